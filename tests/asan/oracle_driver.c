/* Drives the FP64 oracle's C functions over a small input, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer: direct sums, list sums with
 * particle-only lists (every group's list is every particle, so they must
 * equal the direct sums), list sums with cells and textbook tensors (plain and
 * expanded), point fields, quadrupole fields and derivatives, SPH sums, and a
 * malformed list.  Prints "ok". */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_direct(int64_t n, const double *pos, const double *mass, double eps, int64_t n_tgt,
                   const int64_t *tgt, double *acc, double *pot);
int oracle_list_force(int64_t n, const double *pos, const double *mass, int64_t n_groups,
                      const int64_t *group_off, const int64_t *list_off, const int64_t *list_idx,
                      int64_t n_cells, const double *cell_com, const double *cell_mass,
                      const int64_t *n_cellent, const int64_t *pair_off, const double *quad, double eps,
                      int64_t n_tgt, const int64_t *tgt, double *acc, double *pot);
int oracle_list_force_expanded(int64_t n, const double *pos, const double *mass, int64_t n_groups,
                               const int64_t *group_off, const int64_t *list_off, const int64_t *list_idx,
                               int64_t n_cells, const double *cell_com, const double *cell_mass,
                               const int64_t *n_cellent, const int64_t *pair_off, const double *quad,
                               double eps, int64_t n_tgt, const int64_t *tgt, double *acc, double *pot);
void oracle_point_field(int64_t n_pts, const double *x, const int64_t *src_off, const int64_t *src_idx,
                        const double *pos, const double *mass, double eps, double *acc, double *pot);
void oracle_quad_field(int64_t n_pts, const double *x, const double *centre, const double *quad, double eps,
                       double *acc, double *pot);
void oracle_quad_derivs(int64_t n_pts, const double *x, const double *centre, const double *quad, double eps,
                        double *acc, double *jac, double *hess, double *pot);
void oracle_sph_sum(int64_t n, const double *pos, const double *h, const double *q, int64_t n_tgt,
                    const int64_t *tgt, double *out);

static uint64_t state = 0x2545F4914F6CDD1Dull;
static double uniform(void) { /* xorshift64* */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 0x2545F4914F6CDD1Dull) >> 11) * 0x1.0p-53;
}

static int fails = 0;
static void expect(int ok, const char *what) {
    if (!ok) {
        printf("FAILED: %s\n", what);
        fails++;
    }
}

int main(void) {
    enum { N = 400, G = 13, C = 5 };
    double *pos = malloc(3 * N * sizeof(double)), *mass = malloc(N * sizeof(double));
    for (int i = 0; i < N; i++) {
        for (int k = 0; k < 3; k++) pos[3 * i + k] = uniform();
        mass[i] = 0.5 + uniform();
    }
    double *ad = malloc(3 * N * sizeof(double)), *pd = malloc(N * sizeof(double));
    oracle_direct(N, pos, mass, 0.01, N, NULL, ad, pd);

    /* G groups of ragged size, each listing every particle */
    int64_t group_off[G + 1], list_off[G + 1];
    for (int g = 0; g <= G; g++) group_off[g] = (int64_t)g * N / G;
    int64_t *list_idx = malloc((size_t)G * N * sizeof(int64_t));
    for (int g = 0; g < G; g++) {
        list_off[g] = (int64_t)g * N;
        for (int j = 0; j < N; j++) list_idx[(int64_t)g * N + j] = j;
    }
    list_off[G] = (int64_t)G * N;
    double *al = malloc(3 * N * sizeof(double)), *pl = malloc(N * sizeof(double));
    expect(oracle_list_force(N, pos, mass, G, group_off, list_off, list_idx, 0, NULL, NULL, NULL, NULL, NULL, 0.01,
                             N, NULL, al, pl) == 0, "list force");
    double worst = 0;
    for (int i = 0; i < 3 * N; i++) worst = fmax(worst, fabs(al[i] - ad[i]) / (fabs(ad[i]) + 1e-300));
    expect(worst < 1e-9, "full lists equal the direct sum");

    /* one group with C cells first (far away) and its own particles after */
    double cell_com[3 * C], cell_mass[C], quad[6 * C];
    for (int c = 0; c < C; c++) {
        for (int k = 0; k < 3; k++) cell_com[3 * c + k] = 5.0 + c + uniform();
        cell_mass[c] = 1.0 + c;
        for (int k = 0; k < 6; k++) quad[6 * c + k] = 0.01 * (uniform() - 0.5);
    }
    const int ng = 20;
    int64_t go1[2] = {0, ng}, lo1[2] = {0, C + ng}, li1[C + ng], nce[1] = {C}, po[2] = {0, C};
    for (int c = 0; c < C; c++) li1[c] = N + c;
    for (int j = 0; j < ng; j++) li1[C + j] = j;
    int64_t tgt[ng];
    for (int j = 0; j < ng; j++) tgt[j] = j;
    double a1[3 * ng], p1[ng], a2[3 * ng], p2[ng];
    expect(oracle_list_force(N, pos, mass, 1, go1, lo1, li1, C, cell_com, cell_mass, nce, po, quad, 0.01, ng, tgt,
                             a1, p1) == 0, "cells + quadrupoles");
    expect(oracle_list_force_expanded(N, pos, mass, 1, go1, lo1, li1, C, cell_com, cell_mass, nce, po, quad, 0.01,
                                      ng, tgt, a2, p2) == 0, "expanded");
    for (int i = 0; i < 3 * ng; i++) expect(isfinite(a1[i]) && isfinite(a2[i]), "finite fields");
    li1[3] = N + C;   /* a cell past the table */
    expect(oracle_list_force(N, pos, mass, 1, go1, lo1, li1, C, cell_com, cell_mass, NULL, NULL, NULL, 0.01, ng,
                             tgt, a1, p1) != 0, "out-of-range cell rejected");

    /* point fields, quadrupole fields and derivatives, SPH sums */
    int64_t so[3] = {0, 10, 30}, si[30];
    for (int k = 0; k < 30; k++) si[k] = 7 * k % N;
    double x[6] = {0.1, 0.2, 0.3, 2.0, 2.0, 2.0}, ap[6], pp[2];
    oracle_point_field(2, x, so, si, pos, mass, 0.01, ap, pp);
    double centre[6] = {0, 0, 0, 1, 1, 1}, aq[6], pq[2], jac[12], hess[20], pq2[2];
    oracle_quad_field(2, x, centre, quad, 0.01, aq, pq);
    oracle_quad_derivs(2, x, centre, quad, 0.01, aq, jac, hess, pq2);
    double *h = malloc(N * sizeof(double)), *out = malloc(N * sizeof(double));
    for (int i = 0; i < N; i++) h[i] = 0.1 + 0.1 * uniform();
    oracle_sph_sum(N, pos, h, mass, N, NULL, out);
    for (int i = 0; i < N; i++) expect(out[i] > 0, "SPH density positive");

    free(pos); free(mass); free(ad); free(pd); free(list_idx); free(al); free(pl); free(h); free(out);
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
