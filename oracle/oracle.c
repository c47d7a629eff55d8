/*
 * FP64 CPU oracle for the octree gravity force path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * call this file.  It shares no code, header or constant with the HIP library.
 * Every loop is plain, in a fixed order, in double precision, with no blocking
 * or vector intrinsics; the outer loop over target particles may run on
 * several OpenMP threads (each target's sum is still taken in list order).
 *
 * Units: G = 1.  Softening is Plummer's: a source of mass m at y acts on a
 * target at x with
 *     acceleration  m (y - x) (|y - x|^2 + eps^2)^(-3/2)
 *     potential    -m (|y - x|^2 + eps^2)^(-1/2).
 * The paper only says that particle-particle interactions use a
 * gravitational softening length (Sec. 3.4, description of the r_b slot);
 * the Plummer form is the reading taken here.
 *
 *   oracle_direct      O(N^2) direct summation over all j != i (Sec. 2: the
 *                      brute-force method the tree replaces).
 *   oracle_list_force  the same sums over a group's interaction list, where
 *                      index e < n is particle e and index e >= n is cell
 *                      e - n acting as a virtual particle of mass M_c at its
 *                      centre of mass (monopole, Sec. 2; unified particle/cell
 *                      index space, Sec. 3.2).  The target's own entry is
 *                      skipped (self pair excluded).  Optionally each cell
 *                      entry also carries a symmetric tensor Qt (6 numbers per
 *                      (group, cell) pair) whose quadrupole-form field is added:
 *                          phi_Q = -1/2 d^T Qt d r^-5,
 *                          a_Q   = Qt d r^-5 - 5/2 (d^T Qt d) d r^-7,
 *                      with d = x - COM_c and r^2 = |d|^2 + eps^2.  This is the
 *                      quadrupole term of the multipole expansion the paper
 *                      names (orders up to p = 3, Sec. 2), softened like the
 *                      monopole.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

/* one softened source acting on one target: adds to a[3] and *phi */
static void pair_monopole(const double x[3], const double y[3], double m, double eps2,
                          double a[3], double *phi)
{
    double dx = y[0] - x[0];
    double dy = y[1] - x[1];
    double dz = y[2] - x[2];
    double r2 = dx * dx + dy * dy + dz * dz + eps2;
    double r = sqrt(r2);
    double inv_r = 1.0 / r;
    double inv_r3 = inv_r / r2;
    a[0] += m * dx * inv_r3;
    a[1] += m * dy * inv_r3;
    a[2] += m * dz * inv_r3;
    *phi -= m * inv_r;
}

/* quadrupole-form field of tensor q = (xx, yy, zz, xy, xz, yz) centred at c */
static void pair_quadrupole(const double x[3], const double c[3], const double q[6], double eps2,
                            double a[3], double *phi)
{
    double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
    double inv_r2 = 1.0 / r2;
    double inv_r = sqrt(inv_r2);
    double inv_r5 = inv_r * inv_r2 * inv_r2;
    double inv_r7 = inv_r5 * inv_r2;
    /* Qd */
    double qd[3];
    qd[0] = q[0] * d[0] + q[3] * d[1] + q[4] * d[2];
    qd[1] = q[3] * d[0] + q[1] * d[1] + q[5] * d[2];
    qd[2] = q[4] * d[0] + q[5] * d[1] + q[2] * d[2];
    double dqd = d[0] * qd[0] + d[1] * qd[1] + d[2] * qd[2];
    for (int k = 0; k < 3; k++)
        a[k] += qd[k] * inv_r5 - 2.5 * dqd * d[k] * inv_r7;
    *phi += -0.5 * dqd * inv_r5;
}

/*
 * Quadrupole-form field of tensor q centred at c, at point x, with its first
 * two derivatives.  phi = -1/2 u rho with u = d.Qd, rho = r^-5, d = x - c,
 * r^2 = |d|^2 + eps^2; a = -grad phi, J_ab = -d_a d_b phi (stored xx, yy, zz,
 * xy, xz, yz) and H_abc = -d_a d_b d_c phi (fully symmetric, stored xxx, yyy,
 * zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz).  Since u has constant second
 * derivatives 2Q and vanishing third ones, Leibniz's rule gives
 *   a_a    = (Qd)_a rho + 1/2 u rho_a
 *   J_ab   = Q_ab rho + (Qd)_a rho_b + (Qd)_b rho_a + 1/2 u rho_ab
 *   H_abc  = Q_ab rho_c + Q_ac rho_b + Q_bc rho_a
 *            + (Qd)_a rho_bc + (Qd)_b rho_ac + (Qd)_c rho_ab + 1/2 u rho_abc
 * with rho_a = -5 r^-7 d_a, rho_ab = -5 r^-7 delta_ab + 35 r^-9 d_a d_b,
 * rho_abc = 35 r^-9 (delta_ab d_c + delta_ac d_b + delta_bc d_a) - 315 r^-11 d_a d_b d_c.
 */
static const int H_IDX[10][3] = {{0, 0, 0}, {1, 1, 1}, {2, 2, 2}, {0, 0, 1}, {0, 0, 2},
                                 {0, 1, 1}, {1, 1, 2}, {0, 2, 2}, {1, 2, 2}, {0, 1, 2}};

static void quad_field_derivs(const double x[3], const double c[3], const double q[6], double eps2,
                              double a[3], double J[6], double H[10], double *phi)
{
    double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
    double inv_r2 = 1.0 / r2;
    double inv_r = sqrt(inv_r2);
    double r5 = inv_r * inv_r2 * inv_r2;
    double r7 = r5 * inv_r2;
    double r9 = r7 * inv_r2;
    double r11 = r9 * inv_r2;
    double Q[3][3] = {{q[0], q[3], q[4]}, {q[3], q[1], q[5]}, {q[4], q[5], q[2]}};
    double qd[3];
    for (int k = 0; k < 3; k++)
        qd[k] = Q[k][0] * d[0] + Q[k][1] * d[1] + Q[k][2] * d[2];
    double u = d[0] * qd[0] + d[1] * qd[1] + d[2] * qd[2];
    double rho = r5, rho1[3], rho2[3][3];
    for (int k = 0; k < 3; k++)
        rho1[k] = -5.0 * r7 * d[k];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            rho2[i][j] = (i == j ? -5.0 * r7 : 0.0) + 35.0 * r9 * d[i] * d[j];
    for (int k = 0; k < 3; k++)
        a[k] = qd[k] * rho + 0.5 * u * rho1[k];
    static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int m = 0; m < 6; m++) {
        int i = ia[m], j = ib[m];
        J[m] = Q[i][j] * rho + qd[i] * rho1[j] + qd[j] * rho1[i] + 0.5 * u * rho2[i][j];
    }
    for (int m = 0; m < 10; m++) {
        int i = H_IDX[m][0], j = H_IDX[m][1], k = H_IDX[m][2];
        double rho3 = 35.0 * r9 * ((i == j ? d[k] : 0.0) + (i == k ? d[j] : 0.0) + (j == k ? d[i] : 0.0)) -
                      315.0 * r11 * d[i] * d[j] * d[k];
        H[m] = Q[i][j] * rho1[k] + Q[i][k] * rho1[j] + Q[j][k] * rho1[i] + qd[i] * rho2[j][k] +
               qd[j] * rho2[i][k] + qd[k] * rho2[i][j] + 0.5 * u * rho3;
    }
    *phi = -0.5 * u * rho;
}

/* the stored component of the symmetric H for index triple (i, j, k) */
static double H_at(const double H[10], int i, int j, int k)
{
    int s[3] = {i, j, k};
    /* sort the three indices */
    for (int p = 0; p < 2; p++)
        for (int q = 0; q < 2 - p; q++)
            if (s[q] > s[q + 1]) {
                int tmp = s[q];
                s[q] = s[q + 1];
                s[q + 1] = tmp;
            }
    for (int m = 0; m < 10; m++)
        if (H_IDX[m][0] == s[0] && H_IDX[m][1] == s[1] && H_IDX[m][2] == s[2])
            return H[m];
    return 0.0;
}

/*
 * Direct sum.  pos[n][3], mass[n]; targets tgt[n_tgt] (NULL = all particles,
 * then n_tgt must equal n).  Writes acc[n_tgt][3], pot[n_tgt].
 */
void oracle_direct(int64_t n, const double *pos, const double *mass, double eps,
                   int64_t n_tgt, const int64_t *tgt, double *acc, double *pot)
{
    double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_tgt; t++) {
        int64_t i = tgt ? tgt[t] : t;
        double a[3] = {0.0, 0.0, 0.0};
        double phi = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i)
                continue;
            pair_monopole(&pos[3 * i], &pos[3 * j], mass[j], eps2, a, &phi);
        }
        acc[3 * t + 0] = a[0];
        acc[3 * t + 1] = a[1];
        acc[3 * t + 2] = a[2];
        pot[t] = phi;
    }
}

/* group containing particle i: largest g with group_off[g] <= i */
static int64_t find_group(int64_t n_groups, const int64_t *group_off, int64_t i)
{
    int64_t lo = 0, hi = n_groups - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (group_off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

/*
 * List force.  Particles pos[n][3], mass[n]; groups are the ranges
 * [group_off[g], group_off[g+1]) of particle indices; group g's list is
 * list_idx[list_off[g] .. list_off[g+1]).  Cells: cell_com[n_cells][3],
 * cell_mass[n_cells].  Optional quadrupole-form tensors: the first
 * n_cellent[g] entries of a group's list are cells that carry a tensor, the
 * k-th of them quad[(pair_off[g] + k) * 6 ...]; cell entries after them
 * (the far cells of a list whose near cells lead it) act as monopoles only;
 * pass quad = NULL for monopole only.  Targets tgt[n_tgt] (NULL = all
 * particles).  Returns 0, or -1 if an index is out of range or a cell
 * tensor is requested for a particle entry.
 */
int oracle_list_force(int64_t n, const double *pos, const double *mass,
                      int64_t n_groups, const int64_t *group_off,
                      const int64_t *list_off, const int64_t *list_idx,
                      int64_t n_cells, const double *cell_com, const double *cell_mass,
                      const int64_t *n_cellent, const int64_t *pair_off, const double *quad,
                      double eps, int64_t n_tgt, const int64_t *tgt,
                      double *acc, double *pot)
{
    double eps2 = eps * eps;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t t = 0; t < n_tgt; t++) {
        int64_t i = tgt ? tgt[t] : t;
        int64_t g = find_group(n_groups, group_off, i);
        double a[3] = {0.0, 0.0, 0.0};
        double phi = 0.0;
        for (int64_t k = list_off[g]; k < list_off[g + 1]; k++) {
            int64_t e = list_idx[k];
            int64_t kk = k - list_off[g];
            if (e < 0 || e >= n + n_cells) {
                bad = 1;
                continue;
            }
            if (e < n) {
                if (quad && kk < n_cellent[g])
                    bad = 1;
                if (e == i)
                    continue;
                pair_monopole(&pos[3 * i], &pos[3 * e], mass[e], eps2, a, &phi);
            } else {
                int64_t c = e - n;
                pair_monopole(&pos[3 * i], &cell_com[3 * c], cell_mass[c], eps2, a, &phi);
                if (quad && kk < n_cellent[g])
                    pair_quadrupole(&pos[3 * i], &cell_com[3 * c], &quad[6 * (pair_off[g] + kk)],
                                    eps2, a, &phi);
            }
        }
        acc[3 * t + 0] = a[0];
        acc[3 * t + 1] = a[1];
        acc[3 * t + 2] = a[2];
        pot[t] = phi;
    }
    return bad ? -1 : 0;
}

/*
 * List force whose cell tensors act through a second-order local expansion
 * about the centre c_g of group g's bounding box (the form the device
 * applies).  With A_g, J_g, H_g and Phi_g the sums over the group's cell
 * entries of the quadrupole-form field, its first and second derivatives
 * and potential at c_g, and delta = x_i - c_g:
 *     a_i   += A_g + J_g delta + 1/2 H_g[delta, delta]
 *     phi_i += Phi_g - A_g . delta - 1/2 delta . J_g delta
 * (a = -grad phi, so the potential's expansion uses -A and -J), on top of
 * the monopole list sums of oracle_list_force.  Arguments as for
 * oracle_list_force with quad required.  Returns 0 or -1 (malformed lists).
 */
int oracle_list_force_expanded(int64_t n, const double *pos, const double *mass,
                               int64_t n_groups, const int64_t *group_off,
                               const int64_t *list_off, const int64_t *list_idx,
                               int64_t n_cells, const double *cell_com, const double *cell_mass,
                               const int64_t *n_cellent, const int64_t *pair_off, const double *quad,
                               double eps, int64_t n_tgt, const int64_t *tgt,
                               double *acc, double *pot)
{
    int rc = oracle_list_force(n, pos, mass, n_groups, group_off, list_off, list_idx, n_cells, cell_com,
                               cell_mass, NULL, NULL, NULL, eps, n_tgt, tgt, acc, pot);
    if (rc)
        return rc;
    double eps2 = eps * eps;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t t = 0; t < n_tgt; t++) {
        int64_t i = tgt ? tgt[t] : t;
        int64_t g = find_group(n_groups, group_off, i);
        double lo[3], hi[3], cg[3];
        for (int k = 0; k < 3; k++)
            lo[k] = hi[k] = pos[3 * group_off[g] + k];
        for (int64_t p = group_off[g]; p < group_off[g + 1]; p++)
            for (int k = 0; k < 3; k++) {
                double v = pos[3 * p + k];
                lo[k] = v < lo[k] ? v : lo[k];
                hi[k] = v > hi[k] ? v : hi[k];
            }
        for (int k = 0; k < 3; k++)
            cg[k] = 0.5 * (lo[k] + hi[k]);
        double A[3] = {0, 0, 0}, J[6] = {0}, H[10] = {0}, Phi = 0.0;
        for (int64_t kk = 0; kk < n_cellent[g]; kk++) {
            int64_t e = list_idx[list_off[g] + kk];
            if (e < n || e >= n + n_cells) {
                bad = 1;
                continue;
            }
            double a1[3], J1[6], H1[10], p1;
            quad_field_derivs(cg, &cell_com[3 * (e - n)], &quad[6 * (pair_off[g] + kk)], eps2, a1, J1, H1, &p1);
            for (int k = 0; k < 3; k++)
                A[k] += a1[k];
            for (int k = 0; k < 6; k++)
                J[k] += J1[k];
            for (int k = 0; k < 10; k++)
                H[k] += H1[k];
            Phi += p1;
        }
        double dl[3] = {pos[3 * i] - cg[0], pos[3 * i + 1] - cg[1], pos[3 * i + 2] - cg[2]};
        double Jm[3][3] = {{J[0], J[3], J[4]}, {J[3], J[1], J[5]}, {J[4], J[5], J[2]}};
        double quadform = 0.0;
        for (int a = 0; a < 3; a++) {
            double lin = 0.0, sec = 0.0;
            for (int b = 0; b < 3; b++) {
                lin += Jm[a][b] * dl[b];
                for (int c = 0; c < 3; c++)
                    sec += H_at(H, a, b, c) * dl[b] * dl[c];
            }
            acc[3 * t + a] += A[a] + lin + 0.5 * sec;
            quadform += dl[a] * lin;
        }
        pot[t] += Phi - (A[0] * dl[0] + A[1] * dl[1] + A[2] * dl[2]) - 0.5 * quadform;
    }
    return bad ? -1 : 0;
}

/* quadrupole-form field with its Jacobian and Hessian at points (pins them) */
void oracle_quad_derivs(int64_t n_pts, const double *x, const double *centre, const double *quad,
                        double eps, double *acc, double *jac, double *hess, double *pot)
{
    double eps2 = eps * eps;
    for (int64_t t = 0; t < n_pts; t++)
        quad_field_derivs(&x[3 * t], &centre[3 * t], &quad[6 * t], eps2, &acc[3 * t], &jac[6 * t],
                          &hess[10 * t], &pot[t]);
}

/*
 * Exact field of a set of sources at arbitrary points: for each target point
 * x[t], sum over sources src_idx[src_off[t] .. src_off[t+1]) of the softened
 * monopole field (no self exclusion: the targets are points, not particles).
 * Used to compute the exact field of a cell's particles (the truth the
 * learned correction is fitted to).
 */
void oracle_point_field(int64_t n_pts, const double *x, const int64_t *src_off,
                        const int64_t *src_idx, const double *pos, const double *mass,
                        double eps, double *acc, double *pot)
{
    double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < n_pts; t++) {
        double a[3] = {0.0, 0.0, 0.0};
        double phi = 0.0;
        for (int64_t k = src_off[t]; k < src_off[t + 1]; k++) {
            int64_t j = src_idx[k];
            pair_monopole(&x[3 * t], &pos[3 * j], mass[j], eps2, a, &phi);
        }
        acc[3 * t + 0] = a[0];
        acc[3 * t + 1] = a[1];
        acc[3 * t + 2] = a[2];
        pot[t] = phi;
    }
}

/* quadrupole-form field alone at points (used to test it against -grad phi) */
void oracle_quad_field(int64_t n_pts, const double *x, const double *centre, const double *quad,
                       double eps, double *acc, double *pot)
{
    double eps2 = eps * eps;
    for (int64_t t = 0; t < n_pts; t++) {
        double a[3] = {0.0, 0.0, 0.0};
        double phi = 0.0;
        pair_quadrupole(&x[3 * t], &centre[3 * t], &quad[6 * t], eps2, a, &phi);
        acc[3 * t + 0] = a[0];
        acc[3 * t + 1] = a[1];
        acc[3 * t + 2] = a[2];
        pot[t] = phi;
    }
}

/*
 * SPH-style gather sums (Sec. 2.3, Eq. 4): for each target i,
 *     s_i = sum over all j (i included) of q_j Wbar_ij,
 *     Wbar_ij = (W(r_ij, h_i) + W(r_ij, h_j)) / 2,
 * with the cubic B-spline kernel of compact support h (Monaghan & Lattanzio
 * 1985):  W(r, h) = 8 / (pi h^3) w(r / h),
 *     w(u) = 1 - 6 u^2 + 6 u^3    for 0 <= u <= 1/2,
 *            2 (1 - u)^3          for 1/2 < u <= 1,
 *            0                    beyond.
 * The paper leaves the kernel open (bell-shaped, zero beyond the neighbour
 * radius h); this kernel and the symmetrised pair weight are the reading
 * taken.  Brute force over all j: no tree and no lists.
 */
static const double kPi = 3.14159265358979323846;

static double sph_w(double r, double h)
{
    double u = r / h;
    double w;
    if (u <= 0.5) {
        w = 1.0 - 6.0 * u * u + 6.0 * u * u * u;
    } else if (u <= 1.0) {
        double v = 1.0 - u;
        w = 2.0 * v * v * v;
    } else {
        w = 0.0;
    }
    return 8.0 / (kPi * h * h * h) * w;
}

double oracle_sph_kernel(double r, double h) { return sph_w(r, h); }

void oracle_sph_sum(int64_t n, const double *pos, const double *h, const double *q, int64_t n_tgt,
                    const int64_t *tgt, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_tgt; k++) {
        int64_t i = tgt ? tgt[k] : k;
        double s = 0.0;
        for (int64_t j = 0; j < n; j++) {
            double dx = pos[3 * j + 0] - pos[3 * i + 0];
            double dy = pos[3 * j + 1] - pos[3 * i + 1];
            double dz = pos[3 * j + 2] - pos[3 * i + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            s += q[j] * 0.5 * (sph_w(r, h[i]) + sph_w(r, h[j]));
        }
        out[k] = s;
    }
}
