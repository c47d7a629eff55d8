// Drives the host tree build and walks of libotoo over a small clustered
// input with coincident points (which reach the depth cap), for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer.  Every list is checked for
// index range and for holding its own group's particles.  Prints "ok".
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "otoo.h"

namespace {

uint64_t state = 0x9E3779B97F4A7C15ull;
double uniform() {   // xorshift64*
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 0x2545F4914F6CDD1Dull) >> 11) * 0x1.0p-53;
}

int fails = 0;
void expect(bool ok, const char* what) {
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        fails++;
    }
}

void check_lists(const otoo_lists* L, int64_t n, int64_t n_cells, const char* what) {
    expect(L->list_off[0] == 0 && L->list_off[L->n_groups] == L->n_entries, what);
    for (int32_t g = 0; g < L->n_groups; g++) {
        const int32_t g0 = L->group_off[g], g1 = L->group_off[g + 1];
        expect(g1 > g0 && g1 - g0 <= OTOO_MAX_GROUP, what);
        int64_t own = 0;
        for (int64_t e = L->list_off[g]; e < L->list_off[g + 1]; e++) {
            const int32_t j = L->list_idx[e];
            expect(j >= 0 && j < n + n_cells, what);
            if (j >= g0 && j < g1) own++;
        }
        expect(own == g1 - g0, what);
    }
}

}  // namespace

int main() {
    const int64_t n = 6000;
    std::vector<double> pos(3 * n), mass(n, 1.0 / n);
    for (int64_t i = 0; i < n; i++) {
        if (i < n / 2) {   // uniform cube
            for (int k = 0; k < 3; k++) pos[3 * i + k] = uniform();
        } else if (i < n - 200) {   // a tight cluster
            for (int k = 0; k < 3; k++) pos[3 * i + k] = 0.3 + 1e-3 * (uniform() - 0.5);
        } else {   // 200 coincident points
            for (int k = 0; k < 3; k++) pos[3 * i + k] = 0.7;
        }
    }
    otoo_tree* t = nullptr;
    expect(otoo_tree_build(pos.data(), mass.data(), n, 16, &t) == OTOO_OK, "build");
    if (!t) return 1;
    int64_t nn = 0, nc = 0;
    int32_t depth = 0;
    double lo[3], side = 0;
    expect(otoo_tree_info(t, &nn, &nc, &depth, lo, &side) == OTOO_OK && nn == n && nc > 0, "info");
    std::vector<int64_t> perm(n), first(nc), count(nc), ijk(3 * nc), next(n + nc), more(n + nc);
    std::vector<float> p32(3 * n), m32(n), cm(12 * nc);
    std::vector<int32_t> level(nc);
    std::vector<double> com(3 * nc), cmass(nc), cside(nc), s(nc), S6(6 * nc), bmax(nc);
    expect(otoo_tree_export(t, perm.data(), p32.data(), m32.data(), cm.data(), 12) == OTOO_OK, "export");
    expect(otoo_tree_cells(t, first.data(), count.data(), level.data(), ijk.data(), com.data(), cmass.data(),
                           cside.data(), s.data(), S6.data(), bmax.data()) == OTOO_OK, "cells");
    expect(otoo_tree_links(t, next.data(), more.data()) == OTOO_OK, "links");

    for (int32_t mode : {OTOO_GROUP_CHUNK, OTOO_GROUP_CELL})
        for (int32_t g_max : {1, 17, 64, 256})
            for (double theta : {0.0, 0.5, 0.9})
                for (double near_ratio : {0.0, 0.4}) {
                    otoo_walk_params wp{OTOO_MAC_BH, theta, 0.0, INFINITY, mode, g_max, near_ratio};
                    otoo_lists* L = nullptr;
                    expect(otoo_tree_walk(t, &wp, &L) == OTOO_OK && L, "walk");
                    if (L) {
                        check_lists(L, n, nc, "walk lists");
                        for (int32_t g = 0; g < L->n_groups; g++)
                            expect(L->n_near[g] >= 0 && L->n_near[g] <= L->n_cellent[g] &&
                                       (near_ratio > 0.0 || L->n_near[g] == 0),
                                   "near cells within the cells");
                    }
                    otoo_lists_free(L);
                }
    for (double m_limit : {(double)INFINITY, 0.05}) {
        otoo_walk_params wp{OTOO_MAC_ABSOLUTE, 0.0, 0.01, m_limit, OTOO_GROUP_CHUNK, 64};
        otoo_lists* L = nullptr;
        expect(otoo_tree_walk(t, &wp, &L) == OTOO_OK && L, "absolute walk");
        if (L) check_lists(L, n, nc, "absolute walk lists");
        otoo_lists_free(L);
    }
    int32_t ng = 0;
    expect(otoo_tree_groups(t, OTOO_GROUP_CHUNK, 64, &ng) == OTOO_OK && ng > 10, "groups");
    for (int32_t b : {0, 3, ng - 1}) {
        otoo_walk_params wp{OTOO_MAC_BH, 0.6, 0.0, INFINITY, OTOO_GROUP_CHUNK, 64};
        otoo_lists* L = nullptr;
        expect(otoo_tree_walk_range(t, &wp, b, b + 7, &L) == OTOO_OK && L, "walk range");
        if (L) check_lists(L, n, nc, "walk range lists");
        otoo_lists_free(L);
    }
    std::vector<double> h(n, 0.05);
    otoo_lists* L = nullptr;
    expect(otoo_tree_walk_sph(t, h.data(), OTOO_GROUP_CELL, 32, &L) == OTOO_OK && L, "sph walk");
    if (L) check_lists(L, n, 0, "sph lists");
    otoo_lists_free(L);

    // rejected arguments
    otoo_walk_params bad{OTOO_MAC_BH, -1.0, 0.0, INFINITY, OTOO_GROUP_CHUNK, 64};
    L = nullptr;
    expect(otoo_tree_walk(t, &bad, &L) == OTOO_EINVAL && !L, "negative theta");
    bad.theta = 0.5;
    bad.g_max = 0;
    expect(otoo_tree_walk(t, &bad, &L) == OTOO_EINVAL, "g_max 0");
    expect(otoo_tree_walk_range(t, &bad, 5, 5, &L) == OTOO_EINVAL, "empty range");
    bad.g_max = 64;
    bad.near_ratio = -0.5;
    expect(otoo_tree_walk(t, &bad, &L) == OTOO_EINVAL, "negative near ratio");
    bad.near_ratio = NAN;
    expect(otoo_tree_walk(t, &bad, &L) == OTOO_EINVAL, "NaN near ratio");
    h[17] = 0.0;
    expect(otoo_tree_walk_sph(t, h.data(), OTOO_GROUP_CELL, 32, &L) == OTOO_EINVAL, "h = 0");
    otoo_tree* t2 = nullptr;
    expect(otoo_tree_build(pos.data(), mass.data(), 0, 16, &t2) == OTOO_EINVAL && !t2, "n = 0");

    otoo_tree_free(t);
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
