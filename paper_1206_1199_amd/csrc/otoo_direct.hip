// Direct summation at selected targets in FP64: the O(N^2) sum of Sec. 2
// that the tree approximates, used as the accuracy reference of the tree
// force (the "median force error" of a walk setting).
#include "otoo_internal.h"

using namespace otoo_detail;

namespace {

constexpr int kDirTargets = 4;                    // targets per workgroup
constexpr int kDirSlices = kBlock / kDirTargets;  // source slices per target

// Thread t takes target t % kDirTargets of its workgroup and sources
// j = slice, slice + kDirSlices, ...; the slices of one target are combined
// by a fixed-order tree in LDS, so results do not depend on timing.
__global__ __launch_bounds__(kBlock) void k_direct(int32_t n, const float* __restrict__ pos,
                                                   const float* __restrict__ mass, int32_t n_tgt,
                                                   const int32_t* __restrict__ tgt, double eps2,
                                                   double* __restrict__ out_acc, double* __restrict__ out_pot,
                                                   int32_t* err) {
    __shared__ double red[4][kBlock];
    const int t = threadIdx.x, k = t % kDirTargets, sl = t / kDirTargets;
    const int64_t it = (int64_t)blockIdx.x * kDirTargets + k;
    int64_t i = -1;
    if (it < n_tgt) {
        i = tgt[it];
        if (i < 0 || i >= n) {
            if (sl == 0) atomicOr(err, kErrIndex);
            i = -1;
        }
    }
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    if (i >= 0) {
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        for (int64_t j = sl; j < n; j += kDirSlices) {
            if (j == i) continue;
            const double dx = (double)pos[3 * j] - xi;
            const double dy = (double)pos[3 * j + 1] - yi;
            const double dz = (double)pos[3 * j + 2] - zi;
            const double r2 = dx * dx + dy * dy + dz * dz + eps2;
            const double rinv = 1.0 / sqrt(r2);
            const double mr = (double)mass[j] * rinv;
            const double mr3 = mr * rinv * rinv;
            ax += mr3 * dx;
            ay += mr3 * dy;
            az += mr3 * dz;
            ph -= mr;
        }
    }
    red[0][t] = ax;
    red[1][t] = ay;
    red[2][t] = az;
    red[3][t] = ph;
    __syncthreads();
    for (int s2 = kDirSlices / 2; s2 > 0; s2 >>= 1) {
        if (sl < s2)
            for (int c = 0; c < 4; c++) red[c][t] += red[c][t + s2 * kDirTargets];
        __syncthreads();
    }
    if (sl == 0 && it < n_tgt) {
        out_acc[3 * it] = red[0][k];
        out_acc[3 * it + 1] = red[1][k];
        out_acc[3 * it + 2] = red[2][k];
        out_pot[it] = red[3][k];
    }
}

}  // namespace

extern "C" int otoo_direct(otoo_ctx* c, int32_t n, const float* pos, const float* mass, int32_t n_tgt,
                           const int32_t* tgt, float eps, double* out_acc, double* out_pot) {
    if (!c) return OTOO_EINVAL;
    c->err.clear();
    if (n < 1 || n_tgt < 0) return fail(c, OTOO_EINVAL, "bad sizes");
    if (!(eps > 0.f) || !std::isfinite(eps)) return fail(c, OTOO_EINVAL, "eps must be positive and finite");
    if (!pos || !mass || (n_tgt && (!tgt || !out_acc || !out_pot)))
        return fail(c, OTOO_EINVAL, "null pointer argument");
    if (n_tgt == 0) return OTOO_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    const double e = eps;
    const int64_t blocks = ((int64_t)n_tgt + kDirTargets - 1) / kDirTargets;
    hipLaunchKernelGGL(k_direct, dim3((unsigned)blocks), dim3(kBlock), 0, c->stream, n, pos, mass, n_tgt, tgt, e * e,
                       out_acc, out_pot, c->errflag);
    HIP_TRY(c, hipGetLastError());
    return OTOO_OK;
}
