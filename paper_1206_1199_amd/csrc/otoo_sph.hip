// SPH-style gather sums over neighbour lists (Sec. 2.3, Eq. 4): the second
// workload on the group/list machinery of the gravity path.  Particles only,
// no cells (a cell is opened or skipped whole by the SPH walk).
#include "otoo_internal.h"

using namespace otoo_detail;

namespace {

constexpr int kSphTile = 256;   // list entries staged in LDS per step
constexpr float kInvPi = 0.318309886183790672f;

// cubic B-spline shape: w(u) = 1 - 6u^2 + 6u^3 on [0, 1/2], 2 (1 - u)^3 on
// [1/2, 1], 0 beyond, written as 2 a^3 - 8 b^3 with a = max(1 - u, 0) and
// b = max(1/2 - u, 0) (the two truncated cubics agree with the pieces)
__device__ __forceinline__ float spline_w(float u) {
    const float a = fmaxf(1.f - u, 0.f);
    const float b = fmaxf(0.5f - u, 0.f);
    return fmaf(2.f * a * a, a, -8.f * b * b * b);
}

// Source record of one list entry, as staged in LDS: position and 1/h,
// then q and q sigma (sigma = 8 / (pi h^3)).  Entries that are not particles
// get q = 0.
struct SphSrc {
    float4 x;
    float2 q;
};

__device__ __forceinline__ SphSrc load_src(const float* __restrict__ pos, const float* __restrict__ hh,
                                           const float* __restrict__ q, const int32_t* __restrict__ list_idx,
                                           int64_t e, int32_t n, int32_t* err) {
    SphSrc r;
    const int32_t j = list_idx[e];
    if (j >= 0 && j < n) {
        const float ih = 1.f / hh[j];
        const float qj = q[j];
        r.x = make_float4(pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], ih);
        r.q = make_float2(qj, qj * (8.f * kInvPi) * ih * ih * ih);
    } else {
        atomicOr(err, kErrIndex);
        r.x = make_float4(0.f, 0.f, 0.f, 0.f);
        r.q = make_float2(0.f, 0.f);
    }
    return r;
}

// One workgroup per group (grid-stride).  Lanes are (target, slice): with
// n_g targets, S = 256 / n_g slices split each staged tile into S
// contiguous runs of `rows` entries, padded with zero-weight entries, so
// every lane runs the same trip count over consecutive LDS records.  Tiles
// are double-buffered: each thread gathers its entry of the next tile into
// registers while the workgroup works on the current one (one barrier per
// tile).  Per target the slices' partial sums are combined in slice order,
// so results are reproducible.  Sums A = sum q_j w(r/h_i) and
// B = sum q_j sigma_j w(r/h_j) give out_i = (sigma_i A + B) / 2 with
// sigma = 8 / (pi h^3).
__global__ __launch_bounds__(kBlock) void k_sph(int32_t n, const float* __restrict__ pos,
                                                const float* __restrict__ hh, const float* __restrict__ q,
                                                int32_t n_groups, const int32_t* __restrict__ group_off,
                                                int64_t n_entries, const int64_t* __restrict__ list_off,
                                                const int32_t* __restrict__ list_idx, float* __restrict__ out,
                                                int32_t* err) {
    __shared__ float4 sX[2][kSphTile];   // x, y, z, 1/h
    __shared__ float2 sQ[2][kSphTile];   // q, q sigma
    __shared__ float2 red[kBlock];
    const int t = threadIdx.x;
    const SphSrc zero{make_float4(0.f, 0.f, 0.f, 0.f), make_float2(0.f, 0.f)};
    for (int g = blockIdx.x; g < n_groups; g += gridDim.x) {
        const int g0 = group_off[g];
        const int ng = group_off[g + 1] - g0;
        const bool gok = ng >= 1 && ng <= kBlock && g0 >= 0 && g0 + ng <= n;
        if (!gok) {
            if (t == 0) atomicOr(err, kErrGroup);
            continue;   // uniform across the workgroup
        }
        const int S = kBlock / ng;
        const int ti = t % ng, sl = t / ng;
        const bool lane_on = sl < S;
        const int tstride = S * (kSphTile / S);   // entries per tile, a multiple of S
        const int i = g0 + ti;
        const float xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        const float ihi = 1.f / hh[i];
        float A = 0.f, B = 0.f;
        int64_t lb, le;
        list_range(list_off, n_entries, g, lb, le);
        const int64_t len = le - lb;
        __syncthreads();   // the previous group's buffers and reduction have been read
        SphSrc r = (t < tstride && t < len) ? load_src(pos, hh, q, list_idx, lb + t, n, err) : zero;
        int cur = 0;
        for (int64_t base = 0; base < len; base += tstride) {
            const int tl = (int)((len - base) < tstride ? (len - base) : tstride);
            const int rows = (tl + S - 1) / S;
            sX[cur][t] = r.x;     // entries at or beyond tl are zero weight
            sQ[cur][t] = r.q;
            __syncthreads();
            // gather this thread's entry of the next tile (lands while this one is computed)
            const int64_t nxt = base + tstride + t;
            r = (t < tstride && nxt < len) ? load_src(pos, hh, q, list_idx, lb + nxt, n, err) : zero;
            if (lane_on) {
                const float4* xp = sX[cur] + sl * rows;
                const float2* qp = sQ[cur] + sl * rows;
#pragma unroll 8
                for (int m = 0; m < rows; m++) {
                    const float4 s4 = xp[m];
                    const float2 w = qp[m];
                    const float dx = s4.x - xi, dy = s4.y - yi, dz = s4.z - zi;
                    const float rr = __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
                    A = fmaf(w.x, spline_w(rr * ihi), A);
                    B = fmaf(w.y, spline_w(rr * s4.w), B);
                }
            }
            cur ^= 1;
        }
        red[t] = make_float2(A, B);
        __syncthreads();
        if (t < ng) {
            float a = 0.f, b = 0.f;
            for (int s = 0; s < S; s++) {
                const float2 v = red[s * ng + t];
                a += v.x;
                b += v.y;
            }
            const float sig = (8.f * kInvPi) * ihi * ihi * ihi;
            out[i] = 0.5f * fmaf(sig, a, b);
        }
    }
}

}  // namespace

extern "C" int otoo_sph_sum(otoo_ctx* c, int32_t n, const float* pos, const float* h, const float* q,
                            int32_t n_groups, const int32_t* group_off, int64_t n_entries, const int64_t* list_off,
                            const int32_t* list_idx, float* out) {
    if (!c) return OTOO_EINVAL;
    c->err.clear();
    if (n < 1 || n_groups < 1 || n_groups > n || n_entries < 0) return fail(c, OTOO_EINVAL, "bad sizes");
    if (!pos || !h || !q || !group_off || !list_off || !out || (n_entries && !list_idx))
        return fail(c, OTOO_EINVAL, "null pointer argument");
    HIP_TRY(c, hipSetDevice(c->device));
    const int blocks = (int)std::min<int64_t>((int64_t)8 * c->num_cu, n_groups);
    hipLaunchKernelGGL(k_sph, dim3(blocks), dim3(kBlock), 0, c->stream, n, pos, h, q, n_groups, group_off, n_entries,
                       list_off, list_idx, out, c->errflag);
    HIP_TRY(c, hipGetLastError());
    return OTOO_OK;
}
