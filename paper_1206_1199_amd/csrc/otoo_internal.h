// Internal declarations shared by the device sources of libotoo (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "otoo.h"

namespace otoo_detail {

constexpr int kBlock = 256;   // threads per force workgroup = largest group
static_assert(kBlock == OTOO_MAX_GROUP, "a workgroup holds one whole group");

enum : int { kErrGroup = 1, kErrIndex = 2, kErrCapacity = 4 };

constexpr int kClasses = 40;   // longest-first cost classes (log2 buckets)

// device-side queue and schedule counters of one context
struct Meta {
    int64_t n_items;
    int64_t n_parts;
    int32_t head;
    int32_t pad;
    int32_t hist[kClasses];
    int32_t cursor[kClasses];
};
// The context's 4 KiB counter block: Meta at 0, the SPH counters at 1024,
// the error flag at 2048.
static_assert(sizeof(Meta) <= 1024, "Meta must fit below the SPH counters");

__device__ __forceinline__ void kahan_add(float& sum, float& comp, float x) {
    // sum + comp carries the running value; comp holds what rounding dropped
    const float y = x + comp;
    const float t = sum + y;
    comp = y - (t - sum);
    sum = t;
}

__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// list range of group g, clamped to [0, n_entries]
__device__ __forceinline__ void list_range(const int64_t* list_off, int64_t n_entries, int g, int64_t& b,
                                           int64_t& e) {
    b = clamp64(list_off[g], 0, n_entries);
    e = clamp64(list_off[g + 1], b, n_entries);
}

__device__ __forceinline__ int64_t n_chunks(int64_t len, int chunk) {
    return len <= chunk ? 1 : (len + chunk - 1) / chunk;
}

// Quadrupole-form field of tensor Q (xx, yy, zz, xy, xz, yz) about a COM,
// at the point whose offset from the COM is d, with its first two
// derivatives, accumulated into f[kCorrTerms] = {ax, ay, az, phi, J (xx, yy,
// zz, xy, xz, yz), H (xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz)},
// where a = -grad phi, J = -grad grad phi, H = -grad grad grad phi and
// phi = -1/2 (d.Qd) r^-5, r^2 = |d|^2 + eps^2.  Written with e = d/r
// (|e| <= 1) so that no power of 1/r beyond the sixth is formed:
//   a_a   = r^-4 [(Qe)_a - 5/2 (e.Qe) e_a]
//   J_ab  = r^-5 [Q_ab - 5 ((Qe)_a e_b + (Qe)_b e_a) + 1/2 (e.Qe) R2_ab]
//   H_abc = r^-6 [-5 (Q_ab e_c + Q_ac e_b + Q_bc e_a)
//                 + (Qe)_a R2_bc + (Qe)_b R2_ac + (Qe)_c R2_ab + 1/2 (e.Qe) R3_abc]
//   phi   = -1/2 (e.Qe) r^-3
// with R2_ab = -5 delta_ab + 35 e_a e_b and
// R3_abc = 35 (delta_ab e_c + delta_ac e_b + delta_bc e_a) - 315 e_a e_b e_c
// (the derivatives of r^-5 divided by the matching powers of 1/r).
constexpr int kCorrTerms = 20;
constexpr int kCorrStride = 24;   // floats per group: the 20 terms, then the centre xyz, pad

__device__ __forceinline__ void quad_expand_add(float dx, float dy, float dz, const float* qp, float eps2,
                                                float* f) {
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float ri2 = ri * ri;
    const float ri3 = ri2 * ri;
    const float ri4 = ri2 * ri2;
    const float ri5 = ri4 * ri;
    const float ri6 = ri3 * ri3;
    const float e[3] = {dx * ri, dy * ri, dz * ri};
    const float Q[3][3] = {{qp[0], qp[3], qp[4]}, {qp[3], qp[1], qp[5]}, {qp[4], qp[5], qp[2]}};
    float qe[3];
#pragma unroll
    for (int k = 0; k < 3; k++) qe[k] = Q[k][0] * e[0] + Q[k][1] * e[1] + Q[k][2] * e[2];
    const float u = e[0] * qe[0] + e[1] * qe[1] + e[2] * qe[2];
    const float hu = 0.5f * u;
    float R2[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) R2[i][j] = (i == j ? -5.f : 0.f) + 35.f * e[i] * e[j];
#pragma unroll
    for (int k = 0; k < 3; k++) f[k] += ri4 * (qe[k] - 2.5f * u * e[k]);
    f[3] += -hu * ri3;
    constexpr int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int m = 0; m < 6; m++) {
        const int i = ia[m], j = ib[m];
        f[4 + m] += ri5 * (Q[i][j] - 5.f * (qe[i] * e[j] + qe[j] * e[i]) + hu * R2[i][j]);
    }
    constexpr int ha[10] = {0, 1, 2, 0, 0, 0, 1, 0, 1, 0}, hb[10] = {0, 1, 2, 0, 0, 1, 1, 2, 2, 1},
                  hc[10] = {0, 1, 2, 1, 2, 1, 2, 2, 2, 2};
#pragma unroll
    for (int m = 0; m < 10; m++) {
        const int i = ha[m], j = hb[m], k = hc[m];
        const float R3 = 35.f * ((i == j ? e[k] : 0.f) + (i == k ? e[j] : 0.f) + (j == k ? e[i] : 0.f)) -
                         315.f * e[i] * e[j] * e[k];
        f[10 + m] += ri6 * (-5.f * (Q[i][j] * e[k] + Q[i][k] * e[j] + Q[j][k] * e[i]) + qe[i] * R2[j][k] +
                            qe[j] * R2[i][k] + qe[k] * R2[i][j] + hu * R3);
    }
}

// The two halves of quad_expand_add, for two lanes sharing one pair:
// part 0 adds {a, phi, J} (f[0..9]), part 1 adds H (f[10..19]).
__device__ __forceinline__ void quad_expand_add_part(int part, float dx, float dy, float dz, const float* qp,
                                                     float eps2, float* f) {
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float ri2 = ri * ri;
    const float ri3 = ri2 * ri;
    const float e[3] = {dx * ri, dy * ri, dz * ri};
    const float Q[3][3] = {{qp[0], qp[3], qp[4]}, {qp[3], qp[1], qp[5]}, {qp[4], qp[5], qp[2]}};
    float qe[3];
#pragma unroll
    for (int k = 0; k < 3; k++) qe[k] = Q[k][0] * e[0] + Q[k][1] * e[1] + Q[k][2] * e[2];
    const float u = e[0] * qe[0] + e[1] * qe[1] + e[2] * qe[2];
    const float hu = 0.5f * u;
    float R2[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) R2[i][j] = (i == j ? -5.f : 0.f) + 35.f * e[i] * e[j];
    if (part == 0) {
        const float ri4 = ri2 * ri2;
        const float ri5 = ri4 * ri;
#pragma unroll
        for (int k = 0; k < 3; k++) f[k] += ri4 * (qe[k] - 2.5f * u * e[k]);
        f[3] += -hu * ri3;
        constexpr int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int m = 0; m < 6; m++) {
            const int i = ia[m], j = ib[m];
            f[4 + m] += ri5 * (Q[i][j] - 5.f * (qe[i] * e[j] + qe[j] * e[i]) + hu * R2[i][j]);
        }
    } else {
        const float ri6 = ri3 * ri3;
        constexpr int ha[10] = {0, 1, 2, 0, 0, 0, 1, 0, 1, 0}, hb[10] = {0, 1, 2, 0, 0, 1, 1, 2, 2, 1},
                      hc[10] = {0, 1, 2, 1, 2, 1, 2, 2, 2, 2};
#pragma unroll
        for (int m = 0; m < 10; m++) {
            const int i = ha[m], j = hb[m], k = hc[m];
            const float R3 = 35.f * ((i == j ? e[k] : 0.f) + (i == k ? e[j] : 0.f) + (j == k ? e[i] : 0.f)) -
                             315.f * e[i] * e[j] * e[k];
            f[10 + m] += ri6 * (-5.f * (Q[i][j] * e[k] + Q[i][k] * e[j] + Q[j][k] * e[i]) + qe[i] * R2[j][k] +
                                qe[j] * R2[i][k] + qe[k] * R2[i][j] + hu * R3);
        }
    }
}

}  // namespace otoo_detail

struct otoo_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    otoo_tuning tune{1024, 8, 1, 0, 256, 0};
    int num_cu = 0;
    // scratch
    void* buf = nullptr;
    size_t buf_bytes = 0;
    otoo_detail::Meta* meta = nullptr;
    int32_t* errflag = nullptr;
    // timing
    bool timing = false;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    // SPH gather sums: work-queue counters (inside the 4 KiB block of meta)
    // and scratch for the item lists and chunk partials, grown on demand
    void* sph_meta = nullptr;
    void* sph_buf = nullptr;
    size_t sph_bytes = 0;
};


namespace otoo_detail {

inline int fail(otoo_ctx* c, int code, const char* fmt, ...) {
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    if (c) c->err = msg;
    return code;
}

}  // namespace otoo_detail

#define HIP_TRY(c, expr)                                                                             \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return otoo_detail::fail((c), OTOO_EHIP, "%s: %s", #expr, hipGetErrorString(e_));           \
    } while (0)


