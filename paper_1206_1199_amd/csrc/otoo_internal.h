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
    int32_t n_split;   // groups whose list is split into several items (listed for the reduction)
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

// Per-pair quantities shared by the terms: e = d/r, Qe, u = e.Qe and the
// powers of 1/r.  The terms are the formulas above with e_a e_b formed once,
// the delta terms of H gathered into V = r^-6 (-5 Qe + 35/2 u e), and the
// constant factors carried by scaled vectors, so that each J term costs four
// fused multiply-adds and each H term four to six.
struct QuadPair {
    float e0, e1, e2, q0, q1, q2, u, ri3, ri4, ri5, ri6;
};
__device__ __forceinline__ void quad_pair_setup(float dx, float dy, float dz, float ri, const float* qp, QuadPair& p) {
    const float ri2 = ri * ri;
    p.ri3 = ri2 * ri;
    p.ri4 = ri2 * ri2;
    p.ri5 = p.ri4 * ri;
    p.ri6 = p.ri3 * p.ri3;
    p.e0 = dx * ri;
    p.e1 = dy * ri;
    p.e2 = dz * ri;
    p.q0 = fmaf(qp[0], p.e0, fmaf(qp[3], p.e1, qp[4] * p.e2));
    p.q1 = fmaf(qp[3], p.e0, fmaf(qp[1], p.e1, qp[5] * p.e2));
    p.q2 = fmaf(qp[4], p.e0, fmaf(qp[5], p.e1, qp[2] * p.e2));
    p.u = fmaf(p.e0, p.q0, fmaf(p.e1, p.q1, p.e2 * p.q2));
}
// a (3), phi and J (6): f[0..9]
__device__ __forceinline__ void quad_add_low(const QuadPair& p, const float* qp, float* f) {
    const float e0 = p.e0, e1 = p.e1, e2 = p.e2;
    const float a2 = -2.5f * p.u * p.ri4;
    f[0] = fmaf(p.ri4, p.q0, fmaf(a2, e0, f[0]));
    f[1] = fmaf(p.ri4, p.q1, fmaf(a2, e1, f[1]));
    f[2] = fmaf(p.ri4, p.q2, fmaf(a2, e2, f[2]));
    f[3] = fmaf(-0.5f * p.u, p.ri3, f[3]);
    const float s = -5.f * p.ri5;
    const float qs0 = s * p.q0, qs1 = s * p.q1, qs2 = s * p.q2;
    const float ur5 = p.u * p.ri5;
    const float j3 = 17.5f * ur5, jd = -2.5f * ur5;
    const float E00 = e0 * e0, E11 = e1 * e1, E22 = e2 * e2, E01 = e0 * e1, E02 = e0 * e2, E12 = e1 * e2;
    f[4] = fmaf(p.ri5, qp[0], fmaf(2.f * qs0, e0, fmaf(j3, E00, f[4] + jd)));
    f[5] = fmaf(p.ri5, qp[1], fmaf(2.f * qs1, e1, fmaf(j3, E11, f[5] + jd)));
    f[6] = fmaf(p.ri5, qp[2], fmaf(2.f * qs2, e2, fmaf(j3, E22, f[6] + jd)));
    f[7] = fmaf(p.ri5, qp[3], fmaf(qs0, e1, fmaf(qs1, e0, fmaf(j3, E01, f[7]))));
    f[8] = fmaf(p.ri5, qp[4], fmaf(qs0, e2, fmaf(qs2, e0, fmaf(j3, E02, f[8]))));
    f[9] = fmaf(p.ri5, qp[5], fmaf(qs1, e2, fmaf(qs2, e1, fmaf(j3, E12, f[9]))));
}
// H (10): f[10..19] in the order xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz
__device__ __forceinline__ void quad_add_high(const QuadPair& p, const float* qp, float* f) {
    const float e0 = p.e0, e1 = p.e1, e2 = p.e2;
    const float Q00 = qp[0], Q11 = qp[1], Q22 = qp[2], Q01 = qp[3], Q02 = qp[4], Q12 = qp[5];
    const float E00 = e0 * e0, E11 = e1 * e1, E22 = e2 * e2, E01 = e0 * e1, E02 = e0 * e2, E12 = e1 * e2;
    const float s1 = -5.f * p.ri6, s2 = 35.f * p.ri6;
    const float es0 = s1 * e0, es1 = s1 * e1, es2 = s1 * e2;         // -5 r^-6 e
    const float qh0 = s2 * p.q0, qh1 = s2 * p.q1, qh2 = s2 * p.q2;   // 35 r^-6 Qe
    const float ur6 = p.u * p.ri6;
    const float c3 = -157.5f * ur6, t = 17.5f * ur6;
    const float ce0 = c3 * e0, ce1 = c3 * e1, ce2 = c3 * e2;          // -157.5 u r^-6 e
    const float V0 = fmaf(t, e0, s1 * p.q0), V1 = fmaf(t, e1, s1 * p.q1), V2 = fmaf(t, e2, s1 * p.q2);
    const float qc0 = qh0 + ce0, qc1 = qh1 + ce1, qc2 = qh2 + ce2;
    // (a, a, a): 3 (Q_aa es_a + qh_a E_aa + V_a) + E_aa ce_a
    f[10] = fmaf(3.f, fmaf(Q00, es0, fmaf(qh0, E00, V0)), fmaf(E00, ce0, f[10]));
    f[11] = fmaf(3.f, fmaf(Q11, es1, fmaf(qh1, E11, V1)), fmaf(E11, ce1, f[11]));
    f[12] = fmaf(3.f, fmaf(Q22, es2, fmaf(qh2, E22, V2)), fmaf(E22, ce2, f[12]));
    // (a, a, b): Q_aa es_b + 2 (Q_ab es_a + qh_a E_ab) + E_aa (qh_b + ce_b) + V_b
    f[13] = fmaf(2.f, fmaf(Q01, es0, qh0 * E01), fmaf(Q00, es1, fmaf(E00, qc1, f[13] + V1)));   // xxy
    f[14] = fmaf(2.f, fmaf(Q02, es0, qh0 * E02), fmaf(Q00, es2, fmaf(E00, qc2, f[14] + V2)));   // xxz
    f[15] = fmaf(2.f, fmaf(Q01, es1, qh1 * E01), fmaf(Q11, es0, fmaf(E11, qc0, f[15] + V0)));   // xyy = (y, y, x)
    f[16] = fmaf(2.f, fmaf(Q12, es1, qh1 * E12), fmaf(Q11, es2, fmaf(E11, qc2, f[16] + V2)));   // yyz
    f[17] = fmaf(2.f, fmaf(Q02, es2, qh2 * E02), fmaf(Q22, es0, fmaf(E22, qc0, f[17] + V0)));   // xzz = (z, z, x)
    f[18] = fmaf(2.f, fmaf(Q12, es2, qh2 * E12), fmaf(Q22, es1, fmaf(E22, qc1, f[18] + V1)));   // yzz = (z, z, y)
    // (x, y, z)
    f[19] = fmaf(Q01, es2, fmaf(Q02, es1, fmaf(Q12, es0, fmaf(qh0, E12, fmaf(qh1, E02, fmaf(E01, qc2, f[19]))))));
}

__device__ __forceinline__ void quad_expand_add(float dx, float dy, float dz, const float* qp, float eps2,
                                                float* f) {
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
    QuadPair p;
    quad_pair_setup(dx, dy, dz, __builtin_amdgcn_rsqf(r2), qp, p);
    quad_add_low(p, qp, f);
    quad_add_high(p, qp, f);
}

// The two halves of quad_expand_add, for two lanes sharing one pair:
// part 0 adds {a, phi, J} (f[0..9]), part 1 adds H (f[10..19]).
__device__ __forceinline__ void quad_expand_add_part(int part, float dx, float dy, float dz, const float* qp,
                                                     float eps2, float* f) {
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
    QuadPair p;
    quad_pair_setup(dx, dy, dz, __builtin_amdgcn_rsqf(r2), qp, p);
    if (part == 0)
        quad_add_low(p, qp, f);
    else
        quad_add_high(p, qp, f);
}

}  // namespace otoo_detail

struct otoo_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    otoo_tuning tune{1024, 8, 1, 0, 256, 2, 0};
    int num_cu = 0;
    size_t scratch_cap = 0;   // largest scratch buffer allowed (0: no cap)
    // bumped whenever a scratch buffer of the context (or of a network bound
    // to it) is allocated anew: a graph captured before names freed memory
    int64_t scratch_gen = 0;
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
    // and scratch for the item lists and chunk partials; cell corrections:
    // scratch for the partial expansions of groups that straddle work items;
    // both grown on demand
    void* sph_meta = nullptr;
    void* sph_buf = nullptr;
    size_t sph_bytes = 0;
    void* corr_buf = nullptr;
    size_t corr_bytes = 0;
    // device address of the no-allocation entry point's scratch array on
    // this context's device (shared by every context on that device)
    void* noalloc = nullptr;
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


