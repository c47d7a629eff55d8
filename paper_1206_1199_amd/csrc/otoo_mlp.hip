// Learned cell correction on gfx950.
//
// For every (group g, accepted cell c) pair a small network predicts a
// symmetric traceless tensor Qt_gc whose quadrupole-form field, applied
// through the group's local expansion, corrects the cell's monopole toward
// the cell's exact direct sum (the paper uses monopoles only and names higher
// multipoles without using them, Sec. 2).  A fixed skip term makes the
// network's tensor the textbook quadrupole plus a learned correction, and a
// gate on l/|d| limits the layers to near cells.
//
//   k_corr_box      bounding box of each group (the expansion centre), or
//                   k_corr_box_given from the boxes the walk returns
//   k_corr_net      per item of consecutive cell pairs: features, gated
//                   network (register-resident, v_mfma_f32_16x16x32_bf16)
//                   and the local expansion
//   k_corr_wave     the same items with given tensors or the textbook
//                   quadrupole
//   k_corr_merge    item sums of the groups that straddle items, in item
//                   order, and the rows of groups without cell pairs
//   k_corr_group    per group, LDS-staged: the network (alternative kernel)
//   k_group_geom    bounding-box centre and half-diagonal of each group
//   k_mlp_infer     Qt of every pair (for checks and external use)
//   k_mlp_forward_raw network outputs for given BF16 features
//   k_train_samples exact cell sums at target particles (FP64) and features
//   k_mlp_train     forward, loss through the expansion, backward (MFMA for
//                   every product), per-workgroup gradient partials
//   k_grad_reduce   fixed-order sum of the partials
//   k_adam          Adam on FP32 master weights, BF16 operand copies
#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <vector>

#include "otoo_internal.h"

using namespace otoo_detail;

namespace {

constexpr int NIN = 32, NFEAT = 12, NH = 64, NOUT = 6, NOUTP = 16, NO32 = 32;
// FP32 master parameters: W1 [NIN][NH], b1 [NH], W2 [NH][NH], b2 [NH], W3 [NH][NOUT], b3 [NOUT]
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NIN * NH;
constexpr int OFF_W2 = OFF_B1 + NH;
constexpr int OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH;
constexpr int OFF_B3 = OFF_W3 + NH * NOUT;
constexpr int NPARAM = OFF_B3 + NOUT;
// BF16 operand copies: out-major for the forward products, in-major for the backward ones
constexpr int OFFB_W1T = 0;                     // [NH][NIN]
constexpr int OFFB_W2T = OFFB_W1T + NH * NIN;   // [NH][NH]
constexpr int OFFB_W3T = OFFB_W2T + NH * NH;    // [NOUTP][NH], rows >= NOUT zero
constexpr int OFFB_W2 = OFFB_W3T + NOUTP * NH;  // [NH][NH]
constexpr int OFFB_W3 = OFFB_W2 + NH * NH;      // [NH][NO32], columns >= NOUT zero
constexpr int NBF = OFFB_W3 + NH * NO32;
constexpr int AUX = 12;          // per training sample: D xyz, delta xyz, target xyz, scale, weight, pad
constexpr float kFeatLimit = 8.f;
constexpr float GELU_C = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float GELU_A = 0.044715f;

static_assert(NPARAM == 6662, "parameter count");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // v_cvt_pk_bf16_f32: round to nearest even
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
__device__ __forceinline__ float bf_round(float f) { return bf2f(f2bf(f)); }

// The network's fixed skip term: output m (< NOUT) gets 3 s_m, where s is
// the BF16 normalised second-moment tensor (features kSkip0 ..), so that
// M l^2 P(3 s) = 3 S - tr(S) I, the textbook quadrupole; the layers add the
// learned correction to it.
constexpr int kSkip0 = NFEAT - NOUT;
__device__ __forceinline__ float skip_term(const uint16_t* xrow, int m) {
    return m < NOUT ? 3.f * bf2f(xrow[kSkip0 + m]) : 0.f;
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {  // 8 contiguous BF16, 16-byte aligned
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

__device__ __forceinline__ bf16x8 ld8s(const uint16_t* p, int stride) {  // 8 BF16 at a stride
    uint16_t v[8];
#pragma unroll
    for (int j = 0; j < 8; j++) v[j] = p[j * stride];
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// tanh-form GELU (Hendrycks & Gimpel): z/2 (1 + tanh(y)) = z sigmoid(2y),
// y = sqrt(2/pi) (z + 0.044715 z^3).  sigmoid(2y) = 1 / (1 + 2^(-2 y log2 e))
// and -2 y log2 e = z (G1 + G2 z^2): three VALU, one v_exp_f32, one add and
// one v_rcp_f32.
constexpr double kLog2e = 1.4426950408889634;
constexpr float GELU_G1 = (float)(-2.0 * 0.7978845608028654 * kLog2e);
constexpr float GELU_G2 = (float)(-2.0 * 0.7978845608028654 * kLog2e * 0.044715);
__device__ __forceinline__ float gelu_sig(float z) {
    const float e = __builtin_amdgcn_exp2f(z * fmaf(GELU_G2, z * z, GELU_G1));
    return __builtin_amdgcn_rcpf(1.f + e);
}
__device__ __forceinline__ float gelu(float z) { return z * gelu_sig(z); }
__device__ __forceinline__ float gelu_grad(float z) {
    const float s = gelu_sig(z);
    return s + 2.f * z * s * (1.f - s) * GELU_C * fmaf(3.f * GELU_A * z, z, 1.f);
}

// Features of a (group, cell) pair: d = COM - c_g, n = |d|:
// d/n, l/n, eps/n, h_g/n, S/(M l^2).  cm is the cell's stride-12 moment row.
__device__ __forceinline__ bool pair_features(float cx, float cy, float cz, float h, const float* cm, float eps,
                                              float f[NFEAT], float& scale) {
    const float dx = cm[0] - cx, dy = cm[1] - cy, dz = cm[2] - cz;
    const float n2 = dx * dx + dy * dy + dz * dz;
    const float inv = n2 > 0.f ? __builtin_amdgcn_rsqf(n2) : 0.f;
    const float M = cm[3], l = cm[4];
    const float sc = M * l * l;
    const float isc = sc > 0.f ? 1.f / sc : 0.f;
    f[0] = dx * inv;
    f[1] = dy * inv;
    f[2] = dz * inv;
    f[3] = l * inv;
    f[4] = eps * inv;
    f[5] = h * inv;
#pragma unroll
    for (int k = 0; k < 6; k++) f[6 + k] = cm[5 + k] * isc;
    scale = sc;
    bool ok = n2 > 0.f && sc > 0.f;
#pragma unroll
    for (int k = 0; k < NFEAT; k++) ok = ok && fabsf(f[k]) <= kFeatLimit;  // also false for NaN
    return ok;
}

// group containing pair p: the g with pair_off[g] <= p < pair_off[g+1]
__device__ __forceinline__ int group_of_pair(const int64_t* pair_off, int n_groups, int64_t p) {
    int lo = 0, hi = n_groups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pair_off[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Evaluate a correction expansion f[kCorrTerms] (about the expansion point)
// at offset delta: acceleration only.
__device__ __forceinline__ void expand_accel(const float* f, float dx, float dy, float dz, float& ax, float& ay,
                                             float& az) {
    const float* J = f + 4;
    const float* H = f + 10;
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz, xy = 2.f * dx * dy, xz = 2.f * dx * dz, yz = 2.f * dy * dz;
    ax = f[0] + J[0] * dx + J[3] * dy + J[4] * dz +
         0.5f * (H[0] * xx + H[5] * yy + H[7] * zz + H[3] * xy + H[4] * xz + H[9] * yz);
    ay = f[1] + J[3] * dx + J[1] * dy + J[5] * dz +
         0.5f * (H[3] * xx + H[1] * yy + H[8] * zz + H[5] * xy + H[9] * xz + H[6] * yz);
    az = f[2] + J[4] * dx + J[5] * dy + J[2] * dz +
         0.5f * (H[4] * xx + H[6] * yy + H[2] * zz + H[9] * xy + H[7] * xz + H[8] * yz);
}

// ---------------------------------------------------------------- geometry

__global__ __launch_bounds__(256) void k_group_geom(const float* __restrict__ pos, int32_t n,
                                                    const int32_t* __restrict__ group_off,
                                                    float4* __restrict__ geom, int32_t* err) {
    __shared__ float red[6][256];
    const int g = blockIdx.x, t = threadIdx.x;
    const int g0 = group_off[g];
    const int ng = group_off[g + 1] - g0;
    const bool ok = ng >= 1 && ng <= kBlock && g0 >= 0 && g0 + ng <= n;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (ok && t < ng)
        for (int k = 0; k < 3; k++) lo[k] = hi[k] = pos[3 * (g0 + t) + k];
    for (int k = 0; k < 3; k++) {
        red[k][t] = lo[k];
        red[3 + k][t] = hi[k];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 3; k++) {
                red[k][t] = fminf(red[k][t], red[k][t + w]);
                red[3 + k][t] = fmaxf(red[3 + k][t], red[3 + k][t + w]);
            }
        __syncthreads();
    }
    if (t == 0) {
        if (!ok) {
            atomicOr(err, kErrGroup);
            geom[g] = make_float4(0.f, 0.f, 0.f, 0.f);
            return;
        }
        const float ex = red[3][0] - red[0][0], ey = red[4][0] - red[1][0], ez = red[5][0] - red[2][0];
        geom[g] = make_float4(0.5f * (red[0][0] + red[3][0]), 0.5f * (red[1][0] + red[4][0]),
                              0.5f * (red[2][0] + red[5][0]), 0.5f * sqrtf(ex * ex + ey * ey + ez * ez));
    }
}

// ---------------------------------------------------------------- forward

struct NetLDS {
    alignas(16) uint16_t w1t[NH * NIN];
    alignas(16) uint16_t w2t[NH * NH];
    alignas(16) uint16_t w3t[NOUTP * NH];
    float b1[NH], b2[NH], b3[NOUTP];
};

__device__ void load_net(NetLDS& s, const uint16_t* __restrict__ wbf, const float* __restrict__ master) {
    const int t = threadIdx.x;
    for (int i = t; i < NH * NIN; i += blockDim.x) s.w1t[i] = wbf[OFFB_W1T + i];
    for (int i = t; i < NH * NH; i += blockDim.x) s.w2t[i] = wbf[OFFB_W2T + i];
    for (int i = t; i < NOUTP * NH; i += blockDim.x) s.w3t[i] = wbf[OFFB_W3T + i];
    for (int i = t; i < NH; i += blockDim.x) {
        s.b1[i] = master[OFF_B1 + i];
        s.b2[i] = master[OFF_B2 + i];
    }
    for (int i = t; i < NOUTP; i += blockDim.x) s.b3[i] = i < NOUT ? master[OFF_B3 + i] : 0.f;
}

// One wave computes rows [r0, r0+16) of Z = A W + b with A row-major in LDS
// (lda elements per row, K = 32 * KS) and W given out-major (Wt[n][k]).
// acc[nt][i] holds Z[r0 + q*4 + i][nt*16 + r16].
template <int KS, int NT>
__device__ __forceinline__ void wave_dense(const uint16_t* A, int lda, const uint16_t* Wt, int ldw, const float* bias,
                                           int r0, floatx4 acc[NT]) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, q = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
        const float b = bias[nt * 16 + r16];
        acc[nt] = floatx4{b, b, b, b};
    }
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
        const bf16x8 a = ld8(A + (r0 + r16) * lda + ks * 32 + q * 8);
#pragma unroll
        for (int nt = 0; nt < NT; nt++) acc[nt] = mfma(a, ld8(Wt + (nt * 16 + r16) * ldw + ks * 32 + q * 8), acc[nt]);
    }
}

struct InferArgs {
    int32_t n;
    int32_t n_groups;
    const int64_t* list_off;
    int64_t n_entries;
    const int32_t* list_idx;
    const int64_t* pair_off;
    int64_t n_pairs;
    int32_t n_cells;
    const float* cell_mom;
    float eps;
    const float4* geom;
    const uint16_t* wbf;
    const float* master;
    float gate;               // the layers run only where the BF16 feature l/n >= gate
    float* corr;
    int32_t* err;
};

__global__ __launch_bounds__(256) void k_mlp_infer(InferArgs a) {
    __shared__ NetLDS net;
    __shared__ __align__(16) uint16_t sX[64 * NIN];
    __shared__ __align__(16) uint16_t sH[64 * NH];
    __shared__ float sO[64 * NOUTP];
    __shared__ float sScale[64];
    __shared__ int sOk[64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, r16 = lane & 15, q = lane >> 4;
    load_net(net, a.wbf, a.master);
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * 64; base < a.n_pairs; base += (int64_t)gridDim.x * 64) {
        {
            const int row = t >> 2, part = t & 3;
            const int64_t p = base + row;
            float f[NFEAT];
            float sc = 0.f;
            bool ok = false;
            if (p < a.n_pairs) {
                const int g = group_of_pair(a.pair_off, a.n_groups, p);
                int64_t lb, le;
                list_range(a.list_off, a.n_entries, g, lb, le);
                const int64_t k = p - a.pair_off[g];
                if (k >= 0 && k < le - lb) {
                    const int64_t c = (int64_t)a.list_idx[lb + k] - a.n;
                    if (c >= 0 && c < a.n_cells) {
                        const float4 gm = a.geom[g];
                        ok = pair_features(gm.x, gm.y, gm.z, gm.w, a.cell_mom + 12 * c, a.eps, f, sc);
                    } else if (part == 0) {
                        atomicOr(a.err, kErrIndex);
                    }
                } else if (part == 0) {
                    atomicOr(a.err, kErrIndex);
                }
            }
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int fi = part * 8 + j;
                sX[row * NIN + fi] = f2bf(ok && fi < NFEAT ? f[fi < NFEAT ? fi : 0] : 0.f);
            }
            if (part == 0) {
                sScale[row] = sc;
                sOk[row] = ok;
            }
        }
        __syncthreads();
        const int r0 = 16 * w;
        floatx4 acc[4];
        wave_dense<1, 4>(sX, NIN, net.w1t, NIN, net.b1, r0, acc);
#pragma unroll
        for (int nt = 0; nt < 4; nt++)
#pragma unroll
            for (int i = 0; i < 4; i++) sH[(r0 + q * 4 + i) * NH + nt * 16 + r16] = f2bf(gelu(acc[nt][i]));
        __syncthreads();
        wave_dense<2, 4>(sH, NH, net.w2t, NH, net.b2, r0, acc);
        __syncthreads();
#pragma unroll
        for (int nt = 0; nt < 4; nt++)
#pragma unroll
            for (int i = 0; i < 4; i++) sH[(r0 + q * 4 + i) * NH + nt * 16 + r16] = f2bf(gelu(acc[nt][i]));
        __syncthreads();
        floatx4 o[1];
        wave_dense<2, 1>(sH, NH, net.w3t, NH, net.b3, r0, o);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint16_t* xr = sX + (r0 + q * 4 + i) * NIN;
            const bool on = bf2f(xr[3]) >= a.gate;
            sO[(r0 + q * 4 + i) * NOUTP + r16] = (on ? o[0][i] : 0.f) + skip_term(xr, r16);
        }
        __syncthreads();
        if (t < 64) {
            const int64_t p = base + t;
            if (p < a.n_pairs) {
                const float* ov = sO + t * NOUTP;
                const float tr = (ov[0] + ov[1] + ov[2]) * (1.f / 3.f);
                const float sc = sOk[t] ? sScale[t] : 0.f;
                float* out = a.corr + 6 * p;
                out[0] = (ov[0] - tr) * sc;
                out[1] = (ov[1] - tr) * sc;
                out[2] = (ov[2] - tr) * sc;
                out[3] = ov[3] * sc;
                out[4] = ov[4] * sc;
                out[5] = ov[5] * sc;
            }
        }
        __syncthreads();
    }
}

// Raw network outputs (no projection or scaling) for given BF16 features.
__global__ __launch_bounds__(256) void k_mlp_forward_raw(const uint16_t* __restrict__ X, int64_t rows,
                                                         const uint16_t* __restrict__ wbf,
                                                         const float* __restrict__ master, float* __restrict__ out) {
    __shared__ NetLDS net;
    __shared__ __align__(16) uint16_t sX[64 * NIN];
    __shared__ __align__(16) uint16_t sH[64 * NH];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, r16 = lane & 15, q = lane >> 4;
    load_net(net, wbf, master);
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * 64; base < rows; base += (int64_t)gridDim.x * 64) {
        for (int i = t; i < 64 * NIN; i += 256) {
            const int64_t r = base + i / NIN;
            sX[i] = r < rows ? X[r * NIN + i % NIN] : 0;
        }
        __syncthreads();
        const int r0 = 16 * w;
        floatx4 acc[4];
        wave_dense<1, 4>(sX, NIN, net.w1t, NIN, net.b1, r0, acc);
        for (int nt = 0; nt < 4; nt++)
            for (int i = 0; i < 4; i++) sH[(r0 + q * 4 + i) * NH + nt * 16 + r16] = f2bf(gelu(acc[nt][i]));
        __syncthreads();
        wave_dense<2, 4>(sH, NH, net.w2t, NH, net.b2, r0, acc);
        __syncthreads();
        for (int nt = 0; nt < 4; nt++)
            for (int i = 0; i < 4; i++) sH[(r0 + q * 4 + i) * NH + nt * 16 + r16] = f2bf(gelu(acc[nt][i]));
        __syncthreads();
        floatx4 o[1];
        wave_dense<2, 1>(sH, NH, net.w3t, NH, net.b3, r0, o);
        if (r16 < NOUT)
            for (int i = 0; i < 4; i++) {
                const int64_t r = base + r0 + q * 4 + i;
                if (r < rows) out[r * NOUT + r16] = o[0][i] + skip_term(sX + (r0 + q * 4 + i) * NIN, r16);
            }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- fused per-group correction

enum { kCorrPairs = 0, kCorrQuad = 1, kCorrMlp = 2 };

// Work items of the per-wave correction kernels: the cell pairs of all
// groups, in pair order (pair_off is their prefix sum), cut into items of
// `seg` pairs, taken statically by the waves.  A group whose pairs lie in
// one item writes its row of gcorr there; a group that straddles items leaves
// a partial expansion in each: in slot R of its first item, and in slot L of
// every later one.  k_corr_merge adds them in item order, so the result does
// not depend on the schedule.  seg is kCorrSeg, halved down to kCorrSegMin
// while there are fewer than four items per resident wave (small inputs
// would otherwise leave most waves of the chip without an item); it follows
// from the pair count and the kernels' occupancy alone.
constexpr int kCorrSeg = 1024;
constexpr int kCorrSegMin = 256;
struct CorrPlan {
    int64_t n_items;
    int32_t seg;     // pairs per item
    int32_t chunked; // two-pass learned correction: pair-parallel chunks (sparse pairs), else one group at a time
    float* part_l;   // [n_items][kCorrStride]: 20 terms, centre xyz, pad
    float* part_r;   // [n_items][kCorrStride]
    float4* box;     // [n_groups]: box centre xyz and half-diagonal, -1 for a malformed group
    uint4* crec;     // [n_cells][2]: the cells' records of the two-pass learned correction
};

struct CorrArgs {
    int32_t n;
    const float* pos;
    int32_t n_groups;
    const int32_t* group_off;
    const float* gbox;        // [n_groups][6] lo xyz, hi xyz, or NULL (found in pos)
    const int64_t* list_off;
    int64_t n_entries;
    const int32_t* list_idx;
    const int64_t* pair_off;
    int64_t n_pairs;
    int32_t n_cells;
    const float* cell_mom;
    int32_t stride;
    float eps;
    const float* corr;        // kCorrPairs: given tensors [n_pairs][6]
    const uint16_t* wbf;      // kCorrMlp: network
    const float* master;
    float gate;               // kCorrMlp: the layers run only where the BF16 feature l/n >= gate
    float* gcorr;             // [n_groups][kCorrStride]
    int32_t* err;
    CorrPlan plan;            // work items of the wave kernels
};

// The network through LDS, one workgroup per group (grid-stride over
// groups): the centre c_g of the group's bounding box, then the network's
// tensor for 128 (group, cell) pairs at a time on MFMA with the activations
// staged in LDS, and each pair's quadrupole-form field, Jacobian, Hessian
// and potential at c_g, summed in a fixed order into the group's local
// expansion.  No per-pair tensor touches HBM.  (The register-resident
// k_corr_net below is the default; this one is the reference variant.)
constexpr int kCorrRows = 128;   // pairs per chunk in the network variant (2 row tiles per wave)

// LDS of the network variant: the features (X) and hidden activations (H)
// of one chunk; the outputs (O) reuse X once layer 1 has read it, and the
// per-group reductions reuse the whole area between chunks.
union CorrScratch {
    struct {
        alignas(16) uint16_t x[kCorrRows * NIN];
        alignas(16) uint16_t h[kCorrRows * NH];
    } net;
    float o[kCorrRows * NOUTP];
    float red[kCorrTerms][256];
};

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_corr_group(CorrArgs a) {
    __shared__ NetLDS net;
    __shared__ CorrScratch scr;
    __shared__ float sScale[kCorrRows];
    __shared__ int sCell[kCorrRows];
    __shared__ float sSkip[kCorrRows * NOUT];   // skip term of each row; the layers' part is
    __shared__ int sOn[kCorrRows];              // kept only for rows the gate lets through
    uint16_t* sX = scr.net.x;
    uint16_t* sH = scr.net.h;
    float* sO = scr.o;
    auto& red = scr.red;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, r16 = lane & 15, q = lane >> 4;
    const float eps2 = a.eps * a.eps;
    load_net(net, a.wbf, a.master);
    for (int g = blockIdx.x; g < a.n_groups; g += gridDim.x) {
        const int g0 = a.group_off[g];
        const int ng = a.group_off[g + 1] - g0;
        const bool ok = ng >= 1 && ng <= kBlock && g0 >= 0 && g0 + ng <= a.n;
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (ok && t < ng)
            for (int k = 0; k < 3; k++) lo[k] = hi[k] = a.pos[3 * (g0 + t) + k];
        __syncthreads();   // the previous group's reduction has been read
        for (int k = 0; k < 3; k++) {
            red[k][t] = lo[k];
            red[3 + k][t] = hi[k];
        }
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if (t < s2)
                for (int k = 0; k < 3; k++) {
                    red[k][t] = fminf(red[k][t], red[k][t + s2]);
                    red[3 + k][t] = fmaxf(red[3 + k][t], red[3 + k][t + s2]);
                }
            __syncthreads();
        }
        const float cx = 0.5f * (red[0][0] + red[3][0]);
        const float cy = 0.5f * (red[1][0] + red[4][0]);
        const float cz = 0.5f * (red[2][0] + red[5][0]);
        const float ex = red[3][0] - red[0][0], ey = red[4][0] - red[1][0], ez = red[5][0] - red[2][0];
        const float h = 0.5f * sqrtf(ex * ex + ey * ey + ez * ez);
        __syncthreads();
        float f[kCorrTerms];
#pragma unroll
        for (int k = 0; k < kCorrTerms; k++) f[k] = 0.f;
        int64_t lb = 0, le = 0, p0 = 0, nce = 0;
        if (ok) {
            list_range(a.list_off, a.n_entries, g, lb, le);
            p0 = clamp64(a.pair_off[g], 0, a.n_pairs);
            const int64_t p1 = clamp64(a.pair_off[g + 1], p0, a.n_pairs);
            nce = (p1 - p0) < (le - lb) ? (p1 - p0) : (le - lb);
        } else if (t == 0) {
            atomicOr(a.err, kErrGroup);
        }
        for (int64_t base = 0; base < nce; base += kCorrRows) {
            if (t >= kCorrRows) {  // zero the padding columns (X shares its space with O and the reductions)
                const int row = t - kCorrRows;
                for (int j = NFEAT; j < NIN; j++) sX[row * NIN + j] = 0;
            } else {               // features: one thread per row
                const int64_t k = base + t;
                float fe[NFEAT];
                float sc = 0.f;
                bool fok = false;
                int64_t c = -1;
                if (k < nce) {
                    c = (int64_t)a.list_idx[lb + k] - a.n;
                    if (c >= 0 && c < a.n_cells) {
                        fok = pair_features(cx, cy, cz, h, a.cell_mom + 12 * c, a.eps, fe, sc);
                    } else {
                        atomicOr(a.err, kErrIndex);
                        c = -1;
                    }
                }
#pragma unroll
                for (int j = 0; j < NFEAT; j++) sX[t * NIN + j] = f2bf(fok ? fe[j] : 0.f);
#pragma unroll
                for (int m = 0; m < NOUT; m++) sSkip[t * NOUT + m] = fok ? 3.f * bf_round(fe[kSkip0 + m]) : 0.f;
                sOn[t] = fok && bf_round(fe[3]) >= a.gate;
                sScale[t] = fok ? sc : 0.f;
                sCell[t] = (int)c;
            }
            __syncthreads();
            floatx4 acc[4];
#pragma unroll
            for (int mt = 0; mt < 2; mt++) {
                const int r0 = 32 * w + 16 * mt;
                wave_dense<1, 4>(sX, NIN, net.w1t, NIN, net.b1, r0, acc);
#pragma unroll
                for (int nt = 0; nt < 4; nt++)
#pragma unroll
                    for (int i = 0; i < 4; i++)
                        sH[(r0 + q * 4 + i) * NH + nt * 16 + r16] = f2bf(gelu(acc[nt][i]));
            }
            __syncthreads();
            floatx4 acc2[2][4];
#pragma unroll
            for (int mt = 0; mt < 2; mt++) wave_dense<2, 4>(sH, NH, net.w2t, NH, net.b2, 32 * w + 16 * mt, acc2[mt]);
            __syncthreads();
#pragma unroll
            for (int mt = 0; mt < 2; mt++) {
                const int r0 = 32 * w + 16 * mt;
#pragma unroll
                for (int nt = 0; nt < 4; nt++)
#pragma unroll
                    for (int i = 0; i < 4; i++)
                        sH[(r0 + q * 4 + i) * NH + nt * 16 + r16] = f2bf(gelu(acc2[mt][nt][i]));
            }
            __syncthreads();
#pragma unroll
            for (int mt = 0; mt < 2; mt++) {
                const int r0 = 32 * w + 16 * mt;
                floatx4 o[1];
                wave_dense<2, 1>(sH, NH, net.w3t, NH, net.b3, r0, o);
#pragma unroll
                for (int i = 0; i < 4; i++) sO[(r0 + q * 4 + i) * NOUTP + r16] = o[0][i];
            }
            __syncthreads();
            {   // two threads per row share the expansion: {a, phi, J} and H
                const int row = t >> 1, part = t & 1;
                if (base + row < nce && sCell[row] >= 0 && sScale[row] > 0.f) {
                    const float* on = sO + row * NOUTP;
                    const bool lay = sOn[row] != 0;
                    float ov[NOUT];
#pragma unroll
                    for (int m = 0; m < NOUT; m++) ov[m] = (lay ? on[m] : 0.f) + sSkip[row * NOUT + m];
                    const float tr = (ov[0] + ov[1] + ov[2]) * (1.f / 3.f);
                    const float sc = sScale[row];
                    const float Q[6] = {(ov[0] - tr) * sc, (ov[1] - tr) * sc, (ov[2] - tr) * sc,
                                        ov[3] * sc,        ov[4] * sc,        ov[5] * sc};
                    const float* cm = a.cell_mom + 12 * (int64_t)sCell[row];
                    quad_expand_add_part(part, cx - cm[0], cy - cm[1], cz - cm[2], Q, eps2, f);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < kCorrTerms; k++) red[k][t] = f[k];
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if (t < s2)
                for (int k = 0; k < kCorrTerms; k++) red[k][t] += red[k][t + s2];
            __syncthreads();
        }
        float* out = a.gcorr + (int64_t)kCorrStride * g;
        if (t < kCorrTerms) out[t] = red[t][0];
        if (t == kCorrTerms) out[kCorrTerms] = cx;
        if (t == kCorrTerms + 1) out[kCorrTerms + 1] = cy;
        if (t == kCorrTerms + 2) out[kCorrTerms + 2] = cz;
        if (t == kCorrTerms + 3) out[kCorrTerms + 3] = 0.f;
    }
}

// Register-resident network variant of the learned correction.  Each wave
// evaluates the network for 64 pairs at a time with the activations kept in
// registers: the products are written transposed (weights are the MFMA's A
// operand, held in registers for the whole kernel; pairs are the N
// dimension), so the output layout of one layer is the B layout of the next
// once the next layer's K index is permuted to match:  K slot q*8 + j of
// step ks holds hidden unit (2 ks + j/4)*16 + q*4 + j%4.  Features go in and
// outputs come out through lane shuffles; no LDS and no workgroup barrier
// inside the network.
__device__ __forceinline__ bf16x8 pack8(const floatx4& a, const floatx4& b) {
    bf16x8 r;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        r[i] = (__bf16)gelu(a[i]);
        r[4 + i] = (__bf16)gelu(b[i]);
    }
    return r;
}

// 8 BF16 of row `row` of an out-major weight copy: units (2ks)*16 + q*4 .. +3
// then (2ks+1)*16 + q*4 .. +3 (the permuted K order above)
__device__ __forceinline__ bf16x8 ld_perm(const uint16_t* W, int ld, int row, int ks, int q) {
    const uint2 lo = *reinterpret_cast<const uint2*>(W + row * ld + (2 * ks) * 16 + q * 4);
    const uint2 hi = *reinterpret_cast<const uint2*>(W + row * ld + (2 * ks + 1) * 16 + q * 4);
    const uint4 v = make_uint4(lo.x, lo.y, hi.x, hi.y);
    return __builtin_bit_cast(bf16x8, v);
}

// Traceless tensor of a pair from its outputs o (skip term included), times
// the pair's scale M l^2, added to the group's expansion at offset d.
__device__ __forceinline__ void expand_outputs(const float o[NOUT], float sc, float dx, float dy, float dz,
                                               float eps2, float* f) {
    const float tr = (o[0] + o[1] + o[2]) * (1.f / 3.f);
    const float Q[6] = {(o[0] - tr) * sc, (o[1] - tr) * sc, (o[2] - tr) * sc, o[3] * sc, o[4] * sc, o[5] * sc};
    quad_expand_add(dx, dy, dz, Q, eps2, f);
}

// Wave-level reductions on the VALU through DPP lane moves, in a fixed
// order, the result the same in every lane: within each row of 16 lanes the
// partner lanes xor 1 and xor 2 (quad permutes), then the half-row and row
// mirrors; the four row totals are then combined through the broadcasts of
// lanes 15 and 31 into rows 1 and 3, and 2 and 3, and lane 63's value is
// read into a scalar register.  `id` is the operation's identity, taken by
// the rows a broadcast does not write.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float old, float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, x),
                                                                  CTRL, ROW_MASK, 0xF, false));
}
template <typename Op>
__device__ __forceinline__ float wave_reduce(float v, float id, Op op) {
    v = op(v, dpp_move<0xB1, 0xF>(id, v));    // quad_perm [1, 0, 3, 2]: lane xor 1
    v = op(v, dpp_move<0x4E, 0xF>(id, v));    // quad_perm [2, 3, 0, 1]: lane xor 2
    v = op(v, dpp_move<0x141, 0xF>(id, v));   // row_half_mirror: the other quad of each half-row
    v = op(v, dpp_move<0x140, 0xF>(id, v));   // row_mirror: the other half of each row
    v = op(v, dpp_move<0x142, 0xA>(id, v));   // row_bcast:15 into rows 1 and 3
    v = op(v, dpp_move<0x143, 0xC>(id, v));   // row_bcast:31 into rows 2 and 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ float wave_sum(float v) {
    return wave_reduce(v, 0.f, [](float x, float y) { return x + y; });
}
__device__ __forceinline__ float wave_min(float v) {
    return wave_reduce(v, INFINITY, [](float x, float y) { return fminf(x, y); });
}
__device__ __forceinline__ float wave_max(float v) {
    return wave_reduce(v, -INFINITY, [](float x, float y) { return fmaxf(x, y); });
}

// Centre and half-diagonal of the box [lo, hi].
__device__ __forceinline__ void box_centre(const float lo[3], const float hi[3], float& cx, float& cy, float& cz,
                                           float& h) {
    cx = 0.5f * (lo[0] + hi[0]);
    cy = 0.5f * (lo[1] + hi[1]);
    cz = 0.5f * (lo[2] + hi[2]);
    const float ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    h = 0.5f * sqrtf(ex * ex + ey * ey + ez * ez);
}

// Geometry of group g for one wave: centre and half-diagonal of the
// bounding box of its particles; false for a malformed group.
__device__ __forceinline__ bool wave_group_box(const CorrArgs& a, int g, int lane, float& cx, float& cy, float& cz,
                                               float& h) {
    const int g0 = a.group_off[g];
    const int ng = a.group_off[g + 1] - g0;
    const bool ok = ng >= 1 && ng <= kBlock && g0 >= 0 && g0 + ng <= a.n;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (ok)
        for (int p = lane; p < ng; p += 64)
            for (int k = 0; k < 3; k++) {
                const float x = a.pos[3 * (g0 + p) + k];
                lo[k] = fminf(lo[k], x);
                hi[k] = fmaxf(hi[k], x);
            }
    for (int k = 0; k < 3; k++) {
        lo[k] = wave_min(lo[k]);
        hi[k] = wave_max(hi[k]);
    }
    box_centre(lo, hi, cx, cy, cz, h);
    return ok;
}

// Each group's bounding box once, for every item that holds pairs of it:
// one wave per group.
__global__ __launch_bounds__(256) void k_corr_box(CorrArgs a) {
    const int lane = threadIdx.x & 63;
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= a.n_groups) return;   // whole waves: g is the same for the wave's lanes
    float cx, cy, cz, h;
    const bool ok = wave_group_box(a, g, lane, cx, cy, cz, h);
    if (lane == 0) {
        a.plan.box[g] = make_float4(cx, cy, cz, ok ? h : -1.f);
        if (!ok) atomicOr(a.err, kErrGroup);
    }
}

// The same from the boxes the walk returns: one thread per group.
__global__ __launch_bounds__(256) void k_corr_box_given(CorrArgs a) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= a.n_groups) return;
    const int g0 = a.group_off[g];
    const int ng = a.group_off[g + 1] - g0;
    const bool ok = ng >= 1 && ng <= kBlock && g0 >= 0 && g0 + ng <= a.n;
    const float lo[3] = {a.gbox[6 * g], a.gbox[6 * g + 1], a.gbox[6 * g + 2]};
    const float hi[3] = {a.gbox[6 * g + 3], a.gbox[6 * g + 4], a.gbox[6 * g + 5]};
    float cx, cy, cz, h;
    box_centre(lo, hi, cx, cy, cz, h);
    a.plan.box[g] = make_float4(cx, cy, cz, ok ? h : -1.f);
    if (!ok) atomicOr(a.err, kErrGroup);
}

// Group g's box from k_corr_box; false for a malformed group.
__device__ __forceinline__ bool group_box(const CorrArgs& a, int g, float& cx, float& cy, float& cz, float& h) {
    const float4 b = a.plan.box[g];
    cx = b.x;
    cy = b.y;
    cz = b.z;
    h = b.w;
    return b.w >= 0.f;
}

// Sum the lanes' expansion terms into a partial slot (lane 0).
__device__ __forceinline__ void wave_store_part(float* out, int lane, float f[kCorrTerms], float cx, float cy,
                                                float cz) {
#pragma unroll
    for (int k = 0; k < kCorrTerms; k++) f[k] = wave_sum(f[k]);
    static_assert(kCorrTerms == 20 && kCorrStride == 24, "row layout");
    if (lane == 0) {   // rows are 96 bytes: six 16-byte stores
        float4* o4 = reinterpret_cast<float4*>(out);
#pragma unroll
        for (int k = 0; k < 5; k++) o4[k] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
        o4[5] = make_float4(cx, cy, cz, 0.f);
    }
}

// Pair range of group g in pair order, clamped to [0, n_pairs] and made
// non-decreasing from its start, the same way in every kernel.
__device__ __forceinline__ void pair_range(const CorrArgs& a, int g, int64_t& p0, int64_t& p1) {
    p0 = clamp64(a.pair_off[g], 0, a.n_pairs);
    p1 = clamp64(a.pair_off[g + 1], p0, a.n_pairs);
}

// The group holding pair q: the last g with pair_off[g] <= q (binary search,
// wave-uniform).
__device__ __forceinline__ int group_of_pair(const CorrArgs& a, int64_t q) {
    int lo = 0, hi = a.n_groups;   // pair_off[lo] <= q is assumed, the answer is in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (clamp64(a.pair_off[mid], 0, a.n_pairs) <= q)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Where the expansion of group g over pairs [q0, q1) of item `it` goes.
__device__ __forceinline__ float* corr_target(const CorrArgs& a, int g, int64_t it, int64_t p0, int64_t p1,
                                              int64_t q0, int64_t q1) {
    if (p0 >= q0 && p1 <= q1) return a.gcorr + (int64_t)kCorrStride * g;   // whole group
    if (p0 < q0) return a.plan.part_l + (int64_t)kCorrStride * it;         // continues from an earlier item
    return a.plan.part_r + (int64_t)kCorrStride * it;                        // starts here, continues later
}

// The groups of the pairs of chunk [c0, c1) (c1 - c0 <= 64): map[j] is the
// group of pair c0 + j.  The wave's lanes take 64 consecutive groups from
// gcur (wave-uniform, the group of pair c0) at a time, and each writes its
// group into map[] at the chunk positions of its pairs; groups without pairs
// in the chunk write nothing.  On return gcur is the group of pair c1 - 1,
// from which the next chunk's groups start.
__device__ __forceinline__ void chunk_groups(const CorrArgs& a, int lane, int64_t c0, int64_t c1, int& gcur,
                                             int* map) {
    map[lane] = gcur;   // a valid group for every slot (malformed pair offsets leave slots unwritten)
    __builtin_amdgcn_wave_barrier();
    for (;;) {
        const int g = gcur + lane;
        int64_t p0 = a.n_pairs, p1 = a.n_pairs;
        if (g < a.n_groups) pair_range(a, g, p0, p1);
        const int64_t lo = p0 > c0 ? p0 : c0, hi = p1 < c1 ? p1 : c1;
        for (int64_t p = lo; p < hi; p++) map[p - c0] = g;
        // the run covers the chunk once its last group ends at or after c1
        const int64_t last = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)p1 >> 32), 63) << 32) |
                                       (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)p1, 63));
        if (last >= c1 || gcur + 64 >= a.n_groups) break;
        gcur += 64;
    }
    __builtin_amdgcn_wave_barrier();
    gcur = __builtin_amdgcn_readfirstlane(map[c1 - 1 - c0]);
}

// Rows of the groups that straddle items (partials added in item order) and
// of the groups without cell pairs (zero terms, their box centre): one
// thread per group.
__global__ __launch_bounds__(256) void k_corr_merge(CorrArgs a) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < a.n_groups; g += gridDim.x * blockDim.x) {
        int64_t p0, p1;
        pair_range(a, g, p0, p1);
        float* row = a.gcorr + (int64_t)kCorrStride * g;
        if (p1 == p0) {
            const float4 b = a.plan.box[g];
            for (int k = 0; k < kCorrTerms; k++) row[k] = 0.f;
            row[kCorrTerms] = b.x;
            row[kCorrTerms + 1] = b.y;
            row[kCorrTerms + 2] = b.z;
            row[kCorrTerms + 3] = 0.f;
            continue;
        }
        const int64_t i0 = p0 / a.plan.seg, i1 = (p1 - 1) / a.plan.seg;
        if (i0 == i1) continue;   // written whole by its item
        const float* r = a.plan.part_r + (int64_t)kCorrStride * i0;
        float v[kCorrTerms];
        for (int k = 0; k < kCorrTerms; k++) v[k] = r[k];
        for (int64_t i = i0 + 1; i <= i1; i++) {
            const float* l = a.plan.part_l + (int64_t)kCorrStride * i;
            for (int k = 0; k < kCorrTerms; k++) v[k] += l[k];
        }
        for (int k = 0; k < kCorrTerms; k++) row[k] = v[k];
        for (int k = 0; k < 4; k++) row[kCorrTerms + k] = r[kCorrTerms + k];
    }
}

// Static, XCD-aware assignment of work items to the waves of a grid of
// 256-thread workgroups.  The dispatcher deals workgroups to the chip's
// eight XCDs in turn (workgroup b to XCD b mod 8), and each XCD has its own
// L2; so each XCD takes a contiguous eighth of the items, and the waves that
// share an L2 work on neighbouring items, whose groups gather the same
// cells.  Within an XCD the waves take its items in turn.  Every item goes
// to exactly one wave for any grid size.
struct ItemRange {
    int64_t first, end, step;
};
__device__ __forceinline__ ItemRange xcd_items(int64_t n_items) {
    const int nx = gridDim.x < 8 ? (int)gridDim.x : 8;
    const int b = blockIdx.x, x = b % nx, j = b / nx;
    const int nblk = ((int)gridDim.x - x + nx - 1) / nx;   // workgroups of this XCD
    const int64_t per = (n_items + nx - 1) / nx;
    const int64_t lo = (int64_t)x * per < n_items ? (int64_t)x * per : n_items;
    const int64_t hi = lo + per < n_items ? lo + per : n_items;
    const int64_t first = lo + (int64_t)j * 4 + (threadIdx.x >> 6);
    return ItemRange{__builtin_amdgcn_readfirstlane(first), hi, (int64_t)nblk * 4};
}

// One (group, cell) pair of the given or textbook kind as gathered: the
// cell's COM and either the given tensor or the cell's second moments S
// (raw, so that a prefetched pair costs no arithmetic until it is used).  A
// position past the item, or an entry that is not a cell (flagged), is not
// valid.
struct CorrCell {
    float com[3];
    float t[6];
    bool valid;
};

// Branch-free gathers for the software pipeline below: every load reads a
// clamped, in-range address, and whether the pair counts is decided from
// positions alone (pv) or once the loaded value is used, so that a load
// issued ahead is not waited for until its pair is summed.
struct CorrEntry {
    int64_t e;   // list entry (loaded)
    bool pv;     // the position is a pair of this item
};

// The list entry at pair position p (k = p - p0 of the group's list, whose
// last position is kmax >= 0).
__device__ __forceinline__ CorrEntry corr_list_entry(const CorrArgs& a, int64_t p, int64_t a1, int64_t p0, int64_t lb,
                                                     int64_t kmax) {
    const int64_t k = p - p0;   // the group's cells lead its list
    return CorrEntry{(int64_t)a.list_idx[lb + (k < kmax ? k : kmax)], p < a1 && k <= kmax};
}

// The pair's cell record; an entry that is not a cell makes the pair invalid
// and sets bad (cell 0 stands in for its loads).  pmax is the item's last
// pair position (for the given tensors).
template <int KIND>
__device__ __forceinline__ CorrCell load_corr_cell(const CorrArgs& a, CorrEntry en, int64_t p, int64_t pmax, bool& bad) {
    const int64_t c = en.e - a.n;
    const bool ok = en.pv && c >= 0 && c < a.n_cells;
    bad |= en.pv && !ok;
    const float* cm = a.cell_mom + (int64_t)a.stride * (ok ? c : 0);
    const float* src = KIND == kCorrPairs ? a.corr + 6 * (p < pmax ? p : pmax) : cm + 5;
    CorrCell r;
    for (int m = 0; m < 3; m++) r.com[m] = cm[m];
    for (int m = 0; m < 6; m++) r.t[m] = src[m];
    r.valid = ok;
    return r;
}

// The tensor of a gathered pair: given, or 3 S - tr(S) I.
template <int KIND>
__device__ __forceinline__ void corr_tensor(const CorrCell& cc, float Q[6]) {
    if (KIND == kCorrPairs) {
        for (int m = 0; m < 6; m++) Q[m] = cc.t[m];
    } else {
        const float tr = cc.t[0] + cc.t[1] + cc.t[2];
        Q[0] = 3.f * cc.t[0] - tr;
        Q[1] = 3.f * cc.t[1] - tr;
        Q[2] = 3.f * cc.t[2] - tr;
        Q[3] = 3.f * cc.t[3];
        Q[4] = 3.f * cc.t[4];
        Q[5] = 3.f * cc.t[5];
    }
}

// Given or textbook tensors, one wave per item (items wave w, w + W, ...):
// for each group with pairs in the item, its box, then its pairs of the item;
// no workgroup barrier; the box and the expansion terms are reduced with
// lane shuffles in a fixed order.
template <int KIND>
__global__ __launch_bounds__(256) void k_corr_wave(CorrArgs a) {
    const int lane = threadIdx.x & 63;
    const float eps2 = a.eps * a.eps;
    const ItemRange ir = xcd_items(a.plan.n_items);
    for (int64_t it = ir.first; it < ir.end; it += ir.step) {
        const int64_t q0 = it * a.plan.seg;
        const int64_t q1 = q0 + a.plan.seg < a.n_pairs ? q0 + a.plan.seg : a.n_pairs;
        for (int g = group_of_pair(a, q0); g < a.n_groups; g++) {
            int64_t p0, p1;
            pair_range(a, g, p0, p1);
            if (p0 >= q1) break;
            const int64_t a0 = p0 > q0 ? p0 : q0, a1 = p1 < q1 ? p1 : q1;
            if (a1 <= a0) continue;   // no pairs of this group in the item
            float cx, cy, cz, h;
            const bool ok = group_box(a, g, cx, cy, cz, h);
            float f[kCorrTerms];
#pragma unroll
            for (int k = 0; k < kCorrTerms; k++) f[k] = 0.f;
            int64_t lb, le;
            list_range(a.list_off, a.n_entries, g, lb, le);
            if (ok && le > lb && a.n_cells > 0) {
                // software pipeline: while a pair is summed, the next pair's cell record and the
                // list entry of the pair after it are in flight (a lane's loads retire in order,
                // and nothing waits for them before its pair is summed)
                const int64_t kmax = le - lb - 1, pmax = a1 - 1;
                const int64_t p_first = a0 + lane;
                bool bad = false;
                CorrCell cur = load_corr_cell<KIND>(a, corr_list_entry(a, p_first, a1, p0, lb, kmax), p_first, pmax, bad);
                CorrEntry e_next = corr_list_entry(a, p_first + 64, a1, p0, lb, kmax);
                for (int64_t p = p_first; p < a1; p += 64) {
                    const CorrEntry e_after = corr_list_entry(a, p + 128, a1, p0, lb, kmax);
                    const CorrCell nxt = load_corr_cell<KIND>(a, e_next, p + 64, pmax, bad);
                    // keeps these loads ahead of the sum below: the compiler would otherwise move
                    // them into the next iteration, next to their use, and wait for them there
                    __asm__ volatile("" ::: "memory");
                    float Q[6];
                    corr_tensor<KIND>(cur, Q);
                    const float w = cur.valid ? 1.f : 0.f;   // an invalid pair adds zero
#pragma unroll
                    for (int m = 0; m < 6; m++) Q[m] *= w;
                    quad_expand_add(cx - cur.com[0], cy - cur.com[1], cz - cur.com[2], Q, eps2, f);
                    cur = nxt;
                    e_next = e_after;
                }
                if (bad) atomicOr(a.err, kErrIndex);
            }   // a malformed group was flagged by k_corr_box
            wave_store_part(corr_target(a, g, it, p0, p1, q0, q1), lane, f, cx, cy, cz);
        }
    }
}

// Register-resident network, one wave per item (the items of k_corr_wave).
// For each group with pairs in the item the wave walks those cell entries 64
// at a time: a pair the gate keeps out gets the skip term alone (the textbook
// quadrupole) at once; a gated pair is appended to the wave's LDS queue
// (ballot order).  Whenever 64 are queued, and once at the end of the
// group's part of the item, the wave runs the network on them: weights are the
// MFMA's A operand, held in registers for the whole kernel; the 64 pairs are
// the N dimension in four steps of 16, and each layer's output layout is
// the next layer's B layout once the K index is permuted (K slot q*8 + j of
// step ks holds hidden unit (2 ks + j/4)*16 + q*4 + j%4).  No workgroup
// barrier after the weights are loaded.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_corr_net(CorrArgs a) {
    constexpr int kQueue = 128;
    __shared__ float sb[NH + NH + NOUTP];
    __shared__ int32_t sPend[4][kQueue];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, r16 = lane & 15, q = lane >> 4;
    int32_t* pendq = sPend[w];
    const float eps2 = a.eps * a.eps;
    for (int i = t; i < NH; i += 256) {
        sb[i] = a.master[OFF_B1 + i];
        sb[NH + i] = a.master[OFF_B2 + i];
    }
    if (t < NOUTP) sb[2 * NH + t] = t < NOUT ? a.master[OFF_B3 + t] : 0.f;
    bf16x8 w1a[4], w2a[4][2], w3a[2];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        w1a[mt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(a.wbf + OFFB_W1T + (mt * 16 + r16) * NIN + q * 8));
#pragma unroll
        for (int ks = 0; ks < 2; ks++) w2a[mt][ks] = ld_perm(a.wbf + OFFB_W2T, NH, mt * 16 + r16, ks, q);
    }
#pragma unroll
    for (int ks = 0; ks < 2; ks++) w3a[ks] = ld_perm(a.wbf + OFFB_W3T, NH, r16, ks, q);
    __syncthreads();
    const ItemRange ir = xcd_items(a.plan.n_items);
    for (int64_t it = ir.first; it < ir.end; it += ir.step)
    for (int g = group_of_pair(a, it * a.plan.seg); g < a.n_groups; g++) {
        const int64_t q0 = it * a.plan.seg;
        const int64_t q1 = q0 + a.plan.seg < a.n_pairs ? q0 + a.plan.seg : a.n_pairs;
        int64_t p0, p1;
        pair_range(a, g, p0, p1);
        if (p0 >= q1) break;
        const int64_t a0 = p0 > q0 ? p0 : q0, a1 = p1 < q1 ? p1 : q1;
        if (a1 <= a0) continue;   // no pairs of this group in the item
        float cx, cy, cz, h;
        const bool ok = group_box(a, g, cx, cy, cz, h);
        float f[kCorrTerms];
#pragma unroll
        for (int k = 0; k < kCorrTerms; k++) f[k] = 0.f;
        int64_t lb = 0, k0 = 0, k1 = 0;   // this item's part of the group's list: positions [k0, k1)
        if (ok) {
            int64_t le;
            list_range(a.list_off, a.n_entries, g, lb, le);
            k0 = a0 - p0;
            k1 = (a1 - p0) < (le - lb) ? (a1 - p0) : (le - lb);
            if (k1 > INT32_MAX) {   // queue slots hold 32-bit list positions
                k1 = INT32_MAX;
                if (lane == 0) atomicOr(a.err, kErrCapacity);
            }
        }   // a malformed group was flagged by k_corr_box
        // the network on queue slots [0, cnt): features, layers, skip term, expansion
        auto run_net = [&](int cnt) {
            const bool has = lane < cnt;
            float fe[NFEAT], sc = 0.f, mx = 0.f, my = 0.f, mz = 0.f;
#pragma unroll
            for (int j = 0; j < NFEAT; j++) fe[j] = 0.f;
            if (has) {
                const int64_t c = (int64_t)a.list_idx[lb + pendq[lane]] - a.n;   // checked when queued
                const float* cm = a.cell_mom + 12 * c;
                pair_features(cx, cy, cz, h, cm, a.eps, fe, sc);
                mx = cm[0];
                my = cm[1];
                mz = cm[2];
            }
            float ov[NOUT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int tau = 0; tau < 4; tau++) {
                const int src = tau * 16 + r16;
                float v[NFEAT];
#pragma unroll
                for (int j = 0; j < NFEAT; j++) v[j] = __shfl(fe[j], src);
                bf16x8 xb;
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    const float x = q == 0 ? v[j] : (q == 1 && j < 4 ? v[8 + j] : 0.f);
                    xb[j] = (__bf16)x;
                }
                floatx4 acc[4];
#pragma unroll
                for (int mt = 0; mt < 4; mt++) {
                    const float4 bb = *reinterpret_cast<const float4*>(sb + mt * 16 + q * 4);
                    acc[mt] = mfma(w1a[mt], xb, floatx4{bb.x, bb.y, bb.z, bb.w});
                }
                const bf16x8 h0 = pack8(acc[0], acc[1]), h1 = pack8(acc[2], acc[3]);
#pragma unroll
                for (int mt = 0; mt < 4; mt++) {
                    const float4 bb = *reinterpret_cast<const float4*>(sb + NH + mt * 16 + q * 4);
                    acc[mt] = mfma(w2a[mt][0], h0, floatx4{bb.x, bb.y, bb.z, bb.w});
                    acc[mt] = mfma(w2a[mt][1], h1, acc[mt]);
                }
                const bf16x8 g0b = pack8(acc[0], acc[1]), g1b = pack8(acc[2], acc[3]);
                const float4 b3 = *reinterpret_cast<const float4*>(sb + 2 * NH + q * 4);
                floatx4 o = mfma(w3a[0], g0b, floatx4{b3.x, b3.y, b3.z, b3.w});
                o = mfma(w3a[1], g1b, o);
                // outputs 0..3 of pair (tau, r16) sit in lane r16, outputs 4, 5 in lane r16 + 16
                float sv[NOUT];
#pragma unroll
                for (int i = 0; i < 4; i++) sv[i] = __shfl(o[i], r16);
                sv[4] = __shfl(o[0], r16 + 16);
                sv[5] = __shfl(o[1], r16 + 16);
                if (q == tau)
#pragma unroll
                    for (int i = 0; i < NOUT; i++) ov[i] = sv[i];
            }
            if (has && sc > 0.f) {
#pragma unroll
                for (int m = 0; m < NOUT; m++) ov[m] += 3.f * bf_round(fe[kSkip0 + m]);
                expand_outputs(ov, sc, cx - mx, cy - my, cz - mz, eps2, f);
            }
        };
        int pend = 0;   // uniform within the wave
        for (int64_t base = k0; base < k1; base += 64) {
            const int64_t k = base + lane;
            bool gated = false;
            if (k < k1) {
                const int64_t c = (int64_t)a.list_idx[lb + k] - a.n;
                if (c >= 0 && c < a.n_cells) {
                    const float* cm = a.cell_mom + 12 * c;
                    float fe[NFEAT], sc;
                    if (pair_features(cx, cy, cz, h, cm, a.eps, fe, sc)) {
                        if (bf_round(fe[3]) >= a.gate) {
                            gated = true;
                        } else {
                            float o[NOUT];
#pragma unroll
                            for (int m = 0; m < NOUT; m++) o[m] = 3.f * bf_round(fe[kSkip0 + m]);
                            expand_outputs(o, sc, cx - cm[0], cy - cm[1], cz - cm[2], eps2, f);
                        }
                    }
                } else {
                    atomicOr(a.err, kErrIndex);
                }
            }
            const uint64_t mask = __ballot(gated);
            if (gated) pendq[pend + __popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)k;   // pend < 64
            pend += __popcll(mask);
            __builtin_amdgcn_wave_barrier();
            if (pend >= 64) {
                run_net(64);
                const int rest = pend - 64;   // < 64, moved from [64, pend) to the front
                const int32_t moved = lane < rest ? pendq[64 + lane] : 0;
                __builtin_amdgcn_wave_barrier();
                if (lane < rest) pendq[lane] = moved;
                __builtin_amdgcn_wave_barrier();
                pend = rest;
            }
        }
        if (pend > 0) run_net(pend);
        wave_store_part(corr_target(a, g, it, p0, p1, q0, q1), lane, f, cx, cy, cz);
    }
}

// ---------------------------------------------------------------- learned correction in two passes

// The learned correction split into a network pass and an expansion pass,
// so that neither carries the other's registers.
//
// k_corr_gnet: every wave takes the items of seg pairs in turn (as the
// wave kernels do) and decides per pair whether the gate sends it through
// the layers (features in range and finite, BF16 l/n at least the gate).
// The pairs that go are appended to the wave's queue in LDS with their BF16
// features, scale M l^2 and pair number; each full batch of 64 runs the
// network with the weights as the MFMA's A operand held in registers (the
// layout of k_corr_net) and the features read from the queue as the B
// operand, and each pair's traceless tensor M l^2 P(o + 3 s) goes to its row
// of the pair buffer.  The queue carries over from group to group and item
// to item, so only a wave's last batch runs partly empty.
//
// k_corr_apply: per item and group, the pairs in order, four-deep software
// pipelined like k_corr_wave; a pair the gate keeps out gets the skip term
// alone (the textbook quadrupole of the BF16 features) at once, a gated pair
// is listed in LDS with its cell's COM, and whenever the list fills, and at
// the end of the group's part of the item, the listed pairs' tensors are
// read from the pair buffer and expanded.  The order of the sums is fixed by
// the item alone.
// Per-cell record of the two-pass learned correction, 32 bytes: COM xyz, l,
// the scale M l^2 (0 when the cell's part of the features -- the normalised
// second moments s = S / (M l^2) -- is out of range or not finite, or
// M l^2 <= 0, so that none of its pairs counts), then s in BF16 (xx, yy, zz,
// xy, xz, yz).  The pair features are those of pair_features: the same FP32
// operations, split between the cell and the pair.
__global__ __launch_bounds__(256) void k_corr_cells(CorrArgs a) {
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < a.n_cells; c += (int64_t)gridDim.x * 256) {
        const float* cm = a.cell_mom + 12 * c;
        const float4 u0 = *reinterpret_cast<const float4*>(cm);
        const float4 u1 = *reinterpret_cast<const float4*>(cm + 4);
        const float4 u2 = *reinterpret_cast<const float4*>(cm + 8);
        const float M = u0.w, l = u1.x;
        const float sc = M * l * l;
        const float isc = sc > 0.f ? 1.f / sc : 0.f;
        const float S[6] = {u1.y, u1.z, u1.w, u2.x, u2.y, u2.z};
        float f[6];
        bool ok = sc > 0.f;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            f[k] = S[k] * isc;
            ok = ok && fabsf(f[k]) <= kFeatLimit;   // also false for NaN
        }
        uint4* r = a.plan.crec + 2 * c;
        r[0] = make_uint4(__float_as_uint(u0.x), __float_as_uint(u0.y), __float_as_uint(u0.z), __float_as_uint(l));
        r[1] = make_uint4(__float_as_uint(ok ? sc : 0.f), (uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16),
                          (uint32_t)f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16),
                          (uint32_t)f2bf(f[4]) | ((uint32_t)f2bf(f[5]) << 16));
    }
}

// A cell record as gathered: COM, l, scale (0: the cell's pairs do not count)
// and the BF16 normalised second moments (three words).
struct CellRec {
    float com[3], l, sc;
    uint32_t s[3];
};
__device__ __forceinline__ CellRec load_cell_rec(const uint4* crec, int64_t c) {
    const uint4 r0 = crec[2 * c], r1 = crec[2 * c + 1];
    return CellRec{{__uint_as_float(r0.x), __uint_as_float(r0.y), __uint_as_float(r0.z)}, __uint_as_float(r0.w),
                   __uint_as_float(r1.x), {r1.y, r1.z, r1.w}};
}
// BF16 normalised second moment m (0..5) of a record
__device__ __forceinline__ float rec_s(const CellRec& r, int m) {
    return bf2f((uint16_t)(r.s[m >> 1] >> (16 * (m & 1))));
}
// The pair's own features d/n, l/n, eps/n, h/n (FP32) and whether the pair
// counts (the conditions of pair_features).
__device__ __forceinline__ bool rec_features(float cx, float cy, float cz, float h, const CellRec& r, float eps,
                                             float f[6]) {
    const float dx = r.com[0] - cx, dy = r.com[1] - cy, dz = r.com[2] - cz;
    const float n2 = dx * dx + dy * dy + dz * dz;
    const float inv = n2 > 0.f ? __builtin_amdgcn_rsqf(n2) : 0.f;
    f[0] = dx * inv;
    f[1] = dy * inv;
    f[2] = dz * inv;
    f[3] = r.l * inv;
    f[4] = eps * inv;
    f[5] = h * inv;
    bool ok = n2 > 0.f && r.sc > 0.f;
#pragma unroll
    for (int k = 0; k < 6; k++) ok = ok && fabsf(f[k]) <= kFeatLimit;
    return ok;
}

constexpr int kQRow = 8;     // floats per row of the pair buffer (6 used, 32-byte rows)
constexpr int kGQ = 128;     // queue slots per wave of k_corr_gnet
constexpr int kApList = 256; // listed gated pairs per wave of k_corr_apply

struct GnetQueue {
    alignas(16) uint16_t x[kGQ][16];   // BF16 features 0..11, then zeros (the first 16 of the K = 32 inputs)
    float sc[kGQ];
    int64_t p[kGQ];
    int map[64];                       // chunked passes: the group of each pair of the chunk
};

// The network inputs of a pair as queued: its features in BF16 (the pair's
// own six, then the cell's normalised second moments), zeros after them.
__device__ __forceinline__ void pack_inputs(const float fe[6], const CellRec& r, uint4& x0, uint4& x1) {
    x0 = make_uint4((uint32_t)f2bf(fe[0]) | ((uint32_t)f2bf(fe[1]) << 16),
                    (uint32_t)f2bf(fe[2]) | ((uint32_t)f2bf(fe[3]) << 16),
                    (uint32_t)f2bf(fe[4]) | ((uint32_t)f2bf(fe[5]) << 16), r.s[0]);
    x1 = make_uint4(r.s[1], r.s[2], 0u, 0u);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_corr_gnet(CorrArgs a, float* __restrict__ qbuf) {
    __shared__ float sb[NH + NH + NOUTP];
    __shared__ __align__(16) uint16_t sw3[NOUTP * NH];   // the last layer's weights (out-major), read per batch
    __shared__ GnetQueue sq[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, r16 = lane & 15, q = lane >> 4;
    GnetQueue& Q = sq[w];
    for (int i = t; i < NH; i += 256) {
        sb[i] = a.master[OFF_B1 + i];
        sb[NH + i] = a.master[OFF_B2 + i];
    }
    if (t < NOUTP) sb[2 * NH + t] = t < NOUT ? a.master[OFF_B3 + t] : 0.f;
    for (int i = t; i < NOUTP * NH; i += 256) sw3[i] = a.wbf[OFFB_W3T + i];
    bf16x8 w1a[4], w2a[4][2];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        w1a[mt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(a.wbf + OFFB_W1T + (mt * 16 + r16) * NIN + q * 8));
#pragma unroll
        for (int ks = 0; ks < 2; ks++) w2a[mt][ks] = ld_perm(a.wbf + OFFB_W2T, NH, mt * 16 + r16, ks, q);
    }
    __syncthreads();

    // the network on queue slots [0, cnt)
    auto run_net = [&](int cnt) __attribute__((always_inline)) {
#pragma unroll
        for (int tau = 0; tau < 4; tau++) {
            const int slot = tau * 16 + r16;
            bf16x8 xb = {};
            if (q < 2) xb = ld8(&Q.x[slot][q * 8]);   // K rows q*8 .. q*8+7 of pair column r16; rows >= 16 are zero
            floatx4 acc[4];
#pragma unroll
            for (int mt = 0; mt < 4; mt++) {
                const float4 bb = *reinterpret_cast<const float4*>(sb + mt * 16 + q * 4);
                acc[mt] = mfma(w1a[mt], xb, floatx4{bb.x, bb.y, bb.z, bb.w});
            }
            const bf16x8 h0 = pack8(acc[0], acc[1]), h1 = pack8(acc[2], acc[3]);
#pragma unroll
            for (int mt = 0; mt < 4; mt++) {
                const float4 bb = *reinterpret_cast<const float4*>(sb + NH + mt * 16 + q * 4);
                acc[mt] = mfma(w2a[mt][0], h0, floatx4{bb.x, bb.y, bb.z, bb.w});
                acc[mt] = mfma(w2a[mt][1], h1, acc[mt]);
            }
            const bf16x8 g0b = pack8(acc[0], acc[1]), g1b = pack8(acc[2], acc[3]);
            const float4 b3 = *reinterpret_cast<const float4*>(sb + 2 * NH + q * 4);
            floatx4 o = mfma(ld_perm(sw3, NH, r16, 0, q), g0b, floatx4{b3.x, b3.y, b3.z, b3.w});
            o = mfma(ld_perm(sw3, NH, r16, 1, q), g1b, o);
            // lane (r16, q) holds outputs q*4 .. q*4+3 of the slot's pair: q = 0 has 0..3, q = 1 has 4, 5
            if (slot < cnt && q < 2) {
                const uint16_t* xr = Q.x[slot];
                const float sc = Q.sc[slot];
                float* row = qbuf + (int64_t)kQRow * Q.p[slot];
                if (q == 0) {
                    const float o0 = o[0] + 3.f * bf2f(xr[kSkip0]), o1 = o[1] + 3.f * bf2f(xr[kSkip0 + 1]);
                    const float o2 = o[2] + 3.f * bf2f(xr[kSkip0 + 2]), o3 = o[3] + 3.f * bf2f(xr[kSkip0 + 3]);
                    const float tr = (o0 + o1 + o2) * (1.f / 3.f);
                    *reinterpret_cast<float4*>(row) = make_float4((o0 - tr) * sc, (o1 - tr) * sc, (o2 - tr) * sc, o3 * sc);
                } else {
                    const float o4 = o[0] + 3.f * bf2f(xr[kSkip0 + 4]), o5 = o[1] + 3.f * bf2f(xr[kSkip0 + 5]);
                    *reinterpret_cast<float2*>(row + 4) = make_float2(o4 * sc, o5 * sc);
                }
            }
        }
    };

    int pend = 0;   // queued pairs, uniform within the wave
    // the pair of this lane (global pair number p, its BF16 inputs x0 | x1
    // and scale sc) joins the queue if `gated`; a full batch runs the network
    auto offer = [&](bool gated, uint4 x0, uint4 x1, float sc, int64_t p) __attribute__((always_inline)) {
        const uint64_t mask = __ballot(gated);
        if (gated) {
            const int slot = pend + __popcll(mask & ((1ull << lane) - 1ull));   // pend < 64
            uint4* dst = reinterpret_cast<uint4*>(Q.x[slot]);
            dst[0] = x0;
            dst[1] = x1;
            Q.sc[slot] = sc;
            Q.p[slot] = p;
        }
        pend += __popcll(mask);
        __builtin_amdgcn_wave_barrier();
        if (pend >= 64) {
            run_net(64);
            const int rest = pend - 64;   // < 64, moved from [64, pend) to the front
            uint4 x0 = {}, x1 = {};
            float s = 0.f;
            int64_t pp = 0;
            if (lane < rest) {
                x0 = reinterpret_cast<const uint4*>(Q.x[64 + lane])[0];
                x1 = reinterpret_cast<const uint4*>(Q.x[64 + lane])[1];
                s = Q.sc[64 + lane];
                pp = Q.p[64 + lane];
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < rest) {
                reinterpret_cast<uint4*>(Q.x[lane])[0] = x0;
                reinterpret_cast<uint4*>(Q.x[lane])[1] = x1;
                Q.sc[lane] = s;
                Q.p[lane] = pp;
            }
            __builtin_amdgcn_wave_barrier();
            pend = rest;
        }
    };
    const ItemRange ir = xcd_items(a.plan.n_items);
    if (a.plan.chunked) {
        // pair-parallel: chunks of 64 consecutive pairs, each lane with its own group
        for (int64_t it = ir.first; it < ir.end; it += ir.step) {
            const int64_t q0 = it * a.plan.seg;
            const int64_t q1 = q0 + a.plan.seg < a.n_pairs ? q0 + a.plan.seg : a.n_pairs;
            int gcur = group_of_pair(a, q0);
            for (int64_t c0 = q0; c0 < q1; c0 += 64) {
                const int64_t c1 = c0 + 64 < q1 ? c0 + 64 : q1;
                chunk_groups(a, lane, c0, c1, gcur, Q.map);
                const int64_t p = c0 + lane;
                bool gated = false;
                float fe[6];
                CellRec r{};
                if (p < c1) {
                    const int g = Q.map[lane];
                    int64_t p0, p1, lb, le;
                    pair_range(a, g, p0, p1);
                    list_range(a.list_off, a.n_entries, g, lb, le);
                    float cx, cy, cz, h;
                    const int64_t k = p - p0;
                    if (group_box(a, g, cx, cy, cz, h) && k >= 0 && k < le - lb) {
                        const int64_t c = (int64_t)a.list_idx[lb + k] - a.n;   // a bad entry is flagged by k_corr_apply
                        if (c >= 0 && c < a.n_cells) {
                            r = load_cell_rec(a.plan.crec, c);
                            if (rec_features(cx, cy, cz, h, r, a.eps, fe)) gated = bf_round(fe[3]) >= a.gate;
                        }
                    }
                }
                uint4 x0 = {}, x1 = {};
                if (gated) pack_inputs(fe, r, x0, x1);
                offer(gated, x0, x1, r.sc, p);
            }
        }
    } else {
        for (int64_t it = ir.first; it < ir.end; it += ir.step)
        for (int g = group_of_pair(a, it * a.plan.seg); g < a.n_groups; g++) {
            const int64_t q0 = it * a.plan.seg;
            const int64_t q1 = q0 + a.plan.seg < a.n_pairs ? q0 + a.plan.seg : a.n_pairs;
            int64_t p0, p1;
            pair_range(a, g, p0, p1);
            if (p0 >= q1) break;
            const int64_t a0 = p0 > q0 ? p0 : q0, a1 = p1 < q1 ? p1 : q1;
            if (a1 <= a0) continue;   // no pairs of this group in the item
            float cx, cy, cz, h;
            if (!group_box(a, g, cx, cy, cz, h)) continue;   // flagged by k_corr_box
            int64_t lb, le;
            list_range(a.list_off, a.n_entries, g, lb, le);
            const int64_t k0 = a0 - p0, k1 = (a1 - p0) < (le - lb) ? (a1 - p0) : (le - lb);
            for (int64_t base = k0; base < k1; base += 64) {
                const int64_t k = base + lane;
                bool gated = false;
                float fe[6];
                CellRec r{};
                if (k < k1) {
                    const int64_t c = (int64_t)a.list_idx[lb + k] - a.n;   // a bad entry is flagged by k_corr_apply
                    if (c >= 0 && c < a.n_cells) {
                        r = load_cell_rec(a.plan.crec, c);
                        if (rec_features(cx, cy, cz, h, r, a.eps, fe)) gated = bf_round(fe[3]) >= a.gate;
                    }
                }
                uint4 x0 = {}, x1 = {};
                if (gated) pack_inputs(fe, r, x0, x1);
                offer(gated, x0, x1, r.sc, p0 + k);
            }
        }
    }
    if (pend > 0) run_net(pend);
}

// The cell record of a pair for k_corr_apply (branch-free, as in
// load_corr_cell: a position past the item, or an entry that is not a cell,
// reads cell 0 and is not valid).
struct ApCell {
    CellRec r;
    bool valid;
};
__device__ __forceinline__ ApCell load_ap_cell(const CorrArgs& a, CorrEntry en, bool& bad) {
    const int64_t c = en.e - a.n;
    const bool ok = en.pv && c >= 0 && c < a.n_cells;
    bad |= en.pv && !ok;
    return ApCell{load_cell_rec(a.plan.crec, ok ? c : 0), ok};
}

struct ApList {
    float4 com[kApList];   // COM xyz, the pair's offset from the item segment's first pair (as float bits)
    int map[64];           // chunked pass: the group of each pair of the chunk
    float carry[kCorrTerms];   // chunked pass: the open group's sum over the item's earlier chunks
};

__global__ __launch_bounds__(256) void k_corr_apply(CorrArgs a, const float* __restrict__ qbuf) {
    __shared__ ApList sl[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    ApList& L = sl[w];
    const float eps2 = a.eps * a.eps;
    const ItemRange ir = xcd_items(a.plan.n_items);
    if (a.plan.chunked) {
        // pair-parallel: chunks of 64 consecutive pairs, each lane with its own group; the lanes'
        // expansion terms are summed per group by a segmented scan across the wave, a group that
        // continues into the next chunk is carried over, and each group's sum over the item goes
        // where corr_target puts it
        bool bad = false;
        for (int64_t it = ir.first; it < ir.end; it += ir.step) {
            const int64_t q0 = it * a.plan.seg;
            const int64_t q1 = q0 + a.plan.seg < a.n_pairs ? q0 + a.plan.seg : a.n_pairs;
            int gcur = group_of_pair(a, q0);
            int carry_g = -1;   // uniform
            for (int64_t c0 = q0; c0 < q1; c0 += 64) {
                const int64_t c1 = c0 + 64 < q1 ? c0 + 64 : q1;
                chunk_groups(a, lane, c0, c1, gcur, L.map);
                const int64_t p = c0 + lane;
                const bool act = p < c1;
                const int g = act ? L.map[lane] : -1;
                float f[kCorrTerms];
#pragma unroll
                for (int k = 0; k < kCorrTerms; k++) f[k] = 0.f;
                float cx = 0.f, cy = 0.f, cz = 0.f, h = 0.f;
                int64_t p0 = 0, p1 = 0;
                if (act) {
                    pair_range(a, g, p0, p1);
                    const bool ok = group_box(a, g, cx, cy, cz, h);
                    int64_t lb, le;
                    list_range(a.list_off, a.n_entries, g, lb, le);
                    const int64_t k = p - p0;   // the group's cells lead its list
                    if (ok && a.n_cells > 0 && k >= 0 && k < le - lb) {
                        const int64_t c = (int64_t)a.list_idx[lb + k] - a.n;
                        if (c >= 0 && c < a.n_cells) {
                            const CellRec r = load_cell_rec(a.plan.crec, c);
                            float fe[6];
                            if (rec_features(cx, cy, cz, h, r, a.eps, fe)) {
                                if (bf_round(fe[3]) >= a.gate) {
                                    const float* row = qbuf + (int64_t)kQRow * p;
                                    const float4 r0 = *reinterpret_cast<const float4*>(row);
                                    const float2 r1 = *reinterpret_cast<const float2*>(row + 4);
                                    const float Qv[6] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y};
                                    quad_expand_add(cx - r.com[0], cy - r.com[1], cz - r.com[2], Qv, eps2, f);
                                } else {
                                    float o[NOUT];
#pragma unroll
                                    for (int m = 0; m < NOUT; m++) o[m] = 3.f * rec_s(r, m);
                                    expand_outputs(o, r.sc, cx - r.com[0], cy - r.com[1], cz - r.com[2], eps2, f);
                                }
                            }
                        } else {
                            bad = true;
                        }
                    }
                }
                if (lane == 0 && carry_g >= 0 && g == carry_g) {
#pragma unroll
                    for (int k = 0; k < kCorrTerms; k++) f[k] += L.carry[k];
                }
                // segmented inclusive scan: the lanes of one group are contiguous.  Every lane
                // takes part in each shuffle (a permute reads nothing from a lane that is off)
                const int g_prev = __shfl(g, lane > 0 ? lane - 1 : 0);
                const bool head = (lane == 0) | (g != g_prev);
                const uint64_t heads = __ballot(head);
                const int first = 63 - __clzll(heads & ((2ull << lane) - 1ull));
                for (int d = 1; d < 64; d <<= 1) {
                    const int src = lane >= d ? lane - d : 0;
#pragma unroll
                    for (int k = 0; k < kCorrTerms; k++) {
                        const float v = __shfl(f[k], src);
                        if (lane - d >= first) f[k] += v;
                    }
                }
                const bool seg_last = lane == 63 || ((heads >> (lane + 1)) & 1ull);
                const int64_t end = p1 < q1 ? p1 : q1;   // one past the group's last pair in this item
                const bool cont = act && seg_last && end > c1;
                const uint64_t cm = __ballot(cont);
                __builtin_amdgcn_wave_barrier();
                if (cont) {
#pragma unroll
                    for (int k = 0; k < kCorrTerms; k++) L.carry[k] = f[k];
                }
                carry_g = cm ? __builtin_amdgcn_readlane(g, (int)(c1 - c0 - 1)) : -1;
                if (act && seg_last && !cont) {
                    float4* o4 = reinterpret_cast<float4*>(corr_target(a, g, it, p0, p1, q0, q1));
#pragma unroll
                    for (int k = 0; k < 5; k++) o4[k] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
                    o4[5] = make_float4(cx, cy, cz, 0.f);
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (bad) atomicOr(a.err, kErrIndex);
        return;
    }
    for (int64_t it = ir.first; it < ir.end; it += ir.step) {
        const int64_t q0 = it * a.plan.seg;
        const int64_t q1 = q0 + a.plan.seg < a.n_pairs ? q0 + a.plan.seg : a.n_pairs;
        for (int g = group_of_pair(a, q0); g < a.n_groups; g++) {
            int64_t p0, p1;
            pair_range(a, g, p0, p1);
            if (p0 >= q1) break;
            const int64_t a0 = p0 > q0 ? p0 : q0, a1 = p1 < q1 ? p1 : q1;
            if (a1 <= a0) continue;   // no pairs of this group in the item
            float cx, cy, cz, h;
            const bool ok = group_box(a, g, cx, cy, cz, h);
            float f[kCorrTerms];
#pragma unroll
            for (int k = 0; k < kCorrTerms; k++) f[k] = 0.f;
            int64_t lb, le;
            list_range(a.list_off, a.n_entries, g, lb, le);
            // the listed gated pairs [0, cnt): tensors from the pair buffer, expanded in list order
            auto drain = [&](int cnt) {
                for (int j0 = 0; j0 < cnt; j0 += 64) {
                    const int j = j0 + lane;
                    float Qv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    float4 cm = make_float4(cx, cy, cz, 0.f);
                    if (j < cnt) {
                        cm = L.com[j];
                        const float* row = qbuf + (int64_t)kQRow * (a0 + (int64_t)__float_as_int(cm.w));
                        const float4 r0 = *reinterpret_cast<const float4*>(row);
                        const float2 r1 = *reinterpret_cast<const float2*>(row + 4);
                        Qv[0] = r0.x; Qv[1] = r0.y; Qv[2] = r0.z; Qv[3] = r0.w; Qv[4] = r1.x; Qv[5] = r1.y;
                    }
                    quad_expand_add(cx - cm.x, cy - cm.y, cz - cm.z, Qv, eps2, f);
                }
                __builtin_amdgcn_wave_barrier();
            };
            int listed = 0;   // uniform within the wave
            if (ok && le > lb && a.n_cells > 0) {
                const int64_t kmax = le - lb - 1;
                const int64_t p_first = a0 + lane;
                bool bad = false;
                ApCell cur = load_ap_cell(a, corr_list_entry(a, p_first, a1, p0, lb, kmax), bad);
                CorrEntry e_next = corr_list_entry(a, p_first + 64, a1, p0, lb, kmax);
                for (int64_t p = p_first; p - lane < a1; p += 64) {
                    const CorrEntry e_after = corr_list_entry(a, p + 128, a1, p0, lb, kmax);
                    const ApCell nxt = load_ap_cell(a, e_next, bad);
                    // keeps these loads ahead of the sum below (see k_corr_wave)
                    __asm__ volatile("" ::: "memory");
                    float fe[6];
                    const CellRec& r = cur.r;
                    const bool valid = cur.valid && rec_features(cx, cy, cz, h, r, a.eps, fe);
                    const bool gated = valid && bf_round(fe[3]) >= a.gate;
                    const uint64_t mask = __ballot(gated);
                    if (gated)
                        L.com[listed + __popcll(mask & ((1ull << lane) - 1ull))] =
                            make_float4(r.com[0], r.com[1], r.com[2], __int_as_float((int)(p - a0)));
                    listed += __popcll(mask);
                    const bool skip = valid && !gated;
                    float o[NOUT];
#pragma unroll
                    for (int m = 0; m < NOUT; m++) o[m] = skip ? 3.f * rec_s(r, m) : 0.f;
                    expand_outputs(o, skip ? r.sc : 0.f, cx - r.com[0], cy - r.com[1], cz - r.com[2], eps2, f);
                    __builtin_amdgcn_wave_barrier();
                    if (listed > kApList - 64) {
                        drain(listed);
                        listed = 0;
                    }
                    cur = nxt;
                    e_next = e_after;
                }
                if (bad) atomicOr(a.err, kErrIndex);
                if (listed > 0) drain(listed);
            }   // a malformed group was flagged by k_corr_box
            wave_store_part(corr_target(a, g, it, p0, p1, q0, q1), lane, f, cx, cy, cz);
        }
    }
}

// ---------------------------------------------------------------- training data

// Per sample (pair p, target particle i of p's group): features of the pair,
// D = c_g - COM, delta = x_i - c_g, target t = a_exact(x_i) - a_mono(x_i)
// (the cell's exact softened sum over its particles minus its monopole, FP64),
// scale M l^2 and a unit loss weight (0 for a pair outside the feature range).
__global__ __launch_bounds__(256) void k_train_samples(
    const float* __restrict__ pos, const float* __restrict__ mass, int32_t n, const int32_t* __restrict__ group_off,
    int32_t n_groups, const int64_t* __restrict__ list_off, int64_t n_entries, const int32_t* __restrict__ list_idx,
    const int64_t* __restrict__ pair_off, int64_t n_pairs, int32_t n_cells, const float* __restrict__ cell_mom,
    const int32_t* __restrict__ cell_first, const int32_t* __restrict__ cell_count, float eps,
    const int64_t* __restrict__ samples, int64_t n_samples, uint16_t* __restrict__ X, float* __restrict__ aux,
    int32_t* err) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_samples) return;
    uint16_t* xs = X + s * NIN;
    float* ax = aux + s * AUX;
    for (int k = 0; k < NIN; k++) xs[k] = 0;
    for (int k = 0; k < AUX; k++) ax[k] = 0.f;
    const int64_t p = samples[2 * s], i = samples[2 * s + 1];
    if (p < 0 || p >= n_pairs) {
        atomicOr(err, kErrIndex);
        return;
    }
    const int g = group_of_pair(pair_off, n_groups, p);
    const int g0 = group_off[g], ng = group_off[g + 1] - g0;
    if (ng < 1 || ng > kBlock || g0 < 0 || g0 + ng > n || i < g0 || i >= g0 + ng) {
        atomicOr(err, kErrGroup);
        return;
    }
    int64_t lb, le;
    list_range(list_off, n_entries, g, lb, le);
    const int64_t k = p - pair_off[g];
    const int64_t c = (k >= 0 && k < le - lb) ? (int64_t)list_idx[lb + k] - n : -1;
    if (c < 0 || c >= n_cells) {
        atomicOr(err, kErrIndex);
        return;
    }
    const int64_t f0 = cell_first[c], cnt = cell_count[c];
    if (f0 < 0 || cnt < 1 || f0 + cnt > n) {
        atomicOr(err, kErrIndex);
        return;
    }
    // group bounding box (same operations as k_group_geom)
    float lo[3], hi[3];
    for (int d = 0; d < 3; d++) lo[d] = hi[d] = pos[3 * g0 + d];
    for (int j = 1; j < ng; j++)
        for (int d = 0; d < 3; d++) {
            lo[d] = fminf(lo[d], pos[3 * (g0 + j) + d]);
            hi[d] = fmaxf(hi[d], pos[3 * (g0 + j) + d]);
        }
    const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
    const float ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    const float h = 0.5f * sqrtf(ex * ex + ey * ey + ez * ez);
    const float* cm = cell_mom + 12 * c;
    float f[NFEAT], sc;
    const bool ok = pair_features(cx, cy, cz, h, cm, eps, f, sc);
    // exact and monopole fields at x_i in FP64
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const double e2 = (double)eps * (double)eps;
    double sx = 0, sy = 0, sz = 0;
    for (int64_t j = f0; j < f0 + cnt; j++) {
        const double dx = pos[3 * j] - x, dy = pos[3 * j + 1] - y, dz = pos[3 * j + 2] - z;
        const double r2 = dx * dx + dy * dy + dz * dz + e2;
        const double w = (double)mass[j] / (r2 * sqrt(r2));
        sx += w * dx;
        sy += w * dy;
        sz += w * dz;
    }
    const double mx = cm[0] - x, my = cm[1] - y, mz = cm[2] - z;
    const double m2 = mx * mx + my * my + mz * mz;
    const double mw = (double)cm[3] / ((m2 + e2) * sqrt(m2 + e2));
    for (int k2 = 0; k2 < NFEAT; k2++) xs[k2] = f2bf(ok ? f[k2] : 0.f);
    ax[0] = cx - cm[0];
    ax[1] = cy - cm[1];
    ax[2] = cz - cm[2];
    ax[3] = (float)(x - cx);
    ax[4] = (float)(y - cy);
    ax[5] = (float)(z - cz);
    ax[6] = (float)(sx - mw * mx);
    ax[7] = (float)(sy - mw * my);
    ax[8] = (float)(sz - mw * mz);
    ax[9] = ok ? sc : 0.f;
    ax[10] = ok ? 1.f : 0.f;   // unit weight until otoo_mlp_sample_weights sets the training weight
}

// ---------------------------------------------------------------- training weights

// Loss weights and the gate's selection of training samples.  A sample s
// (target particle i, cell target t_s = a_exact - a_mono) is kept when its
// BF16 feature l/n reaches the gate; its weight is W / |a_i|^2, a_i the total
// force on the target, with W = (kept samples) / sum over kept samples of
// |t_s|^2 / |a_i|^2, so that the kept set's zero-correction loss is 1.
// Three passes: per-block kept counts and FP64 partial sums (fixed tree
// order), one block that scans the counts and forms W, then the weights and
// the kept indices in ascending sample order.
constexpr int kSwBlock = 256;

struct SwArgs {
    int64_t n_samples;
    const int64_t* samples;   // [n_samples][2]: pair, target particle
    int32_t n;
    const float* acc;         // [n][3]
    const uint16_t* X;        // [n_samples][NIN]
    float* aux;               // [n_samples][AUX]
    float gate;
    double* part_q;           // [blocks]
    int64_t* part_c;          // [blocks], then exclusive offsets
    double* scale;            // [1]: W
    int64_t* n_keep;          // [1]
    int64_t* keep;            // [n_samples]
    int32_t* err;
};

// Whether sample s is kept, and |t|^2 / |a_i|^2 (FP64) and 1 / |a_i|^2.
__device__ __forceinline__ bool sw_sample(const SwArgs& a, int64_t s, double& q, double& inv_a2) {
    q = 0.0;
    inv_a2 = 0.0;
    if (s >= a.n_samples) return false;
    const int64_t i = a.samples[2 * s + 1];
    if (i < 0 || i >= a.n) {
        atomicOr(a.err, kErrIndex);
        return false;
    }
    const double ax = a.acc[3 * i], ay = a.acc[3 * i + 1], az = a.acc[3 * i + 2];
    double a2 = ax * ax + ay * ay + az * az;
    a2 = a2 > 1e-300 ? a2 : 1e-300;   // a target at rest keeps a finite weight
    inv_a2 = 1.0 / a2;
    if (!(bf2f(a.X[s * NIN + 3]) >= a.gate)) return false;
    const float* t = a.aux + s * AUX + 6;
    const double t2 = (double)t[0] * t[0] + (double)t[1] * t[1] + (double)t[2] * t[2];
    q = t2 * inv_a2;
    return true;
}

__global__ __launch_bounds__(kSwBlock) void k_sw_count(SwArgs a) {
    __shared__ double sq[kSwBlock];
    __shared__ int sc[kSwBlock];
    const int t = threadIdx.x;
    double q, ia;
    const bool kept = sw_sample(a, (int64_t)blockIdx.x * kSwBlock + t, q, ia);
    sq[t] = q;
    sc[t] = kept ? 1 : 0;
    __syncthreads();
    for (int h = kSwBlock / 2; h > 0; h >>= 1) {   // fixed tree order
        if (t < h) {
            sq[t] += sq[t + h];
            sc[t] += sc[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        a.part_q[blockIdx.x] = sq[0];
        a.part_c[blockIdx.x] = sc[0];
    }
}

// One workgroup: exclusive scan of the block counts (in place), the total of
// the partial sums in a fixed order, and W.
__global__ __launch_bounds__(kSwBlock) void k_sw_scale(SwArgs a, int32_t blocks) {
    __shared__ double sq[kSwBlock];
    __shared__ int64_t sc[kSwBlock];
    __shared__ int64_t carry;
    const int t = threadIdx.x;
    double q = 0.0;
    for (int b = t; b < blocks; b += kSwBlock) q += a.part_q[b];   // each thread's blocks in order
    sq[t] = q;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int h = kSwBlock / 2; h > 0; h >>= 1) {
        if (t < h) sq[t] += sq[t + h];
        __syncthreads();
    }
    for (int base = 0; base < blocks; base += kSwBlock) {
        const int b = base + t;
        const int64_t v = b < blocks ? a.part_c[b] : 0;
        sc[t] = v;
        __syncthreads();
        for (int off = 1; off < kSwBlock; off <<= 1) {   // Hillis-Steele inclusive scan
            const int64_t add = t >= off ? sc[t - off] : 0;
            __syncthreads();
            sc[t] += add;
            __syncthreads();
        }
        if (b < blocks) a.part_c[b] = carry + sc[t] - v;
        __syncthreads();
        if (t == kSwBlock - 1) carry += sc[kSwBlock - 1];
        __syncthreads();
    }
    if (t == 0) {
        *a.n_keep = carry;
        *a.scale = sq[0] > 0.0 ? (double)carry / sq[0] : 1.0;
    }
}

__global__ __launch_bounds__(kSwBlock) void k_sw_write(SwArgs a) {
    __shared__ int wcount[kSwBlock / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t s = (int64_t)blockIdx.x * kSwBlock + t;
    double q, ia;
    const bool kept = sw_sample(a, s, q, ia);
    if (s < a.n_samples) a.aux[s * AUX + 10] = (float)(*a.scale * ia);
    const uint64_t mask = __ballot(kept);
    if (lane == 0) wcount[w] = __popcll(mask);
    __syncthreads();
    int64_t pos = a.part_c[blockIdx.x] + __popcll(mask & ((1ull << lane) - 1ull));
    for (int v = 0; v < w; v++) pos += wcount[v];
    if (kept) a.keep[pos] = s;
}

// ---------------------------------------------------------------- training step

struct TrainLDS {
    NetLDS net;
    alignas(16) uint16_t w2[NH * NH];      // in-major, for dH1 = dZ2 W2^T
    alignas(16) uint16_t w3[NH * NO32];    // in-major, outputs padded to 32, for dH2 = dO W3^T
    alignas(16) uint16_t x[64 * NIN];
    float z1[64 * NH];
    alignas(16) uint16_t h1[64 * NH];
    float z2[64 * NH];
    alignas(16) uint16_t h2[64 * NH];
    float o[64 * NOUTP];
    alignas(16) uint16_t d_o[64 * NO32];
    alignas(16) uint16_t dz2[64 * NH];
    alignas(16) uint16_t dz1[64 * NH];
    float red[4][NH + NH + NOUTP];  // bias-gradient partials per wave
    float lossred[256];
};

struct TrainArgs {
    const uint16_t* X;
    const float* aux;
    int64_t n_samples;
    float inv_total;   // 1 / number of samples in the batch (the loss is their mean)
    float eps2;
    const uint16_t* wbf;
    const float* master;
    float* part;       // [gridDim.x][NPARAM + 1] gradient partials, then the loss partial
};

// dW tile (mi, ni) of a matrix [K_in x N_out] stored at master offset `off`
// with row length `ncols` (only columns < ncols exist).
__device__ __forceinline__ void store_tile(float* dst, const floatx4& acc, int mi, int ni, int ncols, int nrows) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, q = lane >> 4;
    const int col = ni * 16 + r16;
    if (col >= ncols) return;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int row = mi * 16 + q * 4 + i;
        if (row < nrows) dst[row * ncols + col] = acc[i];
    }
}

__global__ __launch_bounds__(256) void k_mlp_train(TrainArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    TrainLDS& S = *reinterpret_cast<TrainLDS*>(smem);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, r16 = lane & 15, q = lane >> 4;
    load_net(S.net, a.wbf, a.master);
    for (int i = t; i < NH * NH; i += 256) S.w2[i] = a.wbf[OFFB_W2 + i];
    for (int i = t; i < NH * NO32; i += 256) S.w3[i] = a.wbf[OFFB_W3 + i];
    // weight-gradient accumulators: 28 tiles (dW1 2x4, dW2 4x4, dW3 4x1), wave w owns tiles w, w+4, ...
    floatx4 gacc[7];
#pragma unroll
    for (int k = 0; k < 7; k++) gacc[k] = floatx4{0.f, 0.f, 0.f, 0.f};
    float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gb3 = 0.f, lsum = 0.f;
    __syncthreads();
    const int r0 = 16 * w;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < a.n_samples; base += (int64_t)gridDim.x * 64) {
        for (int i = t; i < 64 * NIN; i += 256) {
            const int64_t r = base + i / NIN;
            S.x[i] = r < a.n_samples ? a.X[r * NIN + i % NIN] : 0;
        }
        __syncthreads();
        floatx4 acc[4];
        wave_dense<1, 4>(S.x, NIN, S.net.w1t, NIN, S.net.b1, r0, acc);
#pragma unroll
        for (int nt = 0; nt < 4; nt++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int idx = (r0 + q * 4 + i) * NH + nt * 16 + r16;
                S.z1[idx] = acc[nt][i];
                S.h1[idx] = f2bf(gelu(acc[nt][i]));
            }
        __syncthreads();
        wave_dense<2, 4>(S.h1, NH, S.net.w2t, NH, S.net.b2, r0, acc);
#pragma unroll
        for (int nt = 0; nt < 4; nt++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int idx = (r0 + q * 4 + i) * NH + nt * 16 + r16;
                S.z2[idx] = acc[nt][i];
                S.h2[idx] = f2bf(gelu(acc[nt][i]));
            }
        __syncthreads();
        floatx4 o1[1];
        wave_dense<2, 1>(S.h2, NH, S.net.w3t, NH, S.net.b3, r0, o1);
#pragma unroll
        for (int i = 0; i < 4; i++)
            S.o[(r0 + q * 4 + i) * NOUTP + r16] = o1[0][i] + skip_term(S.x + (r0 + q * 4 + i) * NIN, r16);
        __syncthreads();
        // loss layer: one thread per sample
        if (t < 64) {
            const int64_t s = base + t;
            float dov[NOUT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (s < a.n_samples) {
                const float* ax = a.aux + s * AUX;
                const float sc = ax[9], wt = ax[10];
                if (sc > 0.f) {
                    const float* ov = S.o + t * NOUTP;
                    const float tr = (ov[0] + ov[1] + ov[2]) * (1.f / 3.f);
                    const float qv[NOUT] = {(ov[0] - tr) * sc, (ov[1] - tr) * sc, (ov[2] - tr) * sc,
                                            ov[3] * sc,        ov[4] * sc,        ov[5] * sc};
                    // the applied correction is linear in the tensor: columns B[:, m] for unit tensors
                    float B[3][NOUT];
#pragma unroll
                    for (int m = 0; m < NOUT; m++) {
                        float e[NOUT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                        e[m] = 1.f;
                        float f[kCorrTerms];
#pragma unroll
                        for (int k = 0; k < kCorrTerms; k++) f[k] = 0.f;
                        quad_expand_add(ax[0], ax[1], ax[2], e, a.eps2, f);
                        expand_accel(f, ax[3], ax[4], ax[5], B[0][m], B[1][m], B[2][m]);
                    }
                    float r[3];
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        float v = -ax[6 + k];
#pragma unroll
                        for (int m = 0; m < NOUT; m++) v = fmaf(B[k][m], qv[m], v);
                        r[k] = v;
                    }
                    lsum += wt * (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                    const float gscale = 2.f * wt * a.inv_total;
                    float dq[NOUT];
#pragma unroll
                    for (int m = 0; m < NOUT; m++) dq[m] = gscale * (B[0][m] * r[0] + B[1][m] * r[1] + B[2][m] * r[2]);
                    const float mean = (dq[0] + dq[1] + dq[2]) * (1.f / 3.f);
                    dov[0] = (dq[0] - mean) * sc;
                    dov[1] = (dq[1] - mean) * sc;
                    dov[2] = (dq[2] - mean) * sc;
                    dov[3] = dq[3] * sc;
                    dov[4] = dq[4] * sc;
                    dov[5] = dq[5] * sc;
                }
            }
#pragma unroll
            for (int m = 0; m < NO32; m++) S.d_o[t * NO32 + m] = f2bf(m < NOUT ? dov[m] : 0.f);
            // the last layer's bias gradient is summed in FP32 from these (the row's outputs are spent)
            for (int m = 0; m < NOUT; m++) S.o[t * NOUTP + m] = dov[m];
        }
        __syncthreads();
        // db3: per-output sums over the chunk's samples (threads 0..5, fixed order)
        if (t < NOUT)
            for (int s2 = 0; s2 < 64; s2++) gb3 += S.o[s2 * NOUTP + t];
        // dW3 (tiles: 4 x 1) += H2^T dO over the 64 samples (K)
        // dH2 = dO W3^T for this wave's rows, then dZ2
        {
            floatx4 dh[4];
#pragma unroll
            for (int nt = 0; nt < 4; nt++) dh[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
            const bf16x8 av = ld8(S.d_o + (r0 + r16) * NO32 + q * 8);
#pragma unroll
            for (int nt = 0; nt < 4; nt++) dh[nt] = mfma(av, ld8(S.w3 + (nt * 16 + r16) * NO32 + q * 8), dh[nt]);
#pragma unroll
            for (int nt = 0; nt < 4; nt++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int idx = (r0 + q * 4 + i) * NH + nt * 16 + r16;
                    const float dz = dh[nt][i] * gelu_grad(S.z2[idx]);
                    S.dz2[idx] = f2bf(dz);
                    gb2[nt] += dz;
                }
        }
        __syncthreads();
        // dH1 = dZ2 W2^T for this wave's rows, then dZ1
        {
            floatx4 dh[4];
#pragma unroll
            for (int nt = 0; nt < 4; nt++) dh[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ks++) {
                const bf16x8 av = ld8(S.dz2 + (r0 + r16) * NH + ks * 32 + q * 8);
#pragma unroll
                for (int nt = 0; nt < 4; nt++)
                    dh[nt] = mfma(av, ld8(S.w2 + (nt * 16 + r16) * NH + ks * 32 + q * 8), dh[nt]);
            }
#pragma unroll
            for (int nt = 0; nt < 4; nt++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int idx = (r0 + q * 4 + i) * NH + nt * 16 + r16;
                    const float dz = dh[nt][i] * gelu_grad(S.z1[idx]);
                    S.dz1[idx] = f2bf(dz);
                    gb1[nt] += dz;
                }
        }
        __syncthreads();
        // weight gradients: K = the chunk's 64 samples, operands read across rows
#pragma unroll
        for (int k = 0; k < 7; k++) {
            const int tile = w + 4 * k;   // 0..27
            const uint16_t *Am, *Bm;
            int lda, ldb, mi, ni;
            if (tile < 8) {               // dW1 [32 x 64]: X^T dZ1
                mi = tile >> 2, ni = tile & 3;
                Am = S.x + mi * 16 + r16;
                lda = NIN;
                Bm = S.dz1 + ni * 16 + r16;
                ldb = NH;
            } else if (tile < 24) {       // dW2 [64 x 64]: H1^T dZ2
                mi = (tile - 8) >> 2, ni = (tile - 8) & 3;
                Am = S.h1 + mi * 16 + r16;
                lda = NH;
                Bm = S.dz2 + ni * 16 + r16;
                ldb = NH;
            } else {                      // dW3 [64 x 16]: H2^T dO
                mi = tile - 24, ni = 0;
                Am = S.h2 + mi * 16 + r16;
                lda = NH;
                Bm = S.d_o + r16;
                ldb = NO32;
            }
#pragma unroll
            for (int ks = 0; ks < 2; ks++) {
                const int s0 = ks * 32 + q * 8;
                gacc[k] = mfma(ld8s(Am + s0 * lda, lda), ld8s(Bm + s0 * ldb, ldb), gacc[k]);
            }
        }
        __syncthreads();
    }
    // write this workgroup's partial gradient
    float* dst = a.part + (int64_t)blockIdx.x * (NPARAM + 1);
#pragma unroll
    for (int k = 0; k < 7; k++) {
        const int tile = w + 4 * k;
        if (tile < 8) store_tile(dst + OFF_W1, gacc[k], tile >> 2, tile & 3, NH, NIN);
        else if (tile < 24) store_tile(dst + OFF_W2, gacc[k], (tile - 8) >> 2, (tile - 8) & 3, NH, NH);
        else store_tile(dst + OFF_W3, gacc[k], tile - 24, 0, NOUT, NH);
    }
    // bias gradients: lane (r16, q) of wave w holds column sums over rows q*4+i of its rows
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        // reduce over q within the wave through LDS (fixed order)
        __syncthreads();
        S.lossred[t] = gb1[nt];
        __syncthreads();
        if (q == 0) {
            float v = 0.f;
            for (int qq = 0; qq < 4; qq++) v += S.lossred[w * 64 + qq * 16 + r16];
            S.red[w][nt * 16 + r16] = v;
        }
        __syncthreads();
        S.lossred[t] = gb2[nt];
        __syncthreads();
        if (q == 0) {
            float v = 0.f;
            for (int qq = 0; qq < 4; qq++) v += S.lossred[w * 64 + qq * 16 + r16];
            S.red[w][NH + nt * 16 + r16] = v;
        }
    }
    __syncthreads();
    if (t < NH) {
        dst[OFF_B1 + t] = S.red[0][t] + S.red[1][t] + S.red[2][t] + S.red[3][t];
        dst[OFF_B2 + t] = S.red[0][NH + t] + S.red[1][NH + t] + S.red[2][NH + t] + S.red[3][NH + t];
    }
    if (t < NOUT) dst[OFF_B3 + t] = gb3;
    __syncthreads();
    S.lossred[t] = lsum;
    __syncthreads();
    if (t == 0) {
        float v = 0.f;
        for (int k = 0; k < 64; k++) v += S.lossred[k];
        dst[NPARAM] = v * a.inv_total;
    }
}

// Fixed-order FP64 sum of the per-workgroup partial rows: a workgroup takes
// kGradCols consecutive entries (parameters, then the loss) and kGradSlices
// interleaved subsets of the rows; the slices are then added in slice order.
constexpr int kGradCols = 32, kGradSlices = 8;
__global__ __launch_bounds__(kGradCols * kGradSlices) void k_grad_reduce(const float* __restrict__ part,
                                                                         int32_t n_parts, float* __restrict__ grad) {
    __shared__ double red[kGradSlices][kGradCols];
    const int c = threadIdx.x % kGradCols, sl = threadIdx.x / kGradCols;
    const int i = blockIdx.x * kGradCols + c;
    double s = 0.0;
    if (i <= NPARAM)
        for (int b = sl; b < n_parts; b += kGradSlices) s += (double)part[(int64_t)b * (NPARAM + 1) + i];
    red[sl][c] = s;
    __syncthreads();
    if (sl == 0 && i <= NPARAM) {
        double tot = 0.0;
        for (int k = 0; k < kGradSlices; k++) tot += red[k][c];
        grad[i] = (float)tot;
    }
}

// BF16 operand copies of parameter i of the FP32 master vector
__device__ __forceinline__ void write_bf16_copies(uint16_t* wbf, int i, float v) {
    const uint16_t b = f2bf(v);
    if (i < OFF_B1) {
        const int in = i / NH, out = i % NH;
        wbf[OFFB_W1T + out * NIN + in] = b;
    } else if (i >= OFF_W2 && i < OFF_B2) {
        const int j = i - OFF_W2, in = j / NH, out = j % NH;
        wbf[OFFB_W2T + out * NH + in] = b;
        wbf[OFFB_W2 + in * NH + out] = b;
    } else if (i >= OFF_W3 && i < OFF_B3) {
        const int j = i - OFF_W3, in = j / NOUT, out = j % NOUT;
        wbf[OFFB_W3T + out * NH + in] = b;
        wbf[OFFB_W3 + in * NO32 + out] = b;
    }
}

// Adam (Kingma & Ba): omb1 = 1 - beta1 and omb2 = 1 - beta2 come from the
// host in double precision (1 - 0.999f in FP32 would be off by 1.3e-5).
__global__ void k_adam(float* __restrict__ master, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, uint16_t* __restrict__ wbf, float lr, float beta1, float beta2,
                       float omb1, float omb2, float adam_eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    const float g = grad[i];
    const float mi = beta1 * m[i] + omb1 * g;
    const float vi = beta2 * v[i] + omb2 * g * g;
    m[i] = mi;
    v[i] = vi;
    const float p = master[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + adam_eps);
    master[i] = p;
    write_bf16_copies(wbf, i, p);
}

__global__ void k_bf16_clear(uint16_t* __restrict__ wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NBF) wbf[i] = 0;   // padding rows/columns stay zero
}

__global__ void k_bf16_fill(const float* __restrict__ master, uint16_t* __restrict__ wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NPARAM) write_bf16_copies(wbf, i, master[i]);
}

}  // namespace

// ================================================================ runtime

struct otoo_mlp {
    otoo_ctx* ctx = nullptr;   // must outlive every call except otoo_mlp_destroy
    int device = 0;
    float* master = nullptr;   // device [NPARAM]
    float* m = nullptr;        // device [NPARAM]
    float* v = nullptr;        // device [NPARAM]
    float* grad = nullptr;     // device [NPARAM + 1] (last gradient, then the loss)
    uint16_t* wbf = nullptr;   // device [NBF]
    float* part = nullptr;     // device gradient partials
    int part_rows = 0;
    float4* geom = nullptr;    // device per-group geometry
    int64_t geom_cap = 0;
    void* sw = nullptr;        // device block sums of otoo_mlp_sample_weights
    int64_t sw_blocks = 0;
    int64_t step = 0;
    bool has_params = false;
    float gate = 0.f;          // the layers run only for pairs whose BF16 l/n is at least this
};

namespace {

int mlp_check(otoo_mlp* m) {
    if (!m || !m->ctx) return OTOO_EINVAL;
    HIP_TRY(m->ctx, hipSetDevice(m->ctx->device));
    return OTOO_OK;
}

int mlp_upload(otoo_mlp* m, const float* host_params, const float* host_m, const float* host_v) {
    otoo_ctx* c = m->ctx;
    hipStream_t s = c->stream;
    HIP_TRY(c, hipMemcpyAsync(m->master, host_params, sizeof(float) * NPARAM, hipMemcpyHostToDevice, s));
    if (host_m) HIP_TRY(c, hipMemcpyAsync(m->m, host_m, sizeof(float) * NPARAM, hipMemcpyHostToDevice, s));
    if (host_v) HIP_TRY(c, hipMemcpyAsync(m->v, host_v, sizeof(float) * NPARAM, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bf16_clear, dim3((NBF + 255) / 256), dim3(256), 0, s, m->wbf);
    hipLaunchKernelGGL(k_bf16_fill, dim3((NPARAM + 255) / 256), dim3(256), 0, s, m->master, m->wbf);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(s));
    m->has_params = true;
    return OTOO_OK;
}

int run_backward(otoo_mlp* m, const uint16_t* X, const float* aux, int64_t n_samples, float eps) {
    otoo_ctx* c = m->ctx;
    const int blocks = (int)std::min<int64_t>((int64_t)c->num_cu, (n_samples + 63) / 64);
    if (blocks > m->part_rows) {
        if (m->part) HIP_TRY(c, hipFree(m->part));
        m->part = nullptr;
        m->part_rows = 0;   // stays 0 if the allocation fails
        HIP_TRY(c, hipMalloc(&m->part, sizeof(float) * (size_t)(NPARAM + 1) * blocks));
        m->part_rows = blocks;
    }
    TrainArgs ta{X, aux, n_samples, 1.f / (float)n_samples, eps * eps, m->wbf, m->master, m->part};
    // set on every call: the attribute belongs to the current device
    HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_train),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(TrainLDS)));
    hipLaunchKernelGGL(k_mlp_train, dim3(blocks), dim3(256), sizeof(TrainLDS), c->stream, ta);
    hipLaunchKernelGGL(k_grad_reduce, dim3((NPARAM + 1 + kGradCols - 1) / kGradCols), dim3(kGradCols * kGradSlices), 0,
                       c->stream, m->part, blocks, m->grad);
    HIP_TRY(c, hipGetLastError());
    return OTOO_OK;
}

int ensure_corr_scratch(otoo_ctx* c, size_t bytes) {
    if (bytes <= c->corr_bytes) return OTOO_OK;
    if (c->scratch_cap && bytes > c->scratch_cap)
        return fail(c, OTOO_ENOMEM, "correction scratch of %zu bytes exceeds the cap of %zu", bytes, c->scratch_cap);
    if (c->corr_buf) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipFree(c->corr_buf));
        c->corr_buf = nullptr;
        c->corr_bytes = 0;
    }
    const size_t want = c->scratch_cap ? std::min(bytes + bytes / 4, c->scratch_cap) : bytes + bytes / 4;
    if (hipMalloc(&c->corr_buf, want) != hipSuccess) {
        (void)hipGetLastError();
        c->corr_buf = nullptr;
        return fail(c, OTOO_ENOMEM, "correction scratch of %zu bytes could not be allocated", want);
    }
    c->corr_bytes = want;
    c->scratch_gen++;
    return OTOO_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }


}  // namespace

extern "C" {

int otoo_mlp_create(otoo_ctx* c, otoo_mlp** out) {
    if (!c || !out) return OTOO_EINVAL;
    *out = nullptr;
    HIP_TRY(c, hipSetDevice(c->device));
    otoo_mlp* m = new (std::nothrow) otoo_mlp();
    if (!m) return OTOO_ENOMEM;
    m->ctx = c;
    m->device = c->device;
    void* p = nullptr;
    const size_t bytes = sizeof(float) * (4 * (size_t)NPARAM + 1) + sizeof(uint16_t) * NBF + 1024;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        delete m;
        return fail(c, OTOO_ENOMEM, "network buffers");
    }
    char* b = static_cast<char*>(p);
    m->master = reinterpret_cast<float*>(b);
    m->m = m->master + NPARAM;
    m->v = m->m + NPARAM;
    m->grad = m->v + NPARAM;
    m->wbf = reinterpret_cast<uint16_t*>(b + ((sizeof(float) * (4 * (size_t)NPARAM + 1) + 255) & ~(size_t)255));
    if (hipMemset(p, 0, bytes) != hipSuccess) {
        (void)hipFree(p);
        delete m;
        return fail(c, OTOO_EHIP, "hipMemset");
    }
    *out = m;
    return OTOO_OK;
}

int otoo_mlp_destroy(otoo_mlp* m) {
    if (!m) return OTOO_EINVAL;
    // does not touch the context (it may already be gone); hipFree waits for the device
    (void)hipSetDevice(m->device);
    if (m->master) (void)hipFree(m->master);
    if (m->part) (void)hipFree(m->part);
    if (m->geom) (void)hipFree(m->geom);
    if (m->sw) (void)hipFree(m->sw);
    delete m;
    return OTOO_OK;
}

int otoo_mlp_num_params(void) { return NPARAM; }

int otoo_mlp_set_params(otoo_mlp* m, const float* params) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (!params) return fail(m->ctx, OTOO_EINVAL, "params is null");
    for (int i = 0; i < NPARAM; i++)
        if (!std::isfinite(params[i])) return fail(m->ctx, OTOO_EINVAL, "parameter %d is not finite", i);
    std::vector<float> zero(NPARAM, 0.f);
    m->step = 0;
    return mlp_upload(m, params, zero.data(), zero.data());
}

int otoo_mlp_set_gate(otoo_mlp* m, float gate) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (!(gate >= 0.f)) return fail(m->ctx, OTOO_EINVAL, "gate must be >= 0 (or +inf)");
    m->gate = gate;
    return OTOO_OK;
}

int otoo_mlp_get_params(otoo_mlp* m, float* params, float* adam_m, float* adam_v, int64_t* step) {
    int rc = mlp_check(m);
    if (rc) return rc;
    otoo_ctx* c = m->ctx;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (params) HIP_TRY(c, hipMemcpy(params, m->master, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    if (adam_m) HIP_TRY(c, hipMemcpy(adam_m, m->m, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    if (adam_v) HIP_TRY(c, hipMemcpy(adam_v, m->v, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    if (step) *step = m->step;
    return OTOO_OK;
}

int otoo_mlp_save(otoo_mlp* m, const char* path) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (!path) return fail(m->ctx, OTOO_EINVAL, "path is null");
    std::vector<float> buf(3 * (size_t)NPARAM);
    int64_t step = 0;
    rc = otoo_mlp_get_params(m, buf.data(), buf.data() + NPARAM, buf.data() + 2 * NPARAM, &step);
    if (rc) return rc;
    FILE* f = fopen(path, "wb");
    if (!f) return fail(m->ctx, OTOO_EINVAL, "cannot open %s", path);
    const char magic[8] = {'O', 'T', 'O', 'O', 'M', 'L', 'P', '1'};
    const int32_t np = NPARAM;
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&np, 4, 1, f) == 1 && fwrite(&step, 8, 1, f) == 1 &&
              fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? OTOO_OK : fail(m->ctx, OTOO_EINVAL, "write to %s failed", path);
}

int otoo_mlp_load(otoo_mlp* m, const char* path) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (!path) return fail(m->ctx, OTOO_EINVAL, "path is null");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(m->ctx, OTOO_EINVAL, "cannot open %s", path);
    char magic[8];
    int32_t np = 0;
    int64_t step = 0;
    std::vector<float> buf(3 * (size_t)NPARAM);
    bool ok = fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "OTOOMLP1", 8) == 0 && fread(&np, 4, 1, f) == 1 &&
              np == NPARAM && fread(&step, 8, 1, f) == 1 &&
              fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    fclose(f);
    if (!ok) return fail(m->ctx, OTOO_EINVAL, "%s is not a network checkpoint of this layout", path);
    for (float x : buf)
        if (!std::isfinite(x)) return fail(m->ctx, OTOO_EINVAL, "%s holds non-finite values", path);
    rc = mlp_upload(m, buf.data(), buf.data() + NPARAM, buf.data() + 2 * NPARAM);
    if (rc) return rc;
    m->step = step;
    return OTOO_OK;
}

int otoo_mlp_forward(otoo_mlp* m, const uint16_t* X, int64_t rows, float* out) {
    int rc = mlp_check(m);
    if (rc) return rc;
    if (!m->has_params) return fail(m->ctx, OTOO_EINVAL, "no parameters loaded");
    if (rows < 0 || (rows && (!X || !out))) return fail(m->ctx, OTOO_EINVAL, "bad arguments");
    if (!rows) return OTOO_OK;
    const int blocks = (int)std::min<int64_t>(4 * (int64_t)m->ctx->num_cu, (rows + 63) / 64);
    hipLaunchKernelGGL(k_mlp_forward_raw, dim3(blocks), dim3(256), 0, m->ctx->stream, X, rows, m->wbf, m->master,
                       out);
    HIP_TRY(m->ctx, hipGetLastError());
    return OTOO_OK;
}

int otoo_mlp_infer(otoo_mlp* m, int32_t n, const float* pos, int32_t n_groups, const int32_t* group_off,
                   int64_t n_entries, const int64_t* list_off, const int32_t* list_idx, int64_t n_pairs,
                   const int64_t* pair_off, int32_t n_cells, const float* cell_mom, int32_t cell_stride, float eps,
                   float* corr) {
    int rc = mlp_check(m);
    if (rc) return rc;
    otoo_ctx* c = m->ctx;
    c->err.clear();
    if (!m->has_params) return fail(c, OTOO_EINVAL, "no parameters loaded");
    if (n < 1 || n_groups < 1 || n_groups > n || n_entries < 0 || n_pairs < 0 || n_pairs > n_entries || n_cells < 0)
        return fail(c, OTOO_EINVAL, "bad sizes");
    if (cell_stride != 12) return fail(c, OTOO_EINVAL, "the network needs cell moments of stride 12");
    if (!(eps > 0.f) || !std::isfinite(eps)) return fail(c, OTOO_EINVAL, "eps must be positive and finite");
    if (!pos || !group_off || !list_off || !pair_off || (n_entries && !list_idx) || (n_cells && !cell_mom) ||
        (n_pairs && !corr))
        return fail(c, OTOO_EINVAL, "null pointer argument");
    if (!n_pairs) return OTOO_OK;
    if (n_groups > m->geom_cap) {
        if (m->geom) HIP_TRY(c, hipFree(m->geom));
        m->geom = nullptr;
        m->geom_cap = 0;   // stays 0 if the allocation fails
        HIP_TRY(c, hipMalloc(&m->geom, sizeof(float4) * (size_t)n_groups));
        m->geom_cap = n_groups;
        c->scratch_gen++;
    }
    hipLaunchKernelGGL(k_group_geom, dim3(n_groups), dim3(256), 0, c->stream, pos, n, group_off, m->geom,
                       c->errflag);
    InferArgs ia{n,        n_groups, list_off, n_entries, list_idx,  pair_off, n_pairs, n_cells,
                 cell_mom, eps,      m->geom,  m->wbf,    m->master, m->gate, corr,    c->errflag};
    const int blocks = (int)std::min<int64_t>(4 * (int64_t)c->num_cu, (n_pairs + 63) / 64);
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks), dim3(256), 0, c->stream, ia);
    HIP_TRY(c, hipGetLastError());
    return OTOO_OK;
}

int otoo_correction(otoo_ctx* c, int32_t kind, otoo_mlp* m, int32_t n, const float* pos, int32_t n_groups,
                    const int32_t* group_off, const float* group_box, int64_t n_entries, const int64_t* list_off,
                    const int32_t* list_idx,
                    int64_t n_pairs, const int64_t* pair_off, int32_t n_cells, const float* cell_mom,
                    int32_t cell_stride, float eps, const float* corr, float* gcorr) {
    if (!c) return OTOO_EINVAL;
    c->err.clear();
    HIP_TRY(c, hipSetDevice(c->device));
    if (kind != OTOO_CORR_PAIRS && kind != OTOO_CORR_QUAD && kind != OTOO_CORR_MLP)
        return fail(c, OTOO_EINVAL, "unknown correction kind %d", kind);
    if (n < 1 || n_groups < 1 || n_groups > n || n_entries < 0 || n_pairs < 0 || n_pairs > n_entries || n_cells < 0)
        return fail(c, OTOO_EINVAL, "bad sizes");
    if (cell_stride != 4 && cell_stride != 12) return fail(c, OTOO_EINVAL, "cell_stride must be 4 or 12");
    if (kind != OTOO_CORR_PAIRS && cell_stride != 12)
        return fail(c, OTOO_EINVAL, "this correction needs cell moments of stride 12");
    if (!(eps > 0.f) || !std::isfinite(eps)) return fail(c, OTOO_EINVAL, "eps must be positive and finite");
    if (!pos || !group_off || !list_off || !pair_off || !gcorr || (n_entries && !list_idx) ||
        (n_cells && !cell_mom) || (kind == OTOO_CORR_PAIRS && n_pairs && !corr))
        return fail(c, OTOO_EINVAL, "null pointer argument");
    if (kind == OTOO_CORR_MLP) {
        if (!m || m->ctx != c) return fail(c, OTOO_EINVAL, "a network of this context is required");
        if (!m->has_params) return fail(c, OTOO_EINVAL, "no parameters loaded");
    }
    CorrArgs ca{n,        pos,     n_groups, group_off, group_box, list_off, n_entries, list_idx,
                pair_off, n_pairs, n_cells,  cell_mom,  cell_stride, eps,   corr,
                m ? m->wbf : nullptr, m ? m->master : nullptr, m ? m->gate : 0.f, gcorr, c->errflag, CorrPlan{}};
    if (kind == OTOO_CORR_MLP && c->tune.net_kernel == 1) {   // one workgroup per group, LDS-staged network
        hipLaunchKernelGGL(k_corr_group, dim3((int)std::min<int64_t>(3LL * c->num_cu, n_groups)), dim3(256), 0,
                           c->stream, ca);
        HIP_TRY(c, hipGetLastError());
        return OTOO_OK;
    }
    // one wave per item of seg pairs (items taken statically), then the rows of the groups
    // that straddle items or have no pairs
    CorrPlan& pl = ca.plan;
    const bool split = kind == OTOO_CORR_MLP && c->tune.net_kernel == 2;   // network pass + expansion pass
    // resident workgroups per CU of each kernel (the same for every device of this build)
    static std::atomic<int> occ[5] = {0, 0, 0, 0, 0};
    auto resident = [&](int which, const void* fn, int& per_cu) -> int {
        per_cu = occ[which].load(std::memory_order_relaxed);
        if (!per_cu) {
            HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0));
            per_cu = std::max(per_cu, 1);
            occ[which].store(per_cu, std::memory_order_relaxed);
        }
        return OTOO_OK;
    };
    const int which = kind == OTOO_CORR_PAIRS ? 0 : kind == OTOO_CORR_QUAD ? 1 : split ? 3 : 2;
    const void* fn = which == 0   ? reinterpret_cast<const void*>(&k_corr_wave<kCorrPairs>)
                     : which == 1 ? reinterpret_cast<const void*>(&k_corr_wave<kCorrQuad>)
                     : which == 2 ? reinterpret_cast<const void*>(&k_corr_net)
                                  : reinterpret_cast<const void*>(&k_corr_apply);
    int per_cu = 0, per_cu_net = 0;
    int rc = resident(which, fn, per_cu);
    if (rc) return rc;
    if (split) {
        rc = resident(4, reinterpret_cast<const void*>(&k_corr_gnet), per_cu_net);
        if (rc) return rc;
    }
    const int64_t waves = 4LL * std::max(per_cu, per_cu_net) * c->num_cu;
    pl.seg = kCorrSeg;
    while (pl.seg > kCorrSegMin && (n_pairs + pl.seg - 1) / pl.seg < 4 * waves) pl.seg /= 2;
    pl.n_items = (n_pairs + pl.seg - 1) / pl.seg;
    // pair-parallel chunks for sparse pairs (fewer than 32 per group, e.g. the nearest cells only), and
    // for fewer than 128 per group when even items of kCorrSegMin pairs leave waves without four items
    const bool underfull = (n_pairs + kCorrSegMin - 1) / kCorrSegMin < 4 * waves;
    const bool sparse = n_pairs < 32LL * n_groups || (underfull && n_pairs < 128LL * n_groups);
    pl.chunked = split && (c->tune.corr_chunks == 2 || (c->tune.corr_chunks == 0 && sparse));
    const size_t part_bytes = align256(sizeof(float) * kCorrStride * (size_t)std::max<int64_t>(pl.n_items, 1));
    const size_t box_bytes = align256(sizeof(float4) * (size_t)n_groups);
    const size_t qbuf_bytes = split ? align256(sizeof(float) * kQRow * (size_t)std::max<int64_t>(n_pairs, 1)) : 0;
    const size_t crec_bytes = split ? align256(2 * sizeof(uint4) * (size_t)std::max<int32_t>(n_cells, 1)) : 0;
    rc = ensure_corr_scratch(c, 2 * part_bytes + box_bytes + qbuf_bytes + crec_bytes);
    if (rc) return rc;
    pl.part_l = static_cast<float*>(c->corr_buf);
    pl.part_r = reinterpret_cast<float*>(static_cast<char*>(c->corr_buf) + part_bytes);
    pl.box = reinterpret_cast<float4*>(static_cast<char*>(c->corr_buf) + 2 * part_bytes);
    float* qbuf = split ? reinterpret_cast<float*>(static_cast<char*>(c->corr_buf) + 2 * part_bytes + box_bytes)
                        : nullptr;
    pl.crec = split ? reinterpret_cast<uint4*>(static_cast<char*>(c->corr_buf) + 2 * part_bytes + box_bytes + qbuf_bytes)
                    : nullptr;
    if (group_box)
        hipLaunchKernelGGL(k_corr_box_given, dim3((unsigned)(((int64_t)n_groups + 255) / 256)), dim3(256), 0,
                           c->stream, ca);
    else
        hipLaunchKernelGGL(k_corr_box, dim3((unsigned)(((int64_t)n_groups + 3) / 4)), dim3(256), 0, c->stream, ca);
    const int64_t item_blocks = std::max<int64_t>((pl.n_items + 3) / 4, 1);
    const dim3 grid((unsigned)std::min<int64_t>((int64_t)per_cu * c->num_cu, item_blocks));
    if (which == 0) {
        hipLaunchKernelGGL(k_corr_wave<kCorrPairs>, grid, dim3(256), 0, c->stream, ca);
    } else if (which == 1) {
        hipLaunchKernelGGL(k_corr_wave<kCorrQuad>, grid, dim3(256), 0, c->stream, ca);
    } else if (which == 2) {
        hipLaunchKernelGGL(k_corr_net, grid, dim3(256), 0, c->stream, ca);
    } else {
        const dim3 grid_net((unsigned)std::min<int64_t>((int64_t)per_cu_net * c->num_cu, item_blocks));
        if (n_cells > 0)
            hipLaunchKernelGGL(k_corr_cells, dim3((unsigned)std::min<int64_t>(4LL * c->num_cu, ((int64_t)n_cells + 255) / 256)),
                               dim3(256), 0, c->stream, ca);
        hipLaunchKernelGGL(k_corr_gnet, grid_net, dim3(256), 0, c->stream, ca, qbuf);
        hipLaunchKernelGGL(k_corr_apply, grid, dim3(256), 0, c->stream, ca, static_cast<const float*>(qbuf));
    }
    const int merge_blocks = (int)std::min<int64_t>(4LL * c->num_cu, ((int64_t)n_groups + 255) / 256);
    hipLaunchKernelGGL(k_corr_merge, dim3(merge_blocks), dim3(256), 0, c->stream, ca);
    HIP_TRY(c, hipGetLastError());
    return OTOO_OK;
}

int otoo_mlp_train_samples(otoo_mlp* m, int32_t n, const float* pos, const float* mass, int32_t n_groups,
                           const int32_t* group_off, int64_t n_entries, const int64_t* list_off,
                           const int32_t* list_idx, int64_t n_pairs, const int64_t* pair_off, int32_t n_cells,
                           const float* cell_mom, int32_t cell_stride, const int32_t* cell_first,
                           const int32_t* cell_count, float eps, int64_t n_samples, const int64_t* samples,
                           uint16_t* X, float* aux) {
    int rc = mlp_check(m);
    if (rc) return rc;
    otoo_ctx* c = m->ctx;
    c->err.clear();
    if (n < 1 || n_groups < 1 || n_groups > n || n_entries < 0 || n_pairs < 0 || n_pairs > n_entries ||
        n_cells < 0 || n_samples < 0)
        return fail(c, OTOO_EINVAL, "bad sizes");
    if (cell_stride != 12) return fail(c, OTOO_EINVAL, "cell moments of stride 12 are required");
    if (!(eps > 0.f) || !std::isfinite(eps)) return fail(c, OTOO_EINVAL, "eps must be positive and finite");
    if (!pos || !mass || !group_off || !list_off || !pair_off || (n_entries && !list_idx) ||
        (n_cells && (!cell_mom || !cell_first || !cell_count)) || (n_samples && (!samples || !X || !aux)))
        return fail(c, OTOO_EINVAL, "null pointer argument");
    if (!n_samples) return OTOO_OK;
    hipLaunchKernelGGL(k_train_samples, dim3((unsigned)((n_samples + 255) / 256)), dim3(256), 0, c->stream, pos, mass,
                       n, group_off, n_groups, list_off, n_entries, list_idx, pair_off, n_pairs, n_cells, cell_mom,
                       cell_first, cell_count, eps, samples, n_samples, X, aux, c->errflag);
    HIP_TRY(c, hipGetLastError());
    return OTOO_OK;
}

int otoo_mlp_sample_weights(otoo_mlp* m, int64_t n_samples, const int64_t* samples, int32_t n, const float* acc,
                            const uint16_t* X, float* aux, float gate, int64_t* keep, int64_t* n_keep) {
    int rc = mlp_check(m);
    if (rc) return rc;
    otoo_ctx* c = m->ctx;
    c->err.clear();
    if (n_samples < 0 || n < 1) return fail(c, OTOO_EINVAL, "bad sizes");
    if (!(gate >= 0.f)) return fail(c, OTOO_EINVAL, "the gate must be non-negative");
    if (!n_keep || (n_samples && (!samples || !acc || !X || !aux || !keep)))
        return fail(c, OTOO_EINVAL, "null pointer argument");
    *n_keep = 0;
    if (!n_samples) return OTOO_OK;
    const int64_t blocks = (n_samples + kSwBlock - 1) / kSwBlock;
    if (blocks > INT32_MAX) return fail(c, OTOO_EINVAL, "too many samples");
    if (blocks > m->sw_blocks) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (m->sw) HIP_TRY(c, hipFree(m->sw));
        m->sw = nullptr;
        m->sw_blocks = 0;   // stays 0 if the allocation fails
        HIP_TRY(c, hipMalloc(&m->sw, 16 * (size_t)blocks + 256));
        m->sw_blocks = blocks;
    }
    char* b = static_cast<char*>(m->sw);
    SwArgs a{n_samples, samples, n, acc, X, aux, gate, reinterpret_cast<double*>(b),
             reinterpret_cast<int64_t*>(b + 8 * (size_t)blocks), reinterpret_cast<double*>(b + 16 * (size_t)blocks),
             reinterpret_cast<int64_t*>(b + 16 * (size_t)blocks + 8), keep, c->errflag};
    hipLaunchKernelGGL(k_sw_count, dim3((unsigned)blocks), dim3(kSwBlock), 0, c->stream, a);
    hipLaunchKernelGGL(k_sw_scale, dim3(1), dim3(kSwBlock), 0, c->stream, a, (int32_t)blocks);
    hipLaunchKernelGGL(k_sw_write, dim3((unsigned)blocks), dim3(kSwBlock), 0, c->stream, a);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(n_keep, a.n_keep, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return OTOO_OK;
}

int otoo_mlp_backward(otoo_mlp* m, const uint16_t* X, const float* aux, int64_t n_samples, float eps,
                      float* grad_out, float* loss_out) {
    int rc = mlp_check(m);
    if (rc) return rc;
    otoo_ctx* c = m->ctx;
    c->err.clear();
    if (!m->has_params) return fail(c, OTOO_EINVAL, "no parameters loaded");
    if (n_samples < 1 || !X || !aux) return fail(c, OTOO_EINVAL, "bad arguments");
    if (!(eps > 0.f) || !std::isfinite(eps)) return fail(c, OTOO_EINVAL, "eps must be positive and finite");
    rc = run_backward(m, X, aux, n_samples, eps);
    if (rc) return rc;
    if (grad_out || loss_out) {
        std::vector<float> g(NPARAM + 1);
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipMemcpy(g.data(), m->grad, sizeof(float) * (NPARAM + 1), hipMemcpyDeviceToHost));
        if (grad_out) std::memcpy(grad_out, g.data(), sizeof(float) * NPARAM);
        if (loss_out) *loss_out = g[NPARAM];
    }
    return OTOO_OK;
}

int otoo_mlp_train_step(otoo_mlp* m, const uint16_t* X, const float* aux, int64_t n_samples, float eps, float lr,
                        float* loss_out) {
    int rc = mlp_check(m);
    if (rc) return rc;
    otoo_ctx* c = m->ctx;
    c->err.clear();
    if (!m->has_params) return fail(c, OTOO_EINVAL, "no parameters loaded");
    if (n_samples < 1 || !X || !aux) return fail(c, OTOO_EINVAL, "bad arguments");
    if (!(eps > 0.f) || !std::isfinite(eps) || !(lr >= 0.f) || !std::isfinite(lr))
        return fail(c, OTOO_EINVAL, "eps must be positive and lr non-negative");
    rc = run_backward(m, X, aux, n_samples, eps);
    if (rc) return rc;
    m->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = (float)(1.0 - std::pow(b1, (double)m->step));
    const float bc2 = (float)(1.0 - std::pow(b2, (double)m->step));
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, c->stream, m->master, m->m, m->v, m->grad,
                       m->wbf, lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, bc1, bc2);
    HIP_TRY(c, hipGetLastError());
    if (loss_out) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipMemcpy(loss_out, m->grad + NPARAM, sizeof(float), hipMemcpyDeviceToHost));
    }
    return OTOO_OK;
}

}  // extern "C"
