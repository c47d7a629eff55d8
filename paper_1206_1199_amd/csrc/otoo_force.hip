// Device half of libotoo: the grouped gravity force evaluation on gfx950.
//
// Per call (all on the context stream, no host synchronisation):
//   k_pack        unified source table src[e] = (x, y, z, m): particles 0..n-1,
//                 then cell monopoles (COM, M) at n + c (the index space of
//                 Sec. 3.2, the (r, m) words of Sec. 3.4); clears the queue.
//   k_sched_*     work items (group g, chunk k of its list), their partial-row
//                 offsets, and an optional longest-first order.
//   k_force       persistent workgroups pull items from a device queue; the
//                 group's targets sit in registers, list tiles are gathered
//                 with coalesced loads into LDS and read back as broadcasts;
//                 FP32 pair arithmetic, per-tile FP32 partials, Kahan across
//                 tiles.  A group whose list is one item writes its results
//                 directly; longer lists leave per-item partial rows.
//   k_reduce      per particle of the groups whose list was split: Kahan
//                 over the item partials in item order, potential in FP64,
//                 self pair removed.
// The pair term is the Plummer-softened monopole; an optional per-group
// second-order local expansion (from otoo_correction) adds a cell correction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "otoo.h"
#include "otoo_internal.h"

using namespace otoo_detail;

namespace {

constexpr int kScanBlock = 1024;      // groups per scan block (256 threads x 4)

// ---------------------------------------------------------------- K1 pack

__global__ void k_pack(const float* __restrict__ pos, const float* __restrict__ mass, int32_t n,
                       const float* __restrict__ cell_mom, int32_t n_cells, int32_t stride,
                       float4* __restrict__ src, Meta* meta) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) {
        meta->head = 0;
        meta->n_split = 0;
        for (int c = 0; c < kClasses; c++) {
            meta->hist[c] = 0;
            meta->cursor[c] = 0;
        }
    }
    if (e < n) {
        src[e] = make_float4(pos[3 * e], pos[3 * e + 1], pos[3 * e + 2], mass[e]);
    } else if (e < (int64_t)n + n_cells) {
        const float* c = cell_mom + (e - n) * stride;
        src[e] = make_float4(c[0], c[1], c[2], c[3]);
    }
}

// ---------------------------------------------------------------- scheduling

// Per group: items c_g and partial rows p_g (only for groups split in >1
// items); block-local exclusive prefix sums and block totals.
__global__ __launch_bounds__(256) void k_sched_scan1(const int32_t* __restrict__ group_off,
                                                     const int64_t* __restrict__ list_off, int64_t n_entries,
                                                     int32_t n_groups, int32_t chunk, int64_t* item_base,
                                                     int64_t* part_base, int64_t* block_tot) {
    __shared__ int64_t s_i[256], s_p[256];
    const int t = threadIdx.x;
    const int64_t g0 = (int64_t)blockIdx.x * kScanBlock + 4 * t;
    int64_t ci[4], cp[4], si = 0, sp = 0;
    for (int k = 0; k < 4; k++) {
        const int64_t g = g0 + k;
        ci[k] = cp[k] = 0;
        if (g < n_groups) {
            int64_t b, e;
            list_range(list_off, n_entries, (int)g, b, e);
            const int64_t c = n_chunks(e - b, chunk);
            int ng = group_off[g + 1] - group_off[g];
            ng = ng < 0 ? 0 : (ng > kBlock ? kBlock : ng);
            ci[k] = c;
            cp[k] = c > 1 ? c * ng : 0;
        }
        si += ci[k];
        sp += cp[k];
    }
    s_i[t] = si;
    s_p[t] = sp;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 256 thread sums
    for (int off = 1; off < 256; off <<= 1) {
        int64_t ai = 0, ap = 0;
        if (t >= off) {
            ai = s_i[t - off];
            ap = s_p[t - off];
        }
        __syncthreads();
        s_i[t] += ai;
        s_p[t] += ap;
        __syncthreads();
    }
    int64_t ri = s_i[t] - si, rp = s_p[t] - sp;  // exclusive
    for (int k = 0; k < 4; k++) {
        const int64_t g = g0 + k;
        if (g < n_groups) {
            item_base[g] = ri;
            part_base[g] = rp;
        }
        ri += ci[k];
        rp += cp[k];
    }
    if (t == 255) {
        block_tot[2 * blockIdx.x] = s_i[255];
        block_tot[2 * blockIdx.x + 1] = s_p[255];
    }
}

// Exclusive scan of block totals (one workgroup, sequential over 256-wide
// chunks), grand totals into meta.
__global__ __launch_bounds__(256) void k_sched_scan2(int64_t* block_tot, int32_t n_blocks, Meta* meta) {
    __shared__ int64_t s_i[256], s_p[256];
    __shared__ int64_t carry_i, carry_p;
    const int t = threadIdx.x;
    if (t == 0) {
        carry_i = 0;
        carry_p = 0;
    }
    __syncthreads();
    for (int base = 0; base < n_blocks; base += 256) {
        const int b = base + t;
        const int64_t vi = b < n_blocks ? block_tot[2 * b] : 0;
        const int64_t vp = b < n_blocks ? block_tot[2 * b + 1] : 0;
        s_i[t] = vi;
        s_p[t] = vp;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            int64_t ai = 0, ap = 0;
            if (t >= off) {
                ai = s_i[t - off];
                ap = s_p[t - off];
            }
            __syncthreads();
            s_i[t] += ai;
            s_p[t] += ap;
            __syncthreads();
        }
        if (b < n_blocks) {
            block_tot[2 * b] = carry_i + s_i[t] - vi;
            block_tot[2 * b + 1] = carry_p + s_p[t] - vp;
        }
        __syncthreads();
        if (t == 255) {
            carry_i += s_i[255];
            carry_p += s_p[255];
        }
        __syncthreads();
    }
    if (t == 0) {
        meta->n_items = carry_i;
        meta->n_parts = carry_p;
    }
}

__device__ __forceinline__ int cost_class(int64_t cost) {
    int c = cost > 0 ? 63 - __clzll((unsigned long long)cost) : 0;
    return c >= kClasses ? kClasses - 1 : c;
}

// Item table (g, k), the list of groups split into several items (for the
// reduction) and, for longest-first, a histogram of cost classes (counted in
// LDS, one global atomic per class and one for the split list per workgroup).
__global__ __launch_bounds__(256) void k_sched_fill(const int32_t* __restrict__ group_off,
                                                    const int64_t* __restrict__ list_off, int64_t n_entries,
                                                    int32_t n_groups, int32_t chunk, int64_t* item_base,
                                                    int64_t* part_base, const int64_t* __restrict__ block_tot,
                                                    int2* items, int64_t item_cap, int32_t lpt, Meta* meta,
                                                    int32_t* __restrict__ split, int32_t* err) {
    __shared__ int hist[kClasses];
    __shared__ int s_split[256];
    __shared__ int s_nsplit, s_base;
    const int t = threadIdx.x;
    if (t < kClasses) hist[t] = 0;
    if (t == 0) s_nsplit = 0;
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + t;
    if (g < n_groups) {
        const int64_t blk = g / kScanBlock;
        const int64_t ib = item_base[g] + block_tot[2 * blk];
        item_base[g] = ib;
        part_base[g] += block_tot[2 * blk + 1];
        int64_t b, e;
        list_range(list_off, n_entries, (int)g, b, e);
        const int64_t len = e - b;
        const int64_t c = n_chunks(len, chunk);
        int ng = group_off[g + 1] - group_off[g];
        ng = ng < 0 ? 0 : (ng > kBlock ? kBlock : ng);
        for (int64_t k = 0; k < c; k++) {
            const int64_t q = ib + k;
            if (q >= item_cap) {
                atomicOr(err, kErrCapacity);
                break;
            }
            items[q] = make_int2((int)g, (int)k);
            if (lpt) {
                const int64_t l = (k + 1 < c) ? chunk : len - k * (int64_t)chunk;
                atomicAdd(&hist[cost_class((int64_t)ng * (l > 0 ? l : 1))], 1);
            }
        }
        if (c > 1) s_split[atomicAdd(&s_nsplit, 1)] = (int)g;
    }
    __syncthreads();
    if (t == 0) s_base = s_nsplit ? atomicAdd(&meta->n_split, s_nsplit) : 0;
    __syncthreads();
    // n_split never exceeds n_groups, the capacity of the split list
    if (t < s_nsplit) split[s_base + t] = s_split[t];
    if (lpt && t < kClasses && hist[t]) atomicAdd(&meta->hist[t], hist[t]);
}

__device__ __forceinline__ int item_class(const int2 it, const int32_t* group_off, const int64_t* list_off,
                                          int64_t n_entries, int32_t chunk) {
    int64_t b, e;
    list_range(list_off, n_entries, it.x, b, e);
    const int64_t len = e - b;
    const int64_t c = n_chunks(len, chunk);
    int ng = group_off[it.x + 1] - group_off[it.x];
    ng = ng < 0 ? 0 : (ng > kBlock ? kBlock : ng);
    const int64_t l = (it.y + 1 < c) ? chunk : len - it.y * (int64_t)chunk;
    return cost_class((int64_t)ng * (l > 0 ? l : 1));
}

// Scatter items into longest-first order: classes from the most to the least
// expensive.  Each workgroup takes a contiguous range of items, ranks them
// per class in LDS and reserves its slots with one global atomic per class
// (a class's slots start after every more expensive class, summed from the
// histogram).
__global__ __launch_bounds__(256) void k_lpt_scatter(const int2* __restrict__ items, const int32_t* __restrict__ group_off,
                                                     const int64_t* __restrict__ list_off, int64_t n_entries,
                                                     int32_t chunk, int64_t item_cap, Meta* meta,
                                                     int32_t* __restrict__ order) {
    __shared__ int cnt[kClasses], base[kClasses], rank[kClasses], first[kClasses];
    const int t = threadIdx.x;
    if (t == 0) {
        int run = 0;
        for (int c = kClasses - 1; c >= 0; c--) {
            first[c] = run;
            run += meta->hist[c];
        }
    }
    const int64_t n_items = meta->n_items < item_cap ? meta->n_items : item_cap;
    const int64_t per = (n_items + gridDim.x - 1) / gridDim.x;
    const int64_t q0 = (int64_t)blockIdx.x * per;
    const int64_t q1 = (q0 + per < n_items) ? q0 + per : n_items;
    if (t < kClasses) {
        cnt[t] = 0;
        rank[t] = 0;
    }
    __syncthreads();
    for (int64_t q = q0 + t; q < q1; q += blockDim.x)
        atomicAdd(&cnt[item_class(items[q], group_off, list_off, n_entries, chunk)], 1);
    __syncthreads();
    if (t < kClasses) base[t] = cnt[t] ? first[t] + atomicAdd(&meta->cursor[t], cnt[t]) : 0;
    __syncthreads();
    for (int64_t q = q0 + t; q < q1; q += blockDim.x) {
        const int cls = item_class(items[q], group_off, list_off, n_entries, chunk);
        const int p = base[cls] + atomicAdd(&rank[cls], 1);
        if (p < n_items) order[p] = (int32_t)q;
    }
}

// ---------------------------------------------------------------- cell correction

// Textbook quadrupole of each accepted cell, Q = 3 S - tr(S) I from the
// cell's second-moment tensor S, written per (group, cell) pair.
__global__ __launch_bounds__(256) void k_quad_exact(int32_t n, int32_t n_groups, const int64_t* __restrict__ list_off,
                                                    int64_t n_entries, const int32_t* __restrict__ list_idx,
                                                    const int64_t* __restrict__ pair_off, int64_t n_pairs,
                                                    int32_t n_cells, const float* __restrict__ cell_mom,
                                                    float* __restrict__ corr, int32_t* err) {
    const int g = blockIdx.x;
    int64_t lb, le;
    list_range(list_off, n_entries, g, lb, le);
    const int64_t p0 = clamp64(pair_off[g], 0, n_pairs);
    const int64_t p1 = clamp64(pair_off[g + 1], p0, n_pairs);
    const int64_t nce = (p1 - p0) < (le - lb) ? (p1 - p0) : (le - lb);
    for (int64_t k = threadIdx.x; k < nce; k += blockDim.x) {
        const int64_t c = (int64_t)list_idx[lb + k] - n;
        float* q = corr + 6 * (p0 + k);
        if (c < 0 || c >= n_cells) {
            atomicOr(err, kErrIndex);
            for (int m = 0; m < 6; m++) q[m] = 0.f;
            continue;
        }
        const float* S = cell_mom + 12 * c + 5;
        const float tr = S[0] + S[1] + S[2];
        q[0] = 3.f * S[0] - tr;
        q[1] = 3.f * S[1] - tr;
        q[2] = 3.f * S[2] - tr;
        q[3] = 3.f * S[3];
        q[4] = 3.f * S[4];
        q[5] = 3.f * S[5];
    }
}

// Second-order local expansion of group g's cell correction applied at x:
// a += A + J delta + 1/2 H[delta, delta], phi += Phi - A.delta - 1/2 delta.J delta.
__device__ __forceinline__ void apply_corr(const float* __restrict__ gc, float x, float y, float z, float& ax,
                                           float& ay, float& az, double& phi) {
    const float dx = x - gc[kCorrTerms], dy = y - gc[kCorrTerms + 1], dz = z - gc[kCorrTerms + 2];
    const float* J = gc + 4;
    const float* H = gc + 10;   // xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz
    const float jx = J[0] * dx + J[3] * dy + J[4] * dz;
    const float jy = J[3] * dx + J[1] * dy + J[5] * dz;
    const float jz = J[4] * dx + J[5] * dy + J[2] * dz;
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz, xy = 2.f * dx * dy, xz = 2.f * dx * dz,
                yz = 2.f * dy * dz;
    const float hx = H[0] * xx + H[5] * yy + H[7] * zz + H[3] * xy + H[4] * xz + H[9] * yz;
    const float hy = H[3] * xx + H[1] * yy + H[8] * zz + H[5] * xy + H[9] * xz + H[6] * yz;
    const float hz = H[4] * xx + H[6] * yy + H[2] * zz + H[9] * xy + H[7] * xz + H[8] * yz;
    ax += gc[0] + jx + 0.5f * hx;
    ay += gc[1] + jy + 0.5f * hy;
    az += gc[2] + jz + 0.5f * hz;
    phi += (double)gc[3] - (double)(gc[0] * dx + gc[1] * dy + gc[2] * dz) -
           0.5 * (double)(dx * jx + dy * jy + dz * jz);
}

// ---------------------------------------------------------------- K2 force

struct ForceArgs {
    const float4* src;
    int32_t n_src;            // records in src, clamped to the int32 range of the list entries
    int32_t n;
    const int32_t* group_off;
    const int64_t* list_off;
    int64_t n_entries;
    const int32_t* list_idx;
    const int2* items;
    const int32_t* order;     // NULL: items in table order
    int64_t item_cap;
    const int64_t* part_base;
    float4* partial;          // rows of 8 floats: acc sum xyz, pot sum | acc comp xyz, pot comp
    int64_t part_cap;
    Meta* meta;
    int32_t chunk;
    float eps2;
    const float* gcorr;       // per-group correction expansion (NULL: plain monopole)
    float* out_acc;
    double* out_pot;
    int32_t* err;
};

// A 64-bit value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Interaction of one target with one source: Plummer-softened monopole.
// 13 VALU operations and one v_rsq_f32.
__device__ __forceinline__ void pair_mono(float xi, float yi, float zi, float4 s, float eps2, float& ax, float& ay,
                                          float& az, float& ph) {
    const float dx = s.x - xi;
    const float dy = s.y - yi;
    const float dz = s.z - zi;
    float r2 = fmaf(dx, dx, eps2);
    r2 = fmaf(dy, dy, r2);
    r2 = fmaf(dz, dz, r2);
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float mr = s.w * rinv;
    const float mr3 = mr * rinv * rinv;
    ax = fmaf(mr3, dx, ax);
    ay = fmaf(mr3, dy, ay);
    az = fmaf(mr3, dz, az);
    ph += mr;
}

constexpr int kPadRows = 128;  // zero-mass records after each LDS tile

// The wave parts of a group of ng targets that does not divide the
// workgroup: part j takes n[j] consecutive targets and splits each tile into
// S = 64 / n[j] slices, so it runs about TILE / S rows.  The largest part,
// c = 64 / (64 / ceil(ng / 4)) targets, keeps the longest row count to that
// of a workgroup-wide layout; as many parts as fit take c targets, the rest
// of the targets goes to the remaining parts in the largest counts 64 / S
// that fit, and the last part takes what is left.
__host__ __device__ constexpr void part_counts(int ng, int (&n)[4]) {
    const int c = 64 / (64 / ((ng + 3) >> 2));
    const int nfull = ng / c;                // at most 4
    int r = ng - nfull * c;
    for (int j = 0; j < 4; j++) {
        if (j < nfull) {
            n[j] = c;
        } else if (j == 3) {
            n[j] = r;
        } else {
            n[j] = r > 0 ? 64 / (64 / (r + 1) + 1) : 0;   // largest 64 / S <= r
            r -= n[j];
        }
    }
}

// Wave rows of a full tile of `tile` entries: the parts, and the
// workgroup-wide layout with S = 256 / ng slices (the waves whose lanes are
// all past S ng skip the tile).  The parts are used where they run fewer
// rows, and always where the workgroup-wide layout would have more than 64
// slices (its last slice would run past the zero records).
__host__ __device__ constexpr bool use_parts(int ng, int tile) {
    if (kBlock % ng == 0) return false;
    const int S = kBlock / ng;
    if (S > 64) return true;
    int n[4] = {0, 0, 0, 0};
    part_counts(ng, n);
    int part_rows = 0;
    for (int j = 0; j < 4; j++) part_rows += n[j] > 0 ? (tile + 64 / n[j] - 1) / (64 / n[j]) : 0;
    const int shared_rows = ((S * ng + 63) >> 6) * ((tile + S - 1) / S);
    return part_rows < shared_rows;
}

// The lane layout of each group size, fixed at compile time so that items
// decode it with one scalar load instead of integer divisions on the vector
// unit: the part counts, the workgroup-wide slice count 256 / ng, and (bit
// t of `parts`) whether tiles of 256 << t entries use the parts.
struct GroupLayout {
    uint8_t n[4];
    uint16_t S;
    uint8_t parts;
    uint8_t pad;
};
struct LayoutTable {
    GroupLayout e[kBlock + 1];
};
constexpr LayoutTable make_layouts() {
    LayoutTable t{};
    for (int ng = 1; ng <= kBlock; ng++) {
        int n[4] = {0, 0, 0, 0};
        part_counts(ng, n);
        GroupLayout& e = t.e[ng];
        for (int j = 0; j < 4; j++) e.n[j] = (uint8_t)n[j];
        e.S = (uint16_t)(kBlock / ng);
        e.parts = (uint8_t)((use_parts(ng, 256) ? 1 : 0) | (use_parts(ng, 512) ? 2 : 0) |
                            (use_parts(ng, 1024) ? 4 : 0));
    }
    return t;
}
__constant__ LayoutTable kLayouts = make_layouts();

template <int TILE>
constexpr int tile_bit() {
    return TILE == 256 ? 1 : (TILE == 512 ? 2 : 4);
}

// floor(x / d) for 0 <= x <= 2048 and 1 <= d <= 256 through the reciprocal:
// (x + 1/2) / d lies at least 1 / (2 d) >= 2^-9 from an integer, and the
// error of the product stays below 2049 x 2^-22 < 2^-10.
__device__ __forceinline__ int div_small(int x, int d) {
    return (int)(((float)x + 0.5f) * __builtin_amdgcn_rcpf((float)d));
}

// One work item as every thread of the workgroup sees it.  The values are
// the same in every lane (loads of one address); readfirstlane keeps them,
// and the control of the tile loop, in scalar registers (integer division
// and 64-bit compares run on the vector unit).
struct ItemGeo {
    int g, k, g0, ng;
    int S;             // slices of the workgroup-wide layout, 256 / ng
    bool shared;       // lanes (t mod ng, t / ng) across the workgroup, else wave parts
    const GroupLayout* ly;   // the group size's layout
    int clen;          // entries of this item (at most one chunk)
    int64_t nch;       // items of the group's list
    const int32_t* idx;   // the item's entries, idx[0 .. clen)
};

// Decodes queue slot q; false for a malformed group.
template <int TILE>
__device__ __forceinline__ bool decode_item(const ForceArgs& a, int q, ItemGeo& m) {
    const int qi = a.order ? __builtin_amdgcn_readfirstlane(a.order[q]) : q;
    const int2 it = a.items[qi];
    m.g = __builtin_amdgcn_readfirstlane(it.x);
    m.k = __builtin_amdgcn_readfirstlane(it.y);
    m.g0 = __builtin_amdgcn_readfirstlane(a.group_off[m.g]);
    m.ng = __builtin_amdgcn_readfirstlane(a.group_off[m.g + 1]) - m.g0;
    if (m.ng < 1 || m.ng > kBlock || m.g0 < 0 || m.g0 + m.ng > a.n) return false;
    int64_t lb, le;
    list_range(a.list_off, a.n_entries, m.g, lb, le);
    lb = uniform64(lb);
    le = uniform64(le);
    m.nch = n_chunks(le - lb, a.chunk);
    const int64_t cb = lb + (int64_t)m.k * a.chunk;
    const int64_t rest = le - cb;
    m.clen = __builtin_amdgcn_readfirstlane(rest <= 0 ? 0 : (rest < a.chunk ? (int)rest : a.chunk));
    m.idx = a.list_idx + cb;
    const GroupLayout& ly = kLayouts.e[m.ng];
    m.S = ly.S;
    m.shared = (ly.parts & tile_bit<TILE>()) == 0;
    m.ly = &ly;
    return true;
}

// The gather of a tile runs in two stages one tile apart, so that no wave
// waits on memory between tiles: load_idx issues the list-index loads of a
// tile (thread t takes entries base + t + l kBlock; entries past the tile or
// the item are marked absent), and one tile later load_src issues the
// source-record loads for those indices (absent entries are zero mass).
// Waiting for an index load right after issuing it would also wait for every
// load issued before it (the vector memory counter drains in order).
template <int TILE, int L>
__device__ __forceinline__ void load_idx(const ItemGeo& m, int t, int base, int32_t (&j)[L], bool (&has)[L]) {
#pragma unroll
    for (int l = 0; l < L; l++) {
        const int te = t + l * kBlock;
        const int e = base + te;
        has[l] = te < TILE && e < m.clen;
        j[l] = has[l] ? m.idx[e] : 0;
    }
}
template <int L>
__device__ __forceinline__ void load_src(const ForceArgs& a, const int32_t (&j)[L], const bool (&has)[L],
                                         float4 (&pre)[L]) {
    // Every load in flight here is an index load (the previous records were
    // stored to LDS): wait for them in every lane before the branches.  A
    // wait left inside a branch that a wave may skip makes the compiler wait
    // again before the index registers are reloaded, after these record
    // loads are issued, and so for the records as well.
    __builtin_amdgcn_s_waitcnt(0xF70);   // vmcnt(0); expcnt and lgkmcnt not waited for
#pragma unroll
    for (int l = 0; l < L; l++) {
        pre[l] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (has[l]) {
            if (j[l] >= 0 && j[l] < a.n_src) {
                pre[l] = a.src[j[l]];
            } else {
                atomicOr(a.err, kErrIndex);
            }
        }
    }
}

// TILE list entries are staged in LDS per tile (TILE / kBlock per thread),
// followed by kPadRows zero-mass records that the last slice of a target may
// run into (a target's S <= 64 slices of at most ceil(TILE / S) + 1 rows end
// before TILE + 2 S - 1).
template <int TILE>
__device__ __forceinline__ void force_items(const ForceArgs& a) {
    constexpr int L = TILE / kBlock;
    static_assert(L * kBlock == TILE && L >= 1, "tile must be a multiple of the workgroup");
    __shared__ float4 tile[2][TILE + kPadRows];
    __shared__ int s_q;
    const int t = threadIdx.x;
    const int64_t n_items = uniform64(a.meta->n_items < a.item_cap ? a.meta->n_items : a.item_cap);

    for (;;) {
        if (t == 0) s_q = atomicAdd(&a.meta->head, 1);
        __syncthreads();
        const int q = __builtin_amdgcn_readfirstlane(s_q);
        __syncthreads();
        if (q >= n_items) break;
        ItemGeo m;
        if (!decode_item<TILE>(a, q, m)) {
            if (t == 0) atomicOr(a.err, kErrGroup);
            continue;
        }
        const int g = m.g, k = m.k, g0 = m.g0, ng = m.ng;
        const int64_t nch = m.nch;

        // Lanes are (target i, slice sl): the nsl slices of a target split
        // each tile into nsl contiguous runs of `rows` entries, padded with
        // zero-mass entries, so every lane of a wave runs the same trip count.
        // Workgroup-wide, S = 256 / ng slices (thread t: target t mod ng,
        // slice t / ng); or, where that leaves more lanes idle, each wave
        // takes its own part of the targets (part_counts), the parts rotated
        // over the waves from item to item.  The slices of a target sit
        // sstride threads apart.
        int i, sl, nsl, sstride;
        bool active, wave_busy;
        if (m.shared) {
            sl = div_small(t, ng);
            i = t - sl * ng;
            nsl = m.S;
            sstride = ng;
            active = sl < nsl;
            wave_busy = (t & ~63) < nsl * ng;    // some lane of this wave is active
            if (!active) sl = 0;
        } else {
            const int pw = (__builtin_amdgcn_readfirstlane(t >> 6) + q) & 3;
            int pb = 0, pn = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int cj = m.ly->n[j];
                if (j < pw) pb += cj;
                if (j == pw) pn = cj;
            }
            pb = __builtin_amdgcn_readfirstlane(pb);
            pn = __builtin_amdgcn_readfirstlane(pn);
            const int lane = t & 63;
            nsl = pn > 0 ? div_small(64, pn) : 1;
            sstride = pn;
            wave_busy = pn > 0;
            sl = pn > 0 ? div_small(lane, pn) : 0;
            active = wave_busy && sl < nsl;
            i = active ? pb + lane - sl * pn : 0;
            if (!active) sl = 0;
        }
        // Where one wave reads several slices, an odd row count puts their
        // records in different LDS banks (slices of 2^k rows of 16 bytes
        // start in the same bank and serialise the read).  The 128 and 256
        // slices of groups of 2 and 1 keep exact rows.
        const bool skew = m.shared ? (ng & 63) != 0 && nsl <= 64 : nsl > 1;
        const int rows_full = div_small(TILE + nsl - 1, nsl) | (skew ? 1 : 0);
        const float4 xi = a.src[g0 + i];

        float s_ax = 0.f, s_ay = 0.f, s_az = 0.f, s_ph = 0.f;
        float c_ax = 0.f, c_ay = 0.f, c_az = 0.f, c_ph = 0.f;

        // tile 0's records and tile 1's indices in flight
        float4 pre[L];
        int32_t jn[L];
        bool has[L];
        load_idx<TILE>(m, t, 0, jn, has);
        load_src(a, jn, has, pre);
        load_idx<TILE>(m, t, TILE, jn, has);
        int buf = 0;
        for (int tb = 0; tb < m.clen; tb += TILE) {
            const int tl = (m.clen - tb) < TILE ? (m.clen - tb) : TILE;
            const int rows = tl == TILE ? rows_full : div_small(tl + nsl - 1, nsl) | (skew ? 1 : 0);
#pragma unroll
            for (int l = 0; l < L; l++) tile[buf][t + l * kBlock] = pre[l];
            if (t < kPadRows) tile[buf][TILE + t] = make_float4(0.f, 0.f, 0.f, 0.f);
            __syncthreads();
            // the next tile's records (its indices arrived during the previous
            // tile) and the indices of the tile after it load while this tile
            // is summed
            if (tb + TILE < m.clen) {
                load_src(a, jn, has, pre);
                load_idx<TILE>(m, t, tb + 2 * TILE, jn, has);
            }
            float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
            if (wave_busy) {
                const float4* tp = tile[buf] + sl * rows;
#pragma unroll 8
                for (int mm = 0; mm < rows; mm++) pair_mono(xi.x, xi.y, xi.z, tp[mm], a.eps2, ax, ay, az, ph);
            }
            kahan_add(s_ax, c_ax, ax);
            kahan_add(s_ay, c_ay, ay);
            kahan_add(s_az, c_az, az);
            kahan_add(s_ph, c_ph, ph);
            buf ^= 1;
        }
        __syncthreads();  // all reads of the tiles are done before reuse as reduction space

        // combine the j-slices of each target (fixed slice order)
        float* red = reinterpret_cast<float*>(&tile[0][0]);  // >= 2 * 256 float4 = 8 floats per thread
        const bool lead = active && sl == 0;
        if (!m.shared || m.S > 1) {
            red[8 * t + 0] = s_ax;
            red[8 * t + 1] = s_ay;
            red[8 * t + 2] = s_az;
            red[8 * t + 3] = s_ph;
            red[8 * t + 4] = c_ax;
            red[8 * t + 5] = c_ay;
            red[8 * t + 6] = c_az;
            red[8 * t + 7] = c_ph;
            __syncthreads();
            if (lead) {
                for (int s = 1; s < nsl; s++) {
                    const float* r = red + 8 * (t + s * sstride);
                    kahan_add(s_ax, c_ax, r[0] + r[4]);
                    kahan_add(s_ay, c_ay, r[1] + r[5]);
                    kahan_add(s_az, c_az, r[2] + r[6]);
                    kahan_add(s_ph, c_ph, r[3] + r[7]);
                }
            }
        }
        if (lead) {
            const int p = g0 + i;
            if (nch == 1) {
                float ax = s_ax + c_ax, ay = s_ay + c_ay, az = s_az + c_az;
                const float self = xi.w * __builtin_amdgcn_rsqf(a.eps2);
                double phi = -((double)s_ph + (double)c_ph) + (double)self;
                if (a.gcorr) apply_corr(a.gcorr + (int64_t)kCorrStride * g, xi.x, xi.y, xi.z, ax, ay, az, phi);
                a.out_acc[3 * p + 0] = ax;
                a.out_acc[3 * p + 1] = ay;
                a.out_acc[3 * p + 2] = az;
                a.out_pot[p] = phi;
            } else {
                const int64_t row = a.part_base[g] + (int64_t)k * ng + i;
                if (row >= 0 && row < a.part_cap) {
                    a.partial[2 * row] = make_float4(s_ax, s_ay, s_az, s_ph);
                    a.partial[2 * row + 1] = make_float4(c_ax, c_ay, c_az, c_ph);
                } else {
                    atomicOr(a.err, kErrCapacity);
                }
            }
        }
        __syncthreads();  // the reduction space is the next item's tile buffer
    }
}

// Waves per SIMD the compiler is asked to fit: seven at 256- and 512-entry
// tiles (at most 72 VGPRs, no spills; the default budget gave five at
// 512-entry tiles, and seven hide more of the per-item load chain).
// 1024-entry tiles are held to four workgroups per CU by their 36 KB of LDS.
template <int TILE>
struct ForceWaves {
    static constexpr int value = TILE == 1024 ? 1 : 7;
};

template <int TILE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ForceWaves<TILE>::value))) void k_force(
    ForceArgs a) {
    force_items<TILE>(a);
}

// ---------------------------------------------------------------- K3 reduce

// The reduction of particle i of split group g (see k_reduce).
__device__ __forceinline__ void reduce_particle(const float4* __restrict__ src, const int64_t* __restrict__ list_off,
                                                int64_t n_entries, int32_t chunk,
                                                const int64_t* __restrict__ part_base,
                                                const float4* __restrict__ partial, int64_t part_cap, float eps2,
                                                const float* __restrict__ gcorr, int g, int g0, int ng, int i,
                                                float* __restrict__ out_acc, double* __restrict__ out_pot) {
    int64_t lb, le;
    list_range(list_off, n_entries, g, lb, le);
    const int64_t nch = n_chunks(le - lb, chunk);
    if (nch == 1) return;
    const int p = g0 + i;
    float s_ax = 0.f, s_ay = 0.f, s_az = 0.f, c_ax = 0.f, c_ay = 0.f, c_az = 0.f;
    double ph = 0.0;
    for (int64_t k = 0; k < nch; k++) {
        const int64_t row = part_base[g] + k * ng + i;
        if (row < 0 || row >= part_cap) return;
        const float4 s = partial[2 * row];
        const float4 c = partial[2 * row + 1];
        kahan_add(s_ax, c_ax, s.x + c.x);
        kahan_add(s_ay, c_ay, s.y + c.y);
        kahan_add(s_az, c_az, s.z + c.z);
        ph += (double)s.w + (double)c.w;
    }
    const float4 xp = src[p];
    float ax = s_ax + c_ax, ay = s_ay + c_ay, az = s_az + c_az;
    const float self = xp.w * __builtin_amdgcn_rsqf(eps2);
    double phi = -ph + (double)self;
    if (gcorr) apply_corr(gcorr + (int64_t)kCorrStride * g, xp.x, xp.y, xp.z, ax, ay, az, phi);
    out_acc[3 * p + 0] = ax;
    out_acc[3 * p + 1] = ay;
    out_acc[3 * p + 2] = az;
    out_pot[p] = phi;
}

// The groups whose list was split into several items, one workgroup per
// group in turn, one thread per particle: Kahan over the item partials in
// item order (acceleration, FP32) and an FP64 sum for the potential, then the
// self pair is removed.  (The other groups' outputs were written by k_force.)
__global__ __launch_bounds__(256) void k_reduce(const float4* __restrict__ src, const int32_t* __restrict__ group_off,
                                                int32_t n_groups, const int64_t* __restrict__ list_off,
                                                int64_t n_entries, int32_t n, int32_t chunk,
                                                const int64_t* __restrict__ part_base,
                                                const float4* __restrict__ partial, int64_t part_cap, float eps2,
                                                const float* __restrict__ gcorr, const Meta* __restrict__ meta,
                                                const int32_t* __restrict__ split, float* __restrict__ out_acc,
                                                double* __restrict__ out_pot) {
    const int n_split = meta->n_split < n_groups ? meta->n_split : n_groups;
    for (int s = blockIdx.x; s < n_split; s += gridDim.x) {
        const int g = split[s];
        if (g < 0 || g >= n_groups) continue;
        const int g0 = group_off[g];
        const int ng = group_off[g + 1] - g0;
        if (ng < 1 || ng > kBlock || g0 < 0 || g0 + ng > n || (int)threadIdx.x >= ng) continue;
        reduce_particle(src, list_off, n_entries, chunk, part_base, partial, part_cap, eps2, gcorr, g, g0, ng,
                        (int)threadIdx.x, out_acc, out_pot);
    }
}

}  // namespace

// ================================================================ runtime

namespace {

}  // namespace

// Scratch of otoo_force_noalloc: a file-scope device array, one copy per
// GPU, held from the library's load until the process ends.  Host code
// never passes this name to a kernel (on the host it is only a stand-in):
// it uses the device address that hipGetSymbolAddress returns for the
// current device, looked up once per device by otoo_create.
static __device__ __align__(256) unsigned char scratch[OTOO_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (which must be current).
hipError_t noalloc_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_noalloc_ptr[device] = p;
    }
    *out = g_noalloc_ptr[device];
    return hipSuccess;
}

struct Layout {
    size_t src, item_base, part_base, block_tot, items, order, split, partial, total;
    int64_t item_cap, part_cap;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

Layout plan_layout(int32_t n, int32_t n_groups, int64_t n_entries, int32_t n_cells, int32_t chunk) {
    Layout L{};
    const int64_t n_blocks = (n_groups + kScanBlock - 1) / kScanBlock;
    L.item_cap = (int64_t)n_groups + n_entries / chunk + 1;
    // rows are written only for groups split into more than one item; each
    // such group has len > chunk and at most 2 len / chunk items
    const int64_t split_items = std::min<int64_t>(L.item_cap, 2 * (n_entries / chunk) + 1);
    L.part_cap = std::max<int64_t>(1, std::min<int64_t>(split_items * (int64_t)kBlock, (int64_t)n * (n_entries / chunk + 1)));
    size_t off = 0;
    L.src = off;
    off = align_up(off + sizeof(float4) * ((size_t)n + n_cells));
    L.item_base = off;
    off = align_up(off + sizeof(int64_t) * ((size_t)n_groups + 1));
    L.part_base = off;
    off = align_up(off + sizeof(int64_t) * ((size_t)n_groups + 1));
    L.block_tot = off;
    off = align_up(off + 2 * sizeof(int64_t) * ((size_t)n_blocks + 1));
    L.items = off;
    off = align_up(off + sizeof(int2) * (size_t)L.item_cap);
    L.order = off;
    off = align_up(off + sizeof(int32_t) * (size_t)L.item_cap);
    L.split = off;
    off = align_up(off + sizeof(int32_t) * ((size_t)n_groups + 1));
    L.partial = off;
    off = align_up(off + 2 * sizeof(float4) * (size_t)L.part_cap);
    L.total = off;
    return L;
}

int ensure_scratch(otoo_ctx* c, size_t bytes) {
    if (bytes <= c->buf_bytes) return OTOO_OK;
    if (c->scratch_cap && bytes > c->scratch_cap)
        return fail(c, OTOO_ENOMEM, "force scratch of %zu bytes exceeds the cap of %zu", bytes, c->scratch_cap);
    if (c->buf) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        // a captured graph names the old buffer: it cannot be replayed any more
        if (c->gexec) HIP_TRY(c, hipGraphExecDestroy(c->gexec));
        if (c->graph) HIP_TRY(c, hipGraphDestroy(c->graph));
        c->gexec = nullptr;
        c->graph = nullptr;
        HIP_TRY(c, hipFree(c->buf));
        c->buf = nullptr;
        c->buf_bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    if (c->scratch_cap) want = std::min(want, c->scratch_cap);
    if (hipMalloc(&c->buf, want) != hipSuccess) {
        (void)hipGetLastError();
        c->buf = nullptr;
        return fail(c, OTOO_ENOMEM, "device scratch of %zu bytes could not be allocated", want);
    }
    c->buf_bytes = want;
    c->scratch_gen++;
    return OTOO_OK;
}

struct Call {
    int32_t n;
    const float* pos;
    const float* mass;
    int32_t n_groups;
    const int32_t* group_off;
    int64_t n_entries;
    const int64_t* list_off;
    const int32_t* list_idx;
    int32_t n_cells;
    const float* cell_mom;
    int32_t cell_stride;
    float eps;
    const float* gcorr;
    float* out_acc;
    double* out_pot;
};

int check_args(otoo_ctx* c, const Call& a) {
    if (!c) return OTOO_EINVAL;
    if (a.n < 1 || a.n > (1 << 30)) return fail(c, OTOO_EINVAL, "n = %d outside 1..2^30", a.n);
    if (a.n_groups < 1 || a.n_groups > a.n) return fail(c, OTOO_EINVAL, "n_groups = %d outside 1..n", a.n_groups);
    if (a.n_entries < 0) return fail(c, OTOO_EINVAL, "n_entries < 0");
    if (a.n_cells < 0 || (int64_t)a.n + a.n_cells > INT32_MAX)
        return fail(c, OTOO_EINVAL, "n_cells = %d out of range", a.n_cells);
    if (a.cell_stride != 4 && a.cell_stride != 12) return fail(c, OTOO_EINVAL, "cell_stride must be 4 or 12");
    if (!(a.eps > 0.f) || !std::isfinite(a.eps)) return fail(c, OTOO_EINVAL, "eps must be positive and finite");
    if (!a.pos || !a.mass || !a.group_off || !a.list_off || !a.out_acc || !a.out_pot)
        return fail(c, OTOO_EINVAL, "null pointer argument");
    if (a.n_entries > 0 && !a.list_idx) return fail(c, OTOO_EINVAL, "list_idx is null");
    if (a.n_cells > 0 && !a.cell_mom) return fail(c, OTOO_EINVAL, "cell_mom is null");
    return OTOO_OK;
}

// Host-side check of the device CSR (debug mode): copies it back.
int validate_csr(otoo_ctx* c, const Call& a) {
    std::vector<int32_t> go(a.n_groups + 1);
    std::vector<int64_t> lo(a.n_groups + 1);
    std::vector<int32_t> li(a.n_entries);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(go.data(), a.group_off, sizeof(int32_t) * go.size(), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(lo.data(), a.list_off, sizeof(int64_t) * lo.size(), hipMemcpyDeviceToHost));
    if (a.n_entries)
        HIP_TRY(c, hipMemcpy(li.data(), a.list_idx, sizeof(int32_t) * li.size(), hipMemcpyDeviceToHost));
    if (go[0] < 0 || go[a.n_groups] > a.n || go[0] > go[a.n_groups])
        return fail(c, OTOO_EINVAL, "group_off must lie within 0..n");
    if (lo[0] != 0 || lo[a.n_groups] != a.n_entries)
        return fail(c, OTOO_EINVAL, "list_off must run from 0 to n_entries");
    const int64_t n_src = (int64_t)a.n + a.n_cells;
    for (int g = 0; g < a.n_groups; g++) {
        const int ng = go[g + 1] - go[g];
        if (ng < 1 || ng > OTOO_MAX_GROUP) return fail(c, OTOO_EINVAL, "group %d has %d particles", g, ng);
        if (lo[g + 1] < lo[g]) return fail(c, OTOO_EINVAL, "list_off decreases at group %d", g);
        int self = 0;
        for (int64_t e = lo[g]; e < lo[g + 1]; e++) {
            const int32_t j = li[e];
            if (j < 0 || j >= n_src) return fail(c, OTOO_EINVAL, "list entry %lld = %d out of range", (long long)e, j);
            if (j >= go[g] && j < go[g + 1]) self++;
        }
        if (self != ng)
            return fail(c, OTOO_EINVAL, "group %d: list holds %d of its %d own particles", g, self, ng);
    }
    return OTOO_OK;
}

// Launch the force path with its scratch at `buf` (the context's buffer,
// or the no-allocation array), which holds at least the call's layout.
int enqueue(otoo_ctx* c, const Call& a, bool allow_timing, void* buf) {
    const otoo_tuning& tu = c->tune;
    const Layout L = plan_layout(a.n, a.n_groups, a.n_entries, a.n_cells, tu.chunk);
    char* base = static_cast<char*>(buf);
    float4* src = reinterpret_cast<float4*>(base + L.src);
    int64_t* item_base = reinterpret_cast<int64_t*>(base + L.item_base);
    int64_t* part_base = reinterpret_cast<int64_t*>(base + L.part_base);
    int64_t* block_tot = reinterpret_cast<int64_t*>(base + L.block_tot);
    int2* items = reinterpret_cast<int2*>(base + L.items);
    int32_t* order = reinterpret_cast<int32_t*>(base + L.order);
    int32_t* split = reinterpret_cast<int32_t*>(base + L.split);
    float4* partial = reinterpret_cast<float4*>(base + L.partial);
    const float* gcorr = a.gcorr;
    hipStream_t s = c->stream;
    const bool tm = allow_timing && c->timing;

    if (tm) HIP_TRY(c, hipEventRecord(c->ev[0], s));
    const int64_t n_src = (int64_t)a.n + a.n_cells;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((n_src + 255) / 256)), dim3(256), 0, s, a.pos, a.mass, a.n, a.cell_mom,
                       a.n_cells, a.cell_stride, src, c->meta);
    const int n_blocks = (a.n_groups + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_sched_scan1, dim3(n_blocks), dim3(256), 0, s, a.group_off, a.list_off, a.n_entries,
                       a.n_groups, tu.chunk, item_base, part_base, block_tot);
    hipLaunchKernelGGL(k_sched_scan2, dim3(1), dim3(256), 0, s, block_tot, n_blocks, c->meta);
    hipLaunchKernelGGL(k_sched_fill, dim3((a.n_groups + 255) / 256), dim3(256), 0, s, a.group_off, a.list_off,
                       a.n_entries, a.n_groups, tu.chunk, item_base, part_base, block_tot, items, L.item_cap,
                       tu.lpt, c->meta, split, c->errflag);
    if (tu.lpt) {
        const int lpt_grid = (int)std::min<int64_t>(1024, (L.item_cap + 255) / 256);
        hipLaunchKernelGGL(k_lpt_scatter, dim3(lpt_grid), dim3(256), 0, s, items, a.group_off, a.list_off,
                           a.n_entries, tu.chunk, L.item_cap, c->meta, order);
    }
    ForceArgs fa;
    fa.src = src;
    fa.n_src = (int32_t)std::min<int64_t>(n_src, INT32_MAX);
    fa.n = a.n;
    fa.group_off = a.group_off;
    fa.list_off = a.list_off;
    fa.n_entries = a.n_entries;
    fa.list_idx = a.list_idx;
    fa.items = items;
    fa.order = tu.lpt ? order : nullptr;
    fa.item_cap = L.item_cap;
    fa.part_base = part_base;
    fa.partial = partial;
    fa.part_cap = L.part_cap;
    fa.meta = c->meta;
    fa.chunk = tu.chunk;
    fa.eps2 = a.eps * a.eps;
    fa.gcorr = gcorr;
    fa.out_acc = a.out_acc;
    fa.out_pot = a.out_pot;
    fa.err = c->errflag;
    const int grid = c->num_cu * tu.blocks_per_cu;
    if (tm) HIP_TRY(c, hipEventRecord(c->ev[1], s));
    if (tu.tile == 1024)
        hipLaunchKernelGGL(k_force<1024>, dim3(grid), dim3(kBlock), 0, s, fa);
    else if (tu.tile == 512)
        hipLaunchKernelGGL(k_force<512>, dim3(grid), dim3(kBlock), 0, s, fa);
    else
        hipLaunchKernelGGL(k_force<256>, dim3(grid), dim3(kBlock), 0, s, fa);
    if (tm) HIP_TRY(c, hipEventRecord(c->ev[2], s));
    if ((int64_t)tu.chunk < a.n_entries) {   // otherwise no list is split and k_force wrote every output
        const int red_grid = (int)std::min<int64_t>(a.n_groups, 8LL * c->num_cu);
        hipLaunchKernelGGL(k_reduce, dim3(red_grid), dim3(256), 0, s, src, a.group_off, a.n_groups, a.list_off,
                           a.n_entries, a.n, tu.chunk, part_base, partial, L.part_cap, fa.eps2, gcorr, c->meta,
                           split, a.out_acc, a.out_pot);
    }
    HIP_TRY(c, hipGetLastError());
    return OTOO_OK;
}

// The host-side plan of a call: sizes in range and the scratch layout.  The
// queue head, the item table's chunk index and the longest-first order are
// 32-bit: every fetch, including each of the `workgroups` persistent
// workgroups' last one, must stay below 2^31.  Touches no device state.
int plan_call(otoo_ctx* c, int32_t n, int32_t n_groups, int64_t n_entries, int32_t n_cells, int32_t chunk,
              int64_t workgroups, Layout& L) {
    if (n < 1 || n > (1 << 30)) return fail(c, OTOO_EINVAL, "n = %d outside 1..2^30", n);
    if (n_groups < 1 || n_groups > n) return fail(c, OTOO_EINVAL, "n_groups = %d outside 1..n", n_groups);
    if (n_entries < 0) return fail(c, OTOO_EINVAL, "n_entries < 0");
    if (n_cells < 0 || (int64_t)n + n_cells > INT32_MAX) return fail(c, OTOO_EINVAL, "n_cells = %d out of range", n_cells);
    if (chunk < 64 || chunk > (1 << 28)) return fail(c, OTOO_EINVAL, "chunk must be in 64..2^28");
    if (workgroups < 1 || workgroups > (1 << 20)) return fail(c, OTOO_EINVAL, "workgroups out of range");
    L = plan_layout(n, n_groups, n_entries, n_cells, chunk);
    if (L.item_cap + workgroups >= INT32_MAX)
        return fail(c, OTOO_EINVAL, "%lld work items exceed the 32-bit queue; use a longer chunk",
                    (long long)L.item_cap);
    return OTOO_OK;
}

int prepare(otoo_ctx* c, const Call& a) {
    int rc = check_args(c, a);
    if (rc) return rc;
    Layout L;
    rc = plan_call(c, a.n, a.n_groups, a.n_entries, a.n_cells, c->tune.chunk,
                   (int64_t)c->num_cu * c->tune.blocks_per_cu, L);
    if (rc) return rc;
    if (c->tune.debug_validate) {
        rc = validate_csr(c, a);
        if (rc) return rc;
    }
    return ensure_scratch(c, L.total);
}

}  // namespace

extern "C" {

int otoo_create(otoo_ctx** out, int32_t device) {
    if (!out) return OTOO_EINVAL;
    *out = nullptr;
    otoo_ctx* c = new (std::nothrow) otoo_ctx();
    if (!c) return OTOO_ENOMEM;
    c->device = device;
    hipError_t e = hipSetDevice(device);
    int cu = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device);
    void* small = nullptr;
    if (e == hipSuccess) e = hipMalloc(&small, 4096);
    if (e != hipSuccess) {
        delete c;
        (void)hipGetLastError();
        return OTOO_EHIP;
    }
    void* na = nullptr;
    if (noalloc_scratch(device, &na) != hipSuccess) {   // device < 64: the table's size
        (void)hipGetLastError();
        na = nullptr;   // otoo_force_noalloc then reports the missing array
    }
    c->noalloc = na;
    c->num_cu = cu;
    c->meta = static_cast<Meta*>(small);
    c->errflag = reinterpret_cast<int32_t*>(static_cast<char*>(small) + 2048);
    c->sph_meta = static_cast<char*>(small) + 1024;
    if (hipMemset(small, 0, 4096) != hipSuccess) {
        (void)hipFree(small);
        delete c;
        return OTOO_EHIP;
    }
    for (auto& ev : c->ev) {
        if (hipEventCreate(&ev) != hipSuccess) {
            (void)hipFree(small);
            delete c;
            return OTOO_EHIP;
        }
    }
    *out = c;
    return OTOO_OK;
}

int otoo_destroy(otoo_ctx* c) {
    if (!c) return OTOO_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto& ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->buf) (void)hipFree(c->buf);
    if (c->sph_buf) (void)hipFree(c->sph_buf);
    if (c->corr_buf) (void)hipFree(c->corr_buf);
    if (c->meta) (void)hipFree(c->meta);
    delete c;
    return OTOO_OK;
}

int otoo_set_stream(otoo_ctx* c, void* stream) {
    if (!c) return OTOO_EINVAL;
    c->stream = static_cast<hipStream_t>(stream);
    return OTOO_OK;
}

const char* otoo_last_error(const otoo_ctx* c) { return c ? c->err.c_str() : "null context"; }

int otoo_set_tuning(otoo_ctx* c, const otoo_tuning* t) {
    if (!c || !t) return OTOO_EINVAL;
    otoo_tuning nt = c->tune;
    if (t->chunk) nt.chunk = t->chunk;
    if (t->blocks_per_cu) nt.blocks_per_cu = t->blocks_per_cu;
    if (t->tile) nt.tile = t->tile;
    nt.net_kernel = t->net_kernel;
    nt.corr_chunks = t->corr_chunks;
    nt.lpt = t->lpt ? 1 : 0;
    nt.debug_validate = t->debug_validate ? 1 : 0;
    if (nt.chunk < 64 || nt.chunk > (1 << 28)) return fail(c, OTOO_EINVAL, "chunk must be in 64..2^28");
    if (nt.blocks_per_cu < 1 || nt.blocks_per_cu > 16) return fail(c, OTOO_EINVAL, "blocks_per_cu must be in 1..16");
    if (nt.tile != 256 && nt.tile != 512 && nt.tile != 1024) return fail(c, OTOO_EINVAL, "tile must be 256, 512 or 1024");
    if (nt.net_kernel < 0 || nt.net_kernel > 2) return fail(c, OTOO_EINVAL, "net_kernel must be 0, 1 or 2");
    if (nt.corr_chunks < 0 || nt.corr_chunks > 2) return fail(c, OTOO_EINVAL, "corr_chunks must be 0, 1 or 2");
    c->tune = nt;
    return OTOO_OK;
}

int otoo_get_tuning(const otoo_ctx* c, otoo_tuning* t) {
    if (!c || !t) return OTOO_EINVAL;
    *t = c->tune;
    return OTOO_OK;
}

int otoo_set_scratch_limit(otoo_ctx* c, int64_t max_bytes) {
    if (!c) return OTOO_EINVAL;
    if (max_bytes < 0) return fail(c, OTOO_EINVAL, "the scratch cap must not be negative");
    c->scratch_cap = (size_t)max_bytes;
    return OTOO_OK;
}

int otoo_force_plan(int32_t n, int32_t n_groups, int64_t n_entries, int32_t n_cells, int32_t chunk,
                    int32_t workgroups, int64_t* scratch_bytes) {
    Layout L;
    const int rc = plan_call(nullptr, n, n_groups, n_entries, n_cells, chunk, workgroups, L);
    if (rc) return rc;
    if (scratch_bytes) *scratch_bytes = (int64_t)L.total;
    return OTOO_OK;
}

int otoo_group_layout(int32_t ng, int32_t tile, int32_t* wave_parts, int32_t* parts) {
    if (ng < 1 || ng > kBlock || (tile != 256 && tile != 512 && tile != 1024) || !wave_parts || !parts)
        return OTOO_EINVAL;
    static constexpr LayoutTable kHostLayouts = make_layouts();   // the table the kernel reads
    const GroupLayout& e = kHostLayouts.e[ng];
    const int bit = tile == 256 ? 1 : (tile == 512 ? 2 : 4);
    *wave_parts = (e.parts & bit) ? 1 : 0;
    for (int j = 0; j < 4; j++) parts[j] = *wave_parts ? e.n[j] : (j == 0 ? e.S : 0);
    return OTOO_OK;
}

int otoo_scratch_generation(const otoo_ctx* c, int64_t* gen) {
    if (!c || !gen) return OTOO_EINVAL;
    *gen = c->scratch_gen;
    return OTOO_OK;
}

int otoo_force(otoo_ctx* c, int32_t n, const float* pos, const float* mass, int32_t n_groups,
               const int32_t* group_off, int64_t n_entries, const int64_t* list_off, const int32_t* list_idx,
               int32_t n_cells, const float* cell_mom, int32_t cell_stride, float eps, const float* gcorr,
               float* out_acc, double* out_pot) {
    if (!c) return OTOO_EINVAL;
    c->err.clear();
    Call a{n, pos, mass, n_groups, group_off, n_entries, list_off, list_idx, n_cells, cell_mom, cell_stride, eps,
           gcorr, out_acc, out_pot};
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = prepare(c, a);
    if (rc) return rc;
    return enqueue(c, a, true, c->buf);
}

int otoo_force_noalloc(otoo_ctx* c, int32_t n, const float* pos, const float* mass, int32_t n_groups,
                       const int32_t* group_off, int64_t n_entries, const int64_t* list_off,
                       const int32_t* list_idx, int32_t n_cells, const float* cell_mom, int32_t cell_stride,
                       float eps, const float* gcorr, float* out_acc, double* out_pot) {
    if (!c) return OTOO_EINVAL;
    c->err.clear();
    Call a{n, pos, mass, n_groups, group_off, n_entries, list_off, list_idx, n_cells, cell_mom, cell_stride, eps,
           gcorr, out_acc, out_pot};
    int rc = check_args(c, a);
    if (rc) return rc;
    Layout L;
    rc = plan_call(c, a.n, a.n_groups, a.n_entries, a.n_cells, c->tune.chunk,
                   (int64_t)c->num_cu * c->tune.blocks_per_cu, L);
    if (rc) return rc;
    if (L.total > (size_t)OTOO_NOALLOC_SCRATCH_BYTES)
        return fail(c, OTOO_EINVAL,
                    "this call needs %zu bytes of scratch; otoo_force_noalloc holds %zu per GPU (use otoo_force, "
                    "or a longer chunk)",
                    L.total, (size_t)OTOO_NOALLOC_SCRATCH_BYTES);
    if (c->tune.debug_validate)
        return fail(c, OTOO_EINVAL, "debug validation copies the lists to the host; it is off for otoo_force_noalloc");
    if (!c->noalloc) return fail(c, OTOO_EHIP, "the scratch array of device %d could not be located", c->device);
    HIP_TRY(c, hipSetDevice(c->device));
    return enqueue(c, a, true, c->noalloc);
}

int otoo_quad_exact(otoo_ctx* c, int32_t n, int32_t n_groups, int64_t n_entries, const int64_t* list_off,
                    const int32_t* list_idx, int64_t n_pairs, const int64_t* pair_off, int32_t n_cells,
                    const float* cell_mom, int32_t cell_stride, float* corr) {
    if (!c) return OTOO_EINVAL;
    c->err.clear();
    if (n < 1 || n_groups < 1 || n_entries < 0 || n_pairs < 0 || n_pairs > n_entries || n_cells < 0)
        return fail(c, OTOO_EINVAL, "bad sizes");
    if (cell_stride != 12) return fail(c, OTOO_EINVAL, "the quadrupole needs cell moments of stride 12");
    if (!list_off || !pair_off || (n_entries && !list_idx) || (n_cells && !cell_mom) || (n_pairs && !corr))
        return fail(c, OTOO_EINVAL, "null pointer argument");
    if (n_pairs == 0) return OTOO_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_quad_exact, dim3(n_groups), dim3(256), 0, c->stream, n, n_groups, list_off, n_entries,
                       list_idx, pair_off, n_pairs, n_cells, cell_mom, corr, c->errflag);
    HIP_TRY(c, hipGetLastError());
    return OTOO_OK;
}

int otoo_check(otoo_ctx* c) {
    if (!c) return OTOO_EINVAL;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int32_t f = 0;
    HIP_TRY(c, hipMemcpy(&f, c->errflag, sizeof f, hipMemcpyDeviceToHost));
    if (f) {
        const int32_t zero = 0;
        HIP_TRY(c, hipMemcpy(c->errflag, &zero, sizeof zero, hipMemcpyHostToDevice));
        return fail(c, OTOO_EINVAL, "malformed device input skipped (flags 0x%x:%s%s%s)", f,
                    (f & kErrGroup) ? " group size" : "", (f & kErrIndex) ? " list index" : "",
                    (f & kErrCapacity) ? " capacity" : "");
    }
    return OTOO_OK;
}

int otoo_enable_timing(otoo_ctx* c, int32_t enable) {
    if (!c) return OTOO_EINVAL;
    c->timing = enable != 0;
    return OTOO_OK;
}

int otoo_last_timing(otoo_ctx* c, float* ms_kernel, float* ms_total) {
    if (!c) return OTOO_EINVAL;
    if (!c->timing) return fail(c, OTOO_EINVAL, "timing is not enabled");
    HIP_TRY(c, hipEventSynchronize(c->ev[2]));
    float k = 0, t = 0;
    HIP_TRY(c, hipEventElapsedTime(&k, c->ev[1], c->ev[2]));
    HIP_TRY(c, hipEventElapsedTime(&t, c->ev[0], c->ev[2]));
    if (ms_kernel) *ms_kernel = k;
    if (ms_total) *ms_total = t;
    return OTOO_OK;
}

int otoo_graph_capture(otoo_ctx* c, int32_t n, const float* pos, const float* mass, int32_t n_groups,
                       const int32_t* group_off, int64_t n_entries, const int64_t* list_off,
                       const int32_t* list_idx, int32_t n_cells, const float* cell_mom, int32_t cell_stride,
                       float eps, const float* gcorr, float* out_acc, double* out_pot) {
    if (!c) return OTOO_EINVAL;
    c->err.clear();
    Call a{n, pos, mass, n_groups, group_off, n_entries, list_off, list_idx, n_cells, cell_mom, cell_stride, eps,
           gcorr, out_acc, out_pot};
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = prepare(c, a);  // all allocation happens before capture
    if (rc) return rc;
    if (c->gexec) {
        HIP_TRY(c, hipGraphExecDestroy(c->gexec));
        c->gexec = nullptr;
    }
    if (c->graph) {
        HIP_TRY(c, hipGraphDestroy(c->graph));
        c->graph = nullptr;
    }
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue(c, a, false, c->buf);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = user;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(c, OTOO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    c->graph = g;
    HIP_TRY(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    return OTOO_OK;
}

int otoo_graph_launch(otoo_ctx* c) {
    if (!c) return OTOO_EINVAL;
    if (!c->gexec) return fail(c, OTOO_EINVAL, "no graph captured (or the context's scratch grew since the capture)");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
    return OTOO_OK;
}

}  // extern "C"
