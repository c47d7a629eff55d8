// SPH-style gather sums over neighbour lists (Sec. 2.3, Eq. 4): the second
// workload on the group/list machinery of the gravity path.  Particles only,
// no cells (a cell is opened or skipped whole by the SPH walk).
#include <algorithm>
#include <atomic>

#include "otoo_internal.h"

using namespace otoo_detail;

namespace {

constexpr int kSphPer = 2;                   // list entries each thread gathers per tile
constexpr int kSphCap = kSphPer * kBlock;    // records per LDS tile buffer
constexpr float kInvPi = 0.318309886183790672f;
constexpr float kCbrt4 = 1.58740105196819947f;       // k with k^3 = 4
constexpr float kHalfCbrt4 = 0.793700525984099737f;  // k / 2

// Half the cubic B-spline shape at u = r/h: w(u) = 1 - 6u^2 + 6u^3 on
// [0, 1/2], 2 (1 - u)^3 on [1/2, 1], 0 beyond, equals 2 a^3 - 8 b^3 with
// a = max(1 - u, 0), b = max(1/2 - u, 0) (the truncated cubics agree with
// the pieces).  With b' = k b, k^3 = 4, that is 2 (a^3 - b'^3); this returns
// a^3 - b'^3, the factor 2 being carried by the source weights.
__device__ __forceinline__ float spline_half(float r, float ih, float kih) {
    const float a = fmaxf(fmaf(-ih, r, 1.f), 0.f);
    const float b = fmaxf(fmaf(-kih, r, kHalfCbrt4), 0.f);
    return fmaf(a * a, a, -(b * b) * b);
}

// Source record of one list entry as staged in LDS: position and 1/h, then
// 2q and 2q sigma (sigma = 8 / (pi h^3)).  Entries that are not particles,
// and the padding of a tile, get zero weights.
struct SphRec {
    float4 x;
    float2 w;
};

// A 64-bit value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ int64_t sph_uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A tile's records are gathered in three steps, each one tile after the
// previous: the list indices (sph_load_idx), the raw particle data for those
// indices (sph_load_raw), and the record itself (sph_make_rec, the
// arithmetic on the raw data, as the tile is written to LDS).  Waiting for a
// load right after issuing it would also wait for every earlier load (the
// vector memory counter drains in order); the lag leaves no wait between
// tiles.  Entries that are absent or out of range get zero weights and h = 1.
struct SphRaw {
    float x, y, z, h, q;
};

__device__ __forceinline__ void sph_load_idx(const int32_t* __restrict__ list_idx, int64_t lb, int64_t len, int ts,
                                             int t, int64_t base, int32_t (&j)[kSphPer], bool (&has)[kSphPer]) {
#pragma unroll
    for (int p = 0; p < kSphPer; p++) {
        const int e = p * kBlock + t;
        has[p] = e < ts && base + e < len;
        j[p] = has[p] ? list_idx[lb + base + e] : 0;
    }
}

__device__ __forceinline__ void sph_load_raw(const float* __restrict__ pos, const float* __restrict__ hh,
                                             const float* __restrict__ q, int32_t n, int32_t* err,
                                             const int32_t (&j)[kSphPer], const bool (&has)[kSphPer],
                                             SphRaw (&raw)[kSphPer]) {
#pragma unroll
    for (int p = 0; p < kSphPer; p++) {
        raw[p] = SphRaw{0.f, 0.f, 0.f, 1.f, 0.f};
        if (has[p]) {
            if (j[p] >= 0 && j[p] < n) {
                raw[p] = SphRaw{pos[3 * j[p]], pos[3 * j[p] + 1], pos[3 * j[p] + 2], hh[j[p]], q[j[p]]};
            } else {
                atomicOr(err, kErrIndex);
            }
        }
    }
}

__device__ __forceinline__ SphRec sph_make_rec(const SphRaw& r) {
    const float ih = 1.f / r.h;
    const float q2 = 2.f * r.q;
    SphRec c;
    c.x = make_float4(r.x, r.y, r.z, ih);
    c.w = make_float2(q2, q2 * (8.f * kInvPi) * ih * ih * ih);
    return c;
}

// A group's particle range and list range (uniform across the workgroup).
struct Geo {
    int g0, ng;
    int64_t lb, len;
    bool ok;
};

__device__ __forceinline__ Geo load_geo(int g, int32_t n, const int32_t* __restrict__ group_off, int64_t n_entries,
                                        const int64_t* __restrict__ list_off) {
    Geo c;
    c.g0 = group_off[g];
    c.ng = group_off[g + 1] - c.g0;
    c.ok = c.ng >= 1 && c.ng <= kBlock && c.g0 >= 0 && c.g0 + c.ng <= n;
    int64_t le;
    list_range(list_off, n_entries, g, c.lb, le);
    c.len = le - c.lb;
    return c;
}

// Slices of a group of ng targets and the entries per tile (a multiple of
// the slice count).
__device__ __forceinline__ int slices(int ng) { return kBlock / ng; }
__device__ __forceinline__ int tile_len(int ng) {
    const int S = slices(ng);
    return S * (kSphCap / S);
}

// Work items.  A list longer than a quarter chunk is a "long" group: its
// list is cut into chunks of C entries, each an item (g, k, m, nc) with nc
// the chunk count and m the group's slot among the split groups (nc > 1) or
// -1; these items are taken first.  Every other group is one "short" item.
// Chunk partials of a split group go to slots base_m + k ng + i and are
// summed in chunk order by k_sph_merge.
struct SphMeta {
    int32_t head;                 // next item of the queue
    int32_t n_long;               // long items
    int32_t n_short;              // short items
    int32_t n_split;              // split groups
    unsigned long long n_parts;   // partial slots handed out
};

struct SphPlan {
    SphMeta* meta;
    int32_t chunk;
    int64_t cap_long, cap_split, cap_parts;
    int4* items_long;
    int32_t* items_short;
    int32_t* split_g;
    int64_t* split_base;
    float2* parts;
};

__global__ void k_sph_reset(SphMeta* m) {
    if (threadIdx.x == 0) {
        m->head = 0;
        m->n_long = 0;
        m->n_short = 0;
        m->n_split = 0;
        m->n_parts = 0;
    }
}

// One thread per group: classify it and append its items (wave-aggregated
// appends for the short ones).
__global__ __launch_bounds__(256) void k_sph_plan(SphPlan pl, int32_t n, int32_t n_groups,
                                                  const int32_t* __restrict__ group_off, int64_t n_entries,
                                                  const int64_t* __restrict__ list_off, int32_t* err) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool valid = g < n_groups;
    Geo c{};
    if (valid) {
        c = load_geo(g, n, group_off, n_entries, list_off);
        if (!c.ok) {
            atomicOr(err, kErrGroup);
            valid = false;
        }
    }
    const int C = pl.chunk;
    const bool is_long = valid && c.len > C / 4;
    const bool is_short = valid && !is_long;
    const unsigned long long mask = __ballot(is_short);
    if (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&pl.meta->n_short, __popcll(mask));
        base = __shfl(base, leader);
        if (is_short) pl.items_short[base + __popcll(mask & ((1ull << lane) - 1))] = g;
    }
    if (is_long) {
        const int nc = (int)((c.len + C - 1) / C);
        int m = -1;
        if (nc > 1) {
            m = atomicAdd(&pl.meta->n_split, 1);
            const unsigned long long pb = atomicAdd(&pl.meta->n_parts, (unsigned long long)nc * c.ng);
            if (m >= pl.cap_split) {
                atomicOr(err, kErrCapacity);
                return;
            }
            if ((int64_t)(pb + (unsigned long long)nc * c.ng) > pl.cap_parts) {
                pl.split_g[m] = -1;   // k_sph_merge skips the slot
                atomicOr(err, kErrCapacity);
                return;
            }
            pl.split_g[m] = g;
            pl.split_base[m] = (int64_t)pb;
        }
        const int base = atomicAdd(&pl.meta->n_long, nc);
        const bool fits = (int64_t)base + nc <= pl.cap_long;
        if (!fits) atomicOr(err, kErrCapacity);
        for (int k = 0; k < nc && (int64_t)base + k < pl.cap_long; k++)   // slots in range are always written
            pl.items_long[base + k] = fits ? make_int4(g, k, m, nc) : make_int4(-2, 0, -1, 0);
    }
}

// Persistent workgroups pull items from the queue (long items first), a
// batch of consecutive items per atomic.  Per
// item, lanes are (target, slice): with ng targets, S = 256 / ng slices;
// slice s of a staged tile takes entries s, s + S, s + 2S, ..., so the
// slices that share a wave read consecutive records (no bank conflicts) and
// every lane runs the same trip count (the tail is zero-weight padding).
// Tiles are double-buffered: each thread gathers its entries of the next
// tile while the workgroup sums the current one.  Per target the slices'
// partial sums are combined in slice order, so results are reproducible.
// Sums A = sum q_j w(r/h_i) and B = sum q_j sigma_j w(r/h_j) give
// out_i = (sigma_i A + B) / 2 with sigma = 8 / (pi h^3).
__global__ __launch_bounds__(kBlock) void k_sph(SphPlan pl, int32_t batch, int32_t n, const float* __restrict__ pos,
                                                const float* __restrict__ hh, const float* __restrict__ q,
                                                int32_t n_groups, const int32_t* __restrict__ group_off,
                                                int64_t n_entries,
                                                const int64_t* __restrict__ list_off,
                                                const int32_t* __restrict__ list_idx, float* __restrict__ out,
                                                int32_t* err) {
    __shared__ float4 sX[2][kSphCap];   // x, y, z, 1/h
    __shared__ float2 sW[2][kSphCap];   // 2q, 2q sigma
    __shared__ float2 red[kBlock];
    __shared__ int4 s_item;
    const int t = threadIdx.x;
    const int n_long = (int)std::min<int64_t>(pl.meta->n_long, pl.cap_long);
    const int n_items = n_long + pl.meta->n_short;
    int next_it = 0, batch_left = 0;   // thread 0's batch of consecutive items
    for (;;) {
        if (t == 0) {
            if (batch_left == 0) {   // one atomic per batch: a single counter serves every workgroup
                next_it = atomicAdd(&pl.meta->head, batch);
                batch_left = batch;
            }
            const int it = next_it++;
            batch_left--;
            s_item = it < n_long    ? pl.items_long[it]
                     : it < n_items ? make_int4(pl.items_short[it - n_long], 0, -1, 1)
                                    : make_int4(-1, 0, -1, 0);
        }
        __syncthreads();
        // the same item for every thread; readfirstlane makes that visible to the
        // compiler, so the item loop and its exits are wave-uniform scalar branches
        const int4 si = s_item;
        const int4 item = make_int4(__builtin_amdgcn_readfirstlane(si.x), __builtin_amdgcn_readfirstlane(si.y),
                                    __builtin_amdgcn_readfirstlane(si.z), __builtin_amdgcn_readfirstlane(si.w));
        if (item.x == -1) break;
        const bool bad = item.x < 0 || item.x >= n_groups || (item.w > 1 && (item.z < 0 || item.z >= pl.cap_split));
        const Geo c = bad ? Geo{} : load_geo(item.x, n, group_off, n_entries, list_off);
        if (bad || !c.ok) {   // a slot of a failed plan: nothing to sum
            __syncthreads();  // every thread has read s_item before it is rewritten
            continue;
        }
        // the group's ranges are uniform too (loads of one address); readfirstlane
        // keeps them, the slice count and the tile length in scalar registers
        const int g0 = __builtin_amdgcn_readfirstlane(c.g0);
        const int ng = __builtin_amdgcn_readfirstlane(c.ng);
        const int S = __builtin_amdgcn_readfirstlane(slices(ng));
        const int ts = __builtin_amdgcn_readfirstlane(tile_len(ng));
        const int64_t e0 = (int64_t)item.y * pl.chunk;
        const int64_t e1 = std::min<int64_t>(c.len, e0 + pl.chunk);
        const int len = __builtin_amdgcn_readfirstlane((int)std::max<int64_t>(e1 - e0, 0));   // <= chunk
        const int64_t lb = sph_uniform64(c.lb + e0);
        const int ti = t % ng, sl = t / ng;
        const int i = g0 + ti;
        const float xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        const float ihi = 1.f / hh[i];
        const float kihi = kCbrt4 * ihi;
        float A = 0.f, B = 0.f;
        // tile 0's raw data and tile 1's indices in flight
        int32_t jn[kSphPer];
        bool has[kSphPer];
        SphRaw raw[kSphPer];
        sph_load_idx(list_idx, lb, len, ts, t, 0, jn, has);
        sph_load_raw(pos, hh, q, n, err, jn, has, raw);
        sph_load_idx(list_idx, lb, len, ts, t, ts, jn, has);
        int cur = 0;
        for (int base = 0; base < len; base += ts) {
            const int tl = (len - base) < ts ? (len - base) : ts;
            const int rows = __builtin_amdgcn_readfirstlane((tl + S - 1) / S);   // rows * S <= ts: inside the tile
#pragma unroll
            for (int p = 0; p < kSphPer; p++) {
                const SphRec rec = sph_make_rec(raw[p]);   // entries at or beyond tl are zero weight
                sX[cur][p * kBlock + t] = rec.x;
                sW[cur][p * kBlock + t] = rec.w;
            }
            __syncthreads();
            // the next tile's raw data (its indices arrived during the previous
            // tile) and the indices of the tile after it load while this tile
            // is summed
            if (base + ts < len) {
                sph_load_raw(pos, hh, q, n, err, jn, has, raw);
                sph_load_idx(list_idx, lb, len, ts, t, base + 2 * ts, jn, has);
            }
            if (sl < S) {
                const float4* xp = sX[cur] + sl;
                const float2* wp = sW[cur] + sl;
#pragma unroll 4
                for (int m = 0; m < rows; m++) {
                    const float4 s4 = xp[m * S];
                    const float2 w2 = wp[m * S];
                    const float dx = s4.x - xi, dy = s4.y - yi, dz = s4.z - zi;
                    const float rr = __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
                    A = fmaf(w2.x, spline_half(rr, ihi, kihi), A);
                    B = fmaf(w2.y, spline_half(rr, s4.w, kCbrt4 * s4.w), B);
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
            if (item.w == 1) {
                const float sig = (8.f * kInvPi) * ihi * ihi * ihi;
                out[g0 + t] = 0.5f * fmaf(sig, a, b);
            } else {
                pl.parts[pl.split_base[item.z] + (int64_t)item.y * ng + t] = make_float2(a, b);
            }
        }
    }
}

// Split groups: chunk partials summed in chunk order, then the output.
__global__ __launch_bounds__(kBlock) void k_sph_merge(SphPlan pl, int32_t n, const float* __restrict__ hh,
                                                      int32_t n_groups, const int32_t* __restrict__ group_off,
                                                      int64_t n_entries, const int64_t* __restrict__ list_off,
                                                      float* __restrict__ out) {
    const int n_split = pl.meta->n_split;
    const int t = threadIdx.x;
    for (int m = blockIdx.x; m < n_split && m < pl.cap_split; m += gridDim.x) {
        const int g = pl.split_g[m];
        if (g < 0 || g >= n_groups) continue;
        const Geo c = load_geo(g, n, group_off, n_entries, list_off);
        if (!c.ok || t >= c.ng) continue;
        const int nc = (int)((c.len + pl.chunk - 1) / pl.chunk);
        const float2* pp = pl.parts + pl.split_base[m] + t;
        float a = 0.f, b = 0.f;
        for (int k = 0; k < nc; k++) {
            const float2 v = pp[(int64_t)k * c.ng];
            a += v.x;
            b += v.y;
        }
        const float ih = 1.f / hh[c.g0 + t];
        out[c.g0 + t] = 0.5f * fmaf((8.f * kInvPi) * ih * ih * ih, a, b);
    }
}

int ensure_sph_scratch(otoo_ctx* c, size_t bytes) {
    if (bytes <= c->sph_bytes) return OTOO_OK;
    if (c->scratch_cap && bytes > c->scratch_cap)
        return fail(c, OTOO_ENOMEM, "SPH scratch of %zu bytes exceeds the cap of %zu", bytes, c->scratch_cap);
    if (c->sph_buf) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipFree(c->sph_buf));
        c->sph_buf = nullptr;
        c->sph_bytes = 0;
    }
    const size_t want = c->scratch_cap ? std::min(bytes + bytes / 4, c->scratch_cap) : bytes + bytes / 4;
    if (hipMalloc(&c->sph_buf, want) != hipSuccess) {
        (void)hipGetLastError();
        c->sph_buf = nullptr;
        return fail(c, OTOO_ENOMEM, "SPH scratch of %zu bytes could not be allocated", want);
    }
    c->sph_bytes = want;
    c->scratch_gen++;
    return OTOO_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

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
    // Chunk length: 2048 entries, doubled until the partial slots of the
    // split groups (at most 2 kBlock n_entries / C) fit in max(8 n, 2^20).
    const int64_t budget = std::max<int64_t>(8LL * n, 1LL << 20);
    int64_t C = 2048;
    while (2LL * kBlock * (n_entries / C + 1) > budget) C *= 2;
    SphPlan pl{};
    pl.chunk = (int32_t)C;
    pl.cap_long = 5 * (n_entries / C) + n_groups / 64 + 1;
    pl.cap_split = n_entries / C + 1;
    pl.cap_parts = 2LL * kBlock * (n_entries / C + 1);
    const size_t o_short = align256(sizeof(int4) * (size_t)pl.cap_long);
    const size_t o_sg = o_short + align256(sizeof(int32_t) * (size_t)n_groups);
    const size_t o_sb = o_sg + align256(sizeof(int32_t) * (size_t)pl.cap_split);
    const size_t o_parts = o_sb + align256(sizeof(int64_t) * (size_t)pl.cap_split);
    const size_t total = o_parts + sizeof(float2) * (size_t)pl.cap_parts;
    int rc = ensure_sph_scratch(c, total);
    if (rc) return rc;
    char* b = static_cast<char*>(c->sph_buf);
    pl.meta = static_cast<SphMeta*>(c->sph_meta);
    pl.items_long = reinterpret_cast<int4*>(b);
    pl.items_short = reinterpret_cast<int32_t*>(b + o_short);
    pl.split_g = reinterpret_cast<int32_t*>(b + o_sg);
    pl.split_base = reinterpret_cast<int64_t*>(b + o_sb);
    pl.parts = reinterpret_cast<float2*>(b + o_parts);
    // resident workgroups of k_sph per CU (the same for every device of this build)
    static std::atomic<int> occ{0};
    int per_cu = occ.load(std::memory_order_relaxed);
    if (!per_cu) {
        HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sph, kBlock, 0));
        per_cu = std::max(per_cu, 1);
        occ.store(per_cu, std::memory_order_relaxed);
    }
    hipLaunchKernelGGL(k_sph_reset, dim3(1), dim3(64), 0, c->stream, pl.meta);
    hipLaunchKernelGGL(k_sph_plan, dim3((n_groups + 255) / 256), dim3(256), 0, c->stream, pl, n, n_groups, group_off,
                       n_entries, list_off, c->errflag);
    // items per queue access: at least 16 batches per workgroup (there are at least n_groups items)
    const int blocks = per_cu * c->num_cu;
    const int batch = (int)std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)n_groups / (16LL * blocks)));
    hipLaunchKernelGGL(k_sph, dim3(blocks), dim3(kBlock), 0, c->stream, pl, batch, n, pos, h, q, n_groups, group_off,
                       n_entries, list_off, list_idx, out, c->errflag);
    const int merge_blocks = (int)std::min<int64_t>(4LL * c->num_cu, pl.cap_split);
    hipLaunchKernelGGL(k_sph_merge, dim3(merge_blocks), dim3(kBlock), 0, c->stream, pl, n, h, n_groups, group_off,
                       n_entries, list_off, out);
    HIP_TRY(c, hipGetLastError());
    return OTOO_OK;
}
