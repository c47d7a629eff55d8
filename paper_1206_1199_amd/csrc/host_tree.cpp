// Host-side octree build and grouped tree walk (C++17 / OpenMP).
//
// Tree construction follows the four steps of Sec. 3.2 of the paper: the root
// cube from the particles' bounding box, one key per particle (21-bit integer
// coordinates per axis turned into a 63-bit Hilbert key), a parallel sort of
// (key, id) pairs, and the cells read off the sorted keys by slicing equal key
// prefixes level by level.  Cells and particles share one integer index space
// (particles 0..n-1 in key order, cell c at n + c) and are linked by "next"
// (brother, else the parent's next) and "more" (first child, or a leaf's first
// particle) pointers as in Sec. 2.1.  Cell moments (Sec. 3.3) are formed bottom
// up: mass and centre of mass, the second-moment tensor S whose trace is the
// B2 of Eq. (2) (combined through the parallel-axis theorem), and b_max.
//
// The walk (Sec. 2.1 rules 1-4, vectorised over a group of targets as in
// Sec. 3.4) runs one stackless next/more traversal per group of particles on
// the host and emits the group's interaction list: accepted cells first, then
// the particles of opened leaves, each part ascending.
#include "otoo.h"

#include <omp.h>
#include <parallel/algorithm>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

namespace {

constexpr int kBits = 21;                       // bits per axis of the integer coordinates
constexpr int kMaxLevel = kBits;                // cells stop splitting at this depth
constexpr uint32_t kCoordMax = (1u << kBits) - 1u;

// Hilbert index of 3-D integer coordinates with kBits bits per axis, following
// J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707 (2004):
// the coordinates are first transformed in place to the "transpose" form of
// the index (undo excess work, then Gray-encode), whose bits read across the
// three axes from the top give the index three bits per level.
inline uint64_t hilbert_key(uint32_t x0, uint32_t x1, uint32_t x2) {
    uint32_t X[3] = {x0, x1, x2};
    const uint32_t M = 1u << (kBits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; i++) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; i++) X[i] ^= t;
    uint64_t key = 0;
    for (int q = kBits - 1; q >= 0; q--)
        key = (key << 3) | (uint64_t((X[0] >> q) & 1u) << 2) | (uint64_t((X[1] >> q) & 1u) << 1) |
              uint64_t((X[2] >> q) & 1u);
    return key;
}

}  // namespace

namespace {
struct WalkCell;
}

// Walk inputs that depend only on the tree and the opening criterion (the
// per-cell records) or the grouping (group offsets).  They are kept on the
// tree, so that a step walked in batches of groups builds them once; the
// shared pointers keep a set alive for a walk that is still using it.
struct WalkCache {
    std::mutex mu;
    int mac = -1;
    double theta = 0.0, delta = 0.0, m_limit = 0.0;
    std::shared_ptr<const std::vector<WalkCell>> cells;
    int gmode = -1, gmax = -1;
    std::shared_ptr<const std::vector<int64_t>> goff;
};

struct otoo_tree {
    int64_t n = 0;
    double lo[3] = {0, 0, 0};
    double side = 1.0;
    std::vector<int64_t> perm;     // key order k -> original particle id
    std::vector<double> pos;       // [n][3] in key order
    std::vector<double> mass;      // [n] in key order
    std::vector<uint32_t> icoord;  // [n][3] integer coordinates in key order
    std::vector<uint64_t> key;     // [n] sorted Hilbert keys
    // cells in preorder
    std::vector<int64_t> first, count;
    std::vector<int32_t> level;
    std::vector<int32_t> nchild;
    std::vector<int64_t> child0;   // id of first child (children are consecutive in a child table)
    std::vector<int64_t> children; // child table
    std::vector<uint32_t> ijk;     // [n_cells][3] integer cube coordinates at the cell's level
    // links in the unified index space (-1 = null)
    std::vector<int64_t> next;     // [n + n_cells]
    std::vector<int64_t> more;     // [n + n_cells]
    // moments
    std::vector<double> M, com, S6, s, bmax, centre, csize;
    int32_t depth = 0;
    mutable WalkCache cache;
    int64_t n_cells() const { return (int64_t)first.size(); }
};

struct otoo_lists_impl {
    otoo_lists pub;
    std::vector<int32_t> group_off, n_cellent, n_near;
    std::unique_ptr<int32_t[]> list_idx;
    std::vector<int64_t> list_off;
    std::vector<float> group_box;  // [G][6] lo xyz, hi xyz (FP32, rounded outward is not needed: informative)
};

namespace {

int64_t build_cells(otoo_tree& t, int64_t lo, int64_t hi, int level, int n_crit,
                    std::vector<std::vector<int64_t>>& kids) {
    const int64_t c = t.n_cells();
    t.first.push_back(lo);
    t.count.push_back(hi - lo);
    t.level.push_back(level);
    const int sh = kBits - level;
    t.ijk.push_back(t.icoord[3 * lo + 0] >> sh);
    t.ijk.push_back(t.icoord[3 * lo + 1] >> sh);
    t.ijk.push_back(t.icoord[3 * lo + 2] >> sh);
    kids.emplace_back();
    if (level > t.depth) t.depth = level;
    if (hi - lo <= n_crit || level >= kMaxLevel) return c;
    // children: runs of equal 3-bit digit at depth level+1
    const int dshift = 3 * (kBits - level - 1);
    int64_t a = lo;
    while (a < hi) {
        const uint64_t digit = (t.key[a] >> dshift) & 7u;
        // first index in [a, hi) whose digit differs (keys are sorted, digits ascend)
        int64_t b = std::partition_point(t.key.begin() + a, t.key.begin() + hi,
                                         [&](uint64_t k) { return ((k >> dshift) & 7u) == digit; }) -
                    t.key.begin();
        const int64_t ch = build_cells(t, a, b, level + 1, n_crit, kids);
        kids[c].push_back(ch);
        a = b;
    }
    return c;
}

enum WalkAction { kOpen = 0, kAccept = 1, kSkip = 2 };

// groups: contiguous ranges of key order, returned as offsets (size G + 1)
std::vector<int64_t> make_groups(const otoo_tree* t, int mode, int G) {
    const int64_t n = t->n;
    std::vector<int64_t> goff;
    if (mode == OTOO_GROUP_CHUNK) {
        for (int64_t a = 0; a < n; a += G) goff.push_back(a);
    } else {
        // maximal cells with at most G particles, found in preorder; a leaf
        // above G (only possible at the depth cap) is cut into chunks
        std::vector<int64_t> stack{0};
        while (!stack.empty()) {
            const int64_t c = stack.back();
            stack.pop_back();
            if (t->count[c] <= G) {
                goff.push_back(t->first[c]);
            } else if (t->nchild[c] == 0) {
                for (int64_t a = t->first[c]; a < t->first[c] + t->count[c]; a += G) goff.push_back(a);
            } else {
                for (int k = t->nchild[c] - 1; k >= 0; k--) stack.push_back(t->children[t->child0[c] + k]);
            }
        }
    }
    goff.push_back(n);
    if ((int64_t)goff.size() - 1 > INT32_MAX) throw std::bad_alloc();
    return goff;
}

// Per-cell record of the walk, packed into one cache line: COM, two radii
// for the opening criterion, the next/more links and the particle range.
struct alignas(64) WalkCell {
    double com[3];
    double ra, rb;     // criterion radii (meaning set by the caller)
    int64_t next, more;
    int64_t first;     // first particle (key order)
    int32_t count;     // particles in the cell
    int32_t leaf;      // no children
};

std::vector<WalkCell> walk_cells(const otoo_tree* t) {
    const int64_t n = t->n, nc = t->n_cells();
    std::vector<WalkCell> w(nc);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; c++) {
        WalkCell& x = w[c];
        for (int k = 0; k < 3; k++) x.com[k] = t->com[3 * c + k];
        x.ra = x.rb = 0.0;
        x.next = t->next[n + c];
        x.more = t->more[n + c];
        x.first = t->first[c];
        x.count = (int32_t)t->count[c];
        x.leaf = t->nchild[c] == 0;
    }
    return w;
}

// The stackless next/more walk of every group.  decide(cell, d_min, g) says
// what to do with a cell, where d_min is the distance from the cell's COM to
// the group's bounding box: open it, accept it as one entry, or skip it.  An
// opened leaf contributes its particles (a contiguous key range, the same
// entries its more/next chain visits) without visiting them one by one.
// Lists hold the accepted cells, then the particles, each part in walk
// (ascending) order.  With near_ratio > 0 the accepted cells are split,
// each part still ascending: first the near ones, whose side l_c is at least
// near_ratio times the distance from the cell's COM to the centre of the
// group's bounding box (FP64), then the others; n_near counts the first
// part.  Threads take groups in chunks of 8; each keeps its lists in its own
// buffer until they are gathered into one CSR.
template <class Decide>
void walk_groups(const otoo_tree* t, const std::vector<int64_t>& goff, const std::vector<WalkCell>& cells,
                 Decide decide, otoo_lists_impl* L, double near_ratio = 0.0) {
    const int64_t n = t->n;
    const int64_t ng = (int64_t)goff.size() - 1;
    const int nth = omp_get_max_threads();
    std::vector<std::vector<int32_t>> buf(nth);
    std::vector<int64_t> g_thread(ng), g_start(ng), g_ncell(ng), g_nnear(ng), g_len(ng);
    L->group_box.resize(6 * (size_t)ng);
    // an exception cannot leave an OpenMP region: a failed allocation inside
    // it is recorded here and rethrown after the region
    std::atomic<bool> out_of_memory{false};
#pragma omp parallel
    {
        const int tid = omp_get_thread_num();
        std::vector<int32_t>& B = buf[tid];
        std::vector<int32_t> cellv, partv, farv;
#pragma omp for schedule(dynamic, 8)
        for (int64_t g = 0; g < ng; g++) {
            if (out_of_memory.load(std::memory_order_relaxed)) continue;
            try {
                double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
                for (int64_t p = goff[g]; p < goff[g + 1]; p++)
                    for (int k = 0; k < 3; k++) {
                        lo[k] = std::min(lo[k], t->pos[3 * p + k]);
                        hi[k] = std::max(hi[k], t->pos[3 * p + k]);
                    }
                for (int k = 0; k < 3; k++) {
                    L->group_box[6 * g + k] = (float)lo[k];
                    L->group_box[6 * g + 3 + k] = (float)hi[k];
                }
                cellv.clear();
                partv.clear();
                int64_t u = n;  // root cell
                while (u >= 0) {
                    if (u < n) {   // a particle reached through a link (not taken when leaves are expanded whole)
                        partv.push_back((int32_t)u);
                        u = t->next[u];
                        continue;
                    }
                    const WalkCell& c = cells[u - n];
                    double d2 = 0;
                    for (int k = 0; k < 3; k++) {
                        const double dk = std::max(0.0, std::max(lo[k] - c.com[k], c.com[k] - hi[k]));
                        d2 += dk * dk;
                    }
                    const int act = decide(c, std::sqrt(d2), g);
                    const bool open = act == kOpen;
                    if (open && c.leaf)
                        for (int32_t k = 0; k < c.count; k++) partv.push_back((int32_t)(c.first + k));
                    if (act == kAccept) cellv.push_back((int32_t)u);
                    u = (open && !c.leaf) ? c.more : c.next;
                }
                int64_t nnear = 0;
                if (near_ratio > 0.0) {   // near cells first, then the far ones, each part ascending
                    const double cg[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
                    farv.clear();
                    for (const int32_t u : cellv) {
                        const int64_t c = (int64_t)u - n;
                        const double dx = t->com[3 * c] - cg[0], dy = t->com[3 * c + 1] - cg[1],
                                     dz = t->com[3 * c + 2] - cg[2];
                        if (t->csize[c] >= near_ratio * std::sqrt(dx * dx + dy * dy + dz * dz))
                            cellv[nnear++] = u;
                        else
                            farv.push_back(u);
                    }
                    std::copy(farv.begin(), farv.end(), cellv.begin() + nnear);
                }
                g_thread[g] = tid;
                g_start[g] = (int64_t)B.size();
                g_ncell[g] = (int64_t)cellv.size();
                g_nnear[g] = nnear;
                B.insert(B.end(), cellv.begin(), cellv.end());
                B.insert(B.end(), partv.begin(), partv.end());
                g_len[g] = (int64_t)B.size() - g_start[g];
            } catch (const std::bad_alloc&) {
                out_of_memory.store(true, std::memory_order_relaxed);
            }
        }
    }
    if (out_of_memory.load()) throw std::bad_alloc();
    L->group_off.resize(ng + 1);
    L->list_off.resize(ng + 1);
    L->n_cellent.resize(ng);
    L->n_near.resize(ng);
    int64_t tot = 0, inter = 0;
    for (int64_t g = 0; g < ng; g++) {
        L->group_off[g] = (int32_t)goff[g];
        L->list_off[g] = tot;
        L->n_cellent[g] = (int32_t)g_ncell[g];
        L->n_near[g] = (int32_t)g_nnear[g];
        tot += g_len[g];
        inter += (goff[g + 1] - goff[g]) * g_len[g];
    }
    L->group_off[ng] = (int32_t)goff[ng];
    L->list_off[ng] = tot;
    L->list_idx.reset(new int32_t[tot > 0 ? tot : 1]);   // every entry is written below
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t g = 0; g < ng; g++)
        std::memcpy(&L->list_idx[L->list_off[g]], &buf[g_thread[g]][g_start[g]], sizeof(int32_t) * g_len[g]);
    L->pub.n_groups = (int32_t)ng;
    L->pub.n_entries = tot;
    L->pub.interactions = inter;
    L->pub.group_off = L->group_off.data();
    L->pub.list_off = L->list_off.data();
    L->pub.list_idx = L->list_idx.get();
    L->pub.n_cellent = L->n_cellent.data();
    L->pub.group_box = L->group_box.data();
    L->pub.n_near = L->n_near.data();
    L->pub.impl = L;
}

// The per-cell records with the acceptance radius of the criterion (ra:
// accept iff d_min > ra), from the tree's cache or built and cached.
std::shared_ptr<const std::vector<WalkCell>> cached_cells(const otoo_tree* t, const otoo_walk_params& wp) {
    WalkCache& k = t->cache;
    std::lock_guard<std::mutex> lock(k.mu);
    if (k.cells && k.mac == wp.mac && k.theta == wp.theta && k.delta == wp.delta && k.m_limit == wp.m_limit)
        return k.cells;
    auto cells = std::make_shared<std::vector<WalkCell>>(walk_cells(t));
    const int64_t nc = t->n_cells();
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; c++) {
        double& rc = (*cells)[c].ra;
        if (wp.mac == OTOO_MAC_BH) {
            rc = wp.theta > 0.0 ? t->csize[c] / wp.theta + t->s[c] : INFINITY;
        } else if (t->M[c] > wp.m_limit) {
            rc = 2.0 * t->side;
        } else {
            const double b = t->bmax[c], B2 = t->S6[6 * c] + t->S6[6 * c + 1] + t->S6[6 * c + 2];
            rc = b / 2.0 + std::sqrt(b * b / 4.0 + std::sqrt(3.0 * B2 / wp.delta));
        }
    }
    k.mac = wp.mac;
    k.theta = wp.theta;
    k.delta = wp.delta;
    k.m_limit = wp.m_limit;
    k.cells = cells;
    return k.cells;
}

// The group offsets of a grouping, from the tree's cache or built and cached.
std::shared_ptr<const std::vector<int64_t>> cached_groups(const otoo_tree* t, int mode, int g_max) {
    WalkCache& k = t->cache;
    std::lock_guard<std::mutex> lock(k.mu);
    if (k.goff && k.gmode == mode && k.gmax == g_max) return k.goff;
    k.goff = std::make_shared<const std::vector<int64_t>>(make_groups(t, mode, g_max));
    k.gmode = mode;
    k.gmax = g_max;
    return k.goff;
}

}  // namespace

extern "C" {

int otoo_tree_build(const double* pos, const double* mass, int64_t n, int32_t n_crit, otoo_tree** out) {
    if (!pos || !mass || !out || n < 1 || n > (int64_t)INT32_MAX / 2 || n_crit < 1) return OTOO_EINVAL;
    otoo_tree* tp = new (std::nothrow) otoo_tree();
    if (!tp) return OTOO_ENOMEM;
    otoo_tree& t = *tp;
    try {
        t.n = n;
        // 1. root cube: bounding box, side = largest extent, centred on the box
        double mn[3] = {pos[0], pos[1], pos[2]}, mx[3] = {pos[0], pos[1], pos[2]};
        for (int64_t i = 0; i < n; i++)
            for (int k = 0; k < 3; k++)
                if (!std::isfinite(pos[3 * i + k]) || !std::isfinite(mass[i]) || mass[i] < 0) {
                    delete tp;
                    return OTOO_EINVAL;
                }
#pragma omp parallel
        {
            double lmn[3] = {mn[0], mn[1], mn[2]}, lmx[3] = {mx[0], mx[1], mx[2]};
#pragma omp for nowait
            for (int64_t i = 0; i < n; i++)
                for (int k = 0; k < 3; k++) {
                    lmn[k] = std::min(lmn[k], pos[3 * i + k]);
                    lmx[k] = std::max(lmx[k], pos[3 * i + k]);
                }
#pragma omp critical
            for (int k = 0; k < 3; k++) {
                mn[k] = std::min(mn[k], lmn[k]);
                mx[k] = std::max(mx[k], lmx[k]);
            }
        }
        double side = std::max(mx[0] - mn[0], std::max(mx[1] - mn[1], mx[2] - mn[2]));
        if (!(side > 0)) side = 1.0;
        for (int k = 0; k < 3; k++) t.lo[k] = 0.5 * (mn[k] + mx[k]) - 0.5 * side;
        t.side = side;
        // 2. integer coordinates and Hilbert keys
        std::vector<uint32_t> ic(3 * (size_t)n);
        std::vector<std::pair<uint64_t, int64_t>> kv((size_t)n);
        const double scale = (double)(1u << kBits) / side;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            uint32_t c3[3];
            for (int k = 0; k < 3; k++) {
                double f = std::floor((pos[3 * i + k] - t.lo[k]) * scale);
                c3[k] = f <= 0 ? 0u : (f >= (double)kCoordMax ? kCoordMax : (uint32_t)f);
                ic[3 * i + k] = c3[k];
            }
            kv[i] = {hilbert_key(c3[0], c3[1], c3[2]), i};
        }
        // 3. parallel sort of (key, id)
        __gnu_parallel::sort(kv.begin(), kv.end());
        // permute
        t.perm.resize(n);
        t.pos.resize(3 * (size_t)n);
        t.mass.resize(n);
        t.icoord.resize(3 * (size_t)n);
        t.key.resize(n);
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < n; k++) {
            const int64_t i = kv[k].second;
            t.perm[k] = i;
            t.key[k] = kv[k].first;
            t.mass[k] = mass[i];
            for (int d = 0; d < 3; d++) {
                t.pos[3 * k + d] = pos[3 * i + d];
                t.icoord[3 * k + d] = ic[3 * i + d];
            }
        }
        std::vector<std::pair<uint64_t, int64_t>>().swap(kv);
        std::vector<uint32_t>().swap(ic);
        // 4. cells from key prefixes, preorder
        std::vector<std::vector<int64_t>> kids;
        build_cells(t, 0, n, 0, n_crit, kids);
        const int64_t nc = t.n_cells();
        t.nchild.resize(nc);
        t.child0.resize(nc);
        t.children.clear();
        for (int64_t c = 0; c < nc; c++) {
            t.nchild[c] = (int32_t)kids[c].size();
            t.child0[c] = (int64_t)t.children.size();
            t.children.insert(t.children.end(), kids[c].begin(), kids[c].end());
        }
        std::vector<std::vector<int64_t>>().swap(kids);
        // links: next = brother or the parent's next; more = first child / first particle
        t.next.assign(n + nc, -1);
        t.more.assign(n + nc, -1);
        for (int64_t c = 0; c < nc; c++) {  // preorder: a parent is linked before its children
            const int64_t u = n + c;
            if (t.nchild[c] == 0) {
                const int64_t f = t.first[c], e = f + t.count[c];
                t.more[u] = f;
                for (int64_t p = f; p < e - 1; p++) t.next[p] = p + 1;
                t.next[e - 1] = t.next[u];
            } else {
                const int64_t* ch = &t.children[t.child0[c]];
                t.more[u] = n + ch[0];
                for (int k = 0; k < t.nchild[c]; k++)
                    t.next[n + ch[k]] = (k + 1 < t.nchild[c]) ? n + ch[k + 1] : t.next[u];
            }
        }
        // moments, bottom up by level
        t.M.assign(nc, 0.0);
        t.com.assign(3 * nc, 0.0);
        t.S6.assign(6 * nc, 0.0);
        t.s.assign(nc, 0.0);
        t.bmax.assign(nc, 0.0);
        t.centre.assign(3 * nc, 0.0);
        t.csize.assign(nc, 0.0);
        std::vector<std::vector<int64_t>> by_level(t.depth + 1);
        for (int64_t c = 0; c < nc; c++) by_level[t.level[c]].push_back(c);
        for (int L = t.depth; L >= 0; L--) {
            const std::vector<int64_t>& cl = by_level[L];
#pragma omp parallel for schedule(dynamic, 64)
            for (size_t q = 0; q < cl.size(); q++) {
                const int64_t c = cl[q];
                double Mc = 0, cx = 0, cy = 0, cz = 0;
                double S[6] = {0, 0, 0, 0, 0, 0};
                if (t.nchild[c] == 0) {
                    const int64_t f = t.first[c], e = f + t.count[c];
                    for (int64_t p = f; p < e; p++) {
                        Mc += t.mass[p];
                        cx += t.mass[p] * t.pos[3 * p];
                        cy += t.mass[p] * t.pos[3 * p + 1];
                        cz += t.mass[p] * t.pos[3 * p + 2];
                    }
                    if (Mc > 0) {
                        cx /= Mc;
                        cy /= Mc;
                        cz /= Mc;
                    } else {
                        cx = t.pos[3 * f];
                        cy = t.pos[3 * f + 1];
                        cz = t.pos[3 * f + 2];
                    }
                    for (int64_t p = f; p < e; p++) {
                        const double m = t.mass[p];
                        const double rx = t.pos[3 * p] - cx, ry = t.pos[3 * p + 1] - cy, rz = t.pos[3 * p + 2] - cz;
                        S[0] += m * rx * rx;
                        S[1] += m * ry * ry;
                        S[2] += m * rz * rz;
                        S[3] += m * rx * ry;
                        S[4] += m * rx * rz;
                        S[5] += m * ry * rz;
                    }
                } else {
                    const int64_t* ch = &t.children[t.child0[c]];
                    for (int k = 0; k < t.nchild[c]; k++) {
                        const int64_t d = ch[k];
                        Mc += t.M[d];
                        cx += t.M[d] * t.com[3 * d];
                        cy += t.M[d] * t.com[3 * d + 1];
                        cz += t.M[d] * t.com[3 * d + 2];
                    }
                    if (Mc > 0) {
                        cx /= Mc;
                        cy /= Mc;
                        cz /= Mc;
                    } else {
                        cx = t.com[3 * ch[0]];
                        cy = t.com[3 * ch[0] + 1];
                        cz = t.com[3 * ch[0] + 2];
                    }
                    for (int k = 0; k < t.nchild[c]; k++) {
                        const int64_t d = ch[k];
                        const double m = t.M[d];
                        const double rx = t.com[3 * d] - cx, ry = t.com[3 * d + 1] - cy, rz = t.com[3 * d + 2] - cz;
                        S[0] += t.S6[6 * d + 0] + m * rx * rx;
                        S[1] += t.S6[6 * d + 1] + m * ry * ry;
                        S[2] += t.S6[6 * d + 2] + m * rz * rz;
                        S[3] += t.S6[6 * d + 3] + m * rx * ry;
                        S[4] += t.S6[6 * d + 4] + m * rx * rz;
                        S[5] += t.S6[6 * d + 5] + m * ry * rz;
                    }
                }
                t.M[c] = Mc;
                t.com[3 * c] = cx;
                t.com[3 * c + 1] = cy;
                t.com[3 * c + 2] = cz;
                for (int k = 0; k < 6; k++) t.S6[6 * c + k] = S[k];
                const double sz = t.side / (double)(1u << L);
                t.csize[c] = sz;
                double ctr[3];
                for (int k = 0; k < 3; k++) {
                    ctr[k] = t.lo[k] + ((double)t.ijk[3 * c + k] + 0.5) * sz;
                    t.centre[3 * c + k] = ctr[k];
                }
                const double ox = cx - ctr[0], oy = cy - ctr[1], oz = cz - ctr[2];
                t.s[c] = std::sqrt(ox * ox + oy * oy + oz * oz);
                // b_max: largest particle distance from the COM (exact scan)
                double b2 = 0;
                const int64_t f = t.first[c], e = f + t.count[c];
                for (int64_t p = f; p < e; p++) {
                    const double rx = t.pos[3 * p] - cx, ry = t.pos[3 * p + 1] - cy, rz = t.pos[3 * p + 2] - cz;
                    b2 = std::max(b2, rx * rx + ry * ry + rz * rz);
                }
                t.bmax[c] = std::sqrt(b2);
            }
        }
    } catch (const std::bad_alloc&) {
        delete tp;
        return OTOO_ENOMEM;
    }
    *out = tp;
    return OTOO_OK;
}

void otoo_tree_free(otoo_tree* t) { delete t; }

int otoo_tree_info(const otoo_tree* t, int64_t* n, int64_t* n_cells, int32_t* depth, double* root_lo,
                   double* root_side) {
    if (!t) return OTOO_EINVAL;
    if (n) *n = t->n;
    if (n_cells) *n_cells = t->n_cells();
    if (depth) *depth = t->depth;
    if (root_lo)
        for (int k = 0; k < 3; k++) root_lo[k] = t->lo[k];
    if (root_side) *root_side = t->side;
    return OTOO_OK;
}

int otoo_tree_export(const otoo_tree* t, int64_t* perm, float* pos32, float* mass32, float* cell_mom,
                     int32_t stride) {
    if (!t) return OTOO_EINVAL;
    if (cell_mom && stride != 4 && stride != 12) return OTOO_EINVAL;
    const int64_t n = t->n, nc = t->n_cells();
    if (perm) std::memcpy(perm, t->perm.data(), sizeof(int64_t) * n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        if (pos32)
            for (int k = 0; k < 3; k++) pos32[3 * i + k] = (float)t->pos[3 * i + k];
        if (mass32) mass32[i] = (float)t->mass[i];
    }
    if (cell_mom) {
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; c++) {
            float* o = cell_mom + (size_t)stride * c;
            for (int k = 0; k < 3; k++) o[k] = (float)t->com[3 * c + k];
            o[3] = (float)t->M[c];
            if (stride == 12) {
                o[4] = (float)t->csize[c];
                for (int k = 0; k < 6; k++) o[5 + k] = (float)t->S6[6 * c + k];
                o[11] = 0.0f;
            }
        }
    }
    return OTOO_OK;
}

int otoo_tree_cells(const otoo_tree* t, int64_t* first, int64_t* count, int32_t* level, int64_t* ijk,
                    double* com, double* mass, double* side, double* s, double* S6, double* bmax) {
    if (!t) return OTOO_EINVAL;
    const int64_t nc = t->n_cells();
    for (int64_t c = 0; c < nc; c++) {
        if (first) first[c] = t->first[c];
        if (count) count[c] = t->count[c];
        if (level) level[c] = t->level[c];
        if (ijk)
            for (int k = 0; k < 3; k++) ijk[3 * c + k] = t->ijk[3 * c + k];
        if (com)
            for (int k = 0; k < 3; k++) com[3 * c + k] = t->com[3 * c + k];
        if (mass) mass[c] = t->M[c];
        if (side) side[c] = t->csize[c];
        if (s) s[c] = t->s[c];
        if (S6)
            for (int k = 0; k < 6; k++) S6[6 * c + k] = t->S6[6 * c + k];
        if (bmax) bmax[c] = t->bmax[c];
    }
    return OTOO_OK;
}

int otoo_tree_links(const otoo_tree* t, int64_t* next, int64_t* more) {
    if (!t) return OTOO_EINVAL;
    const int64_t m = t->n + t->n_cells();
    if (next) std::memcpy(next, t->next.data(), sizeof(int64_t) * m);
    if (more) std::memcpy(more, t->more.data(), sizeof(int64_t) * m);
    return OTOO_OK;
}

int otoo_tree_groups(const otoo_tree* t, int32_t group_mode, int32_t g_max, int32_t* n_groups) {
    if (!t || !n_groups) return OTOO_EINVAL;
    if (g_max < 1 || g_max > OTOO_MAX_GROUP) return OTOO_EINVAL;
    if (group_mode != OTOO_GROUP_CHUNK && group_mode != OTOO_GROUP_CELL) return OTOO_EINVAL;
    try {
        *n_groups = (int32_t)(make_groups(t, group_mode, g_max).size() - 1);
    } catch (const std::bad_alloc&) {
        return OTOO_ENOMEM;
    }
    return OTOO_OK;
}

int otoo_tree_walk(const otoo_tree* t, const otoo_walk_params* wp, otoo_lists** out) {
    return otoo_tree_walk_range(t, wp, 0, INT32_MAX, out);
}

int otoo_tree_walk_range(const otoo_tree* t, const otoo_walk_params* wp, int32_t g_begin, int32_t g_end,
                         otoo_lists** out) {
    if (!t || !wp || !out) return OTOO_EINVAL;
    if (g_begin < 0 || g_end <= g_begin) return OTOO_EINVAL;
    if (wp->g_max < 1 || wp->g_max > OTOO_MAX_GROUP) return OTOO_EINVAL;
    if (wp->mac == OTOO_MAC_BH) {
        if (!(wp->theta >= 0.0) || !(wp->theta < OTOO_THETA_LIMIT)) return OTOO_EINVAL;
    } else if (wp->mac == OTOO_MAC_ABSOLUTE) {
        if (!(wp->delta > 0.0) || !std::isfinite(wp->delta) || std::isnan(wp->m_limit)) return OTOO_EINVAL;
    } else {
        return OTOO_EINVAL;
    }
    if (wp->group_mode != OTOO_GROUP_CHUNK && wp->group_mode != OTOO_GROUP_CELL) return OTOO_EINVAL;
    if (!(wp->near_ratio >= 0.0) || !std::isfinite(wp->near_ratio)) return OTOO_EINVAL;
    otoo_lists_impl* L = new (std::nothrow) otoo_lists_impl();
    if (!L) return OTOO_ENOMEM;
    try {
        const std::shared_ptr<const std::vector<int64_t>> all = cached_groups(t, wp->group_mode, wp->g_max);
        const int64_t ng_all = (int64_t)all->size() - 1;
        if (g_begin >= ng_all) {
            delete L;
            return OTOO_EINVAL;
        }
        const int64_t g1 = std::min<int64_t>(g_end, ng_all);
        const std::vector<int64_t> goff(all->begin() + g_begin, all->begin() + g1 + 1);
        const std::shared_ptr<const std::vector<WalkCell>> cells = cached_cells(t, *wp);
        walk_groups(t, goff, *cells, [](const WalkCell& w, double dmin, int64_t) { return dmin > w.ra ? kAccept : kOpen; },
                    L, wp->near_ratio);
    } catch (const std::bad_alloc&) {
        delete L;
        return OTOO_ENOMEM;
    }
    *out = &L->pub;
    return OTOO_OK;
}

int otoo_tree_walk_sph(const otoo_tree* t, const double* h, int32_t group_mode, int32_t g_max, otoo_lists** out) {
    if (!t || !h || !out) return OTOO_EINVAL;
    if (g_max < 1 || g_max > OTOO_MAX_GROUP) return OTOO_EINVAL;
    if (group_mode != OTOO_GROUP_CHUNK && group_mode != OTOO_GROUP_CELL) return OTOO_EINVAL;
    const int64_t n = t->n, nc = t->n_cells();
    for (int64_t i = 0; i < n; i++)
        if (!(h[i] > 0.0) || !std::isfinite(h[i])) return OTOO_EINVAL;
    otoo_lists_impl* L = new (std::nothrow) otoo_lists_impl();
    if (!L) return OTOO_ENOMEM;
    try {
        std::vector<double> hk(n);
        for (int64_t p = 0; p < n; p++) hk[p] = h[t->perm[p]];
        // per cell: extent R_c = max |COM_c - x_j| (rb) and the SPH bounding
        // radius r_SPH = max (|COM_c - x_j| + h_j) of Eq. 5 (ra), over the
        // cell's particles
        std::vector<WalkCell> cells = walk_cells(t);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t c = 0; c < nc; c++) {
            const double* cm = &t->com[3 * c];
            double r_max = 0.0, rs_max = 0.0;
            for (int64_t p = t->first[c]; p < t->first[c] + t->count[c]; p++) {
                double d2 = 0.0;
                for (int k = 0; k < 3; k++) {
                    const double dk = t->pos[3 * p + k] - cm[k];
                    d2 += dk * dk;
                }
                const double d = std::sqrt(d2);
                r_max = std::max(r_max, d);
                rs_max = std::max(rs_max, d + hk[p]);
            }
            cells[c].rb = r_max;
            cells[c].ra = rs_max;
        }
        const std::vector<int64_t> goff = make_groups(t, group_mode, g_max);
        const int64_t ng = (int64_t)goff.size() - 1;
        std::vector<double> hg(ng);
        for (int64_t g = 0; g < ng; g++) {
            double m = 0.0;
            for (int64_t p = goff[g]; p < goff[g + 1]; p++) m = std::max(m, hk[p]);
            hg[g] = m;
        }
        // a cell can hold a neighbour of a group particle only if the group's
        // box comes within r_SPH of its COM (the source's support) or within
        // R_c + max_g h (the target's support); otherwise it is skipped whole
        walk_groups(t, goff, cells, [&](const WalkCell& w, double dmin, int64_t g) {
            return dmin >= std::max(w.ra, w.rb + hg[g]) ? kSkip : kOpen;
        }, L);
    } catch (const std::bad_alloc&) {
        delete L;
        return OTOO_ENOMEM;
    }
    *out = &L->pub;
    return OTOO_OK;
}

void otoo_lists_free(otoo_lists* l) {
    if (l) delete static_cast<otoo_lists_impl*>(l->impl);
}

}  // extern "C"
