/*
 * otoo.h -- C ABI of the MI355X octree gravity force library (libotoo.so).
 *
 * The library evaluates, for every group of target particles produced by a
 * grouped tree walk, the Plummer-softened acceleration and potential summed
 * over the group's interaction list of particles and monopole cell moments:
 * the force evaluation that the paper hands to the GPU (Sec. 3.4, with the
 * octree method of Sec. 2).  G = 1 throughout.  A source of mass m at y acts
 * on a target at x with
 *     acceleration  m (y - x) (|y - x|^2 + eps^2)^(-3/2)
 *     potential    -m (|y - x|^2 + eps^2)^(-1/2)
 * and the target's own entry (the self pair) is excluded.
 *
 * Two halves:
 *   host  (C++/OpenMP, host pointers): tree build, cell moments, grouped walk
 *         -> the interaction-list CSR;
 *   device (HIP, gfx950, device pointers): the force evaluation and the
 *         learned cell correction (network inference and training).
 *
 * Conventions
 *   - every function returns OTOO_OK (0) or a negative otoo_status;
 *     nothing throws across the ABI;
 *   - device entry points are asynchronous on the context's stream; device
 *     outputs are valid once that stream has synchronised;
 *   - inputs are never modified; outputs are fully overwritten;
 *   - device pointers belong to the caller; a context owns only its own
 *     scratch memory, grown on demand and freed by otoo_destroy;
 *   - on a non-zero return, otoo_last_error(ctx) names the problem.
 */
#ifndef OTOO_H
#define OTOO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum otoo_status {
    OTOO_OK = 0,
    OTOO_EINVAL = -1,      /* bad argument (null pointer, size, eps, stride, ...) */
    OTOO_ENOMEM = -2,      /* host or device allocation failed, or the scratch cap was hit */
    OTOO_EHIP = -3,        /* a HIP runtime call failed; otoo_last_error has its message */
    OTOO_EUNSUPPORTED = -4 /* option not available in this library */
};

/* Largest group (number of target particles sharing one list) the device
 * kernels accept; a workgroup holds the whole group in registers. */
#define OTOO_MAX_GROUP 256
/* Opening angles at or above 2/sqrt(3) could accept a cell that holds one of
 * the group's own particles; the walk rejects them (see otoo_tree_walk). */
#define OTOO_THETA_LIMIT 1.15

/* ======================================================================
 * Host half: tree build and grouped walk
 * ====================================================================== */

typedef struct otoo_tree otoo_tree;

/* Build the octree of n particles (Sec. 3.2: root cube from the bounding
 * box, 21-bit-per-axis integer coordinates turned into Hilbert keys, parallel
 * sort, cells read off equal key prefixes; a cell with at most n_crit
 * particles, or at depth 21, is a leaf) and its cell moments (Sec. 3.3: mass,
 * centre of mass, second-moment tensor S with trace B2 of Eq. (2), b_max).
 *   pos   [n][3] FP64, original order (host)      mass [n] FP64, >= 0
 *   n     1 .. 2^30                               n_crit >= 1 (the paper uses 16)
 *   *tree receives a handle freed by otoo_tree_free.
 * EINVAL for null pointers, bad sizes, non-finite coordinates or negative
 * masses; ENOMEM when host memory runs out. */
int otoo_tree_build(const double* pos, const double* mass, int64_t n, int32_t n_crit, otoo_tree** tree);
void otoo_tree_free(otoo_tree* tree);

/* Sizes and root cube.  Any output pointer may be NULL. */
int otoo_tree_info(const otoo_tree* tree, int64_t* n, int64_t* n_cells, int32_t* depth,
                   double* root_lo /*[3]*/, double* root_side);

/* Copy out the device-ready arrays (host buffers owned by the caller; NULL skips):
 *   perm     [n]        sorted position k holds original particle perm[k]
 *   pos32    [n][3]     FP32 positions in key (group) order
 *   mass32   [n]        FP32 masses in key order
 *   cell_mom [n_cells][stride], stride 4: COM xyz, M;
 *            stride 12: COM xyz, M, side l, S (xx, yy, zz, xy, xz, yz), 0. */
int otoo_tree_export(const otoo_tree* tree, int64_t* perm, float* pos32, float* mass32, float* cell_mom,
                     int32_t stride);

/* FP64 cell data in preorder (host buffers, NULL skips): first particle and
 * count in key order, level, integer cube coordinates ijk [n_cells][3] at that
 * level, COM [n_cells][3], mass, side, offset s = |COM - centre|,
 * S [n_cells][6], b_max. */
int otoo_tree_cells(const otoo_tree* tree, int64_t* first, int64_t* count, int32_t* level, int64_t* ijk,
                    double* com, double* mass, double* side, double* s, double* S6, double* bmax);

/* The next/more links over the unified index space [0, n + n_cells)
 * (Sec. 2.1; index u < n is particle u in key order, u >= n is cell u - n;
 * -1 is null). */
int otoo_tree_links(const otoo_tree* tree, int64_t* next, int64_t* more);

enum otoo_mac {
    OTOO_MAC_BH = 0,       /* accept iff d_min > l/theta + s  (opening angle theta, COM offset s) */
    OTOO_MAC_ABSOLUTE = 1  /* accept iff d_min > r_b of Eq. (1); r_b = 2 * root side above m_limit */
};
enum otoo_group_mode {
    OTOO_GROUP_CHUNK = 0,  /* consecutive runs of g_max particles in key order */
    OTOO_GROUP_CELL = 1    /* maximal cells holding at most g_max particles */
};

typedef struct {
    int32_t mac;          /* otoo_mac */
    double theta;         /* BH: 0 <= theta < OTOO_THETA_LIMIT (0 opens every cell) */
    double delta;         /* ABSOLUTE: accuracy parameter Delta > 0 */
    double m_limit;       /* ABSOLUTE: cells heavier than this are never accepted (INFINITY = off) */
    int32_t group_mode;   /* otoo_group_mode */
    int32_t g_max;        /* 1 .. OTOO_MAX_GROUP */
    double near_ratio;    /* >= 0; > 0: each list's accepted cells are ordered near first -- those whose
                             side l_c is at least near_ratio times the distance from their COM to the
                             centre of the group's bounding box (FP64) -- then the others, each part
                             ascending, and n_near counts the near ones; 0: no split (n_near = 0) */
} otoo_walk_params;

/* Interaction lists in CSR form, allocated by the library. */
typedef struct {
    int32_t n_groups;
    int64_t n_entries;      /* sum of list lengths */
    int64_t interactions;   /* sum over groups of n_g * |L_g| (self pairs included) */
    int32_t* group_off;     /* [n_groups+1] particle ranges in key order */
    int64_t* list_off;      /* [n_groups+1] */
    int32_t* list_idx;      /* [n_entries]: j < n particle j, j >= n cell j - n */
    int32_t* n_cellent;     /* [n_groups]: the first n_cellent[g] entries of L_g are cells */
    float* group_box;       /* [n_groups][6]: bounding box lo xyz, hi xyz (FP32) */
    int32_t* n_near;        /* [n_groups]: the first n_near[g] of those cells are the near ones
                               (otoo_walk_params.near_ratio); all 0 without the split */
    void* impl;
} otoo_lists;

/* Grouped stackless walk (Sec. 2.1 rules 1-4; group d_min as in Sec. 3.4):
 * for each group, d_min is the distance from a cell's COM to the group's
 * bounding box; accepted cells become one entry, opened leaves contribute
 * their particles.  Each list holds the accepted cells first, then the
 * particles, each part ascending.  Every group particle appears in its own
 * list (its leaf can never be accepted below OTOO_THETA_LIMIT), which the
 * device force relies on to remove the self pair.  *out is freed by
 * otoo_lists_free.  EINVAL on bad parameters, ENOMEM on allocation failure. */
int otoo_tree_walk(const otoo_tree* tree, const otoo_walk_params* params, otoo_lists** out);

/* Number of groups the walk forms for (group_mode, g_max). */
int otoo_tree_groups(const otoo_tree* tree, int32_t group_mode, int32_t g_max, int32_t* n_groups);
/* The walk of otoo_tree_walk restricted to groups [g_begin, g_end) of its
 * grouping (g_end is clamped to the group count), so that a caller can walk
 * in batches and evaluate earlier batches meanwhile.  group_off holds the
 * groups' absolute particle offsets (group_off[0] is the first particle of
 * group g_begin, group_off[n_groups] one past the last of group g_end - 1);
 * list_off starts at 0.  The concatenated batches equal the whole walk.
 * EINVAL if g_begin < 0, g_end <= g_begin or g_begin >= the group count. */
int otoo_tree_walk_range(const otoo_tree* tree, const otoo_walk_params* params, int32_t g_begin, int32_t g_end,
                         otoo_lists** out);

/* Neighbour lists for SPH gather sums (Sec. 2.3, Eq. 4-5): the same grouped
 * walk with the SPH bounding radius in place of the MAC.  There is no
 * particle-cell interaction: a cell is either opened or skipped whole, so
 * lists hold particles only (n_cellent = 0).  With R_c = max |COM_c - x_j|
 * and r_SPH = max (|COM_c - x_j| + h_j) over the cell's particles (Eq. 5),
 * a cell is skipped iff d_min >= max(r_SPH, R_c + max_{i in g} h_i), so every
 * pair closer than max(h_i, h_j) -- every pair with a nonzero symmetrised
 * kernel weight -- is listed.  h [n] (host, FP64, > 0 and finite) is given
 * in the caller's particle order, as passed to otoo_tree_build.  *out is
 * freed by otoo_lists_free.  EINVAL on bad parameters, ENOMEM on allocation
 * failure. */
int otoo_tree_walk_sph(const otoo_tree* tree, const double* h, int32_t group_mode, int32_t g_max,
                       otoo_lists** out);
void otoo_lists_free(otoo_lists* lists);

/* ======================================================================
 * Device half: force evaluation
 * ====================================================================== */

typedef struct otoo_ctx otoo_ctx;
typedef struct otoo_mlp otoo_mlp;   /* the learned correction's network, below */

/* Create a context on HIP device `device` (its stream is the null stream
 * until otoo_set_stream).  EHIP if the device cannot be used. */
int otoo_create(otoo_ctx** ctx, int32_t device);
/* Synchronise the context's stream, free its scratch and the context. */
int otoo_destroy(otoo_ctx* ctx);
/* Use `hip_stream` (a hipStream_t, e.g. torch's current stream) for all work. */
int otoo_set_stream(otoo_ctx* ctx, void* hip_stream);
/* Message of the last failing call on this context ("" if none). */
const char* otoo_last_error(const otoo_ctx* ctx);

/* Kernel schedule knobs (the autotuner's search space).  A zero chunk,
 * blocks_per_cu or tile keeps the current value; lpt, debug_validate,
 * net_kernel and corr_chunks are taken as given. */
typedef struct {
    int32_t chunk;        /* list entries per work item (a long list is split into items); >= 64 */
    int32_t blocks_per_cu;/* persistent workgroups per compute unit, 1..16 */
    int32_t lpt;          /* 1: hand out items longest-first, 0: in group order */
    int32_t debug_validate; /* 1: check the CSR on the host before launching (slow) */
    int32_t tile;         /* list entries staged in LDS per tile: 256, 512 or 1024 */
    int32_t net_kernel;   /* learned correction kernel: 0 fused, registers-resident; 1 fused, LDS-staged;
                             2 (default) a network pass writing the gated pairs' tensors, then the
                             expansion pass */
    int32_t corr_chunks;  /* the two passes of net_kernel 2: 0 (default) by the pairs' density (pair-parallel
                             chunks of 64 pairs across groups when there are fewer than 32 pairs per group,
                             or fewer than 128 when items of 256 pairs would give the resident waves fewer
                             than four each; else one group at a time), 1 one group at a time, 2
                             pair-parallel chunks */
} otoo_tuning;
int otoo_set_tuning(otoo_ctx* ctx, const otoo_tuning* tuning);
int otoo_get_tuning(const otoo_ctx* ctx, otoo_tuning* tuning);

/* Cap, in bytes, on each device scratch buffer of the context (force
 * schedule and partials, SPH items and partials, correction item sums);
 * 0 (the default) means no cap.  A call that would need a larger buffer
 * returns ENOMEM before it enqueues anything.  Buffers already allocated are
 * kept.  EINVAL for a negative cap. */
int otoo_set_scratch_limit(otoo_ctx* ctx, int64_t max_bytes);

/* Force evaluation over interaction lists (device pointers).
 *   n           number of particles, 1 .. 2^30
 *   pos [n][3], mass [n]   FP32 targets and particle sources, in group order
 *   n_groups    >= 1; group_off [n_groups+1] int32: group g is particles
 *               [group_off[g], group_off[g+1]), 1 .. OTOO_MAX_GROUP of them
 *   n_entries   = list_off[n_groups]; list_off [n_groups+1] int64;
 *   list_idx [n_entries] int32: j < n particle j, j >= n cell j - n
 *               (the unified index space of Sec. 3.2).  A group's list must
 *               hold each of the group's own particles exactly once: that
 *               self pair is what the final reduction removes.
 *   n_cells     >= 0; cell_mom [n_cells][cell_stride] FP32, COM xyz then M
 *               (cell_stride 4 or 12)
 *   eps         Plummer softening, > 0 and finite
 *   gcorr       per-group cell correction from otoo_correction
 *               ([n_groups][24] FP32), or NULL for the plain monopole: the
 *               second-order local expansion of the correction field about
 *               the centre c_g of each group's bounding box, applied per
 *               target as a_i += A + J d + 1/2 H[d, d] and
 *               phi_i += Phi - A.d - 1/2 d.J d with d = x_i - c_g
 *   out_acc [n][3] FP32, out_pot [n] FP64 (the potential is reduced in FP64)
 * Arithmetic: FP32 pairs; per-tile FP32 partial sums combined with Kahan
 * compensation across tiles and work items; FP64 for the final potential.
 * The groups may cover a contiguous sub-range [group_off[0],
 * group_off[n_groups]) of the particles (a batch of otoo_tree_walk_range);
 * only those particles' outputs are written, and every group's result is
 * the same as in a call over all groups.
 * Results are bitwise reproducible for fixed tuning.  Malformed device CSR
 * (indices out of range, group sizes outside 1..OTOO_MAX_GROUP) never causes
 * an out-of-bounds access: such entries are skipped and otoo_check(ctx)
 * reports them; with debug_validate the call returns EINVAL instead. */
int otoo_force(otoo_ctx* ctx, int32_t n, const float* pos, const float* mass, int32_t n_groups,
               const int32_t* group_off, int64_t n_entries, const int64_t* list_off, const int32_t* list_idx,
               int32_t n_cells, const float* cell_mom, int32_t cell_stride, float eps, const float* gcorr,
               float* out_acc, double* out_pot);

/* otoo_force without any device allocation, for callers that cannot
 * allocate device memory: code under stream or graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, launches and
 * results (bitwise) as otoo_force with the context's tuning; the scratch is
 * a fixed array of OTOO_NOALLOC_SCRATCH_BYTES in the library's device code,
 * one per GPU (located once per device by otoo_create), instead of the
 * context's buffer.  The context's 4 KiB counter block, made by otoo_create,
 * is used as by otoo_force.  Every call on one GPU shares that array, which
 * keeps the last call's contents (nothing in it needs to start at zero):
 * calls that overlap on one GPU -- from two streams or two contexts -- race.
 * EINVAL, before anything is enqueued, when the call's scratch (the size
 * otoo_force_plan reports) exceeds the array, and when the context's debug
 * validation is on (it copies the lists to the host). */
#define OTOO_NOALLOC_SCRATCH_BYTES (128 * 1024 * 1024)
int otoo_force_noalloc(otoo_ctx* ctx, int32_t n, const float* pos, const float* mass, int32_t n_groups,
                       const int32_t* group_off, int64_t n_entries, const int64_t* list_off,
                       const int32_t* list_idx, int32_t n_cells, const float* cell_mom, int32_t cell_stride,
                       float eps, const float* gcorr, float* out_acc, double* out_pot);

/* Host-only plan of an otoo_force call (no device call, no context): the
 * same size checks otoo_force makes before it touches the device, and the
 * bytes of context scratch such a call needs (unified source table, work
 * items, longest-first order, partial rows of split lists).
 *   n, n_groups, n_entries, n_cells   as for otoo_force
 *   chunk        list entries per work item (otoo_tuning.chunk, 64 .. 2^28)
 *   workgroups   persistent workgroups of the force kernel (CUs x
 *                blocks_per_cu), 1 .. 2^20
 *   *scratch_bytes (may be NULL) receives the scratch size.
 * EINVAL for sizes out of range, and when the work items plus one last
 * queue fetch per workgroup would reach 2^31: the device queue head, the
 * item table and the longest-first order are 32-bit, so such a call is
 * refused before anything is allocated or enqueued. */
int otoo_force_plan(int32_t n, int32_t n_groups, int64_t n_entries, int32_t n_cells, int32_t chunk,
                    int32_t workgroups, int64_t* scratch_bytes);

/* The lanes the force kernel gives a group of ng targets (1 .. OTOO_MAX_GROUP)
 * at tile depth `tile` (256, 512 or 1024 list entries), for tests and tools;
 * host only, no context.  The kernel's workgroup is 256 threads in four
 * waves of 64.
 *   *wave_parts  0: every target has 256 / ng slices across the workgroup
 *                (thread t: target t mod ng, slice t / ng), parts[0] =
 *                256 / ng and parts[1..3] = 0;
 *                1: each wave takes its own part of the targets, parts[j] =
 *                the size of part j (consecutive targets, in order; 0 for an
 *                idle part), each part with 64 / parts[j] slices of a tile.
 * Sizes that divide 256 use the first layout; the others use the parts
 * where these run fewer wave rows per full tile (and whenever 256 / ng
 * exceeds 64).  EINVAL for ng or tile out of range or NULL pointers. */
int otoo_group_layout(int32_t ng, int32_t tile, int32_t* wave_parts, int32_t* parts);

/* Generation of the context's device scratch: a counter raised every time
 * the context allocates a scratch buffer anew (force, SPH and correction
 * scratch, and the per-group geometry of a network bound to it).  A graph
 * captured around calls of this library names the scratch of its
 * generation; after the counter changes it must be captured again. */
int otoo_scratch_generation(const otoo_ctx* ctx, int64_t* gen);

/* Direct summation at selected targets: the O(N^2) sum of Sec. 2 that the
 * tree approximates, used as the accuracy reference of the tree force.  For
 * k < n_tgt and i = tgt[k], with d = x_j - x_i and r^2 = |d|^2 + eps^2:
 *   out_acc[k] = sum_{j != i} m_j d r^-3,   out_pot[k] = -sum_{j != i} m_j r^-1
 * in FP64 over the FP32 inputs.  Device pointers: pos [n][3], mass [n],
 * tgt [n_tgt] int32 indices into pos; out_acc [n_tgt][3] FP64 and
 * out_pot [n_tgt] FP64 are overwritten.  Asynchronous on the context stream;
 * the sum over j runs in fixed slices combined in a fixed order, so results
 * are reproducible.  A target outside [0, n) gives zeros and is flagged for
 * otoo_check.  Returns EINVAL for n < 1, n_tgt < 0, eps not positive and
 * finite, or a null pointer (tgt and the outputs may be NULL when
 * n_tgt == 0). */
int otoo_direct(otoo_ctx* ctx, int32_t n, const float* pos, const float* mass, int32_t n_tgt, const int32_t* tgt,
                float eps, double* out_acc, double* out_pot);

/* SPH-style gather sums over neighbour lists (Sec. 2.3, Eq. 4).  For every
 * particle i of group g:
 *   out[i] = sum over j in L_g of q_j (W(r_ij, h_i) + W(r_ij, h_j)) / 2,
 * with the cubic B-spline kernel of compact support h,
 *   W(r, h) = 8 / (pi h^3) w(r / h),  w(u) = 1 - 6u^2 + 6u^3 (u <= 1/2),
 *   2 (1 - u)^3 (1/2 < u <= 1), 0 beyond.
 * With the lists of otoo_tree_walk_sph, which hold every pair of nonzero
 * weight, this is the sum over all particles, the particle's own term
 * q_i W(0, h_i) included (q = m gives the SPH density).  Device pointers, in
 * the key order of the device arrays: pos [n][3], h [n] (> 0), q [n] FP32;
 * group_off, list_off, list_idx as for otoo_force (particle entries only);
 * out [n] FP32 is overwritten.  FP32 arithmetic; per target the slices of a
 * workgroup are combined in a fixed order, and a long list is cut into
 * chunks whose sums are added in chunk order, so results are reproducible.
 * The context keeps scratch for the work items and chunk sums (grown on
 * demand).
 * Entries that are not particles, and malformed groups, are skipped and
 * flagged for otoo_check.  Asynchronous on the context stream. */
int otoo_sph_sum(otoo_ctx* ctx, int32_t n, const float* pos, const float* h, const float* q, int32_t n_groups,
                 const int32_t* group_off, int64_t n_entries, const int64_t* list_off, const int32_t* list_idx,
                 float* out);

/* Textbook quadrupole tensor of every (group, cell) pair (the p = 2 term of
 * the multipole expansion the paper names in Sec. 2 but does not use):
 * corr[pair_off[g] + k] = 3 S_c - tr(S_c) I for the k-th cell entry c of
 * group g's list, from the second-moment tensor S in cell_mom (cell_stride 12,
 * as exported by otoo_tree_export).  Device pointers; corr [n_pairs][6]
 * (xx, yy, zz, xy, xz, yz) is written; asynchronous on the context stream.
 * Entries that are not cells give a zero tensor and are flagged for
 * otoo_check. */
int otoo_quad_exact(otoo_ctx* ctx, int32_t n, int32_t n_groups, int64_t n_entries, const int64_t* list_off,
                    const int32_t* list_idx, int64_t n_pairs, const int64_t* pair_off, int32_t n_cells,
                    const float* cell_mom, int32_t cell_stride, float* corr);

/* ======================================================================
 * Learned cell correction (not in the paper, which evaluates accepted cells
 * as monopoles, Sec. 2): for every (group g, accepted cell c) pair a network
 * 12 features (zero-padded to 32) -> 64 -> GELU -> 64 -> GELU -> 6, plus the
 * fixed skip term 3 s (s the normalised second moments, features 6..11),
 * gives o and the symmetric traceless tensor Qt = M_c l_c^2 P(o) (P removes
 * the trace) that otoo_force applies through its local expansion.  With zero
 * layers Qt is the textbook quadrupole 3 S_c - tr(S_c) I; the layers learn
 * the correction to it.  Features, with
 * d = COM_c - c_g (c_g the centre of the group's bounding box) and n = |d|:
 *     d/n (3), l_c/n, eps/n, h_g/n (h_g the box half-diagonal),
 *     S_c / (M_c l_c^2) as (xx, yy, zz, xy, xz, yz).
 * A pair whose features are non-finite or exceed 8 in magnitude gets a zero
 * tensor (plain monopole).  A gate (otoo_mlp_set_gate) limits the layers to
 * pairs whose BF16 feature l_c/n is at least the gate; the others keep the
 * skip term alone (the textbook quadrupole).  GELU is the tanh form.  BF16
 * operands on MFMA, FP32 accumulation, FP32 master weights with Adam.
 * ====================================================================== */

/* Number of FP32 parameters (6662): W1 [32][64], b1 [64], W2 [64][64],
 * b2 [64], W3 [64][6], b3 [6], concatenated row-major in that order. */
int otoo_mlp_num_params(void);
/* A network bound to a context (its device, its stream); the context must
 * stay alive for every network call except otoo_mlp_destroy, which may come
 * after otoo_destroy.  No parameters until otoo_mlp_set_params or
 * otoo_mlp_load. */
int otoo_mlp_create(otoo_ctx* ctx, otoo_mlp** mlp);
int otoo_mlp_destroy(otoo_mlp* mlp);
/* Host parameter vector in, optimiser state reset (EINVAL on non-finite values). */
int otoo_mlp_set_params(otoo_mlp* mlp, const float* params);
/* Gate of the layers for otoo_mlp_infer and otoo_correction: the layers run
 * only for pairs whose BF16 feature l_c/n is >= gate (0, the default, runs
 * them for every pair; +INFINITY for none).  A setting of the network object,
 * not part of its checkpoint.  EINVAL for a negative or NaN gate. */
int otoo_mlp_set_gate(otoo_mlp* mlp, float gate);
/* Host copies of parameters, Adam moments and the step count (NULL skips). */
int otoo_mlp_get_params(otoo_mlp* mlp, float* params, float* adam_m, float* adam_v, int64_t* step);
/* Checkpoint: "OTOOMLP1", int32 parameter count, int64 step, then FP32
 * parameters, Adam m and Adam v.  Loading restores the exact training state. */
int otoo_mlp_save(otoo_mlp* mlp, const char* path);
int otoo_mlp_load(otoo_mlp* mlp, const char* path);

/* Network outputs o [rows][6], skip term included and no gate (before
 * projection and scaling), for BF16 features X [rows][32] (device pointers;
 * for parity checks). */
int otoo_mlp_forward(otoo_mlp* mlp, const uint16_t* X, int64_t rows, float* out);

/* Tensors of every (group, cell) pair for otoo_force: corr [n_pairs][6].
 * Arguments as for otoo_force (device pointers; cell_stride must be 12). */
int otoo_mlp_infer(otoo_mlp* mlp, int32_t n, const float* pos, int32_t n_groups, const int32_t* group_off,
                   int64_t n_entries, const int64_t* list_off, const int32_t* list_idx, int64_t n_pairs,
                   const int64_t* pair_off, int32_t n_cells, const float* cell_mom, int32_t cell_stride, float eps,
                   float* corr);

/* Training samples generated by the method itself: for each requested
 * (pair p, particle i) with i a target of p's group (samples [n_samples][2]
 * int64), the pair's BF16 features X [n_samples][32] and aux [n_samples][12]
 * FP32 = {c_g - COM (3), x_i - c_g (3), t (3), M l^2, w, 0}, where
 * t = a_exact(x_i) - a_mono(x_i) is the cell's exact softened direct sum over
 * its particles minus its monopole (FP64 sums; cell_first/cell_count give each
 * cell's particle range in key order, from otoo_tree_cells) and w = 1 (0 for
 * a pair whose features are out of range; otoo_mlp_sample_weights sets the
 * training weight).  Device pointers. */
int otoo_mlp_train_samples(otoo_mlp* mlp, int32_t n, const float* pos, const float* mass, int32_t n_groups,
                           const int32_t* group_off, int64_t n_entries, const int64_t* list_off,
                           const int32_t* list_idx, int64_t n_pairs, const int64_t* pair_off, int32_t n_cells,
                           const float* cell_mom, int32_t cell_stride, const int32_t* cell_first,
                           const int32_t* cell_count, float eps, int64_t n_samples, const int64_t* samples,
                           uint16_t* X, float* aux);

/* Training weights and the gate's selection of samples (the weight is not
 * in the paper; it makes the loss follow the per-particle relative force
 * error by which the method is judged).  For sample s of the samples of
 * otoo_mlp_train_samples (samples [n_samples][2] int64, device; only the
 * target particle i = samples[s][1] is read), with a_i = acc[i] the total
 * force on the target from the same walk (acc [n][3] FP32, device, e.g. from
 * otoo_force):
 *   kept:   the BF16 feature l/n (X[s][3]) is at least gate (>= 0; 0 keeps
 *           every sample with features in range),
 *   weight: aux[s][10] = W / |a_i|^2 (for every sample; |a_i|^2 is taken as
 *           at least 1e-300), with W = K / sum over the K kept samples of
 *           |t_s|^2 / |a_i|^2 (t_s = aux[s][6..8]), so that the kept samples'
 *           zero-correction loss, mean of w |t|^2, is 1 (W = 1 if that sum is
 *           0).
 * The sums are FP64 in a fixed order.  keep [n_samples] int64 (device)
 * receives the kept sample indices in ascending order and *n_keep (host)
 * their number; the call synchronises the context stream.  A target index
 * outside [0, n) drops the sample and is flagged for otoo_check.  EINVAL for
 * a negative or NaN gate, bad sizes or null pointers. */
int otoo_mlp_sample_weights(otoo_mlp* mlp, int64_t n_samples, const int64_t* samples, int32_t n, const float* acc,
                            const uint16_t* X, float* aux, float gate, int64_t* keep, int64_t* n_keep);

/* Loss L = mean over the samples of w |a_corr - t|^2, with a_corr the
 * correction of the sample's predicted tensor through the second-order local
 * expansion about c_g evaluated at x_i, and its gradient with respect to the
 * parameters (host grad [6662] and loss, NULL skips; synchronises).  Sums
 * over samples are taken per workgroup and then in a fixed order. */
int otoo_mlp_backward(otoo_mlp* mlp, const uint16_t* X, const float* aux, int64_t n_samples, float eps,
                      float* grad, float* loss);
/* One Adam step (beta 0.9 / 0.999, epsilon 1e-8, bias-corrected) on that
 * gradient; *loss (if not NULL) receives the loss before the step. */
int otoo_mlp_train_step(otoo_mlp* mlp, const uint16_t* X, const float* aux, int64_t n_samples, float eps, float lr,
                        float* loss);

enum otoo_corr_kind {
    OTOO_CORR_PAIRS = 0,   /* given tensors corr [n_pairs][6], one per (group, cell) pair */
    OTOO_CORR_QUAD = 1,    /* the textbook quadrupole 3 S_c - tr(S_c) I of each accepted cell */
    OTOO_CORR_MLP = 2      /* the learned effective tensor of each (group, cell) pair (otoo_mlp_*) */
};

/* Per-group cell correction for otoo_force.  For every (group, cell) pair
 * (the first pair_off[g+1]-pair_off[g] entries of group g's list are its
 * cells; pair_off [n_groups+1] int64, n_pairs = pair_off[n_groups]) a
 * symmetric tensor Q (xx, yy, zz, xy, xz, yz) -- given, textbook or learned --
 * defines the quadrupole-form field
 *     phi = -1/2 d.Qd r^-5,  a = -grad phi  (d = x - COM_c, r^2 = |d|^2 + eps^2);
 * the field, its first and second derivatives and its potential at the
 * centre c_g of the group's bounding box are summed over the group's cells
 * (fixed order) into gcorr [n_groups][24] = {A xyz, Phi, J (xx yy zz xy xz yz),
 * H (xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz), c_g xyz, 0}.  The multipole
 * expansion beyond the monopole is what the paper names but does not use
 * (Sec. 2).  The work is cut into items of 1024 consecutive (group, cell)
 * pairs in pair order; a group whose pairs span several items has its item
 * sums added in item order, so results do not depend on how the work is
 * scheduled.  group_box [n_groups][6] (lo xyz, hi xyz, FP32) may give each
 * group's bounding box as the walk returns it (the extremes of the group's
 * positions, identical to those of the FP32 pos); NULL has the pass find
 * them in pos.  Device pointers; asynchronous; mlp only for OTOO_CORR_MLP;
 * cell_stride 12 for QUAD and MLP (the second-moment tensor).  The context
 * keeps scratch for the item sums (grown on demand). */
int otoo_correction(otoo_ctx* ctx, int32_t kind, otoo_mlp* mlp, int32_t n, const float* pos, int32_t n_groups,
                    const int32_t* group_off, const float* group_box, int64_t n_entries, const int64_t* list_off,
                    const int32_t* list_idx,
                    int64_t n_pairs, const int64_t* pair_off, int32_t n_cells, const float* cell_mom,
                    int32_t cell_stride, float eps, const float* corr, float* gcorr);

/* Autotuner of the force evaluation (the group size of Sec. 3.4's
 * vectorised walk and the device schedule).  For each group choice, the
 * tree is walked with *walk's criterion and that (group_mode, g_max), the
 * lists and the particle/cell arrays (cell stride 4) are copied to the
 * device, and every schedule in `schedules` is timed as the mean of `reps`
 * replays of a captured force graph (after two warm-up replays) on the
 * context stream.  ms [n_choices][n_schedules] (host, may be NULL) receives
 * every time and interactions [n_choices] (may be NULL) the interaction
 * counts; *best_choice and *best_tuning receive the fastest pair and
 * *best_ms its time.  The context's tuning is restored afterwards and any
 * graph it held (otoo_graph_capture) is discarded.  The library allocates
 * and frees the device copies itself.  Synchronous.
 * EINVAL on bad arguments (a schedule set_tuning rejects included). */
typedef struct {
    int32_t group_mode;   /* otoo_group_mode */
    int32_t g_max;        /* 1 .. OTOO_MAX_GROUP */
} otoo_group_choice;
int otoo_autotune(otoo_ctx* ctx, const otoo_tree* tree, const otoo_walk_params* walk,
                  const otoo_group_choice* choices, int32_t n_choices, const otoo_tuning* schedules,
                  int32_t n_schedules, float eps, int32_t reps, float* ms, int64_t* interactions,
                  otoo_group_choice* best_choice, otoo_tuning* best_tuning, float* best_ms);
/* The same sweep for a corrected evaluation: each timed replay is one graph
 * holding the correction pass (otoo_correction of corr_kind, OTOO_CORR_QUAD
 * or OTOO_CORR_MLP with the network mlp of this context) followed by the
 * force with that correction, captured on the context's stream; the cell
 * moments go with stride 12 and each group's cell-entry counts give the
 * pair offsets (its near cells' counts when walk->near_ratio > 0).  Larger groups cut the (group, cell) pairs the correction
 * pays for and raise the interactions the force pays for, so the corrected
 * step has its own best group size.  corr_kind -1 is otoo_autotune.  The
 * context's tuning (net_kernel included) is restored afterwards.  EINVAL as
 * otoo_autotune, and for another corr_kind or a missing network. */
int otoo_autotune_step(otoo_ctx* ctx, const otoo_tree* tree, const otoo_walk_params* walk,
                       const otoo_group_choice* choices, int32_t n_choices, const otoo_tuning* schedules,
                       int32_t n_schedules, float eps, int32_t corr_kind, otoo_mlp* mlp, int32_t reps, float* ms,
                       int64_t* interactions, otoo_group_choice* best_choice, otoo_tuning* best_tuning,
                       float* best_ms);

/* Synchronise the context's stream and report whether any kernel since the
 * last otoo_check met malformed input (EINVAL) or not (OK); clears the flag. */
int otoo_check(otoo_ctx* ctx);

/* Timing of the last otoo_force on the context stream (ms of the force
 * kernel alone and of the whole call), taken with HIP events when
 * enable != 0 (set with otoo_enable_timing). */
int otoo_enable_timing(otoo_ctx* ctx, int32_t enable);
int otoo_last_timing(otoo_ctx* ctx, float* ms_force_kernel, float* ms_total);

/* Capture the exact sequence otoo_force would enqueue for these arguments
 * into a HIP graph held by the context (replacing any previous one), and
 * replay it with otoo_graph_launch on the context stream.  The pointers are
 * baked into the graph; list contents may change between replays as long as
 * n_groups, n_entries and the pointers stay the same.  The graph also names
 * the context's scratch: a later otoo_force that needs more scratch than the
 * context holds reallocates it and discards the graph (otoo_graph_launch then
 * returns EINVAL).  Graphs that a caller captures around calls of this library
 * must likewise be captured again after a call that grows the context's
 * scratch. */
int otoo_graph_capture(otoo_ctx* ctx, int32_t n, const float* pos, const float* mass, int32_t n_groups,
                       const int32_t* group_off, int64_t n_entries, const int64_t* list_off,
                       const int32_t* list_idx, int32_t n_cells, const float* cell_mom, int32_t cell_stride,
                       float eps, const float* gcorr, float* out_acc, double* out_pot);
int otoo_graph_launch(otoo_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* OTOO_H */
