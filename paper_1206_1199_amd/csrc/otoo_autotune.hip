// Autotuner of the force evaluation: host code on the HIP runtime that
// walks the tree for each group choice and times each device schedule as
// replays of the captured force graph (the group size n_vec of Sec. 3.4's
// vectorised walk and the kernel schedule are the knobs).
#include <algorithm>
#include <cmath>
#include <vector>

#include "otoo_internal.h"

using namespace otoo_detail;

namespace {

// Device buffers of one autotuning call, freed on every exit path once the
// stream that reads them has drained.
struct DeviceBufs {
    hipStream_t stream;
    std::vector<void*> ptrs;
    ~DeviceBufs() {
        (void)hipStreamSynchronize(stream);
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t alloc(T** p, size_t count) {
        void* v = nullptr;
        const hipError_t e = hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) ptrs.push_back(v);
        *p = static_cast<T*>(v);
        return e;
    }
};

struct ListsGuard {
    otoo_lists* l = nullptr;
    ~ListsGuard() {
        if (l) otoo_lists_free(l);
    }
};

// Restores the caller's tuning and drops the graph captured here, whose
// baked-in pointers outlive the buffers they name.
struct CtxGuard {
    otoo_ctx* c;
    otoo_tuning saved;
    ~CtxGuard() {
        (void)hipStreamSynchronize(c->stream);
        if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->gexec = nullptr;
        c->graph = nullptr;
        c->tune = saved;
    }
};

}  // namespace

namespace {

// One timed step under stream capture: the correction pass (if any) and the
// force, as the caller would capture them.  Every scratch buffer is grown by
// an eager call first, so nothing is allocated inside the capture.
struct StepArgs {
    int32_t corr_kind;   // -1: the plain force
    otoo_mlp* mlp;
    int32_t n, n_groups, n_cells, stride;
    int64_t n_entries, n_pairs;
    const float *pos, *mass, *cm;
    const int32_t *go, *li;
    const float* gb;   // the walk's group boxes
    const int64_t *lo, *po;
    float eps;
    float* gcorr;
    float* acc;
    double* pot;
};

int step_enqueue(otoo_ctx* c, const StepArgs& s) {
    if (s.corr_kind >= 0) {
        const int rc = otoo_correction(c, s.corr_kind, s.mlp, s.n, s.pos, s.n_groups, s.go, s.gb, s.n_entries, s.lo,
                                       s.li,
                                       s.n_pairs, s.po, s.n_cells, s.cm, s.stride, s.eps, nullptr, s.gcorr);
        if (rc) return rc;
    }
    return otoo_force(c, s.n, s.pos, s.mass, s.n_groups, s.go, s.n_entries, s.lo, s.li, s.n_cells, s.cm, s.stride,
                      s.eps, s.corr_kind >= 0 ? s.gcorr : nullptr, s.acc, s.pot);
}

// Capture the step on the context's capture stream into an executable graph.
int step_capture(otoo_ctx* c, const StepArgs& s, hipGraphExec_t* exec) {
    int rc = step_enqueue(c, s);   // grows every scratch buffer outside the capture
    if (rc) return rc;
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = step_enqueue(c, s);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = user;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(c, OTOO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(c, OTOO_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    return OTOO_OK;
}

int autotune_impl(otoo_ctx* c, const otoo_tree* tree, const otoo_walk_params* walk, const otoo_group_choice* choices,
                  int32_t n_choices, const otoo_tuning* schedules, int32_t n_schedules, float eps, int32_t corr_kind,
                  otoo_mlp* mlp, int32_t reps, float* ms, int64_t* interactions, otoo_group_choice* best_choice,
                  otoo_tuning* best_tuning, float* best_ms) {
    if (!c) return OTOO_EINVAL;
    c->err.clear();
    if (!tree || !walk || !choices || !schedules || !best_choice || !best_tuning || !best_ms)
        return fail(c, OTOO_EINVAL, "null pointer argument");
    if (n_choices < 1 || n_schedules < 1 || reps < 1) return fail(c, OTOO_EINVAL, "bad sizes");
    if (!(eps > 0.f) || !std::isfinite(eps)) return fail(c, OTOO_EINVAL, "eps must be positive and finite");
    if (corr_kind != -1 && corr_kind != OTOO_CORR_QUAD && corr_kind != OTOO_CORR_MLP)
        return fail(c, OTOO_EINVAL, "corr_kind must be -1 (plain), OTOO_CORR_QUAD or OTOO_CORR_MLP");
    if (corr_kind == OTOO_CORR_MLP && !mlp) return fail(c, OTOO_EINVAL, "the learned correction needs a network");
    HIP_TRY(c, hipSetDevice(c->device));
    int64_t n = 0, n_cells = 0;
    int rc = otoo_tree_info(tree, &n, &n_cells, nullptr, nullptr, nullptr);
    if (rc) return fail(c, rc, "otoo_tree_info failed");
    if (n < 1 || n > (1 << 30)) return fail(c, OTOO_EINVAL, "tree size out of range");
    const int32_t stride = corr_kind >= 0 ? 12 : 4;
    std::vector<float> pos((size_t)n * 3), mass((size_t)n), cm((size_t)std::max<int64_t>(n_cells, 1) * stride);
    rc = otoo_tree_export(tree, nullptr, pos.data(), mass.data(), cm.data(), stride);
    if (rc) return fail(c, rc, "otoo_tree_export failed");

    DeviceBufs dev{c->stream, {}};
    float *d_pos, *d_mass, *d_cm, *d_acc;
    double* d_pot;
    HIP_TRY(c, dev.alloc(&d_pos, pos.size()));
    HIP_TRY(c, dev.alloc(&d_mass, mass.size()));
    HIP_TRY(c, dev.alloc(&d_cm, cm.size()));
    HIP_TRY(c, dev.alloc(&d_acc, pos.size()));
    HIP_TRY(c, dev.alloc(&d_pot, mass.size()));
    HIP_TRY(c, hipMemcpy(d_pos, pos.data(), pos.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(d_mass, mass.data(), mass.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(d_cm, cm.data(), cm.size() * sizeof(float), hipMemcpyHostToDevice));

    CtxGuard tg{c, c->tune};
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    struct EventGuard {
        hipEvent_t a, b;
        ~EventGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } eg{e0, e1};

    float best = -1.f;
    for (int32_t gi = 0; gi < n_choices; gi++) {
        otoo_walk_params wp = *walk;
        wp.group_mode = choices[gi].group_mode;
        wp.g_max = choices[gi].g_max;
        ListsGuard lg;
        rc = otoo_tree_walk(tree, &wp, &lg.l);
        if (rc) return fail(c, rc, "walk failed for group choice %d (mode %d, g_max %d)", gi, wp.group_mode, wp.g_max);
        const otoo_lists& L = *lg.l;
        if (interactions) interactions[gi] = L.interactions;
        DeviceBufs lists{c->stream, {}};
        int32_t *d_go, *d_li;
        int64_t *d_lo, *d_po = nullptr;
        float *d_gc = nullptr, *d_gb = nullptr;
        HIP_TRY(c, lists.alloc(&d_go, (size_t)L.n_groups + 1));
        HIP_TRY(c, lists.alloc(&d_lo, (size_t)L.n_groups + 1));
        HIP_TRY(c, lists.alloc(&d_li, (size_t)L.n_entries));
        HIP_TRY(c, hipMemcpy(d_go, L.group_off, sizeof(int32_t) * (L.n_groups + 1), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(d_lo, L.list_off, sizeof(int64_t) * (L.n_groups + 1), hipMemcpyHostToDevice));
        if (L.n_entries)
            HIP_TRY(c, hipMemcpy(d_li, L.list_idx, sizeof(int32_t) * L.n_entries, hipMemcpyHostToDevice));
        int64_t n_pairs = 0;
        if (corr_kind >= 0) {   // the (group, cell) pairs: prefix sums of the cell-entry counts (the near ones
                                // when the walk splits them)
            const int32_t* cnt = wp.near_ratio > 0.0 ? L.n_near : L.n_cellent;
            std::vector<int64_t> po((size_t)L.n_groups + 1, 0);
            for (int32_t g = 0; g < L.n_groups; g++) po[g + 1] = po[g] + cnt[g];
            n_pairs = po[L.n_groups];
            HIP_TRY(c, lists.alloc(&d_po, po.size()));
            HIP_TRY(c, lists.alloc(&d_gc, (size_t)L.n_groups * kCorrStride));
            HIP_TRY(c, lists.alloc(&d_gb, (size_t)L.n_groups * 6));
            HIP_TRY(c, hipMemcpy(d_po, po.data(), sizeof(int64_t) * po.size(), hipMemcpyHostToDevice));
            HIP_TRY(c, hipMemcpy(d_gb, L.group_box, sizeof(float) * 6 * (size_t)L.n_groups, hipMemcpyHostToDevice));
        }
        const StepArgs sa{corr_kind, mlp,  (int32_t)n, L.n_groups, (int32_t)n_cells, stride, L.n_entries, n_pairs,
                          d_pos,     d_mass, d_cm,   d_go,        d_li,             d_gb,   d_lo,        d_po,
                          eps,       d_gc,   d_acc,  d_pot};
        for (int32_t si = 0; si < n_schedules; si++) {
            otoo_tuning t = schedules[si];
            t.debug_validate = 0;
            t.net_kernel = tg.saved.net_kernel;
            t.corr_chunks = tg.saved.corr_chunks;
            c->tune = tg.saved;   // a zero field means the caller's value, not the previous schedule's
            rc = otoo_set_tuning(c, &t);
            if (rc) return rc;
            hipGraphExec_t exec = nullptr;
            rc = step_capture(c, sa, &exec);
            if (rc) return rc;
            struct ExecGuard {
                hipGraphExec_t e;
                hipStream_t s;
                ~ExecGuard() {
                    (void)hipStreamSynchronize(s);
                    (void)hipGraphExecDestroy(e);
                }
            } xg{exec, c->stream};
            for (int w = 0; w < 2; w++) HIP_TRY(c, hipGraphLaunch(exec, c->stream));
            HIP_TRY(c, hipEventRecord(e0, c->stream));
            for (int r = 0; r < reps; r++) HIP_TRY(c, hipGraphLaunch(exec, c->stream));
            HIP_TRY(c, hipEventRecord(e1, c->stream));
            HIP_TRY(c, hipEventSynchronize(e1));
            float t_ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&t_ms, e0, e1));
            t_ms /= (float)reps;
            if (ms) ms[(int64_t)gi * n_schedules + si] = t_ms;
            if (best < 0.f || t_ms < best) {
                best = t_ms;
                *best_choice = choices[gi];
                *best_tuning = c->tune;
            }
        }
        rc = otoo_check(c);
        if (rc) return rc;
    }
    *best_ms = best;
    return OTOO_OK;
}

}  // namespace

extern "C" int otoo_autotune(otoo_ctx* c, const otoo_tree* tree, const otoo_walk_params* walk,
                             const otoo_group_choice* choices, int32_t n_choices, const otoo_tuning* schedules,
                             int32_t n_schedules, float eps, int32_t reps, float* ms, int64_t* interactions,
                             otoo_group_choice* best_choice, otoo_tuning* best_tuning, float* best_ms) {
    return autotune_impl(c, tree, walk, choices, n_choices, schedules, n_schedules, eps, -1, nullptr, reps, ms,
                         interactions, best_choice, best_tuning, best_ms);
}

extern "C" int otoo_autotune_step(otoo_ctx* c, const otoo_tree* tree, const otoo_walk_params* walk,
                                  const otoo_group_choice* choices, int32_t n_choices, const otoo_tuning* schedules,
                                  int32_t n_schedules, float eps, int32_t corr_kind, otoo_mlp* mlp, int32_t reps,
                                  float* ms, int64_t* interactions, otoo_group_choice* best_choice,
                                  otoo_tuning* best_tuning, float* best_ms) {
    return autotune_impl(c, tree, walk, choices, n_choices, schedules, n_schedules, eps, corr_kind, mlp, reps, ms,
                         interactions, best_choice, best_tuning, best_ms);
}
