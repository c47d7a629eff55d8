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

extern "C" int otoo_autotune(otoo_ctx* c, const otoo_tree* tree, const otoo_walk_params* walk,
                             const otoo_group_choice* choices, int32_t n_choices, const otoo_tuning* schedules,
                             int32_t n_schedules, float eps, int32_t reps, float* ms, int64_t* interactions,
                             otoo_group_choice* best_choice, otoo_tuning* best_tuning, float* best_ms) {
    if (!c) return OTOO_EINVAL;
    c->err.clear();
    if (!tree || !walk || !choices || !schedules || !best_choice || !best_tuning || !best_ms)
        return fail(c, OTOO_EINVAL, "null pointer argument");
    if (n_choices < 1 || n_schedules < 1 || reps < 1) return fail(c, OTOO_EINVAL, "bad sizes");
    if (!(eps > 0.f) || !std::isfinite(eps)) return fail(c, OTOO_EINVAL, "eps must be positive and finite");
    HIP_TRY(c, hipSetDevice(c->device));
    int64_t n = 0, n_cells = 0;
    int rc = otoo_tree_info(tree, &n, &n_cells, nullptr, nullptr, nullptr);
    if (rc) return fail(c, rc, "otoo_tree_info failed");
    if (n < 1 || n > (1 << 30)) return fail(c, OTOO_EINVAL, "tree size out of range");
    std::vector<float> pos((size_t)n * 3), mass((size_t)n), cm((size_t)std::max<int64_t>(n_cells, 1) * 4);
    rc = otoo_tree_export(tree, nullptr, pos.data(), mass.data(), cm.data(), 4);
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
        int64_t* d_lo;
        HIP_TRY(c, lists.alloc(&d_go, (size_t)L.n_groups + 1));
        HIP_TRY(c, lists.alloc(&d_lo, (size_t)L.n_groups + 1));
        HIP_TRY(c, lists.alloc(&d_li, (size_t)L.n_entries));
        HIP_TRY(c, hipMemcpy(d_go, L.group_off, sizeof(int32_t) * (L.n_groups + 1), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(d_lo, L.list_off, sizeof(int64_t) * (L.n_groups + 1), hipMemcpyHostToDevice));
        if (L.n_entries)
            HIP_TRY(c, hipMemcpy(d_li, L.list_idx, sizeof(int32_t) * L.n_entries, hipMemcpyHostToDevice));
        for (int32_t si = 0; si < n_schedules; si++) {
            otoo_tuning t = schedules[si];
            t.debug_validate = 0;
            t.net_kernel = tg.saved.net_kernel;
            c->tune = tg.saved;   // a zero field means the caller's value, not the previous schedule's
            rc = otoo_set_tuning(c, &t);
            if (rc) return rc;
            rc = otoo_graph_capture(c, (int32_t)n, d_pos, d_mass, L.n_groups, d_go, L.n_entries, d_lo, d_li,
                                    (int32_t)n_cells, d_cm, 4, eps, nullptr, d_acc, d_pot);
            if (rc) return rc;
            for (int w = 0; w < 2; w++) {
                rc = otoo_graph_launch(c);
                if (rc) return rc;
            }
            HIP_TRY(c, hipEventRecord(e0, c->stream));
            for (int r = 0; r < reps; r++) {
                rc = otoo_graph_launch(c);
                if (rc) return rc;
            }
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
