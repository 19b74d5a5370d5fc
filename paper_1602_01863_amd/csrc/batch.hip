// Batched Haydock chains: many plans (Hamiltonians of different sizes, with their
// right-hand sides) advanced by a few HIP graphs that run side by side.
//
// bse_batch_create deals the plans to n_branches branches, largest first (by the
// bytes of one step), and records each branch's runs (chain start, n_steps steps of
// coarse product, prolong, update + restrict and collapse, chain report; plan after
// plan) by stream capture into one graph per branch, instantiated once.
// bse_batch_launch forks the caller's stream onto the batch's own streams (one per
// branch, default priority), launches each branch's graph there and joins back, so
// the host issues one graph launch per branch instead of thousands of kernel
// launches, and the branches run concurrently on the device.  (Parallel branches
// inside a single graph ran largely one after another on this runtime; separate
// graphs on separate streams overlap.)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "bse_plan.hpp"

struct bse_batch {
    int n_plans;
    int n_branches;
    hipGraph_t graph[16];
    hipGraphExec_t exec[16];
    hipStream_t stream[16];
    hipEvent_t join[16];
    hipEvent_t fork;
};

static void batch_release(bse_batch* bt) {
    for (int k = 0; k < 16; ++k) {
        if (bt->exec[k]) (void)hipGraphExecDestroy(bt->exec[k]);
        if (bt->graph[k]) (void)hipGraphDestroy(bt->graph[k]);
        if (bt->join[k]) (void)hipEventDestroy(bt->join[k]);
        if (bt->stream[k]) (void)hipStreamDestroy(bt->stream[k]);
    }
    if (bt->fork) (void)hipEventDestroy(bt->fork);
    delete bt;
}

namespace bse {

// bytes one step of a plan streams (coarse kernel + overlaps twice + vectors), for balancing
static double step_cost(const Plan& p, int n_rhs) {
    const double kb = p.g.dtype == BSE_F64 ? 16.0 : (kc_lowp(p.g.dtype) ? 4.0 : 8.0);
    const double vb = vec_is_f32(p.g.dtype) ? 8.0 : 16.0;
    return kb * (double)p.g.Nc * (double)p.g.Nc + 2.0 * 8.0 * p.g.ncells * 8.0 * p.g.ne * p.g.ndiv3 +
           6.0 * vb * (double)p.g.N * n_rhs;
}

}  // namespace bse

using namespace bse;

extern "C" {

bse_status bse_batch_create(bse_plan* const* plans, int32_t n_plans, const double* const* P, const int32_t* n_rhs,
                            int32_t n_steps, double* const* a, double* const* b, double* const* pnorm2,
                            int32_t* const* steps_done, int32_t* const* status, int32_t n_branches,
                            bse_batch** batch_out) {
    if (!batch_out) {
        set_error("bse_batch_create: batch_out is NULL");
        return BSE_ERR_INVALID_ARG;
    }
    *batch_out = nullptr;
    if (!plans || !P || !n_rhs || !a || !b || !pnorm2 || !steps_done || !status || n_plans < 1 || n_steps < 1 ||
        n_branches < 1 || n_branches > 16) {
        set_error("bse_batch_create: NULL array, n_plans < 1, n_steps < 1 or n_branches outside [1, 16]");
        return BSE_ERR_INVALID_ARG;
    }
    for (int i = 0; i < n_plans; ++i) {
        if (!plans[i] || !P[i] || !a[i] || !b[i] || !pnorm2[i] || !steps_done[i] || !status[i]) {
            set_error("bse_batch_create: NULL entry for plan %d", i);
            return BSE_ERR_INVALID_ARG;
        }
        const Plan& p = *reinterpret_cast<const Plan*>(plans[i]);
        if (n_rhs[i] < 1 || n_rhs[i] > p.g.max_rhs) {
            set_error("bse_batch_create: n_rhs of plan %d must be in [1, %d]", i, p.g.max_rhs);
            return BSE_ERR_INVALID_ARG;
        }
        if (p.timing) {
            set_error("bse_batch_create: plan %d has kernel timing enabled", i);
            return BSE_ERR_INVALID_ARG;
        }
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) {
                set_error("bse_batch_create: plan %d appears twice (its workspace would be shared)", i);
                return BSE_ERR_INVALID_ARG;
            }
    }
    n_branches = std::min(n_branches, n_plans);
    // largest first, each to the branch with the least load so far
    std::vector<int> order(n_plans);
    for (int i = 0; i < n_plans; ++i) order[i] = i;
    std::vector<double> cost(n_plans);
    for (int i = 0; i < n_plans; ++i) cost[i] = step_cost(*reinterpret_cast<const Plan*>(plans[i]), n_rhs[i]);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<double> load(n_branches, 0.0);
    std::vector<int> branch(n_plans, 0);
    for (int i : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        branch[i] = k;
        load[k] += cost[i];
    }

    bse_batch* bt = new (std::nothrow) bse_batch();
    if (!bt) {
        set_error("bse_batch_create: out of host memory");
        return BSE_ERR_INVALID_ARG;
    }
    bt->n_plans = n_plans;
    bt->n_branches = n_branches;
    hipError_t e = hipEventCreateWithFlags(&bt->fork, hipEventDisableTiming);
    for (int k = 0; k < n_branches && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&bt->stream[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->join[k], hipEventDisableTiming);
    }
    // one capture per branch: its plans' runs, in dealing order
    for (int k = 0; k < n_branches && e == hipSuccess; ++k) {
        e = hipStreamBeginCapture(bt->stream[k], hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) break;
        for (int i : order) {
            if (branch[i] != k || e != hipSuccess) continue;
            Plan& p = *reinterpret_cast<Plan*>(plans[i]);
            e = enqueue_haydock(p, P[i], n_rhs[i], n_steps, a[i], b[i], pnorm2[i], steps_done[i], status[i],
                                bt->stream[k]);
        }
        const hipError_t e2 = hipStreamEndCapture(bt->stream[k], &bt->graph[k]);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&bt->exec[k], bt->graph[k], nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
        batch_release(bt);
        return hip_fail_status(e, "bse_batch_create");
    }
    *batch_out = bt;
    return BSE_OK;
}

bse_status bse_batch_launch(bse_batch* batch, hipStream_t stream) {
    if (!batch) {
        set_error("bse_batch_launch: NULL batch");
        return BSE_ERR_INVALID_ARG;
    }
    hipError_t e = hipEventRecord(batch->fork, stream);
    for (int k = 0; k < batch->n_branches && e == hipSuccess; ++k) e = hipStreamWaitEvent(batch->stream[k], batch->fork, 0);
    for (int k = 0; k < batch->n_branches && e == hipSuccess; ++k) e = hipGraphLaunch(batch->exec[k], batch->stream[k]);
    for (int k = 0; k < batch->n_branches && e == hipSuccess; ++k) e = hipEventRecord(batch->join[k], batch->stream[k]);
    for (int k = 0; k < batch->n_branches && e == hipSuccess; ++k) e = hipStreamWaitEvent(stream, batch->join[k], 0);
    return e == hipSuccess ? BSE_OK : hip_fail_status(e, "bse_batch_launch");
}

void bse_batch_destroy(bse_batch* batch) {
    if (!batch) return;
    batch_release(batch);
}

}  // extern "C"
