// Closing a chain step on the device (Eq. bi): b_{i+1} = ||u_{i+1}|| from the restrict's
// per-cell partials of ||u||^2, the breakdown test, s_{i+1} = 1 / b_{i+1}, and the next
// copy of the chain state.  Every block that calls it adds the partials in the same fixed
// order, so all blocks agree on the scales; block 0 writes b_{i+1} and the state.
#pragma once

#include <hip/hip_runtime.h>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

// LDS of one call: the wavefront sums, then the scale of every right-hand side
struct CloseLds {
    double red[2 * kMaxRhs][kBlock / kWave];
    double scale[kMaxRhs];
};

// Requires every thread of the block, blockDim.x a multiple of 64 and at most kBlock; MODE
// is COLLAPSE_INIT or COLLAPSE_STEP.  Thread r < n_rhs handles chain r; its state and step scalars are loaded
// before the partial sums, so their latency overlaps them.  On return lds.scale[r] holds
// s_{i+1} of chain r (0 for a chain that stopped), valid in every thread.
template <int MODE>
__device__ __forceinline__ void close_chain_step(const double* __restrict__ rpart, int ncells,
                                                 const ChainState* __restrict__ cs_in,
                                                 const StepScalars* __restrict__ pend, ChainState* __restrict__ cs_out,
                                                 double* __restrict__ beta, int ldb, int step, double tol2, int n_rhs,
                                                 CloseLds& lds) {
    const int r = threadIdx.x;
    ChainState st{};
    StepScalars sc{};
    if (MODE != COLLAPSE_INIT && r < n_rhs) {
        st = cs_in[r];
        sc = pend[r];
    }
    // per-thread partial sums of ||u||^2 (and ||P||^2) for every right-hand side, then
    // one block reduction in a fixed order
    const int nval = 2 * n_rhs;
    double acc[2 * kMaxRhs];
#pragma unroll
    for (int q = 0; q < 2 * kMaxRhs; ++q) acc[q] = 0.0;
    const int nt = blockDim.x;
    for (int c0 = 0; c0 < ncells; c0 += 2 * nt) {
        double v[2][2 * kMaxRhs];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = min(c0 + (int)threadIdx.x + u * nt, ncells - 1);
#pragma unroll
            for (int q = 0; q < 2 * kMaxRhs; ++q) v[u][q] = q < nval ? rpart[(int64_t)c * nval + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (c0 + (int)threadIdx.x + u * nt < ncells)
#pragma unroll
                for (int q = 0; q < 2 * kMaxRhs; ++q) acc[q] += v[u][q];
    }
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < 2 * kMaxRhs; ++q) {
        if (q >= nval) break;
        const double w = wave_sum(acc[q]);
        if (threadIdx.x % kWave == 0) lds.red[q][wave] = w;
    }
    __syncthreads();
    if (r < n_rhs) {
        double uu = 0.0, pp = 0.0;
        for (int w = 0; w < nt / kWave; ++w) {
            uu += lds.red[2 * r][w];
            pp += lds.red[2 * r + 1][w];
        }
        ChainState nx;
        double b = 0.0;
        if (MODE == COLLAPSE_INIT) {
            nx.pnorm2 = pp;
            nx.s_prev = 0.0;
            nx.b_cur = 0.0;
            nx.steps = 0;
            nx.pad = 0;
            if (uu > 0.0 && isfinite(uu)) {
                nx.active = 1;
                nx.s_cur = 1.0 / sqrt(uu);
                nx.status = BSE_OK;
            } else {
                nx.active = 0;
                nx.s_cur = 0.0;
                nx.status = (uu == 0.0) ? BSE_INFO_ZERO_START : BSE_ERR_NONFINITE;
            }
        } else {
            nx = st;
            nx.s_prev = st.s_cur;
            nx.s_cur = 0.0;
            nx.b_cur = 0.0;
            if (st.active) {
                if (!sc.ok) {
                    nx.status = BSE_ERR_NONFINITE;
                    nx.active = 0;
                } else {
                    nx.steps = step + 1;   // a_{step+1} is valid
                    if (!isfinite(uu)) {
                        nx.status = BSE_ERR_NONFINITE;
                        nx.active = 0;
                    } else if (uu <= tol2 * sc.ww) {
                        nx.status = BSE_INFO_INVARIANT_SUBSPACE;  // b_{i+1} = 0: exact chain end
                        nx.active = 0;
                    } else {
                        b = sqrt(uu);
                        nx.b_cur = b;
                        nx.s_cur = 1.0 / b;
                    }
                }
            }
        }
        lds.scale[r] = nx.s_cur;
        if (blockIdx.x == 0) {
            cs_out[r] = nx;
            if (MODE == COLLAPSE_STEP && b > 0.0) beta[(int64_t)r * ldb + step + 1] = b;
        }
    }
    __syncthreads();
}

}  // namespace bse
