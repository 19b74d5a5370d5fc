// Step orchestration pieces of the interpolated BSE matvec and Haydock chain (gfx950).
//
// One step of the chain (Sec. 4, Eqs. matmul1-matmul3 inside Eqs. ai-ci).  The
// chain keeps unnormalised vectors u_j, psi_j = s_j u_j, with the scales in a
// small device-side state, so that b_{i+1} is the norm of the vector actually
// formed without an extra pass over memory:
//   k_gemv2     r = K_c qbar           (gemv.hip; Eq. matmul2, corner sum collapsed)
//   k_prolong2  w = delta psi_i + C^H r - b_i psi_{i-1} and a_i   (prolong.hip;
//               Eq. matmul3, Eq. bse1 diagonal, Eq. ai)
//   k_restrict2 u_{i+1} = w - a_i psi_i, b_{i+1} = ||u_{i+1}||, then the
//               per-(cell, corner) coarse vectors of u_{i+1}  (restrict.hip;
//               Eqs. bi, ci, matmul1)
//   k_collapse  qbar(k~) = s_{i+1} x sum of the 8 (cell, corner) vectors on k~
// This file holds the collapse, the chain report, counter reset and the dispatch
// on band counts and storage precision.  Every sum is FP64; reductions use fixed
// trees, so results do not depend on scheduling.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

// ------------------------------------------------------------------------------------
// collapse: qbar[(k~ NP + p) n_rhs + r] = sum_z qpart[cell_of_corner(k~, z)][z][r][p]
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_collapse(const double2* __restrict__ qpart,
                                                  double2* __restrict__ qbar, const ChainState* __restrict__ chain,
                                                  int n_c, int np, int n_rhs, int64_t total) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int r = (int)(i % n_rhs);
    const int64_t T = i / n_rhs;
    const int p = (int)(T % np);
    const int k = (int)(T / np);
    double re = 0.0, im = 0.0;
    for (int z = 0; z < 8; ++z) {
        const int cell = cell_of_corner(k, z, n_c);
        const double2 v = qpart[((int64_t)(cell * 8 + z) * n_rhs + r) * np + p];
        re += v.x;
        im += v.y;
    }
    const double s = chain ? chain[r].s_cur : 1.0;   // psi = s u in a chain
    qbar[i] = make_double2(s * re, s * im);
}

// ------------------------------------------------------------------------------------
// chain outputs and counters
// ------------------------------------------------------------------------------------
__global__ void k_chain_report(const ChainState* __restrict__ chain, double* pnorm2, int32_t* steps,
                               int32_t* status, int n_rhs) {
    const int r = threadIdx.x;
    if (r < n_rhs) {
        pnorm2[r] = chain[r].pnorm2;
        steps[r] = chain[r].steps;
        status[r] = chain[r].status;
    }
}

__global__ void k_zero_u32(unsigned int* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ------------------------------------------------------------------------------------
// dispatch on band counts and storage precision
// ------------------------------------------------------------------------------------
bool supported_bands(int nv, int nc) {
#define BSE_CHECK(a, b) \
    if (nv == a && nc == b) return true;
    BSE_BANDS(BSE_CHECK)
#undef BSE_CHECK
    return false;
}

template <int NV, int NC>
static hipError_t restrict_dt(const Plan& p, int mode, const void* x, const void* w, const void* psi,
                              const double* P, void* out, int step, double* a, double* b, int lda, int ldb,
                              int n_rhs, hipStream_t s) {
    switch (p.g.dtype) {
        case BSE_F64:
            return restrict_launch<double2, double2, NV, NC>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
        case BSE_F32:
            return restrict_launch<float2, float2, NV, NC>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
        default:
            return restrict_launch<float2, double2, NV, NC>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
    }
}

template <int NV, int NC>
static hipError_t prolong_dt(const Plan& p, int mode, const void* x, void* out, int step, double* a, int lda,
                             int n_rhs, hipStream_t s) {
    switch (p.g.dtype) {
        case BSE_F64: return prolong_launch<double2, double2, NV, NC>(p, mode, x, out, step, a, lda, n_rhs, s);
        case BSE_F32: return prolong_launch<float2, float2, NV, NC>(p, mode, x, out, step, a, lda, n_rhs, s);
        default: return prolong_launch<float2, double2, NV, NC>(p, mode, x, out, step, a, lda, n_rhs, s);
    }
}

hipError_t launch_restrict(const Plan& p, int mode, const void* x, const void* w, const void* psi,
                           const double* P, void* out, int step, double* a, double* b, int lda, int ldb,
                           int n_rhs, hipStream_t s) {
    const int nv = p.g.nv, nc = p.g.nc;
#define BSE_CASE(a_, b_) \
    if (nv == a_ && nc == b_) return restrict_dt<a_, b_>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
    BSE_BANDS(BSE_CASE)
#undef BSE_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_prolong(const Plan& p, int mode, const void* x, void* out, int step, double* a,
                          double* b, int lda, int ldb, int n_rhs, hipStream_t s) {
    (void)b;
    (void)ldb;
    const int nv = p.g.nv, nc = p.g.nc;
#define BSE_CASE(a_, b_) \
    if (nv == a_ && nc == b_) return prolong_dt<a_, b_>(p, mode, x, out, step, a, lda, n_rhs, s);
    BSE_BANDS(BSE_CASE)
#undef BSE_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_collapse(const Plan& p, int n_rhs, bool scaled, hipStream_t s) {
    const Geometry& g = p.g;
    const int64_t total = g.Nc * n_rhs;
    const int nb = (int)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_collapse, dim3(nb), dim3(kBlock), 0, s,
                       reinterpret_cast<const double2*>(p.ws + p.L.qpart),
                       reinterpret_cast<double2*>(p.ws + p.L.qbar),
                       scaled ? reinterpret_cast<const ChainState*>(p.ws + p.L.chain) : nullptr, g.n_c, g.np, n_rhs,
                       total);
    return hipGetLastError();
}

hipError_t launch_chain_report(const Plan& p, double* pnorm2, int32_t* steps, int32_t* status, int n_rhs,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_chain_report, dim3(1), dim3(kWave), 0, s,
                       reinterpret_cast<const ChainState*>(p.ws + p.L.chain), pnorm2, steps, status, n_rhs);
    return hipGetLastError();
}

hipError_t launch_zero_counters(const Plan& p, hipStream_t s) {
    // counters are contiguous: gcount, pcount, rcount (256-byte regions)
    const int64_t n = (int64_t)((p.L.rcount + 256 - p.L.gcount) / sizeof(unsigned int));
    hipLaunchKernelGGL(k_zero_u32, dim3(8), dim3(kBlock), 0, s,
                       reinterpret_cast<unsigned int*>(p.ws + p.L.gcount), n);
    return hipGetLastError();
}

}  // namespace bse
