// Step orchestration pieces of the interpolated BSE matvec and Haydock chain (gfx950).
//
// One step of the chain (Sec. 4, Eqs. matmul1-matmul3 inside Eqs. ai-ci).  The
// chain keeps unnormalised vectors u_j, psi_j = s_j u_j, with the scales in a
// small device-side state, so that b_{i+1} is the norm of the vector actually
// formed without an extra pass over memory:
//   k_gemv2     r = K_c qbar by column splits, k_gemv_reduce adds the splits
//               (gemv.hip; Eq. matmul2, corner sum collapsed)
//   k_prolong3  w = delta psi_i + C^H r - b_i psi_{i-1} and a_i   (prolong.hip;
//               Eq. matmul3, Eq. bse1 diagonal, Eq. ai)
//   k_restrict3 u_{i+1} = w - a_i psi_i, b_{i+1} = ||u_{i+1}||, then the
//               per-(cell, corner) coarse vectors of u_{i+1}  (restrict.hip;
//               Eqs. bi, ci, matmul1)
//   k_collapse  qbar(k~) = s_{i+1} x sum of the 8 (cell, corner) vectors on k~
// No kernel waits on another block: each kernel leaves per-block partials that the
// next kernel in the stream adds in a fixed order.  This file holds the collapse
// (which closes a chain step), the chain report and the dispatch on band counts and
// storage precision.  Every sum is FP64; reductions use fixed
// trees, so results do not depend on scheduling.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "bse_device.hpp"
#include "bse_plan.hpp"
#include "chain_close.hpp"

namespace bse {

// ------------------------------------------------------------------------------------
// collapse: qbar[(k~ NP + p) n_rhs + r] = s_r sum_z qpart[cell_of_corner(k~, z)][z][r][p]
//
// In a chain the collapse closes the step (chain_close.hpp): every block adds the
// restrict's per-cell ||u||^2 partials (same fixed order in every block), so all blocks
// agree on b_{i+1} = ||u_{i+1}|| (Eq. bi), the breakdown test and s_{i+1} = 1 / b_{i+1};
// block 0 writes b_{i+1} and the next copy of the chain state.
// ------------------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_collapse(const double2* __restrict__ qpart, double2* __restrict__ qbar,
                                                  const ChainState* __restrict__ cs_in,
                                                  const StepScalars* __restrict__ pend,
                                                  const double* __restrict__ rpart, ChainState* __restrict__ cs_out,
                                                  double* __restrict__ beta, int ldb, int step, double tol2,
                                                  int n_c, int np, int n_rhs, int64_t total,
                                                  unsigned short* __restrict__ qfrag, int qfmt,
                                                  float* __restrict__ qsinv) {
    __shared__ CloseLds cl;
    __shared__ unsigned smax[kMaxRhs];
    // this thread's 8 (cell, corner) vectors: loaded first (indices clamped), so their
    // latency overlaps the chain reductions below
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ic = i < total ? i : total - 1;
    const int r0 = (int)(ic % n_rhs);
    const int64_t T = ic / n_rhs;
    const int p = (int)(T % np);
    const int k = (int)(T / np);
    double2 qv[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) qv[z] = qpart[((int64_t)(cell_of_corner(k, z, n_c) * 8 + z) * n_rhs + r0) * np + p];
    if (MODE != COLLAPSE_PLAIN)
        close_chain_step<MODE>(rpart, n_c * n_c * n_c, cs_in, pend, cs_out, beta, ldb, step, tol2, n_rhs, cl);
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        re += qv[z].x;
        im += qv[z].y;
    }
    const double sc = (MODE == COLLAPSE_PLAIN) ? 1.0 : cl.scale[r0];   // psi = s u in a chain
    re *= sc;
    im *= sc;
    double qs = 1.0;
    if (qfmt == BSE_F16_KC) {
        // FP16: the block is one 64-column group of qbar (64 n_rhs threads); each
        // right-hand side of the group gets the power of two that puts its largest entry
        // in [2^14, 2^15), so no encoding overflows whatever the vector's norm; the
        // product divides it out with the block scale of K_c
        if ((int)threadIdx.x < n_rhs) smax[threadIdx.x] = 0u;
        __syncthreads();
        if (i < total) atomicMax(&smax[r0], __float_as_uint((float)fmax(fabs(re), fabs(im))));
        __syncthreads();
        // m < 2^e; a zero or non-finite group keeps the scale 1
        auto expo = [](float m) { return (m > 0.0f && isfinite(m)) ? ilogbf(m) + 1 : 15; };
        qs = ldexp(1.0, 15 - expo(__uint_as_float(smax[r0])));
        if ((int)threadIdx.x < n_rhs)
            qsinv[(int64_t)blockIdx.x * kMaxRhs + threadIdx.x] = ldexpf(1.0f, expo(__uint_as_float(smax[threadIdx.x])) - 15);
    }
    if (i >= total) return;
    qbar[i] = make_double2(re, im);
    if (qfmt != 0) {
        // low-precision forms: qbar as matrix-core B fragments (see gemv.hip), leading
        // part and remainder in the storage format, two variants per 32-column step
        const double vr = re * qs, vi = im * qs;
        const unsigned short hr = enc_lowp(qfmt, (float)vr), hi = enc_lowp(qfmt, (float)vi);
        const unsigned short lr = enc_lowp(qfmt, (float)(vr - (double)dec_lowp(qfmt, hr)));
        const unsigned short li = enc_lowp(qfmt, (float)(vi - (double)dec_lowp(qfmt, hi)));
        const int64_t j = T;  // column of K_c
        const int64_t g = j / 32;
        const int kk = (int)(j % 32), lg = kk / 8, ent = kk % 8;
        unsigned short* b1 = qfrag + ((g * 2 + 0) * kWave + lg * 16) * 8 + ent;
        unsigned short* b2 = qfrag + ((g * 2 + 1) * kWave + lg * 16) * 8 + ent;
        const unsigned short sign = 0x8000;
        b1[(r0) * 8] = hr;
        b1[(4 + r0) * 8] = hi;
        b1[(8 + r0) * 8] = lr;
        b1[(12 + r0) * 8] = li;
        b2[(r0) * 8] = hi ^ sign;
        b2[(4 + r0) * 8] = hr;
        b2[(8 + r0) * 8] = li ^ sign;
        b2[(12 + r0) * 8] = lr;
    }
}

__global__ void k_chain_report(const ChainState* __restrict__ chain, double* pnorm2, int32_t* steps,
                               int32_t* status, int n_rhs) {
    const int r = threadIdx.x;
    if (r < n_rhs) {
        pnorm2[r] = chain[r].pnorm2;
        steps[r] = chain[r].steps;
        status[r] = chain[r].status;
    }
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
        case BSE_BF16_KC:
        case BSE_F16_KC:
            return restrict_launch<float2, float2, NV, NC>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
        default:
            return restrict_launch<float2, double2, NV, NC>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
    }
}

template <int NV, int NC>
static hipError_t prolong_dt(const Plan& p, int mode, const void* x, void* out, int step, int n_rhs,
                             hipStream_t s) {
    switch (p.g.dtype) {
        case BSE_F64: return prolong_launch<double2, double2, NV, NC>(p, mode, x, out, step, n_rhs, s);
        case BSE_F32:
        case BSE_BF16_KC:
        case BSE_F16_KC: return prolong_launch<float2, float2, NV, NC>(p, mode, x, out, step, n_rhs, s);
        default: return prolong_launch<float2, double2, NV, NC>(p, mode, x, out, step, n_rhs, s);
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
    switch (p.g.dtype) {
        case BSE_F64:
            return restrict_any_launch<double2, double2>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
        case BSE_F32:
        case BSE_BF16_KC:
        case BSE_F16_KC:
            return restrict_any_launch<float2, float2>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
        default:
            return restrict_any_launch<float2, double2>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
    }
}

hipError_t launch_prolong(const Plan& p, int mode, const void* x, void* out, int step, int n_rhs, hipStream_t s) {
    const int nv = p.g.nv, nc = p.g.nc;
#define BSE_CASE(a_, b_) \
    if (nv == a_ && nc == b_) return prolong_dt<a_, b_>(p, mode, x, out, step, n_rhs, s);
    BSE_BANDS(BSE_CASE)
#undef BSE_CASE
    switch (p.g.dtype) {
        case BSE_F64: return prolong_any_launch<double2, double2>(p, mode, x, out, step, n_rhs, s);
        case BSE_F32:
        case BSE_BF16_KC:
        case BSE_F16_KC: return prolong_any_launch<float2, float2>(p, mode, x, out, step, n_rhs, s);
        default: return prolong_any_launch<float2, double2>(p, mode, x, out, step, n_rhs, s);
    }
}

hipError_t launch_collapse(const Plan& p, int mode, int step, double* b, int ldb, int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    const int64_t total = g.Nc * n_rhs;
    // FP16 coarse kernel: one block per 64-column group of qbar (see k_collapse)
    const bool grouped = g.dtype == BSE_F16_KC;
    const int bt = grouped ? kKqBlock * n_rhs : kBlock;
    const int nb = grouped ? kq_shape(g.Nc).nb : (int)((total + kBlock - 1) / kBlock);
    float* qsinv = grouped ? reinterpret_cast<float*>(p.ws + p.L.qsinv) : nullptr;
    const double2* qpart = reinterpret_cast<const double2*>(p.ws + p.L.qpart);
    double2* qbar = reinterpret_cast<double2*>(p.ws + p.L.qbar);
    ChainState* cs = reinterpret_cast<ChainState*>(p.ws + p.L.chain);
    const StepScalars* pend = reinterpret_cast<const StepScalars*>(p.ws + p.L.pend);
    const double* rpart = reinterpret_cast<const double*>(p.ws + p.L.rpart);
    const double tol = breakdown_tol(g.dtype);
    unsigned short* qf = kc_lowp(g.dtype) ? reinterpret_cast<unsigned short*>(p.ws + p.L.qfrag) : nullptr;
    const int qfmt = kc_lowp(g.dtype) ? g.dtype : 0;
    // the chain start writes copy 0, step i reads copy i % 2 and writes copy (i + 1) % 2
    const ChainState* cin = cs + state_in(step) * kMaxRhs;
    ChainState* cout = (mode == COLLAPSE_INIT) ? cs : cs + state_out(step) * kMaxRhs;
    if (mode == COLLAPSE_PLAIN)
        hipLaunchKernelGGL(k_collapse<COLLAPSE_PLAIN>, dim3(nb), dim3(bt), 0, s, qpart, qbar, cin, pend, rpart,
                           cout, b, ldb, step, tol * tol, g.n_c, g.np, n_rhs, total, qf, qfmt, qsinv);
    else if (mode == COLLAPSE_INIT)
        hipLaunchKernelGGL(k_collapse<COLLAPSE_INIT>, dim3(nb), dim3(bt), 0, s, qpart, qbar, cin, pend, rpart,
                           cout, b, ldb, step, tol * tol, g.n_c, g.np, n_rhs, total, qf, qfmt, qsinv);
    else
        hipLaunchKernelGGL(k_collapse<COLLAPSE_STEP>, dim3(nb), dim3(bt), 0, s, qpart, qbar, cin, pend, rpart,
                           cout, b, ldb, step, tol * tol, g.n_c, g.np, n_rhs, total, qf, qfmt, qsinv);
    return hipGetLastError();
}

hipError_t launch_chain_report(const Plan& p, int n_steps, double* pnorm2, int32_t* steps, int32_t* status,
                               int n_rhs, hipStream_t s) {
    const ChainState* cs = reinterpret_cast<const ChainState*>(p.ws + p.L.chain) + state_in(n_steps) * kMaxRhs;
    hipLaunchKernelGGL(k_chain_report, dim3(1), dim3(kWave), 0, s, cs, pnorm2, steps, status, n_rhs);
    return hipGetLastError();
}

}  // namespace bse
