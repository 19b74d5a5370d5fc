// Coarse product r = K_c qbar (Eq. matmul2 with the corner sum collapsed) on gfx950.
//
// K_c is Hermitian and row-major, so r[i] = sum_j conj(K[j][i]) qbar[j]: a lane owns
// output rows and walks down columns j, and every load instruction of a wavefront
// reads one contiguous 1 KiB strip of row j (16 bytes per lane).  The product is
// bound by the HBM stream of K_c (n_rhs <= 4 right-hand sides per read), so the
// kernel is built for bytes in flight: one non-temporal 16-byte load per lane and
// column, 8 columns per lane in flight, <= 128 VGPRs (4 wavefronts per SIMD).  Sums
// are FP64.
//
// Grid: row blocks x column splits.  A block = 4 wavefronts on the same rows and
// interleaved columns of one column chunk; qbar for the chunk sits in LDS.  The 4
// wavefront partials are added in LDS in a fixed order and every block writes its
// split partial; k_gemv_reduce then adds the splits of each output in a fixed order.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

template <class M2>
struct Gv;
template <>
struct Gv<float2> {
    static constexpr int E = 2;  // complex entries per 16-byte load
    __device__ static inline void load(const float2* p, bool nt, f4v& v) {
        v = nt ? __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p)) : *reinterpret_cast<const f4v*>(p);
    }
    __device__ static inline cd get(const f4v& v, int i) { return i == 0 ? cd{v.x, v.y} : cd{v.z, v.w}; }
    using raw = f4v;
};
template <>
struct Gv<double2> {
    static constexpr int E = 1;
    __device__ static inline void load(const double2* p, bool nt, d2v& v) {
        v = nt ? __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p)) : *reinterpret_cast<const d2v*>(p);
    }
    __device__ static inline cd get(const d2v& v, int) { return cd{v.x, v.y}; }
    using raw = d2v;
};

constexpr int kGemvUnroll = 8;

// lane l of a block owns rows base + l*E + e, e < E (one 16-byte load per column)
template <class M2, int NRHS, bool FULL>
__device__ __forceinline__ void gemv_stream(const M2* __restrict__ kp, const double2* qs, int Nc, int ncol, int row,
                                            int valid, int wave, cd (&acc)[Gv<M2>::E][NRHS]) {
    using G = Gv<M2>;
    using raw = typename G::raw;
    constexpr int E = G::E;
    auto load_col = [&](int c, raw& v) {
        const M2* colp = kp + (int64_t)c * Nc + row;
        if (FULL) {
            G::load(colp, true, v);
        } else if constexpr (E == 2) {
            // ragged tail or rows not 16-byte aligned: element loads, zeros past the end
            const cd a = valid > 0 ? ld(colp) : cmake(0.0, 0.0);
            const cd b = valid > 1 ? ld(colp + 1) : cmake(0.0, 0.0);
            v = raw{(float)a.re, (float)a.im, (float)b.re, (float)b.im};
        } else {
            const cd a = valid > 0 ? ld(colp) : cmake(0.0, 0.0);
            v = raw{a.re, a.im};
        }
    };
    auto fma_col = [&](const raw& v, int c) {
#pragma unroll
        for (int r = 0; r < NRHS; ++r) {
            const double2 q = qs[c * NRHS + r];
            const cd qc = cmake(q.x, q.y);
#pragma unroll
            for (int e = 0; e < E; ++e) cfma_cj(acc[e][r], G::get(v, e), qc);
        }
    };
    int c = wave;
    for (; c + 4 * (kGemvUnroll - 1) < ncol; c += 4 * kGemvUnroll) {
        raw v[kGemvUnroll];
#pragma unroll
        for (int u = 0; u < kGemvUnroll; ++u) load_col(c + 4 * u, v[u]);
#pragma unroll
        for (int u = 0; u < kGemvUnroll; ++u) {
            // keep each column's LDS reads and widening next to its FMAs
            __builtin_amdgcn_sched_barrier(0);
            fma_col(v[u], c + 4 * u);
        }
    }
    for (; c < ncol; c += 4) {
        raw v;
        load_col(c, v);
        fma_col(v, c);
    }
}

template <class M2, int NRHS, bool VEC>
__global__ __launch_bounds__(256, 4) void k_gemv2(const M2* __restrict__ K, const double2* __restrict__ qbar,
                                                  double2* __restrict__ part, int Nc, int col_chunk, int n_rowblk) {
    constexpr int E = Gv<M2>::E;
    constexpr int RW = kWave * E;
    extern __shared__ double2 smem[];
    const int rb = blockIdx.x % n_rowblk;
    const int s = blockIdx.x / n_rowblk;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int c_begin = s * col_chunk;
    const int c_end = min(Nc, c_begin + col_chunk);
    const int ncol = c_end - c_begin;

    for (int i = threadIdx.x; i < ncol * NRHS; i += blockDim.x) smem[i] = qbar[(int64_t)c_begin * NRHS + i];
    __syncthreads();

    const int row = rb * RW + lane * E;
    const int valid = max(0, min(E, Nc - row));
    cd acc[E][NRHS];
#pragma unroll
    for (int e = 0; e < E; ++e)
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc[e][r] = cmake(0.0, 0.0);
    const M2* kp = K + (int64_t)c_begin * Nc;
    if (VEC && (rb + 1) * RW <= Nc)
        gemv_stream<M2, NRHS, true>(kp, smem, Nc, ncol, row, valid, wave, acc);
    else if (valid > 0)
        gemv_stream<M2, NRHS, false>(kp, smem, Nc, ncol, row, valid, wave, acc);

    // cross-wave sum in fixed order (waves 1..3 into LDS, wave 0 adds)
    __syncthreads();
    constexpr int PER = E * NRHS;
    double2* red = smem;  // 3 * 64 * PER entries
    if (wave > 0) {
        int o = ((wave - 1) * kWave + lane) * PER;
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
            for (int r = 0; r < NRHS; ++r) red[o++] = make_double2(acc[e][r].re, acc[e][r].im);
    }
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < 4; ++w) {
            int o = ((w - 1) * kWave + lane) * PER;
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int r = 0; r < NRHS; ++r) {
                    const double2 v = red[o++];
                    acc[e][r].re += v.x;
                    acc[e][r].im += v.y;
                }
        }
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e < valid)
#pragma unroll
                for (int r = 0; r < NRHS; ++r)
                    part[((int64_t)s * Nc + row + e) * NRHS + r] = make_double2(acc[e][r].re, acc[e][r].im);
    }

}

// r[o] = sum over the splits of part[split][o], o = row * NRHS + rhs, fixed order
__global__ __launch_bounds__(256) void k_gemv_reduce(const double2* __restrict__ part, double2* __restrict__ rout,
                                                     int64_t n_out, int n_split) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_out) return;
    double re = 0.0, im = 0.0;
    // batches of 8 splits, loads unconditional (clamped) so a batch is in flight at once
    for (int t0 = 0; t0 < n_split; t0 += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)min(t0 + u, n_split - 1) * n_out + o];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (t0 + u < n_split) {
                re += v[u].x;
                im += v[u].y;
            }
    }
    rout[o] = make_double2(re, im);
}

static void gemv_shape(const Plan& p, int rw, int* n_rowblk, int* n_split, int* col_chunk) {
    const int Nc = (int)p.g.Nc;
    *n_rowblk = (Nc + rw - 1) / rw;
    int ns = p.n_split;
    if (ns <= 0) ns = (2048 + *n_rowblk - 1) / *n_rowblk;
    ns = std::max(1, std::min(ns, kMaxSplit));
    ns = std::min(ns, std::max(1, Nc / 32));
    int chunk = (Nc + ns - 1) / ns;
    chunk = (chunk + 31) / 32 * 32;
    *col_chunk = chunk;
    *n_split = (Nc + chunk - 1) / chunk;
}

template <class M2, int NRHS>
static hipError_t gemv_t(Plan& p, hipStream_t s) {
    const Geometry& g = p.g;
    constexpr int RW = kWave * Gv<M2>::E;
    int n_rowblk, n_split, chunk;
    gemv_shape(p, RW, &n_rowblk, &n_split, &chunk);
    const size_t lds = std::max((size_t)chunk * NRHS, (size_t)3 * kWave * Gv<M2>::E * NRHS) * sizeof(double2);
    const bool vec = (g.Nc * (int64_t)sizeof(M2)) % 16 == 0;
    const M2* K = reinterpret_cast<const M2*>(p.Kc);
    const double2* qbar = reinterpret_cast<const double2*>(p.ws + p.L.qbar);
    double2* part = reinterpret_cast<double2*>(p.ws + p.L.gpart);
    double2* rvec = reinterpret_cast<double2*>(p.ws + p.L.rvec);
    dim3 grid(n_rowblk * n_split), block(kBlock);
    if (vec)
        hipLaunchKernelGGL((k_gemv2<M2, NRHS, true>), grid, block, lds, s, K, qbar, part, (int)g.Nc, chunk, n_rowblk);
    else
        hipLaunchKernelGGL((k_gemv2<M2, NRHS, false>), grid, block, lds, s, K, qbar, part, (int)g.Nc, chunk, n_rowblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n_out = g.Nc * NRHS;
    hipLaunchKernelGGL(k_gemv_reduce, dim3((unsigned)((n_out + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, part, rvec,
                       n_out, n_split);
    return hipGetLastError();
}

template <class M2>
static hipError_t gemv_r(Plan& p, int n_rhs, hipStream_t s) {
    switch (n_rhs) {
        case 1: return gemv_t<M2, 1>(p, s);
        case 2: return gemv_t<M2, 2>(p, s);
        case 3: return gemv_t<M2, 3>(p, s);
        default: return gemv_t<M2, 4>(p, s);
    }
}

hipError_t launch_gemv(Plan& p, int n_rhs, hipStream_t s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (p.timing && p.ev && p.ev_used + 2 <= p.ev_cap) {
        e0 = p.ev[p.ev_used];
        e1 = p.ev[p.ev_used + 1];
        p.ev_used += 2;
        (void)hipEventRecord(e0, s);
    }
    hipError_t err = (p.g.dtype == BSE_F64) ? gemv_r<double2>(p, n_rhs, s) : gemv_r<float2>(p, n_rhs, s);
    if (e1) (void)hipEventRecord(e1, s);
    return err;
}

}  // namespace bse
