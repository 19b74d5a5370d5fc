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

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

// Launch of a coarse product's streaming kernel (the kernel before the one that adds the
// partials).  In kernel timing mode 3 the launch itself carries the event pair: the runtime
// stamps the two events with that kernel's own start and end, so the timed span holds the
// kernel alone, without the gap that an event recorded between two launches puts in front.
template <typename F, typename... Args>
static inline void launch_stream(const Plan& p, F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                                 Args... args) {
    if (p.split_ev)
        hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, s, p.split_start, p.split_ev, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

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
constexpr int kGemvLdsCols = 2048;  // qbar entries (double2) staged in LDS at a time: 32 KiB

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

// MULTI: the split's columns do not fit in LDS at once and are staged in pieces
template <class M2, int NRHS, bool FULL, bool MULTI>
__device__ __forceinline__ void gemv_pieces(const M2* __restrict__ K, const double2* __restrict__ qbar, double2* smem,
                                            int Nc, int c_begin, int c_end, int row, int valid, int wave,
                                            cd (&acc)[Gv<M2>::E][NRHS]) {
    if (!MULTI) {
        const int ncol = c_end - c_begin;
        for (int i = threadIdx.x; i < ncol * NRHS; i += blockDim.x) smem[i] = qbar[(int64_t)c_begin * NRHS + i];
        __syncthreads();
        if (FULL || valid > 0)
            gemv_stream<M2, NRHS, FULL>(K + (int64_t)c_begin * Nc, smem, Nc, ncol, row, valid, wave, acc);
        __syncthreads();
        return;
    }
    for (int c0 = c_begin; c0 < c_end; c0 += kGemvLdsCols / NRHS) {
        const int ncol = min(c_end - c0, kGemvLdsCols / NRHS);
        for (int i = threadIdx.x; i < ncol * NRHS; i += blockDim.x) smem[i] = qbar[(int64_t)c0 * NRHS + i];
        __syncthreads();
        if (FULL || valid > 0) gemv_stream<M2, NRHS, FULL>(K + (int64_t)c0 * Nc, smem, Nc, ncol, row, valid, wave, acc);
        __syncthreads();
    }
}

template <class M2, int NRHS, bool VEC, bool MULTI>
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

    const int row = rb * RW + lane * E;
    const int valid = max(0, min(E, Nc - row));
    cd acc[E][NRHS];
#pragma unroll
    for (int e = 0; e < E; ++e)
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc[e][r] = cmake(0.0, 0.0);
    // the split's columns in LDS-sized pieces of qbar
    if (VEC && (rb + 1) * RW <= Nc)
        gemv_pieces<M2, NRHS, true, MULTI>(K, qbar, smem, Nc, c_begin, c_end, row, valid, wave, acc);
    else
        gemv_pieces<M2, NRHS, false, MULTI>(K, qbar, smem, Nc, c_begin, c_end, row, valid, wave, acc);

    // cross-wave sum in fixed order (waves 1..3 into LDS, wave 0 adds)
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

// Automatic column splits: at least 2048 blocks, except that a product whose columns
// can all be staged at once (single-stage blocks) takes the splits that make one round
// of resident blocks (4 per compute unit) if that round is at least 85% full: every
// block starts at once and no small last round is left as a tail (measured: C1 FP32
// 0.214 -> 0.209 ms per step; blocks that stage their columns in pieces did better
// with more of them).
static int auto_splits(int n_rowblk, int single_stage_cols, int Nc) {
    const int resident = 4 * cu_count();
    const int ns1 = resident / n_rowblk;
    if (ns1 >= 1 && (double)ns1 * n_rowblk >= 0.85 * resident && (Nc + ns1 - 1) / ns1 <= single_stage_cols)
        return ns1;
    return (2048 + n_rowblk - 1) / n_rowblk;
}

static void gemv_shape(const Plan& p, int rw, int nrhs, int* n_rowblk, int* n_split, int* col_chunk) {
    const int Nc = (int)p.g.Nc;
    *n_rowblk = (Nc + rw - 1) / rw;
    int ns = p.n_split;
    if (ns <= 0) ns = auto_splits(*n_rowblk, kGemvLdsCols / nrhs - 4, Nc);
    ns = std::max(1, std::min(ns, kMaxSplit));
    ns = std::min(ns, std::max(1, Nc / 32));
    int chunk = (Nc + ns - 1) / ns;
    chunk = (chunk + 3) / 4 * 4;   // whole columns per wavefront of a block
    *col_chunk = chunk;
    *n_split = (Nc + chunk - 1) / chunk;
}

template <class M2, int NRHS>
static hipError_t gemv_t(Plan& p, hipStream_t s) {
    const Geometry& g = p.g;
    constexpr int RW = kWave * Gv<M2>::E;
    int n_rowblk, n_split, chunk;
    gemv_shape(p, RW, NRHS, &n_rowblk, &n_split, &chunk);
    const size_t lds =
        std::max((size_t)std::min(chunk, kGemvLdsCols / NRHS) * NRHS, (size_t)3 * kWave * Gv<M2>::E * NRHS) *
        sizeof(double2);
    const bool vec = (g.Nc * (int64_t)sizeof(M2)) % 16 == 0;
    const M2* K = reinterpret_cast<const M2*>(p.Kc);
    const double2* qbar = reinterpret_cast<const double2*>(p.ws + p.L.qbar);
    double2* part = reinterpret_cast<double2*>(p.ws + p.L.gpart);
    double2* rvec = reinterpret_cast<double2*>(p.ws + p.L.rvec);
    dim3 grid(n_rowblk * n_split), block(kBlock);
    const bool multi = chunk > kGemvLdsCols / NRHS;
    if (vec && !multi)
        launch_stream(p, (k_gemv2<M2, NRHS, true, false>), grid, block, lds, s, K, qbar, part, (int)g.Nc, chunk,
                           n_rowblk);
    else if (vec)
        launch_stream(p, (k_gemv2<M2, NRHS, true, true>), grid, block, lds, s, K, qbar, part, (int)g.Nc, chunk,
                           n_rowblk);
    else if (!multi)
        launch_stream(p, (k_gemv2<M2, NRHS, false, false>), grid, block, lds, s, K, qbar, part, (int)g.Nc, chunk,
                           n_rowblk);
    else
        launch_stream(p, (k_gemv2<M2, NRHS, false, true>), grid, block, lds, s, K, qbar, part, (int)g.Nc, chunk,
                           n_rowblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n_out = g.Nc * NRHS;
    hipLaunchKernelGGL(k_gemv_reduce, dim3((unsigned)((n_out + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, part, rvec,
                       n_out, n_split);
    return hipGetLastError();
}

// ---- low-precision forms: block-scaled BF16 / FP16 coarse kernel on the matrix cores ----
//
// r = K_c qbar in real arithmetic: with K = Kr + i Ki and the coarse vectors split as
// q = q_hi + q_lo (each part in the storage format),
//   D = Kr [qr_hi qi_hi qr_lo qi_lo] + Ki [-qi_hi qr_hi -qi_lo qr_lo]
// gives Re r = D[:, rhs] + D[:, 8 + rhs] and Im r = D[:, 4 + rhs] + D[:, 12 + rhs]
// (16 columns: 4 right-hand sides x {re, im} x {hi, lo}).  One wavefront owns 16 rows
// of a 64-row block row; per 64 x 64 block it issues four 16x16x32 matrix-core
// products (two 32-column steps x {Kr, Ki}) into a fresh FP32 tile, then adds
// scale x tile into FP64 accumulators.
//
// Operand layouts (16x16x32, 8 entries per lane): A[m][k] in lane 16 (k / 8) + m,
// entry k % 8; B[k][n] in lane 16 (k / 8) + n, entry k % 8; D[m][n] in lane
// 16 (m / 4) + n, entry m % 4.  The plan stores every block as 16 A fragments of
// 1 KiB (fragment (rg, ks, part) = rows 16 rg.., columns 32 ks.., real or imaginary
// part) and the collapse writes qbar as B fragments, two variants per 32-column step.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int FMT>
struct Lowp;
template <>
struct Lowp<BSE_BF16_KC> {
    static constexpr bool grouped = false;   // qbar unscaled (BF16 has FP32's range)
    __device__ static inline unsigned short enc(float v) { return enc_lowp(BSE_BF16_KC, v); }
    __device__ static inline f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                       0, 0, 0);
    }
};
template <>
struct Lowp<BSE_F16_KC> {
    static constexpr bool grouped = true;    // qbar x a power of two per 64-column group and rhs
    __device__ static inline unsigned short enc(float v) { return enc_lowp(BSE_F16_KC, v); }
    __device__ static inline f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    }
};

// block (bi, bj) of the padded coarse kernel: scale = smallest power of two >= the
// largest |Re| or |Im| entry (1 for a zero block), entries K / scale in the format
template <int FMT>
__global__ __launch_bounds__(256) void k_quantize(const float2* __restrict__ K, unsigned short* __restrict__ kq,
                                                  float* __restrict__ kscale, int64_t Nc, int nb) {
    __shared__ float smax[kBlock / kWave];
    const int bi = blockIdx.x / nb, bj = blockIdx.x % nb;
    const int t = threadIdx.x;
    constexpr int PER = kKqBlock * kKqBlock / kBlock;  // 16 entries per thread
    float2 v[PER];
    float mx = 0.0f;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = t + u * kBlock;
        const int64_t row = (int64_t)bi * kKqBlock + e / kKqBlock, col = (int64_t)bj * kKqBlock + e % kKqBlock;
        v[u] = (row < Nc && col < Nc) ? K[row * Nc + col] : make_float2(0.0f, 0.0f);
        mx = fmaxf(mx, fmaxf(fabsf(v[u].x), fabsf(v[u].y)));
    }
    for (int off = kWave / 2; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
    if (t % kWave == 0) smax[t / kWave] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
    int ex = 0;
    if (mx > 0.0f) {
        (void)frexpf(mx, &ex);          // mx = f 2^ex, f in [1/2, 1)
        if (ldexpf(1.0f, ex - 1) >= mx) ex -= 1;  // exact powers of two map to themselves
    }
    const float sc = mx > 0.0f ? ldexpf(1.0f, ex) : 1.0f;
    const float inv = 1.0f / sc;       // a power of two: exact
    unsigned short* tile = kq + ((int64_t)bi * nb + bj) * (kKqBlock * kKqBlock * 2);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = t + u * kBlock;
        const int row = e / kKqBlock, col = e % kKqBlock;
        const int rg = row / 16, m = row % 16, ks = col / 32, kk = col % 32;
        const int lane = (kk / 8) * 16 + m, ent = kk % 8;
        const int fr_re = (rg * 2 + ks) * 2, fr_im = fr_re + 1;
        tile[(fr_re * kWave + lane) * 8 + ent] = Lowp<FMT>::enc(v[u].x * inv);
        tile[(fr_im * kWave + lane) * 8 + ent] = Lowp<FMT>::enc(v[u].y * inv);
    }
    if (t == 0) kscale[(int64_t)bi * nb + bj] = sc;
}

__global__ void k_zero_u32(unsigned int* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_hm_table(int* __restrict__ runs, int* __restrict__ row0, int nb, int len);

hipError_t launch_quantize(const Plan& p, hipStream_t s) {
    const Geometry& g = p.g;
    if (!kc_lowp(g.dtype)) return hipSuccess;
    const KqShape k = kq_shape(g.Nc);
    unsigned short* kq = reinterpret_cast<unsigned short*>(p.ws + p.L.kq);
    float* ksc = reinterpret_cast<float*>(p.ws + p.L.kscale);
    const float2* K = reinterpret_cast<const float2*>(p.Kc);
    if (g.dtype == BSE_BF16_KC)
        hipLaunchKernelGGL(k_quantize<BSE_BF16_KC>, dim3((unsigned)(k.nb * k.nb)), dim3(kBlock), 0, s, K, kq, ksc, g.Nc,
                           k.nb);
    else
        hipLaunchKernelGGL(k_quantize<BSE_F16_KC>, dim3((unsigned)(k.nb * k.nb)), dim3(kBlock), 0, s, K, kq, ksc, g.Nc,
                           k.nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nw = (int64_t)(p.L.qfrag_bytes / 4);
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((nw + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       reinterpret_cast<unsigned int*>(p.ws + p.L.qfrag), nw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const HmShape h = hm_shape(g.Nc);
    int* runs = reinterpret_cast<int*>(p.ws + p.L.mtab);
    hipLaunchKernelGGL(k_hm_table, dim3(1), dim3(kWave), 0, s, runs, runs + h.runs, h.nb, h.run_len);
    return hipGetLastError();
}

constexpr int kMfmaUnroll = 2;  // 64-column blocks whose operands are in flight together

template <int FMT>
__global__ __launch_bounds__(256) void k_gemv_mfma(const u32x4* __restrict__ kq, const float* __restrict__ kscale,
                                                   const u32x4* __restrict__ qf, const float* __restrict__ qsinv,
                                                   double* __restrict__ part, int Nc, int nb, int cpb, int n_rhs) {
    const int bi = blockIdx.x % nb;
    const int sp = blockIdx.x / nb;
    const int rg = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int bj0 = sp * cpb, bj1 = min(nb, bj0 + cpb);
    // this wavefront's 4 A fragments of block (bi, bj): (ks, part) = (0, re), (0, im), (1, re), (1, im)
    const u32x4* arow = kq + (int64_t)bi * nb * 16 * kWave + (rg * 4) * kWave + lane;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // this lane's output column n = lane % 16 belongs to right-hand side n % 4; the FP16
    // form divides out the scale the collapse gave that rhs in column group bj
    const int rq = (lane % 16) & 3;
    auto qinv = [&](int bj) -> float { return Lowp<FMT>::grouped ? qsinv[(int64_t)bj * kMaxRhs + rq] : 1.0f; };
    int bj = bj0;
    for (; bj + kMfmaUnroll <= bj1; bj += kMfmaUnroll) {
        u32x4 a[kMfmaUnroll][4], b[kMfmaUnroll][4];
        float sc[kMfmaUnroll], qi[kMfmaUnroll];
#pragma unroll
        for (int u = 0; u < kMfmaUnroll; ++u) {
            const u32x4* ab = arow + (int64_t)(bj + u) * 16 * kWave;
#pragma unroll
            for (int f = 0; f < 4; ++f) a[u][f] = __builtin_nontemporal_load(ab + f * kWave);
            // B fragments of the block's two 32-column steps: (step, variant)
#pragma unroll
            for (int f = 0; f < 4; ++f) b[u][f] = qf[((int64_t)(2 * (bj + u) + (f >> 1)) * 2 + (f & 1)) * kWave + lane];
            sc[u] = kscale[(int64_t)bi * nb + bj + u];
            qi[u] = qinv(bj + u);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kMfmaUnroll; ++u) {
            f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
            d = Lowp<FMT>::mfma(a[u][0], b[u][0], d);  // Kr x B1, first 32 columns
            d = Lowp<FMT>::mfma(a[u][1], b[u][1], d);  // Ki x B2
            d = Lowp<FMT>::mfma(a[u][2], b[u][2], d);  // second 32 columns
            d = Lowp<FMT>::mfma(a[u][3], b[u][3], d);
            const double w = (double)sc[u] * (double)qi[u];   // powers of two: exact
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = fma(w, (double)d[e], acc[e]);
        }
    }
    for (; bj < bj1; ++bj) {
        const u32x4* ab = arow + (int64_t)bj * 16 * kWave;
        f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int f = 0; f < 4; ++f)
            d = Lowp<FMT>::mfma(ab[f * kWave], qf[((int64_t)(2 * bj + (f >> 1)) * 2 + (f & 1)) * kWave + lane], d);
        const double w = (double)kscale[(int64_t)bi * nb + bj] * (double)qinv(bj);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = fma(w, (double)d[e], acc[e]);
    }
    // column n = lane % 16 holds (hi, lo) parts in n and n + 8: add them; rows 4 (lane / 16) + e
    const int n = lane % 16;
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e] += __shfl_xor(acc[e], 8, kWave);
    if (n < 8) {
        const int r = n & 3, comp = n >> 2;  // n = r: real part, n = 4 + r: imaginary part
        if (r < n_rhs) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = bi * kKqBlock + rg * 16 + 4 * (lane / 16) + e;
                if (row < Nc) part[(((int64_t)sp * Nc + row) * n_rhs + r) * 2 + comp] = acc[e];
            }
        }
    }
}

// ---- packed Hermitian product on the matrix cores (block-scaled BF16/FP16 K_c) ---------
//
// K_c is Hermitian, so the blocks (bi, bj) with bi <= bj of the block-scaled layout hold
// all of it; the others are never read.  A wavefront takes a band of two block rows
// (bi0 = 2 bp, bi1 = bi0 + 1) and a run of block columns bj, and for each stored block
//   P1: r_bi += K_(bi,bj) q_bj     (the stored A fragments, as k_gemv_mfma, all 64 rows),
//   P2: r_bj += K_(bi,bj)^H q_bi   (off-diagonal blocks; the diagonal block is P1's whole).
// P2 contracts over the block's rows, so it needs the block as the B operand with k = row:
// the wavefront writes its 16 fragments into its own LDS planes (re, im) transposed,
// T[col][row], and reads B fragments back as contiguous 16-byte runs.  The fragments of
// q_bi, which the collapse writes as B operands, serve unchanged as the A operands of P2
// (the A fragment of a 16 x 32 matrix holds the same lane data as the B fragment of its
// transpose).  Conjugation: with the variants [qr, qi] (V1) and [-qi, qr] (V2) of q,
//   Re r2 = sum Kr qr + Ki qi = (V1 Kr - V2 Ki) on the qr rows,  Im r2 = the same on the qi rows.
// A block's FP32 product times its scale (a power of two, as is the FP16 q scale) is exact
// in FP32.  P1 is summed over the run in FP64 and written once per run and row; the P2 of
// the band's two blocks in a column are added in FP32 and written once per (band, column);
// k_hm_reduce adds both kinds in a fixed order.

constexpr int kHmPitch = 72;     // bf16 per row of a transposed LDS plane (16-byte rows, spread banks)
constexpr int kHmWaves = 2048;   // wavefronts the runs aim at: one round at 2 waves per SIMD
constexpr int kHmBlock = 128;    // 2 independent wavefronts per workgroup: 36 KiB of LDS planes

// column partials: one per (band bp, column block bj) with 2 bp < bj, stored by column block
// (those of column bj are contiguous; column bj has ceil(bj / 2) of them)
__host__ __device__ inline int64_t hm_p2_index(int bp, int bj) {
    const int64_t m = bj / 2;
    return m * (m + (bj & 1)) + bp;
}
__host__ __device__ inline int hm_runs_in_band(int nb, int bp, int len) { return (nb - 2 * bp + len - 1) / len; }

HmShape hm_shape(int64_t Nc) {
    HmShape h;
    h.nb = kq_shape(Nc).nb;
    h.bands = (h.nb + 1) / 2;
    h.p2 = hm_p2_index(0, h.nb);
    auto runs = [&](int len) {
        int64_t r = 0;
        for (int bp = 0; bp < h.bands; ++bp) r += hm_runs_in_band(h.nb, bp, len);
        return r;
    };
    h.run_len = 1;
    while (runs(h.run_len) > kHmWaves && h.run_len < h.nb) ++h.run_len;
    h.runs = runs(h.run_len);
    return h;
}

// run -> bp | bj0 << 16, runs band by band; band0[bp] = first run of band bp
__global__ void k_hm_table(int* __restrict__ runs, int* __restrict__ band0, int nb, int len) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int r = 0;
    const int bands = (nb + 1) / 2;
    for (int bp = 0; bp < bands; ++bp) {
        band0[bp] = r;
        for (int bj = 2 * bp; bj < nb; bj += len) runs[r++] = bp | (bj << 16);
    }
    band0[bands] = r;
}

template <int FMT>
__global__ __launch_bounds__(kHmBlock, 2) void k_hemv_mfma(const u32x4* __restrict__ kq, const float* __restrict__ kscale,
                                                      const u32x4* __restrict__ qf, const float* __restrict__ qsinv,
                                                      const int* __restrict__ runs, int nruns, int run_len,
                                                      double* __restrict__ p1part, float* __restrict__ p2part,
                                                      int nb, int n_rhs) {
    extern __shared__ unsigned short hm_lds[];   // per wavefront: planes re, im of [64][kHmPitch]
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int run = blockIdx.x * (kHmBlock / kWave) + wave;
    if (run >= nruns) return;   // wavefront-uniform; the kernel has no block barrier
    const int code = runs[run];
    const int bp = code & 0xffff, bj0 = code >> 16;
    const int bi0 = 2 * bp;
    const int nrow = (bi0 + 1 < nb) ? 2 : 1;
    const int bj1 = min(nb, bj0 + run_len);
    unsigned short* pre = hm_lds + (size_t)wave * 2 * 64 * kHmPitch;
    unsigned short* pim = pre + 64 * kHmPitch;
    const int n = lane % 16, g = lane / 16;
    // q of the band's rows as the A operands of P2: (row, step, variant), and their FP16 scales
    // (P2's output rows m = 4 g + e hold right-hand side e; P1's column n holds rhs n % 4)
    u32x4 a2[2][2][2];
    float qs2[2][4];
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const int bi = min(bi0 + rr, nb - 1);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int v = 0; v < 2; ++v) a2[rr][ks][v] = qf[((int64_t)(2 * bi + ks) * 2 + v) * kWave + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) qs2[rr][e] = Lowp<FMT>::grouped ? qsinv[(int64_t)bi * kMaxRhs + e] : 1.0f;
    }
    double acc[2][4][4];
#pragma unroll
    for (int rr = 0; rr < 2; ++rr)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[rr][rg][e] = 0.0;
#pragma unroll 1
    for (int bj = bj0; bj < bj1; ++bj) {
        u32x4 b[2][2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int v = 0; v < 2; ++v) b[ks][v] = qf[((int64_t)(2 * bj + ks) * 2 + v) * kWave + lane];
        const float q1 = Lowp<FMT>::grouped ? qsinv[(int64_t)bj * kMaxRhs + (n & 3)] : 1.0f;
        float p2v[4][4];
#pragma unroll
        for (int cg = 0; cg < 4; ++cg)
#pragma unroll
            for (int e = 0; e < 4; ++e) p2v[cg][e] = 0.0f;
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int bi = bi0 + rr;
            if (rr >= nrow || bj < bi) continue;   // wavefront-uniform: no such row, or a block below the diagonal
            const u32x4* ab = kq + ((int64_t)bi * nb + bj) * 16 * kWave + lane;
            u32x4 a[16];
#pragma unroll
            for (int f = 0; f < 16; ++f) a[f] = __builtin_nontemporal_load(ab + f * kWave);
            const float sc = kscale[(int64_t)bi * nb + bj];
            __builtin_amdgcn_sched_barrier(0);
            // P1: row group rg, fragments (rg, step, part) = a[(rg * 2 + ks) * 2 + part]
            const double w1 = (double)sc * (double)q1;   // powers of two: exact
#pragma unroll
            for (int rg = 0; rg < 4; ++rg) {
                f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    d = Lowp<FMT>::mfma(a[(rg * 2 + ks) * 2 + 0], b[ks][0], d);
                    d = Lowp<FMT>::mfma(a[(rg * 2 + ks) * 2 + 1], b[ks][1], d);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[rr][rg][e] = fma(w1, (double)d[e], acc[rr][rg][e]);
            }
            if (bj == bi) continue;   // wavefront-uniform: the diagonal block
            // the block into LDS, transposed: fragment (rg, ks, part), entry e holds
            // K_part[row 16 rg + n][col 32 ks + 8 g + e] -> plane[col][row]
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // the previous block's reads are done
#pragma unroll
            for (int rg = 0; rg < 4; ++rg)
#pragma unroll
                for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                    for (int part = 0; part < 2; ++part) {
                        const u32x4 v = a[(rg * 2 + ks) * 2 + part];
                        unsigned short* pl = (part ? pim : pre) + (32 * ks + 8 * g) * kHmPitch + 16 * rg + n;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const unsigned int wv = v[e / 2];
                            pl[e * kHmPitch] = (unsigned short)((e & 1) ? (wv >> 16) : (wv & 0xffffu));
                        }
                    }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // writes before the reads of other lanes
            // P2 per column group cg: B[k = row][n = col] = plane[16 cg + n][32 ks + 8 g .. + 7]
#pragma unroll
            for (int cg = 0; cg < 4; ++cg) {
                f32x4 da = {0.0f, 0.0f, 0.0f, 0.0f}, db = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int o = (16 * cg + n) * kHmPitch + 32 * ks + 8 * g;
                    const u32x4 kre = *reinterpret_cast<const u32x4*>(pre + o);
                    const u32x4 kim = *reinterpret_cast<const u32x4*>(pim + o);
                    da = Lowp<FMT>::mfma(a2[rr][ks][0], kre, da);
                    db = Lowp<FMT>::mfma(a2[rr][ks][1], kim, db);
                }
                // D2[m = 4 g + e][col]: g = 0 qr_hi, 1 qi_hi, 2 qr_lo, 3 qi_lo rows of rhs e;
                // the lo rows (lanes g + 2) are added to the hi rows
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = (da[e] - db[e]) * (sc * qs2[rr][e]);
                    v += __shfl_xor(v, 32, kWave);
                    p2v[cg][e] += v;
                }
            }
        }
        if (bj > bi0 && g < 2) {   // the band's column partial of bj
            float* out = p2part + hm_p2_index(bp, bj) * kKqBlock * n_rhs * 2;
#pragma unroll
            for (int cg = 0; cg < 4; ++cg)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e < n_rhs) out[((int64_t)(16 * cg + n) * n_rhs + e) * 2 + g] = p2v[cg][e];
        }
    }
    // P1 partials of the run, one per row: column n holds (hi, lo) parts in n and n + 8; rows
    // 4 (lane / 16) + e of row group rg
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        double* out1 = p1part + ((int64_t)run * 2 + rr) * kKqBlock * n_rhs * 2;
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double v = acc[rr][rg][e] + __shfl_xor(acc[rr][rg][e], 8, kWave);
                const int r = n & 3, comp = (n >> 2) & 1;
                if (n < 8 && r < n_rhs) out1[((int64_t)(16 * rg + 4 * g + e) * n_rhs + r) * 2 + comp] = v;
            }
    }
}

// r[i][rhs] = the P1 partials of the runs of band b / 2 for row b = i / 64 (in order), then
// the P2 partials of the bands bp with 2 bp < b; eight lanes per output and a fixed butterfly
template <int NRHS>
__global__ __launch_bounds__(256) void k_hm_reduce(const double2* __restrict__ p1, const float2* __restrict__ p2,
                                                   const int* __restrict__ band0, double2* __restrict__ rout, int Nc) {
    constexpr int LN = 8;
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LN;
    const int k = threadIdx.x % LN;
    const int64_t oc = min(o, (int64_t)Nc * NRHS - 1);   // lanes past the end: same work, no store
    const int i = (int)(oc / NRHS), r = (int)(oc % NRHS);
    const int b = i / kKqBlock, w = i % kKqBlock;
    const int bp = b / 2, rr = b & 1;
    const int r0 = band0[bp], n1 = band0[bp + 1] - r0;
    const int n = n1 + (b + 1) / 2;
    const double2* q1 = p1 + (((int64_t)r0 * 2 + rr) * kKqBlock + w) * NRHS + r;   // run t at t 2 64 NRHS
    const float2* q2 = p2 + (hm_p2_index(0, b) * kKqBlock + w) * NRHS + r;          // band t at t 64 NRHS
    double re = 0.0, im = 0.0;
    for (int t0 = k; t0 < n; t0 += 4 * LN) {
        double2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = min(t0 + u * LN, n - 1);
            if (t < n1) {
                v[u] = q1[(int64_t)t * 2 * kKqBlock * NRHS];
            } else {
                const float2 f = q2[(int64_t)(t - n1) * kKqBlock * NRHS];
                v[u] = make_double2(f.x, f.y);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t0 + u * LN < n) {
                re += v[u].x;
                im += v[u].y;
            }
    }
#pragma unroll
    for (int off = 1; off < LN; off <<= 1) {
        re += __shfl_xor(re, off, kWave);
        im += __shfl_xor(im, off, kWave);
    }
    if (k == 0 && o < (int64_t)Nc * NRHS) rout[o] = make_double2(re, im);
}

static hipError_t hemv_lowp(Plan& p, int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    const HmShape h = hm_shape(g.Nc);
    const u32x4* kq = reinterpret_cast<const u32x4*>(p.ws + p.L.kq);
    const float* ksc = reinterpret_cast<const float*>(p.ws + p.L.kscale);
    const u32x4* qf = reinterpret_cast<const u32x4*>(p.ws + p.L.qfrag);
    const float* qsi = reinterpret_cast<const float*>(p.ws + p.L.qsinv);
    const int* runs = reinterpret_cast<const int*>(p.ws + p.L.mtab);
    double* p1 = reinterpret_cast<double*>(p.ws + p.L.mp1);
    float* p2 = reinterpret_cast<float*>(p.ws + p.L.mp2);
    constexpr int wpb = kHmBlock / kWave;
    const dim3 grid((unsigned)((h.runs + wpb - 1) / wpb)), block(kHmBlock);
    const size_t lds = (size_t)wpb * 2 * 64 * kHmPitch * sizeof(unsigned short);
    if (g.dtype == BSE_BF16_KC)
        launch_stream(p, k_hemv_mfma<BSE_BF16_KC>, grid, block, lds, s, kq, ksc, qf, qsi, runs, (int)h.runs,
                           h.run_len, p1, p2, h.nb, n_rhs);
    else
        launch_stream(p, k_hemv_mfma<BSE_F16_KC>, grid, block, lds, s, kq, ksc, qf, qsi, runs, (int)h.runs,
                           h.run_len, p1, p2, h.nb, n_rhs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n_thr = g.Nc * n_rhs * 8;
    const dim3 rg((unsigned)((n_thr + kBlock - 1) / kBlock)), rblock(kBlock);
    const double2* q1 = reinterpret_cast<const double2*>(p1);
    const float2* q2 = reinterpret_cast<const float2*>(p2);
    double2* rvec = reinterpret_cast<double2*>(p.ws + p.L.rvec);
    const int* row0 = runs + h.runs;
    switch (n_rhs) {
        case 1: hipLaunchKernelGGL(k_hm_reduce<1>, rg, rblock, 0, s, q1, q2, row0, rvec, (int)g.Nc); break;
        case 2: hipLaunchKernelGGL(k_hm_reduce<2>, rg, rblock, 0, s, q1, q2, row0, rvec, (int)g.Nc); break;
        case 3: hipLaunchKernelGGL(k_hm_reduce<3>, rg, rblock, 0, s, q1, q2, row0, rvec, (int)g.Nc); break;
        default: hipLaunchKernelGGL(k_hm_reduce<4>, rg, rblock, 0, s, q1, q2, row0, rvec, (int)g.Nc); break;
    }
    return hipGetLastError();
}

static hipError_t gemv_lowp(Plan& p, int n_rhs, hipStream_t s) {
    if (use_packed_lowp(p)) return hemv_lowp(p, n_rhs, s);
    const Geometry& g = p.g;
    const KqShape k = kq_shape(g.Nc);
    int ns = p.n_split;
    if (ns <= 0) ns = (2048 + k.nb - 1) / k.nb;
    ns = std::max(1, std::min(std::min(ns, kMaxSplit), k.nb));
    const int cpb = (k.nb + ns - 1) / ns;
    ns = (k.nb + cpb - 1) / cpb;
    const u32x4* kq = reinterpret_cast<const u32x4*>(p.ws + p.L.kq);
    const float* ksc = reinterpret_cast<const float*>(p.ws + p.L.kscale);
    const u32x4* qf = reinterpret_cast<const u32x4*>(p.ws + p.L.qfrag);
    const float* qsi = reinterpret_cast<const float*>(p.ws + p.L.qsinv);
    double* part = reinterpret_cast<double*>(p.ws + p.L.gpart);
    double2* rvec = reinterpret_cast<double2*>(p.ws + p.L.rvec);
    dim3 grid((unsigned)(k.nb * ns)), block(kBlock);
    if (g.dtype == BSE_BF16_KC)
        launch_stream(p, k_gemv_mfma<BSE_BF16_KC>, grid, block, 0, s, kq, ksc, qf, qsi, part, (int)g.Nc, k.nb, cpb,
                           n_rhs);
    else
        launch_stream(p, k_gemv_mfma<BSE_F16_KC>, grid, block, 0, s, kq, ksc, qf, qsi, part, (int)g.Nc, k.nb, cpb,
                           n_rhs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n_out = g.Nc * n_rhs;
    hipLaunchKernelGGL(k_gemv_reduce, dim3((unsigned)((n_out + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       reinterpret_cast<const double2*>(part), rvec, n_out, ns);
    return hipGetLastError();
}

// ---- packed Hermitian product (FP32 coarse kernel; the FP64 form follows) --------------
//
// K_c is Hermitian (Eqs. bse1-bse2), so its 128 x 128 tiles (I, J) with I <= J hold all of
// it: half the bytes of the full stream.  One wavefront streams one 64-column half of a
// tile and does both products it serves,
//   P1: r_I += K_IJ q_J          (rows of the tile),
//   P2: r_J += K_IJ^H q_I        (columns; not on the diagonal tile, which P1 covers whole).
// Lane L owns tile rows L and 64 + L.  At step s of column half h it holds column
// 64 h + (L + s) mod 64 of both rows: one 16-byte load of two complex FP32 entries, and the
// tile is stored in that order, so every load instruction of the wavefront reads one
// contiguous 1 KiB run.  P1 accumulates per lane (its rows).  P2's partial of a column
// moves one lane per step with a DPP wavefront rotate, so each lane adds into the column it
// holds; after 64 steps every partial is back on the lane of its column.
// Arithmetic: products and sums in FP32 over runs of kHemvFlush steps (P1: kHemvFlush terms
// per row, P2: 2 kHemvFlush terms per column), then added into FP64 (P1 in registers, P2 in
// LDS).  A block is 4 wavefronts on the two halves of 2 tpw consecutive tiles of one tile
// row, each wavefront taking tpw of them in turn: their P1 sums are added in LDS
// in a fixed order and written as one partial of r_I; every off-diagonal tile writes its P2
// partial of r_J.  k_hemv_reduce adds, for each output, the
// partials of its tile row and of its tile column in a fixed order.

constexpr int kHemvTile = 128;
// Tiles each wavefront streams one after another (tpw): a block covers 2 tpw consecutive
// tiles of its tile row.  The plan takes the smallest tpw that keeps the grid within
// kHemvBlocks blocks, a single round on the device with room to spare: a second, partial
// round of blocks left the HBM stream short of loads in flight, and so did fewer, longer
// blocks (9216-row kernel, FP32: 77.3 us at tpw 1 with 1332 blocks, 74.2 us at tpw 3 with
// 468, 85.6 us at tpw 4 with 360).
constexpr int kHemvBlocks = 512;
constexpr int kHemvFlush = 16;   // steps per FP32 run before the FP64 sums
constexpr int kHemvUnroll = 8;   // 16-byte loads of a lane in flight

__host__ __device__ inline int64_t hemv_tile_index(int I, int J, int nbk) {
    return (int64_t)I * nbk - (int64_t)I * (I - 1) / 2 + (J - I);
}

// rotate a float across the wavefront: lane L receives lane L + 1 (mod 64)
__device__ __forceinline__ float wave_rol1(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x134, 0xF, 0xF, false));
}

// packed tiles from the row-major FP32 K_c: one block per (tile, half, 4 steps)
__global__ __launch_bounds__(256) void k_hemv_pack(const float2* __restrict__ K, f4v* __restrict__ kp, int64_t Nc,
                                                   int nbk) {
    const int64_t unit = blockIdx.x;   // (tile, half, step group of 4)
    const int64_t tile = unit / 32;
    const int hs = (int)(unit % 32);
    const int h = hs / 16, s = (hs % 16) * 4 + threadIdx.x / kWave;
    const int L = threadIdx.x % kWave;
    int I = 0;
    while (I + 1 < nbk && hemv_tile_index(I + 1, I + 1, nbk) <= tile) ++I;
    const int J = I + (int)(tile - hemv_tile_index(I, I, nbk));
    const int64_t col = (int64_t)J * kHemvTile + 64 * h + ((L + s) & 63);
    const int64_t r0 = (int64_t)I * kHemvTile + L, r1 = r0 + 64;
    const float2 a = (r0 < Nc && col < Nc) ? K[r0 * Nc + col] : make_float2(0.0f, 0.0f);
    const float2 b = (r1 < Nc && col < Nc) ? K[r1 * Nc + col] : make_float2(0.0f, 0.0f);
    kp[((tile * 2 + h) * 64 + s) * kWave + L] = f4v{a.x, a.y, b.x, b.y};
}

__host__ __device__ inline int hemv_groups(int nbk, int I, int tpw) { return (nbk - I + 2 * tpw - 1) / (2 * tpw); }

// block -> (tile row I, group g of 2 tpw tiles): table[b] = I | g << 16; band0[I] = first block of row I
__global__ void k_hemv_table(int* __restrict__ table, int* __restrict__ band0, int nbk, int tpw) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int b = 0;
    for (int I = 0; I < nbk; ++I) {
        band0[I] = b;
        const int ng = hemv_groups(nbk, I, tpw);
        for (int g = 0; g < ng; ++g) table[b++] = I | (g << 16);
    }
    band0[nbk] = b;
}

// one wavefront streams column half h of tile (I, J): P1 row sums into d1 (FP64), P2
// (OFFDIAG) into its FP64 column sums in LDS (p2, the half's 64 columns), then the half's
// P2 partial of r_J.  qj holds q_J of the half's 64 columns.
template <int NRHS, bool OFFDIAG>
__device__ __forceinline__ void hemv_half(const f4v* __restrict__ kp, const float2* qj, double2* p2,
                                          const float2 (&qi)[2][NRHS], double (&d1)[2][NRHS][2],
                                          float2* __restrict__ r2part, int I, int J, int h, int nbk, int L) {
    const f4v* tp = kp + (hemv_tile_index(I, J, nbk) * 2 + h) * (64 * kWave) + L;
    float a1[2][NRHS][2], a2[NRHS][2];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int r = 0; r < NRHS; ++r) a1[e][r][0] = a1[e][r][1] = 0.0f;
#pragma unroll
    for (int r = 0; r < NRHS; ++r) a2[r][0] = a2[r][1] = 0.0f;
#pragma unroll 1
    for (int sf = 0; sf < 64; sf += kHemvFlush) {
#pragma unroll
        for (int s0 = sf; s0 < sf + kHemvFlush; s0 += kHemvUnroll) {
            f4v kv[kHemvUnroll];
#pragma unroll
            for (int u = 0; u < kHemvUnroll; ++u) kv[u] = __builtin_nontemporal_load(tp + (int64_t)((s0 + u) * kWave));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < kHemvUnroll; ++u) {
                // keep each step's LDS reads next to its arithmetic
                __builtin_amdgcn_sched_barrier(0);
                const int c = (L + s0 + u) & 63;
                const float k0r = kv[u].x, k0i = kv[u].y, k1r = kv[u].z, k1i = kv[u].w;
#pragma unroll
                for (int r = 0; r < NRHS; ++r) {
                    const float2 q = qj[r * 64 + c];
                    // P1: row L and row 64 + L times q_J[c]
                    a1[0][r][0] = fmaf(k0r, q.x, a1[0][r][0]);
                    a1[0][r][0] = fmaf(-k0i, q.y, a1[0][r][0]);
                    a1[0][r][1] = fmaf(k0r, q.y, a1[0][r][1]);
                    a1[0][r][1] = fmaf(k0i, q.x, a1[0][r][1]);
                    a1[1][r][0] = fmaf(k1r, q.x, a1[1][r][0]);
                    a1[1][r][0] = fmaf(-k1i, q.y, a1[1][r][0]);
                    a1[1][r][1] = fmaf(k1r, q.y, a1[1][r][1]);
                    a1[1][r][1] = fmaf(k1i, q.x, a1[1][r][1]);
                }
                if (OFFDIAG) {
                    // P2: column c gets conj(K[L][c]) q_I[L] + conj(K[64 + L][c]) q_I[64 + L]
#pragma unroll
                    for (int r = 0; r < NRHS; ++r) {
                        float re = a2[r][0], im = a2[r][1];
                        re = fmaf(k0r, qi[0][r].x, re);
                        re = fmaf(k0i, qi[0][r].y, re);
                        re = fmaf(k1r, qi[1][r].x, re);
                        re = fmaf(k1i, qi[1][r].y, re);
                        im = fmaf(k0r, qi[0][r].y, im);
                        im = fmaf(-k0i, qi[0][r].x, im);
                        im = fmaf(k1r, qi[1][r].y, im);
                        im = fmaf(-k1i, qi[1][r].x, im);
                        // the partial moves on with its column: lane L now holds column
                        // (L + s + 1) mod 64 of the half
                        a2[r][0] = wave_rol1(re);
                        a2[r][1] = wave_rol1(im);
                    }
                }
            }
        }
        // end of a run: FP32 sums into FP64
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int r = 0; r < NRHS; ++r) {
                d1[e][r][0] += (double)a1[e][r][0];
                d1[e][r][1] += (double)a1[e][r][1];
                a1[e][r][0] = a1[e][r][1] = 0.0f;
            }
        if (OFFDIAG) {
            // the P2 sums of a column are read and written by different lanes at different
            // runs: keep this wavefront's LDS accesses in order
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const int cn = (L + sf + kHemvFlush) & 63;
#pragma unroll
            for (int r = 0; r < NRHS; ++r) {
                double2 v = p2[r * 64 + cn];
                v.x += (double)a2[r][0];
                v.y += (double)a2[r][1];
                p2[r * 64 + cn] = v;
                a2[r][0] = a2[r][1] = 0.0f;
            }
        }
    }
    // P2 partial of r_J for the half's 64 columns (the last run left column L on lane L)
    if (OFFDIAG) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        float2* out = r2part + hemv_tile_index(I, J, nbk) * kHemvTile * NRHS;
#pragma unroll
        for (int r = 0; r < NRHS; ++r) {
            const double2 v = p2[r * 64 + L];
            out[(64 * h + L) * NRHS + r] = make_float2((float)v.x, (float)v.y);
        }
    }
}

// Block = 4 wavefronts on 2 tpw consecutive tiles of tile row I: wavefront w takes column
// half w % 2 of the tiles J = I + 2 tpw g + w / 2 + 2 k, k < tpw, one after another.
template <int NRHS>
__global__ __launch_bounds__(256, 4) void k_hemv(const f4v* __restrict__ kp, const double2* __restrict__ qbar,
                                                 const int* __restrict__ table, float2* __restrict__ r1part,
                                                 float2* __restrict__ r2part, int Nc, int nbk, int tpw) {
    extern __shared__ double2 hsm[];
    const int wave = threadIdx.x / kWave;
    const int L = threadIdx.x % kWave;
    const int code = table[blockIdx.x];
    const int I = code & 0xffff, g = code >> 16;
    const int h = wave & 1;
    // LDS: q_J of each wavefront's 64 columns [4][NRHS][64] (float2), then the FP64 P2 sums
    // [4][NRHS][64]; at the end the P1 sums [4][128][NRHS] (double2) over all of them
    float2* qj = reinterpret_cast<float2*>(hsm) + wave * NRHS * 64;
    double2* p2 = hsm + 4 * NRHS * 64 / 2 + wave * NRHS * 64;
    // q_I of this lane's two rows (FP32)
    float2 qi[2][NRHS];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int row = I * kHemvTile + 64 * e + L;
#pragma unroll
        for (int r = 0; r < NRHS; ++r) {
            const double2 q = row < Nc ? qbar[(int64_t)row * NRHS + r] : make_double2(0.0, 0.0);
            qi[e][r] = make_float2((float)q.x, (float)q.y);
        }
    }
    double d1[2][NRHS][2];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int r = 0; r < NRHS; ++r) d1[e][r][0] = d1[e][r][1] = 0.0;
#pragma unroll 1
    for (int k = 0; k < tpw; ++k) {
        const int J = I + 2 * tpw * g + (wave >> 1) + 2 * k;
        const bool active = J < nbk;   // wavefront-uniform
        // q_J of the half's columns and cleared P2 sums in this wavefront's LDS (the
        // barriers order them after the previous tile's reads; the trip count is uniform)
        __syncthreads();
        if (active) {
            const int col = J * kHemvTile + 64 * h + L;
#pragma unroll
            for (int r = 0; r < NRHS; ++r) {
                const double2 q = col < Nc ? qbar[(int64_t)col * NRHS + r] : make_double2(0.0, 0.0);
                qj[r * 64 + L] = make_float2((float)q.x, (float)q.y);
                p2[r * 64 + L] = make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
        if (active) {
            if (J != I)
                hemv_half<NRHS, true>(kp, qj, p2, qi, d1, r2part, I, J, h, nbk, L);
            else
                hemv_half<NRHS, false>(kp, qj, p2, qi, d1, r2part, I, J, h, nbk, L);
        }
    }
    // P1 partial of r_I: the 4 wavefronts' row sums added in LDS in a fixed order
    __syncthreads();
    double2* red = hsm;   // [4][128][NRHS]
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int r = 0; r < NRHS; ++r)
            red[(wave * kHemvTile + 64 * e + L) * NRHS + r] = make_double2(d1[e][r][0], d1[e][r][1]);
    __syncthreads();
    for (int o = threadIdx.x; o < kHemvTile * NRHS; o += blockDim.x) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const double2 v = red[w * kHemvTile * NRHS + o];
            re += v.x;
            im += v.y;
        }
        r1part[(int64_t)blockIdx.x * kHemvTile * NRHS + o] = make_float2((float)re, (float)im);
    }
}

// ---- the same product for the FP64 coarse kernel ----------------------------------------
// Same tiles and lane roles; an entry is 16 bytes, so a step is two loads (rows L and
// 64 + L, each a contiguous 1 KiB run of the wavefront), layout [tile][h][s][row][L].  Every
// product and sum is FP64: the column partials stay in registers for the whole half (a 64-bit
// rotate is two 32-bit DPP moves) and the partials are FP64.

__device__ __forceinline__ double wave_rol1_d(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x134, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x134, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

__global__ __launch_bounds__(256) void k_hemv_pack64(const double2* __restrict__ K, d2v* __restrict__ kp, int64_t Nc,
                                                     int nbk) {
    const int64_t unit = blockIdx.x;   // (tile, half, step group of 4)
    const int64_t tile = unit / 32;
    const int hs = (int)(unit % 32);
    const int h = hs / 16, s = (hs % 16) * 4 + threadIdx.x / kWave;
    const int L = threadIdx.x % kWave;
    int I = 0;
    while (I + 1 < nbk && hemv_tile_index(I + 1, I + 1, nbk) <= tile) ++I;
    const int J = I + (int)(tile - hemv_tile_index(I, I, nbk));
    const int64_t col = (int64_t)J * kHemvTile + 64 * h + ((L + s) & 63);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int64_t row = (int64_t)I * kHemvTile + 64 * e + L;
        const double2 v = (row < Nc && col < Nc) ? K[row * Nc + col] : make_double2(0.0, 0.0);
        kp[(((tile * 2 + h) * 64 + s) * 2 + e) * kWave + L] = d2v{v.x, v.y};
    }
}

template <int NRHS, bool OFFDIAG>
__device__ __forceinline__ void hemv_half64(const d2v* __restrict__ kp, const double2* qj,
                                            const double2 (&qi)[2][NRHS], double (&d1)[2][NRHS][2],
                                            double2* __restrict__ r2part, int I, int J, int h, int nbk, int L) {
    constexpr int U = 4;   // steps whose loads are in flight together
    const d2v* tp = kp + (hemv_tile_index(I, J, nbk) * 2 + h) * (64 * 2 * kWave) + L;
    double a2[NRHS][2];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) a2[r][0] = a2[r][1] = 0.0;
#pragma unroll 1
    for (int s0 = 0; s0 < 64; s0 += U) {
        d2v kv[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < 2; ++e) kv[u][e] = __builtin_nontemporal_load(tp + (int64_t)(((s0 + u) * 2 + e) * kWave));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            __builtin_amdgcn_sched_barrier(0);
            const int c = (L + s0 + u) & 63;
            const double k0r = kv[u][0].x, k0i = kv[u][0].y, k1r = kv[u][1].x, k1i = kv[u][1].y;
#pragma unroll
            for (int r = 0; r < NRHS; ++r) {
                const double2 q = qj[r * 64 + c];
                d1[0][r][0] = fma(k0r, q.x, d1[0][r][0]);
                d1[0][r][0] = fma(-k0i, q.y, d1[0][r][0]);
                d1[0][r][1] = fma(k0r, q.y, d1[0][r][1]);
                d1[0][r][1] = fma(k0i, q.x, d1[0][r][1]);
                d1[1][r][0] = fma(k1r, q.x, d1[1][r][0]);
                d1[1][r][0] = fma(-k1i, q.y, d1[1][r][0]);
                d1[1][r][1] = fma(k1r, q.y, d1[1][r][1]);
                d1[1][r][1] = fma(k1i, q.x, d1[1][r][1]);
            }
            if (OFFDIAG) {
#pragma unroll
                for (int r = 0; r < NRHS; ++r) {
                    double re = a2[r][0], im = a2[r][1];
                    re = fma(k0r, qi[0][r].x, re);
                    re = fma(k0i, qi[0][r].y, re);
                    re = fma(k1r, qi[1][r].x, re);
                    re = fma(k1i, qi[1][r].y, re);
                    im = fma(k0r, qi[0][r].y, im);
                    im = fma(-k0i, qi[0][r].x, im);
                    im = fma(k1r, qi[1][r].y, im);
                    im = fma(-k1i, qi[1][r].x, im);
                    a2[r][0] = wave_rol1_d(re);
                    a2[r][1] = wave_rol1_d(im);
                }
            }
        }
    }
    // after 64 steps every column partial is back on the lane of its column
    if (OFFDIAG) {
        double2* out = r2part + hemv_tile_index(I, J, nbk) * kHemvTile * NRHS;
#pragma unroll
        for (int r = 0; r < NRHS; ++r) out[(64 * h + L) * NRHS + r] = make_double2(a2[r][0], a2[r][1]);
    }
}

template <int NRHS>
__global__ __launch_bounds__(256, NRHS > 3 ? 2 : 4) void k_hemv64(const d2v* __restrict__ kp, const double2* __restrict__ qbar,
                                                   const int* __restrict__ table, double2* __restrict__ r1part,
                                                   double2* __restrict__ r2part, int Nc, int nbk, int tpw) {
    extern __shared__ double2 hsm[];
    const int wave = threadIdx.x / kWave;
    const int L = threadIdx.x % kWave;
    const int code = table[blockIdx.x];
    const int I = code & 0xffff, g = code >> 16;
    const int h = wave & 1;
    double2* qj = hsm + wave * NRHS * 64;   // q_J of the half's 64 columns
    double2 qi[2][NRHS];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int row = I * kHemvTile + 64 * e + L;
#pragma unroll
        for (int r = 0; r < NRHS; ++r) qi[e][r] = row < Nc ? qbar[(int64_t)row * NRHS + r] : make_double2(0.0, 0.0);
    }
    double d1[2][NRHS][2];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int r = 0; r < NRHS; ++r) d1[e][r][0] = d1[e][r][1] = 0.0;
#pragma unroll 1
    for (int k = 0; k < tpw; ++k) {
        const int J = I + 2 * tpw * g + (wave >> 1) + 2 * k;
        const bool active = J < nbk;   // wavefront-uniform
        __syncthreads();
        if (active) {
            const int col = J * kHemvTile + 64 * h + L;
#pragma unroll
            for (int r = 0; r < NRHS; ++r)
                qj[r * 64 + L] = col < Nc ? qbar[(int64_t)col * NRHS + r] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (active) {
            if (J != I)
                hemv_half64<NRHS, true>(kp, qj, qi, d1, r2part, I, J, h, nbk, L);
            else
                hemv_half64<NRHS, false>(kp, qj, qi, d1, r2part, I, J, h, nbk, L);
        }
    }
    __syncthreads();
    double2* red = hsm;   // [4][128][NRHS]
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int r = 0; r < NRHS; ++r)
            red[(wave * kHemvTile + 64 * e + L) * NRHS + r] = make_double2(d1[e][r][0], d1[e][r][1]);
    __syncthreads();
    for (int o = threadIdx.x; o < kHemvTile * NRHS; o += blockDim.x) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const double2 v = red[w * kHemvTile * NRHS + o];
            re += v.x;
            im += v.y;
        }
        r1part[(int64_t)blockIdx.x * kHemvTile * NRHS + o] = make_double2(re, im);
    }
}

// r[i][rhs] = sum of the P1 partials of tile row b = i / 128 (its blocks in order), then of
// the P2 partials of tiles (I, b), I < b, in order of I.  Eight lanes per output: lane k
// adds partials k, k + 8, ... (FP64), then the eight sums are added in a fixed butterfly.
constexpr int kHemvRedLanes = 8;

template <int NRHS, class PT>
__global__ __launch_bounds__(256) void k_hemv_reduce(const PT* __restrict__ r1part, const PT* __restrict__ r2part,
                                                     const int* __restrict__ band0, double2* __restrict__ rout, int Nc,
                                                     int nbk) {
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kHemvRedLanes;
    const int k = threadIdx.x % kHemvRedLanes;
    const int64_t oc = min(o, (int64_t)Nc * NRHS - 1);   // lanes past the end: same work, no store
    const int i = (int)(oc / NRHS), r = (int)(oc % NRHS);
    const int b = i / kHemvTile, w = i % kHemvTile;
    const int p0 = band0[b], np1 = band0[b + 1] - p0;
    const int n = np1 + b;   // P1 partials, then P2 partials of tiles (0, b) .. (b - 1, b)
    double re = 0.0, im = 0.0;
    for (int t0 = k; t0 < n; t0 += 4 * kHemvRedLanes) {
        PT v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = min(t0 + u * kHemvRedLanes, n - 1);
            const int64_t src = t < np1 ? (int64_t)(p0 + t) : hemv_tile_index(t - np1, b, nbk);
            v[u] = (t < np1 ? r1part : r2part)[(src * kHemvTile + w) * NRHS + r];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t0 + u * kHemvRedLanes < n) {
                re += (double)v[u].x;
                im += (double)v[u].y;
            }
    }
#pragma unroll
    for (int off = 1; off < kHemvRedLanes; off <<= 1) {
        re += __shfl_xor(re, off, kWave);
        im += __shfl_xor(im, off, kWave);
    }
    if (k == 0 && o < (int64_t)Nc * NRHS) rout[o] = make_double2(re, im);
}

HemvShape hemv_shape(int64_t Nc, int dtype) {
    HemvShape h;
    h.nbk = (int)((Nc + kHemvTile - 1) / kHemvTile);
    h.tiles = (int64_t)h.nbk * (h.nbk + 1) / 2;
    auto blocks = [&](int tpw) {
        int64_t b = 0;
        for (int I = 0; I < h.nbk; ++I) b += hemv_groups(h.nbk, I, tpw);
        return b;
    };
    h.tpw = 1;
    while (blocks(h.tpw) > kHemvBlocks && 2 * h.tpw < h.nbk) ++h.tpw;
    h.blocks = blocks(h.tpw);
    h.elem_bytes = dtype == BSE_F64 ? sizeof(double2) : sizeof(float2);
    h.tile_bytes = (size_t)kHemvTile * kHemvTile * h.elem_bytes;
    return h;
}

hipError_t launch_hemv_pack(const Plan& p, hipStream_t s) {
    if (p.L.kp_bytes == 0) return hipSuccess;
    const HemvShape h = hemv_shape(p.g.Nc, p.g.dtype);
    if (p.g.dtype == BSE_F64)
        hipLaunchKernelGGL(k_hemv_pack64, dim3((unsigned)(h.tiles * 32)), dim3(kBlock), 0, s,
                           reinterpret_cast<const double2*>(p.Kc), reinterpret_cast<d2v*>(p.ws + p.L.kp), p.g.Nc,
                           h.nbk);
    else
        hipLaunchKernelGGL(k_hemv_pack, dim3((unsigned)(h.tiles * 32)), dim3(kBlock), 0, s,
                           reinterpret_cast<const float2*>(p.Kc), reinterpret_cast<f4v*>(p.ws + p.L.kp), p.g.Nc,
                           h.nbk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hemv_table, dim3(1), dim3(kWave), 0, s, reinterpret_cast<int*>(p.ws + p.L.htab),
                       reinterpret_cast<int*>(p.ws + p.L.htab) + h.blocks, h.nbk, h.tpw);
    return hipGetLastError();
}

template <int NRHS>
static hipError_t hemv_t(Plan& p, hipStream_t s) {
    const Geometry& g = p.g;
    const HemvShape h = hemv_shape(g.Nc, g.dtype);
    const int* tab = reinterpret_cast<const int*>(p.ws + p.L.htab);
    const double2* qbar = reinterpret_cast<const double2*>(p.ws + p.L.qbar);
    double2* rvec = reinterpret_cast<double2*>(p.ws + p.L.rvec);
    const int64_t n_out = g.Nc * NRHS;
    const dim3 rgrid((unsigned)((n_out * kHemvRedLanes + kBlock - 1) / kBlock));
    hipError_t e;
    if (g.dtype == BSE_F64) {
        double2* r1 = reinterpret_cast<double2*>(p.ws + p.L.hpart);
        double2* r2 = r1 + (size_t)h.blocks * kHemvTile * NRHS;
        // q_J of 4 wavefronts x 64 columns, or the P1 sums of 4 x 128 rows
        const size_t lds = (size_t)4 * kHemvTile * NRHS * sizeof(double2);
        launch_stream(p, (k_hemv64<NRHS>), dim3((unsigned)h.blocks), dim3(kBlock), lds, s,
                           reinterpret_cast<const d2v*>(p.ws + p.L.kp), qbar, tab, r1, r2, (int)g.Nc, h.nbk,
                           h.tpw);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_hemv_reduce<NRHS, double2>), rgrid, dim3(kBlock), 0, s, r1, r2, tab + h.blocks, rvec,
                           (int)g.Nc, h.nbk);
        return hipGetLastError();
    }
    float2* r1 = reinterpret_cast<float2*>(p.ws + p.L.hpart);
    float2* r2 = r1 + (size_t)h.blocks * kHemvTile * NRHS;
    // q_J and P2 sums of 4 wavefronts x 64 columns, or the P1 sums of 4 x 128 rows
    const size_t lds = std::max((size_t)4 * NRHS * 64 * (sizeof(float2) + sizeof(double2)),
                                (size_t)4 * kHemvTile * NRHS * sizeof(double2));
    launch_stream(p, (k_hemv<NRHS>), dim3((unsigned)h.blocks), dim3(kBlock), lds, s,
                       reinterpret_cast<const f4v*>(p.ws + p.L.kp), qbar, tab, r1, r2, (int)g.Nc, h.nbk, h.tpw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_hemv_reduce<NRHS, float2>), rgrid, dim3(kBlock), 0, s, r1, r2, tab + h.blocks, rvec,
                       (int)g.Nc, h.nbk);
    return hipGetLastError();
}

static hipError_t hemv_r(Plan& p, int n_rhs, hipStream_t s) {
    switch (n_rhs) {
        case 1: return hemv_t<1>(p, s);
        case 2: return hemv_t<2>(p, s);
        case 3: return hemv_t<3>(p, s);
        default: return hemv_t<4>(p, s);
    }
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
    if ((p.timing == 1 || p.timing == 3) && p.ev && p.ev_used + 2 <= p.ev_cap) {
        e0 = p.ev[p.ev_used];
        e1 = p.ev[p.ev_used + 1];
        p.ev_used += 2;
        if (p.timing == 1) (void)hipEventRecord(e0, s);
    }
    // mode 1 times the whole product between two recorded events; mode 3 hands the pair to
    // the launch of the streaming kernel (launch_stream)
    p.split_start = p.timing == 3 ? e0 : nullptr;
    p.split_ev = p.timing == 3 ? e1 : nullptr;
    hipError_t err = kc_lowp(p.g.dtype)        ? gemv_lowp(p, n_rhs, s)
                     : use_packed(p)          ? hemv_r(p, n_rhs, s)
                     : (p.g.dtype == BSE_F64) ? gemv_r<double2>(p, n_rhs, s)
                                              : gemv_r<float2>(p, n_rhs, s);
    if (e1 && p.timing == 1) (void)hipEventRecord(e1, s);
    p.split_start = p.split_ev = nullptr;
    return err;
}

}  // namespace bse
