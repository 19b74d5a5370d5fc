// Method 3 (Sec. 4): the divergence of the kernel treated in a band along the diagonal.
//
// Pairs of dense points farther apart than w d (d = 1 / n_c, the smallest distance
// between coarse points, reduced units, minimum image) keep the Method 1 kernel
// K^i = interp(K_c) of Eq. (interp1).  Inside the band the coefficients of
// Eq. (diverg) are interpolated and combined with the dense q.  For the model
// kernel the split is K_c = a_c s(q) + c_c with s(q) = 1 / (|q|^2 + kappa^2) (see
// setup.hip), so inside the band
//     K^{M3}(k, k') = interp(a_c)(k, k') s(q_dense) + interp(c_c)(k, k')
//                   = K^i(k, k') + Delta(k, k'),
//     Delta(k, k') = sum_{z z'} f(k, z) f(k', z') [s(q_dense) - S_c(k~z, k~'z')]
//                    L_{kz} a_c(k~z, k~'z') L_{k'z'}^H,
// with L_{kz}[(v c), (n1 n2)] = d_{vk}^{n1 k~z} conj(d_{ck}^{n2 k~z}) and S_c the
// coarse value of s (the mini-cell mean at q = 0, as for s(q_dense) at k = k').
//
// The band is sparse with a fixed stencil: the offsets o of the dense mesh with
// |o|^2 <= (w n_div)^2, the same for every k.  bse_build_m3_band evaluates every
// block Delta(k, k + o) once (Table tab:scalings: O(N~_k N_div^2) work for the sparse
// form); each matvec then adds y_k = sum_o Delta(k, k + o) x_{k+o}, computed by
// k_m3_apply before the prolong, which adds y (times the chain scale) to its output.
//
// Band buffer (caller-owned, 256-byte aligned sections):
//   offset table  int4 [n_off_pad] (o1, o2, o3, 1), n_off_pad = n_off rounded up to
//                 even; a padding entry is (0, 0, 0, 0) with a zero block
//   blocks        per k (n_off_pad np^2 entries, storage precision), chunks of
//                 kM3Chunk offsets (the last one W <= kM3Chunk wide); inside a chunk
//                 row n holds its W np entries (o_local, m) contiguously
//   product       double2 [max_rhs][N]: y of the last matvec or step

#include <hip/hip_runtime.h>

#include <cmath>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

constexpr int kM3Chunk = 16;    // offsets per chunk of the block layout
constexpr int kM3MaxNE = 52;    // nv^2 + nc^2 for the largest compiled bands (4v6c)
constexpr int kM3MaxNP = 32;    // nv nc of the builder (its block has nv^2 nc^2 threads)
constexpr int kM3MaxR = 16;     // floor(w n_div) <= 16

static inline size_t up256(size_t b) { return (b + 255) / 256 * 256; }

struct BandLayout {
    int r;            // floor(w n_div)
    double R2;        // (w n_div)^2
    int n_off, n_off_pad, n_chunks;
    size_t table, blocks, yb, total;  // byte offsets / total
};

static int count_offsets(int r, double R2) {
    int n = 0;
    for (int a = -r; a <= r; ++a)
        for (int b = -r; b <= r; ++b)
            for (int c = -r; c <= r; ++c)
                if (a * a + b * b + c * c <= R2 * (1.0 + 1e-12) + 1e-12) ++n;
    return n;
}

static size_t band_elem_bytes(int dtype) { return dtype == BSE_F64 ? 16 : 8; }

// false (with the error set) when w does not give a valid band for g
static bool band_layout(const Geometry& g, double w, BandLayout* L) {
    if (!(w >= 0.0) || !std::isfinite(w)) {
        set_error("Method 3: the width w must be finite and >= 0");
        return false;
    }
    L->R2 = (w * g.n_div) * (w * g.n_div);
    L->r = (int)std::floor(w * g.n_div + 1e-9);
    if (L->r > kM3MaxR || 2 * L->r >= g.n_c * g.n_div) {
        set_error("Method 3: floor(w n_div) = %d must be <= %d and below half the dense mesh (%d)", L->r, kM3MaxR,
                  g.n_c * g.n_div);
        return false;
    }
    if (g.np > kM3MaxNP || g.ne > kM3MaxNE) {
        set_error("Method 3: nv nc <= %d and nv^2 + nc^2 <= %d", kM3MaxNP, kM3MaxNE);
        return false;
    }
    L->n_off = count_offsets(L->r, L->R2);
    L->n_off_pad = (L->n_off + 1) / 2 * 2;
    L->n_chunks = (L->n_off_pad + kM3Chunk - 1) / kM3Chunk;
    L->table = 0;
    L->blocks = up256((size_t)L->n_off_pad * sizeof(int4));
    L->yb = L->blocks + up256((size_t)g.nk * L->n_off_pad * g.np * g.np * band_elem_bytes(g.dtype));
    L->total = L->yb + up256((size_t)g.max_rhs * g.N * sizeof(double2));
    return true;
}

// s(q) = 1 / (|q|^2 + kappa^2), and its mean over the dense mini-cell (midpoint rule)
static double s_q0_mean(int n_c, int n_div, double kappa2, int nq) {
    const double h = 1.0 / ((double)n_c * n_div);
    double sum = 0.0;
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b)
            for (int c = 0; c < nq; ++c) {
                const double x = ((a + 0.5) / nq - 0.5) * h, y = ((b + 0.5) / nq - 0.5) * h,
                             z = ((c + 0.5) / nq - 0.5) * h;
                sum += 1.0 / (x * x + y * y + z * z + kappa2);
            }
    return sum / ((double)nq * nq * nq);
}

// offset table: lexicographic (o1, o2, o3) over the cube, kept when |o|^2 <= R2
__global__ void k_m3_offsets(int4* __restrict__ table, int r, double R2, int n_off_pad) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int n = 0;
    for (int a = -r; a <= r; ++a)
        for (int b = -r; b <= r; ++b)
            for (int c = -r; c <= r; ++c)
                if (a * a + b * b + c * c <= R2 * (1.0 + 1e-12) + 1e-12) table[n++] = make_int4(a, b, c, 1);
    for (; n < n_off_pad; ++n) table[n] = make_int4(0, 0, 0, 0);
}

__device__ __forceinline__ int fold_m3(int d, int n) {
    const int h = n / 2;
    return ((d + h) % n + n) % n - h;
}

// dense index (cell-major) and integer coordinates i n_div + j
__device__ __forceinline__ void dense_coords(int64_t kd, int n_c, int n_div, int* x) {
    const int ndiv3 = n_div * n_div * n_div;
    const int cell = (int)(kd / ndiv3), sub = (int)(kd % ndiv3);
    x[0] = (cell / (n_c * n_c)) * n_div + sub / (n_div * n_div);
    x[1] = ((cell / n_c) % n_c) * n_div + (sub / n_div) % n_div;
    x[2] = (cell % n_c) * n_div + sub % n_div;
}
__device__ __forceinline__ int64_t dense_index(const int* x, int n_c, int n_div) {
    const int nd = n_c * n_div;
    int c[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) c[i] = ((x[i] % nd) + nd) % nd;
    const int cell = ((c[0] / n_div) * n_c + c[1] / n_div) * n_c + c[2] / n_div;
    const int sub = ((c[0] % n_div) * n_div + c[1] % n_div) * n_div + c[2] % n_div;
    return (int64_t)cell * (n_div * n_div * n_div) + sub;
}

// ---- builder: one block per (k, offset), one thread per entry of the np x np block ----
template <class M2>
__global__ __launch_bounds__(1024) void k_m3_band(const M2* __restrict__ d, const M2* __restrict__ acoef,
                                                  const int4* __restrict__ table, M2* __restrict__ band, int n_c,
                                                  int n_div, int nv, int nc, int neighbours, int n_off_pad,
                                                  double kappa2, double s0) {
    __shared__ double2 dk[8][kM3MaxNE], dq[8][kM3MaxNE];
    __shared__ double2 X[kM3MaxNP * kM3MaxNP], Rb[kM3MaxNP * kM3MaxNP], Yl[kM3MaxNP * kM3MaxNP];
    __shared__ double gzz[64];
    __shared__ int ck[8], cq[8];
    const int np = nv * nc, ne = nv * nv + nc * nc;
    const int ndiv3 = n_div * n_div * n_div;
    const int64_t Nc = (int64_t)n_c * n_c * n_c * np;
    const int64_t bid = blockIdx.x;
    const int64_t k = bid / n_off_pad;
    const int o = (int)(bid % n_off_pad);
    const int t = threadIdx.x;
    const bool act = t < np * np;
    const int row = act ? t / np : 0, col = act ? t % np : 0;
    const int chunk = o / kM3Chunk, ol = o % kM3Chunk;
    const int W = min(kM3Chunk, n_off_pad - chunk * kM3Chunk);   // offsets of this chunk
    M2* out = band + ((int64_t)k * n_off_pad + chunk * kM3Chunk) * np * np + (int64_t)ol * np;
    const int4 off = table[o];
    if (off.w == 0) {   // padding offset: zero block
        if (act) st(out + (int64_t)row * W * np + col, cmake(0.0, 0.0));
        return;
    }
    int x[3];
    dense_coords(k, n_c, n_div, x);
    const int cell = (int)(k / ndiv3), sub = (int)(k % ndiv3);
    const int xq[3] = {x[0] + off.x, x[1] + off.y, x[2] + off.z};
    const int64_t kq = dense_index(xq, n_c, n_div);
    const int cellq = (int)(kq / ndiv3), subq = (int)(kq % ndiv3);
    for (int i = t; i < 8 * ne; i += blockDim.x) {
        const int z = i / ne, e = i % ne;
        const cd a = ld(d + ((int64_t)(cell * 8 + z) * ne + e) * ndiv3 + sub);
        const cd b = ld(d + ((int64_t)(cellq * 8 + z) * ne + e) * ndiv3 + subq);
        dk[z][e] = make_double2(a.re, a.im);
        dq[z][e] = make_double2(b.re, b.im);
    }
    if (t < 8) {
        ck[t] = corner_index(cell, t, n_c);
        cq[t] = corner_index(cellq, t, n_c);
    }
    __syncthreads();
    if (t < 64) {
        const int z = t / 8, zq = t % 8;
        const double f = prefactor(sub, z, n_div, neighbours) * prefactor(subq, zq, n_div, neighbours);
        const int nd = n_c * n_div;
        double sd = s0;
        if (off.x != 0 || off.y != 0 || off.z != 0) {
            const double qx = (double)off.x / nd, qy = (double)off.y / nd, qz = (double)off.z / nd;
            sd = 1.0 / (qx * qx + qy * qy + qz * qz + kappa2);
        }
        const int a = ck[z], b = cq[zq];
        double sc = s0;
        if (a != b) {
            const double qx = (double)fold_m3(a / (n_c * n_c) - b / (n_c * n_c), n_c) / n_c;
            const double qy = (double)fold_m3((a / n_c) % n_c - (b / n_c) % n_c, n_c) / n_c;
            const double qz = (double)fold_m3(a % n_c - b % n_c, n_c) / n_c;
            sc = 1.0 / (qx * qx + qy * qy + qz * qz + kappa2);
        }
        gzz[t] = f * (sd - sc);
    }
    __syncthreads();

    cd acc = cmake(0.0, 0.0);
    for (int z = 0; z < 8; ++z) {
        bool any = false;
        for (int zq = 0; zq < 8; ++zq) any |= gzz[z * 8 + zq] != 0.0;
        if (!any) continue;   // uniform
        // Y[(n1 n2), (v' c')] = sum_z' g_zz' sum_{(n3 n4)} a_c[(n1 n2), (n3 n4)] conj(R_z')[(v' c'), (n3 n4)]
        cd y = cmake(0.0, 0.0);
        for (int zq = 0; zq < 8; ++zq) {
            const double g = gzz[z * 8 + zq];
            if (g == 0.0) continue;   // uniform
            __syncthreads();
            if (act) {
                const cd a = ld(acoef + ((int64_t)ck[z] * np + row) * Nc + (int64_t)cq[zq] * np + col);
                X[t] = make_double2(a.re, a.im);
                // Rb[(v' c'), (n3 n4)] = conj(Dv'[v'][n3]) Dc'[c'][n4]
                const int v2 = row / nc, c2 = row % nc, n3 = col / nc, n4 = col % nc;
                const double2 dv = dq[zq][v2 * nv + n3], dc = dq[zq][nv * nv + c2 * nc + n4];
                cd r = cmake(0.0, 0.0);
                cfma_cj(r, cmake(dv.x, dv.y), cmake(dc.x, dc.y));
                Rb[t] = make_double2(r.re, r.im);
            }
            __syncthreads();
            if (act) {
                cd s = cmake(0.0, 0.0);
                for (int q = 0; q < np; ++q) {
                    const double2 a = X[row * np + q], b = Rb[col * np + q];
                    cfma(s, cmake(a.x, a.y), cmake(b.x, b.y));
                }
                y.re = fma(g, s.re, y.re);
                y.im = fma(g, s.im, y.im);
            }
        }
        // acc[(v c), (v' c')] += sum_{(n1 n2)} Dv[v][n1] conj(Dc[c][n2]) Y[(n1 n2), (v' c')]
        __syncthreads();
        if (act) Yl[t] = make_double2(y.re, y.im);
        __syncthreads();
        if (act) {
            const int v = row / nc, c = row % nc;
            for (int n1 = 0; n1 < nv; ++n1) {
                const double2 dv = dk[z][v * nv + n1];
                for (int n2 = 0; n2 < nc; ++n2) {
                    const double2 dc = dk[z][nv * nv + c * nc + n2];
                    cd l = cmake(0.0, 0.0);
                    cfma_jc(l, cmake(dv.x, dv.y), cmake(dc.x, dc.y));
                    const double2 yy = Yl[(n1 * nc + n2) * np + col];
                    cfma(acc, l, cmake(yy.x, yy.y));
                }
            }
        }
    }
    if (act) st(out + (int64_t)row * W * np + col, acc);
}

// ---- product: y_k = sum_o Delta(k, k + o) x_{k+o} -----------------------------------------
//
// Every wavefront owns RG consecutive rows of the block row of one dense point k and
// works alone (no LDS, no barrier).  Per chunk of offsets it loads its rows (one
// contiguous run per row, 16-byte units, a lane per unit) and the x_{k+o}[m] of the
// entries its lanes hold, straight from memory (x stays in the caches: every
// x_{k'} serves all k of its band); the dense index of k + o is computed once per
// chunk by the first lanes and shuffled.  The x of an entry is used by all RG rows.
// Each lane accumulates in FP64; the lanes of a row are added at the end in a fixed
// order.  Wavefronts are numbered so that each XCD takes a contiguous range of k.
// Rows per wavefront: the x of an entry serves all of them, so more rows cut the
// cache traffic of x (measured on 8^3 x 4, 3v6c, w = 1: 3 rows 4.9 TB/s, 6 rows 5.8 TB/s,
// no x loads at all 6.1 TB/s).  Up to 6 rows for FP32 blocks, balanced over the groups;
// 3 for FP64 blocks, whose 16-byte units hold one entry and need more registers.
template <int NP, int P>
constexpr int m3_rows() {
    constexpr int cap = P == 2 ? 6 : 3;
    constexpr int groups = (NP + cap - 1) / cap;
    return (NP + groups - 1) / groups;
}

template <class V2, int NP, int P>
struct XPair;   // the x values of the P entries of one 16-byte unit of the band
template <int NP>
struct XPair<float2, NP, 2> {   // FP32 band and vectors: entries e, e + 1
    __device__ static inline void load(const float2* x, int64_t rowbase, int e0, int kq0, int kq1, float2* out) {
        if constexpr (NP % 2 == 0) {   // e0 even: both entries in one offset, 16 bytes
            const f4v v = *reinterpret_cast<const f4v*>(x + rowbase + (int64_t)kq0 * NP + e0 % NP);
            out[0] = make_float2(v.x, v.y);
            out[1] = make_float2(v.z, v.w);
        } else {
            out[0] = x[rowbase + (int64_t)kq0 * NP + e0 % NP];
            out[1] = x[rowbase + (int64_t)kq1 * NP + (e0 + 1) % NP];
        }
    }
};
template <int NP>
struct XPair<double2, NP, 2> {   // FP32 band, FP64 vectors
    __device__ static inline void load(const double2* x, int64_t rowbase, int e0, int kq0, int kq1, double2* out) {
        out[0] = x[rowbase + (int64_t)kq0 * NP + e0 % NP];
        out[1] = x[rowbase + (int64_t)kq1 * NP + (e0 + 1) % NP];
    }
};
template <int NP>
struct XPair<double2, NP, 1> {   // FP64 band and vectors: one entry per unit
    __device__ static inline void load(const double2* x, int64_t rowbase, int e0, int kq0, int, double2* out) {
        out[0] = x[rowbase + (int64_t)kq0 * NP + e0 % NP];
    }
};

template <class M2, class V2, int NV, int NC, int NR>
__global__ __launch_bounds__(256) void k_m3_apply(const M2* __restrict__ band, const int4* __restrict__ table,
                                                  const V2* __restrict__ x, double2* __restrict__ yb, int n_c,
                                                  int n_div, int n_off_pad, int64_t N, int64_t n_items,
                                                  int64_t blocks_per_xcd) {
    constexpr int NP = NV * NC;
    constexpr int OC = kM3Chunk;
    using U = Unit16<M2>;
    using Rw = typename U::t;
    constexpr int P = U::P;
    constexpr int RU = OC * NP / P;                  // 16-byte units of one row of a full chunk
    constexpr int IT = (RU + kWave - 1) / kWave;     // units per lane
    constexpr int RG = m3_rows<NP, P>();
    constexpr int NG = (NP + RG - 1) / RG;           // row groups of a block row
    static_assert((2 * NP) % P == 0 && (OC * NP) % P == 0, "whole 16-byte units per row and chunk");
    static_assert(OC <= kWave, "one lane per offset of a chunk");
    const int64_t blk = (int64_t)(blockIdx.x % 8) * blocks_per_xcd + blockIdx.x / 8;
    const int64_t item = blk * 4 + threadIdx.x / kWave;
    if (item >= n_items) return;   // whole wavefront; the kernel has no barrier
    const int64_t k = item / NG;
    const int g = (int)(item % NG);
    const int lane = threadIdx.x % kWave;
    int xk[3];
    dense_coords(k, n_c, n_div, xk);
    const Rw* bk = reinterpret_cast<const Rw*>(band) + (int64_t)k * n_off_pad * NP * NP / P;

    cd acc[RG][NR];
#pragma unroll
    for (int rr = 0; rr < RG; ++rr)
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[rr][r] = cmake(0.0, 0.0);

    for (int c0 = 0; c0 < n_off_pad; c0 += OC) {
        const int ru = min(OC, n_off_pad - c0) * NP / P;   // units of one row of this chunk
        const Rw* bc = bk + (int64_t)c0 * NP * NP / P;
        // dense index of k + o for the chunk's offsets (lane l < OC holds offset c0 + l)
        int kq_l;
        {
            const int4 o = table[min(c0 + lane, n_off_pad - 1)];
            const int xq[3] = {xk[0] + o.x, xk[1] + o.y, xk[2] + o.z};
            kq_l = (int)dense_index(xq, n_c, n_div);
        }
        Rw bu[RG][IT];
#pragma unroll
        for (int rr = 0; rr < RG; ++rr) {
            const int n = min(g * RG + rr, NP - 1);
#pragma unroll
            for (int it = 0; it < IT; ++it) bu[rr][it] = bc[(int64_t)n * ru + min(lane + it * kWave, ru - 1)];
        }
        V2 xv[IT][NR][P];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e0 = min(lane + it * kWave, ru - 1) * P;
            const int kq0 = __shfl(kq_l, e0 / NP, kWave);
            const int kq1 = __shfl(kq_l, min((e0 + P - 1) / NP, OC - 1), kWave);
#pragma unroll
            for (int r = 0; r < NR; ++r) XPair<V2, NP, P>::load(x, (int64_t)r * N, e0, kq0, kq1, xv[it][r]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            if (lane + it * kWave >= ru) break;
#pragma unroll
            for (int pp = 0; pp < P; ++pp)
#pragma unroll
                for (int rr = 0; rr < RG; ++rr) {
                    const cd bv = cv(U::get(bu[rr][it], pp));
#pragma unroll
                    for (int r = 0; r < NR; ++r) cfma(acc[rr][r], bv, cv(xv[it][r][pp]));
                }
        }
    }
#pragma unroll
    for (int rr = 0; rr < RG; ++rr) {
        const int n = g * RG + rr;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double re = wave_sum(acc[rr][r].re), im = wave_sum(acc[rr][r].im);
            if (lane == 0 && n < NP) yb[(int64_t)r * N + k * NP + n] = make_double2(re, im);
        }
    }
}

template <class M2, class V2, int NV, int NC>
static hipError_t m3_apply_go(const Plan& p, const void* x, int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    const M2* band = reinterpret_cast<const M2*>(p.m3_band + up256((size_t)p.m3_noff_pad * sizeof(int4)));
    const int4* table = reinterpret_cast<const int4*>(p.m3_band);
    const V2* xv = reinterpret_cast<const V2*>(x);
    constexpr int NP = NV * NC;
    constexpr int RG = m3_rows<NP, Unit16<M2>::P>();
    const int64_t n_items = g.nk * ((NP + RG - 1) / RG);   // (k, row group) wavefronts
    const int64_t nblk = (n_items + 3) / 4;
    const int64_t per_xcd = (nblk + 7) / 8;
    dim3 grid((unsigned)(8 * per_xcd)), block(256);
#define BSE_M3_GO(R)                                                                                              \
    hipLaunchKernelGGL((k_m3_apply<M2, V2, NV, NC, R>), grid, block, 0, s, band, table, xv, p.m3_yb, g.n_c, g.n_div, \
                       p.m3_noff_pad, g.N, n_items, per_xcd)
    switch (n_rhs) {
        case 1: BSE_M3_GO(1); break;
        case 2: BSE_M3_GO(2); break;
        case 3: BSE_M3_GO(3); break;
        default: BSE_M3_GO(4); break;
    }
#undef BSE_M3_GO
    return hipGetLastError();
}

// Band pairs without a compiled form: nv nc at run time, one thread per output entry
// (k, row n, right-hand side) summing its row of every block in the band, in FP64.
template <class M2, class V2>
__global__ __launch_bounds__(256) void k_m3_apply_any(const M2* __restrict__ band, const int4* __restrict__ table,
                                                      const V2* __restrict__ x, double2* __restrict__ yb, int n_c,
                                                      int n_div, int n_off_pad, int64_t N, int64_t nk, int np,
                                                      int n_rhs) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nk * np * n_rhs) return;
    const int r = (int)(idx % n_rhs);
    const int64_t rest = idx / n_rhs;
    const int n = (int)(rest % np);
    const int64_t k = rest / np;
    int xk[3];
    dense_coords(k, n_c, n_div, xk);
    const M2* bk = band + k * n_off_pad * np * np;
    cd acc = cmake(0.0, 0.0);
    for (int c0 = 0; c0 < n_off_pad; c0 += kM3Chunk) {
        const int W = min(kM3Chunk, n_off_pad - c0);
        const M2* row = bk + ((int64_t)c0 * np + (int64_t)n * W) * np;   // row n of the chunk: (o_local, m)
        for (int ol = 0; ol < W; ++ol) {
            const int4 o = table[c0 + ol];
            const int xq[3] = {xk[0] + o.x, xk[1] + o.y, xk[2] + o.z};
            const V2* xr = x + (int64_t)r * N + dense_index(xq, n_c, n_div) * np;
            for (int m = 0; m < np; ++m) cfma(acc, ld(row + ol * np + m), ld(xr + m));
        }
    }
    yb[(int64_t)r * N + k * np + n] = make_double2(acc.re, acc.im);
}

template <class M2, class V2>
static hipError_t m3_apply_any_go(const Plan& p, const void* x, int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    const M2* band = reinterpret_cast<const M2*>(p.m3_band + up256((size_t)p.m3_noff_pad * sizeof(int4)));
    const int4* table = reinterpret_cast<const int4*>(p.m3_band);
    const int64_t total = g.nk * g.np * n_rhs;
    hipLaunchKernelGGL((k_m3_apply_any<M2, V2>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, band, table,
                       reinterpret_cast<const V2*>(x), p.m3_yb, g.n_c, g.n_div, p.m3_noff_pad, g.N, g.nk, g.np, n_rhs);
    return hipGetLastError();
}

template <int NV, int NC>
static hipError_t m3_apply_dt(const Plan& p, const void* x, int n_rhs, hipStream_t s) {
    switch (p.g.dtype) {
        case BSE_F64: return m3_apply_go<double2, double2, NV, NC>(p, x, n_rhs, s);
        case BSE_F32:
        case BSE_BF16_KC:
        case BSE_F16_KC: return m3_apply_go<float2, float2, NV, NC>(p, x, n_rhs, s);
        default: return m3_apply_go<float2, double2, NV, NC>(p, x, n_rhs, s);
    }
}

hipError_t launch_m3_apply(Plan& p, const void* x, int n_rhs, hipStream_t s) {
    if (!p.m3_band) return hipSuccess;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (p.timing == 2 && p.ev && p.ev_used + 2 <= p.ev_cap) {
        e0 = p.ev[p.ev_used];
        e1 = p.ev[p.ev_used + 1];
        p.ev_used += 2;
        (void)hipEventRecord(e0, s);
    }
    hipError_t err = hipErrorInvalidValue;
    const int nv = p.g.nv, nc = p.g.nc;
    if (supported_bands(nv, nc)) {
#define BSE_CASE(a_, b_) \
    if (nv == a_ && nc == b_) err = m3_apply_dt<a_, b_>(p, x, n_rhs, s);
        BSE_BANDS(BSE_CASE)
#undef BSE_CASE
    } else {
        switch (p.g.dtype) {
            case BSE_F64: err = m3_apply_any_go<double2, double2>(p, x, n_rhs, s); break;
            case BSE_F32:
            case BSE_BF16_KC:
            case BSE_F16_KC: err = m3_apply_any_go<float2, float2>(p, x, n_rhs, s); break;
            default: err = m3_apply_any_go<float2, double2>(p, x, n_rhs, s); break;
        }
    }
    if (e1) (void)hipEventRecord(e1, s);
    return err;
}

}  // namespace bse

using namespace bse;

extern "C" {

bse_status bse_build_divergence_coefficient(const bse_dims* dims, const double* vecs_coarse, const double* tau,
                                            const bse_kernel_model* model, void* a_out, hipStream_t stream) {
    Geometry g;
    if (!make_geometry(dims, &g)) return BSE_ERR_INVALID_ARG;
    if (!vecs_coarse || !tau || !model || !a_out) {
        set_error("bse_build_divergence_coefficient: NULL pointer");
        return BSE_ERR_INVALID_ARG;
    }
    if (g.n_orb_input < 1 || g.n_orb_input > 16 || g.nv + g.nc > 16 || g.np > 32) {
        set_error("bse_build_divergence_coefficient: needs n_orb <= 16, nv + nc <= 16, nv * nc <= 32");
        return BSE_ERR_UNSUPPORTED;
    }
    if (!(model->eps_inf > 0) || model->g2_max < 0 || model->g2_max > 4) {
        set_error("bse_build_divergence_coefficient: model parameters out of range");
        return BSE_ERR_INVALID_ARG;
    }
    hipError_t e = launch_divergence_coefficient(g, vecs_coarse, tau, *model, a_out, stream);
    return e == hipSuccess ? BSE_OK : hip_fail_status(e, "bse_build_divergence_coefficient");
}

bse_status bse_m3_band_info(const bse_dims* dims, double w, int32_t* n_offsets, size_t* band_bytes) {
    Geometry g;
    if (!make_geometry(dims, &g)) return BSE_ERR_INVALID_ARG;
    BandLayout L;
    if (!band_layout(g, w, &L)) return BSE_ERR_INVALID_ARG;
    if (n_offsets) *n_offsets = L.n_off;
    if (band_bytes) *band_bytes = L.total;
    return BSE_OK;
}

bse_status bse_build_m3_band(const bse_dims* dims, const void* d, const void* a_coef, const bse_kernel_model* model,
                             double w, void* band, size_t band_bytes, hipStream_t stream) {
    Geometry g;
    if (!make_geometry(dims, &g)) return BSE_ERR_INVALID_ARG;
    if (!d || !a_coef || !model || !band) {
        set_error("bse_build_m3_band: NULL pointer");
        return BSE_ERR_INVALID_ARG;
    }
    if (!(model->eps_inf > 0) || !(model->lambda >= 0) || model->q0_quad < 1 || model->q0_quad > 256) {
        set_error("bse_build_m3_band: model parameters out of range");
        return BSE_ERR_INVALID_ARG;
    }
    BandLayout L;
    if (!band_layout(g, w, &L)) return BSE_ERR_INVALID_ARG;
    if (((uintptr_t)band & 255) != 0 || band_bytes < L.total) {
        set_error("bse_build_m3_band: band must be 256-byte aligned and >= %zu bytes", L.total);
        return BSE_ERR_WORKSPACE;
    }
    const double kappa2 = model->lambda * model->lambda / (4.0 * M_PI * M_PI * model->eps_inf);
    const double s0 = s_q0_mean(g.n_c, g.n_div, kappa2, model->q0_quad);
    char* base = reinterpret_cast<char*>(band);
    int4* table = reinterpret_cast<int4*>(base + L.table);
    hipLaunchKernelGGL(k_m3_offsets, dim3(1), dim3(64), 0, stream, table, L.r, L.R2, L.n_off_pad);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        const int threads = (g.np * g.np + kWave - 1) / kWave * kWave;
        const dim3 grid((unsigned)(g.nk * L.n_off_pad));
        if (g.dtype == BSE_F64)
            hipLaunchKernelGGL(k_m3_band<double2>, grid, dim3(threads), 0, stream, reinterpret_cast<const double2*>(d),
                               reinterpret_cast<const double2*>(a_coef), table,
                               reinterpret_cast<double2*>(base + L.blocks), g.n_c, g.n_div, g.nv, g.nc, g.neighbours,
                               L.n_off_pad, kappa2, s0);
        else
            hipLaunchKernelGGL(k_m3_band<float2>, grid, dim3(threads), 0, stream, reinterpret_cast<const float2*>(d),
                               reinterpret_cast<const float2*>(a_coef), table,
                               reinterpret_cast<float2*>(base + L.blocks), g.n_c, g.n_div, g.nv, g.nc, g.neighbours,
                               L.n_off_pad, kappa2, s0);
        e = hipGetLastError();
    }
    return e == hipSuccess ? BSE_OK : hip_fail_status(e, "bse_build_m3_band");
}

bse_status bse_plan_set_m3_band(bse_plan* plan, void* band, double w) {
    if (!plan) {
        set_error("bse_plan_set_m3_band: NULL plan");
        return BSE_ERR_INVALID_ARG;
    }
    Plan& p = *reinterpret_cast<Plan*>(plan);
    if (!band) {
        p.m3_band = nullptr;
        p.m3_yb = nullptr;
        p.m3_noff_pad = 0;
        return BSE_OK;
    }
    if (p.g.np > kM3MaxNP || p.g.ne > kM3MaxNE) {   // the builder's limits
        set_error("bse_plan_set_m3_band: Method 3 takes nv nc <= %d and nv^2 + nc^2 <= %d", kM3MaxNP, kM3MaxNE);
        return BSE_ERR_UNSUPPORTED;
    }
    BandLayout L;
    if (!band_layout(p.g, w, &L)) return BSE_ERR_INVALID_ARG;
    if (((uintptr_t)band & 255) != 0) {
        set_error("bse_plan_set_m3_band: band must be 256-byte aligned");
        return BSE_ERR_INVALID_ARG;
    }
    p.m3_band = reinterpret_cast<const char*>(band);
    p.m3_yb = reinterpret_cast<double2*>(reinterpret_cast<char*>(band) + L.yb);
    p.m3_noff_pad = L.n_off_pad;
    return BSE_OK;
}

}  // extern "C"
