// Restrict (Eq. matmul1) with the Lanczos update or the chain start in front.
//
//   q^{z}_{cell}[n3][n4] = sum_{sub in S(cell)} f(sub, z) sum_{v c} conj(Dv[v][n3]) x[v][c] Dc[c][n4]
//
// One block per (cell, right-hand side), 4 wavefronts.  A lane owns one corner z, one
// subpoint column j and one half h of the conduction index n4 (lane = 8 z + 2 j + h)
// and walks the subpoints sub = 4 s + j; the wavefronts take interleaved s.  Each
// lane therefore accumulates the whole sub-sum of its corner and half in registers;
// only 4 lanes (xor 2, 4) and then 4 wavefronts (LDS, fixed order) are added at the
// end.  Every (sub, corner) overlap block is read by one lane pair, as 4-subpoint
// contiguous segments.
//
// In chain modes the block first forms its slice of the new vector with coalesced
// element-wise accesses (u_{i+1} = w - a_i psi_i, or u_1 = P) and writes the slice's
// squared norm; the collapse that follows adds those into b_{i+1}.  a_i itself is
// the sum of the prolong's per-cell partials, added by every block in the same
// fixed order (so every block holds the same bits); the block of cell 0 records it.
// No block waits on another: kernel boundaries order the steps.
//
// Block order is XCD-aware: the n_rhs blocks of one cell carry indices that are equal
// modulo 8, so they run on the same XCD and share its L2 copy of the cell's overlaps.

#include <hip/hip_runtime.h>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

// sum over the 4 subpoint columns j of a corner (lane bits 1 and 2)
__device__ __forceinline__ double xor_sum_j(double v) {
    v += __shfl_xor(v, 2, kWave);
    v += __shfl_xor(v, 4, kWave);
    return v;
}

template <class M2, class V2, int NV, int NC, int MODE>
__global__ __launch_bounds__(256, (NV * NC > 18) ? 2 : 3) void k_restrict2(
    const M2* __restrict__ d, const V2* x, const V2* __restrict__ psi, const double2* __restrict__ P, V2* out,
    double2* __restrict__ qpart, const ChainState* __restrict__ cs, StepScalars* __restrict__ pend,
    const double* __restrict__ ppart, double* __restrict__ rpart, double* __restrict__ alpha,
    double* __restrict__ beta, int lda, int ldb, int step, int n_c, int n_div, int neighbours, int64_t N,
    int n_rhs) {
    constexpr int NP = NV * NC;
    constexpr int NE = NV * NV + NC * NC;
    constexpr int NW = kBlock / kWave;
    __shared__ double2 red[NW][8][NP];
    __shared__ double sred[NW];
    const int ndiv3 = n_div * n_div * n_div;
    const int ncells = n_c * n_c * n_c;
    // XCD-aware block -> (cell, rhs)
    const int bid = blockIdx.x;
    const int rest = bid / 8;
    const int rhs = rest % n_rhs;
    const int cell = (rest / n_rhs) * 8 + bid % 8;
    if (cell >= ncells) return;  // padding blocks (not counted below)
    const int t = threadIdx.x;
    const int wave = t / kWave;
    const int lane = t % kWave;
    const int64_t base = (int64_t)rhs * N + (int64_t)cell * ndiv3 * NP;
    const int nelem = ndiv3 * NP;
    double uu = 0.0, pp = 0.0;

    if (MODE == RESTRICT_INIT) {
        // chain coefficients start at zero
        const int64_t tid = (int64_t)(cell * n_rhs + rhs) * blockDim.x + t;
        const int64_t nth = (int64_t)ncells * n_rhs * blockDim.x;
        for (int64_t i = tid; i < (int64_t)n_rhs * lda; i += nth) alpha[i] = 0.0;
        for (int64_t i = tid; i < (int64_t)n_rhs * ldb; i += nth) beta[i] = 0.0;
    }
    if (MODE != RESTRICT_PLAIN) {
        // init: u_1 = P.  update: u_{i+1} = w - a_i psi_i = w - a_i s_i u_i  (Eq. bi), with
        // a_i = s_i sum_cells <u_i|w>_cell  (Eq. ai)
        double coef = 0.0;
        bool ok = true;
        if (MODE == RESTRICT_UPDATE) {
            const double pw = block_sum_strided(ppart + rhs * 2, ncells, n_rhs * 2, sred);
            const double ww = block_sum_strided(ppart + rhs * 2 + 1, ncells, n_rhs * 2, sred);
            const ChainState st = cs[rhs];
            const double a = st.s_cur * pw;
            ok = st.active && isfinite(a) && isfinite(ww);
            coef = ok ? a * st.s_cur : 0.0;
            if (cell == 0 && t == 0 && st.active) {
                StepScalars sc;
                sc.a = a;
                sc.ww = ww;
                sc.ok = ok;
                sc.pad[0] = sc.pad[1] = sc.pad[2] = 0;
                pend[rhs] = sc;
                if (ok) alpha[(int64_t)rhs * lda + step] = a;
            }
        }
        for (int i = t; i < nelem; i += blockDim.x) {
            cd u = cmake(0.0, 0.0);
            if (MODE == RESTRICT_INIT) {
                u = ld(P + base + i);
                pp = fma(u.re, u.re, pp);
                pp = fma(u.im, u.im, pp);
            } else if (ok) {
                u = ld(x + base + i);
                const cd ps = ld(psi + base + i);
                u.re = fma(-coef, ps.re, u.re);
                u.im = fma(-coef, ps.im, u.im);
            }
            st(out + base + i, u);
            const cd ur = rounded(u, out);
            uu = fma(ur.re, ur.re, uu);
            uu = fma(ur.im, ur.im, uu);
        }
        __syncthreads();  // the block's slice of u is visible to all its lanes
    }
    const V2* src = (MODE == RESTRICT_PLAIN) ? x : out;

    constexpr int NCH = (NC + 1) / 2;   // conduction columns per lane half
    const int z = lane >> 3;
    const int j = (lane >> 1) & 3;
    const int h = lane & 1;
    const int S = (ndiv3 + 3) / 4;
    cd acc[NV][NCH];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int q = 0; q < NCH; ++q) acc[v][q] = cmake(0.0, 0.0);
    // overlaps of (cell, z) and the block's vector slice through buffer resources:
    // one per-lane offset, element strides in scalar offsets
    // (the resource must be wavefront-uniform: the cell's 8 corner blocks, corner in the lane offset)
    const __amdgpu_buffer_rsrc_t rd =
        make_rsrc(d + (int64_t)cell * 8 * NE * ndiv3, (uint32_t)(8 * NE * ndiv3 * sizeof(M2)));
    const __amdgpu_buffer_rsrc_t rx = make_rsrc(src + base, (uint32_t)(nelem * sizeof(V2)));
    const int es = ndiv3 * (int)sizeof(M2);
#pragma unroll 1
    for (int s = wave; s < S; s += NW) {
        const int sub = 4 * s + j;
        if (sub >= ndiv3) continue;
        const double f = prefactor(sub, z, n_div, neighbours);
        const int vd = (z * NE * ndiv3 + sub) * (int)sizeof(M2);
        const int vx = sub * NP * (int)sizeof(V2);
        M2 dv[NV * NV];
#pragma unroll
        for (int e = 0; e < NV * NV; ++e) dv[e] = bload<M2>(rd, vd, e * es);
        // T[v][q] = sum_c x[v][c] Dc[c][n4(q)] over this lane's half of n4
        cd T[NV][NCH];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < NCH; ++q) T[v][q] = cmake(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            __builtin_amdgcn_sched_barrier(0);
            cd xc[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) xc[v] = cv(bload<V2>(rx, vx, (v * NC + c) * (int)sizeof(V2)));
#pragma unroll
            for (int q = 0; q < NCH; ++q) {
                const int n4 = h * NCH + q;
                if (n4 >= NC) break;
                const cd dc = cv(bload<M2>(rd, vd, (NV * NV + c * NC + n4) * es));
#pragma unroll
                for (int v = 0; v < NV; ++v) cfma(T[v][q], xc[v], dc);
            }
        }
        // acc[n3][q] += f sum_v conj(Dv[v][n3]) T[v][q]
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < NCH; ++q) T[v][q] = cscale(T[v][q], f);
#pragma unroll
        for (int n3 = 0; n3 < NV; ++n3)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const cd dvv = cv(dv[v * NV + n3]);
#pragma unroll
                for (int q = 0; q < NCH; ++q) cfma_cj(acc[n3][q], dvv, T[v][q]);
            }
    }
    // sum the 4 subpoint columns of each (corner, half), then the wavefronts
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
            acc[v][q].re = xor_sum_j(acc[v][q].re);
            acc[v][q].im = xor_sum_j(acc[v][q].im);
        }
    if (j == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < NCH; ++q) {
                const int n4 = h * NCH + q;
                if (n4 < NC) red[wave][z][v * NC + n4] = make_double2(acc[v][q].re, acc[v][q].im);
            }
    }
    __syncthreads();
    for (int o = t; o < 8 * NP; o += blockDim.x) {
        const int zz = o / NP, p = o % NP;
        double re = 0.0, im = 0.0;
        for (int w = 0; w < NW; ++w) {
            re += red[w][zz][p].x;
            im += red[w][zz][p].y;
        }
        qpart[((int64_t)(cell * 8 + zz) * n_rhs + rhs) * NP + p] = make_double2(re, im);
    }
    if (MODE == RESTRICT_PLAIN) return;

    // ||u||^2 (and ||P||^2 at the start) of this block's slice, for the collapse
    uu = block_sum(uu, sred);
    pp = block_sum(pp, sred);
    if (t == 0) {
        rpart[((int64_t)cell * n_rhs + rhs) * 2] = uu;
        rpart[((int64_t)cell * n_rhs + rhs) * 2 + 1] = pp;
    }
}

template <class M2, class V2, int NV, int NC>
hipError_t restrict_launch(const Plan& p, int mode, const void* x, const void* w, const void* psi, const double* P,
                           void* out, int step, double* a, double* b, int lda, int ldb, int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    double2* qpart = reinterpret_cast<double2*>(p.ws + p.L.qpart);
    const ChainState* cs = reinterpret_cast<const ChainState*>(p.ws + p.L.chain) + state_in(step) * kMaxRhs;
    StepScalars* pend = reinterpret_cast<StepScalars*>(p.ws + p.L.pend);
    const double* ppart = reinterpret_cast<const double*>(p.ws + p.L.ppart);
    double* rpart = reinterpret_cast<double*>(p.ws + p.L.rpart);
    const M2* d = reinterpret_cast<const M2*>(p.d);
    const int groups = (g.ncells + 7) / 8;
    dim3 grid(groups * 8 * n_rhs), block(kBlock);
    if (mode == RESTRICT_PLAIN)
        hipLaunchKernelGGL((k_restrict2<M2, V2, NV, NC, RESTRICT_PLAIN>), grid, block, 0, s, d,
                           reinterpret_cast<const V2*>(x), nullptr, nullptr, nullptr, qpart, cs, pend, ppart, rpart,
                           nullptr, nullptr, 0, 0, 0, g.n_c, g.n_div, g.neighbours, g.N, n_rhs);
    else if (mode == RESTRICT_UPDATE)
        hipLaunchKernelGGL((k_restrict2<M2, V2, NV, NC, RESTRICT_UPDATE>), grid, block, 0, s, d,
                           reinterpret_cast<const V2*>(w), reinterpret_cast<const V2*>(psi), nullptr,
                           reinterpret_cast<V2*>(out), qpart, cs, pend, ppart, rpart, a, b, lda, ldb, step, g.n_c,
                           g.n_div, g.neighbours, g.N, n_rhs);
    else
        hipLaunchKernelGGL((k_restrict2<M2, V2, NV, NC, RESTRICT_INIT>), grid, block, 0, s, d, nullptr, nullptr,
                           reinterpret_cast<const double2*>(P), reinterpret_cast<V2*>(out), qpart, cs, pend, ppart,
                           rpart, a, b, lda, ldb, 0, g.n_c, g.n_div, g.neighbours, g.N, n_rhs);
    return hipGetLastError();
}

#define BSE_RESTRICT_INST(M2, V2, A, B)                                                                             \
    template hipError_t restrict_launch<M2, V2, A, B>(const Plan&, int, const void*, const void*, const void*, \
                                                      const double*, void*, int, double*, double*, int, int, int, \
                                                      hipStream_t);
#define BSE_RESTRICT_ALL(A, B)                  \
    BSE_RESTRICT_INST(double2, double2, A, B)   \
    BSE_RESTRICT_INST(float2, float2, A, B)     \
    BSE_RESTRICT_INST(float2, double2, A, B)
BSE_BANDS(BSE_RESTRICT_ALL)

}  // namespace bse
