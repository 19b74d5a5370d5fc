// Prolong (Eq. matmul3) plus the diagonal of Eq. (bse1):
//
//   w_k = delta_k (.) psi_k + sum_z f(k, z) Dv_z r_{k~z} Dc_z^H   [- b_i psi_{i-1} in a chain]
//
// One block per coarse cell; wavefront = right-hand side, lane = subpoint, so each
// lane owns its output block and nothing is reduced across lanes.  In a chain the
// block also writes its FP64 partials of <u_i|w> and ||w||^2, from which the next
// kernel forms a_i (Eq. ai).
//
// Main form (n_div^3 <= 64): the block stages the overlaps of one corner at a time
// in LDS with coalesced 16-byte loads, double-buffered (the loads for corner z+1 are
// in flight while corner z is computed), so every wavefront of the cell reads them
// from LDS; the 8 coarse blocks r_{k~z} sit in LDS as well.  Two wavefronts per
// right-hand side split the conduction index c in halves, which halves the FP64
// accumulators each lane holds.  After the corner loop the lanes' sums pass through
// LDS, and the whole block applies the diagonal and the chain terms element by element
// over the cell's contiguous slice of each vector.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

// ---- general form: any number of subpoints per cell, overlaps read from global memory
template <class M2, class V2, int NV, int NC, int MODE>
__global__ __launch_bounds__(256) void k_prolong1(const M2* __restrict__ d, const double* __restrict__ delta,
                                                 const double2* __restrict__ rvec, const V2* __restrict__ x,
                                                 V2* __restrict__ out, double* __restrict__ ppart,
                                                 const ChainState* __restrict__ chain, int n_c, int n_div,
                                                 int neighbours, int64_t N, int n_rhs,
                                                 const double2* __restrict__ yb) {
    constexpr int NP = NV * NC;
    constexpr int NE = NV * NV + NC * NC;
    const int ndiv3 = n_div * n_div * n_div;
    const int rhs = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x % kWave;
    const int cell = blockIdx.x;
    const int64_t kd0 = (int64_t)cell * ndiv3;
    double s_cur = 1.0, c_prev = 0.0;
    if (MODE == PROLONG_LANCZOS) {
        s_cur = chain[rhs].s_cur;                         // psi_i = s_i u_i
        c_prev = chain[rhs].b_cur * chain[rhs].s_prev;    // b_i psi_{i-1} = b_i s_{i-1} u_{i-1}
    }
    const bool use_prev = (MODE == PROLONG_LANCZOS) && c_prev != 0.0;
    double pw = 0.0, ww = 0.0;

    for (int sub = lane; sub < ndiv3; sub += kWave) {
        const int64_t kd = kd0 + sub;
        const int64_t t0 = (int64_t)rhs * N + kd * NP;
        cd acc[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const cd xv = ld(x + t0 + p);
            acc[p] = cscale(xv, delta[kd * NP + p] * s_cur);
            if (use_prev) {
                const cd pv = ld(out + t0 + p);
                acc[p].re = fma(-c_prev, pv.re, acc[p].re);
                acc[p].im = fma(-c_prev, pv.im, acc[p].im);
            }
            if (yb) {   // Method 3 band product of u_i (uniform)
                const double2 y = yb[t0 + p];
                acc[p].re = fma(s_cur, y.x, acc[p].re);
                acc[p].im = fma(s_cur, y.y, acc[p].im);
            }
        }
        for (int z = 0; z < 8; ++z) {
            const double f = prefactor(sub, z, n_div, neighbours);
            const int k = corner_index(cell, z, n_c);
            const double2* rb = rvec + (int64_t)k * NP * n_rhs + rhs;
            const M2* db = d + ((int64_t)(cell * 8 + z) * NE) * ndiv3 + sub;
            cd dv[NV * NV];
#pragma unroll
            for (int e = 0; e < NV * NV; ++e) dv[e] = cscale(ld(db + (int64_t)e * ndiv3), f);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                // t[n1] = sum_{n2} r[n1][n2] conj(Dc[c][n2])
                cd t[NV];
#pragma unroll
                for (int n1 = 0; n1 < NV; ++n1) t[n1] = cmake(0.0, 0.0);
#pragma unroll
                for (int n2 = 0; n2 < NC; ++n2) {
                    const cd dc = ld(db + (int64_t)(NV * NV + c * NC + n2) * ndiv3);
#pragma unroll
                    for (int n1 = 0; n1 < NV; ++n1) {
                        const double2 r = rb[(int64_t)(n1 * NC + n2) * n_rhs];
                        cfma_jc(t[n1], cmake(r.x, r.y), dc);
                    }
                }
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int n1 = 0; n1 < NV; ++n1) cfma(acc[v * NC + c], dv[v * NV + n1], t[n1]);
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            st(out + t0 + p, acc[p]);
            if (MODE == PROLONG_LANCZOS) {
                const cd w = rounded(acc[p], out);
                const cd xv = ld(x + t0 + p);
                pw = fma(xv.re, w.re, pw);
                pw = fma(xv.im, w.im, pw);
                ww = fma(w.re, w.re, ww);
                ww = fma(w.im, w.im, ww);
            }
        }
    }
    if (MODE != PROLONG_LANCZOS) return;

    pw = wave_sum(pw);
    ww = wave_sum(ww);
    if (lane == 0) {
        ppart[((int64_t)cell * n_rhs + rhs) * 2] = pw;
        ppart[((int64_t)cell * n_rhs + rhs) * 2 + 1] = ww;
    }
}

// ---- main form: overlaps staged per corner in LDS ------------------------------------
//
// Block = 2 NR wavefronts (NR right-hand sides x 2 halves of c), so that two blocks
// share a compute unit and no wavefront idles.  The prefactors f(sub, z) of the cell
// sit in an LDS table; the diagonal, the -b_i psi_{i-1} term and the chain partials
// are applied after the corner loop, so psi_i is read once.
// wavefronts per SIMD the register budget allows: 3 (<= 168 VGPRs) where the
// FP32-storage variant fits without spills (FP32 vectors, up to three right-hand
// sides), else 2
template <class M2, class V2, int NV, int NC, int NR>
constexpr int prolong3_waves() {
    return (sizeof(M2) == 8 && sizeof(V2) == 8 && NV * NC <= 18 && !(NV == 3 && NC == 4) && NR < 4) ? 3 : 2;
}

// threads of a block: NPART wavefronts per right-hand side (each takes 1 / NPART of the
// conduction index c), at least 4 wavefronts (the extra ones only help staging)
template <int NR, int NPART>
constexpr int prolong3_threads() {
    return kWave * (NR * NPART < 4 ? 4 : NR * NPART);
}
// wavefronts per right-hand side: 3 for band pairs above 18 products with several
// right-hand sides (4v6c: 100 VGPRs instead of 132, two 9-wavefront blocks per compute
// unit; 100.4 against 105.6 us at 10^3 x 4^3 cells), else 2
template <int NV, int NC, int NR>
constexpr int prolong3_parts() {
    return (NV * NC > 18 && NR >= 2) ? 3 : 2;
}

// NDIV3 > 0: the subpoint count n_div^3 fixed at compile time (the LDS offsets of the
// corner loop become immediates); 0: taken from n_div
template <class M2, class V2, int NV, int NC, int MODE, int NR, int NDIV3, int NPART>
__global__ __launch_bounds__((prolong3_threads<NR, NPART>()), (prolong3_waves<M2, V2, NV, NC, NR>())) void k_prolong3(const M2* __restrict__ d, const double* __restrict__ delta,
                                                         const double2* __restrict__ rvec, const V2* __restrict__ x,
                                                         V2* __restrict__ out, double* __restrict__ ppart,
                                                         const ChainState* __restrict__ chain, int n_c, int n_div,
                                                         int neighbours, int64_t N,
                                                         const double2* __restrict__ yb) {
    constexpr int NP = NV * NC;
    constexpr int NE = NV * NV + NC * NC;
    constexpr int NCH = (NC + NPART - 1) / NPART;
    constexpr int NT = prolong3_threads<NR, NPART>();
    using U = Unit16<M2>;
    using Rw = typename U::t;
    constexpr int PFU = (NE * kWave / U::P + NT - 1) / NT;  // staged 16-byte units per thread (n_div^3 <= 64)
    extern __shared__ double2 lds2[];
    __shared__ double red[NR][NT / kWave][2];
    __shared__ double ftab[8 * kWave];
    const int ndiv3 = NDIV3 > 0 ? NDIV3 : n_div * n_div * n_div;
    const int blk = NE * ndiv3;                // entries of one (cell, corner) block
    const int blku = (blk + U::P - 1) / U::P;  // its 16-byte units (blocks start 16-byte aligned)
    using IT = typename Inner<M2>::t;   // precision of the per-(subpoint, corner) contractions
    using RS = typename std::conditional<sizeof(IT) == 4, float2, double2>::type;
    Rw* dbuf0 = reinterpret_cast<Rw*>(lds2);
    Rw* dbuf1 = dbuf0 + blku;
    RS* rs = reinterpret_cast<RS*>(lds2 + 2 * blku);   // r of the 8 corners, in IT
    const int cell = blockIdx.x;
    const int t = threadIdx.x;
    const int wave = t / kWave;
    const int lane = t % kWave;
    const int rhs = wave / NPART;
    const int h = wave % NPART;
    const bool active = lane < ndiv3 && rhs < NR;

    // coarse blocks r_{k~z} of the 8 corners (rs[z][p][r]), the overlaps of corner 0 and
    // the prefactor table.  The loads are unconditional (indices clamped) and all
    // issued before the first LDS write, so they are in flight together.
    constexpr int per = NP * NR;
    static_assert(8 * per <= 2 * NT, "coarse blocks: two entries per thread");
    const Rw* dcell = reinterpret_cast<const Rw*>(d + (int64_t)cell * 8 * blk);
    {
        double2 rv[2];
        Rw pf[PFU];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int i = min(t + q * NT, 8 * per - 1);
            const int zz = i / per;
            rv[q] = rvec[(int64_t)corner_index(cell, zz, n_c) * per + (i - zz * per)];
        }
#pragma unroll
        for (int q = 0; q < PFU; ++q) pf[q] = dcell[min(t + q * NT, blku - 1)];
        __builtin_amdgcn_sched_barrier(0);
        for (int i = t; i < 8 * ndiv3; i += NT)
            ftab[(i / ndiv3) * kWave + i % ndiv3] = prefactor(i % ndiv3, i / ndiv3, n_div, neighbours);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (t + q * NT < 8 * per) {
                RS v;
                v.x = (decltype(v.x))rv[q].x;
                v.y = (decltype(v.y))rv[q].y;
                rs[t + q * NT] = v;
            }
#pragma unroll
        for (int q = 0; q < PFU; ++q)
            if (t + q * NT < blku) dbuf0[t + q * NT] = pf[q];
    }

    cd acc[NV][NCH];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int q = 0; q < NCH; ++q) acc[v][q] = cmake(0.0, 0.0);

    for (int z = 0; z < 8; ++z) {
        Rw pf[PFU];
        if (z < 7) {
            const Rw* dn = dcell + (int64_t)(z + 1) * blku;
#pragma unroll
            for (int q = 0; q < PFU; ++q) pf[q] = dn[min(t + q * NT, blku - 1)];
        }
        __syncthreads();
        const M2* cur = reinterpret_cast<const M2*>((z & 1) ? dbuf1 : dbuf0);
        if (active && sizeof(IT) == 4) {
            // FP32 overlaps: tt[q][n1] = sum_{n2} r[n1][n2] conj(Dc[c(q)][n2]) and
            // Y[v][q] = f sum_{n1} Dv[v][n1] tt[q][n1] in FP32, Y added into the FP64 sum
            // over the corners
            const IT f = (IT)ftab[z * kWave + lane];
            const RS* rz = rs + z * per + rhs;
            cplx<IT> tt[NCH][NV];
#pragma unroll
            for (int q = 0; q < NCH; ++q)
#pragma unroll
                for (int n1 = 0; n1 < NV; ++n1) tt[q][n1] = czero<IT>();
#pragma unroll
            for (int n2 = 0; n2 < NC; ++n2) {
                __builtin_amdgcn_sched_barrier(0);
                cplx<IT> rc[NV];
#pragma unroll
                for (int n1 = 0; n1 < NV; ++n1) rc[n1] = cl<IT>(rz[(n1 * NC + n2) * NR]);
#pragma unroll
                for (int q = 0; q < NCH; ++q) {
                    const int c = h * NCH + q;
                    if (c >= NC) break;
                    const cplx<IT> dc = cl<IT>(cur[(NV * NV + c * NC + n2) * ndiv3 + lane]);
#pragma unroll
                    for (int n1 = 0; n1 < NV; ++n1) cmac_jc(tt[q][n1], rc[n1], dc);
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                cplx<IT> dvv[NV];
#pragma unroll
                for (int n1 = 0; n1 < NV; ++n1) dvv[n1] = cl<IT>(cur[(v * NV + n1) * ndiv3 + lane]);
#pragma unroll
                for (int q = 0; q < NCH; ++q) {
                    cplx<IT> Y = czero<IT>();
#pragma unroll
                    for (int n1 = 0; n1 < NV; ++n1) cmac(Y, dvv[n1], tt[q][n1]);
                    Y.re *= f;
                    Y.im *= f;
                    cadd_to(acc[v][q], Y);
                }
            }
        } else if (active) {
            const double f = ftab[z * kWave + lane];
            const RS* rz = rs + z * per + rhs;
            M2 dv[NV * NV];   // storage precision, widened at use
#pragma unroll
            for (int e = 0; e < NV * NV; ++e) dv[e] = cur[e * ndiv3 + lane];
            // tt[q][n1] = sum_{n2} r[n1][n2] conj(Dc[c(q)][n2]), one column of r at a time
            cd tt[NCH][NV];
#pragma unroll
            for (int q = 0; q < NCH; ++q)
#pragma unroll
                for (int n1 = 0; n1 < NV; ++n1) tt[q][n1] = cmake(0.0, 0.0);
#pragma unroll
            for (int n2 = 0; n2 < NC; ++n2) {
                __builtin_amdgcn_sched_barrier(0);
                cd rc[NV];
#pragma unroll
                for (int n1 = 0; n1 < NV; ++n1) {
                    const RS r = rz[(n1 * NC + n2) * NR];
                    rc[n1] = cmake(r.x, r.y);
                }
#pragma unroll
                for (int q = 0; q < NCH; ++q) {
                    const int c = h * NCH + q;
                    if (c >= NC) break;
                    const cd dc = cv(cur[(NV * NV + c * NC + n2) * ndiv3 + lane]);
#pragma unroll
                    for (int n1 = 0; n1 < NV; ++n1) cfma_jc(tt[q][n1], rc[n1], dc);
                }
            }
            // acc[v][q] += f sum_{n1} Dv[v][n1] tt[q][n1]
#pragma unroll
            for (int q = 0; q < NCH; ++q)
#pragma unroll
                for (int n1 = 0; n1 < NV; ++n1) tt[q][n1] = cscale(tt[q][n1], f);
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int n1 = 0; n1 < NV; ++n1) {
                    const cd dvv = cv(dv[v * NV + n1]);
#pragma unroll
                    for (int q = 0; q < NCH; ++q) cfma(acc[v][q], dvv, tt[q][n1]);
                }
        }
        if (z < 7) {
            Rw* nxt = (z & 1) ? dbuf0 : dbuf1;
#pragma unroll
            for (int q = 0; q < PFU; ++q) {
                const int i = t + q * NT;
                if (i < blku) nxt[i] = pf[q];
            }
        }
    }

    // w = delta psi_i + C^H r [- b_i psi_{i-1}] [+ s_i y], psi_i = s_i u_i in a chain,
    // element by element: the lanes' C^H r pass through LDS (the staging buffers are
    // free after the corner loop), one right-hand side at a time, so that the vector
    // slices of the cell are read and written in contiguous runs and no lane holds
    // its nine vector entries of every kind at once.
    double2* accs = reinterpret_cast<double2*>(lds2);   // fits: 2 (nv^2 + nc^2) >= nv nc
    const int nelem = ndiv3 * NP;
    const int64_t cbase = (int64_t)cell * nelem;
    double pwr[NR], wwr[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) pwr[r] = wwr[r] = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        __syncthreads();   // earlier readers of the buffers are done
        if (active && rhs == r) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int q = 0; q < NCH; ++q) {
                    const int c = h * NCH + q;
                    if (c < NC) accs[lane * NP + v * NC + c] = make_double2(acc[v][q].re, acc[v][q].im);
                }
        }
        __syncthreads();
        double s_cur = 1.0, c_prev = 0.0;
        if (MODE == PROLONG_LANCZOS) {
            s_cur = chain[r].s_cur;                       // psi_i = s_i u_i
            c_prev = chain[r].b_cur * chain[r].s_prev;    // b_i psi_{i-1} = b_i s_{i-1} u_{i-1}
        }
        const int64_t rbase = (int64_t)r * N + cbase;
        constexpr int EPT = 4;
        for (int e0 = 0; e0 < nelem; e0 += EPT * NT) {
            // all loads of the batch first, clamped (psi_{i-1} unconditionally: before
            // the second step its buffer holds no vector, and the select below drops it)
            V2 xr[EPT], pr[EPT];
            double dr[EPT];
            double2 yr[EPT];
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int e = min(e0 + t + u * NT, nelem - 1);
                xr[u] = x[rbase + e];
                dr[u] = delta[cbase + e];
                if (MODE == PROLONG_LANCZOS) pr[u] = out[rbase + e];
            }
            if (yb) {   // Method 3 band product of u_i (uniform branch)
#pragma unroll
                for (int u = 0; u < EPT; ++u) yr[u] = yb[rbase + min(e0 + t + u * NT, nelem - 1)];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int e = e0 + t + u * NT;
                if (e >= nelem) break;
                const cd xv = cv(xr[u]);
                const double dl = dr[u] * s_cur;
                const double2 a = accs[e];
                cd w = cmake(a.x, a.y);
                w.re = fma(dl, xv.re, w.re);
                w.im = fma(dl, xv.im, w.im);
                if (MODE == PROLONG_LANCZOS) {
                    const cd pv = cv(pr[u]);
                    const double pre = c_prev != 0.0 ? pv.re : 0.0;
                    const double pim = c_prev != 0.0 ? pv.im : 0.0;
                    w.re = fma(-c_prev, pre, w.re);
                    w.im = fma(-c_prev, pim, w.im);
                }
                if (yb) {
                    w.re = fma(s_cur, yr[u].x, w.re);
                    w.im = fma(s_cur, yr[u].y, w.im);
                }
                st(out + rbase + e, w);
                if (MODE == PROLONG_LANCZOS) {
                    const cd wr = rounded(w, out);
                    pwr[r] = fma(xv.re, wr.re, pwr[r]);
                    pwr[r] = fma(xv.im, wr.im, pwr[r]);
                    wwr[r] = fma(wr.re, wr.re, wwr[r]);
                    wwr[r] = fma(wr.im, wr.im, wwr[r]);
                }
            }
        }
    }
    if (MODE != PROLONG_LANCZOS) return;

    // per right-hand side: lanes, then wavefronts in a fixed order
    constexpr int NWV = NT / kWave;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const double pw = wave_sum(pwr[r]), ww = wave_sum(wwr[r]);
        if (lane == 0) {
            red[r][wave][0] = pw;
            red[r][wave][1] = ww;
        }
    }
    __syncthreads();
    if (t < 2 * NR) {
        const int r = t >> 1, comp = t & 1;
        double sum = 0.0;
        for (int w = 0; w < NWV; ++w) sum += red[r][w][comp];
        ppart[((int64_t)cell * NR + r) * 2 + comp] = sum;
    }
}

static size_t prolong3_lds(int ne, int ndiv3, int np, int n_rhs, size_t melem) {
    const size_t blku = ((size_t)ne * ndiv3 * melem + 15) / 16;
    return 2 * blku * 16 + (size_t)8 * np * n_rhs * sizeof(double2);
}

template <class M2, class V2, int NV, int NC, int NR>
static void prolong3_go(const Plan& p, int mode, const V2* xv, V2* ov, const ChainState* cs, size_t lds,
                        hipStream_t s) {
    const Geometry& g = p.g;
    const double2* rvec = reinterpret_cast<const double2*>(p.ws + p.L.rvec);
    double* ppart = reinterpret_cast<double*>(p.ws + p.L.ppart);
    const M2* d = reinterpret_cast<const M2*>(p.d);
    const double2* yb = p.m3_band ? p.m3_yb : nullptr;
    constexpr int NPART = prolong3_parts<NV, NC, NR>();
    dim3 grid(g.ncells), block(prolong3_threads<NR, NPART>());
    if (mode == PROLONG_PLAIN)
        hipLaunchKernelGGL((k_prolong3<M2, V2, NV, NC, PROLONG_PLAIN, NR, 0, NPART>), grid, block, lds, s, d, p.delta, rvec,
                           xv, ov, ppart, cs, g.n_c, g.n_div, g.neighbours, g.N, yb);
    else if (g.ndiv3 == 64)   // 4 divisions per axis, the chain's common case
        hipLaunchKernelGGL((k_prolong3<M2, V2, NV, NC, PROLONG_LANCZOS, NR, 64, NPART>), grid, block, lds, s, d, p.delta,
                           rvec, xv, ov, ppart, cs, g.n_c, g.n_div, g.neighbours, g.N, yb);
    else
        hipLaunchKernelGGL((k_prolong3<M2, V2, NV, NC, PROLONG_LANCZOS, NR, 0, NPART>), grid, block, lds, s, d, p.delta,
                           rvec, xv, ov, ppart, cs, g.n_c, g.n_div, g.neighbours, g.N, yb);
}

template <class M2, class V2, int NV, int NC>
hipError_t prolong_launch(const Plan& p, int mode, const void* x, void* out, int step, int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    const double2* rvec = reinterpret_cast<const double2*>(p.ws + p.L.rvec);
    double* ppart = reinterpret_cast<double*>(p.ws + p.L.ppart);
    const ChainState* cs = reinterpret_cast<const ChainState*>(p.ws + p.L.chain) + state_in(step) * kMaxRhs;
    const M2* d = reinterpret_cast<const M2*>(p.d);
    const V2* xv = reinterpret_cast<const V2*>(x);
    V2* ov = reinterpret_cast<V2*>(out);
    constexpr int NP = NV * NC, NE = NV * NV + NC * NC;
    const size_t lds = prolong3_lds(NE, g.ndiv3, NP, n_rhs, sizeof(M2));
    // staged form: whole 16-byte units per (cell, corner) block and an aligned base
    const bool units = ((size_t)NE * g.ndiv3 * sizeof(M2)) % 16 == 0 && ((uintptr_t)p.d & 15) == 0;
    // prefactor table, per-wavefront chain partials (at most 2 kMaxRhs wavefronts)
    const size_t static_lds = 8 * kWave * sizeof(double) + kMaxRhs * (3 * kMaxRhs) * 2 * sizeof(double);
    if (g.ndiv3 <= kWave && lds + static_lds <= lds_limit() && units) {
        switch (n_rhs) {
            case 1: prolong3_go<M2, V2, NV, NC, 1>(p, mode, xv, ov, cs, lds, s); break;
            case 2: prolong3_go<M2, V2, NV, NC, 2>(p, mode, xv, ov, cs, lds, s); break;
            case 3: prolong3_go<M2, V2, NV, NC, 3>(p, mode, xv, ov, cs, lds, s); break;
            default: prolong3_go<M2, V2, NV, NC, 4>(p, mode, xv, ov, cs, lds, s); break;
        }
    } else {
        dim3 grid(g.ncells), block(kWave * n_rhs);
        const double2* yb = p.m3_band ? p.m3_yb : nullptr;
        if (mode == PROLONG_PLAIN)
            hipLaunchKernelGGL((k_prolong1<M2, V2, NV, NC, PROLONG_PLAIN>), grid, block, 0, s, d, p.delta, rvec, xv,
                               ov, ppart, cs, g.n_c, g.n_div, g.neighbours, g.N, n_rhs, yb);
        else
            hipLaunchKernelGGL((k_prolong1<M2, V2, NV, NC, PROLONG_LANCZOS>), grid, block, 0, s, d, p.delta, rvec,
                               xv, ov, ppart, cs, g.n_c, g.n_div, g.neighbours, g.N, n_rhs, yb);
    }
    return hipGetLastError();
}

#define BSE_PROLONG_INST(M2, V2, A, B)                                                                             \
    template hipError_t prolong_launch<M2, V2, A, B>(const Plan&, int, const void*, void*, int, int, hipStream_t);
#define BSE_PROLONG_ALL(A, B)                 \
    BSE_PROLONG_INST(double2, double2, A, B)  \
    BSE_PROLONG_INST(float2, float2, A, B)    \
    BSE_PROLONG_INST(float2, double2, A, B)
BSE_BANDS(BSE_PROLONG_ALL)

// ---- any band counts: nv and nc at run time ---------------------------------------------
//
// For band pairs without a compiled form.  One block per coarse cell; one thread per vector
// entry (subpoint, v, c) of each right-hand side in turn forms
//   w = delta psi_i + sum_z f(sub, z) sum_{n1} Dv[v][n1] sum_{n2} r_z[n1][n2] conj(Dc[c][n2])
//       [- b_i psi_{i-1}] [+ s_i y]
// in FP64 and, in a chain, the block's partials of <u_i|w> and ||w||^2.
template <class M2, class V2, int MODE>
__global__ __launch_bounds__(256) void k_prolong_any(const M2* __restrict__ d, const double* __restrict__ delta,
                                                     const double2* __restrict__ rvec, const V2* __restrict__ x, V2* out,
                                                     double* __restrict__ ppart, const ChainState* __restrict__ chain,
                                                     int n_c, int n_div, int neighbours, int64_t N, int n_rhs,
                                                     const double2* __restrict__ yb, int nv, int nc) {
    __shared__ double sred[kBlock / kWave];
    const int np = nv * nc, ne = nv * nv + nc * nc;
    const int ndiv3 = n_div * n_div * n_div;
    const int cell = blockIdx.x;
    const int64_t kd0 = (int64_t)cell * ndiv3;
    for (int rhs = 0; rhs < n_rhs; ++rhs) {   // uniform
        double s_cur = 1.0, c_prev = 0.0;
        if (MODE == PROLONG_LANCZOS) {
            s_cur = chain[rhs].s_cur;                        // psi_i = s_i u_i
            c_prev = chain[rhs].b_cur * chain[rhs].s_prev;   // b_i psi_{i-1} = b_i s_{i-1} u_{i-1}
        }
        const bool use_prev = (MODE == PROLONG_LANCZOS) && c_prev != 0.0;
        double pw = 0.0, ww = 0.0;
        for (int o = threadIdx.x; o < ndiv3 * np; o += blockDim.x) {
            const int sub = o / np, pe = o % np, v = pe / nc, c = pe % nc;
            const int64_t kd = kd0 + sub;
            const int64_t t0 = (int64_t)rhs * N + kd * np + pe;
            const cd xv = ld(x + t0);
            cd acc = cscale(xv, delta[kd * np + pe] * s_cur);
            if (use_prev) {
                const cd pv = ld(out + t0);
                acc.re = fma(-c_prev, pv.re, acc.re);
                acc.im = fma(-c_prev, pv.im, acc.im);
            }
            if (yb) {   // Method 3 band product of u_i (uniform)
                const double2 y = yb[t0];
                acc.re = fma(s_cur, y.x, acc.re);
                acc.im = fma(s_cur, y.y, acc.im);
            }
            for (int z = 0; z < 8; ++z) {
                const double f = prefactor(sub, z, n_div, neighbours);
                if (f == 0.0) continue;
                const double2* rb = rvec + (int64_t)corner_index(cell, z, n_c) * np * n_rhs + rhs;
                const M2* db = d + (int64_t)(cell * 8 + z) * ne * ndiv3 + sub;
                cd y = cmake(0.0, 0.0);
                for (int n1 = 0; n1 < nv; ++n1) {
                    cd tt = cmake(0.0, 0.0);   // sum_n2 r[n1][n2] conj(Dc[c][n2])
                    for (int n2 = 0; n2 < nc; ++n2) {
                        const double2 r = rb[(int64_t)(n1 * nc + n2) * n_rhs];
                        cfma_jc(tt, cmake(r.x, r.y), ld(db + (int64_t)(nv * nv + c * nc + n2) * ndiv3));
                    }
                    cfma(y, ld(db + (int64_t)(v * nv + n1) * ndiv3), tt);
                }
                acc.re = fma(f, y.re, acc.re);
                acc.im = fma(f, y.im, acc.im);
            }
            st(out + t0, acc);
            if (MODE == PROLONG_LANCZOS) {
                const cd wr = rounded(acc, out);
                pw = fma(xv.re, wr.re, pw);
                pw = fma(xv.im, wr.im, pw);
                ww = fma(wr.re, wr.re, ww);
                ww = fma(wr.im, wr.im, ww);
            }
        }
        if (MODE == PROLONG_LANCZOS) {
            pw = block_sum(pw, sred);
            ww = block_sum(ww, sred);
            if (threadIdx.x == 0) {
                ppart[((int64_t)cell * n_rhs + rhs) * 2] = pw;
                ppart[((int64_t)cell * n_rhs + rhs) * 2 + 1] = ww;
            }
        }
    }
}

template <class M2, class V2>
hipError_t prolong_any_launch(const Plan& p, int mode, const void* x, void* out, int step, int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    const double2* rvec = reinterpret_cast<const double2*>(p.ws + p.L.rvec);
    double* ppart = reinterpret_cast<double*>(p.ws + p.L.ppart);
    const ChainState* cs = reinterpret_cast<const ChainState*>(p.ws + p.L.chain) + state_in(step) * kMaxRhs;
    const M2* d = reinterpret_cast<const M2*>(p.d);
    const double2* yb = p.m3_band ? p.m3_yb : nullptr;
    dim3 grid(g.ncells), block(kBlock);
    if (mode == PROLONG_PLAIN)
        hipLaunchKernelGGL((k_prolong_any<M2, V2, PROLONG_PLAIN>), grid, block, 0, s, d, p.delta, rvec,
                           reinterpret_cast<const V2*>(x), reinterpret_cast<V2*>(out), ppart, cs, g.n_c, g.n_div,
                           g.neighbours, g.N, n_rhs, yb, g.nv, g.nc);
    else
        hipLaunchKernelGGL((k_prolong_any<M2, V2, PROLONG_LANCZOS>), grid, block, 0, s, d, p.delta, rvec,
                           reinterpret_cast<const V2*>(x), reinterpret_cast<V2*>(out), ppart, cs, g.n_c, g.n_div,
                           g.neighbours, g.N, n_rhs, yb, g.nv, g.nc);
    return hipGetLastError();
}

template hipError_t prolong_any_launch<double2, double2>(const Plan&, int, const void*, void*, int, int, hipStream_t);
template hipError_t prolong_any_launch<float2, float2>(const Plan&, int, const void*, void*, int, int, hipStream_t);
template hipError_t prolong_any_launch<float2, double2>(const Plan&, int, const void*, void*, int, int, hipStream_t);

}  // namespace bse
