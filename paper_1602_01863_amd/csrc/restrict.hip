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

// Chain prefix of the general restricts (one block per (cell, right-hand side)).  At the
// chain start the coefficients are zeroed and u_1 = P; in an update
// u_{i+1} = w - a_i psi_i = w - a_i s_i u_i (Eq. bi) with a_i = s_i sum_cells <u_i|w>_cell
// (Eq. ai), summed from the prolong's per-cell partials by every block in the same fixed
// order; the block of cell 0 records a_i.  The block writes its slice of u to out and adds
// the slice's ||u||^2 (and ||P||^2 at the start) into uu and pp.
template <class V2, int MODE>
__device__ __forceinline__ void restrict_chain_prefix(const V2* x, const V2* __restrict__ psi,
                                                      const double2* __restrict__ P, V2* out,
                                                      const ChainState* __restrict__ cs,
                                                      StepScalars* __restrict__ pend,
                                                      const double* __restrict__ ppart, double* __restrict__ alpha,
                                                      double* __restrict__ beta, int lda, int ldb, int step, int cell,
                                                      int ncells, int rhs, int n_rhs, int64_t base, int nelem,
                                                      double* sred, double& uu, double& pp) {
    const int t = threadIdx.x;
    if (MODE == RESTRICT_INIT) {
        // chain coefficients start at zero
        const int64_t tid = (int64_t)(cell * n_rhs + rhs) * blockDim.x + t;
        const int64_t nth = (int64_t)ncells * n_rhs * blockDim.x;
        for (int64_t i = tid; i < (int64_t)n_rhs * lda; i += nth) alpha[i] = 0.0;
        for (int64_t i = tid; i < (int64_t)n_rhs * ldb; i += nth) beta[i] = 0.0;
    }
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

    if (MODE != RESTRICT_PLAIN) {
        restrict_chain_prefix<V2, MODE>(x, psi, P, out, cs, pend, ppart, alpha, beta, lda, ldb, step, cell, ncells, rhs,
                                        n_rhs, base, nelem, sred, uu, pp);
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

// ---- tiled form: overlaps from restrict tiles, the vector slice from LDS ------------------
//
// Same lane roles as k_restrict2 (lane = 8 z + 2 j + h, subpoint 4 s + j), but every
// value a lane needs comes from a restrict tile (one contiguous 1 KiB run per 16-byte
// load of the wavefront) or from the block's vector slice in LDS.  The tile carries
// f(sub, z) Dv already (f is real, so conj(f Dv) = f conj(Dv)) and each lane of a pair
// h = 0, 1 holds half of the valence block; the halves are exchanged with a DPP
// permutation.  The slice in LDS is padded with zeros to 4 S subpoints.

// tile entry k of lane l in (cell, s): see swz_shape()
template <class M2>
__global__ __launch_bounds__(256) void k_swizzle(const M2* __restrict__ d, M2* __restrict__ dsw, int ndiv3, int n_div,
                                                 int nv, int nc, int neighbours, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const SwzShape z = swz_shape(nv, nc, ndiv3, (int)sizeof(M2));
    const int ne = nv * nv + nc * nc;
    const int nunit = z.kp / z.unit;
    const int kin = (int)(idx % z.unit);
    int64_t rest = idx / z.unit;
    const int lane = (int)(rest % kWave);
    rest /= kWave;
    const int q = (int)(rest % nunit);
    rest /= nunit;
    const int s = (int)(rest % z.S);
    const int64_t cell = rest / z.S;
    const int k = q * z.unit + kin;
    const int corner = lane >> 3, j = (lane >> 1) & 3, h = lane & 1;
    const int sub = 4 * s + j;
    cd v = cmake(0.0, 0.0);
    if (sub < ndiv3 && k < z.kl) {
        const M2* blk = d + (cell * 8 + corner) * ne * ndiv3 + sub;
        if (k < z.ndv) {
            const int e = h * z.ndv + k;
            if (e < nv * nv) v = cscale(ld(blk + (int64_t)e * ndiv3), prefactor(sub, corner, n_div, neighbours));
        } else {
            const int kk = k - z.ndv;
            const int c = kk / z.nch, n2 = h * z.nch + kk % z.nch;
            if (n2 < nc) v = ld(blk + (int64_t)(nv * nv + c * nc + n2) * ndiv3);
        }
    }
    st(dsw + idx, v);
}

// Block = one cell and NR of the n_rhs right-hand sides (rhs0 .. rhs0 + NR - 1), so a
// tile load feeds NR products.  Blocks of one cell carry indices that are equal modulo
// 8 (same XCD, shared L2 copy of the tiles).  LDS: the vector slices xs[NR][4 S][NP]
// (storage precision), then the wavefront partials red[NW][NR][8][NP].
template <class M2, class V2, int NV, int NC, int MODE, int NR>
__global__ __launch_bounds__(256, (NR == 1 && sizeof(M2) == 8 && NV * NC <= 18) ? 3 : 2) void k_restrict3(
    const M2* __restrict__ dsw, const V2* x, const V2* __restrict__ psi, const double2* __restrict__ P, V2* out,
    double2* __restrict__ qpart, const ChainState* __restrict__ cs, StepScalars* __restrict__ pend,
    const double* __restrict__ ppart, double* __restrict__ rpart, double* __restrict__ alpha,
    double* __restrict__ beta, int lda, int ldb, int step, int n_c, int n_div, int64_t N, int n_rhs) {
    constexpr int NP = NV * NC;
    constexpr int NW = kBlock / kWave;
    constexpr int NDV = (NV * NV + 1) / 2;
    constexpr int NCH = (NC + 1) / 2;
    constexpr int KL = NDV + NC * NCH;
    using U = Unit16<M2>;
    using R = typename U::t;
    constexpr int NU = (KL + U::P - 1) / U::P;  // 16-byte loads per lane and tile
    using IT = typename Inner<M2>::t;           // precision of the per-subpoint contractions
    extern __shared__ double2 lds_raw[];
    __shared__ double sred[2 * NR][NW];
    const int ndiv3 = n_div * n_div * n_div;
    const int ncells = n_c * n_c * n_c;
    const int S = (ndiv3 + 3) / 4;
    const int xstride = 4 * S * NP;  // entries of one right-hand side's slice in LDS
    V2* xs = reinterpret_cast<V2*>(lds_raw);
    double2* red = lds_raw + ((size_t)NR * xstride * sizeof(V2) + 15) / 16;
    // XCD-aware block -> (cell, group of NR right-hand sides)
    const int ngrp = n_rhs / NR;
    const int bid = blockIdx.x;
    const int rest = bid / 8;
    const int grp = rest % ngrp;
    const int cell = (rest / ngrp) * 8 + bid % 8;
    if (cell >= ncells) return;  // padding blocks
    const int rhs0 = grp * NR;
    const int t = threadIdx.x;
    const int wave = t / kWave;
    const int lane = t % kWave;
    const int nelem = ndiv3 * NP;  // entries of the cell's slice of one vector
    const int64_t cbase = (int64_t)cell * nelem;
    const int ntot = NR * nelem;

    if (MODE == RESTRICT_INIT) {
        const int64_t tid = (int64_t)(cell * ngrp + grp) * blockDim.x + t;
        const int64_t nth = (int64_t)ncells * ngrp * blockDim.x;
        for (int64_t i = tid; i < (int64_t)n_rhs * lda; i += nth) alpha[i] = 0.0;
        for (int64_t i = tid; i < (int64_t)n_rhs * ldb; i += nth) beta[i] = 0.0;
    }
    const R* tile = reinterpret_cast<const R*>(dsw) + (int64_t)cell * S * NU * kWave + lane;
    // element-wise passes over (rhs, entry) run in batches of EPT entries per thread
    // whose loads are unconditional (clamped indices), so a batch is in flight at once;
    // the first batch is issued before anything waits (the chain scalars below)
    constexpr int EPT = 8;
    cd ua[EPT], pb[EPT];
    auto gidx = [&](int f) {
        const int r = NR == 1 ? 0 : f / nelem;   // one right-hand side: no division
        return (int64_t)(rhs0 + r) * N + cbase + (f - r * nelem);
    };
    auto load_batch = [&](int f0) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t g = gidx(min(f0 + t + e * kBlock, ntot - 1));
            if (MODE == RESTRICT_INIT) {
                ua[e] = ld(P + g);
            } else {
                ua[e] = ld(x + g);
                if (MODE == RESTRICT_UPDATE) pb[e] = ld(psi + g);
            }
        }
    };
    load_batch(0);
    __builtin_amdgcn_sched_barrier(0);

    double uu[NR], pp[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) uu[r] = pp[r] = 0.0;
    if (MODE == RESTRICT_PLAIN) {
        for (int f0 = 0; f0 < ntot; f0 += EPT * kBlock) {
            if (f0 > 0) load_batch(f0);
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int f = f0 + t + e * kBlock;
                if (f >= ntot) continue;
                const int r = NR == 1 ? 0 : f / nelem;
                st(xs + r * xstride + (f - r * nelem), ua[e]);
            }
        }
    } else {
        // init: u_1 = P.  update: u_{i+1} = w - a_i psi_i = w - a_i s_i u_i  (Eq. bi),
        // a_i = s_i sum_cells <u_i|w>_cell  (Eq. ai), from the prolong's per-cell partials
        double coef[NR];
        bool ok[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            coef[r] = 0.0;
            ok[r] = true;
        }
        if (MODE == RESTRICT_UPDATE) {
            double acc2[2 * NR];
#pragma unroll
            for (int q = 0; q < 2 * NR; ++q) acc2[q] = 0.0;
            for (int c0 = 0; c0 < ncells; c0 += 2 * kBlock) {
                double v[2][2 * NR];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int c = min(c0 + t + u * kBlock, ncells - 1);
#pragma unroll
                    for (int q = 0; q < 2 * NR; ++q) v[u][q] = ppart[((int64_t)c * n_rhs + rhs0) * 2 + q];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (c0 + t + u * kBlock < ncells)
#pragma unroll
                        for (int q = 0; q < 2 * NR; ++q) acc2[q] += v[u][q];
            }
#pragma unroll
            for (int q = 0; q < 2 * NR; ++q) {
                const double w = wave_sum(acc2[q]);
                if (lane == 0) sred[q][wave] = w;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                double pw = 0.0, ww = 0.0;
                for (int w = 0; w < NW; ++w) {
                    pw += sred[2 * r][w];
                    ww += sred[2 * r + 1][w];
                }
                const ChainState st0 = cs[rhs0 + r];
                const double a = st0.s_cur * pw;
                ok[r] = st0.active && isfinite(a) && isfinite(ww);
                coef[r] = ok[r] ? a * st0.s_cur : 0.0;
                if (cell == 0 && t == 0 && st0.active) {
                    StepScalars sc;
                    sc.a = a;
                    sc.ww = ww;
                    sc.ok = ok[r];
                    sc.pad[0] = sc.pad[1] = sc.pad[2] = 0;
                    pend[rhs0 + r] = sc;
                    if (ok[r]) alpha[(int64_t)(rhs0 + r) * lda + step] = a;
                }
            }
        }
        for (int f0 = 0; f0 < ntot; f0 += EPT * kBlock) {
            if (f0 > 0) load_batch(f0);
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int f = f0 + t + e * kBlock;
                if (f >= ntot) continue;
                const int r = NR == 1 ? 0 : f / nelem;
                const int i = f - r * nelem;
                double cr = 0.0;
                bool okr = true;
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    if (q == r) {
                        cr = coef[q];
                        okr = ok[q];
                    }
                cd u = cmake(0.0, 0.0);
                if (MODE == RESTRICT_INIT) {
                    u = ua[e];
                } else if (okr) {
                    u = ua[e];
                    u.re = fma(-cr, pb[e].re, u.re);
                    u.im = fma(-cr, pb[e].im, u.im);
                }
                st(out + (int64_t)(rhs0 + r) * N + cbase + i, u);
                st(xs + r * xstride + i, u);
                const cd ur = rounded(u, out);
                const double n2 = fma(ur.re, ur.re, ur.im * ur.im);
                const double p2 = (MODE == RESTRICT_INIT) ? fma(u.re, u.re, u.im * u.im) : 0.0;
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    if (q == r) {
                        uu[q] += n2;
                        pp[q] += p2;
                    }
            }
        }
    }
    for (int r = 0; r < NR; ++r)
        for (int i = nelem + t; i < xstride; i += blockDim.x) st(xs + r * xstride + i, cmake(0.0, 0.0));
    if (MODE != RESTRICT_PLAIN) {
        // ||u||^2 (and ||P||^2 at the start) of the cell's slices, for the collapse
        __syncthreads();  // the chain scalars above have been read from sred
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double a = wave_sum(uu[r]);
            const double b = wave_sum(pp[r]);
            if (lane == 0) {
                sred[2 * r][wave] = a;
                sred[2 * r + 1][wave] = b;
            }
        }
    }
    __syncthreads();
    if (MODE != RESTRICT_PLAIN && t < 2 * NR) {
        double v = 0.0;
        for (int w = 0; w < NW; ++w) v += sred[t][w];
        rpart[((int64_t)cell * n_rhs + rhs0) * 2 + t] = v;
    }

    const int j = (lane >> 1) & 3;
    const int h = lane & 1;
    const int z = lane >> 3;
    cd acc[NR][NV][NCH];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr)
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < NCH; ++q) acc[rr][v][q] = cmake(0.0, 0.0);
#pragma unroll 1
    for (int s = wave; s < S; s += NW) {
        R raw[NU];
        const R* tp = tile + (int64_t)s * NU * kWave;
#pragma unroll
        for (int u = 0; u < NU; ++u) raw[u] = tp[u * kWave];
        // keep the tile's loads together in front of the arithmetic (the scheduler
        // would otherwise issue them one by one, each with its own wait)
        __builtin_amdgcn_sched_barrier(0);
        auto entry = [&](int k) { return U::get(raw[k / U::P], k % U::P); };
        // the pair's halves of f Dv (lanes h = 0, 1 hold one half each), kept in
        // storage precision and widened at use
        M2 dv[NDV * 2];
#pragma unroll
        for (int k = 0; k < NDV; ++k) {
            const M2 mine = entry(k);
            const M2 other = swap_pair(mine);
            dv[k] = h ? other : mine;
            dv[NDV + k] = h ? mine : other;
        }
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            const V2* xrow = xs + rr * xstride + (4 * s + j) * NP;
            if constexpr (sizeof(IT) == 8) {
                // FP64 overlaps: for each v, T[q] = sum_c x[v][c] Dc[c][n2(q)] over this
                // lane's half of n2, then acc[n3][q] += conj(f Dv[v][n3]) T[q]
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    cd T[NCH];
#pragma unroll
                    for (int q = 0; q < NCH; ++q) T[q] = cmake(0.0, 0.0);
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const cd xc = cv(xrow[v * NC + c]);
#pragma unroll
                        for (int q = 0; q < NCH; ++q) cfma(T[q], xc, cv(entry(NDV + c * NCH + q)));
                    }
#pragma unroll
                    for (int n3 = 0; n3 < NV; ++n3) {
                        const cd dvv = cv(dv[v * NV + n3]);
#pragma unroll
                        for (int q = 0; q < NCH; ++q) cfma_cj(acc[rr][n3][q], dvv, T[q]);
                    }
                }
                continue;
            }
            // FP32 overlaps: T[v][q] = sum_c x[v][c] Dc[c][n2(q)] over this lane's half of
            // n2, then Y[n3][q] = sum_v conj(f Dv[v][n3]) T[v][q], both in FP32; Y is added
            // into the FP64 sum over the cell's subpoints
            cplx<IT> T[NV][NCH];
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int q = 0; q < NCH; ++q) T[v][q] = czero<IT>();
#pragma unroll
            for (int c = 0; c < NC; ++c) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const cplx<IT> xc = cl<IT>(xrow[v * NC + c]);
#pragma unroll
                    for (int q = 0; q < NCH; ++q) cmac(T[v][q], xc, cl<IT>(entry(NDV + c * NCH + q)));
                }
            }
#pragma unroll
            for (int n3 = 0; n3 < NV; ++n3)
#pragma unroll
                for (int q = 0; q < NCH; ++q) {
                    cplx<IT> Y = czero<IT>();
#pragma unroll
                    for (int v = 0; v < NV; ++v) cmac_cj(Y, cl<IT>(dv[v * NV + n3]), T[v][q]);
                    cadd_to(acc[rr][n3][q], Y);
                }
        }
    }
    // sum the 4 subpoint columns of each (corner, half), then the wavefronts
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < NCH; ++q) {
                acc[rr][v][q].re = xor_sum_j(acc[rr][v][q].re);
                acc[rr][v][q].im = xor_sum_j(acc[rr][v][q].im);
            }
    }
    if (j == 0) {
#pragma unroll
        for (int rr = 0; rr < NR; ++rr)
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int q = 0; q < NCH; ++q) {
                    const int n4 = h * NCH + q;
                    if (n4 < NC)
                        red[((wave * NR + rr) * 8 + z) * NP + v * NC + n4] =
                            make_double2(acc[rr][v][q].re, acc[rr][v][q].im);
                }
    }
    __syncthreads();
    for (int o = t; o < NR * 8 * NP; o += blockDim.x) {
        const int rr = o / (8 * NP), zp = o % (8 * NP);
        const int zz = zp / NP, p = zp % NP;
        double re = 0.0, im = 0.0;
        for (int w = 0; w < NW; ++w) {
            const double2 v = red[((w * NR + rr) * 8 + zz) * NP + p];
            re += v.x;
            im += v.y;
        }
        qpart[((int64_t)(cell * 8 + zz) * n_rhs + rhs0 + rr) * NP + p] = make_double2(re, im);
    }
}

static size_t restrict3_lds(const Geometry& g, int nr) {
    const size_t vb = vec_is_f32(g.dtype) ? sizeof(float2) : sizeof(double2);
    const size_t xs = (size_t)nr * 4 * ((g.ndiv3 + 3) / 4) * g.np * vb;
    return (xs + 15) / 16 * 16 + (size_t)(kBlock / kWave) * nr * 8 * g.np * sizeof(double2);
}

size_t restrict_tile_lds(const Geometry& g) {
    const size_t bytes = restrict3_lds(g, 1);
    // fixed limit (not the device's): the workspace layout must not depend on the device
    return bytes + 512 <= 64 * 1024 ? bytes : 0;   // 512: the block's static partials
}

hipError_t launch_swizzle(const Plan& p, hipStream_t s) {
    const Geometry& g = p.g;
    if (p.L.dsw_bytes == 0) return hipSuccess;
    const int eb = g.dtype == BSE_F64 ? (int)sizeof(double2) : (int)sizeof(float2);
    const int64_t total = (int64_t)(p.L.dsw_bytes / eb);
    dim3 grid((unsigned)((total + kBlock - 1) / kBlock)), block(kBlock);
    if (g.dtype == BSE_F64)
        hipLaunchKernelGGL(k_swizzle<double2>, grid, block, 0, s, reinterpret_cast<const double2*>(p.d),
                           reinterpret_cast<double2*>(p.ws + p.L.dsw), g.ndiv3, g.n_div, g.nv, g.nc, g.neighbours,
                           total);
    else
        hipLaunchKernelGGL(k_swizzle<float2>, grid, block, 0, s, reinterpret_cast<const float2*>(p.d),
                           reinterpret_cast<float2*>(p.ws + p.L.dsw), g.ndiv3, g.n_div, g.nv, g.nc, g.neighbours,
                           total);
    return hipGetLastError();
}

template <class M2, class V2, int NV, int NC, int NR>
static hipError_t restrict3_go(const Plan& p, int mode, const M2* dsw, const void* x, const void* w, const void* psi,
                               const double* P, void* out, int step, double* a, double* b, int lda, int ldb,
                               int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    double2* qpart = reinterpret_cast<double2*>(p.ws + p.L.qpart);
    const ChainState* cs = reinterpret_cast<const ChainState*>(p.ws + p.L.chain) + state_in(step) * kMaxRhs;
    StepScalars* pend = reinterpret_cast<StepScalars*>(p.ws + p.L.pend);
    const double* ppart = reinterpret_cast<const double*>(p.ws + p.L.ppart);
    double* rpart = reinterpret_cast<double*>(p.ws + p.L.rpart);
    const size_t lds = restrict3_lds(g, NR);
    if (lds + 512 > lds_limit() || n_rhs % NR != 0) return hipErrorInvalidConfiguration;
    const int groups = (g.ncells + 7) / 8;
    dim3 grid(groups * 8 * (n_rhs / NR)), block(kBlock);
    if (mode == RESTRICT_PLAIN)
        hipLaunchKernelGGL((k_restrict3<M2, V2, NV, NC, RESTRICT_PLAIN, NR>), grid, block, lds, s, dsw,
                           reinterpret_cast<const V2*>(x), nullptr, nullptr, nullptr, qpart, cs, pend, ppart, rpart,
                           nullptr, nullptr, 0, 0, 0, g.n_c, g.n_div, g.N, n_rhs);
    else if (mode == RESTRICT_UPDATE)
        hipLaunchKernelGGL((k_restrict3<M2, V2, NV, NC, RESTRICT_UPDATE, NR>), grid, block, lds, s, dsw,
                           reinterpret_cast<const V2*>(w), reinterpret_cast<const V2*>(psi), nullptr,
                           reinterpret_cast<V2*>(out), qpart, cs, pend, ppart, rpart, a, b, lda, ldb, step, g.n_c,
                           g.n_div, g.N, n_rhs);
    else
        hipLaunchKernelGGL((k_restrict3<M2, V2, NV, NC, RESTRICT_INIT, NR>), grid, block, lds, s, dsw, nullptr, nullptr,
                           reinterpret_cast<const double2*>(P), reinterpret_cast<V2*>(out), qpart, cs, pend, ppart,
                           rpart, a, b, lda, ldb, 0, g.n_c, g.n_div, g.N, n_rhs);
    return hipGetLastError();
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
    if (p.L.dsw_bytes > 0) {
        const M2* dsw = reinterpret_cast<const M2*>(p.ws + p.L.dsw);
        // right-hand sides per block: one (default), or all three when the plan asks
        // for it and the tiles fit
        if constexpr (NV * NC <= 18) {   // register budget of the three-rhs form
            if (n_rhs == 3 && p.restrict_group == 3 && restrict3_lds(g, 3) + 512 <= lds_limit())
                return restrict3_go<M2, V2, NV, NC, 3>(p, mode, dsw, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs,
                                                       s);
        }
        return restrict3_go<M2, V2, NV, NC, 1>(p, mode, dsw, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
    }
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

// ---- any band counts: nv and nc at run time ---------------------------------------------
//
// For band pairs without a compiled form.  One block per (cell, right-hand side): the chain
// prefix as above, then one thread per restricted entry (corner z, n3, n4) sums over the
// cell's subpoints
//   q[n3][n4] = sum_sub f(sub, z) sum_v conj(Dv[v][n3]) sum_c x[v][c] Dc[c][n4]
// in FP64, reading the overlaps and the slice from memory (the cache serves the repeats).
template <class M2, class V2, int MODE>
__global__ __launch_bounds__(256) void k_restrict_any(const M2* __restrict__ d, const V2* x, const V2* __restrict__ psi,
                                                      const double2* __restrict__ P, V2* out,
                                                      double2* __restrict__ qpart, const ChainState* __restrict__ cs,
                                                      StepScalars* __restrict__ pend, const double* __restrict__ ppart,
                                                      double* __restrict__ rpart, double* __restrict__ alpha,
                                                      double* __restrict__ beta, int lda, int ldb, int step, int n_c,
                                                      int n_div, int neighbours, int64_t N, int n_rhs, int nv, int nc) {
    __shared__ double sred[kBlock / kWave];
    const int np = nv * nc, ne = nv * nv + nc * nc;
    const int ndiv3 = n_div * n_div * n_div;
    const int ncells = n_c * n_c * n_c;
    const int cell = blockIdx.x / n_rhs, rhs = blockIdx.x % n_rhs;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)rhs * N + (int64_t)cell * ndiv3 * np;
    const int nelem = ndiv3 * np;
    double uu = 0.0, pp = 0.0;
    if (MODE != RESTRICT_PLAIN) {
        restrict_chain_prefix<V2, MODE>(x, psi, P, out, cs, pend, ppart, alpha, beta, lda, ldb, step, cell, ncells, rhs,
                                        n_rhs, base, nelem, sred, uu, pp);
        __syncthreads();  // the block's slice of u is visible to all its threads
    }
    const V2* src = (MODE == RESTRICT_PLAIN) ? x : out;
    for (int o = t; o < 8 * np; o += blockDim.x) {
        const int z = o / np, pe = o % np, n3 = pe / nc, n4 = pe % nc;
        const M2* db = d + (int64_t)(cell * 8 + z) * ne * ndiv3;
        double re = 0.0, im = 0.0;
        for (int sub = 0; sub < ndiv3; ++sub) {
            const double f = prefactor(sub, z, n_div, neighbours);
            if (f == 0.0) continue;
            const V2* xs = src + base + (int64_t)sub * np;
            cd y = cmake(0.0, 0.0);
            for (int v = 0; v < nv; ++v) {
                cd T = cmake(0.0, 0.0);
                for (int c = 0; c < nc; ++c) cfma(T, ld(xs + v * nc + c), ld(db + (int64_t)(nv * nv + c * nc + n4) * ndiv3 + sub));
                cfma_cj(y, ld(db + (int64_t)(v * nv + n3) * ndiv3 + sub), T);
            }
            re = fma(f, y.re, re);
            im = fma(f, y.im, im);
        }
        qpart[((int64_t)(cell * 8 + z) * n_rhs + rhs) * np + pe] = make_double2(re, im);
    }
    if (MODE == RESTRICT_PLAIN) return;
    uu = block_sum(uu, sred);
    pp = block_sum(pp, sred);
    if (t == 0) {
        rpart[((int64_t)cell * n_rhs + rhs) * 2] = uu;
        rpart[((int64_t)cell * n_rhs + rhs) * 2 + 1] = pp;
    }
}

template <class M2, class V2>
hipError_t restrict_any_launch(const Plan& p, int mode, const void* x, const void* w, const void* psi, const double* P,
                               void* out, int step, double* a, double* b, int lda, int ldb, int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    double2* qpart = reinterpret_cast<double2*>(p.ws + p.L.qpart);
    const ChainState* cs = reinterpret_cast<const ChainState*>(p.ws + p.L.chain) + state_in(step) * kMaxRhs;
    StepScalars* pend = reinterpret_cast<StepScalars*>(p.ws + p.L.pend);
    const double* ppart = reinterpret_cast<const double*>(p.ws + p.L.ppart);
    double* rpart = reinterpret_cast<double*>(p.ws + p.L.rpart);
    const M2* d = reinterpret_cast<const M2*>(p.d);
    dim3 grid(g.ncells * n_rhs), block(kBlock);
    if (mode == RESTRICT_PLAIN)
        hipLaunchKernelGGL((k_restrict_any<M2, V2, RESTRICT_PLAIN>), grid, block, 0, s, d,
                           reinterpret_cast<const V2*>(x), nullptr, nullptr, nullptr, qpart, cs, pend, ppart, rpart,
                           nullptr, nullptr, 0, 0, 0, g.n_c, g.n_div, g.neighbours, g.N, n_rhs, g.nv, g.nc);
    else if (mode == RESTRICT_UPDATE)
        hipLaunchKernelGGL((k_restrict_any<M2, V2, RESTRICT_UPDATE>), grid, block, 0, s, d,
                           reinterpret_cast<const V2*>(w), reinterpret_cast<const V2*>(psi), nullptr,
                           reinterpret_cast<V2*>(out), qpart, cs, pend, ppart, rpart, a, b, lda, ldb, step, g.n_c,
                           g.n_div, g.neighbours, g.N, n_rhs, g.nv, g.nc);
    else
        hipLaunchKernelGGL((k_restrict_any<M2, V2, RESTRICT_INIT>), grid, block, 0, s, d, nullptr, nullptr,
                           reinterpret_cast<const double2*>(P), reinterpret_cast<V2*>(out), qpart, cs, pend, ppart,
                           rpart, a, b, lda, ldb, 0, g.n_c, g.n_div, g.neighbours, g.N, n_rhs, g.nv, g.nc);
    return hipGetLastError();
}

template hipError_t restrict_any_launch<double2, double2>(const Plan&, int, const void*, const void*, const void*,
                                                          const double*, void*, int, double*, double*, int, int, int,
                                                          hipStream_t);
template hipError_t restrict_any_launch<float2, float2>(const Plan&, int, const void*, const void*, const void*,
                                                        const double*, void*, int, double*, double*, int, int, int,
                                                        hipStream_t);
template hipError_t restrict_any_launch<float2, double2>(const Plan&, int, const void*, const void*, const void*,
                                                         const double*, void*, int, double*, double*, int, int, int,
                                                         hipStream_t);

}  // namespace bse
