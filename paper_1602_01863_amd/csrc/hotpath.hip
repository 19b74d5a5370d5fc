// Hot path of the interpolated BSE matvec and of the Haydock step (gfx950).
//
// One step of the chain (Sec. 4, Eqs. matmul1-matmul3 inside Eqs. ai-ci).  The
// chain keeps unnormalised vectors u_j, psi_j = s_j u_j, with the scales in a
// small device-side state, so that b_{i+1} is the norm of the vector actually
// formed without an extra pass over memory:
//   k_gemv     r = K_c qbar                       (Eq. matmul2, corner sum collapsed)
//   k_prolong  w = delta psi_i + C^H r - b_i psi_{i-1} (Eq. matmul3, Eq. bse1
//              diagonal); FP64 partials of <u_i|w> and ||w||^2; the last block
//              forms a_i (Eq. ai)
//   k_restrict u_{i+1} = w - a_i psi_i and its ||.||^2 (Eq. bi), then the
//              per-(cell, corner) coarse vectors of u_{i+1} (Eq. matmul1); the last
//              block forms b_{i+1} and s_{i+1} = 1 / b_{i+1} (Eq. ci)
//   k_collapse qbar(k~) = s_{i+1} x sum of the 8 (cell, corner) vectors on k~
//
// Restrict and prolong run one block per coarse cell and one wavefront per
// right-hand side; lane = subpoint of the cell, so the overlap blocks (stored
// component-major per (cell, corner)) are read with unit stride.  Every sum is
// FP64; reductions use fixed trees, so results do not depend on scheduling.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

// ------------------------------------------------------------------------------------
// restrict (Eq. matmul1) with the Lanczos update (or the chain start) in front
// ------------------------------------------------------------------------------------
template <class M2, class V2, int NV, int NC, int MODE>
__global__ __launch_bounds__(256) void k_restrict(const M2* __restrict__ d, const V2* x,
                                                  const V2* __restrict__ psi, const double2* __restrict__ P,
                                                  V2* out, double2* __restrict__ qpart, ChainState* __restrict__ chain,
                                                  double* __restrict__ rpart, unsigned int* __restrict__ rcount,
                                                  double* __restrict__ alpha, double* __restrict__ beta, int lda,
                                                  int ldb, int step, double tol2, int n_c, int n_div,
                                                  int neighbours, int64_t N, int n_rhs) {
    constexpr int NP = NV * NC;
    constexpr int NE = NV * NV + NC * NC;
    __shared__ double red[kBlock / kWave];
    __shared__ int flag;
    const int ndiv3 = n_div * n_div * n_div;
    const int rhs = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x % kWave;
    const int cell = blockIdx.x;
    const int64_t kd0 = (int64_t)cell * ndiv3;
    const V2* src = x;
    double uu = 0.0, pp = 0.0;

    if (MODE == RESTRICT_INIT) {
        // chain coefficients start at zero
        const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const int64_t nth = (int64_t)gridDim.x * blockDim.x;
        for (int64_t i = tid; i < (int64_t)n_rhs * lda; i += nth) alpha[i] = 0.0;
        for (int64_t i = tid; i < (int64_t)n_rhs * ldb; i += nth) beta[i] = 0.0;
    }
    if (MODE != RESTRICT_PLAIN) {
        // init: u_1 = P.  update: u_{i+1} = w - a_i psi_i = w - a_i s_i u_i (Eq. bi)
        const double coef = (MODE == RESTRICT_UPDATE) ? chain[rhs].a * chain[rhs].s_cur : 0.0;
        for (int sub = lane; sub < ndiv3; sub += kWave) {
            const int64_t t0 = (int64_t)rhs * N + (kd0 + sub) * NP;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                cd u;
                if (MODE == RESTRICT_INIT) {
                    u = ld(P + t0 + p);
                    pp = fma(u.re, u.re, pp);
                    pp = fma(u.im, u.im, pp);
                } else {
                    u = ld(x + t0 + p);
                    const cd ps = ld(psi + t0 + p);
                    u.re = fma(-coef, ps.re, u.re);
                    u.im = fma(-coef, ps.im, u.im);
                }
                st(out + t0 + p, u);
                const cd ur = rounded(u, out);
                uu = fma(ur.re, ur.re, uu);
                uu = fma(ur.im, ur.im, uu);
            }
        }
        src = out;
    }

    // per corner: q^{z}_{cell}[n3][n4] = sum_sub f(sub,z) sum_{v c} conj(Dv[v][n3]) x[v][c] Dc[c][n4]
    for (int z = 0; z < 8; ++z) {
        cd acc[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[p] = cmake(0.0, 0.0);
        for (int sub = lane; sub < ndiv3; sub += kWave) {
            const double f = prefactor(sub, z, n_div, neighbours);
            const int64_t t0 = (int64_t)rhs * N + (kd0 + sub) * NP;
            const M2* db = d + ((int64_t)(cell * 8 + z) * NE) * ndiv3 + sub;
            cd xv[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) xv[p] = ld(src + t0 + p);
            cd dv[NV * NV];
#pragma unroll
            for (int e = 0; e < NV * NV; ++e) dv[e] = cscale(ld(db + (int64_t)e * ndiv3), f);
#pragma unroll
            for (int n4 = 0; n4 < NC; ++n4) {
                // column n4 of x Dc
                cd t[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) t[v] = cmake(0.0, 0.0);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const cd dc = ld(db + (int64_t)(NV * NV + c * NC + n4) * ndiv3);
#pragma unroll
                    for (int v = 0; v < NV; ++v) cfma(t[v], xv[v * NC + c], dc);
                }
#pragma unroll
                for (int n3 = 0; n3 < NV; ++n3)
#pragma unroll
                    for (int v = 0; v < NV; ++v) cfma_cj(acc[n3 * NC + n4], dv[v * NV + n3], t[v]);
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            acc[p].re = wave_sum(acc[p].re);
            acc[p].im = wave_sum(acc[p].im);
        }
        if (lane == 0) {
            double2* q = qpart + ((int64_t)(cell * 8 + z) * n_rhs + rhs) * NP;
#pragma unroll
            for (int p = 0; p < NP; ++p) q[p] = make_double2(acc[p].re, acc[p].im);
        }
    }
    if (MODE == RESTRICT_PLAIN) return;

    // ||u||^2 (and ||P||^2 at the start): block partials, last block closes the step
    uu = wave_sum(uu);
    pp = wave_sum(pp);
    if (lane == 0) {
        rpart[((int64_t)cell * n_rhs + rhs) * 2] = uu;
        rpart[((int64_t)cell * n_rhs + rhs) * 2 + 1] = pp;
    }
    const int ncells = gridDim.x;
    if (!last_block_arrival(rcount, (unsigned)ncells, &flag)) return;
    for (int r = 0; r < n_rhs; ++r) {
        double s2[2];
        for (int comp = 0; comp < 2; ++comp) {
            double v = 0.0;
            for (int c = threadIdx.x; c < ncells; c += blockDim.x) v += rpart[((int64_t)c * n_rhs + r) * 2 + comp];
            s2[comp] = block_sum(v, red);
        }
        if (threadIdx.x != 0) continue;
        ChainState st;
        if (MODE == RESTRICT_INIT) {
            st.pnorm2 = s2[1];
            st.a = 0.0;
            st.b_cur = 0.0;
            st.s_prev = 0.0;
            st.ww = 0.0;
            st.steps = 0;
            st.pad = 0;
            if (s2[0] > 0.0 && isfinite(s2[0])) {
                st.active = 1;
                st.s_cur = 1.0 / sqrt(s2[0]);
                st.status = BSE_OK;
            } else {
                st.active = 0;
                st.s_cur = 0.0;
                st.status = (s2[0] == 0.0) ? BSE_INFO_ZERO_START : BSE_ERR_NONFINITE;
            }
        } else {
            st = chain[r];
            st.s_prev = st.s_cur;
            st.s_cur = 0.0;
            st.b_cur = 0.0;
            if (st.active) {
                const double b2 = s2[0];
                if (!isfinite(b2)) {
                    st.status = BSE_ERR_NONFINITE;
                    st.active = 0;
                } else if (b2 <= tol2 * st.ww) {
                    st.status = BSE_INFO_INVARIANT_SUBSPACE;  // b_{i+1} = 0: exact chain end
                    st.active = 0;
                } else {
                    const double bb = sqrt(b2);
                    beta[(int64_t)r * ldb + step + 1] = bb;
                    st.b_cur = bb;
                    st.s_cur = 1.0 / bb;
                }
            }
        }
        chain[r] = st;
    }
}

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
// coarse product r = K_c qbar (Eq. matmul2).  K_c is Hermitian and row-major, so
// r[i] = sum_j conj(K[j][i]) qbar[j]: lanes own consecutive i and every load of a
// column strip is contiguous.  Block = 4 wavefronts on the same rows and
// interleaved columns of one column chunk; FP64 accumulation; split partials are
// summed in a fixed order by the last block of each row block.
// ------------------------------------------------------------------------------------
template <class M2>
struct GemvTraits;
template <>
struct GemvTraits<float2> {
    static constexpr int RPT = 4;  // rows per lane: two 16-byte loads
};
template <>
struct GemvTraits<double2> {
    static constexpr int RPT = 2;
};

__device__ __forceinline__ void load_rows(const float2* p, cd* v, bool full, int valid) {
    if (full) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        const float4 b = *reinterpret_cast<const float4*>(p + 2);
        v[0] = cd{a.x, a.y};
        v[1] = cd{a.z, a.w};
        v[2] = cd{b.x, b.y};
        v[3] = cd{b.z, b.w};
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = (i < valid) ? ld(p + i) : cmake(0.0, 0.0);
    }
}
__device__ __forceinline__ void load_rows(const double2* p, cd* v, bool full, int valid) {
    if (full) {
        v[0] = ld(p);
        v[1] = ld(p + 1);
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i) v[i] = (i < valid) ? ld(p + i) : cmake(0.0, 0.0);
    }
}

template <class M2, int NRHS, bool VEC>
__global__ __launch_bounds__(256) void k_gemv(const M2* __restrict__ K, const double2* __restrict__ qbar,
                                              double2* __restrict__ part, double2* __restrict__ rout,
                                              unsigned int* __restrict__ counters, int Nc, int col_chunk,
                                              int n_split, int n_rowblk) {
    constexpr int RPT = GemvTraits<M2>::RPT;
    constexpr int RW = kWave * RPT;  // rows per block
    extern __shared__ double2 smem[];
    __shared__ int flag;
    const int rb = blockIdx.x % n_rowblk;
    const int s = blockIdx.x / n_rowblk;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int c_begin = s * col_chunk;
    const int c_end = min(Nc, c_begin + col_chunk);
    const int ncol = c_end - c_begin;

    for (int i = threadIdx.x; i < ncol * NRHS; i += blockDim.x) smem[i] = qbar[(int64_t)c_begin * NRHS + i];
    __syncthreads();

    const int row0 = rb * RW + lane * RPT;
    const int valid = min(RPT, Nc - row0);
    const bool full = VEC && valid == RPT;
    cd acc[RPT][NRHS];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc[i][r] = cmake(0.0, 0.0);

    if (valid > 0) {
        const M2* kp = K + (int64_t)c_begin * Nc + row0;
        int c = wave;
        for (; c + 12 < ncol; c += 16) {
            cd kv[4][RPT];
#pragma unroll
            for (int u = 0; u < 4; ++u) load_rows(kp + (int64_t)(c + 4 * u) * Nc, kv[u], full, valid);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int r = 0; r < NRHS; ++r) {
                    const double2 q = smem[(c + 4 * u) * NRHS + r];
                    const cd qc = cmake(q.x, q.y);
#pragma unroll
                    for (int i = 0; i < RPT; ++i) cfma_cj(acc[i][r], kv[u][i], qc);
                }
            }
        }
        for (; c < ncol; c += 4) {
            cd kv[RPT];
            load_rows(kp + (int64_t)c * Nc, kv, full, valid);
#pragma unroll
            for (int r = 0; r < NRHS; ++r) {
                const double2 q = smem[c * NRHS + r];
                const cd qc = cmake(q.x, q.y);
#pragma unroll
                for (int i = 0; i < RPT; ++i) cfma_cj(acc[i][r], kv[i], qc);
            }
        }
    }

    // cross-wave sum in fixed order (waves 1..3 into LDS, wave 0 adds)
    __syncthreads();
    double2* red = smem;  // reuse: 3 * 64 * RPT * NRHS entries
    if (wave > 0) {
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int r = 0; r < NRHS; ++r)
                red[(((wave - 1) * kWave + lane) * RPT + i) * NRHS + r] = make_double2(acc[i][r].re, acc[i][r].im);
    }
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < 4; ++w) {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int r = 0; r < NRHS; ++r) {
                    const double2 v = red[(((w - 1) * kWave + lane) * RPT + i) * NRHS + r];
                    acc[i][r].re += v.x;
                    acc[i][r].im += v.y;
                }
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i)
            if (i < valid)
#pragma unroll
                for (int r = 0; r < NRHS; ++r)
                    part[((int64_t)s * Nc + row0 + i) * NRHS + r] = make_double2(acc[i][r].re, acc[i][r].im);
    }

    if (last_block_arrival(counters + rb, (unsigned)n_split, &flag)) {
        const int rbase = rb * RW;
        const int nrow = min(RW, Nc - rbase);
        for (int o = threadIdx.x; o < nrow * NRHS; o += blockDim.x) {
            double re = 0.0, im = 0.0;
            for (int t = 0; t < n_split; ++t) {
                const double2 v = part[((int64_t)t * Nc + rbase) * NRHS + o];
                re += v.x;
                im += v.y;
            }
            rout[(int64_t)rbase * NRHS + o] = make_double2(re, im);
        }
    }
}

// ------------------------------------------------------------------------------------
// prolong (Eq. matmul3) + diagonal (Eq. bse1); Lanczos mode scales the stored
// vectors, subtracts b_i psi_{i-1} and forms a_i in the last block.
// ------------------------------------------------------------------------------------
template <class M2, class V2, int NV, int NC, int MODE>
__global__ __launch_bounds__(256) void k_prolong(const M2* __restrict__ d, const double* __restrict__ delta,
                                                 const double2* __restrict__ rvec, const V2* __restrict__ x,
                                                 V2* __restrict__ out, double* __restrict__ ppart,
                                                 unsigned int* __restrict__ pcount, ChainState* __restrict__ chain,
                                                 double* __restrict__ alpha, int lda, int step, int n_c, int n_div,
                                                 int neighbours, int64_t N, int n_rhs) {
    constexpr int NP = NV * NC;
    constexpr int NE = NV * NV + NC * NC;
    __shared__ double red[kBlock / kWave];
    __shared__ int flag;
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
    const int ncells = gridDim.x;
    if (!last_block_arrival(pcount, (unsigned)ncells, &flag)) return;
    for (int r = 0; r < n_rhs; ++r) {
        double s2[2];
        for (int comp = 0; comp < 2; ++comp) {
            double v = 0.0;
            for (int c = threadIdx.x; c < ncells; c += blockDim.x) v += ppart[((int64_t)c * n_rhs + r) * 2 + comp];
            s2[comp] = block_sum(v, red);
        }
        if (threadIdx.x != 0) continue;
        ChainState st = chain[r];
        st.a = 0.0;
        st.ww = 0.0;
        if (st.active) {
            const double a = st.s_cur * s2[0];   // a_i = Re <psi_i | w>  (Eq. ai)
            if (!isfinite(a) || !isfinite(s2[1])) {
                st.status = BSE_ERR_NONFINITE;
                st.active = 0;
                st.s_cur = 0.0;
            } else {
                alpha[(int64_t)r * lda + step] = a;
                st.a = a;
                st.ww = s2[1];
                st.steps = step + 1;
            }
        }
        chain[r] = st;
    }
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
// dispatch
// ------------------------------------------------------------------------------------
#define BSE_BANDS(X) X(1, 1) X(1, 2) X(2, 2) X(2, 3) X(3, 3) X(3, 4) X(3, 6) X(4, 6)

bool supported_bands(int nv, int nc) {
#define BSE_CHECK(a, b) \
    if (nv == a && nc == b) return true;
    BSE_BANDS(BSE_CHECK)
#undef BSE_CHECK
    return false;
}

template <class M2, class V2, int NV, int NC>
static hipError_t restrict_t(const Plan& p, int mode, const void* x, const void* w, const void* psi,
                             const double* P, void* out, int step, double* a, double* b, int lda, int ldb,
                             int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    double2* qpart = reinterpret_cast<double2*>(p.ws + p.L.qpart);
    ChainState* chain = reinterpret_cast<ChainState*>(p.ws + p.L.chain);
    double* rpart = reinterpret_cast<double*>(p.ws + p.L.rpart);
    unsigned int* rcount = reinterpret_cast<unsigned int*>(p.ws + p.L.rcount);
    const M2* d = reinterpret_cast<const M2*>(p.d);
    // breakdown: b_{i+1} <= tol ||w||
    const double tol = (sizeof(V2) == sizeof(float2)) ? 1e-6 : 1e-12;
    dim3 grid(g.ncells), block(kWave * n_rhs);
    if (mode == RESTRICT_PLAIN)
        hipLaunchKernelGGL((k_restrict<M2, V2, NV, NC, RESTRICT_PLAIN>), grid, block, 0, s, d,
                           reinterpret_cast<const V2*>(x), nullptr, nullptr, nullptr, qpart, chain, rpart, rcount,
                           nullptr, nullptr, 0, 0, 0, 0.0, g.n_c, g.n_div, g.neighbours, g.N, n_rhs);
    else if (mode == RESTRICT_UPDATE)
        hipLaunchKernelGGL((k_restrict<M2, V2, NV, NC, RESTRICT_UPDATE>), grid, block, 0, s, d,
                           reinterpret_cast<const V2*>(w), reinterpret_cast<const V2*>(psi), nullptr,
                           reinterpret_cast<V2*>(out), qpart, chain, rpart, rcount, a, b, lda, ldb, step, tol * tol,
                           g.n_c, g.n_div, g.neighbours, g.N, n_rhs);
    else
        hipLaunchKernelGGL((k_restrict<M2, V2, NV, NC, RESTRICT_INIT>), grid, block, 0, s, d, nullptr, nullptr,
                           reinterpret_cast<const double2*>(P), reinterpret_cast<V2*>(out), qpart, chain, rpart,
                           rcount, a, b, lda, ldb, 0, tol * tol, g.n_c, g.n_div, g.neighbours, g.N, n_rhs);
    return hipGetLastError();
}

template <class M2, class V2, int NV, int NC>
static hipError_t prolong_t(const Plan& p, int mode, const void* x, void* out, int step, double* a, int lda,
                            int n_rhs, hipStream_t s) {
    const Geometry& g = p.g;
    const double2* rvec = reinterpret_cast<const double2*>(p.ws + p.L.rvec);
    double* ppart = reinterpret_cast<double*>(p.ws + p.L.ppart);
    unsigned int* pcount = reinterpret_cast<unsigned int*>(p.ws + p.L.pcount);
    ChainState* chain = reinterpret_cast<ChainState*>(p.ws + p.L.chain);
    const M2* d = reinterpret_cast<const M2*>(p.d);
    dim3 grid(g.ncells), block(kWave * n_rhs);
    if (mode == PROLONG_PLAIN)
        hipLaunchKernelGGL((k_prolong<M2, V2, NV, NC, PROLONG_PLAIN>), grid, block, 0, s, d, p.delta, rvec,
                           reinterpret_cast<const V2*>(x), reinterpret_cast<V2*>(out), ppart, pcount, chain,
                           nullptr, 0, 0, g.n_c, g.n_div, g.neighbours, g.N, n_rhs);
    else
        hipLaunchKernelGGL((k_prolong<M2, V2, NV, NC, PROLONG_LANCZOS>), grid, block, 0, s, d, p.delta, rvec,
                           reinterpret_cast<const V2*>(x), reinterpret_cast<V2*>(out), ppart, pcount, chain, a, lda,
                           step, g.n_c, g.n_div, g.neighbours, g.N, n_rhs);
    return hipGetLastError();
}

template <int NV, int NC>
static hipError_t restrict_dt(const Plan& p, int mode, const void* x, const void* w, const void* psi,
                              const double* P, void* out, int step, double* a, double* b, int lda, int ldb,
                              int n_rhs, hipStream_t s) {
    switch (p.g.dtype) {
        case BSE_F64:
            return restrict_t<double2, double2, NV, NC>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
        case BSE_F32:
            return restrict_t<float2, float2, NV, NC>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
        default:
            return restrict_t<float2, double2, NV, NC>(p, mode, x, w, psi, P, out, step, a, b, lda, ldb, n_rhs, s);
    }
}

template <int NV, int NC>
static hipError_t prolong_dt(const Plan& p, int mode, const void* x, void* out, int step, double* a, int lda,
                             int n_rhs, hipStream_t s) {
    switch (p.g.dtype) {
        case BSE_F64: return prolong_t<double2, double2, NV, NC>(p, mode, x, out, step, a, lda, n_rhs, s);
        case BSE_F32: return prolong_t<float2, float2, NV, NC>(p, mode, x, out, step, a, lda, n_rhs, s);
        default: return prolong_t<float2, double2, NV, NC>(p, mode, x, out, step, a, lda, n_rhs, s);
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

static void gemv_shape(const Plan& p, int rpt, int* n_rowblk, int* n_split, int* col_chunk) {
    const int Nc = (int)p.g.Nc;
    const int rw = kWave * rpt;
    *n_rowblk = (Nc + rw - 1) / rw;
    int ns = p.n_split;
    if (ns <= 0) ns = (1024 + *n_rowblk - 1) / *n_rowblk;
    ns = std::max(1, std::min(ns, kMaxSplit));
    ns = std::min(ns, std::max(1, Nc / 16));
    int chunk = (Nc + ns - 1) / ns;
    chunk = (chunk + 15) / 16 * 16;
    *col_chunk = chunk;
    *n_split = (Nc + chunk - 1) / chunk;
}

template <class M2, int NRHS>
static hipError_t gemv_t(Plan& p, hipStream_t s) {
    const Geometry& g = p.g;
    constexpr int RPT = GemvTraits<M2>::RPT;
    int n_rowblk, n_split, chunk;
    gemv_shape(p, RPT, &n_rowblk, &n_split, &chunk);
    const size_t lds = std::max((size_t)chunk * NRHS, (size_t)3 * kWave * RPT * NRHS) * sizeof(double2);
    const bool vec = (sizeof(M2) == sizeof(double2)) || (g.Nc % 2 == 0);
    const M2* K = reinterpret_cast<const M2*>(p.Kc);
    const double2* qbar = reinterpret_cast<const double2*>(p.ws + p.L.qbar);
    double2* part = reinterpret_cast<double2*>(p.ws + p.L.gpart);
    double2* rvec = reinterpret_cast<double2*>(p.ws + p.L.rvec);
    unsigned int* cnt = reinterpret_cast<unsigned int*>(p.ws + p.L.gcount);
    dim3 grid(n_rowblk * n_split), block(kBlock);
    if (vec)
        hipLaunchKernelGGL((k_gemv<M2, NRHS, true>), grid, block, lds, s, K, qbar, part, rvec, cnt, (int)g.Nc,
                           chunk, n_split, n_rowblk);
    else
        hipLaunchKernelGGL((k_gemv<M2, NRHS, false>), grid, block, lds, s, K, qbar, part, rvec, cnt, (int)g.Nc,
                           chunk, n_split, n_rowblk);
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
