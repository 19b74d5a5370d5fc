// Once-per-Hamiltonian setup kernels: overlaps (Eq. completeness), transition
// energies (Eq. bse1 diagonal) and the model coarse kernel (Eqs. bse2-bse3b).
// All arithmetic in FP64; results are rounded to the storage precision on store.

#include <hip/hip_runtime.h>
#include <math.h>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

// d[((cell*8 + z)*NE + e)*ndiv3 + sub] = <u_{n' k~z} | u_{n kd}>
template <class M2>
__global__ __launch_bounds__(256) void k_overlaps(const double2* __restrict__ vc, const double2* __restrict__ vd,
                                                  M2* __restrict__ dout, int n_c, int n_div, int nv, int nc,
                                                  int n_orb, int64_t total) {
    const int ndiv3 = n_div * n_div * n_div;
    const int ne = nv * nv + nc * nc;
    const int nb = nv + nc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int sub = (int)(i % ndiv3);
        int64_t rest = i / ndiv3;
        const int e = (int)(rest % ne);
        rest /= ne;
        const int z = (int)(rest % 8);
        const int cell = (int)(rest / 8);
        const int64_t kd = (int64_t)cell * ndiv3 + sub;
        const int kc = corner_index(cell, z, n_c);
        int n, nprime;
        if (e < nv * nv) {
            n = e / nv;
            nprime = e % nv;
        } else {
            const int e2 = e - nv * nv;
            n = nv + e2 / nc;
            nprime = nv + e2 % nc;
        }
        const double2* a = vc + ((int64_t)kc * nb + nprime) * n_orb;
        const double2* b = vd + (kd * nb + n) * n_orb;
        cd s = cmake(0.0, 0.0);
        for (int o = 0; o < n_orb; ++o) cfma_cj(s, cmake(a[o].x, a[o].y), cmake(b[o].x, b[o].y));
        st(dout + i, s);
    }
}

__global__ __launch_bounds__(256) void k_transition_energies(const double* __restrict__ eps, double* __restrict__ out,
                                                             int nv, int nc, int64_t N) {
    const int np = nv * nc, nb = nv + nc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t kd = i / np;
        const int p = (int)(i % np);
        const int v = p / nc, c = p % nc;
        out[i] = eps[kd * nb + nv + c] - eps[kd * nb + v];
    }
}

// ---- model coarse kernel -----------------------------------------------------------------
constexpr int kMaxOrb = 16;
constexpr int kMaxBands = 16;
constexpr int kMaxG = 33;     // |G|^2 <= 4
constexpr int kMaxPair = 32;  // nv * nc
constexpr int kMaxOut = 4;    // outputs per thread: NP^2 <= 1024

__device__ __forceinline__ int fold_int(int d, int n) {
    const int h = n / 2;
    int r = (d + h) % n;
    if (r < 0) r += n;
    return r - h;
}

// the n-th integer vector with |G|^2 <= g2max, enumerated x-major over [-r, r]^3
__device__ __forceinline__ int enumerate_g(int g2max, int* gx, int* gy, int* gz) {
    int r = 0;
    while ((r + 1) * (r + 1) <= g2max) ++r;
    int n = 0;
    for (int x = -r; x <= r; ++x)
        for (int y = -r; y <= r; ++y)
            for (int z = -r; z <= r; ++z)
                if (x * x + y * y + z * z <= g2max && n < kMaxG) {
                    gx[n] = x;
                    gy[n] = y;
                    gz[n] = z;
                    ++n;
                }
    return n;
}

// COEF = false: the coarse kernel K_c.  COEF = true: the coefficient a_c of the
// divergent part of Eq. (diverg) for this model, i.e. the G = 0 direct term with W
// replaced by 1 / (pi eps_inf) (W(q) = s(q) / (pi eps_inf), s = 1 / (|q|^2 + kappa^2)),
// so that the G = 0 direct term of K_c is a_c s(q); no exchange.
template <class M2, bool COEF>
__global__ __launch_bounds__(256) void k_coarse_kernel(const double2* __restrict__ vecs, const double* __restrict__ tau,
                                                       M2* __restrict__ K, int n_c, int n_div, int nv, int nc, int n_orb,
                                                       double eps_inf, double lam, double scale, int g2max, int q0q) {
    __shared__ double2 A[kMaxBands * kMaxOrb], B[kMaxBands * kMaxOrb];
    __shared__ double tauS[kMaxOrb * 3];
    __shared__ int gx[kMaxG], gy[kMaxG], gz[kMaxG];
    __shared__ int ng_s;
    __shared__ double2 mx[2][kMaxG * kMaxPair];   // exchange densities [g][c][v] at k and kp
    __shared__ double2 ph[kMaxOrb];
    __shared__ double2 mcc[kMaxBands * kMaxBands], mvv[kMaxBands * kMaxBands];
    __shared__ double red[kBlock / kWave];
    double2* mxa = mx[0];
    double2* mxb = mx[1];
    double2* blk = mx[0];   // diagonal block, after the exchange sums are done

    const int nk = n_c * n_c * n_c;
    const int np = nv * nc, nb = nv + nc;
    const int64_t Nc = (int64_t)nk * np;
    // block -> (k, kp) with k <= kp, row-major over the upper triangle
    const int64_t idx = blockIdx.x;
    const double tn = 2.0 * nk + 1.0;
    int k = (int)floor((tn - sqrt(tn * tn - 8.0 * (double)idx)) / 2.0);
    auto row_start = [nk](int64_t r) { return r * nk - r * (r - 1) / 2; };
    while (k > 0 && row_start(k) > idx) --k;
    while (row_start(k + 1) <= idx) ++k;
    const int kp = k + (int)(idx - row_start(k));

    for (int i = threadIdx.x; i < nb * n_orb; i += blockDim.x) {
        A[i] = vecs[(int64_t)k * nb * n_orb + i];
        B[i] = vecs[(int64_t)kp * nb * n_orb + i];
    }
    for (int i = threadIdx.x; i < n_orb * 3; i += blockDim.x) tauS[i] = tau[i];
    if (threadIdx.x == 0) ng_s = enumerate_g(g2max, gx, gy, gz);
    __syncthreads();
    const int ng = ng_s;

    // q = k - kp folded into [-1/2, 1/2) per axis
    const int k1 = k / (n_c * n_c), k2 = (k / n_c) % n_c, k3 = k % n_c;
    const int p1 = kp / (n_c * n_c), p2 = (kp / n_c) % n_c, p3 = kp % n_c;
    const double q[3] = {(double)fold_int(k1 - p1, n_c) / n_c, (double)fold_int(k2 - p2, n_c) / n_c,
                         (double)fold_int(k3 - p3, n_c) / n_c};

    // W(q -> 0) averaged over the dense mini-cell, midpoint rule (diagonal blocks only)
    double wq0 = 0.0;
    if (!COEF && k == kp) {
        const int nq3 = q0q * q0q * q0q;
        const double h = 1.0 / ((double)n_c * n_div);
        double s = 0.0;
        for (int i = threadIdx.x; i < nq3; i += blockDim.x) {
            const int a = i / (q0q * q0q), b = (i / q0q) % q0q, c = i % q0q;
            const double x = ((a + 0.5) / q0q - 0.5) * h, y = ((b + 0.5) / q0q - 0.5) * h,
                         zz = ((c + 0.5) / q0q - 0.5) * h;
            const double Q2 = 4.0 * M_PI * M_PI * (x * x + y * y + zz * zz);
            s += 4.0 * M_PI / (eps_inf * Q2 + lam * lam);
        }
        wq0 = block_sum(s, red) / (double)nq3;
    }

    // exchange densities M_cv(k,k;G) and M_c'v'(kp,kp;G), G != 0
    for (int i = threadIdx.x; i < ng * np; i += blockDim.x) {
        const int g = i / np, pc = i % np;
        const int c = pc / nv, v = pc % nv;   // stored [g][c][v]
        double2 sa = make_double2(0.0, 0.0), sb = make_double2(0.0, 0.0);
        if (gx[g] != 0 || gy[g] != 0 || gz[g] != 0) {
            cd ca = cmake(0.0, 0.0), cb = cmake(0.0, 0.0);
            for (int o = 0; o < n_orb; ++o) {
                double sn, cs;
                sincospi(2.0 * (gx[g] * tauS[o * 3] + gy[g] * tauS[o * 3 + 1] + gz[g] * tauS[o * 3 + 2]), &sn, &cs);
                const cd e = cmake(cs, sn);
                cd t = cmake(0.0, 0.0);
                cfma(t, e, cmake(A[v * n_orb + o].x, A[v * n_orb + o].y));
                cfma_cj(ca, cmake(A[(nv + c) * n_orb + o].x, A[(nv + c) * n_orb + o].y), t);
                cd u = cmake(0.0, 0.0);
                cfma(u, e, cmake(B[v * n_orb + o].x, B[v * n_orb + o].y));
                cfma_cj(cb, cmake(B[(nv + c) * n_orb + o].x, B[(nv + c) * n_orb + o].y), u);
            }
            sa = make_double2(ca.re, ca.im);
            sb = make_double2(cb.re, cb.im);
        }
        mxa[i] = sa;
        mxb[i] = sb;
    }
    __syncthreads();

    const int nout = np * np;
    cd accx[kMaxOut], accd[kMaxOut];
    for (int j = 0; j < kMaxOut; ++j) {
        accx[j] = cmake(0.0, 0.0);
        accd[j] = cmake(0.0, 0.0);
    }
    // exchange: X[(v c),(v' c')] = sum_{G != 0} v(G) M_cv(k;G) conj(M_c'v'(kp;G))
    for (int j = 0; j < kMaxOut && !COEF; ++j) {
        const int o = threadIdx.x + j * blockDim.x;
        if (o >= nout) break;
        const int pr = o / np, pc = o % np;
        const int v = pr / nc, c = pr % nc, v2 = pc / nc, c2 = pc % nc;
        for (int g = 0; g < ng; ++g) {
            const int G2 = gx[g] * gx[g] + gy[g] * gy[g] + gz[g] * gz[g];
            if (G2 == 0) continue;
            const double vg = 1.0 / (M_PI * (double)G2);    // 4 pi / |2 pi G|^2
            const double2 a = mxa[g * np + c * nv + v];
            const double2 b = mxb[g * np + c2 * nv + v2];
            cd t = cmake(0.0, 0.0);
            cfma_jc(t, cmake(a.x, a.y), cmake(b.x, b.y));
            accx[j].re = fma(vg, t.re, accx[j].re);
            accx[j].im = fma(vg, t.im, accx[j].im);
        }
    }
    // direct: D[(v c),(v' c')] = sum_G W(q+G) M_cc'(k,kp;q+G) conj(M_vv'(k,kp;q+G))
    for (int g = 0; g < ng; ++g) {
        if (COEF && (gx[g] != 0 || gy[g] != 0 || gz[g] != 0)) continue;   // uniform
        const double Qx = q[0] + gx[g], Qy = q[1] + gy[g], Qz = q[2] + gz[g];
        double W = 4.0 * M_PI / (eps_inf * 4.0 * M_PI * M_PI * (Qx * Qx + Qy * Qy + Qz * Qz) + lam * lam);
        if (k == kp && gx[g] == 0 && gy[g] == 0 && gz[g] == 0) W = wq0;
        if (COEF) W = 1.0 / (M_PI * eps_inf);
        if (threadIdx.x < n_orb) {
            double sn, cs;
            const int o = threadIdx.x;
            sincospi(2.0 * (Qx * tauS[o * 3] + Qy * tauS[o * 3 + 1] + Qz * tauS[o * 3 + 2]), &sn, &cs);
            ph[o] = make_double2(cs, sn);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nc * nc + nv * nv; i += blockDim.x) {
            int r0, r1;
            if (i < nc * nc) {
                r0 = nv + i / nc;
                r1 = nv + i % nc;
            } else {
                r0 = (i - nc * nc) / nv;
                r1 = (i - nc * nc) % nv;
            }
            cd s = cmake(0.0, 0.0);
            for (int o = 0; o < n_orb; ++o) {
                cd t = cmake(0.0, 0.0);
                cfma(t, cmake(ph[o].x, ph[o].y), cmake(B[r1 * n_orb + o].x, B[r1 * n_orb + o].y));
                cfma_cj(s, cmake(A[r0 * n_orb + o].x, A[r0 * n_orb + o].y), t);
            }
            if (i < nc * nc)
                mcc[i] = make_double2(s.re, s.im);
            else
                mvv[i - nc * nc] = make_double2(s.re, s.im);
        }
        __syncthreads();
        for (int j = 0; j < kMaxOut; ++j) {
            const int o = threadIdx.x + j * blockDim.x;
            if (o >= nout) break;
            const int pr = o / np, pc = o % np;
            const int v = pr / nc, c = pr % nc, v2 = pc / nc, c2 = pc % nc;
            const double2 a = mcc[c * nc + c2];
            const double2 b = mvv[v * nv + v2];
            cd t = cmake(0.0, 0.0);
            cfma_jc(t, cmake(a.x, a.y), cmake(b.x, b.y));
            accd[j].re = fma(W, t.re, accd[j].re);
            accd[j].im = fma(W, t.im, accd[j].im);
        }
        __syncthreads();
    }

    // K = scale (2 X - D); Hermitian by construction
    for (int j = 0; j < kMaxOut; ++j) {
        const int o = threadIdx.x + j * blockDim.x;
        if (o >= nout) break;
        const cd val = cmake(scale * (2.0 * accx[j].re - accd[j].re), scale * (2.0 * accx[j].im - accd[j].im));
        const int pr = o / np, pc = o % np;
        if (k != kp) {
            st(K + ((int64_t)k * np + pr) * Nc + (int64_t)kp * np + pc, val);
            st(K + ((int64_t)kp * np + pc) * Nc + (int64_t)k * np + pr, cconj(val));
        } else {
            blk[o] = make_double2(val.re, val.im);
        }
    }
    if (k == kp) {
        __syncthreads();
        for (int o = threadIdx.x; o < nout; o += blockDim.x) {
            const int pr = o / np, pc = o % np;
            const double2 a = blk[pr * np + pc], b = blk[pc * np + pr];
            const cd v = cmake(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
            st(K + ((int64_t)k * np + pr) * Nc + (int64_t)k * np + pc, v);
        }
    }
}

hipError_t launch_overlaps(const Geometry& g, const double* vc, const double* vd, void* dout, hipStream_t s) {
    const int64_t total = (int64_t)g.ncells * 8 * g.ne * g.ndiv3;
    const int nb = (int)std::min<int64_t>((total + kBlock - 1) / kBlock, 65536);
    if (g.dtype == BSE_F64)
        hipLaunchKernelGGL(k_overlaps<double2>, dim3(nb), dim3(kBlock), 0, s, reinterpret_cast<const double2*>(vc),
                           reinterpret_cast<const double2*>(vd), reinterpret_cast<double2*>(dout), g.n_c, g.n_div, g.nv,
                           g.nc, g.n_orb_input, total);
    else
        hipLaunchKernelGGL(k_overlaps<float2>, dim3(nb), dim3(kBlock), 0, s, reinterpret_cast<const double2*>(vc),
                           reinterpret_cast<const double2*>(vd), reinterpret_cast<float2*>(dout), g.n_c, g.n_div, g.nv,
                           g.nc, g.n_orb_input, total);
    return hipGetLastError();
}

hipError_t launch_transition_energies(const Geometry& g, const double* eps, double* out, hipStream_t s) {
    const int nb = (int)std::min<int64_t>((g.N + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_transition_energies, dim3(nb), dim3(kBlock), 0, s, eps, out, g.nv, g.nc, g.N);
    return hipGetLastError();
}

template <bool COEF>
static hipError_t coarse_kernel_go(const Geometry& g, const double* vecs, const double* tau,
                                   const bse_kernel_model& m, void* K, hipStream_t s) {
    const int64_t nk = (int64_t)g.n_c * g.n_c * g.n_c;
    const int64_t npairs = nk * (nk + 1) / 2;
    const double scale = m.kernel_energy / (double)g.nk;
    if (g.dtype == BSE_F64)
        hipLaunchKernelGGL((k_coarse_kernel<double2, COEF>), dim3((unsigned)npairs), dim3(kBlock), 0, s,
                           reinterpret_cast<const double2*>(vecs), tau, reinterpret_cast<double2*>(K), g.n_c, g.n_div,
                           g.nv, g.nc, g.n_orb_input, m.eps_inf, m.lambda, scale, m.g2_max, m.q0_quad);
    else
        hipLaunchKernelGGL((k_coarse_kernel<float2, COEF>), dim3((unsigned)npairs), dim3(kBlock), 0, s,
                           reinterpret_cast<const double2*>(vecs), tau, reinterpret_cast<float2*>(K), g.n_c, g.n_div,
                           g.nv, g.nc, g.n_orb_input, m.eps_inf, m.lambda, scale, m.g2_max, m.q0_quad);
    return hipGetLastError();
}

hipError_t launch_coarse_kernel(const Geometry& g, const double* vecs, const double* tau,
                                const bse_kernel_model& m, void* K, hipStream_t s) {
    return coarse_kernel_go<false>(g, vecs, tau, m, K, s);
}

hipError_t launch_divergence_coefficient(const Geometry& g, const double* vecs, const double* tau,
                                         const bse_kernel_model& m, void* A, hipStream_t s) {
    return coarse_kernel_go<true>(g, vecs, tau, m, A, s);
}

}  // namespace bse
