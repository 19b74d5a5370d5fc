// C ABI of the double-grid BSE library: argument checks, workspace layout and
// the stream-ordered drivers of the matvec and of the Haydock chain.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

static bse_status hip_fail(hipError_t e, const char* what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return BSE_ERR_HIP;
}

bse_status hip_fail_status(hipError_t e, const char* what) { return hip_fail(e, what); }

bool make_geometry(const bse_dims* d, Geometry* g) {
    if (!d) {
        set_error("dims is NULL");
        return false;
    }
    if (d->n_coarse < 1 || d->n_coarse > 64 || d->n_div < 1 || d->n_div > 16) {
        set_error("n_coarse must be in [1, 64] and n_div in [1, 16]");
        return false;
    }
    if (d->nv < 1 || d->nc < 1) {
        set_error("nv and nc must be positive");
        return false;
    }
    if (d->max_rhs < 1 || d->max_rhs > kMaxRhs) {
        set_error("max_rhs must be in [1, %d]", kMaxRhs);
        return false;
    }
    if (d->dtype != BSE_F64 && d->dtype != BSE_F32 && d->dtype != BSE_F32_VEC64 && d->dtype != BSE_BF16_KC &&
        d->dtype != BSE_F16_KC) {
        set_error("unknown dtype %d", d->dtype);
        return false;
    }
    if (d->neighbours != 8 && d->neighbours != 1) {
        set_error("neighbours must be 8 or 1");
        return false;
    }
    g->n_c = d->n_coarse;
    g->n_div = d->n_div;
    g->ndiv3 = d->n_div * d->n_div * d->n_div;
    g->ncells = d->n_coarse * d->n_coarse * d->n_coarse;
    g->nv = d->nv;
    g->nc = d->nc;
    g->np = d->nv * d->nc;
    g->ne = d->nv * d->nv + d->nc * d->nc;
    g->neighbours = d->neighbours;
    g->dtype = d->dtype;
    g->n_orb_input = d->n_orb;
    g->nk = (int64_t)g->ncells * g->ndiv3;
    g->N = g->nk * g->np;
    g->Nc = (int64_t)g->ncells * g->np;
    g->max_rhs = d->max_rhs;
    if (g->Nc > (int64_t)1 << 30) {
        set_error("coarse transition space too large");
        return false;
    }
    return true;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static constexpr int kWaveHost = 64;  // lanes of a wavefront (restrict tile width)

size_t lds_limit() {
    // shared memory one block may use on the current device (queried once per device)
    static size_t cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
    if (cache[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        cache[dev] = (size_t)v;
    }
    return cache[dev];
}
int cu_count() {
    // compute units of the current device (queried once per device)
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}
static size_t vec_elem_bytes(int dtype) { return vec_is_f32(dtype) ? sizeof(float2) : sizeof(double2); }
static size_t mat_elem_bytes(int dtype) { return dtype == BSE_F64 ? sizeof(double2) : sizeof(float2); }

Layout make_layout(const Geometry& g) {
    Layout L;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t R = (size_t)g.max_rhs;
    L.qpart = take((size_t)g.ncells * 8 * R * g.np * sizeof(double2));
    L.qbar = take((size_t)g.Nc * R * sizeof(double2));
    L.rvec = take((size_t)g.Nc * R * sizeof(double2));
    L.gpart = take((size_t)kMaxSplit * g.Nc * R * sizeof(double2));
    L.ppart = take((size_t)g.ncells * R * 2 * 2 * sizeof(double));
    L.rpart = take((size_t)g.ncells * R * 2 * sizeof(double));
    L.chain = take((size_t)2 * kMaxRhs * sizeof(ChainState));
    L.pend = take((size_t)kMaxRhs * sizeof(StepScalars));
    L.flags = take((size_t)kMaxRhs * sizeof(int32_t));
    L.cpart = take((size_t)kMaxRhs * kConvBlocks * 2 * sizeof(double));
    L.vec_a = take((size_t)g.N * R * vec_elem_bytes(g.dtype));
    L.vec_b = take((size_t)g.N * R * vec_elem_bytes(g.dtype));
    L.kq = L.kscale = L.qfrag = L.qsinv = L.mp1 = L.mp2 = L.mtab = off;
    L.kq_bytes = L.kscale_bytes = L.qfrag_bytes = 0;
    if (kc_lowp(g.dtype)) {
        const KqShape k = kq_shape(g.Nc);
        L.kq_bytes = (size_t)k.nb * k.nb * kKqBlock * kKqBlock * 4;
        L.kscale_bytes = (size_t)k.nb * k.nb * sizeof(float);
        L.qfrag_bytes = (size_t)k.nstep * 2 * kWaveHost * 16;
        L.kq = take(L.kq_bytes);
        L.kscale = take(L.kscale_bytes);
        L.qfrag = take(L.qfrag_bytes);
        L.qsinv = take((size_t)k.nb * kMaxRhs * sizeof(float));
        const HmShape hm = hm_shape(g.Nc);
        L.mp1 = take((size_t)hm.runs * 2 * kKqBlock * R * sizeof(double2));
        L.mp2 = take((size_t)hm.p2 * kKqBlock * R * sizeof(float2));
        L.mtab = take((size_t)(hm.runs + hm.bands + 1) * sizeof(int));
    }
    L.kp = L.hpart = L.htab = off;
    L.kp_bytes = 0;
    if (kc_packable(g.dtype)) {
        const HemvShape h = hemv_shape(g.Nc, g.dtype);
        L.kp_bytes = (size_t)h.tiles * h.tile_bytes;
        L.kp = take(L.kp_bytes);
        L.hpart = take((size_t)(h.blocks + h.tiles) * 128 * R * h.elem_bytes);
        L.htab = take((size_t)(h.blocks + h.nbk + 1) * sizeof(int));
    }
    L.dsw_bytes = 0;
    L.dsw = off;
    if (supported_bands(g.nv, g.nc) && restrict_tile_lds(g) > 0) {
        const int eb = (int)mat_elem_bytes(g.dtype);
        const SwzShape z = swz_shape(g.nv, g.nc, g.ndiv3, eb);
        L.dsw_bytes = (size_t)g.ncells * z.S * kWaveHost * z.kp * eb;
        L.dsw = take(L.dsw_bytes);
    }
    L.total = off;
    return L;
}

// ---- continued fraction (Eq. fraccont) ------------------------------------------------
__global__ __launch_bounds__(256) void k_continued_fraction(const double* __restrict__ a, const double* __restrict__ b,
                                                            int lda, int ldb, const double* __restrict__ pnorm2,
                                                            const int32_t* __restrict__ steps, int n_chains,
                                                            double prefactor, const double* __restrict__ omega,
                                                            int n_omega, double eta, double* __restrict__ eps_re,
                                                            double* __restrict__ eps_im) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_chains * n_omega) return;
    const int ch = (int)(i / n_omega);
    const int w = (int)(i % n_omega);
    const int m = min(steps[ch], lda);
    const double pn = pnorm2[ch];
    if (m <= 0 || pn == 0.0) {
        eps_re[i] = 1.0;
        eps_im[i] = 0.0;
        return;
    }
    const double zr = omega[w], zi = eta;
    const double* ac = a + (int64_t)ch * lda;
    const double* bc = b + (int64_t)ch * ldb;
    // t_m = z - a_m; t_i = z - a_i - b_{i+1}^2 / t_{i+1}
    double tr = zr - ac[m - 1], ti = zi;
    for (int j = m - 2; j >= 0; --j) {
        const double b2 = bc[j + 1] * bc[j + 1];
        const double den = tr * tr + ti * ti;
        const double ur = b2 * tr / den, ui = -b2 * ti / den;   // b^2 / t
        tr = zr - ac[j] - ur;
        ti = zi - ui;
    }
    // eps = 1 - C ||P||^2 / t
    const double den = tr * tr + ti * ti;
    const double cr = prefactor * pn * tr / den, ci = -prefactor * pn * ti / den;
    eps_re[i] = 1.0 - cr;
    eps_im[i] = -ci;
}

hipError_t launch_continued_fraction(const double* a, const double* b, int lda, int ldb, const double* pnorm2,
                                     const int32_t* steps, int n_chains, double prefactor, const double* omega,
                                     int n_omega, double eta, double* eps_re, double* eps_im, hipStream_t s) {
    const int64_t total = (int64_t)n_chains * n_omega;
    const int nb = (int)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_continued_fraction, dim3(nb), dim3(kBlock), 0, s, a, b, lda, ldb, pnorm2, steps, n_chains,
                       prefactor, omega, n_omega, eta, eps_re, eps_im);
    return hipGetLastError();
}

// chain start: u_1 = P, ||u_1||, ||P||, coarse vector of psi_1; zero-fills a and b
static hipError_t enqueue_chain_start(Plan& p, const double* P, int n_rhs, double* a, double* b, int lda, int ldb,
                                      hipStream_t stream) {
    void* B = p.ws + p.L.vec_b;  // u_1
    hipError_t e = launch_restrict(p, RESTRICT_INIT, nullptr, nullptr, nullptr, P, B, 0, a, b, lda, ldb, n_rhs,
                                   stream);
    if (e == hipSuccess) e = launch_collapse(p, COLLAPSE_INIT, 0, b, ldb, n_rhs, stream);
    return e;
}

// steps i0 .. i1 - 1 of the chain (Eqs. ai-ci); the two vector buffers alternate: before
// step i, buffer (i even ? vec_b : vec_a) holds u_i and the other u_{i-1}
static hipError_t enqueue_chain_steps(Plan& p, int i0, int i1, int n_rhs, double* a, double* b, int lda, int ldb,
                                      hipStream_t stream) {
    hipError_t e = hipSuccess;
    for (int i = i0; i < i1 && e == hipSuccess; ++i) {
        void* B = p.ws + ((i & 1) ? p.L.vec_a : p.L.vec_b);  // u_i
        void* A = p.ws + ((i & 1) ? p.L.vec_b : p.L.vec_a);  // u_{i-1}, then w, then u_{i+1}
        e = launch_m3_apply(p, B, n_rhs, stream);   // Method 3 band of u_i (no-op without a band)
        if (e == hipSuccess) e = launch_gemv(p, n_rhs, stream);
        if (e == hipSuccess) e = launch_prolong(p, PROLONG_LANCZOS, B, A, i, n_rhs, stream);
        if (e == hipSuccess)
            e = launch_restrict(p, RESTRICT_UPDATE, nullptr, A, B, nullptr, A, i, a, b, lda, ldb, n_rhs, stream);
        if (e == hipSuccess) e = launch_collapse(p, COLLAPSE_STEP, i, b, ldb, n_rhs, stream);
    }
    return e;
}

hipError_t enqueue_haydock(Plan& p, const double* P, int n_rhs, int n_steps, double* a, double* b, double* pnorm2,
                           int32_t* steps_done, int32_t* status, hipStream_t stream) {
    const int lda = n_steps, ldb = n_steps + 1;
    hipError_t e = enqueue_chain_start(p, P, n_rhs, a, b, lda, ldb, stream);
    if (e == hipSuccess) e = enqueue_chain_steps(p, 0, n_steps, n_rhs, a, b, lda, ldb, stream);
    if (e == hipSuccess) e = launch_chain_report(p, n_steps, pnorm2, steps_done, status, n_rhs, stream);
    return e;
}

// ---- convergence check of the spectrum (the paper's stop rule, Sec. 2 after Eq. fraccont)
// One block per chain: eps_M(omega) from the coefficients so far (Eq. fraccont), compared
// with the previous check's eps2 at every omega.  A chain whose largest change is at most
// tol times the largest |eps2| stops: its state is made inactive (status BSE_OK), so the
// following steps leave its coefficients alone.  active_out[r] = chain still running.
// Block (chain r, slice q) of the convergence check: eps_M at the frequencies
// w = q blockDim + thread, stride gridDim.y blockDim, from the chain's first m coefficients,
// and the slice's largest change since the last check and largest |eps2|, written to
// part[(r nq + q) 2 + {0, 1}] for k_converge_decide.
__global__ __launch_bounds__(256) void k_converge_check(const double* __restrict__ a, const double* __restrict__ b,
                                                        int lda, int ldb, const ChainState* __restrict__ cs,
                                                        double prefactor, const double* __restrict__ omega,
                                                        int n_omega, double eta, int first, int closure,
                                                        double* __restrict__ eps_re, double* __restrict__ eps_im,
                                                        double* __restrict__ part) {
    __shared__ double sred[2][256 / kWave];
    const int r = blockIdx.x;
    const ChainState st = cs[r];
    const int m = min(st.steps, lda);
    const double pn = st.pnorm2;
    const double* ac = a + (int64_t)r * lda;
    const double* bc = b + (int64_t)r * ldb;
    // the constant chain that closes the fraction: means of the last `closure` steps
    const bool closed = closure > 0 && m >= closure;
    double a_inf = 0.0, b_inf = 0.0, bm2 = 0.0;
    if (closed) {
        for (int j = m - closure; j < m; ++j) {
            a_inf += ac[j];
            b_inf += bc[j + 1];
        }
        a_inf /= closure;
        b_inf /= closure;
        bm2 = bc[m] * bc[m];   // b_{m+1}: 0 after a breakdown, which leaves the fraction exact
    }
    double dmax = 0.0, emax = 0.0;
    for (int w = blockIdx.y * blockDim.x + threadIdx.x; w < n_omega; w += gridDim.y * blockDim.x) {
        double er = 1.0, ei = 0.0;
        if (m > 0 && pn != 0.0) {
            const double zr = omega[w], zi = eta;
            double tr = zr - ac[m - 1], ti = zi;
            if (closed) {   // t_m = z - a_m - b_{m+1}^2 g_inf(z)
                double gr, gi;
                constant_chain(zr, zi, a_inf, b_inf, gr, gi);
                tr -= bm2 * gr;
                ti -= bm2 * gi;
            }
            for (int j = m - 2; j >= 0; --j) {   // t_j = z - a_j - b_{j+1}^2 / t_{j+1}
                const double b2 = bc[j + 1] * bc[j + 1];
                const double g = b2 / (tr * tr + ti * ti);   // one division per level
                tr = zr - ac[j] - g * tr;
                ti = zi + g * ti;
            }
            const double den = tr * tr + ti * ti;
            er = 1.0 - prefactor * pn * tr / den;
            ei = prefactor * pn * ti / den;
        }
        const int64_t o = (int64_t)r * n_omega + w;
        if (!first) dmax = fmax(dmax, fabs(ei - eps_im[o]));
        emax = fmax(emax, fabs(ei));
        eps_re[o] = er;
        eps_im[o] = ei;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        dmax = fmax(dmax, __shfl_xor(dmax, off, kWave));
        emax = fmax(emax, __shfl_xor(emax, off, kWave));
    }
    const int wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    if (threadIdx.x % kWave == 0) {
        sred[0][wave] = dmax;
        sred[1][wave] = emax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < nw; ++w) {
            dmax = fmax(dmax, sred[0][w]);
            emax = fmax(emax, sred[1][w]);
        }
        double* o = part + ((int64_t)r * gridDim.y + blockIdx.y) * 2;
        o[0] = dmax;
        o[1] = emax;
    }
}

// The stop rule of each chain from the slices' maxima (a maximum does not depend on the
// order of its terms): a chain whose spectrum changed by at most tol times its peak since
// the last check stops.  Thread r < n_rhs.
__global__ void k_converge_decide(const double* __restrict__ part, int nq, ChainState* __restrict__ cs, double tol,
                                  int first, int n_rhs, int32_t* __restrict__ active_out) {
    const int r = threadIdx.x;
    if (r >= n_rhs) return;
    double dmax = 0.0, emax = 0.0;
    for (int q = 0; q < nq; ++q) {
        dmax = fmax(dmax, part[((int64_t)r * nq + q) * 2]);
        emax = fmax(emax, part[((int64_t)r * nq + q) * 2 + 1]);
    }
    int active = cs[r].active;
    if (active && !first && dmax <= tol * emax) {
        cs[r].active = 0;   // converged: the chain stops here with status BSE_OK
        active = 0;
    }
    active_out[r] = active;
}

}  // namespace bse

using namespace bse;

extern "C" {

const char* bse_version(void) { return "bse-dg 0.1.0 (gfx950)"; }

const char* bse_last_error(void) { return g_err; }

size_t bse_workspace_bytes(const bse_dims* dims) {
    Geometry g;
    if (!make_geometry(dims, &g)) return 0;
    return make_layout(g).total;
}

size_t bse_coarse_kernel_bytes(const bse_dims* dims) {
    Geometry g;
    if (!make_geometry(dims, &g)) return 0;
    return (size_t)g.Nc * (size_t)g.Nc * mat_elem_bytes(g.dtype);
}

size_t bse_overlaps_bytes(const bse_dims* dims) {
    Geometry g;
    if (!make_geometry(dims, &g)) return 0;
    return (size_t)g.ncells * 8 * g.ne * g.ndiv3 * mat_elem_bytes(g.dtype);
}

bse_status bse_build_overlaps(const bse_dims* dims, const double* vecs_coarse, const double* vecs_dense,
                              void* d_out, hipStream_t stream) {
    Geometry g;
    if (!make_geometry(dims, &g)) return BSE_ERR_INVALID_ARG;
    if (!vecs_coarse || !vecs_dense || !d_out) {
        set_error("bse_build_overlaps: NULL pointer");
        return BSE_ERR_INVALID_ARG;
    }
    if (g.n_orb_input < 1) {
        set_error("bse_build_overlaps: n_orb must be positive");
        return BSE_ERR_INVALID_ARG;
    }
    hipError_t e = launch_overlaps(g, vecs_coarse, vecs_dense, d_out, stream);
    return e == hipSuccess ? BSE_OK : hip_fail(e, "bse_build_overlaps");
}

bse_status bse_build_transition_energies(const bse_dims* dims, const double* eps_dense, double* delta_out,
                                         hipStream_t stream) {
    Geometry g;
    if (!make_geometry(dims, &g)) return BSE_ERR_INVALID_ARG;
    if (!eps_dense || !delta_out) {
        set_error("bse_build_transition_energies: NULL pointer");
        return BSE_ERR_INVALID_ARG;
    }
    hipError_t e = launch_transition_energies(g, eps_dense, delta_out, stream);
    return e == hipSuccess ? BSE_OK : hip_fail(e, "bse_build_transition_energies");
}

bse_status bse_build_coarse_kernel(const bse_dims* dims, const double* vecs_coarse, const double* tau,
                                   const bse_kernel_model* model, void* Kc_out, hipStream_t stream) {
    Geometry g;
    if (!make_geometry(dims, &g)) return BSE_ERR_INVALID_ARG;
    if (!vecs_coarse || !tau || !model || !Kc_out) {
        set_error("bse_build_coarse_kernel: NULL pointer");
        return BSE_ERR_INVALID_ARG;
    }
    if (g.n_orb_input < 1 || g.n_orb_input > 16 || g.nv + g.nc > 16 || g.np > 32) {
        set_error("bse_build_coarse_kernel: needs n_orb <= 16, nv + nc <= 16, nv * nc <= 32");
        return BSE_ERR_UNSUPPORTED;
    }
    if (model->g2_max < 0 || model->g2_max > 4 || model->q0_quad < 1 || model->q0_quad > 256 ||
        !(model->eps_inf > 0) || !(model->lambda >= 0)) {
        set_error("bse_build_coarse_kernel: model parameters out of range (g2_max <= 4)");
        return BSE_ERR_INVALID_ARG;
    }
    hipError_t e = launch_coarse_kernel(g, vecs_coarse, tau, *model, Kc_out, stream);
    return e == hipSuccess ? BSE_OK : hip_fail(e, "bse_build_coarse_kernel");
}

bse_status bse_plan_create(const bse_dims* dims, const void* Kc, const void* d, const double* delta,
                           void* workspace, size_t workspace_bytes, hipStream_t stream, bse_plan** plan_out) {
    if (!plan_out) {
        set_error("bse_plan_create: plan_out is NULL");
        return BSE_ERR_INVALID_ARG;
    }
    *plan_out = nullptr;
    Geometry g;
    if (!make_geometry(dims, &g)) return BSE_ERR_INVALID_ARG;
    if (!bands_in_range(g.nv, g.nc)) {
        set_error("bands nv=%d nc=%d: the hot path takes nv + nc <= 16 and nv nc <= 32", g.nv, g.nc);
        return BSE_ERR_UNSUPPORTED;
    }
    if (!Kc || !d || !delta) {
        set_error("bse_plan_create: NULL input array");
        return BSE_ERR_INVALID_ARG;
    }
    Layout L = make_layout(g);
    if (!workspace || ((uintptr_t)workspace & 255) != 0 || workspace_bytes < L.total) {
        set_error("bse_plan_create: workspace must be 256-byte aligned and >= %zu bytes", L.total);
        return BSE_ERR_WORKSPACE;
    }
    Plan* p = new (std::nothrow) Plan();
    if (!p) {
        set_error("bse_plan_create: out of host memory");
        return BSE_ERR_INVALID_ARG;
    }
    p->g = g;
    p->L = L;
    p->Kc = Kc;
    p->d = d;
    p->delta = delta;
    p->ws = static_cast<char*>(workspace);
    p->n_split = 0;
    p->product_form = 0;
    p->converge_closure = 0;
    p->side = nullptr;
    p->chk[0] = p->chk[1] = nullptr;
    p->restrict_group = 1;
    p->timing = 0;
    p->ev = nullptr;
    p->ev_cap = 0;
    p->ev_used = 0;
    p->split_start = p->split_ev = nullptr;
    p->timed_ms = 0.0;
    p->timed_launches = 0;
    // restrict tiles: a re-ordered copy of the overlaps in the workspace; for the
    // low-precision forms also the block-scaled coarse kernel
    hipError_t e = launch_swizzle(*p, stream);
    if (e == hipSuccess) e = launch_quantize(*p, stream);
    if (e == hipSuccess) e = launch_hemv_pack(*p, stream);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "bse_plan_create");
    }
    *plan_out = reinterpret_cast<bse_plan*>(p);
    return BSE_OK;
}

static void release_events(Plan* p) {
    if (p->ev) {
        for (int i = 0; i < p->ev_cap; ++i) (void)hipEventDestroy(p->ev[i]);
        delete[] p->ev;
    }
    p->ev = nullptr;
    p->ev_cap = 0;
    p->ev_used = 0;
}

void bse_plan_destroy(bse_plan* plan) {
    if (!plan) return;
    Plan* p = reinterpret_cast<Plan*>(plan);
    release_events(p);
    for (int k = 0; k < 2; ++k)
        if (p->chk[k]) (void)hipEventDestroy(p->chk[k]);
    if (p->side) (void)hipStreamDestroy(p->side);
    delete p;
}

bse_status bse_interp_matvec(bse_plan* plan, const void* x, void* y, int32_t n_rhs, hipStream_t stream) {
    if (!plan || !x || !y) {
        set_error("bse_interp_matvec: NULL argument");
        return BSE_ERR_INVALID_ARG;
    }
    Plan& p = *reinterpret_cast<Plan*>(plan);
    if (n_rhs < 1 || n_rhs > p.g.max_rhs) {
        set_error("bse_interp_matvec: n_rhs must be in [1, %d]", p.g.max_rhs);
        return BSE_ERR_INVALID_ARG;
    }
    if (x == y) {
        set_error("bse_interp_matvec: x and y must not alias");
        return BSE_ERR_INVALID_ARG;
    }
    hipError_t e = launch_m3_apply(p, x, n_rhs, stream);   // Method 3 band (no-op without a band)
    if (e == hipSuccess)
        e = launch_restrict(p, RESTRICT_PLAIN, x, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, 0,
                            n_rhs, stream);
    if (e == hipSuccess) e = launch_collapse(p, COLLAPSE_PLAIN, 0, nullptr, 0, n_rhs, stream);
    if (e == hipSuccess) e = launch_gemv(p, n_rhs, stream);
    if (e == hipSuccess) e = launch_prolong(p, PROLONG_PLAIN, x, y, 0, n_rhs, stream);
    return e == hipSuccess ? BSE_OK : hip_fail(e, "bse_interp_matvec");
}

bse_status bse_haydock_run(bse_plan* plan, const double* P, int32_t n_rhs, int32_t n_steps, double* a, double* b,
                           double* pnorm2, int32_t* steps_done, int32_t* status, hipStream_t stream) {
    if (!plan || !P || !a || !b || !pnorm2 || !steps_done || !status) {
        set_error("bse_haydock_run: NULL argument");
        return BSE_ERR_INVALID_ARG;
    }
    Plan& p = *reinterpret_cast<Plan*>(plan);
    if (n_rhs < 1 || n_rhs > p.g.max_rhs || n_steps < 1) {
        set_error("bse_haydock_run: n_rhs must be in [1, %d] and n_steps >= 1", p.g.max_rhs);
        return BSE_ERR_INVALID_ARG;
    }
    hipError_t e = enqueue_haydock(p, P, n_rhs, n_steps, a, b, pnorm2, steps_done, status, stream);
    return e == hipSuccess ? BSE_OK : hip_fail(e, "bse_haydock_run");
}

bse_status bse_haydock_converge(bse_plan* plan, const double* P, int32_t n_rhs, int32_t max_steps,
                                int32_t check_every, double prefactor, const double* omega, int32_t n_omega,
                                double eta, double tol, double* a, double* b, double* pnorm2, int32_t* steps_done,
                                int32_t* status, double* eps_re, double* eps_im, hipStream_t stream) {
    if (!plan || !P || !a || !b || !pnorm2 || !steps_done || !status || !omega || !eps_re || !eps_im) {
        set_error("bse_haydock_converge: NULL argument");
        return BSE_ERR_INVALID_ARG;
    }
    Plan& p = *reinterpret_cast<Plan*>(plan);
    if (n_rhs < 1 || n_rhs > p.g.max_rhs || max_steps < 1 || check_every < 1 || n_omega < 1 || !(eta > 0) ||
        !(tol >= 0)) {
        set_error("bse_haydock_converge: need n_rhs in [1, %d], max_steps, check_every, n_omega >= 1, eta > 0, "
                  "tol >= 0", p.g.max_rhs);
        return BSE_ERR_INVALID_ARG;
    }
    const int lda = max_steps, ldb = max_steps + 1;
    int32_t* flags = reinterpret_cast<int32_t*>(p.ws + p.L.flags);
    hipError_t e = hipSuccess;
    if (!p.side) e = hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking);   // default priority
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        if (!p.chk[k]) e = hipEventCreateWithFlags(&p.chk[k], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "bse_haydock_converge: stream or events");
    e = enqueue_chain_start(p, P, n_rhs, a, b, lda, ldb, stream);
    // i: steps up to the last check; ahead: steps past i already enqueued
    int i = 0, ahead = 0, c = 0;
    bool running = true;
    while (e == hipSuccess && i < max_steps) {
        const int n = std::min(check_every, max_steps - i);
        if (ahead < n) e = enqueue_chain_steps(p, i + ahead, i + n, n_rhs, a, b, lda, ldb, stream);
        i += n;
        if (e != hipSuccess) break;
        ChainState* cs = reinterpret_cast<ChainState*>(p.ws + p.L.chain) + state_in(i) * kMaxRhs;
        // the check over the frequencies in slices of 256, then the stop decision per chain
        const int nq = std::min(kConvBlocks, (n_omega + 255) / 256);
        double* cpart = reinterpret_cast<double*>(p.ws + p.L.cpart);
        hipLaunchKernelGGL(k_converge_check, dim3(n_rhs, nq), dim3(256), 0, stream, a, b, lda, ldb, cs, prefactor,
                           omega, n_omega, eta, c == 0 ? 1 : 0, p.converge_closure, eps_re, eps_im, cpart);
        e = hipGetLastError();
        if (e == hipSuccess)
            hipLaunchKernelGGL(k_converge_decide, dim3(1), dim3(kWave), 0, stream, cpart, nq, cs, tol,
                               c == 0 ? 1 : 0, n_rhs, flags);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(p.chk[c & 1], stream);
        // the first steps of the next chunk keep the device busy while the host reads this
        // check; once every chain has stopped they leave the chains unchanged
        ahead = std::min(kConvAhead, std::min(check_every, max_steps - i));
        if (e == hipSuccess && ahead > 0) e = enqueue_chain_steps(p, i, i + ahead, n_rhs, a, b, lda, ldb, stream);
        if (e == hipSuccess) {
            int32_t act[kMaxRhs] = {0, 0, 0, 0};
            e = hipEventSynchronize(p.chk[c & 1]);
            if (e == hipSuccess) e = hipMemcpyAsync(act, flags, n_rhs * sizeof(int32_t), hipMemcpyDeviceToHost, p.side);
            if (e == hipSuccess) e = hipStreamSynchronize(p.side);
            running = false;
            for (int r = 0; r < n_rhs; ++r) running = running || act[r] != 0;
        }
        ++c;
        if (!running) {
            i += ahead;
            break;
        }
    }
    if (e == hipSuccess) e = launch_chain_report(p, i, pnorm2, steps_done, status, n_rhs, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e == hipSuccess ? BSE_OK : hip_fail(e, "bse_haydock_converge");
}

bse_status bse_continued_fraction(const double* a, const double* b, int32_t lda, int32_t ldb, const double* pnorm2,
                                  const int32_t* steps, int32_t n_chains, double prefactor, const double* omega,
                                  int32_t n_omega, double eta, double* eps_re, double* eps_im, hipStream_t stream) {
    if (!a || !b || !pnorm2 || !steps || !omega || !eps_re || !eps_im) {
        set_error("bse_continued_fraction: NULL argument");
        return BSE_ERR_INVALID_ARG;
    }
    if (n_chains < 1 || n_omega < 1 || lda < 1 || ldb < lda + 1 || !(eta > 0)) {
        set_error("bse_continued_fraction: need n_chains, n_omega >= 1, ldb >= lda + 1, eta > 0");
        return BSE_ERR_INVALID_ARG;
    }
    hipError_t e = launch_continued_fraction(a, b, lda, ldb, pnorm2, steps, n_chains, prefactor, omega, n_omega,
                                             eta, eps_re, eps_im, stream);
    return e == hipSuccess ? BSE_OK : hip_fail(e, "bse_continued_fraction");
}

bse_status bse_plan_set_timing(bse_plan* plan, int32_t enable) {
    if (!plan) {
        set_error("bse_plan_set_timing: NULL plan");
        return BSE_ERR_INVALID_ARG;
    }
    Plan& p = *reinterpret_cast<Plan*>(plan);
    if (enable && !p.ev) {
        const int cap = 4096;
        p.ev = new (std::nothrow) hipEvent_t[cap];
        if (!p.ev) {
            set_error("bse_plan_set_timing: out of host memory");
            return BSE_ERR_INVALID_ARG;
        }
        for (int i = 0; i < cap; ++i) {
            hipError_t e = hipEventCreate(&p.ev[i]);
            if (e != hipSuccess) {
                p.ev_cap = i;
                release_events(&p);
                return hip_fail(e, "bse_plan_set_timing");
            }
        }
        p.ev_cap = cap;
    }
    if (!enable) release_events(&p);
    p.timing = (enable == 2 || enable == 3) ? enable : (enable != 0 ? 1 : 0);
    p.ev_used = 0;
    p.timed_ms = 0.0;
    p.timed_launches = 0;
    return BSE_OK;
}

bse_status bse_plan_get_timing(bse_plan* plan, double* total_ms, int64_t* launches) {
    if (!plan || !total_ms || !launches) {
        set_error("bse_plan_get_timing: NULL argument");
        return BSE_ERR_INVALID_ARG;
    }
    Plan& p = *reinterpret_cast<Plan*>(plan);
    double ms = 0.0;
    for (int i = 0; i + 1 < p.ev_used; i += 2) {
        hipError_t e = hipEventSynchronize(p.ev[i + 1]);
        if (e != hipSuccess) return hip_fail(e, "bse_plan_get_timing");
        float t = 0.0f;
        e = hipEventElapsedTime(&t, p.ev[i], p.ev[i + 1]);
        if (e != hipSuccess) return hip_fail(e, "bse_plan_get_timing");
        ms += t;
    }
    p.timed_ms += ms;
    p.timed_launches += p.ev_used / 2;
    p.ev_used = 0;
    *total_ms = p.timed_ms;
    *launches = p.timed_launches;
    p.timed_ms = 0.0;
    p.timed_launches = 0;
    return BSE_OK;
}

bse_status bse_plan_set_gemv_splits(bse_plan* plan, int32_t n_split) {
    if (!plan || n_split < 0 || n_split > kMaxSplit) {
        set_error("bse_plan_set_gemv_splits: n_split must be in [0, %d]", kMaxSplit);
        return BSE_ERR_INVALID_ARG;
    }
    reinterpret_cast<Plan*>(plan)->n_split = n_split;
    return BSE_OK;
}

bse_status bse_plan_set_coarse_product(bse_plan* plan, int32_t form) {
    if (!plan || (form != 0 && form != 1)) {
        set_error("bse_plan_set_coarse_product: form must be 0 (packed Hermitian tiles) or 1 (full stream)");
        return BSE_ERR_INVALID_ARG;
    }
    reinterpret_cast<Plan*>(plan)->product_form = form;
    return BSE_OK;
}

bse_status bse_plan_set_converge_closure(bse_plan* plan, int32_t k) {
    if (!plan || k < 0 || k > 64) {
        set_error("bse_plan_set_converge_closure: k must be in [0, 64]");
        return BSE_ERR_INVALID_ARG;
    }
    reinterpret_cast<Plan*>(plan)->converge_closure = k;
    return BSE_OK;
}

bse_status bse_plan_set_restrict_group(bse_plan* plan, int32_t rhs_per_block) {
    if (!plan || (rhs_per_block != 1 && rhs_per_block != 3)) {
        set_error("bse_plan_set_restrict_group: rhs_per_block must be 1 or 3");
        return BSE_ERR_INVALID_ARG;
    }
    reinterpret_cast<Plan*>(plan)->restrict_group = rhs_per_block;
    return BSE_OK;
}

}  // extern "C"
