/*
 * bse_dg.h - C ABI of the double-grid on-the-fly BSE / Haydock library (gfx950).
 *
 * The library applies the dense-mesh Tamm-Dancoff BSE Hamiltonian whose kernel
 * is interpolated on the fly from a coarse-mesh kernel (Gillet, Giantomassi,
 * Gonze, "Efficient on-the-fly interpolation technique for Bethe-Salpeter
 * calculations of optical spectra", Sec. 4, Eqs. matmul1-matmul3), runs the
 * Haydock-Lanczos recursion on it (Sec. 2, Eqs. ai-ci) and evaluates the
 * continued fraction for the macroscopic dielectric function (Eq. fraccont).
 *
 * Conventions shared by every call
 * --------------------------------
 * Meshes (Sec. 3): a cubic coarse mesh of n_coarse points per axis and n_div
 * divisions per axis.  Coarse point / cell index cell = (i1 n + i2) n + i3;
 * subpoint sub = (j1 n_div + j2) n_div + j3; dense point kd = cell n_div^3 + sub
 * (cell-major).  Corner z = 4 l + 2 m + n is the coarse point
 * (i1 + l, i2 + m, i3 + n), indices wrapping periodically.
 * Transitions: dense t = (kd nv + v) nc + c; coarse T = (cell nv + n1) nc + n2,
 * N = n_coarse^3 n_div^3 nv nc, Nc = n_coarse^3 nv nc.
 * Complex numbers are interleaved (re, im) pairs of the storage precision.
 * Vectors with several right-hand sides are stored column by column:
 * element (t, r) at offset r * N + t.
 *
 * Memory: every pointer documented "device" must point to device memory of the
 * current HIP device; "host" pointers to host memory.  The library never
 * allocates device memory: scratch space is the caller's workspace (the one
 * exception, bse_dense_backward_noalloc, uses a fixed array in the library's
 * device code instead).  All
 * device work is enqueued on the given stream, in stream order, and the calls
 * return without waiting for it unless stated otherwise.
 *
 * Errors: calls return a bse_status.  Negative values are errors and nothing
 * was enqueued (argument checks happen before any launch) unless the value is
 * BSE_ERR_HIP, which reports a failed HIP call; bse_last_error() then gives a
 * message (thread-local, valid until the next call on the same thread).
 */
#ifndef BSE_DG_H
#define BSE_DG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BSE_OK = 0,
    BSE_INFO_INVARIANT_SUBSPACE = 1, /* chain status: b_{i+1} vanished, chain complete */
    BSE_INFO_ZERO_START = 2,         /* chain status: ||P|| = 0, eps_M = 1 */
    BSE_ERR_INVALID_ARG = -1,
    BSE_ERR_HIP = -2,
    BSE_ERR_NONFINITE = -3,          /* chain status: a_i or b_{i+1} not finite */
    BSE_ERR_UNSUPPORTED = -4,        /* band counts or sizes outside what a call takes */
    BSE_ERR_WORKSPACE = -5           /* workspace missing, misaligned or too small */
} bse_status;

/* Storage precision of the coarse kernel, the overlaps and the Lanczos
 * vectors.  Every sum (restrict, coarse product, prolong, dot products) is
 * accumulated in FP64 whatever the storage, except inside the matrix-core
 * products of the two low-precision forms (see below).
 *
 * Low-precision forms (BSE_BF16_KC, BSE_F16_KC): the plan keeps K_c of Eq.
 * (matmul2) as 64 x 64 blocks B with one FP32 scale s_B each (a power of two
 * >= the block's largest real or imaginary part) and entries K / s_B in BF16 or
 * FP16.  The coarse vector qbar enters the matrix-core product as a sum of two
 * terms of the same format (its leading part and the remainder), so that K's
 * rounding (unit roundoff 2^-8 for BF16; 2^-11 for FP16 above 2^-14 of the block
 * scale, 2^-25 of the scale absolute below) dominates the error.  Products over one block accumulate in FP32 on the
 * matrix cores; block results are scaled and added in FP64.  For FP16, each
 * right-hand side of each 64-entry group of qbar is multiplied by the power of two
 * that puts its largest entry in [2^14, 2^15) before the conversion (the block
 * result is divided by it), so no input norm overflows the format or loses its
 * relative accuracy to subnormals.  The input K_c, the overlaps and the Lanczos
 * vectors are complex FP32. */
typedef enum {
    BSE_F64 = 0,        /* kernel, overlaps, vectors: complex FP64 */
    BSE_F32 = 1,        /* kernel, overlaps, vectors: complex FP32 */
    BSE_F32_VEC64 = 2,  /* kernel, overlaps: complex FP32; Lanczos vectors: complex FP64 */
    BSE_BF16_KC = 3,    /* kernel in block-scaled BF16 (from an FP32 input); rest FP32 */
    BSE_F16_KC = 4      /* kernel in block-scaled FP16 (from an FP32 input); rest FP32 */
} bse_dtype;

typedef struct {
    int32_t n_coarse;   /* coarse points per axis (Sec. 3, k~ mesh), >= 1 */
    int32_t n_div;      /* divisions per axis (n_1 = n_2 = n_3 = n_div, Sec. 3), >= 1 */
    int32_t nv;         /* valence bands of the transition space */
    int32_t nc;         /* conduction bands of the transition space */
    int32_t n_orb;      /* orbital-basis size of the band-structure input (builders only) */
    int32_t max_rhs;    /* largest number of right-hand sides per call, 1..4 */
    int32_t dtype;      /* bse_dtype */
    int32_t neighbours; /* 8: trilinear prefactors (Sec. 3, Eq. interpwfn);
                           1: nearest corner only (Rohlfing-Louie, Eq. eqRL) */
} bse_dims;

typedef struct bse_plan bse_plan; /* opaque, host object owned by the library */

/* Parameters of the model kernel built by bse_build_coarse_kernel. */
typedef struct {
    double eps_inf;        /* screening of W(Q) = 4 pi / (eps_inf |Q|^2 + lambda^2) */
    double lambda;         /* screening wavevector */
    double kernel_energy;  /* energy scale; K_c = kernel_energy / N_k(dense) (2X - D) */
    int32_t g2_max;        /* plane waves: integer G with |G|^2 <= g2_max */
    int32_t q0_quad;       /* midpoint points per axis for the q -> 0 average of W */
} bse_kernel_model;

/* Library version string (static storage). */
const char* bse_version(void);

/* Message of the last error on this thread ("" if none). */
const char* bse_last_error(void);

/* Bytes of device workspace a plan for dims needs (0 if dims is invalid).
 * The workspace must be 256-byte aligned. */
size_t bse_workspace_bytes(const bse_dims* dims);

/* Bytes of one coarse kernel (Nc x Nc complex; FP32 for the low-precision forms,
 * whose block-scaled copy lives in the plan's workspace) and of the overlap array. */
size_t bse_coarse_kernel_bytes(const bse_dims* dims);
size_t bse_overlaps_bytes(const bse_dims* dims);

/*
 * Overlaps d_{nk}^{n'k~} = <u_{n'k~} | u_{nk}> between each dense point and its
 * 8 coarse corners (Sec. 3, Eq. completeness); only valence-valence and
 * conduction-conduction blocks (Eq. expansion).
 *   vecs_coarse  device, complex FP64 [n_coarse^3][nv+nc][n_orb]: coefficient a of
 *                band n at coarse point k~ (bands 0..nv-1 valence, then nc conduction)
 *   vecs_dense   device, complex FP64 [N_k(dense)][nv+nc][n_orb], same layout
 *   d_out        device, storage precision of dims->dtype, bse_overlaps_bytes(dims)
 *                bytes, layout [cell][z][e][sub] with e < nv^2 the valence block
 *                Dv[v][n1] at e = v nv + n1 and e >= nv^2 the conduction block
 *                Dc[c][n2] at e = nv^2 + c nc + n2 (n1, n2 index coarse bands).
 */
bse_status bse_build_overlaps(const bse_dims* dims, const double* vecs_coarse,
                              const double* vecs_dense, void* d_out, hipStream_t stream);

/*
 * Diagonal of Eq. (bse1): delta[t] = eps_{c kd} - eps_{v kd} (FP64).
 *   eps_dense  device FP64 [N_k(dense)][nv+nc] band energies (scissor included)
 *   delta_out  device FP64 [N]
 */
bse_status bse_build_transition_energies(const bse_dims* dims, const double* eps_dense,
                                         double* delta_out, hipStream_t stream);

/*
 * Coarse kernel K_c = kernel_energy / N_k(dense) (2 X - D) (Eqs. bse2, bse3a, bse3b),
 * for point-like orbitals at reduced positions tau in a cubic cell of lattice
 * constant 1, pair densities M_nm(k,k';Q) = sum_a conj(c_{nk,a}) c_{mk',a}
 * exp(i 2 pi Q.tau_a), exchange X over G != 0 with v = 4 pi / |2 pi G|^2 and
 * direct term D with W = 4 pi / (eps_inf |2 pi (q + G)|^2 + lambda^2),
 * q = k~ - k~' folded into [-1/2, 1/2) per axis, W at q = G = 0 replaced by its
 * mean over the dense mini-cell.  Block (k~, k~') is evaluated for k~ <= k~', its
 * mirror is the conjugate transpose and diagonal blocks are (A + A^H)/2, so the
 * result is exactly Hermitian.
 *   vecs_coarse  device, complex FP64 [n_coarse^3][nv+nc][n_orb]
 *   tau          device FP64 [n_orb][3]
 *   Kc_out       device, storage precision, row-major Nc x Nc complex
 */
bse_status bse_build_coarse_kernel(const bse_dims* dims, const double* vecs_coarse,
                                   const double* tau, const bse_kernel_model* model,
                                   void* Kc_out, hipStream_t stream);

/*
 * Plan: binds the inputs of the interpolated Hamiltonian H^i = diag(delta) + K^i
 * (Eqs. bse1, interp1) and a workspace.  The arrays are referenced, not copied:
 * they must stay valid and unchanged while the plan is used.
 *   Kc         device, Nc x Nc complex (storage precision), row-major, Hermitian:
 *              the product reads it by columns and uses Kc[j][i] = conj(Kc[i][j])
 *   d          device, overlaps in the layout of bse_build_overlaps
 *   delta      device FP64 [N]
 *   workspace  device, >= bse_workspace_bytes(dims) bytes, 256-byte aligned; owned
 *              by the plan until bse_plan_destroy; its contents need no
 *              initialisation; one plan must not run on two streams at once.
 *              Besides scratch space it holds the restrict tiles: a copy of d
 *              re-ordered for the restrict kernel, with the valence blocks already
 *              multiplied by the prefactors f (Sec. 3); for BSE_BF16_KC and
 *              BSE_F16_KC also the block-scaled copy of Kc, and for BSE_F32,
 *              BSE_F32_VEC64 and BSE_F64 the packed copy of its 128 x 128 tiles on and
 *              above the diagonal (Kc itself is then not read after plan creation unless
 *              bse_plan_set_coarse_product selects the full stream).
 *   stream     the copies are written by kernels enqueued on this stream; later
 *              calls on the plan must be ordered after them (same stream, or
 *              synchronised).
 * Band counts: any nv, nc with nv + nc <= 16 and nv nc <= 32 (else BSE_ERR_UNSUPPORTED).
 * The pairs (1,1) (1,2) (2,2) (2,3) (3,3) (3,4) (3,6) (4,6) run tuned kernels with the
 * counts fixed at compile time; any other pair runs general kernels that take them at
 * run time (FP64 arithmetic, slower), the Method 3 band product included.
 */
bse_status bse_plan_create(const bse_dims* dims, const void* Kc, const void* d,
                           const double* delta, void* workspace, size_t workspace_bytes,
                           hipStream_t stream, bse_plan** plan_out);
void bse_plan_destroy(bse_plan* plan);

/*
 * y = H^i x for n_rhs right-hand sides (Eq. bse1 diagonal plus Eqs. matmul1-matmul3:
 * restrict onto per-(cell, corner) coarse vectors, collapse them onto coarse
 * points, multiply by K_c, prolong back with the diagonal added).
 *   x, y   device, storage precision of the Lanczos vectors, N x n_rhs; x != y
 *   n_rhs  1 .. max_rhs
 */
bse_status bse_interp_matvec(bse_plan* plan, const void* x, void* y, int32_t n_rhs,
                             hipStream_t stream);

/*
 * Haydock-Lanczos chains (Eqs. ai-ci), one per right-hand side, all steps on
 * the device without host synchronisation: b_1 = 0, psi_1 = P/||P||, then
 * w = H psi_i - b_i psi_{i-1}, a_i = Re<psi_i|w>, b_{i+1} = ||w - a_i psi_i||,
 * psi_{i+1} = (w - a_i psi_i) / b_{i+1}.  Scalars in FP64.
 *   P          device, complex FP64, N x n_rhs (oscillator matrix elements, Eq. epsmacro)
 *   n_steps    chain length m >= 1
 *   a          device FP64 [n_rhs][n_steps]:   a[r*n_steps + i] = a_{i+1}
 *   b          device FP64 [n_rhs][n_steps+1]: b[r*(n_steps+1) + i] = b_{i+1}, b_1 = 0
 *   pnorm2     device FP64 [n_rhs]: ||P||^2
 *   steps_done device int32 [n_rhs]: valid a_i per chain
 *   status     device int32 [n_rhs]: BSE_OK, BSE_INFO_INVARIANT_SUBSPACE (b_{i+1} <=
 *              tol ||w||, the chain stops there), BSE_INFO_ZERO_START or
 *              BSE_ERR_NONFINITE; coefficients past steps_done are 0.
 */
bse_status bse_haydock_run(bse_plan* plan, const double* P, int32_t n_rhs, int32_t n_steps,
                           double* a, double* b, double* pnorm2, int32_t* steps_done,
                           int32_t* status, hipStream_t stream);

/*
 * Haydock chains run until their spectrum has converged (Sec. 2 after Eq. fraccont: the
 * recursion stops when eps_M(omega) is converged at each frequency).  The chains advance
 * as in bse_haydock_run; after every check_every steps a kernel evaluates eps_M of each
 * chain on the omega grid (Eq. fraccont, z = omega + i eta) and compares eps2 = Im eps_M
 * with the previous check: a chain stops (status BSE_OK, steps_done = its steps) once
 * max_omega |eps2 - eps2_previous| <= tol max_omega |eps2| (the paper gives 1% without a
 * denominator; here the change is measured against the spectrum's largest value), or
 * after max_steps steps.  Breakdown and zero start end a chain as in bse_haydock_run.
 * The fraction of each check is truncated after a_m (Eq. fraccont) unless
 * bse_plan_set_converge_closure selects the constant-chain closure.
 *   P, a, b, pnorm2, steps_done, status   as bse_haydock_run with n_steps = max_steps
 *                                          (lda = max_steps, ldb = max_steps + 1)
 *   omega      device FP64 [n_omega]
 *   eps_re, eps_im  device FP64 [n_rhs][n_omega]: eps_M of the last check (the converged
 *              spectrum), also the previous spectrum between checks
 * The host reads one flag per chain at each check while the first 4 steps of the next
 * chunk run, so at most 4 steps past the convergence of the last chain are enqueued (they
 * leave the stopped chains unchanged).  The call returns after the stream has finished the
 * run.
 */
bse_status bse_haydock_converge(bse_plan* plan, const double* P, int32_t n_rhs, int32_t max_steps,
                                int32_t check_every, double prefactor, const double* omega,
                                int32_t n_omega, double eta, double tol, double* a, double* b,
                                double* pnorm2, int32_t* steps_done, int32_t* status, double* eps_re,
                                double* eps_im, hipStream_t stream);

/*
 * eps_M(omega) = 1 - prefactor ||P||^2 / (z - a_1 - b_2^2 / (z - a_2 - ...)),
 * z = omega + i eta, truncated after a_m with m = steps[chain] (Eq. fraccont).
 * All pointers device; chains are stored with leading dimensions lda (a) and
 * ldb (b) as returned by bse_haydock_run (lda = n_steps, ldb = n_steps + 1).
 *   eps_re, eps_im  device FP64 [n_chains][n_omega]
 */
bse_status bse_continued_fraction(const double* a, const double* b, int32_t lda, int32_t ldb,
                                  const double* pnorm2, const int32_t* steps,
                                  int32_t n_chains, double prefactor, const double* omega,
                                  int32_t n_omega, double eta, double* eps_re, double* eps_im,
                                  hipStream_t stream);

/* Kernel timing: with enable = 1 the plan records HIP events around every launch
 * of the coarse product (the dominant kernel of Method 1: the split product and
 * the kernel that adds its splits) on the stream it is launched on; with enable = 3
 * it times the product's streaming kernel alone, by launching it with an event pair
 * that the runtime stamps with that kernel's own start and end (hipExtLaunchKernel);
 * with enable = 2 around every launch of the Method 3 band product instead;
 * 0 turns timing off.
 * bse_plan_get_timing synchronises those events and returns the total time in
 * milliseconds and the number of timed launches since the last reset. */
bse_status bse_plan_set_timing(bse_plan* plan, int32_t enable);
bse_status bse_plan_get_timing(bse_plan* plan, double* total_ms, int64_t* launches);

/*
 * Batched chains: one Haydock run (Eqs. ai-ci, as bse_haydock_run with n_steps
 * steps) per plan, for many plans of any sizes, recorded once into HIP graphs and
 * submitted by a single call.  Plan i starts from P[i] (n_rhs[i] right-hand
 * sides) and writes a[i], b[i], pnorm2[i], steps_done[i], status[i] with the
 * layouts of bse_haydock_run.  The runs are dealt to n_branches (1..16) branches,
 * largest first; each branch is recorded once into its own HIP graph.  A launch
 * forks `stream` onto the batch's own streams (default priority), launches every
 * branch's graph there and joins back into `stream`, so small Hamiltonians run
 * beside large ones.  All pointers are recorded in the graphs: they, the plans and
 * their inputs must stay valid and unchanged until bse_batch_destroy, which must
 * come after the last launch has completed; a plan may appear once, must have
 * kernel timing disabled, and must not be used elsewhere while a launch runs.
 * Every launch recomputes all chains from their starts.
 */
typedef struct bse_batch bse_batch;
bse_status bse_batch_create(bse_plan* const* plans, int32_t n_plans, const double* const* P,
                            const int32_t* n_rhs, int32_t n_steps, double* const* a,
                            double* const* b, double* const* pnorm2, int32_t* const* steps_done,
                            int32_t* const* status, int32_t n_branches, bse_batch** batch_out);
bse_status bse_batch_launch(bse_batch* batch, hipStream_t stream);
void bse_batch_destroy(bse_batch* batch);

/* ---- Learned continued-fraction terminator -------------------------------------
 * The paper leaves the tail of Eq. (fraccont) open (the chain is run until the
 * spectrum has converged).  These calls serve a small dense network that predicts
 * the coefficients after the first m from the first m, and the continued fraction
 * closed by a constant tail.  All arrays are device pointers, row-major.
 *
 * Dense layer y = act(x W^T + b): x [batch][n_in], W [n_out][n_in], b [n_out],
 * z and y [batch][n_out] (FP32).  act: BSE_ACT_NONE, or BSE_ACT_GELU (the exact
 * z Phi(z) form).  z receives the pre-activation (may be NULL when y is given and
 * no backward pass follows); y may be NULL when z is given.
 */
typedef enum { BSE_ACT_NONE = 0, BSE_ACT_GELU = 1 } bse_act;
bse_status bse_dense_forward(const float* x, const float* W, const float* b, float* z, float* y,
                             int32_t batch, int32_t n_in, int32_t n_out, int32_t act,
                             hipStream_t stream);

/* Backward pass of the same layer for a scalar loss L with dL/dy = dy:
 * dW = dz^T x, db = column sums of dz, dx = dz W (skipped when dx is NULL), with
 * dz = dy * act'(z) written to work [batch][n_out] (caller-owned scratch). */
bse_status bse_dense_backward(const float* x, const float* W, const float* z, const float* dy,
                              float* dx, float* dW, float* db, int32_t batch, int32_t n_in,
                              int32_t n_out, int32_t act, float* work, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the same backward pass as
 * bse_dense_backward without the caller's `work` buffer.  dz lives in a scratch array
 * the library holds in device memory, one per device, from the first call on that
 * device until the process ends (4 MiB: batch * n_out <= 2^20 entries; larger calls
 * return BSE_ERR_WORKSPACE before any launch).  The call allocates nothing.  Every call
 * on one device shares that device's array: calls that overlap on one device (two
 * streams, or two threads) race and must be ordered by the caller.  Results equal
 * bse_dense_backward's bit for bit (same kernels, same order). */
bse_status bse_dense_backward_noalloc(const float* x, const float* W, const float* z, const float* dy,
                                      float* dx, float* dW, float* db, int32_t batch, int32_t n_in,
                                      int32_t n_out, int32_t act, hipStream_t stream);

/* Mean squared error over n entries: *loss = mean (y - t)^2 (FP64, fixed-order
 * sum, one device double) and dy = 2 (y - t) / n (skipped when dy is NULL). */
bse_status bse_mse_loss(const float* y, const float* t, float* dy, double* loss, int64_t n,
                        hipStream_t stream);

/* One Adam update (Kingma and Ba, Alg. 1) of n parameters p with gradient g and
 * moments m, v (updated in place); t >= 1 is the step count for the bias correction. */
bse_status bse_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                         float beta1, float beta2, float eps, int32_t t, hipStream_t stream);

/* FP32 -> BF16 (round to nearest even), n entries; y holds the 16-bit patterns. */
bse_status bse_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t stream);

/* Inference layer on the matrix cores: x [batch][n_in] and W [n_out][n_in] in BF16
 * (16-byte aligned, n_in a multiple of 32), FP32 accumulation, y = act(x W^T + b)
 * written as BF16 (y_bf16, the next layer's input) and/or FP32 (y_f32). */
bse_status bse_dense_forward_bf16(const uint16_t* x, const uint16_t* W, const float* b,
                                  uint16_t* y_bf16, float* y_f32, int32_t batch, int32_t n_in,
                                  int32_t n_out, int32_t act, hipStream_t stream);

/* eps_M (Eq. fraccont) from the first m coefficients a_1..a_m, b_1..b_{m+1} of each
 * chain (rows of a [n_chains][lda], b [n_chains][ldb]) closed by the constant chain
 * (a_inf, b_inf) of that chain: t_m = z - a_m - b_{m+1}^2 g(z) with g the root of
 * b_inf^2 g^2 - (z - a_inf) g + 1 = 0 that has Im g <= 0, then t_i = z - a_i -
 * b_{i+1}^2 / t_{i+1} and eps_M = 1 - prefactor ||P||^2 / t_1.  eta > 0. */
bse_status bse_continued_fraction_terminated(const double* a, const double* b, int32_t lda,
                                             int32_t ldb, int32_t m, const double* pnorm2,
                                             const double* a_inf, const double* b_inf,
                                             int32_t n_chains, double prefactor, const double* omega,
                                             int32_t n_omega, double eta, double* eps_re,
                                             double* eps_im, hipStream_t stream);

/* ---- Method 3: the divergence treated in a band along the diagonal (Sec. 4) ------
 * Dense pairs with ||k - k'|| <= w d (d = 1 / n_coarse, the smallest distance between
 * coarse points; reduced coordinates of the cubic cell, minimum image) take the
 * coefficients of Eq. (diverg) interpolated like K_c (Eq. interp1) and combined with
 * the dense-mesh q; all other pairs keep Method 1.  For the model kernel of
 * bse_build_coarse_kernel the divergent part is the G = 0 direct term:
 * K_c = a_c s(q) + c_c with s(q) = 1 / (|q|^2 + kappa^2), kappa^2 = lambda^2 /
 * (4 pi^2 eps_inf), q reduced (the screened form of a / q^2; b = 0 because W is
 * diagonal in G), and s at q = 0 replaced by its mean over the dense mini-cell
 * (midpoint rule, q0_quad points per axis), as W is in K_c.  Inside the band
 *   K^{M3}(k, k') = interp(a_c)(k, k') s(k - k') + interp(K_c - a_c S_c)(k, k'),
 * i.e. the Method 1 kernel plus a block Delta(k, k + o) per dense point k and band
 * offset o (integer offsets of the dense mesh with |o|^2 <= (w n_div)^2). */

/* a_c (same layout and precision as K_c of bse_build_coarse_kernel): the coarse
 * coefficient of s(q), -kernel_energy / N_k(dense) / (pi eps_inf) M_cc'(k~,k~';q)
 * conj(M_vv'(k~,k~';q)) with the Hermitian construction of K_c. */
bse_status bse_build_divergence_coefficient(const bse_dims* dims, const double* vecs_coarse,
                                            const double* tau, const bse_kernel_model* model,
                                            void* a_out, hipStream_t stream);

/* Number of band offsets for width w >= 0 and the bytes of the band buffer for dims
 * (BSE_ERR_INVALID_ARG when floor(w n_div) > 16, when 2 floor(w n_div) reaches the
 * dense mesh n_coarse n_div, or when nv nc > 32 or nv^2 + nc^2 > 52). */
bse_status bse_m3_band_info(const bse_dims* dims, double w, int32_t* n_offsets, size_t* band_bytes);

/* Builds the band: the blocks Delta(k, k + o) from the overlaps d (layout of
 * bse_build_overlaps), a_c and the model's eps_inf, lambda and q0_quad, in the
 * storage precision of dims->dtype (FP64 for BSE_F64, FP32 otherwise), FP64
 * arithmetic.  band: device, 256-byte aligned, >= band_bytes of bse_m3_band_info;
 * it holds the offset table, the blocks and the scratch of the band product (one
 * FP64 complex vector per right-hand side), so one band serves one plan at a time.
 * The kernels are enqueued on `stream`. */
bse_status bse_build_m3_band(const bse_dims* dims, const void* d, const void* a_coef,
                             const bse_kernel_model* model, double w, void* band,
                             size_t band_bytes, hipStream_t stream);

/* Attaches a band built for the plan's dims and this w (band = NULL detaches it).
 * From then on bse_interp_matvec and bse_haydock_run (and batches recorded later)
 * apply H^{M3} = diag(delta) + K^i + Delta: before the prolong, a kernel forms
 * y_k = sum_o Delta(k, k + o) x_{k+o} in FP64, and the prolong adds it.  The band
 * must stay valid while the plan uses it.  BSE_ERR_UNSUPPORTED for band counts beyond
 * the builder's (nv nc > 32 or nv^2 + nc^2 > 52). */
bse_status bse_plan_set_m3_band(bse_plan* plan, void* band, double w);

/* Tunables of the coarse product: column splits (0 = automatic).  For sweeps. */
bse_status bse_plan_set_gemv_splits(bse_plan* plan, int32_t n_split);

/* Coarse product of Eq. (matmul2) for the FP32 and FP64 coarse kernels (BSE_F32,
 * BSE_F32_VEC64, BSE_F64): form 0 (default) reads the plan's packed copy of the tiles on
 * and above the diagonal (K_c is Hermitian, Eqs. bse1-bse2: half the bytes); for FP32
 * with FP32 products and FP32 sums over runs of 16 tile columns (32 rows for the
 * conjugate-transposed tiles) added in FP64, for FP64 in FP64 throughout.  Form 1 streams
 * the whole Kc with FP64 products and sums.  For the block-scaled forms (BSE_BF16_KC,
 * BSE_F16_KC) form 0 reads only the 64 x 64 blocks on and above the diagonal and forms
 * both products on the matrix cores (the column product through a transposed LDS copy of
 * each block), form 1 every block.  For comparisons and sweeps. */
bse_status bse_plan_set_coarse_product(bse_plan* plan, int32_t form);

/* Tail of the continued fraction in bse_haydock_converge.  k = 0 (default): truncated
 * after a_m, as Eq. (fraccont) is written.  1 <= k <= 64: closed beyond a_m by a chain
 * with constant coefficients a_inf = mean(a_{m-k+1} .. a_m), b_inf = mean(b_{m-k+2} ..
 * b_{m+1}) of the chain's own last k steps, whose resolvent is the root of
 * b_inf^2 g^2 - (z - a_inf) g + 1 = 0 with Im g <= 0 (the standard square-root closure
 * of a Lanczos fraction; the paper leaves the tail open): t_m = z - a_m - b_{m+1}^2 g.
 * Both the stop rule and the returned spectrum then use the closed fraction; a check
 * with m < k uses the truncated one.  BSE_ERR_INVALID_ARG for other k. */
bse_status bse_plan_set_converge_closure(bse_plan* plan, int32_t k);

/* Tunable of the restrict (Eq. matmul1): right-hand sides handled by one block, 1
 * (default) or 3 (used only when a call has exactly three right-hand sides).  Both
 * give the same results; only the speed differs.  For sweeps. */
bse_status bse_plan_set_restrict_group(bse_plan* plan, int32_t rhs_per_block);

#ifdef __cplusplus
}
#endif

#endif /* BSE_DG_H */
