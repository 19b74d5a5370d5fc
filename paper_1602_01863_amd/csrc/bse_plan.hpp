// Host-side plan, workspace layout and launch interface of the BSE library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "bse_dg.h"

namespace bse {

constexpr int kMaxRhs = 4;
constexpr int kMaxSplit = 64;        // column splits of the coarse product
constexpr int kConvBlocks = 64;      // blocks per chain of the convergence check (at most)
constexpr int kConvAhead = 4;        // chain steps enqueued past a convergence check before its flags are read
constexpr int kBlock = 256;          // threads of the reduction / product blocks

// Per-chain Lanczos state kept on the device between kernels.  The chain stores
// unnormalised vectors u_j with psi_j = s_j u_j; the scales live here.  Two copies
// alternate between steps: the kernels of step i read copy i % 2 and the last kernel
// of the step (the collapse) writes copy (i + 1) % 2, so no kernel reads a field that
// another block of the same kernel writes.
struct ChainState {
    double s_cur;   // scale of the buffer holding psi_i (1 / b_i; 1 / ||u_1|| for i = 1)
    double s_prev;  // scale of the buffer holding psi_{i-1}
    double b_cur;   // b_i (0 for i = 1)
    double pnorm2;  // ||P||^2
    int32_t active;
    int32_t steps;
    int32_t status;
    int32_t pad;
};

// a_i and ||w||^2 of the current step, recorded by the restrict for the collapse
struct StepScalars {
    double a;
    double ww;
    int32_t ok;   // chain active and both values finite
    int32_t pad[3];
};

struct Geometry {
    int n_c, n_div, ndiv3, ncells, nv, nc, np, ne, neighbours, dtype, n_orb_input;
    int64_t nk, N, Nc;
    int max_rhs;
};

bool make_geometry(const bse_dims* d, Geometry* g);

// Restrict tiles: the overlaps re-ordered for the restrict's lanes (see restrict.hip).
// Tile (cell, s) covers subpoints 4 s .. 4 s + 3 of the cell; every lane of the
// wavefront owns kp entries, stored as 16-byte units.
struct SwzShape {
    int ndv;   // valence-block entries per lane (half of nv^2, rounded up)
    int nch;   // conduction columns n2 per lane (half of nc, rounded up)
    int kl;    // entries per lane: ndv + nc * nch
    int unit;  // complex entries per 16-byte unit (2 for FP32, 1 for FP64 storage)
    int kp;    // kl rounded up to a multiple of unit
    int S;     // tiles per cell: ceil(n_div^3 / 4)
};
__host__ __device__ inline SwzShape swz_shape(int nv, int nc, int ndiv3, int elem_bytes) {
    SwzShape z;
    z.ndv = (nv * nv + 1) / 2;
    z.nch = (nc + 1) / 2;
    z.kl = z.ndv + nc * z.nch;
    z.unit = 16 / elem_bytes;
    z.kp = (z.kl + z.unit - 1) / z.unit * z.unit;
    z.S = (ndiv3 + 3) / 4;
    return z;
}

// Low-precision coarse kernel (BSE_BF16_KC, BSE_F16_KC): 64 x 64 blocks, one FP32
// scale each; the coarse index padded with zeros to a multiple of 64.  qbar enters the
// matrix-core product as fragments for 32-column steps (see gemv.hip).
constexpr int kKqBlock = 64;
struct KqShape {
    int nb;     // blocks per side: ceil(Nc / 64)
    int nstep;  // 32-column steps: 2 nb
};
inline KqShape kq_shape(int64_t Nc) {
    KqShape k;
    k.nb = (int)((Nc + kKqBlock - 1) / kKqBlock);
    k.nstep = 2 * k.nb;
    return k;
}
inline bool kc_lowp(int dtype) { return dtype == BSE_BF16_KC || dtype == BSE_F16_KC; }
// Packed Hermitian form of the block-scaled product (gemv.hip): runs of block columns over
// bands of two block rows, blocks (bi, bj) with bi <= bj only; one wavefront per run
struct HmShape {
    int nb;         // blocks per side
    int bands;      // bands of two block rows: ceil(nb / 2)
    int run_len;    // block columns per run
    int64_t runs;   // runs over all bands
    int64_t p2;     // column partials: one per (band, column block) right of the band
};
HmShape hm_shape(int64_t Nc);
// Lanczos vectors in FP32 storage
inline bool vec_is_f32(int dtype) { return dtype == BSE_F32 || kc_lowp(dtype); }

// Packed Hermitian coarse product (FP32 or FP64 coarse kernel): 128 x 128 tiles on and above the
// diagonal, their partial sums and the block table (see gemv.hip)
struct HemvShape {
    int nbk;            // tile rows: ceil(Nc / 128)
    int64_t tiles;      // nbk (nbk + 1) / 2
    int tpw;            // tiles each wavefront streams in turn (gemv.hip)
    int64_t blocks;     // groups of 2 tpw consecutive tiles of one tile row
    size_t elem_bytes;  // one complex entry (and one partial): FP32 or FP64
    size_t tile_bytes;  // 128 x 128 complex entries
};
HemvShape hemv_shape(int64_t Nc, int dtype);
inline bool kc_packable(int dtype) { return dtype == BSE_F32 || dtype == BSE_F32_VEC64 || dtype == BSE_F64; }

// workspace regions (byte offsets from the workspace base); dsw_bytes == 0 when the
// restrict reads the overlaps in their input layout; kq, kscale, qfrag, qsinv (the FP16
// form's qbar scales) and mp1, mp2, mtab (partials and run table of their packed product)
// only for the low-precision forms; kp, hpart, htab only for the FP32 and FP64 coarse kernels
struct Layout {
    size_t qpart, qbar, rvec, gpart, ppart, rpart, chain, pend, flags, cpart, vec_a, vec_b, dsw, kq, kscale, qfrag, qsinv, kp,
        hpart, htab, mp1, mp2, mtab;
    size_t dsw_bytes, kq_bytes, kscale_bytes, qfrag_bytes, kp_bytes;
    size_t total;
};
Layout make_layout(const Geometry& g);

struct Plan {
    Geometry g;
    Layout L;
    const void* Kc;
    const void* d;
    const double* delta;
    char* ws;
    int n_split;  // 0 = automatic
    int product_form;  // coarse product of the FP32/FP64 coarse kernel: 0 packed Hermitian tiles, 1 full stream
    int restrict_group;  // right-hand sides per restrict block (1, or 3 for three)
    // kernel timing: 0 off, 1 the coarse product, 2 the Method 3 band product, 3 the coarse
    // product's streaming kernel alone
    int timing;
    int ev_used;
    double timed_ms;
    int64_t timed_launches;
    hipEvent_t* ev;
    int ev_cap;
    hipEvent_t split_start, split_ev;   // timing mode 3: the pair the streaming kernel's launch stamps
    // Method 3 band (m3.hip); m3_band == nullptr: Method 1 only
    const char* m3_band;  // caller's band buffer: offset table, then the blocks
    double2* m3_yb;       // band product [rhs][N] (FP64), the tail of the band buffer
    int m3_noff_pad;      // band offsets, padded to whole chunks
    // chains run to convergence: a side stream for reading the check flags, two events,
    // and the tail of the checked fraction (0 truncated, k: constant chain of the last k)
    hipStream_t side;
    hipEvent_t chk[2];
    int converge_closure;
};

// launches implemented in hotpath.hip (return hipSuccess or the launch error)
hipError_t launch_restrict(const Plan& p, int mode, const void* x, const void* w, const void* psi,
                           const double* P, void* out, int step, double* a, double* b, int lda, int ldb,
                           int n_rhs, hipStream_t s);
hipError_t launch_collapse(const Plan& p, int mode, int step, double* b, int ldb, int n_rhs, hipStream_t s);
hipError_t launch_gemv(Plan& p, int n_rhs, hipStream_t s);
hipError_t launch_prolong(const Plan& p, int mode, const void* x, void* out_prev, int step, int n_rhs,
                          hipStream_t s);
hipError_t launch_chain_report(const Plan& p, int n_steps, double* pnorm2, int32_t* steps, int32_t* status,
                               int n_rhs, hipStream_t s);
bool supported_bands(int nv, int nc);

// Method 3 band product y_band = Band x (m3.hip), before the prolong, which adds it
hipError_t launch_m3_apply(Plan& p, const void* x, int n_rhs, hipStream_t s);

// restrict tiles from the overlaps (restrict.hip), enqueued at plan creation
hipError_t launch_swizzle(const Plan& p, hipStream_t s);
// block-scaled coarse kernel and cleared qbar fragments (gemv.hip), at plan creation
hipError_t launch_quantize(const Plan& p, hipStream_t s);
// packed Hermitian tiles and their block table (gemv.hip), at plan creation
hipError_t launch_hemv_pack(const Plan& p, hipStream_t s);
inline bool use_packed(const Plan& p) { return p.L.kp_bytes > 0 && p.product_form == 0; }
inline bool use_packed_lowp(const Plan& p) { return kc_lowp(p.g.dtype) && p.product_form == 0; }
// vector slice of a cell held in LDS by the tiled restrict: bytes, or 0 if it does not fit
size_t restrict_tile_lds(const Geometry& g);

// setup launches implemented in setup.hip
hipError_t launch_overlaps(const Geometry& g, const double* vc, const double* vd, void* dout, hipStream_t s);
hipError_t launch_transition_energies(const Geometry& g, const double* eps, double* out, hipStream_t s);
hipError_t launch_coarse_kernel(const Geometry& g, const double* vecs, const double* tau,
                                const bse_kernel_model& m, void* K, hipStream_t s);
hipError_t launch_divergence_coefficient(const Geometry& g, const double* vecs, const double* tau,
                                         const bse_kernel_model& m, void* A, hipStream_t s);
hipError_t launch_continued_fraction(const double* a, const double* b, int lda, int ldb, const double* pnorm2,
                                     const int32_t* steps, int n_chains, double prefactor, const double* omega,
                                     int n_omega, double eta, double* eps_re, double* eps_im, hipStream_t s);

// band pairs (nv, nc) compiled into the hot-path kernels
#define BSE_BANDS(X) X(1, 1) X(1, 2) X(2, 2) X(2, 3) X(3, 3) X(3, 4) X(3, 6) X(4, 6)

// per-precision, per-band launchers (restrict.hip, prolong.hip)
template <class M2, class V2, int NV, int NC>
hipError_t restrict_launch(const Plan& p, int mode, const void* x, const void* w, const void* psi, const double* P,
                           void* out, int step, double* a, double* b, int lda, int ldb, int n_rhs, hipStream_t s);
template <class M2, class V2, int NV, int NC>
hipError_t prolong_launch(const Plan& p, int mode, const void* x, void* out, int step, int n_rhs, hipStream_t s);
// band pairs without a compiled form: nv, nc at run time (restrict.hip, prolong.hip)
template <class M2, class V2>
hipError_t restrict_any_launch(const Plan& p, int mode, const void* x, const void* w, const void* psi, const double* P,
                               void* out, int step, double* a, double* b, int lda, int ldb, int n_rhs, hipStream_t s);
template <class M2, class V2>
hipError_t prolong_any_launch(const Plan& p, int mode, const void* x, void* out, int step, int n_rhs, hipStream_t s);
// band counts the hot path takes: the compiled pairs at full speed, any other pair with
// nv + nc <= 16 and nv nc <= 32 through the run-time forms
inline bool bands_in_range(int nv, int nc) { return nv >= 1 && nc >= 1 && nv + nc <= 16 && nv * nc <= 32; }

// chain-state copy read by the kernels of a step, written by its collapse
__host__ __device__ inline int state_in(int step) { return step & 1; }
__host__ __device__ inline int state_out(int step) { return (step + 1) & 1; }
// breakdown threshold: b_{i+1} <= tol ||w||, by vector storage precision
inline double breakdown_tol(int dtype) { return vec_is_f32(dtype) ? 1e-6 : 1e-12; }

// modes of the restrict launch
enum { RESTRICT_PLAIN = 0, RESTRICT_UPDATE = 1, RESTRICT_INIT = 2 };
// modes of the collapse launch
enum { COLLAPSE_PLAIN = 0, COLLAPSE_INIT = 1, COLLAPSE_STEP = 2 };
// modes of the prolong launch
enum { PROLONG_PLAIN = 0, PROLONG_LANCZOS = 1 };

void set_error(const char* fmt, ...);
// every launch of one Haydock run (Eqs. ai-ci) on `stream`, as bse_haydock_run
hipError_t enqueue_haydock(Plan& p, const double* P, int n_rhs, int n_steps, double* a, double* b, double* pnorm2,
                           int32_t* steps_done, int32_t* status, hipStream_t stream);
bse_status hip_fail_status(hipError_t e, const char* what);
// bytes of shared memory (static + dynamic) one block may use on the current device
size_t lds_limit();
// compute units of the current device
int cu_count();

}  // namespace bse
