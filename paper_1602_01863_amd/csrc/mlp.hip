// Kernels of the learned continued-fraction terminator: a small dense network trained
// and evaluated on the device, and the continued fraction closed by a constant tail.
//
// Training (FP32): dense layers y = act(x W^T + b) with a tiled GEMM (64 x 64 output
// tiles, 16-deep K steps staged in LDS, 4 x 4 outputs per thread), GELU in its exact
// erf form, the mean squared error with a fixed-order reduction, and Adam.  Inference
// (BF16): x and W in BF16 on the 16x16x32 matrix cores with FP32 accumulation.  No
// kernel uses atomics: every result has one writer and sums run in a fixed order.

#include <hip/hip_runtime.h>

#include <math.h>

#include <mutex>

#include "bse_device.hpp"
#include "bse_plan.hpp"

namespace bse {

constexpr int kTile = 64;   // output tile per block
constexpr int kKStep = 16;  // K per LDS stage

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// C[M][N] = sum_k A(m, k) B(k, n) (+ bias[n]) ; A(m, k) = TA ? A[k][M] : A[m][K];
// B(k, n) = TB ? B[n][K] : B[k][N].  Epilogue: Z = C + bias (stored if Z != null),
// Y = act(Z).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, const float* __restrict__ B,
                                              const float* __restrict__ bias, float* __restrict__ Z,
                                              float* __restrict__ Y, int M, int N, int K, int act) {
    __shared__ float As[kKStep][kTile + 1];
    __shared__ float Bs[kKStep][kTile + 1];
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int t = threadIdx.x;
    const int tm = (t / 16) * 4, tn = (t % 16) * 4;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += kKStep) {
        // stage a 16 x 64 slice of A and of B (4 entries per thread each), zero past the edges
        for (int i = t; i < kKStep * kTile; i += 256) {
            const int kk = i / kTile, mm = i % kTile;
            const int k = k0 + kk, m = m0 + mm, n = n0 + mm;
            As[kk][mm] = (k < K && m < M) ? (TA ? A[(int64_t)k * M + m] : A[(int64_t)m * K + k]) : 0.0f;
            Bs[kk][mm] = (k < K && n < N) ? (TB ? B[(int64_t)n * K + k] : B[(int64_t)k * N + n]) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKStep; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[kk][tm + i];
                b[i] = Bs[kk][tn + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + tm + i, n = n0 + tn + j;
            if (m >= M || n >= N) continue;
            const float z = acc[i][j] + (bias ? bias[n] : 0.0f);
            if (Z) Z[(int64_t)m * N + n] = z;
            if (Y) Y[(int64_t)m * N + n] = act == BSE_ACT_GELU ? gelu_f(z) : z;
        }
}

// dz = dy * act'(z)
__global__ __launch_bounds__(256) void k_act_grad(const float* __restrict__ z, const float* __restrict__ dy,
                                                  float* __restrict__ dz, int64_t n, int act) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dz[i] = act == BSE_ACT_GELU ? dy[i] * gelu_grad_f(z[i]) : dy[i];
}

// db[j] = sum over rows of dz[row][j], rows in order
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ dz, float* __restrict__ db, int rows,
                                                int cols) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.0f;
    for (int r = 0; r < rows; ++r) s += dz[(int64_t)r * cols + j];
    db[j] = s;
}

// one block: loss = mean (y - t)^2 (FP64 sums in a fixed tree), dy = 2 (y - t) / n
__global__ __launch_bounds__(1024) void k_mse(const float* __restrict__ y, const float* __restrict__ tg,
                                              float* __restrict__ dy, double* __restrict__ loss, int64_t n) {
    __shared__ double sred[1024 / kWave];
    double s = 0.0;
    const float scale = 2.0f / (float)n;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const float d = y[i] - tg[i];
        s += (double)d * (double)d;
        if (dy) dy[i] = scale * d;
    }
    s = block_sum(s, sred);
    if (threadIdx.x == 0) *loss = s / (double)n;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                              float beta1, float beta2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ x, unsigned short* __restrict__ y,
                                                 int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = enc_lowp(BSE_BF16_KC, x[i]);
}

// BF16 inference: one wavefront per 16 x 16 output tile, K in steps of 32 on the
// matrix cores (lane layouts as in the coarse product: A[m][k] in lane 16 (k / 8) + m,
// B[k][n] in lane 16 (k / 8) + n, D[m][n] in lane 16 (m / 4) + n, entry m % 4)
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_dense_bf16(const unsigned short* __restrict__ x,
                                                    const unsigned short* __restrict__ W,
                                                    const float* __restrict__ bias, unsigned short* __restrict__ yb,
                                                    float* __restrict__ yf, int B, int n_in, int n_out, int act) {
    const int wave = blockIdx.x * 4 + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int tiles_n = (n_out + 15) / 16;
    const int tm = wave / tiles_n, tn = wave % tiles_n;
    if (tm * 16 >= B) return;  // whole wavefront: uniform exit
    const int ma = tm * 16 + lane % 16;  // row of x this lane feeds
    const int nb = tn * 16 + lane % 16;  // row of W (output column) this lane feeds
    const int kq = 8 * (lane / 16);
    f32x4_t d = {0.0f, 0.0f, 0.0f, 0.0f};
    const u32x4_t zero = {0u, 0u, 0u, 0u};
    for (int k0 = 0; k0 < n_in; k0 += 32) {
        const u32x4_t a = ma < B ? *reinterpret_cast<const u32x4_t*>(x + (int64_t)ma * n_in + k0 + kq) : zero;
        const u32x4_t b = nb < n_out ? *reinterpret_cast<const u32x4_t*>(W + (int64_t)nb * n_in + k0 + kq) : zero;
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                    d, 0, 0, 0);
    }
    const int n = tn * 16 + lane % 16;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int m = tm * 16 + 4 * (lane / 16) + e;
        if (m >= B || n >= n_out) continue;
        float z = d[e] + bias[n];
        if (act == BSE_ACT_GELU) z = gelu_f(z);
        if (yf) yf[(int64_t)m * n_out + n] = z;
        if (yb) yb[(int64_t)m * n_out + n] = enc_lowp(BSE_BF16_KC, z);
    }
}

// eps_M from m coefficients closed by the constant chain (a_inf, b_inf) (see header)
__global__ __launch_bounds__(256) void k_cf_terminated(const double* __restrict__ a, const double* __restrict__ b,
                                                       int lda, int ldb, int m, const double* __restrict__ pnorm2,
                                                       const double* __restrict__ a_inf,
                                                       const double* __restrict__ b_inf, int n_chains,
                                                       double prefactor, const double* __restrict__ omega,
                                                       int n_omega, double eta, double* __restrict__ eps_re,
                                                       double* __restrict__ eps_im) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_chains * n_omega) return;
    const int ch = (int)(i / n_omega);
    const int w = (int)(i % n_omega);
    const double pn = pnorm2[ch];
    if (m <= 0 || pn == 0.0) {
        eps_re[i] = 1.0;
        eps_im[i] = 0.0;
        return;
    }
    const double zr = omega[w], zi = eta;
    const double* ac = a + (int64_t)ch * lda;
    const double* bc = b + (int64_t)ch * ldb;
    double gr, gi;
    constant_chain(zr, zi, a_inf[ch], b_inf[ch], gr, gi);
    const double bm2 = bc[m] * bc[m];
    // t_m = z - a_m - b_{m+1}^2 g_inf ; t_i = z - a_i - b_{i+1}^2 / t_{i+1}
    double tr = zr - ac[m - 1] - bm2 * gr, ti = zi - bm2 * gi;
    for (int k = m - 2; k >= 0; --k) {
        const double b2 = bc[k + 1] * bc[k + 1];
        const double den = tr * tr + ti * ti;
        const double qr = b2 * tr / den, qi = -b2 * ti / den;
        tr = zr - ac[k] - qr;
        ti = zi - qi;
    }
    const double den = tr * tr + ti * ti;
    const double c = prefactor * pn;
    eps_re[i] = 1.0 - c * tr / den;
    eps_im[i] = c * ti / den;
}

// ---- scratch of bse_dense_backward_noalloc --------------------------------------------
// dz = dy act'(z) of one call, in a file-scope device array instead of a caller buffer.
// Every device that runs the library holds its own copy until the process ends.  In
// host code the array's name is not a device address: host code uses only the address
// hipGetSymbolAddress returns for the current device (kept per device below).
constexpr int64_t kNoAllocMaxEntries = (int64_t)1 << 20;   // batch * n_out <= 2^20 (4 MiB)
static __device__ __align__(256) float scratch[kNoAllocMaxEntries];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once per device)
static hipError_t scratch_address(float** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// dz, dW, db and dx of the layer (see bse_dense_backward), dz in `work`
static hipError_t enqueue_dense_backward(const float* x, const float* W, const float* z, const float* dy, float* dx,
                                         float* dW, float* db, int batch, int n_in, int n_out, int act, float* work,
                                         hipStream_t stream) {
    const int64_t n = (int64_t)batch * n_out;
    hipLaunchKernelGGL(k_act_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, z, dy, work, n, act);
    // dW [n_out][n_in] = dz^T x ; db = column sums of dz ; dx [batch][n_in] = dz W
    hipLaunchKernelGGL((k_gemm<true, false>), dim3((n_in + kTile - 1) / kTile, (n_out + kTile - 1) / kTile), dim3(256),
                       0, stream, work, x, nullptr, nullptr, dW, n_out, n_in, batch, (int)BSE_ACT_NONE);
    hipLaunchKernelGGL(k_colsum, dim3((n_out + 255) / 256), dim3(256), 0, stream, work, db, batch, n_out);
    if (dx)
        hipLaunchKernelGGL((k_gemm<false, false>), dim3((n_in + kTile - 1) / kTile, (batch + kTile - 1) / kTile),
                           dim3(256), 0, stream, work, W, nullptr, nullptr, dx, batch, n_in, n_out, (int)BSE_ACT_NONE);
    return hipGetLastError();
}

static bool dense_backward_args_ok(const float* x, const float* W, const float* z, const float* dy, const float* dW,
                                   const float* db, int batch, int n_in, int n_out, int act) {
    return x && W && dy && dW && db && !(act == BSE_ACT_GELU && !z) && batch >= 1 && n_in >= 1 && n_out >= 1 &&
           (act == BSE_ACT_NONE || act == BSE_ACT_GELU);
}

}  // namespace bse

using namespace bse;

static bse_status fail(hipError_t e, const char* what) { return hip_fail_status(e, what); }

extern "C" {

bse_status bse_dense_forward(const float* x, const float* W, const float* b, float* z, float* y, int32_t batch,
                             int32_t n_in, int32_t n_out, int32_t act, hipStream_t stream) {
    if (!x || !W || !b || (!z && !y) || batch < 1 || n_in < 1 || n_out < 1 ||
        (act != BSE_ACT_NONE && act != BSE_ACT_GELU)) {
        set_error("bse_dense_forward: NULL array, empty size or unknown activation");
        return BSE_ERR_INVALID_ARG;
    }
    dim3 grid((n_out + kTile - 1) / kTile, (batch + kTile - 1) / kTile);
    hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, stream, x, W, b, z, y, batch, n_out, n_in, act);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BSE_OK : fail(e, "bse_dense_forward");
}

bse_status bse_dense_backward(const float* x, const float* W, const float* z, const float* dy, float* dx, float* dW,
                              float* db, int32_t batch, int32_t n_in, int32_t n_out, int32_t act, float* work,
                              hipStream_t stream) {
    if (!work || !dense_backward_args_ok(x, W, z, dy, dW, db, batch, n_in, n_out, act)) {
        set_error("bse_dense_backward: NULL array, empty size or unknown activation");
        return BSE_ERR_INVALID_ARG;
    }
    const hipError_t e = enqueue_dense_backward(x, W, z, dy, dx, dW, db, batch, n_in, n_out, act, work, stream);
    return e == hipSuccess ? BSE_OK : fail(e, "bse_dense_backward");
}

bse_status bse_dense_backward_noalloc(const float* x, const float* W, const float* z, const float* dy, float* dx,
                                      float* dW, float* db, int32_t batch, int32_t n_in, int32_t n_out, int32_t act,
                                      hipStream_t stream) {
    if (!dense_backward_args_ok(x, W, z, dy, dW, db, batch, n_in, n_out, act)) {
        set_error("bse_dense_backward_noalloc: NULL array, empty size or unknown activation");
        return BSE_ERR_INVALID_ARG;
    }
    if ((int64_t)batch * n_out > kNoAllocMaxEntries) {
        set_error("bse_dense_backward_noalloc: batch * n_out = %lld exceeds the scratch limit %lld",
                  (long long)batch * n_out, (long long)kNoAllocMaxEntries);
        return BSE_ERR_WORKSPACE;
    }
    float* work = nullptr;
    hipError_t e = scratch_address(&work);
    if (e != hipSuccess) return fail(e, "bse_dense_backward_noalloc: scratch address");
    e = enqueue_dense_backward(x, W, z, dy, dx, dW, db, batch, n_in, n_out, act, work, stream);
    return e == hipSuccess ? BSE_OK : fail(e, "bse_dense_backward_noalloc");
}

bse_status bse_mse_loss(const float* y, const float* t, float* dy, double* loss, int64_t n, hipStream_t stream) {
    if (!y || !t || !loss || n < 1) {
        set_error("bse_mse_loss: NULL array or n < 1");
        return BSE_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, stream, y, t, dy, loss, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BSE_OK : fail(e, "bse_mse_loss");
}

bse_status bse_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                         float eps, int32_t t, hipStream_t stream) {
    if (!p || !g || !m || !v || n < 1 || t < 1) {
        set_error("bse_adam_step: NULL array, n < 1 or t < 1");
        return BSE_ERR_INVALID_ARG;
    }
    const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, g, m, v, n, lr, beta1,
                       beta2, eps, c1, c2);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BSE_OK : fail(e, "bse_adam_step");
}

bse_status bse_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t stream) {
    if (!x || !y || n < 1) {
        set_error("bse_to_bf16: NULL array or n < 1");
        return BSE_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, x,
                       reinterpret_cast<unsigned short*>(y), n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BSE_OK : fail(e, "bse_to_bf16");
}

bse_status bse_dense_forward_bf16(const uint16_t* x, const uint16_t* W, const float* b, uint16_t* y_bf16,
                                  float* y_f32, int32_t batch, int32_t n_in, int32_t n_out, int32_t act,
                                  hipStream_t stream) {
    if (!x || !W || !b || (!y_bf16 && !y_f32) || batch < 1 || n_in < 32 || n_in % 32 != 0 || n_out < 1 ||
        (act != BSE_ACT_NONE && act != BSE_ACT_GELU) || ((uintptr_t)x & 15) || ((uintptr_t)W & 15)) {
        set_error("bse_dense_forward_bf16: NULL array, n_in not a multiple of 32, unaligned input or bad activation");
        return BSE_ERR_INVALID_ARG;
    }
    const int64_t waves = (int64_t)((batch + 15) / 16) * ((n_out + 15) / 16);
    hipLaunchKernelGGL(k_dense_bf16, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, stream,
                       reinterpret_cast<const unsigned short*>(x), reinterpret_cast<const unsigned short*>(W), b,
                       reinterpret_cast<unsigned short*>(y_bf16), y_f32, batch, n_in, n_out, act);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BSE_OK : fail(e, "bse_dense_forward_bf16");
}

bse_status bse_continued_fraction_terminated(const double* a, const double* b, int32_t lda, int32_t ldb, int32_t m,
                                             const double* pnorm2, const double* a_inf, const double* b_inf,
                                             int32_t n_chains, double prefactor, const double* omega,
                                             int32_t n_omega, double eta, double* eps_re, double* eps_im,
                                             hipStream_t stream) {
    if (!a || !b || !pnorm2 || !a_inf || !b_inf || !omega || !eps_re || !eps_im || n_chains < 1 || n_omega < 1 ||
        m < 1 || lda < m || ldb < m + 1 || !(eta > 0.0)) {
        set_error("bse_continued_fraction_terminated: NULL array, m < 1, lda < m, ldb < m + 1 or eta <= 0");
        return BSE_ERR_INVALID_ARG;
    }
    const int64_t total = (int64_t)n_chains * n_omega;
    hipLaunchKernelGGL(k_cf_terminated, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, a, b, lda, ldb,
                       m, pnorm2, a_inf, b_inf, n_chains, prefactor, omega, n_omega, eta, eps_re, eps_im);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BSE_OK : fail(e, "bse_continued_fraction_terminated");
}

}  // extern "C"
