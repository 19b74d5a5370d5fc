// Device-side helpers shared by the kernels of the double-grid BSE library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bse_dg.h"

namespace bse {

constexpr int kWave = 64;

// ---- complex arithmetic in FP64 --------------------------------------------------
struct cd {
    double re, im;
};

__device__ __forceinline__ cd cmake(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.re * s, a.im * s}; }
__device__ __forceinline__ cd cconj(cd a) { return cd{a.re, -a.im}; }
// acc += a * b
__device__ __forceinline__ void cfma(cd& acc, cd a, cd b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
__device__ __forceinline__ void cfma_cj(cd& acc, cd a, cd b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}
// acc += a * conj(b)
__device__ __forceinline__ void cfma_jc(cd& acc, cd a, cd b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.im, b.re, acc.im);
    acc.im = fma(-a.re, b.im, acc.im);
}

// ---- complex arithmetic in the inner type of a short contraction --------------------
// The restrict and the prolong form their <= 6-term contractions per (subpoint, corner)
// in the storage's precision (FP32 for FP32 overlaps, FP64 for FP64) and add the results
// into FP64 accumulators.
template <class T>
struct cplx {
    T re, im;
};
template <class M2>
struct Inner;
template <>
struct Inner<float2> {
    using t = float;
};
template <>
struct Inner<double2> {
    using t = double;
};
template <class T>
__device__ __forceinline__ cplx<T> cl(float2 v) {
    return cplx<T>{(T)v.x, (T)v.y};
}
template <class T>
__device__ __forceinline__ cplx<T> cl(double2 v) {
    return cplx<T>{(T)v.x, (T)v.y};
}
template <class T>
__device__ __forceinline__ cplx<T> czero() {
    return cplx<T>{(T)0, (T)0};
}
// acc += a * b
template <class T>
__device__ __forceinline__ void cmac(cplx<T>& acc, cplx<T> a, cplx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <class T>
__device__ __forceinline__ void cmac_cj(cplx<T>& acc, cplx<T> a, cplx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}
// acc += a * conj(b)
template <class T>
__device__ __forceinline__ void cmac_jc(cplx<T>& acc, cplx<T> a, cplx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.im, b.re, acc.im);
    acc.im = fma(-a.re, b.im, acc.im);
}
// FP64 accumulator += inner-precision value
template <class T>
__device__ __forceinline__ void cadd_to(cd& acc, cplx<T> v) {
    acc.re += (double)v.re;
    acc.im += (double)v.im;
}

// ---- storage precision ------------------------------------------------------------
template <class S>
struct cstore;
template <>
struct cstore<double> {
    using t2 = double2;
};
template <>
struct cstore<float> {
    using t2 = float2;
};

__device__ __forceinline__ cd ld(const double2* p) {
    double2 v = *p;
    return cd{v.x, v.y};
}
__device__ __forceinline__ cd ld(const float2* p) {
    float2 v = *p;
    return cd{(double)v.x, (double)v.y};
}
__device__ __forceinline__ void st(double2* p, cd v) { *p = make_double2(v.re, v.im); }
__device__ __forceinline__ void st(float2* p, cd v) { *p = make_float2((float)v.re, (float)v.im); }
__device__ __forceinline__ cd cv(double2 v) { return cd{v.x, v.y}; }
__device__ __forceinline__ cd cv(float2 v) { return cd{(double)v.x, (double)v.y}; }
// value after a round trip through the storage type
__device__ __forceinline__ cd rounded(cd v, const double2*) { return v; }
__device__ __forceinline__ cd rounded(cd v, const float2*) {
    return cd{(double)(float)v.re, (double)(float)v.im};
}

// ---- buffer loads: per-lane 32-bit offset, uniform offset in a scalar register ----------
// The resource covers `bytes` from `base`; loads past it return zero (hardware check).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <class T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ float2 bload<float2>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double2 bload<double2>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// ---- 16-byte load units ---------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

// complex entries per 16-byte unit and the unit's type, by storage precision
template <class M2>
struct Unit16;
template <>
struct Unit16<float2> {
    static constexpr int P = 2;
    using t = f4v;
    __device__ static inline float2 get(const f4v& v, int i) {
        return i == 0 ? make_float2(v.x, v.y) : make_float2(v.z, v.w);
    }
};
template <>
struct Unit16<double2> {
    static constexpr int P = 1;
    using t = d2v;
    __device__ static inline double2 get(const d2v& v, int) { return make_double2(v.x, v.y); }
};

// ---- lane-pair exchange (lanes 2i <-> 2i+1) through DPP quad permutation [1,0,3,2] ------
__device__ __forceinline__ int swap_pair_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ float2 swap_pair(float2 v) {
    return make_float2(__builtin_bit_cast(float, swap_pair_i(__builtin_bit_cast(int, v.x))),
                       __builtin_bit_cast(float, swap_pair_i(__builtin_bit_cast(int, v.y))));
}
__device__ __forceinline__ double swap_pair_d(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = swap_pair_i((int)(b & 0xffffffffll));
    const int hi = swap_pair_i((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double2 swap_pair(double2 v) { return make_double2(swap_pair_d(v.x), swap_pair_d(v.y)); }

// ---- 16-bit storage formats of the low-precision coarse kernel (BSE_BF16_KC,
// BSE_F16_KC): round to nearest even from FP32, and back ----------------------------------
__device__ __forceinline__ unsigned short enc_lowp(int fmt, float v) {
    return fmt == BSE_BF16_KC ? __builtin_bit_cast(unsigned short, (__bf16)v)
                              : __builtin_bit_cast(unsigned short, (_Float16)v);
}
__device__ __forceinline__ float dec_lowp(int fmt, unsigned short v) {
    return fmt == BSE_BF16_KC ? (float)__builtin_bit_cast(__bf16, v) : (float)__builtin_bit_cast(_Float16, v);
}

// ---- interpolation prefactors (Sec. 3) ----------------------------------------------
// f^l_j = 1 - j/n for l = 0 and j/n for l = 1, so the trilinear
// f^{lmn}(sub) = f^l_{j1} f^m_{j2} f^n_{j3} (corner z = 4l + 2m + n) is an integer
// product over n^3: one correctly rounded division.
// neighbours == 1: one-hot on the nearest corner (j/n <= 1/2 picks l = 0 per axis).
__device__ __forceinline__ double prefactor(int sub, int z, int n_div, int neighbours) {
    int j3 = sub % n_div;
    int j2 = (sub / n_div) % n_div;
    int j1 = sub / (n_div * n_div);
    int l = (z >> 2) & 1, m = (z >> 1) & 1, n = z & 1;
    if (neighbours == 1) {
        int l1 = (2 * j1 > n_div), m1 = (2 * j2 > n_div), n1 = (2 * j3 > n_div);
        return (l == l1 && m == m1 && n == n1) ? 1.0 : 0.0;
    }
    const int num = (l ? j1 : n_div - j1) * (m ? j2 : n_div - j2) * (n ? j3 : n_div - j3);
    return (double)num / (double)(n_div * n_div * n_div);
}

// coarse index of corner z of a cell (periodic wrap), Eq. (neighborhood)
__device__ __forceinline__ int corner_index(int cell, int z, int n_c) {
    int i3 = cell % n_c;
    int i2 = (cell / n_c) % n_c;
    int i1 = cell / (n_c * n_c);
    i1 = (i1 + ((z >> 2) & 1)) % n_c;
    i2 = (i2 + ((z >> 1) & 1)) % n_c;
    i3 = (i3 + (z & 1)) % n_c;
    return (i1 * n_c + i2) * n_c + i3;
}
// the cell whose corner z is coarse point k (inverse of corner_index)
__device__ __forceinline__ int cell_of_corner(int k, int z, int n_c) {
    int i3 = k % n_c;
    int i2 = (k / n_c) % n_c;
    int i1 = k / (n_c * n_c);
    i1 = (i1 - ((z >> 2) & 1) + n_c) % n_c;
    i2 = (i2 - ((z >> 1) & 1) + n_c) % n_c;
    i3 = (i3 - (z & 1) + n_c) % n_c;
    return (i1 * n_c + i2) * n_c + i3;
}

// resolvent of the constant chain (a_inf, b_inf): root of b^2 g^2 - (z - a) g + 1 = 0
// with Im g <= 0 (vanishes as |z| grows)
__device__ __forceinline__ void constant_chain(double zr, double zi, double a_inf, double b_inf, double& gr,
                                               double& gi) {
    const double xr = zr - a_inf, xi = zi;
    if (b_inf == 0.0) {
        const double den = xr * xr + xi * xi;
        gr = xr / den;
        gi = -xi / den;
        return;
    }
    // w = x^2 - 4 b^2, s = sqrt(w) (principal)
    const double wr = xr * xr - xi * xi - 4.0 * b_inf * b_inf, wi = 2.0 * xr * xi;
    const double r = hypot(wr, wi);
    double sr = sqrt(0.5 * (r + wr)), si = sqrt(0.5 * fmax(r - wr, 0.0));
    if (wi < 0.0) si = -si;
    const double inv = 1.0 / (2.0 * b_inf * b_inf);
    double g1r = (xr - sr) * inv, g1i = (xi - si) * inv;
    if (g1i > 0.0) {  // the other root
        g1r = (xr + sr) * inv;
        g1i = (xi + si) * inv;
    }
    gr = g1r;
    gi = g1i;
}

// ---- wavefront reductions -------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Block-wide sum of one double per thread in a fixed tree order.  `lds` must
// hold blockDim.x / 64 doubles.  Result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* lds) {
    v = wave_sum(v);
    int wave = threadIdx.x / kWave;
    int nw = blockDim.x / kWave;
    __syncthreads();
    if ((threadIdx.x % kWave) == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[w];
    __syncthreads();
    return s;
}

// Sum of n doubles at p[i * stride] (i < n) by the whole block, in an order that
// depends only on n and blockDim: every block that calls it on the same data gets
// the same bits.  `lds` holds blockDim.x / 64 doubles.  Loads go in batches of 4
// per thread with clamped indices, so a batch is in flight at once.
__device__ __forceinline__ double block_sum_strided(const double* p, int n, int stride, double* lds) {
    double v = 0.0;
    for (int i0 = 0; i0 < n; i0 += 4 * (int)blockDim.x) {
        double x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = p[(int64_t)min(i0 + (int)threadIdx.x + q * (int)blockDim.x, n - 1) * stride];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (i0 + (int)threadIdx.x + q * (int)blockDim.x < n) v += x[q];
    }
    return block_sum(v, lds);
}

}  // namespace bse
