// FP32 pair arithmetic, precision-mode accumulators and output records shared
// by the direct-sum and tree-code force kernels (device code only).  See
// accel.hip for the instruction count and the precision modes.
#pragma once

#include "internal.h"

namespace nbi {
namespace {

enum { M_F32 = 1, M_KAHAN = 2, M_F64ACC = 3 };

template <int MODE>
struct Run;

template <>
struct Run<M_F32> {
    float s;
    __device__ void zero() { s = 0.0f; }
    __device__ void fold(float p) { s += p; }
    __device__ double get() const { return s; }
};

// Classic Kahan: y = p - c; t = s + y; c = (t - s) - y; s = t.  The reported
// value applies the final compensation, s - c, formed in FP64.
template <>
struct Run<M_KAHAN> {
    float s, c;
    __device__ void zero() { s = 0.0f; c = 0.0f; }
    __device__ void fold(float p)
    {
        const float y = p - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ double get() const { return (double)s - (double)c; }
};

template <>
struct Run<M_F64ACC> {
    double s;
    __device__ void zero() { s = 0.0; }
    __device__ void fold(float p) { s += (double)p; }
    __device__ double get() const { return s; }
};

template <typename T, int TPL>
struct Targets {
    T x[TPL], y[TPL], z[TPL];
    int i[TPL];
};

template <typename T, int TPL>
struct Sums {
    T ax[TPL], ay[TPL], az[TPL], ph[TPL];
    __device__ void zero()
    {
#pragma unroll
        for (int t = 0; t < TPL; ++t) ax[t] = ay[t] = az[t] = ph[t] = T(0);
    }
};

// ---- FP32 pair ---------------------------------------------------------------
template <int TPL, bool MASK>
__device__ __forceinline__ void pair_f32(const float4 b, const int j, const Targets<float, TPL> &T,
                                         const float eps2, Sums<float, TPL> &S)
{
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const float dx = b.x - T.x[t];
        const float dy = b.y - T.y[t];
        const float dz = b.z - T.z[t];
        const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
        float rho = __builtin_amdgcn_rsqf(r2);
        if (MASK) rho = (j == T.i[t]) ? 0.0f : rho;
        const float mr = b.w * rho;
        const float s = mr * (rho * rho);
        S.ph[t] = __builtin_fmaf(b.w, rho, S.ph[t]);
        S.ax[t] = __builtin_fmaf(s, dx, S.ax[t]);
        S.ay[t] = __builtin_fmaf(s, dy, S.ay[t]);
        S.az[t] = __builtin_fmaf(s, dz, S.az[t]);
    }
}

// SEQ: a scheduling barrier after each source keeps the per-source chain
// that the compiler otherwise chooses (it sometimes interleaves the sources
// of an unrolled step over twice the registers instead, which measured about
// 18% slower).
template <int TPL, bool MASK, bool SEQ = false>
__device__ __forceinline__ void sweep_f32(const float4 *__restrict__ src, int j0, int j1,
                                          const Targets<float, TPL> &T, float eps2,
                                          Sums<float, TPL> &S)
{
    int j = j0;
    for (; j + kUnroll <= j1; j += kUnroll) {
        float4 b[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) b[u] = src[j + u];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            pair_f32<TPL, MASK>(b[u], j + u, T, eps2, S);
            if constexpr (SEQ) __builtin_amdgcn_sched_barrier(0);
        }
    }
    for (; j < j1; ++j) pair_f32<TPL, MASK>(src[j], j, T, eps2, S);
}

// Sources [j0, j1) against the wave's targets [d0, d1): only the overlap runs
// the masked variant.
template <int TPL, bool SEQ = false>
__device__ __forceinline__ void range_f32(const float4 *__restrict__ src, int j0, int j1, int d0,
                                          int d1, const Targets<float, TPL> &T, float eps2,
                                          Sums<float, TPL> &S)
{
    const int lo = min(max(d0, j0), j1);
    const int hi = min(max(d1, j0), j1);
    sweep_f32<TPL, false, SEQ>(src, j0, lo, T, eps2, S);
    sweep_f32<TPL, true, SEQ>(src, lo, hi, T, eps2, S);
    sweep_f32<TPL, false, SEQ>(src, hi, j1, T, eps2, S);
}

// ---- output records ------------------------------------------------------------
__device__ __forceinline__ void put(float4 *out, long k, const double (&r)[4], double G)
{
    out[k] = make_float4((float)(G * r[0]), (float)(G * r[1]), (float)(G * r[2]), (float)(-G * r[3]));
}
__device__ __forceinline__ void put(double4 *out, long k, const double (&r)[4], double G)
{
    out[k] = make_double4(G * r[0], G * r[1], G * r[2], -G * r[3]);
}
// Pure FP32 mode scales in FP32.
__device__ __forceinline__ void put_f32(float4 *out, long k, const double (&r)[4], float G)
{
    out[k] = make_float4(G * (float)r[0], G * (float)r[1], G * (float)r[2], -G * (float)r[3]);
}

}  // namespace
}  // namespace nbi
