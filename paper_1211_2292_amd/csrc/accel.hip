// Direct-sum force and potential kernels for gfx950.
//
// Computes, for each target i, the paper's force calculation (Section IV.B,
// Calculate_forces) with every other body on the interaction list, i.e. the
// exact softened pair sum
//     a_i   =  G sum_{j != i} m_j d_ij (|d_ij|^2 + eps^2)^(-3/2),  d_ij = x_j - x_i
//     phi_i = -G sum_{j != i} m_j (|d_ij|^2 + eps^2)^(-1/2)
//
// Design (CDNA4, wave64):
// * A wave owns 64*TPL targets held in VGPRs.  Sources are streamed with
//   wave-uniform addresses, so every source record arrives through a scalar
//   load into SGPRs and feeds the VALU directly as the one scalar operand an
//   instruction may take: no LDS staging, no barriers, and the 16-byte source
//   record is fetched once per wave for 64*TPL interactions.
// * Pair arithmetic (FP32 modes): 3 sub, 3 FMA, 1 v_rsq_f32, 2 mul, 1 mul,
//   1 FMA (potential), 3 FMA = 14 VALU instructions = 20 flop by the usual
//   count.  The library is built with contraction off and every fused
//   multiply-add is written out, so the same arithmetic is emitted in every
//   kernel that shares these routines (batched results equal standalone ones
//   bit for bit).
// * Sources are processed in tiles of `jtile`; the FP32 partial sum of a tile
//   is folded into the running per-target sum by the precision mode (plain
//   FP32, Kahan-compensated FP32, or FP64).
// * The self pair is removed exactly: only the sub-range of sources that
//   overlaps the wave's own targets runs the masked variant (one compare and
//   one select per pair); every other source range runs unmasked.
// * Small problems split the source range over gridDim.y workgroup rows; the
//   per-split records go to scratch and are reduced in split order by a
//   second kernel, so the result never depends on scheduling.
#include <mutex>

#include "internal.h"
#include "pair.h"

namespace nbi {
namespace {

// Sums over sources [jb, je) of one system (records src[0..n)) for the wave
// whose first target is t0; returns the unscaled sums per target and
// component (ax, ay, az, sum m rho) through `res`.
template <int TPL, int MODE>
__device__ __forceinline__ void wave_f32(const float4 *__restrict__ src, int n, int t0, int jb,
                                         int je, int jtile, float eps2_in, double (&res)[TPL][4])
{
    const int lane = threadIdx.x & 63;
    const float eps2 = lane_copy(eps2_in);
    Targets<float, TPL> T;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        T.i[t] = i;
        const float4 p = src[min(i, n - 1)];
        T.x[t] = p.x;
        T.y[t] = p.y;
        T.z[t] = p.z;
    }
    const int d0 = t0, d1 = t0 + 64 * TPL;
    Sums<float, TPL> S;
    Run<MODE> R[TPL][4];
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) R[t][c].zero();
    for (int jc = jb, ce; jc < je; jc = ce) {
        ce = je - jc > jtile ? jc + jtile : je;  // no jc + jtile past je (int range)
        S.zero();
        // pure FP32 pins the per-source schedule (see sweep_f32)
        range_f32<TPL, MODE == M_F32>(src, jc, ce, d0, d1, T, eps2, S);
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            R[t][0].fold(S.ax[t]);
            R[t][1].fold(S.ay[t]);
            R[t][2].fold(S.az[t]);
            R[t][3].fold(S.ph[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) res[t][c] = R[t][c].get();
}

// ---- FP64 pair ---------------------------------------------------------------
// 1/sqrt(q) from the hardware estimate and two Newton-Raphson steps
// y <- y + y (1 - q y^2) / 2.
__device__ __forceinline__ double rsqrt_f64(double q)
{
    double y = __builtin_amdgcn_rsq(q);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = __builtin_fma(-q, y * y, 1.0);
        y = __builtin_fma(0.5 * y, e, y);
    }
    return y;
}

template <int TPL, bool MASK>
__device__ __forceinline__ void pair_f64(const double4 b, const int j, const Targets<double, TPL> &T,
                                         const double eps2, Sums<double, TPL> &S)
{
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const double dx = b.x - T.x[t];
        const double dy = b.y - T.y[t];
        const double dz = b.z - T.z[t];
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, eps2)));
        double rho = rsqrt_f64(r2);
        if (MASK) rho = (j == T.i[t]) ? 0.0 : rho;
        const double mr = b.w * rho;
        const double s = mr * (rho * rho);
        S.ph[t] = __builtin_fma(b.w, rho, S.ph[t]);
        S.ax[t] = __builtin_fma(s, dx, S.ax[t]);
        S.ay[t] = __builtin_fma(s, dy, S.ay[t]);
        S.az[t] = __builtin_fma(s, dz, S.az[t]);
    }
}

template <int TPL, bool MASK>
__device__ __forceinline__ void sweep_f64(const double4 *__restrict__ src, int j0, int j1,
                                          const Targets<double, TPL> &T, double eps2,
                                          Sums<double, TPL> &S)
{
    int j = j0;
    for (; j + kUnroll <= j1; j += kUnroll) {
        double4 b[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) b[u] = src[j + u];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) pair_f64<TPL, MASK>(b[u], j + u, T, eps2, S);
    }
    for (; j < j1; ++j) pair_f64<TPL, MASK>(src[j], j, T, eps2, S);
}

template <int TPL>
__device__ __forceinline__ void wave_f64(const double4 *__restrict__ src, int n, int t0, int jb,
                                         int je, int jtile, double eps2, double (&res)[TPL][4])
{
    const int lane = threadIdx.x & 63;
    Targets<double, TPL> T;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        T.i[t] = i;
        const double4 p = src[min(i, n - 1)];
        T.x[t] = p.x;
        T.y[t] = p.y;
        T.z[t] = p.z;
    }
    const int d0 = t0, d1 = t0 + 64 * TPL;
    double R[TPL][4];
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) R[t][c] = 0.0;
    Sums<double, TPL> S;
    for (int jc = jb, ce; jc < je; jc = ce) {
        ce = je - jc > jtile ? jc + jtile : je;  // no jc + jtile past je (int range)
        S.zero();
        const int lo = min(max(d0, jc), ce);
        const int hi = min(max(d1, jc), ce);
        sweep_f64<TPL, false>(src, jc, lo, T, eps2, S);
        sweep_f64<TPL, true>(src, lo, hi, T, eps2, S);
        sweep_f64<TPL, false>(src, hi, ce, T, eps2, S);
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            R[t][0] += S.ax[t];
            R[t][1] += S.ay[t];
            R[t][2] += S.az[t];
            R[t][3] += S.ph[t];
        }
    }
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) res[t][c] = R[t][c];
}

// ---- FP32 sweep with sources staged in LDS ----------------------------------
// Same pair arithmetic and the same order of every sum as the scalar-load
// sweep (identical results), but each source record reaches the VALU as a
// VGPR from a broadcast LDS read instead of as an SGPR: on gfx950 VALU
// instructions whose operands are all VGPRs can issue about twice per clock
// per CU, while those that read an SGPR stay near one.
constexpr int kLdsTile = 256;  // sources per LDS buffer (one per thread)

template <int TPL, bool MASK>
__device__ __forceinline__ void sweep_lds(const float4 *tl, int jbase, int u0, int u1,
                                          const Targets<float, TPL> &T, float eps2,
                                          Sums<float, TPL> &S)
{
    int u = u0;
    for (; u + kUnroll <= u1; u += kUnroll) {
        float4 b[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) b[k] = tl[u + k];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) pair_f32<TPL, MASK>(b[k], jbase + u + k, T, eps2, S);
    }
    for (; u < u1; ++u) pair_f32<TPL, MASK>(tl[u], jbase + u, T, eps2, S);
}

// Whole workgroup: all four waves sweep the same source range [jb, je); the
// tiles are double-buffered through LDS with a register prefetch.  jtile is
// a multiple of kLdsTile, so the partial sums fold at the same source
// indices as in the scalar-load sweep.
template <int TPL, int MODE>
__device__ __forceinline__ void block_lds_f32(const float4 *__restrict__ src, int n, int t0, int jb,
                                              int je, int jtile, float eps2_in,
                                              float4 (*tile)[kLdsTile], double (&res)[TPL][4])
{
    const int lane = threadIdx.x & 63;
    const float eps2 = lane_copy(eps2_in);
    Targets<float, TPL> T;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        T.i[t] = i;
        const float4 p = src[min(i, n - 1)];
        T.x[t] = p.x;
        T.y[t] = p.y;
        T.z[t] = p.z;
    }
    const int d0 = t0, d1 = t0 + 64 * TPL;
    Sums<float, TPL> S;
    S.zero();
    Run<MODE> R[TPL][4];
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) R[t][c].zero();
    float4 pre = make_float4(0.f, 0.f, 0.f, 0.f);
    if (jb + (int)threadIdx.x < je) pre = src[jb + threadIdx.x];
    tile[0][threadIdx.x] = pre;
    __syncthreads();
    int buf = 0, since = 0;
    for (int j0 = jb; j0 < je; j0 += kLdsTile) {
        const int cnt = min(kLdsTile, je - j0);
        const int jn = j0 + kLdsTile;
        if (jn + (int)threadIdx.x < je) pre = src[jn + threadIdx.x];
        const int lo = min(max(d0, j0), j0 + cnt) - j0;
        const int hi = min(max(d1, j0), j0 + cnt) - j0;
        sweep_lds<TPL, false>(tile[buf], j0, 0, lo, T, eps2, S);
        sweep_lds<TPL, true>(tile[buf], j0, lo, hi, T, eps2, S);
        sweep_lds<TPL, false>(tile[buf], j0, hi, cnt, T, eps2, S);
        since += cnt;
        if (since >= jtile || jn >= je) {
#pragma unroll
            for (int t = 0; t < TPL; ++t) {
                R[t][0].fold(S.ax[t]);
                R[t][1].fold(S.ay[t]);
                R[t][2].fold(S.az[t]);
                R[t][3].fold(S.ph[t]);
            }
            S.zero();
            since = 0;
        }
        if (jn < je) tile[buf ^ 1][threadIdx.x] = pre;
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) res[t][c] = R[t][c].get();
}

// ---- kernels -------------------------------------------------------------------
// The chip hands workgroups to its 8 XCDs in turn (linear workgroup id modulo
// 8), and each XCD has its own L2.  When the source range is split in a
// multiple of 8, workgroup (bx, by) = (target block, source split) is taken
// from the linear id so that XCD x runs only the splits x J/8 .. (x + 1) J/8
// - 1, one after the other with the target blocks fastest: the waves on an
// XCD then stream one source segment at a time, which stays in that L2, and
// each segment is fetched from memory about once instead of once per pass of
// the resident waves.  Any other split count, or sources that fit in one
// XCD's L2 anyway (there the new order measured up to 18% slower, at 2^12),
// keeps the plain mapping.  Either way every (bx, by) is run exactly once, so
// results do not depend on it.
constexpr int kXcds = 8;
constexpr long kXcdL2Bytes = 4l << 20;

__device__ __forceinline__ void xcd_block(long src_bytes, int &bx, int &by)
{
    const int gx = gridDim.x, J = gridDim.y;
    if (J % kXcds || src_bytes <= kXcdL2Bytes) {
        bx = blockIdx.x;
        by = blockIdx.y;
        return;
    }
    const long L = (long)blockIdx.y * gx + blockIdx.x;
    const long i = L / kXcds;  // this workgroup's place in its XCD's sequence
    by = (int)(L % kXcds) * (J / kXcds) + (int)(i / gx);
    bx = (int)(i % gx);
}

// Source range of split `split` out of `js` over n sources.
__device__ __forceinline__ void split_range(int n, int js, int split, int &jb, int &je)
{
    const long per = ((long)n + js - 1) / js;
    jb = (int)min((long)n, (long)split * per);
    je = (int)min((long)n, (long)jb + per);
}

template <int TPL, int MODE>
__global__ __launch_bounds__(kBlock) void k_accel_f32(const float4 *__restrict__ src, int n,
                                                      float eps2, double G, int tbeg, int tcount,
                                                      int jtile, float4 *__restrict__ out,
                                                      void *__restrict__ partial)
{
    constexpr int WT = 64 * TPL;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int bx, by;
    xcd_block((long)n * sizeof(float4), bx, by);
    const int t0 = tbeg + (bx * (kBlock / 64) + wave) * WT;
    const int tend = tbeg + tcount;
    if (t0 >= tend) return;
    int jb, je;
    split_range(n, gridDim.y, by, jb, je);
    double res[TPL][4];
    wave_f32<TPL, MODE>(src, n, t0, jb, je, jtile, eps2, res);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        if (i >= tend) continue;
        const long k = i - tbeg;
        if (gridDim.y == 1) {
            if constexpr (MODE == M_F32)
                put_f32(out, k, res[t], (float)G);
            else
                put(out, k, res[t], G);
        } else if constexpr (MODE == M_F32) {
            reinterpret_cast<float4 *>(partial)[(long)by * tcount + k] =
                make_float4((float)res[t][0], (float)res[t][1], (float)res[t][2], (float)res[t][3]);
        } else {
            reinterpret_cast<double4 *>(partial)[(long)by * tcount + k] =
                make_double4(res[t][0], res[t][1], res[t][2], res[t][3]);
        }
    }
}

template <int TPL, int MODE>
__global__ __launch_bounds__(kBlock) void k_accel_lds_f32(const float4 *__restrict__ src, int n,
                                                          float eps2, double G, int tbeg, int tcount,
                                                          int jtile, float4 *__restrict__ out,
                                                          void *__restrict__ partial)
{
    __shared__ float4 tile[2][kLdsTile];
    constexpr int WT = 64 * TPL;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tend = tbeg + tcount;
    // waves past the last target still take part in the shared tile loop
    // (on a valid target range) but store nothing
    int bx, by;
    xcd_block((long)n * sizeof(float4), bx, by);
    const long t0l = (long)tbeg + ((long)bx * (kBlock / 64) + wave) * WT;
    const bool active = t0l < tend;
    const int t0 = active ? (int)t0l : tbeg;
    int jb, je;
    split_range(n, gridDim.y, by, jb, je);
    double res[TPL][4];
    block_lds_f32<TPL, MODE>(src, n, t0, jb, je, jtile, eps2, tile, res);
    if (!active) return;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        if (i >= tend) continue;
        const long k = i - tbeg;
        if (gridDim.y == 1) {
            if constexpr (MODE == M_F32)
                put_f32(out, k, res[t], (float)G);
            else
                put(out, k, res[t], G);
        } else if constexpr (MODE == M_F32) {
            reinterpret_cast<float4 *>(partial)[(long)by * tcount + k] =
                make_float4((float)res[t][0], (float)res[t][1], (float)res[t][2], (float)res[t][3]);
        } else {
            reinterpret_cast<double4 *>(partial)[(long)by * tcount + k] =
                make_double4(res[t][0], res[t][1], res[t][2], res[t][3]);
        }
    }
}

template <int TPL>
__global__ __launch_bounds__(kBlock) void k_accel_f64(const double4 *__restrict__ src, int n,
                                                      double eps2, double G, int tbeg, int tcount,
                                                      int jtile, double4 *__restrict__ out,
                                                      double4 *__restrict__ partial)
{
    constexpr int WT = 64 * TPL;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int bx, by;
    xcd_block((long)n * sizeof(double4), bx, by);
    const int t0 = tbeg + (bx * (kBlock / 64) + wave) * WT;
    const int tend = tbeg + tcount;
    if (t0 >= tend) return;
    int jb, je;
    split_range(n, gridDim.y, by, jb, je);
    double res[TPL][4];
    wave_f64<TPL>(src, n, t0, jb, je, jtile, eps2, res);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        if (i >= tend) continue;
        const long k = i - tbeg;
        if (gridDim.y == 1)
            put(out, k, res[t], G);
        else
            partial[(long)by * tcount + k] = make_double4(res[t][0], res[t][1], res[t][2], res[t][3]);
    }
}

// Fixed-order reduction of the per-split records.
template <typename OUT>
__global__ __launch_bounds__(kBlock) void k_split_reduce(const double4 *__restrict__ partial,
                                                         int js, int tcount, double G,
                                                         OUT *__restrict__ out)
{
    const long k = (long)blockIdx.x * kBlock + threadIdx.x;
    if (k >= tcount) return;
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < js; ++s) {
        const double4 p = partial[(long)s * tcount + k];
        r[0] += p.x;
        r[1] += p.y;
        r[2] += p.z;
        r[3] += p.w;
    }
    put(out, k, r, G);
}

__global__ __launch_bounds__(kBlock) void k_split_reduce_f32(const float4 *__restrict__ partial,
                                                             int js, int tcount, float G,
                                                             float4 *__restrict__ out)
{
    const long k = (long)blockIdx.x * kBlock + threadIdx.x;
    if (k >= tcount) return;
    float r[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int s = 0; s < js; ++s) {
        const float4 p = partial[(long)s * tcount + k];
        r[0] += p.x;
        r[1] += p.y;
        r[2] += p.z;
        r[3] += p.w;
    }
    out[k] = make_float4(G * r[0], G * r[1], G * r[2], -G * r[3]);
}

// ---- batched persistent kernel -------------------------------------------------
// Each wave pops (system, first target) units from a longest-first list with
// one integer atomic; a unit is one wave's worth of targets of one system
// swept over that system's sources with the same tiles as k_accel_f32 with
// one split, so each system's result equals its standalone evaluation
// bit for bit.  The wave that finishes last returns both counters to zero,
// which keeps repeated launches and graph replays self-contained.
template <int TPL, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_batched_f32(const float4 *__restrict__ pm,
                                                        const int64_t *__restrict__ offsets,
                                                        const int2 *__restrict__ units, int nunits,
                                                        const float *__restrict__ eps_sys,
                                                        float eps2_all, double G, int jtile,
                                                        float4 *__restrict__ out,
                                                        unsigned *__restrict__ counter)
{
    constexpr int WT = 64 * TPL;
    const int lane = threadIdx.x & 63;
    const unsigned nwaves = gridDim.x * (kBlock / 64);
    for (;;) {
        unsigned u = 0;
        if (lane == 0) u = atomicAdd(&counter[0], 1u);
        u = __builtin_amdgcn_readfirstlane(u);
        if (u >= (unsigned)nunits) break;
        const int2 w = units[u];
        const int64_t base = offsets[w.x];
        const int n = (int)(offsets[w.x + 1] - base);
        const float4 *src = pm + base;
        float eps2 = eps2_all;
        if (eps_sys) {
            const double e = eps_sys[w.x];
            eps2 = (float)(e * e);
        }
        double res[TPL][4];
        wave_f32<TPL, MODE>(src, n, w.y, 0, n, jtile, eps2, res);
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            const int i = w.y + t * 64 + lane;
            if (i >= n) continue;
            if constexpr (MODE == M_F32)
                put_f32(out + base, i, res[t], (float)G);
            else
                put(out + base, i, res[t], G);
        }
    }
    (void)WT;
    if (lane == 0) {
        const unsigned done = atomicAdd(&counter[1], 1u);
        if (done == nwaves - 1) {
            atomicExch(&counter[0], 0u);
            atomicExch(&counter[1], 0u);
        }
    }
}

template <int TPL>
__global__ __launch_bounds__(kBlock) void k_batched_f64(const double4 *__restrict__ pm,
                                                        const int64_t *__restrict__ offsets,
                                                        const int2 *__restrict__ units, int nunits,
                                                        const float *__restrict__ eps_sys,
                                                        double eps2_all, double G, int jtile,
                                                        double4 *__restrict__ out,
                                                        unsigned *__restrict__ counter)
{
    const int lane = threadIdx.x & 63;
    const unsigned nwaves = gridDim.x * (kBlock / 64);
    for (;;) {
        unsigned u = 0;
        if (lane == 0) u = atomicAdd(&counter[0], 1u);
        u = __builtin_amdgcn_readfirstlane(u);
        if (u >= (unsigned)nunits) break;
        const int2 w = units[u];
        const int64_t base = offsets[w.x];
        const int n = (int)(offsets[w.x + 1] - base);
        double eps2 = eps2_all;
        if (eps_sys) {
            const double e = eps_sys[w.x];
            eps2 = e * e;
        }
        double res[TPL][4];
        wave_f64<TPL>(pm + base, n, w.y, 0, n, jtile, eps2, res);
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            const int i = w.y + t * 64 + lane;
            if (i < n) put(out + base, i, res[t], G);
        }
    }
    if (lane == 0) {
        const unsigned done = atomicAdd(&counter[1], 1u);
        if (done == nwaves - 1) {
            atomicExch(&counter[0], 0u);
            atomicExch(&counter[1], 0u);
        }
    }
}

template <int TPL, int MODE>
hipError_t go_f32(const float4 *pm, int n, float eps2, double G, float4 *out, int tbeg, int tcount,
                  const Tune &t, void *partial, bool reduce, hipStream_t s)
{
    const int per_block = (kBlock / 64) * 64 * TPL;
    dim3 grid((tcount + per_block - 1) / per_block, t.jsplit);
    if (t.variant == 1)
        hipLaunchKernelGGL((k_accel_lds_f32<TPL, MODE>), grid, dim3(kBlock), 0, s, pm, n, eps2, G,
                           tbeg, tcount, t.jtile, out, partial);
    else
        hipLaunchKernelGGL((k_accel_f32<TPL, MODE>), grid, dim3(kBlock), 0, s, pm, n, eps2, G, tbeg,
                           tcount, t.jtile, out, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || t.jsplit == 1 || !reduce) return e;
    const int rb = (tcount + kBlock - 1) / kBlock;
    if constexpr (MODE == M_F32)
        hipLaunchKernelGGL(k_split_reduce_f32, dim3(rb), dim3(kBlock), 0, s,
                           (const float4 *)partial, t.jsplit, tcount, (float)G, out);
    else
        hipLaunchKernelGGL(k_split_reduce<float4>, dim3(rb), dim3(kBlock), 0, s,
                           (const double4 *)partial, t.jsplit, tcount, G, out);
    return hipGetLastError();
}

template <int TPL>
hipError_t go_f64(const double4 *pm, int n, double eps2, double G, double4 *out, int tbeg,
                  int tcount, const Tune &t, void *partial, bool reduce, hipStream_t s)
{
    const int per_block = (kBlock / 64) * 64 * TPL;
    dim3 grid((tcount + per_block - 1) / per_block, t.jsplit);
    hipLaunchKernelGGL((k_accel_f64<TPL>), grid, dim3(kBlock), 0, s, pm, n, eps2, G, tbeg, tcount,
                       t.jtile, out, (double4 *)partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || t.jsplit == 1 || !reduce) return e;
    const int rb = (tcount + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_split_reduce<double4>, dim3(rb), dim3(kBlock), 0, s,
                       (const double4 *)partial, t.jsplit, tcount, G, out);
    return hipGetLastError();
}

template <int MODE>
hipError_t by_tpl_f32(const float4 *pm, int n, float eps2, double G, float4 *out, int tbeg,
                      int tcount, const Tune &t, void *partial, bool reduce, hipStream_t s)
{
    switch (t.tpl) {
    case 1: return go_f32<1, MODE>(pm, n, eps2, G, out, tbeg, tcount, t, partial, reduce, s);
    case 2: return go_f32<2, MODE>(pm, n, eps2, G, out, tbeg, tcount, t, partial, reduce, s);
    default: return go_f32<4, MODE>(pm, n, eps2, G, out, tbeg, tcount, t, partial, reduce, s);
    }
}

template <int TPL, int MODE>
hipError_t go_batched_f32(const float4 *pm, const int64_t *off, const int2 *units, int nunits,
                          const float *eps_sys, float eps2, double G, float4 *out, const Tune &t,
                          unsigned *counter, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_batched_f32<TPL, MODE>), dim3(grid), dim3(kBlock), 0, s, pm, off, units,
                       nunits, eps_sys, eps2, G, t.jtile, out, counter);
    return hipGetLastError();
}

template <int MODE>
hipError_t batched_by_tpl(const float4 *pm, const int64_t *off, const int2 *units, int nunits,
                          const float *eps_sys, float eps2, double G, float4 *out, const Tune &t,
                          unsigned *counter, int grid, hipStream_t s)
{
    switch (t.tpl) {
    case 1: return go_batched_f32<1, MODE>(pm, off, units, nunits, eps_sys, eps2, G, out, t, counter, grid, s);
    case 2: return go_batched_f32<2, MODE>(pm, off, units, nunits, eps_sys, eps2, G, out, t, counter, grid, s);
    default: return go_batched_f32<4, MODE>(pm, off, units, nunits, eps_sys, eps2, G, out, t, counter, grid, s);
    }
}

}  // namespace

bool tune_valid(const Tune &t)
{
    return (t.tpl == 1 || t.tpl == 2 || t.tpl == 4) && t.jsplit >= 1 && t.jsplit <= 32 &&
           t.jtile >= 8 && t.jtile % kUnroll == 0 && t.jtile <= (1 << 24) &&
           (t.variant == 0 || (t.variant == 1 && t.jtile % kLdsTile == 0));
}

size_t accel_partial_bytes(int prec, int tcount, const Tune &t)
{
    if (t.jsplit <= 1) return 0;
    const size_t rec = (prec == NBODY_F32) ? sizeof(float4) : sizeof(double4);
    return rec * (size_t)t.jsplit * (size_t)tcount;
}

static float eps2_f32(double eps) { return (float)((double)eps * (double)eps); }

hipError_t launch_accel(int prec, const void *pm, int n, double G, double eps, void *out, int tbeg,
                        int tcount, const Tune &t, void *partial, hipStream_t s, bool reduce)
{
    if (prec == NBODY_F64) {
        const double4 *p = (const double4 *)pm;
        double4 *o = (double4 *)out;
        const double e2 = eps * eps;
        switch (t.tpl) {
        case 1: return go_f64<1>(p, n, e2, G, o, tbeg, tcount, t, partial, reduce, s);
        default: return go_f64<2>(p, n, e2, G, o, tbeg, tcount, t, partial, reduce, s);
        }
    }
    const float4 *p = (const float4 *)pm;
    float4 *o = (float4 *)out;
    const float e2 = eps2_f32(eps);
    switch (prec) {
    case NBODY_F32: return by_tpl_f32<M_F32>(p, n, e2, G, o, tbeg, tcount, t, partial, reduce, s);
    case NBODY_F32_KAHAN: return by_tpl_f32<M_KAHAN>(p, n, e2, G, o, tbeg, tcount, t, partial, reduce, s);
    default: return by_tpl_f32<M_F64ACC>(p, n, e2, G, o, tbeg, tcount, t, partial, reduce, s);
    }
}

hipError_t launch_batched(int prec, const void *pm, const int64_t *offsets, const int2 *units,
                          int nunits, double G, const float *eps_sys, double eps, void *out,
                          const Tune &t, unsigned *counter, int grid, hipStream_t s)
{
    if (prec == NBODY_F64) {
        const double4 *p = (const double4 *)pm;
        double4 *o = (double4 *)out;
        if (t.tpl == 1)
            hipLaunchKernelGGL((k_batched_f64<1>), dim3(grid), dim3(kBlock), 0, s, p, offsets, units,
                               nunits, eps_sys, eps * eps, G, t.jtile, o, counter);
        else
            hipLaunchKernelGGL((k_batched_f64<2>), dim3(grid), dim3(kBlock), 0, s, p, offsets, units,
                               nunits, eps_sys, eps * eps, G, t.jtile, o, counter);
        return hipGetLastError();
    }
    const float4 *p = (const float4 *)pm;
    float4 *o = (float4 *)out;
    const float e2 = eps2_f32(eps);
    switch (prec) {
    case NBODY_F32: return batched_by_tpl<M_F32>(p, offsets, units, nunits, eps_sys, e2, G, o, t, counter, grid, s);
    case NBODY_F32_KAHAN: return batched_by_tpl<M_KAHAN>(p, offsets, units, nunits, eps_sys, e2, G, o, t, counter, grid, s);
    default: return batched_by_tpl<M_F64ACC>(p, offsets, units, nunits, eps_sys, e2, G, o, t, counter, grid, s);
    }
}

// ---- static split scratch (nbody_accel_noalloc) -------------------------------
// The split partials of the entry point that allocates nothing live in this
// file-scope device array; every GPU the library runs on holds its own copy
// for the life of the process.  Host code never passes the array's name to a
// kernel: its device address is looked up once per device with
// hipGetSymbolAddress and that address is what the kernels receive.
__device__ __align__(256) static unsigned char g_split_scratch[kStaticScratchBytes];

void *static_split_scratch()
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the static scratch table covers", dev, kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_split_scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(static split scratch): %s", hipGetErrorString(e));
            return nullptr;
        }
        addr[dev] = p;
    }
    return addr[dev];
}

}  // namespace nbi
