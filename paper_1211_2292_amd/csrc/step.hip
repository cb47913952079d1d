// Elementwise kernels around the force evaluation: the leapfrog kicks and
// drift (the paper's Move_bodies, Section IV.B pseudo-code, read as
// kick-drift-kick with one force evaluation per step), the FP64 energy
// diagnostics, and record permutations for the ORB order.
//
// All are HBM-bound streams over 16- or 32-byte records: one record per lane,
// coalesced 16-byte vector loads and stores, workgroups of 256 lanes.
#include <type_traits>

#include "internal.h"

namespace nbi {
namespace {

// Fixed-order block reduction of two doubles; thread 0 holds the result.
__device__ __forceinline__ void block_sum2(double &a, double &b)
{
    __shared__ double sa[kBlock], sb[kBlock];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] += sa[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    a = sa[0];
    b = sb[0];
}

// close: v += h a;  energy partials (1/2 m |v|^2, 1/2 m phi) in FP64;
// open: v += h a; x += dt v.
template <typename V, typename S>
__device__ __forceinline__ void step_one(V *__restrict__ pm, V *__restrict__ vel, int i, const V a,
                                         S h, S dt, int close, int open, bool energy, double &ek,
                                         double &eu)
{
    V x = pm[i];
    V v = vel[i];
    if (close) {
        v.x = v.x + h * a.x;
        v.y = v.y + h * a.y;
        v.z = v.z + h * a.z;
    }
    if (energy) {
        const double vx = v.x, vy = v.y, vz = v.z, m = x.w;
        ek = 0.5 * m * ((vx * vx + vy * vy) + vz * vz);
        eu = 0.5 * m * (double)a.w;
    }
    if (open) {
        v.x = v.x + h * a.x;
        v.y = v.y + h * a.y;
        v.z = v.z + h * a.z;
        x.x = x.x + dt * v.x;
        x.y = x.y + dt * v.y;
        x.z = x.z + dt * v.z;
        pm[i] = x;
    }
    if (close || open) vel[i] = v;
}

template <typename V, typename S>
__global__ __launch_bounds__(kBlock) void k_step(V *__restrict__ pm, V *__restrict__ vel,
                                                 const V *__restrict__ acc, int n, S h, S dt,
                                                 int close, int open, double *__restrict__ epart)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double ek = 0.0, eu = 0.0;
    if (i < n) step_one(pm, vel, i, acc[i], h, dt, close, open, epart != nullptr, ek, eu);
    if (epart) {
        block_sum2(ek, eu);
        if (threadIdx.x == 0) {
            epart[2 * blockIdx.x] = ek;
            epart[2 * blockIdx.x + 1] = eu;
        }
    }
}

// The force kernel's source-split reduction and the step in one pass: the
// js partial records of body i are summed in split order and scaled exactly
// as the stand-alone reduction does (R = the partials' type, GT = the type G
// is applied in), the record is stored to acc, and the same value drives the
// kick, drift and energy partials.  Results equal reduce-then-step bit for
// bit; one launch and one pass over acc fewer.
template <typename V, typename S, typename P, typename R, typename GT>
__global__ __launch_bounds__(kBlock) void k_reduce_step(const P *__restrict__ partial, int js, GT G,
                                                        V *__restrict__ pm, V *__restrict__ vel,
                                                        V *__restrict__ acc, int n, S h, S dt,
                                                        int close, int open,
                                                        double *__restrict__ epart)
{
    using E = typename std::conditional<sizeof(V) == 16, float, double>::type;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double ek = 0.0, eu = 0.0;
    if (i < n) {
        R r[4] = {R(0), R(0), R(0), R(0)};
        for (int k = 0; k < js; ++k) {
            const P q = partial[(long)k * n + i];
            r[0] += q.x;
            r[1] += q.y;
            r[2] += q.z;
            r[3] += q.w;
        }
        V a;
        a.x = (E)(G * r[0]);
        a.y = (E)(G * r[1]);
        a.z = (E)(G * r[2]);
        a.w = (E)(-G * r[3]);
        acc[i] = a;
        step_one(pm, vel, i, a, h, dt, close, open, epart != nullptr, ek, eu);
    }
    if (epart) {
        block_sum2(ek, eu);
        if (threadIdx.x == 0) {
            epart[2 * blockIdx.x] = ek;
            epart[2 * blockIdx.x + 1] = eu;
        }
    }
}

// One workgroup: each lane sums a strided subset of the block partials in
// order, then a fixed-order tree.
__global__ __launch_bounds__(kBlock) void k_energy_final(const double *__restrict__ epart,
                                                         int nblocks, double *__restrict__ out)
{
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += kBlock) {
        a += epart[2 * k];
        b += epart[2 * k + 1];
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_permute(const R *__restrict__ src, R *__restrict__ dst,
                                                    const int32_t *__restrict__ perm, int n,
                                                    int inverse)
{
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int q = perm[p];
    if ((unsigned)q >= (unsigned)n) return;  // not a permutation entry: no access
    if (inverse)
        dst[q] = src[p];
    else
        dst[p] = src[q];
}

__global__ __launch_bounds__(kBlock) void k_copy16(const float4 *__restrict__ src,
                                                   float4 *__restrict__ dst, size_t nrec)
{
    const size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < nrec) dst[k] = src[k];
}

__global__ __launch_bounds__(kBlock) void k_zero4(uint32_t *__restrict__ p, size_t nwords)
{
    const size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < nwords) p[k] = 0u;
}

}  // namespace

// Zero fill as a kernel (no memset node in captured graphs); bytes must be a
// multiple of 4.
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    const size_t nw = bytes / 4;
    const size_t nb = (nw + kBlock - 1) / kBlock;
    if (nw) hipLaunchKernelGGL(k_zero4, dim3((unsigned)nb), dim3(kBlock), 0, s, (uint32_t *)p, nw);
    return hipGetLastError();
}

int step_blocks(int n) { return (n + kBlock - 1) / kBlock; }

hipError_t launch_step(int prec, void *pm, void *vel, const void *acc, int n, double h, double dt,
                       bool close, bool open, double *epart, int *eblocks, hipStream_t s)
{
    const int nb = step_blocks(n);
    if (eblocks) *eblocks = nb;
    if (prec == NBODY_F64)
        hipLaunchKernelGGL((k_step<double4, double>), dim3(nb), dim3(kBlock), 0, s, (double4 *)pm,
                           (double4 *)vel, (const double4 *)acc, n, h, dt, (int)close, (int)open,
                           epart);
    else
        hipLaunchKernelGGL((k_step<float4, float>), dim3(nb), dim3(kBlock), 0, s, (float4 *)pm,
                           (float4 *)vel, (const float4 *)acc, n, (float)h, (float)dt, (int)close,
                           (int)open, epart);
    return hipGetLastError();
}

hipError_t launch_reduce_step(int prec, const void *partial, int js, double G, void *pm, void *vel,
                              void *acc, int n, double h, double dt, bool close, bool open,
                              double *epart, int *eblocks, hipStream_t s)
{
    const int nb = step_blocks(n);
    if (eblocks) *eblocks = nb;
    if (prec == NBODY_F64)
        hipLaunchKernelGGL((k_reduce_step<double4, double, double4, double, double>), dim3(nb),
                           dim3(kBlock), 0, s, (const double4 *)partial, js, G, (double4 *)pm,
                           (double4 *)vel, (double4 *)acc, n, h, dt, (int)close, (int)open, epart);
    else if (prec == NBODY_F32)
        hipLaunchKernelGGL((k_reduce_step<float4, float, float4, float, float>), dim3(nb),
                           dim3(kBlock), 0, s, (const float4 *)partial, js, (float)G, (float4 *)pm,
                           (float4 *)vel, (float4 *)acc, n, (float)h, (float)dt, (int)close,
                           (int)open, epart);
    else
        hipLaunchKernelGGL((k_reduce_step<float4, float, double4, double, double>), dim3(nb),
                           dim3(kBlock), 0, s, (const double4 *)partial, js, G, (float4 *)pm,
                           (float4 *)vel, (float4 *)acc, n, (float)h, (float)dt, (int)close,
                           (int)open, epart);
    return hipGetLastError();
}

hipError_t launch_energy_final(const double *epart, int nblocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s, epart, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_permute(const void *src, void *dst, const int32_t *perm, int n, int rec_bytes,
                          bool inverse, hipStream_t s)
{
    const int nb = (n + kBlock - 1) / kBlock;
    if (rec_bytes == 16)
        hipLaunchKernelGGL((k_permute<float4>), dim3(nb), dim3(kBlock), 0, s, (const float4 *)src,
                           (float4 *)dst, perm, n, (int)inverse);
    else
        hipLaunchKernelGGL((k_permute<double4>), dim3(nb), dim3(kBlock), 0, s,
                           (const double4 *)src, (double4 *)dst, perm, n, (int)inverse);
    return hipGetLastError();
}

// Device-to-device copy as a kernel (16-byte records), so that it can sit in
// captured graphs without a memcpy node.
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t nrec = bytes / 16;
    const size_t nb = (nrec + kBlock - 1) / kBlock;
    if (nrec) hipLaunchKernelGGL(k_copy16, dim3((unsigned)nb), dim3(kBlock), 0, s, (const float4 *)src, (float4 *)dst, nrec);
    return hipGetLastError();
}

}  // namespace nbi
