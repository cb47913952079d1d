// Bit-reversible kick-drift-kick with fixed-point state, and its adjoint
// without checkpoints (gfx950).
//
// The leapfrog of the paper's Move_bodies step (Section IV.B), with
// positions and velocities held as integers in units of 2^-sx and 2^-sv (the
// integer-state idea of Rein and Tamayo's JANUS integrator):
//   kick:  V += round(h G 2^sv * a(x)),   drift: X += round(V * dt 2^(sx-sv))
// rounded to nearest even in FP64.  Every increment depends only on the
// state it does not change, so subtracting the same integers undoes a step
// exactly: the adjoint rebuilds every position bit for bit from the final
// state alone, and needs no checkpoints.
//
// Exact undoing needs the same force bits in the reverse pass.  The reverse
// pass gets the force from the fused VJP kernel (mass-scaled form), which
// uses the force kernel's pair arithmetic, tiles and split order; both are
// launched with G = 1 (G sits in the kick and in the cotangent scale), in
// NBODY_F32_F64ACC, with one explicit kernel shape, so the two forces are the
// same FP32 values.  Masses must be positive (the general VJP form used for
// zero masses rounds the force differently); the adjoint checks this once.
//
// State layout: 2n longlong4 records, [0, n) = (X, Y, Z, 0), [n, 2n) =
// (VX, VY, VZ, 0).  Positions and masses for the force kernels are decoded
// into a float4 array (x = X 2^-sx rounded to FP32, w = m).
#include <cmath>

#include "internal.h"

namespace nbi {
namespace {

__device__ __forceinline__ long long kick_inc(float a, double kick_scale)
{
    return __double2ll_rn(kick_scale * (double)a);
}

__device__ __forceinline__ long long drift_inc(long long v, double drift_scale)
{
    return __double2ll_rn((double)v * drift_scale);
}

__global__ __launch_bounds__(kBlock) void k_janus_encode(const float4 *__restrict__ pm,
                                                         const float4 *__restrict__ vel, int n,
                                                         double sx_scale, double sv_scale, double inv_sx,
                                                         longlong4 *__restrict__ st,
                                                         float4 *__restrict__ dec)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float4 p = pm[i], v = vel[i];
    longlong4 X, V;
    X.x = __double2ll_rn((double)p.x * sx_scale);
    X.y = __double2ll_rn((double)p.y * sx_scale);
    X.z = __double2ll_rn((double)p.z * sx_scale);
    X.w = 0;
    V.x = __double2ll_rn((double)v.x * sv_scale);
    V.y = __double2ll_rn((double)v.y * sv_scale);
    V.z = __double2ll_rn((double)v.z * sv_scale);
    V.w = 0;
    st[i] = X;
    st[n + i] = V;
    dec[i] = make_float4((float)((double)X.x * inv_sx), (float)((double)X.y * inv_sx),
                         (float)((double)X.z * inv_sx), p.w);
}

// Decoded positions with the masses of pm.
__global__ __launch_bounds__(kBlock) void k_janus_decode(const longlong4 *__restrict__ st,
                                                         const float4 *__restrict__ pm, int n,
                                                         double inv_sx, float4 *__restrict__ dec)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const longlong4 X = st[i];
    dec[i] = make_float4((float)((double)X.x * inv_sx), (float)((double)X.y * inv_sx),
                         (float)((double)X.z * inv_sx), pm[i].w);
}

// sign +1: `kicks` kicks with acc, then a drift if `drift`; sign -1: the exact
// inverse (un-kick, then un-drift).  Re-decodes the positions after a drift.
__global__ __launch_bounds__(kBlock) void k_janus_step(longlong4 *__restrict__ st,
                                                       const float4 *__restrict__ acc, int n,
                                                       double kick_scale, int kicks, int drift,
                                                       double drift_scale, double inv_sx, int sign,
                                                       float4 *__restrict__ dec)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    longlong4 V = st[n + i];
    if (kicks) {
        const float4 a = acc[i];
        const long long k = (long long)kicks * sign;
        V.x += k * kick_inc(a.x, kick_scale);
        V.y += k * kick_inc(a.y, kick_scale);
        V.z += k * kick_inc(a.z, kick_scale);
        st[n + i] = V;
    }
    if (drift) {
        longlong4 X = st[i];
        X.x += sign * drift_inc(V.x, drift_scale);
        X.y += sign * drift_inc(V.y, drift_scale);
        X.z += sign * drift_inc(V.z, drift_scale);
        st[i] = X;
        const float m = dec[i].w;
        dec[i] = make_float4((float)((double)X.x * inv_sx), (float)((double)X.y * inv_sx),
                             (float)((double)X.z * inv_sx), m);
    }
}

// Decoded velocities (v = V 2^-sv rounded to FP32).
__global__ __launch_bounds__(kBlock) void k_janus_velocity(const longlong4 *__restrict__ st, int n,
                                                           double inv_sv, float4 *__restrict__ vel)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const longlong4 V = st[n + i];
    vel[i] = make_float4((float)((double)V.x * inv_sv), (float)((double)V.y * inv_sv),
                         (float)((double)V.z * inv_sv), 0.0f);
}

struct Scales {
    double sx_scale, sv_scale, inv_sx, inv_sv, kick_scale, drift_scale;
};

Scales scales(int sx, int sv, double G, double dt)
{
    Scales c;
    c.sx_scale = std::ldexp(1.0, sx);
    c.sv_scale = std::ldexp(1.0, sv);
    c.inv_sx = std::ldexp(1.0, -sx);
    c.inv_sv = std::ldexp(1.0, -sv);
    c.kick_scale = 0.5 * dt * G * c.sv_scale;
    c.drift_scale = dt * std::ldexp(1.0, sx - sv);
    return c;
}

hipError_t step(longlong4 *st, const float4 *acc, int n, const Scales &c, int kicks, int drift, int sign,
                float4 *dec, hipStream_t s)
{
    hipLaunchKernelGGL(k_janus_step, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, st, acc, n,
                       c.kick_scale, kicks, drift, c.drift_scale, c.inv_sx, sign, dec);
    return hipGetLastError();
}

}  // namespace

// One kernel shape for both the force kernel and the fused VJP.
Tune janus_tune(const Tune &vjp_default)
{
    Tune t = vjp_default;
    t.tpl = 1;
    t.variant = 0;
    return t;
}

int janus_forward(const void *pm, const void *vel, int n, double G, double eps, double dt, int nsteps, int sx,
                  int sv, const Tune &t, void *state, void *pm_out, void *vel_out, void *acc, void *partial,
                  hipStream_t s)
{
    const Scales c = scales(sx, sv, G, dt);
    longlong4 *st = (longlong4 *)state;
    float4 *dec = (float4 *)pm_out;
    const dim3 grid((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_janus_encode, grid, dim3(kBlock), 0, s, (const float4 *)pm, (const float4 *)vel, n,
                       c.sx_scale, c.sv_scale, c.inv_sx, st, dec);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_accel(NBODY_F32_F64ACC, dec, n, 1.0, eps, acc, 0, n, t, partial, s);
    if (e != hipSuccess) return hip_fail(e, "janus forward");
    for (int k = 0; k < nsteps; ++k) {
        e = step(st, (const float4 *)acc, n, c, k == 0 ? 1 : 2, 1, 1, dec, s);
        if (e == hipSuccess) e = launch_accel(NBODY_F32_F64ACC, dec, n, 1.0, eps, acc, 0, n, t, partial, s);
        if (e != hipSuccess) return hip_fail(e, "janus step");
    }
    if (nsteps > 0) {
        e = step(st, (const float4 *)acc, n, c, 1, 0, 1, dec, s);
        if (e != hipSuccess) return hip_fail(e, "janus step");
    }
    if (vel_out) {
        hipLaunchKernelGGL(k_janus_velocity, grid, dim3(kBlock), 0, s, (const longlong4 *)st, n, c.inv_sv,
                           (float4 *)vel_out);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "janus velocity");
    }
    return NBODY_OK;
}

int janus_decode(const void *state, const void *pm, int n, int sx, void *dec, hipStream_t s)
{
    hipLaunchKernelGGL(k_janus_decode, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       (const longlong4 *)state, (const float4 *)pm, n, std::ldexp(1.0, -sx), (float4 *)dec);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "janus decode");
}

int janus_unstep(void *state, const void *acc, int n, double G, double dt, int sx, int sv, int kicks, int drift,
                 void *dec, hipStream_t s)
{
    const Scales c = scales(sx, sv, G, dt);
    const hipError_t e = step((longlong4 *)state, (const float4 *)acc, n, c, kicks, drift, -1, (float4 *)dec, s);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "janus reverse step");
}

}  // namespace nbi
