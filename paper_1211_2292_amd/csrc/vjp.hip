// Fused force + vector-Jacobian product of the direct sum (gfx950).
//
// The paper has no derivatives; this is the reverse-mode derivative of the
// force law of Section IV (see nbody.h).  With d = x_j - x_k,
// q = |d|^2 + eps^2, rho = q^(-1/2), w = rho^3, u = rho^5 and
// T_kj = w I - 3 u d d^T:
//     xbar_k = G sum_{j != k} T_kj (m_k abar_j - m_j abar_k)
//              - G m_k sum_{j != k} phibar_j w d  - phibar_k a_k
//     mbar_k = -G sum_{j != k} w d . abar_j  - G sum_{j != k} phibar_j rho
// and, in the same sweep, the forward a_k and phi_k.
//
// Per wave: 64*TPL targets in VGPRs; each source brings its position/mass
// and its cotangent record through wave-uniform scalar loads.  Per pair the
// sweep accumulates
//     P  += w e                 e = m_k abar_j - m_j abar_k
//     Q  += (w rho^2)(d . e) d  -> xbar = G (P - 3 Q) + ...
//     M  += w (d . abar_j)      -> mbar = -G M + ...
//     A  += m_j w d, F += m_j rho        (forward force and potential)
//     B  += phibar_j w d, H += phibar_j rho   (only with phibar)
// FP32 tile partials are folded into FP64 running sums for the FP32 modes;
// the FP64 mode runs the same sweep in FP64.
//
// `scale` multiplies the cotangent (the product is linear in it) and
// `accumulate` adds the result into the existing pos_cot/mass_cot, which is
// how the trajectory adjoint applies one VJP per position without extra
// passes.
#include "internal.h"

namespace nbi {
namespace {

constexpr int kVjpUnroll = 2;  // sources per unrolled step (measured: 2 beats 1, 3 and 4)

// eps^2 is kept in a vector register in FP32 (see lane_copy); FP64 keeps the
// compiler's choice.
template <typename T>
__device__ __forceinline__ T lane_copy_t(T x) { return x; }
template <>
__device__ __forceinline__ float lane_copy_t<float>(float x) { return lane_copy(x); }

template <typename T, int TPL, bool PHI>
struct VAcc {
    T P[TPL][3], Q[TPL][3], M[TPL], A[TPL][3], F[TPL];
    T B[TPL][3], H[TPL];
    __device__ void zero()
    {
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
#pragma unroll
            for (int c = 0; c < 3; ++c) P[t][c] = Q[t][c] = A[t][c] = B[t][c] = T(0);
            M[t] = F[t] = H[t] = T(0);
        }
    }
};

template <typename T, int TPL>
struct VTgt {
    T x[TPL][3], m[TPL], ab[TPL][3], pb[TPL];
    int i[TPL];
};

// Fused multiply-add in the precision of T (no promotion of float to double).
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T rsq_t(T q);
template <>
__device__ __forceinline__ float rsq_t<float>(float q)
{
    return __builtin_amdgcn_rsqf(q);
}
template <>
__device__ __forceinline__ double rsq_t<double>(double q)
{
    double y = __builtin_amdgcn_rsq(q);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = __builtin_fma(-q, y * y, 1.0);
        y = __builtin_fma(0.5 * y, e, y);
    }
    return y;
}

template <typename T, typename V, int TPL, bool PHI, bool MASK>
__device__ __forceinline__ void vpair(const V p, const V c, const int j, const VTgt<T, TPL> &K,
                                      const T eps2, VAcc<T, TPL, PHI> &S)
{
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const T d0 = p.x - K.x[t][0];
        const T d1 = p.y - K.x[t][1];
        const T d2 = p.z - K.x[t][2];
        const T q = fmat(d2, d2, fmat(d1, d1, fmat(d0, d0, eps2)));
        T rho = rsq_t<T>(q);
        if (MASK) rho = (j == K.i[t]) ? T(0) : rho;
        const T r2 = rho * rho;
        const T w = rho * r2;
        const T e0 = fmat(-p.w, K.ab[t][0], K.m[t] * c.x);
        const T e1 = fmat(-p.w, K.ab[t][1], K.m[t] * c.y);
        const T e2 = fmat(-p.w, K.ab[t][2], K.m[t] * c.z);
        const T de = fmat(d2, e2, fmat(d1, e1, d0 * e0));
        const T da = fmat(d2, c.z, fmat(d1, c.y, d0 * c.x));
        const T uq = (w * r2) * de;
        S.P[t][0] = fmat(w, e0, S.P[t][0]);
        S.P[t][1] = fmat(w, e1, S.P[t][1]);
        S.P[t][2] = fmat(w, e2, S.P[t][2]);
        S.Q[t][0] = fmat(uq, d0, S.Q[t][0]);
        S.Q[t][1] = fmat(uq, d1, S.Q[t][1]);
        S.Q[t][2] = fmat(uq, d2, S.Q[t][2]);
        S.M[t] = fmat(w, da, S.M[t]);
        const T mw = p.w * w;
        S.A[t][0] = fmat(mw, d0, S.A[t][0]);
        S.A[t][1] = fmat(mw, d1, S.A[t][1]);
        S.A[t][2] = fmat(mw, d2, S.A[t][2]);
        S.F[t] = fmat(p.w, rho, S.F[t]);
        if (PHI) {
            const T pw = c.w * w;
            S.B[t][0] = fmat(pw, d0, S.B[t][0]);
            S.B[t][1] = fmat(pw, d1, S.B[t][1]);
            S.B[t][2] = fmat(pw, d2, S.B[t][2]);
            S.H[t] = fmat(c.w, rho, S.H[t]);
        }
    }
}

template <typename T, typename V, int TPL, bool PHI, bool MASK>
__device__ __forceinline__ void vsweep(const V *__restrict__ pm, const V *__restrict__ cot, int j0,
                                       int j1, const VTgt<T, TPL> &K, T eps2,
                                       VAcc<T, TPL, PHI> &S)
{
    int j = j0;
    for (; j + kVjpUnroll <= j1; j += kVjpUnroll) {
        V p[kVjpUnroll], c[kVjpUnroll];
#pragma unroll
        for (int u = 0; u < kVjpUnroll; ++u) {
            p[u] = pm[j + u];
            c[u] = cot[j + u];
        }
#pragma unroll
        for (int u = 0; u < kVjpUnroll; ++u) vpair<T, V, TPL, PHI, MASK>(p[u], c[u], j + u, K, eps2, S);
    }
    for (; j < j1; ++j) vpair<T, V, TPL, PHI, MASK>(pm[j], cot[j], j, K, eps2, S);
}

// Number of accumulated scalars per target.
constexpr int kVN = 17;

template <typename T, int TPL, bool PHI>
__device__ __forceinline__ void vflatten(const VAcc<T, TPL, PHI> &S, int t, T (&f)[kVN])
{
    f[0] = S.P[t][0]; f[1] = S.P[t][1]; f[2] = S.P[t][2];
    f[3] = S.Q[t][0]; f[4] = S.Q[t][1]; f[5] = S.Q[t][2];
    f[6] = S.M[t];
    f[7] = S.A[t][0]; f[8] = S.A[t][1]; f[9] = S.A[t][2];
    f[10] = S.F[t];
    f[11] = S.B[t][0]; f[12] = S.B[t][1]; f[13] = S.B[t][2];
    f[14] = S.H[t];
    f[15] = 0; f[16] = 0;
}

// Output of one target: xbar (3), mbar, a (3), phi, all linear in the sums,
// so per-split values add up to the full result.
__device__ __forceinline__ void apply_out(double (&o)[8], double scale, int accumulate, int i,
                                          float4 *pos_cot, float *mass_cot, float4 *acc_out)
{
    double gx = o[0] * scale, gy = o[1] * scale, gz = o[2] * scale, gm = o[3] * scale;
    if (accumulate) {
        const float4 p = pos_cot[i];
        gx += (double)p.x;
        gy += (double)p.y;
        gz += (double)p.z;
        gm += (double)mass_cot[i];
    }
    pos_cot[i] = make_float4((float)gx, (float)gy, (float)gz, 0.0f);
    mass_cot[i] = (float)gm;
    if (acc_out) acc_out[i] = make_float4((float)o[4], (float)o[5], (float)o[6], (float)o[7]);
}
__device__ __forceinline__ void apply_out(double (&o)[8], double scale, int accumulate, int i,
                                          double4 *pos_cot, double *mass_cot, double4 *acc_out)
{
    double gx = o[0] * scale, gy = o[1] * scale, gz = o[2] * scale, gm = o[3] * scale;
    if (accumulate) {
        const double4 p = pos_cot[i];
        gx += p.x;
        gy += p.y;
        gz += p.z;
        gm += mass_cot[i];
    }
    pos_cot[i] = make_double4(gx, gy, gz, 0.0);
    mass_cot[i] = gm;
    if (acc_out) acc_out[i] = make_double4(o[4], o[5], o[6], o[7]);
}

template <typename T, typename V, typename MT, int TPL, bool PHI>
__device__ __forceinline__ void vjp_general(const V *__restrict__ pm, const V *__restrict__ cot,
                                            int n, T eps2_in, double G, int jtile, double scale,
                                            int accumulate, V *__restrict__ pos_cot,
                                            MT *__restrict__ mass_cot, V *__restrict__ acc_out,
                                            double4 *__restrict__ partial)
{
    constexpr int WT = 64 * TPL;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t0 = (blockIdx.x * (kBlock / 64) + wave) * WT;
    if (t0 >= n) return;
    const T eps2 = lane_copy_t(eps2_in);
    // source range of this split
    const long per = ((long)n + gridDim.y - 1) / gridDim.y;
    const int jb = (int)min((long)n, (long)blockIdx.y * per);
    const int je = (int)min((long)n, (long)jb + per);
    VTgt<T, TPL> K;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        K.i[t] = i;
        const int ic = min(i, n - 1);
        const V p = pm[ic];
        const V c = cot[ic];
        K.x[t][0] = p.x; K.x[t][1] = p.y; K.x[t][2] = p.z;
        K.m[t] = p.w;
        K.ab[t][0] = c.x; K.ab[t][1] = c.y; K.ab[t][2] = c.z;
        K.pb[t] = c.w;
    }
    const int d0 = t0, d1 = t0 + WT;
    double R[TPL][kVN];
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < kVN; ++c) R[t][c] = 0.0;
    VAcc<T, TPL, PHI> S;
    for (int jc = jb, ce; jc < je; jc = ce) {
        ce = je - jc > jtile ? jc + jtile : je;  // no jc + jtile past je (int range)
        const int lo = min(max(d0, jc), ce);
        const int hi = min(max(d1, jc), ce);
        S.zero();
        vsweep<T, V, TPL, PHI, false>(pm, cot, jc, lo, K, eps2, S);
        vsweep<T, V, TPL, PHI, true>(pm, cot, lo, hi, K, eps2, S);
        vsweep<T, V, TPL, PHI, false>(pm, cot, hi, ce, K, eps2, S);
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            T f[kVN];
            vflatten(S, t, f);
#pragma unroll
            for (int c = 0; c < 15; ++c) R[t][c] += (double)f[c];
        }
    }
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        if (i >= n) continue;
        const double mk = K.m[t];
        const double pbk = PHI ? (double)K.pb[t] : 0.0;
        double o[8];
        o[4] = G * R[t][7];
        o[5] = G * R[t][8];
        o[6] = G * R[t][9];
        o[7] = -G * R[t][10];
        o[0] = G * (R[t][0] - 3.0 * R[t][3]);
        o[1] = G * (R[t][1] - 3.0 * R[t][4]);
        o[2] = G * (R[t][2] - 3.0 * R[t][5]);
        o[3] = -G * R[t][6];
        if (PHI) {
            o[0] += -G * mk * R[t][11] - pbk * o[4];
            o[1] += -G * mk * R[t][12] - pbk * o[5];
            o[2] += -G * mk * R[t][13] - pbk * o[6];
            o[3] += -G * R[t][14];
        }
        if (gridDim.y == 1) {
            apply_out(o, scale, accumulate, i, pos_cot, mass_cot, acc_out);
        } else {
            double4 *dst = partial + 2 * ((long)blockIdx.y * n + i);
            dst[0] = make_double4(o[0], o[1], o[2], o[3]);
            dst[1] = make_double4(o[4], o[5], o[6], o[7]);
        }
    }
}

template <typename T, typename V, typename MT, int TPL, bool PHI>
__global__ __launch_bounds__(kBlock) void k_vjp(const V *__restrict__ pm, const V *__restrict__ cot,
                                                int n, T eps2, double G, int jtile, double scale,
                                                int accumulate, V *__restrict__ pos_cot,
                                                MT *__restrict__ mass_cot, V *__restrict__ acc_out,
                                                double4 *__restrict__ partial)
{
    vjp_general<T, V, MT, TPL, PHI>(pm, cot, n, eps2, G, jtile, scale, accumulate, pos_cot, mass_cot,
                                    acc_out, partial);
}

// ---- mass-scaled form (all masses positive) ----------------------------------
// With at = abar / m per body, e = at_j - at_k and s1 = m_j w:
//   xbar_k = G m_k [sum s1 e - 3 sum (s1 rho^2)(d . e) d]
//   mbar_k = -G [sum s1 (d . e) + at_k . sum s1 d],   a_k = G sum s1 d
// 28 VALU per pair (no potential), against 34 for the general form.
template <typename T, int TPL>
struct SAcc {
    T P[TPL][3], Q[TPL][3], M[TPL], F[TPL][3];
    __device__ void zero()
    {
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
#pragma unroll
            for (int c = 0; c < 3; ++c) P[t][c] = Q[t][c] = F[t][c] = T(0);
            M[t] = T(0);
        }
    }
};

template <typename T, typename V, int TPL, bool MASK>
__device__ __forceinline__ void spair(const V p, const V c, const int j, const VTgt<T, TPL> &K,
                                      const T eps2, SAcc<T, TPL> &S)
{
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const T d0 = p.x - K.x[t][0];
        const T d1 = p.y - K.x[t][1];
        const T d2 = p.z - K.x[t][2];
        const T q = fmat(d2, d2, fmat(d1, d1, fmat(d0, d0, eps2)));
        T rho = rsq_t<T>(q);
        if (MASK) rho = (j == K.i[t]) ? T(0) : rho;
        const T r2 = rho * rho;
        const T s1 = (p.w * rho) * r2;
        const T e0 = c.x - K.ab[t][0];
        const T e1 = c.y - K.ab[t][1];
        const T e2 = c.z - K.ab[t][2];
        const T de = fmat(d2, e2, fmat(d1, e1, d0 * e0));
        const T tq = (s1 * r2) * de;
        S.P[t][0] = fmat(s1, e0, S.P[t][0]);
        S.P[t][1] = fmat(s1, e1, S.P[t][1]);
        S.P[t][2] = fmat(s1, e2, S.P[t][2]);
        S.Q[t][0] = fmat(tq, d0, S.Q[t][0]);
        S.Q[t][1] = fmat(tq, d1, S.Q[t][1]);
        S.Q[t][2] = fmat(tq, d2, S.Q[t][2]);
        S.M[t] = fmat(s1, de, S.M[t]);
        S.F[t][0] = fmat(s1, d0, S.F[t][0]);
        S.F[t][1] = fmat(s1, d1, S.F[t][1]);
        S.F[t][2] = fmat(s1, d2, S.F[t][2]);
    }
}

template <typename T, typename V, int TPL, bool MASK>
__device__ __forceinline__ void ssweep(const V *__restrict__ pm, const V *__restrict__ cot, int j0,
                                       int j1, const VTgt<T, TPL> &K, T eps2, SAcc<T, TPL> &S)
{
    int j = j0;
    for (; j + kVjpUnroll <= j1; j += kVjpUnroll) {
        V p[kVjpUnroll], c[kVjpUnroll];
#pragma unroll
        for (int u = 0; u < kVjpUnroll; ++u) {
            p[u] = pm[j + u];
            c[u] = cot[j + u];
        }
#pragma unroll
        for (int u = 0; u < kVjpUnroll; ++u) spair<T, V, TPL, MASK>(p[u], c[u], j + u, K, eps2, S);
    }
    for (; j < j1; ++j) spair<T, V, TPL, MASK>(pm[j], cot[j], j, K, eps2, S);
}

template <typename T, typename V, typename MT, int TPL>
__device__ __forceinline__ void vjp_scaled(const V *__restrict__ pm, const V *__restrict__ sc,
                                           int n, T eps2_in, double G, int jtile, double scale,
                                           int accumulate, V *__restrict__ pos_cot,
                                           MT *__restrict__ mass_cot, V *__restrict__ acc_out,
                                           double4 *__restrict__ partial)
{
    constexpr int WT = 64 * TPL;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t0 = (blockIdx.x * (kBlock / 64) + wave) * WT;
    if (t0 >= n) return;
    const T eps2 = lane_copy_t(eps2_in);
    const long per = ((long)n + gridDim.y - 1) / gridDim.y;
    const int jb = (int)min((long)n, (long)blockIdx.y * per);
    const int je = (int)min((long)n, (long)jb + per);
    VTgt<T, TPL> K;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        K.i[t] = i;
        const int ic = min(i, n - 1);
        const V p = pm[ic];
        const V c = sc[ic];
        K.x[t][0] = p.x; K.x[t][1] = p.y; K.x[t][2] = p.z;
        K.m[t] = p.w;
        K.ab[t][0] = c.x; K.ab[t][1] = c.y; K.ab[t][2] = c.z;
        K.pb[t] = T(0);
    }
    const int d0 = t0, d1 = t0 + WT;
    double R[TPL][10];
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int c = 0; c < 10; ++c) R[t][c] = 0.0;
    SAcc<T, TPL> S;
    for (int jc = jb, ce; jc < je; jc = ce) {
        ce = je - jc > jtile ? jc + jtile : je;  // no jc + jtile past je (int range)
        const int lo = min(max(d0, jc), ce);
        const int hi = min(max(d1, jc), ce);
        S.zero();
        ssweep<T, V, TPL, false>(pm, sc, jc, lo, K, eps2, S);
        ssweep<T, V, TPL, true>(pm, sc, lo, hi, K, eps2, S);
        ssweep<T, V, TPL, false>(pm, sc, hi, ce, K, eps2, S);
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                R[t][c] += (double)S.P[t][c];
                R[t][3 + c] += (double)S.Q[t][c];
                R[t][6 + c] += (double)S.F[t][c];
            }
            R[t][9] += (double)S.M[t];
        }
    }
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = t0 + t * 64 + lane;
        if (i >= n) continue;
        const double gm_k = G * (double)K.m[t];
        double o[8];
        o[0] = gm_k * (R[t][0] - 3.0 * R[t][3]);
        o[1] = gm_k * (R[t][1] - 3.0 * R[t][4]);
        o[2] = gm_k * (R[t][2] - 3.0 * R[t][5]);
        o[3] = -G * (R[t][9] + (double)K.ab[t][0] * R[t][6] + (double)K.ab[t][1] * R[t][7] +
                     (double)K.ab[t][2] * R[t][8]);
        o[4] = G * R[t][6];
        o[5] = G * R[t][7];
        o[6] = G * R[t][8];
        o[7] = 0.0;
        if (gridDim.y == 1) {
            apply_out(o, scale, accumulate, i, pos_cot, mass_cot, acc_out);
        } else {
            double4 *dst = partial + 2 * ((long)blockIdx.y * n + i);
            dst[0] = make_double4(o[0], o[1], o[2], o[3]);
            dst[1] = make_double4(o[4], o[5], o[6], o[7]);
        }
    }
}

// Adjoint VJP: mass-scaled form unless some mass is not positive (flag set
// by the scaling pass), then the general form on the raw cotangent.  The
// branch is uniform over the launch.
template <typename T, typename V, typename MT, int TPL>
__global__ __launch_bounds__(kBlock) void k_vjp_adj(const V *__restrict__ pm, const V *__restrict__ raw,
                                                    const V *__restrict__ sc,
                                                    const int *__restrict__ nonpos, int n, T eps2,
                                                    double G, int jtile, double scale, int accumulate,
                                                    V *__restrict__ pos_cot, MT *__restrict__ mass_cot,
                                                    V *__restrict__ acc_out,
                                                    double4 *__restrict__ partial)
{
    if (*nonpos)
        vjp_general<T, V, MT, TPL, false>(pm, raw, n, eps2, G, jtile, scale, accumulate, pos_cot,
                                          mass_cot, acc_out, partial);
    else
        vjp_scaled<T, V, MT, TPL>(pm, sc, n, eps2, G, jtile, scale, accumulate, pos_cot, mass_cot,
                                  acc_out, partial);
}

// at = abar / m for every body; any non-positive mass sets *nonpos.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_prescale(const V *__restrict__ cot,
                                                     const V *__restrict__ pm, int n,
                                                     V *__restrict__ sc, int *__restrict__ nonpos)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const V c = cot[i];
    const V p = pm[i];
    V o;
    o.x = c.x / p.w;
    o.y = c.y / p.w;
    o.z = c.z / p.w;
    o.w = 0;
    sc[i] = o;
    if (!(p.w > 0)) atomicOr(nonpos, 1);
}

// Fixed-order sum of the per-split records, then the same output step.
template <typename V, typename MT>
__global__ __launch_bounds__(kBlock) void k_vjp_reduce(const double4 *__restrict__ partial, int js,
                                                       int n, double scale, int accumulate,
                                                       V *__restrict__ pos_cot,
                                                       MT *__restrict__ mass_cot,
                                                       V *__restrict__ acc_out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < js; ++s) {
        const double4 *src = partial + 2 * ((long)s * n + i);
        const double4 a = src[0], b = src[1];
        o[0] += a.x; o[1] += a.y; o[2] += a.z; o[3] += a.w;
        o[4] += b.x; o[5] += b.y; o[6] += b.z; o[7] += b.w;
    }
    apply_out(o, scale, accumulate, i, pos_cot, mass_cot, acc_out);
}

// y += a x, and ysc = y / m with m from the records pm (next scaled cotangent)
template <typename V, typename S>
__global__ __launch_bounds__(kBlock) void k_axpy(V *__restrict__ y, const V *__restrict__ x, S a,
                                                 const V *__restrict__ pm, V *__restrict__ ysc,
                                                 int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    V v = y[i];
    const V u = x[i];
    v.x = v.x + a * u.x;
    v.y = v.y + a * u.y;
    v.z = v.z + a * u.z;
    y[i] = v;
    const S m = pm[i].w;
    V o;
    o.x = v.x / m;
    o.y = v.y / m;
    o.z = v.z / m;
    o.w = 0;
    ysc[i] = o;
}

// Split reduction fused with the elementwise step that follows every adjoint
// VJP, so that one launch finishes the step:
//   POST 1 (segment recompute):  vbar += dt xbar,  vsc = vbar / m
//   POST 3 (integer reversal):    as POST 1, and the force is written to vh
//   POST 2 (time reversal):      vh -= hk a;  x -= dt vh;  vbar += dt xbar;
//                                vsc = vbar / m
// The stored (rounded) xbar and a are the values used, as in the separate
// kernels.
template <typename V, typename MT, typename S, int POST>
__global__ __launch_bounds__(kBlock) void k_vjp_reduce_post(
    const double4 *__restrict__ partial, int js, int n, double scale, V *__restrict__ pos_cot,
    MT *__restrict__ mass_cot, V *__restrict__ x, V *__restrict__ vh, V *__restrict__ vbar,
    V *__restrict__ vsc, S hk, S dt)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < js; ++s) {
        const double4 *src = partial + 2 * ((long)s * n + i);
        const double4 a = src[0], b = src[1];
        o[0] += a.x; o[1] += a.y; o[2] += a.z; o[3] += a.w;
        o[4] += b.x; o[5] += b.y; o[6] += b.z; o[7] += b.w;
    }
    V g = pos_cot[i];
    g.x = (S)(o[0] * scale + (double)g.x);
    g.y = (S)(o[1] * scale + (double)g.y);
    g.z = (S)(o[2] * scale + (double)g.z);
    g.w = 0;
    pos_cot[i] = g;
    mass_cot[i] = (MT)(o[3] * scale + (double)mass_cot[i]);
    V p = x[i], w = vbar[i];
    if (POST == 2) {
        V v = vh[i];
        const S ax = (S)o[4], ay = (S)o[5], az = (S)o[6];
        v.x = v.x - hk * ax;
        v.y = v.y - hk * ay;
        v.z = v.z - hk * az;
        p.x = p.x - dt * v.x;
        p.y = p.y - dt * v.y;
        p.z = p.z - dt * v.z;
        vh[i] = v;
        x[i] = p;
    }
    if (POST == 3) {  // the force alone, for a reversal done elsewhere (vh receives it)
        V f;
        f.x = (S)o[4];
        f.y = (S)o[5];
        f.z = (S)o[6];
        f.w = 0;
        vh[i] = f;
    }
    w.x = w.x + dt * g.x;
    w.y = w.y + dt * g.y;
    w.z = w.z + dt * g.z;
    vbar[i] = w;
    V q;
    q.x = w.x / p.w;
    q.y = w.y / p.w;
    q.z = w.z / p.w;
    q.w = 0;
    vsc[i] = q;
}

// One reverse step of the leapfrog by exact time reversal (scheme used by
// the reversal adjoint):  given x_{s+1}, the force a_{s+1} and either the
// synchronised velocity v_{s+1} (first step of a segment) or v_{s+3/2},
//   v_{s+1/2} = v_{s+1} - h a_{s+1}   or   v_{s+3/2} - 2h a_{s+1}
//   x_s       = x_{s+1} - dt v_{s+1/2}
// and the adjoint of the drift, vbar += dt xbar.
template <typename V, typename S>
__global__ __launch_bounds__(kBlock) void k_reverse(V *__restrict__ x, V *__restrict__ vh,
                                                    const V *__restrict__ acc,
                                                    const V *__restrict__ xbar,
                                                    V *__restrict__ vbar, V *__restrict__ vsc,
                                                    int n, S hk, S dt)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    V p = x[i], v = vh[i], w = vbar[i];
    const V a = acc[i], g = xbar[i];
    v.x = v.x - hk * a.x;
    v.y = v.y - hk * a.y;
    v.z = v.z - hk * a.z;
    p.x = p.x - dt * v.x;
    p.y = p.y - dt * v.y;
    p.z = p.z - dt * v.z;
    w.x = w.x + dt * g.x;
    w.y = w.y + dt * g.y;
    w.z = w.z + dt * g.z;
    x[i] = p;
    vh[i] = v;
    vbar[i] = w;
    V o;
    o.x = w.x / p.w;
    o.y = w.y / p.w;
    o.z = w.z / p.w;
    o.w = 0;
    vsc[i] = o;
}

template <typename T, typename V, typename MT, int TPL>
hipError_t go_vjp(const void *pm, const void *cot, int n, T eps2, double G, const Tune &t, double scale,
                  int accumulate, bool phi, void *pos_cot, void *mass_cot, void *acc_out,
                  void *partial, hipStream_t s)
{
    const int per_block = (kBlock / 64) * 64 * TPL;
    const dim3 grid((n + per_block - 1) / per_block, t.jsplit);
    if (phi)
        hipLaunchKernelGGL((k_vjp<T, V, MT, TPL, true>), grid, dim3(kBlock), 0, s, (const V *)pm,
                           (const V *)cot, n, eps2, G, t.jtile, scale, accumulate, (V *)pos_cot,
                           (MT *)mass_cot, (V *)acc_out, (double4 *)partial);
    else
        hipLaunchKernelGGL((k_vjp<T, V, MT, TPL, false>), grid, dim3(kBlock), 0, s, (const V *)pm,
                           (const V *)cot, n, eps2, G, t.jtile, scale, accumulate, (V *)pos_cot,
                           (MT *)mass_cot, (V *)acc_out, (double4 *)partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || t.jsplit == 1) return e;
    hipLaunchKernelGGL((k_vjp_reduce<V, MT>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       (const double4 *)partial, t.jsplit, n, scale, accumulate, (V *)pos_cot,
                       (MT *)mass_cot, (V *)acc_out);
    return hipGetLastError();
}

}  // namespace

size_t vjp_partial_bytes(int n, const Tune &t)
{
    return t.jsplit > 1 ? 2 * sizeof(double4) * (size_t)t.jsplit * (size_t)n : 0;
}

// Internal entry with scale/accumulate, used by the trajectory adjoint.
hipError_t launch_vjp_ex(int prec, const void *pm, const void *cot, int n, double G, double eps,
                         bool phi, double scale, bool accumulate, void *pos_cot, void *mass_cot,
                         void *acc_out, const Tune &t, void *partial, hipStream_t s)
{
    if (prec == NBODY_F64) {
        if (t.tpl == 1)
            return go_vjp<double, double4, double, 1>(pm, cot, n, eps * eps, G, t, scale, accumulate,
                                                      phi, pos_cot, mass_cot, acc_out, partial, s);
        return go_vjp<double, double4, double, 2>(pm, cot, n, eps * eps, G, t, scale, accumulate, phi,
                                                  pos_cot, mass_cot, acc_out, partial, s);
    }
    const float e2 = (float)(eps * eps);
    if (t.tpl == 1)
        return go_vjp<float, float4, float, 1>(pm, cot, n, e2, G, t, scale, accumulate, phi, pos_cot,
                                               mass_cot, acc_out, partial, s);
    return go_vjp<float, float4, float, 2>(pm, cot, n, e2, G, t, scale, accumulate, phi, pos_cot,
                                           mass_cot, acc_out, partial, s);
}

hipError_t launch_vjp(int prec, const void *pm, const void *cot, int n, double G, double eps,
                      void *pos_cot, void *mass_cot, void *acc_out, const Tune &t, void *partial,
                      hipStream_t s)
{
    return launch_vjp_ex(prec, pm, cot, n, G, eps, true, 1.0, false, pos_cot, mass_cot, acc_out, t,
                         partial, s);
}

hipError_t launch_reverse_step(int prec, void *x, void *vh, const void *acc, const void *xbar,
                               void *vbar, void *vsc, int n, double hk, double dt, hipStream_t s)
{
    const dim3 grid((n + kBlock - 1) / kBlock);
    if (prec == NBODY_F64)
        hipLaunchKernelGGL((k_reverse<double4, double>), grid, dim3(kBlock), 0, s, (double4 *)x,
                           (double4 *)vh, (const double4 *)acc, (const double4 *)xbar,
                           (double4 *)vbar, (double4 *)vsc, n, hk, dt);
    else
        hipLaunchKernelGGL((k_reverse<float4, float>), grid, dim3(kBlock), 0, s, (float4 *)x,
                           (float4 *)vh, (const float4 *)acc, (const float4 *)xbar, (float4 *)vbar,
                           (float4 *)vsc, n, (float)hk, (float)dt);
    return hipGetLastError();
}

hipError_t launch_adj_axpy(int prec, void *y, const void *x, double a, const void *pm, void *ysc,
                           int n, hipStream_t s)
{
    const dim3 grid((n + kBlock - 1) / kBlock);
    if (prec == NBODY_F64)
        hipLaunchKernelGGL((k_axpy<double4, double>), grid, dim3(kBlock), 0, s, (double4 *)y,
                           (const double4 *)x, a, (const double4 *)pm, (double4 *)ysc, n);
    else
        hipLaunchKernelGGL((k_axpy<float4, float>), grid, dim3(kBlock), 0, s, (float4 *)y,
                           (const float4 *)x, (float)a, (const float4 *)pm, (float4 *)ysc, n);
    return hipGetLastError();
}

// (0, 0, 0, w) of every record: the potential cotangent alone.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_phibar_only(const V *__restrict__ src, int n, V *__restrict__ dst)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    V o;
    o.x = 0;
    o.y = 0;
    o.z = 0;
    o.w = src[i].w;
    dst[i] = o;
}

hipError_t launch_phibar_only(int prec, const void *src, int n, void *dst, hipStream_t s)
{
    const dim3 grid((n + kBlock - 1) / kBlock);
    if (prec == NBODY_F64)
        hipLaunchKernelGGL((k_phibar_only<double4>), grid, dim3(kBlock), 0, s, (const double4 *)src, n,
                           (double4 *)dst);
    else
        hipLaunchKernelGGL((k_phibar_only<float4>), grid, dim3(kBlock), 0, s, (const float4 *)src, n,
                           (float4 *)dst);
    return hipGetLastError();
}

hipError_t launch_prescale(int prec, const void *cot, const void *pm, int n, void *sc, int *nonpos,
                           hipStream_t s)
{
    const dim3 grid((n + kBlock - 1) / kBlock);
    if (prec == NBODY_F64)
        hipLaunchKernelGGL((k_prescale<double4>), grid, dim3(kBlock), 0, s, (const double4 *)cot,
                           (const double4 *)pm, n, (double4 *)sc, nonpos);
    else
        hipLaunchKernelGGL((k_prescale<float4>), grid, dim3(kBlock), 0, s, (const float4 *)cot,
                           (const float4 *)pm, n, (float4 *)sc, nonpos);
    return hipGetLastError();
}

template <typename T, typename V, typename MT, int TPL>
hipError_t go_vjp_adj(const void *pm, const void *raw, const void *sc, const int *nonpos, int n,
                      T eps2, double G, const Tune &t, double scale, void *pos_cot, void *mass_cot,
                      void *acc_out, void *partial, hipStream_t s)
{
    const int per_block = (kBlock / 64) * 64 * TPL;
    const dim3 grid((n + per_block - 1) / per_block, t.jsplit);
    hipLaunchKernelGGL((k_vjp_adj<T, V, MT, TPL>), grid, dim3(kBlock), 0, s, (const V *)pm,
                       (const V *)raw, (const V *)sc, nonpos, n, eps2, G, t.jtile, scale, 1,
                       (V *)pos_cot, (MT *)mass_cot, (V *)acc_out, (double4 *)partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || t.jsplit == 1) return e;
    hipLaunchKernelGGL((k_vjp_reduce<V, MT>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       (const double4 *)partial, t.jsplit, n, scale, 1, (V *)pos_cot,
                       (MT *)mass_cot, (V *)acc_out);
    return hipGetLastError();
}

// Adjoint VJP plus its elementwise step (post = 1: vbar update, post = 2:
// time reversal; x is the position array the VJP was evaluated at and vh
// the half-step velocity).  With a source split the step runs inside the
// reduction launch; otherwise as its own kernel after the VJP.
hipError_t launch_vjp_adj_step(int prec, int post, void *pm, void *raw, void *sc, const int *nonpos,
                               int n, double G, double eps, double scale, void *pos_cot,
                               void *mass_cot, void *acc, void *vh, double hk, double dt,
                               const Tune &t, void *partial, hipStream_t s)
{
    if (t.jsplit == 1) {
        hipError_t e = launch_vjp_adj(prec, pm, raw, sc, nonpos, n, G, eps, scale, pos_cot, mass_cot,
                                      post >= 2 ? acc : nullptr, t, partial, s);
        if (e != hipSuccess) return e;
        if (post == 2) return launch_reverse_step(prec, pm, vh, acc, pos_cot, raw, sc, n, hk, dt, s);
        return launch_adj_axpy(prec, raw, pos_cot, dt, pm, sc, n, s);
    }
    // the sweep alone: partial records only (the split path never writes
    // outputs from the sweep kernel)
    const dim3 grid((n + kBlock - 1) / kBlock, t.jsplit);
    if (prec == NBODY_F64) {
        const double e2 = eps * eps;
        hipLaunchKernelGGL((k_vjp_adj<double, double4, double, 1>), grid, dim3(kBlock), 0, s,
                           (const double4 *)pm, (const double4 *)raw, (const double4 *)sc, nonpos, n,
                           e2, G, t.jtile, scale, 1, (double4 *)pos_cot, (double *)mass_cot,
                           (double4 *)nullptr, (double4 *)partial);
    } else {
        const float e2 = (float)(eps * eps);
        hipLaunchKernelGGL((k_vjp_adj<float, float4, float, 1>), grid, dim3(kBlock), 0, s,
                           (const float4 *)pm, (const float4 *)raw, (const float4 *)sc, nonpos, n, e2,
                           G, t.jtile, scale, 1, (float4 *)pos_cot, (float *)mass_cot,
                           (float4 *)nullptr, (double4 *)partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 rg((n + kBlock - 1) / kBlock);
    if (prec == NBODY_F64) {
        if (post == 2)
            hipLaunchKernelGGL((k_vjp_reduce_post<double4, double, double, 2>), rg, dim3(kBlock), 0, s,
                               (const double4 *)partial, t.jsplit, n, scale, (double4 *)pos_cot,
                               (double *)mass_cot, (double4 *)pm, (double4 *)vh, (double4 *)raw,
                               (double4 *)sc, hk, dt);
        else if (post == 3)
            hipLaunchKernelGGL((k_vjp_reduce_post<double4, double, double, 3>), rg, dim3(kBlock), 0, s,
                               (const double4 *)partial, t.jsplit, n, scale, (double4 *)pos_cot,
                               (double *)mass_cot, (double4 *)pm, (double4 *)acc, (double4 *)raw,
                               (double4 *)sc, hk, dt);
        else
            hipLaunchKernelGGL((k_vjp_reduce_post<double4, double, double, 1>), rg, dim3(kBlock), 0, s,
                               (const double4 *)partial, t.jsplit, n, scale, (double4 *)pos_cot,
                               (double *)mass_cot, (double4 *)pm, (double4 *)vh, (double4 *)raw,
                               (double4 *)sc, hk, dt);
    } else {
        if (post == 2)
            hipLaunchKernelGGL((k_vjp_reduce_post<float4, float, float, 2>), rg, dim3(kBlock), 0, s,
                               (const double4 *)partial, t.jsplit, n, scale, (float4 *)pos_cot,
                               (float *)mass_cot, (float4 *)pm, (float4 *)vh, (float4 *)raw,
                               (float4 *)sc, (float)hk, (float)dt);
        else if (post == 3)
            hipLaunchKernelGGL((k_vjp_reduce_post<float4, float, float, 3>), rg, dim3(kBlock), 0, s,
                               (const double4 *)partial, t.jsplit, n, scale, (float4 *)pos_cot,
                               (float *)mass_cot, (float4 *)pm, (float4 *)acc, (float4 *)raw,
                               (float4 *)sc, (float)hk, (float)dt);
        else
            hipLaunchKernelGGL((k_vjp_reduce_post<float4, float, float, 1>), rg, dim3(kBlock), 0, s,
                               (const double4 *)partial, t.jsplit, n, scale, (float4 *)pos_cot,
                               (float *)mass_cot, (float4 *)pm, (float4 *)vh, (float4 *)raw,
                               (float4 *)sc, (float)hk, (float)dt);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_adj(int prec, const void *pm, const void *raw, const void *sc,
                          const int *nonpos, int n, double G, double eps, double scale,
                          void *pos_cot, void *mass_cot, void *acc_out, const Tune &t, void *partial,
                          hipStream_t s)
{
    if (prec == NBODY_F64) {
        if (t.tpl == 1)
            return go_vjp_adj<double, double4, double, 1>(pm, raw, sc, nonpos, n, eps * eps, G, t,
                                                          scale, pos_cot, mass_cot, acc_out, partial, s);
        return go_vjp_adj<double, double4, double, 2>(pm, raw, sc, nonpos, n, eps * eps, G, t, scale,
                                                      pos_cot, mass_cot, acc_out, partial, s);
    }
    const float e2 = (float)(eps * eps);
    if (t.tpl == 1)
        return go_vjp_adj<float, float4, float, 1>(pm, raw, sc, nonpos, n, e2, G, t, scale, pos_cot,
                                                   mass_cot, acc_out, partial, s);
    return go_vjp_adj<float, float4, float, 2>(pm, raw, sc, nonpos, n, e2, G, t, scale, pos_cot,
                                               mass_cot, acc_out, partial, s);
}

}  // namespace nbi
