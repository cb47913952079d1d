// Tree tables shared by the tree walks (tree.hip) and the multi-level fast
// multipole method (fmm.hip): the device view of the ORB node table and its
// per-node moments and cell records, the host plan of the node table, the
// box distance of the opening test, the quadrupole cell's evaluation at a
// target and its M2L into a third-order local expansion.
#pragma once

#include <mutex>
#include <vector>

#include "internal.h"
#include "pair.h"

namespace nbi {

constexpr int kQuadRec = 3;  // float4 records per cell (quadrupole cells)
constexpr int kCellsMono = 0, kCellsPseudo = 2, kCellsQuad = 3, kCellsLocal = 4;

struct TreeDev {
    const int4 *node;    // begin, end, left, right (-1 for a leaf)
    const int *by_height;  // node ids by height (0 = leaves, in ORB order), ascending
    const int *groups;     // group node ids in ORB order
    double4 *sums;       // M, Sx, Sy, Sz
    double4 *comd;       // com (FP64), diag2
    float4 *rec;         // com (FP32), M (FP32): the pseudo-body record
    float4 *lo, *hi;     // box
    double4 *s2a, *s2b;  // second moment about com: (xx, yy, zz, xy), (xz, yz, -, -)
    float4 *pp;          // pseudo-particle cells: kPseudo records (x, y, z, q) per node
    float4 *qr;          // quadrupole cells: (com, M), (Qxx, Qyy, Qzz, Qxy), (Qxz, Qyz, 0, 0)
    int *order;          // dispatch order of the local-expansion walk (group indices)
    unsigned short *obin;  // per group: the diag2 bin that sets the order
    int *ohist;          // per 1024 groups: a histogram of those bins
};

struct HostTree {
    std::vector<int4> node;
    std::vector<int> leaves, groups, height;
    std::vector<int> by_height;    // node ids ordered by height, leaves first in ORB order
    std::vector<int> height_off;   // start of each height in by_height, plus the end
};

// Caller holds tree_mutex(): makes the tables for (n, leaf) current, computes
// the moments with the quadrupole records of every node from the ORB-ordered
// records pm, and returns the device view and the host plan (valid until the
// next call with another shape or tree_release).
int tree_quad_prepare(const void *pm, int n, int leaf, hipStream_t s, TreeDev &d, const HostTree *&h);
std::mutex &tree_mutex();

namespace {

// Distance along one axis from p to the interval [a, b] (0 inside).
__device__ __forceinline__ double box_gap(double p, double a, double b)
{
    return p < a ? a - p : (p > b ? p - b : 0.0);
}

// One quadrupole cell against the lane's TPL targets: c = (com, M),
// q1 = (Qxx, Qyy, Qzz, Qxy), q2 = (Qxz, Qyz, -, -).  With d = com - x and
// s^2 = |d|^2 + eps^2: phi-sum += M/s + d.Q.d / (2 s^5),
// a-sum += M d / s^3 + 5 (d.Q.d) d / (2 s^7) - Q d / s^5.
template <int TPL>
__device__ __forceinline__ void quad_f32(const float4 c, const float4 q1, const float4 q2,
                                         const Targets<float, TPL> &T, float eps2, Sums<float, TPL> &S)
{
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const float dx = c.x - T.x[t];
        const float dy = c.y - T.y[t];
        const float dz = c.z - T.z[t];
        const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float ri2 = ri * ri;
        const float ri3 = ri2 * ri;
        const float ri5 = ri3 * ri2;
        const float qx = __builtin_fmaf(q1.x, dx, __builtin_fmaf(q1.w, dy, q2.x * dz));
        const float qy = __builtin_fmaf(q1.w, dx, __builtin_fmaf(q1.y, dy, q2.y * dz));
        const float qz = __builtin_fmaf(q2.x, dx, __builtin_fmaf(q2.y, dy, q1.z * dz));
        const float dqd = __builtin_fmaf(dx, qx, __builtin_fmaf(dy, qy, dz * qz));
        const float t5 = dqd * ri5;
        S.ph[t] = __builtin_fmaf(0.5f, t5, __builtin_fmaf(c.w, ri, S.ph[t]));
        const float k = __builtin_fmaf(2.5f * t5, ri2, c.w * ri3);
        S.ax[t] = __builtin_fmaf(-qx, ri5, __builtin_fmaf(k, dx, S.ax[t]));
        S.ay[t] = __builtin_fmaf(-qy, ri5, __builtin_fmaf(k, dy, S.ay[t]));
        S.az[t] = __builtin_fmaf(-qz, ri5, __builtin_fmaf(k, dz, S.az[t]));
    }
}

// Third-order local expansion about a centre z: P0, p (x, y, z),
// K (xx, yy, zz, xy, xz, yz), T (xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz,
// yzz, xyz) of the potential sum.
struct Local {
    float c[20];
};

// Folds one quadrupole cell (records (com, M), (Qxx, Qyy, Qzz, Qxy),
// (Qxz, Qyz, -, -)) into L, expanded about zg: with r = zg - com,
// s^2 = |r|^2 + eps^2 and u = r / s,
//   P0   += M/s + (u.Q.u) / (2 s^3)
//   p_k  += u_k (-M/s^2 - 5 (u.Q.u) / (2 s^4)) + (Q u)_k / s^4
//   K_kl += u_k u_l (3 M/s^3 + 35 (u.Q.u) / (2 s^5)) - 5 ((Q u)_k u_l + (Q u)_l u_k) / s^5
//           + Q_kl / s^5 - delta_kl (M/s^3 + 5 (u.Q.u) / (2 s^5))
//   T_klm += A u_k u_l u_m + B (q_k u_l u_m + q_l u_k u_m + q_m u_k u_l)
//            + C (d_kl u_m + d_km u_l + d_lm u_k)
//            + D (Q_kl u_m + Q_km u_l + Q_lm u_k + q_k d_lm + q_l d_km + q_m d_kl)
//     with q = Q u, A = -15 M/s^4 - 315 (u.Q.u) / (2 s^6), B = 35 / s^6,
//     C = 3 M/s^4 + 35 (u.Q.u) / (2 s^6), D = -5 / s^6
// (the derivatives of M/s + (r.Q.r) / (2 s^5) written with u, so that no
// power above s^-6 is formed).
__device__ __forceinline__ void m2l_f32(const float4 *__restrict__ rec, float zx, float zy, float zz, float eps2,
                                        Local &L)
{
    const float4 c = rec[0], q1 = rec[1], q2 = rec[2];
    const float rx = zx - c.x, ry = zy - c.y, rz = zz - c.z;
    const float s2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, __builtin_fmaf(rx, rx, eps2)));
    const float si = __builtin_amdgcn_rsqf(s2);
    const float ux = rx * si, uy = ry * si, uz = rz * si;
    const float si2 = si * si, si3 = si2 * si, si4 = si2 * si2, si5 = si4 * si;
    const float qx = __builtin_fmaf(q1.x, ux, __builtin_fmaf(q1.w, uy, q2.x * uz));
    const float qy = __builtin_fmaf(q1.w, ux, __builtin_fmaf(q1.y, uy, q2.y * uz));
    const float qz = __builtin_fmaf(q2.x, ux, __builtin_fmaf(q2.y, uy, q1.z * uz));
    const float uqu = __builtin_fmaf(ux, qx, __builtin_fmaf(uy, qy, uz * qz));
    const float M = c.w;
    L.c[0] += __builtin_fmaf(0.5f * uqu, si3, M * si);
    const float cp = __builtin_fmaf(-2.5f * uqu, si4, -M * si2);
    L.c[1] += __builtin_fmaf(ux, cp, qx * si4);
    L.c[2] += __builtin_fmaf(uy, cp, qy * si4);
    L.c[3] += __builtin_fmaf(uz, cp, qz * si4);
    const float A = __builtin_fmaf(17.5f * uqu, si5, 3.0f * M * si3);
    const float B = -5.0f * si5;
    const float D = __builtin_fmaf(2.5f * uqu, si5, M * si3);
    L.c[4] += __builtin_fmaf(ux * ux, A, __builtin_fmaf(2.0f * B, qx * ux, __builtin_fmaf(q1.x, si5, -D)));
    L.c[5] += __builtin_fmaf(uy * uy, A, __builtin_fmaf(2.0f * B, qy * uy, __builtin_fmaf(q1.y, si5, -D)));
    L.c[6] += __builtin_fmaf(uz * uz, A, __builtin_fmaf(2.0f * B, qz * uz, __builtin_fmaf(q1.z, si5, -D)));
    L.c[7] += __builtin_fmaf(ux * uy, A, __builtin_fmaf(B, __builtin_fmaf(qx, uy, qy * ux), q1.w * si5));
    L.c[8] += __builtin_fmaf(ux * uz, A, __builtin_fmaf(B, __builtin_fmaf(qx, uz, qz * ux), q2.x * si5));
    L.c[9] += __builtin_fmaf(uy * uz, A, __builtin_fmaf(B, __builtin_fmaf(qy, uz, qz * uy), q2.y * si5));
    const float si6 = si4 * si2;
    const float a3 = __builtin_fmaf(-157.5f * uqu, si6, -15.0f * M * si4);
    const float b3 = 35.0f * si6;
    const float c3 = __builtin_fmaf(17.5f * uqu, si6, 3.0f * M * si4);
    const float d3 = -5.0f * si6;
    // T_kkk = a3 u_k^3 + 3 b3 q_k u_k^2 + 3 c3 u_k + 3 d3 (Q_kk u_k + q_k)
    L.c[10] += __builtin_fmaf(a3 * ux, ux * ux, 3.0f * __builtin_fmaf(b3 * qx, ux * ux, __builtin_fmaf(c3, ux, d3 * __builtin_fmaf(q1.x, ux, qx))));
    L.c[11] += __builtin_fmaf(a3 * uy, uy * uy, 3.0f * __builtin_fmaf(b3 * qy, uy * uy, __builtin_fmaf(c3, uy, d3 * __builtin_fmaf(q1.y, uy, qy))));
    L.c[12] += __builtin_fmaf(a3 * uz, uz * uz, 3.0f * __builtin_fmaf(b3 * qz, uz * uz, __builtin_fmaf(c3, uz, d3 * __builtin_fmaf(q1.z, uz, qz))));
    // T_kkm = a3 u_k^2 u_m + b3 (2 q_k u_k u_m + q_m u_k^2) + c3 u_m + d3 (Q_kk u_m + 2 Q_km u_k + q_m)
    auto tkkm = [&](float uk, float um, float qk, float qm, float Qkk, float Qkm) {
        const float uk2 = uk * uk;
        return __builtin_fmaf(a3 * uk2, um,
                              __builtin_fmaf(b3, __builtin_fmaf(2.0f * qk * uk, um, qm * uk2),
                                             __builtin_fmaf(c3, um, d3 * __builtin_fmaf(Qkk, um, __builtin_fmaf(2.0f * Qkm, uk, qm)))));
    };
    L.c[13] += tkkm(ux, uy, qx, qy, q1.x, q1.w);  // xxy
    L.c[14] += tkkm(ux, uz, qx, qz, q1.x, q2.x);  // xxz
    L.c[15] += tkkm(uy, ux, qy, qx, q1.y, q1.w);  // xyy
    L.c[16] += tkkm(uy, uz, qy, qz, q1.y, q2.y);  // yyz
    L.c[17] += tkkm(uz, ux, qz, qx, q1.z, q2.x);  // xzz
    L.c[18] += tkkm(uz, uy, qz, qy, q1.z, q2.y);  // yzz
    // T_xyz = a3 ux uy uz + b3 (qx uy uz + qy ux uz + qz ux uy) + d3 (Qxy uz + Qxz uy + Qyz ux)
    L.c[19] += __builtin_fmaf(a3 * ux, uy * uz,
                              __builtin_fmaf(b3, __builtin_fmaf(qx, uy * uz, __builtin_fmaf(qy, ux * uz, qz * ux * uy)),
                                             d3 * __builtin_fmaf(q1.w, uz, __builtin_fmaf(q2.x, uy, q2.y * ux))));
}

}  // namespace
}  // namespace nbi
