// Tree-code force on the ORB cells (gfx950).
//
// The paper's force calculation (Section IV.A): a distant group of bodies acts
// as one body of the group's total mass at its centre of mass; the cells that
// are distant enough are found by walking the tree from the root, and the
// force sums over the accepted cells and the remaining nearby bodies.  The
// cells here are the nodes of the ORB recursion of Section IV.B, so they need
// no separate tree build: with the bodies in ORB order (same leaf size) node k
// is the contiguous range [begin, end), and the node table depends only on
// (n, leaf).
//
// Definitions shared with the FP64 oracle (bit-exact decisions):
// * moments in FP64: a leaf sums m and m*x over its bodies in order (product
//   rounded, then added); an inner node adds left + right.  com = S / M, or the
//   box centre when M = 0.  Boxes are exact FP32 minima/maxima, and
//   diag2 = sum over x, y, z of (hi - lo)^2 in FP64.
// * groups: the targets are taken in groups, the maximal nodes of at most 64
//   bodies (one wave each).
// * opening: cell c is accepted for group g iff c and g share no body and
//   diag2_c < theta^2 * D2, D2 the squared distance from com_c to the box of g
//   (per axis lo - com, com - hi or 0; summed x, y, z).  Every body of c lies
//   within sqrt(diag2_c) of com_c and every body of g at least sqrt(D2) from
//   it, so the size-to-distance ratio is below theta for every target.
//
// Kernels:
// * k_tree_leaves, then k_tree_inner once per node height (children are
//   always lower than their parent): one thread per node, left + right.  The
//   kernel boundaries order the levels, so no fences or counters are needed.
// * k_tree_walk: one wave per group.  The walk starts from the siblings of
//   the group's ancestors (every cell disjoint from the group) and pops up to
//   64 cells per step from a 512-entry stack in LDS, one cell per lane: the acceptance
//   test is per cell, so the control flow of the wave stays uniform.
//   Accepted cells go to an LDS batch of pseudo-body records that every lane
//   sweeps with the same FP32 pair code as the direct sum (broadcast LDS
//   reads); rejected leaves go to a batch of contiguous source ranges swept
//   with scalar loads; the group's own bodies are one masked range.  A cell
//   whose children would overflow the stack is summed body by body instead,
//   which is exact.  In inspection mode the same walk writes the node ids of
//   the accepted cells and of the rejected leaves instead of summing.
// * k_order_bins, k_group_order: the order in which the local-expansion walk
//   takes its groups when there are many (largest boxes first; see there).
//
// Order 2 (pseudo-particle multipoles: Makino, J. Comput. Phys. 151, 1999,
// the paper's reference [20], which Section VI cites for the O(N) fast
// multipole method): an
// accepted cell acts as 12 point masses q_j at com + a s_j, s_j the unit
// vertices of the icosahedron, a = half the box diagonal, whose expansion
// about com equals the cell's through the quadrupole term.  With S the
// cell's second moment about com (FP64, bottom-up by the parallel-axis rule:
// a leaf sums m r r^T over its bodies, a parent adds each child's S plus
// m_c d_c d_c^T, d_c = com_c - com), the method's mass formula reduces to
//   q_j = M / 12 + 5 / (24 a^2) (3 s_j.S.s_j - trace S)
// (the dipole term vanishes about com); a = 0 leaves q_j = M / 12.  The walk
// and its acceptance test are unchanged; accepted cell ids are batched in
// LDS and each cell's 12 records are read with scalar loads.
//
// Quadrupole cells: the same expansion through l = 2 evaluated directly from
// the traceless tensor Q = 3 S - trace(S) I, at offset d = com - x and
// softened distance s^2 = |d|^2 + eps^2:
//   potential sum  M / s + d.Q.d / (2 s^5)
//   acceleration   d (M / s^3 + 5 d.Q.d / (2 s^7)) - Q d / s^5
// about 35 VALU per cell and target instead of 12 pair evaluations.  The
// accepted cells' 3 records are staged in LDS and swept after every walk
// step, so the cell values reach the arithmetic as vector operands (read
// from scalar registers they issue at about two thirds of the rate).
//
// Group local expansions (the fast multipole method's M2L and L2P steps at
// the level of the target groups): a cell with diag2_c + diag2_g <
// theta^2 |com_c - z_g|^2 (z_g the group's centre of mass) enters one
// third-order Taylor expansion of its quadrupole potential about z_g (one
// order above the cells', so that the force keeps a third-order error)
// instead of being evaluated at every target.  One lane folds one cell in
// (about 110 VALU, lanes over cells); the twenty coefficients are summed
// over the wave at the end and every lane evaluates the expansion at its
// body.
// The remaining cells go through the quadrupole path or are opened, with
// the same tests as above; every decision is the FP64 expression of the
// definitions, so the lists equal the FP64 definition's.
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"
#include "pair.h"
#include "tree_shared.h"

namespace nbi {
namespace {

constexpr int kGroup = 64;     // targets per group: one per lane
constexpr int kStack = 512;    // LDS stack entries per wave
constexpr int kBuf = 128;      // LDS batch entries (cells, near ranges)
constexpr int kPseudo = 12;    // pseudo-particles per cell (pseudo-particle cells)


__device__ __forceinline__ void finish_node(const TreeDev &T, int c, double M, double sx, double sy,
                                            double sz, float4 lo, float4 hi, double &cx, double &cy,
                                            double &cz)
{
    if (M > 0.0) {
        cx = sx / M;
        cy = sy / M;
        cz = sz / M;
    } else {
        cx = 0.5 * ((double)lo.x + (double)hi.x);
        cy = 0.5 * ((double)lo.y + (double)hi.y);
        cz = 0.5 * ((double)lo.z + (double)hi.z);
    }
    const double ex = (double)hi.x - (double)lo.x;
    const double ey = (double)hi.y - (double)lo.y;
    const double ez = (double)hi.z - (double)lo.z;
    double d2 = 0.0;
    d2 = d2 + ex * ex;
    d2 = d2 + ey * ey;
    d2 = d2 + ez * ez;
    T.sums[c] = make_double4(M, sx, sy, sz);
    T.comd[c] = make_double4(cx, cy, cz, d2);
    T.rec[c] = make_float4((float)cx, (float)cy, (float)cz, (float)M);
    T.lo[c] = lo;
    T.hi[c] = hi;
}

// Leaves: one thread per leaf sums its bodies in position order (Q2: then
// the second moment about the centre of mass).
template <bool Q2>
__global__ __launch_bounds__(256) void k_tree_leaves(const float4 *__restrict__ pm, TreeDev T, int nleaves)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nleaves) return;
    const int c = T.by_height[t];
    const int4 nd = T.node[c];
    const float4 p0 = pm[nd.x];
    float4 lo = make_float4(p0.x, p0.y, p0.z, 0.0f), hi = lo;
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    for (int p = nd.x; p < nd.y; ++p) {
        const float4 b = pm[p];
        const double m = b.w;
        M = M + m;
        const double mx = m * (double)b.x, my = m * (double)b.y, mz = m * (double)b.z;
        sx = sx + mx;
        sy = sy + my;
        sz = sz + mz;
        if (b.x < lo.x) lo.x = b.x;
        if (b.x > hi.x) hi.x = b.x;
        if (b.y < lo.y) lo.y = b.y;
        if (b.y > hi.y) hi.y = b.y;
        if (b.z < lo.z) lo.z = b.z;
        if (b.z > hi.z) hi.z = b.z;
    }
    double cx, cy, cz;
    finish_node(T, c, M, sx, sy, sz, lo, hi, cx, cy, cz);
    if constexpr (Q2) {
        double xx = 0.0, yy = 0.0, zz = 0.0, xy = 0.0, xz = 0.0, yz = 0.0;
        for (int p = nd.x; p < nd.y; ++p) {
            const float4 b = pm[p];
            const double m = b.w;
            const double dx = (double)b.x - cx, dy = (double)b.y - cy, dz = (double)b.z - cz;
            const double mx = m * dx, my = m * dy, mz = m * dz;
            xx = xx + mx * dx;
            yy = yy + my * dy;
            zz = zz + mz * dz;
            xy = xy + mx * dy;
            xz = xz + mx * dz;
            yz = yz + my * dz;
        }
        T.s2a[c] = make_double4(xx, yy, zz, xy);
        T.s2b[c] = make_double4(xz, yz, 0.0, 0.0);
    }
}

// Inner nodes of one height (their children are all lower, so finished by
// the previous launches): left + right (Q2: second moments moved to the
// parent's centre of mass).
template <bool Q2>
__global__ __launch_bounds__(256) void k_tree_inner(TreeDev T, int first, int count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int c = T.by_height[first + t];
    const int4 nd = T.node[c];
    const double4 a = T.sums[nd.z], b = T.sums[nd.w];
    const float4 la = T.lo[nd.z], lb = T.lo[nd.w], ha = T.hi[nd.z], hb = T.hi[nd.w];
    const float4 lo = make_float4(la.x < lb.x ? la.x : lb.x, la.y < lb.y ? la.y : lb.y,
                                  la.z < lb.z ? la.z : lb.z, 0.0f);
    const float4 hi = make_float4(ha.x > hb.x ? ha.x : hb.x, ha.y > hb.y ? ha.y : hb.y,
                                  ha.z > hb.z ? ha.z : hb.z, 0.0f);
    double cx, cy, cz;
    finish_node(T, c, a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w, lo, hi, cx, cy, cz);
    if constexpr (Q2) {
        const double4 ca = T.comd[nd.z], cb = T.comd[nd.w];
        const double4 pa = T.s2a[nd.z], pb = T.s2a[nd.w], qa = T.s2b[nd.z], qb = T.s2b[nd.w];
        const double ax = ca.x - cx, ay = ca.y - cy, az = ca.z - cz;
        const double bx = cb.x - cx, by = cb.y - cy, bz = cb.z - cz;
        const double ma = a.x, mb = b.x;
        const double xx = (pa.x + ma * ax * ax) + (pb.x + mb * bx * bx);
        const double yy = (pa.y + ma * ay * ay) + (pb.y + mb * by * by);
        const double zz = (pa.z + ma * az * az) + (pb.z + mb * bz * bz);
        const double xy = (pa.w + ma * ax * ay) + (pb.w + mb * bx * by);
        const double xz = (qa.x + ma * ax * az) + (qb.x + mb * bx * bz);
        const double yz = (qa.y + ma * ay * az) + (qb.y + mb * by * bz);
        T.s2a[c] = make_double4(xx, yy, zz, xy);
        T.s2b[c] = make_double4(xz, yz, 0.0, 0.0);
    }
}

// Order-2 pseudo-particles, one thread per (node, direction).  Direction j:
// family j / 4 = (0, u, v g), (u, v g, 0), (u g, 0, v), divided by
// sqrt(1 + g^2), g the golden ratio, with (u, v) = (+,+), (+,-), (-,+), (-,-)
// for j % 4 = 0..3.
__global__ __launch_bounds__(256) void k_tree_pseudo(TreeDev T, int nn)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * kPseudo) return;
    const int c = t / kPseudo, j = t - c * kPseudo;
    const double g = 0.5 * (1.0 + sqrt(5.0));
    const double inv = 1.0 / sqrt(1.0 + g * g);
    const double u = (j & 2) ? -1.0 : 1.0, v = (j & 1) ? -1.0 : 1.0;
    double s0, s1, s2;
    if (j < 4) {
        s0 = 0.0;
        s1 = u * inv;
        s2 = v * g * inv;
    } else if (j < 8) {
        s0 = u * inv;
        s1 = v * g * inv;
        s2 = 0.0;
    } else {
        s0 = u * g * inv;
        s1 = 0.0;
        s2 = v * inv;
    }
    const double4 cd = T.comd[c];
    const double M = T.sums[c].x;
    const double a = 0.5 * sqrt(cd.w);
    double q = M / kPseudo;
    if (a > 0.0) {
        const double4 A = T.s2a[c], B = T.s2b[c];
        const double sSs = (s0 * s0 * A.x + s1 * s1 * A.y + s2 * s2 * A.z) +
                           2.0 * (s0 * s1 * A.w + s0 * s2 * B.x + s1 * s2 * B.y);
        const double tr = (A.x + A.y) + A.z;
        q = q + 5.0 / (2.0 * kPseudo * a * a) * (3.0 * sSs - tr);
    }
    T.pp[t] = make_float4((float)(cd.x + a * s0), (float)(cd.y + a * s1), (float)(cd.z + a * s2), (float)q);
}

// Quadrupole records, one thread per node: Q = 3 S - trace(S) I in FP64,
// rounded to FP32.
__global__ __launch_bounds__(256) void k_tree_quad(TreeDev T, int nn)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nn) return;
    const double4 A = T.s2a[c], B = T.s2b[c];
    const double tr = (A.x + A.y) + A.z;
    float4 *o = T.qr + (long)kQuadRec * c;
    o[0] = T.rec[c];
    o[1] = make_float4((float)(3.0 * A.x - tr), (float)(3.0 * A.y - tr), (float)(3.0 * A.z - tr),
                       (float)(3.0 * A.w));
    o[2] = make_float4((float)(3.0 * B.x), (float)(3.0 * B.y), 0.0f, 0.0f);
}

__device__ __forceinline__ unsigned lane_rank(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

struct WalkOut {
    float4 *acc_pot;   // force mode: ORB-ordered output records
    int *far_cnt, *near_cnt, *far_ids, *near_ids;  // inspection mode
    int *loc_cnt;      // inspection of the local-expansion walk
    int max_far, max_near;
};

// Sweeps the batched pseudo-body records in LDS (broadcast reads).
__device__ __forceinline__ void sweep_cells(const float4 *cb, int cnt, const Targets<float, 1> &T,
                                            float eps2, Sums<float, 1> &S)
{
    int j = 0;
    for (; j + kUnroll <= cnt; j += kUnroll) {
        float4 b[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) b[u] = cb[j + u];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) pair_f32<1, false>(b[u], j + u, T, eps2, S);
    }
    for (; j < cnt; ++j) pair_f32<1, false>(cb[j], j, T, eps2, S);
}

// Sweeps the pseudo-particles of the batched cell ids (scalar loads of each
// cell's 12 contiguous records).
__device__ __forceinline__ void sweep_pseudo(const float4 *__restrict__ pp, const int *ids, int cnt,
                                             const Targets<float, 1> &T, float eps2, Sums<float, 1> &S)
{
    for (int r = 0; r < cnt; ++r) {
        const int c = __builtin_amdgcn_readfirstlane(ids[r]);
        const float4 *q = pp + (long)kPseudo * c;
        float4 b[kPseudo];
#pragma unroll
        for (int u = 0; u < kPseudo; ++u) b[u] = q[u];
#pragma unroll
        for (int u = 0; u < kPseudo; ++u) pair_f32<1, false>(b[u], u, T, eps2, S);
    }
}

// Sweeps the quadrupole records batched in LDS (broadcast reads into vector
// registers: the cell values then enter the arithmetic as vector operands).
__device__ __forceinline__ void sweep_quad(const float4 *qb, int cnt, const Targets<float, 1> &T, float eps2,
                                           Sums<float, 1> &S)
{
    for (int r = 0; r < cnt; ++r) {
        const float4 a = qb[kQuadRec * r], b = qb[kQuadRec * r + 1], d = qb[kQuadRec * r + 2];
        quad_f32(a, b, d, T, eps2, S);
    }
}

template <int MODE, bool INSPECT, int CELLS>
// 7 waves per SIMD: 5 KB of LDS per wave and at most 72 VGPRs (measured
// faster than 6 waves, and than 8 waves with register spills).  The local-
// expansion walk keeps 20 expansion coefficients per lane and cannot reach 7;
// asked for 5 it fits in 94 VGPRs without spills (left to itself the
// allocator took 111, 4 waves).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(CELLS == kCellsLocal ? 5 : 7))) void k_tree_walk(const float4 *__restrict__ src, int n, TreeDev T,
                                                  const float4 *__restrict__ cells, float eps2_in, double G,
                                                  double theta2, WalkOut O, const int *__restrict__ order)
{
    __shared__ int stk[kStack];
    __shared__ float4 cbuf[CELLS == kCellsMono ? kBuf : 1];    // monopole cells: the accepted records
    __shared__ int cid[CELLS == kCellsPseudo ? kBuf : 1];      // pseudo-particle cells: the accepted ids
    // quadrupole cells: the records of one step's accepted cells (swept every step)
    __shared__ float4 qbuf[CELLS >= kCellsQuad ? kQuadRec * kGroup : 1];
    // local expansions: the ids of cells waiting to be folded in
    __shared__ int lid[CELLS == kCellsLocal ? kBuf : 1];
    __shared__ int2 nbuf[kBuf];
    const int lane = threadIdx.x;
    const int g = order ? order[blockIdx.x] : (int)blockIdx.x;
    const int gnode = T.groups[g];
    const int4 gn = T.node[gnode];
    const float4 glo = T.lo[gnode], ghi = T.hi[gnode];
    const double ax = glo.x, ay = glo.y, az = glo.z, bx = ghi.x, by = ghi.y, bz = ghi.z;
    const float eps2 = lane_copy(eps2_in);
    const double4 gcd = T.comd[gnode];  // the group's centre of mass and diag2
    const float zgx = (float)gcd.x, zgy = (float)gcd.y, zgz = (float)gcd.z;
    Local Lx;
#pragma unroll
    for (int k = 0; k < 20; ++k) Lx.c[k] = 0.0f;

    Targets<float, 1> TT;
    const int i = gn.x + lane;
    {
        const float4 p = src[min(i, gn.y - 1)];
        TT.x[0] = p.x;
        TT.y[0] = p.y;
        TT.z[0] = p.z;
        TT.i[0] = i;
    }
    Run<MODE> R[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) R[c].zero();
    Sums<float, 1> S;

    // siblings of the ancestors, root first (the deepest ends on top)
    int top = 0;
    for (int c = 0, depth = 0; c != gnode && c >= 0 && depth < 64; ++depth) {
        const int4 nd = T.node[c];
        const int4 ln = T.node[nd.z];
        const bool left = gn.x < ln.y;
        if (lane == 0) stk[top] = left ? nd.w : nd.z;
        ++top;
        c = left ? nd.z : nd.w;
    }
    int nf = 0, nr = 0, tf = 0, tn = 0, nl = 0, tl = 0;

    auto flush_cells = [&]() {
        if constexpr (!INSPECT) {
            S.zero();
            if constexpr (CELLS == kCellsPseudo) {
                sweep_pseudo(cells, cid, nf, TT, eps2, S);
            } else if constexpr (CELLS >= kCellsQuad) {
                sweep_quad(qbuf, nf, TT, eps2, S);
            } else {
                static_assert(CELLS == kCellsMono, "unhandled cell model");
                sweep_cells(cbuf, nf, TT, eps2, S);
            }
            R[0].fold(S.ax[0]);
            R[1].fold(S.ay[0]);
            R[2].fold(S.az[0]);
            R[3].fold(S.ph[0]);
        }
        nf = 0;
    };
    auto flush_near = [&]() {
        if constexpr (!INSPECT) {
            S.zero();
            for (int r = 0; r < nr;) {
                const int2 a = nbuf[r];
                int b = __builtin_amdgcn_readfirstlane(a.x);
                int e = __builtin_amdgcn_readfirstlane(a.y);
                ++r;
                while (r < nr) {  // merge ranges that continue each other
                    const int2 c2 = nbuf[r];
                    const int nb = __builtin_amdgcn_readfirstlane(c2.x);
                    if (nb != e) break;
                    e = __builtin_amdgcn_readfirstlane(c2.y);
                    ++r;
                }
                sweep_f32<1, false>(src, b, e, TT, eps2, S);
            }
            R[0].fold(S.ax[0]);
            R[1].fold(S.ay[0]);
            R[2].fold(S.az[0]);
            R[3].fold(S.ph[0]);
        }
        nr = 0;
    };
    auto flush_local = [&]() {
        if constexpr (CELLS == kCellsLocal && !INSPECT) {
            for (int b = 0; b < nl; b += kGroup)
                if (b + lane < nl) m2l_f32(cells + (long)kQuadRec * lid[b + lane], zgx, zgy, zgz, eps2, Lx);
        }
        nl = 0;
    };

    while (top > 0) {
        const int k = min(kGroup, top);
        top -= k;
        __syncthreads();
        const bool act = lane < k;
        const int c = act ? stk[top + lane] : 0;
        __syncthreads();
        bool acc = false, nearr = false, open = false, loc = false;
        int4 nd = make_int4(0, 0, -1, -1);
        if (act) {
            nd = T.node[c];
            const double4 cd = T.comd[c];
            if constexpr (CELLS == kCellsLocal) {
                const double ex = cd.x - gcd.x, ey = cd.y - gcd.y, ez = cd.z - gcd.z;
                const double dz2 = (ex * ex + ey * ey) + ez * ez;
                loc = cd.w + gcd.w < theta2 * dz2;
            }
            if (!loc) {
                const double dx = box_gap(cd.x, ax, bx);
                const double dy = box_gap(cd.y, ay, by);
                const double dz = box_gap(cd.z, az, bz);
                const double D2 = (dx * dx + dy * dy) + dz * dz;
                acc = cd.w < theta2 * D2;
                if (!acc) {
                    if (nd.z < 0)
                        nearr = true;
                    else
                        open = true;
                }
            }
        }
        // children that would not fit on the stack are summed body by body
        const unsigned long long mo0 = __ballot(open);
        if (open && top + 2 * (int)(lane_rank(mo0) + 1) > kStack) {
            open = false;
            nearr = true;
        }
        const unsigned long long ma = __ballot(acc), mn = __ballot(nearr), mo = __ballot(open);
        const int ca = __popcll(ma), cn = __popcll(mn), co = __popcll(mo);
        const unsigned long long ml = CELLS == kCellsLocal ? __ballot(loc) : 0ull;
        const int cl = __popcll(ml);
        if constexpr (INSPECT) {
            if (acc) {
                const int q = tf + (int)lane_rank(ma);
                if (q < O.max_far) O.far_ids[(long)g * O.max_far + q] = c;
            }
            if (nearr) {
                const int q = tn + (int)lane_rank(mn);
                if (q < O.max_near) O.near_ids[(long)g * O.max_near + q] = c;
            }
        } else {
            if (acc) {
                if constexpr (CELLS >= kCellsQuad) {
                    const int slot = nf + (int)lane_rank(ma);
                    const float4 *r = cells + (long)kQuadRec * c;
                    qbuf[kQuadRec * slot] = r[0];
                    qbuf[kQuadRec * slot + 1] = r[1];
                    qbuf[kQuadRec * slot + 2] = r[2];
                } else if constexpr (CELLS == kCellsPseudo) {
                    cid[nf + (int)lane_rank(ma)] = c;
                } else {
                    static_assert(CELLS == kCellsMono, "unhandled cell model");
                    cbuf[nf + (int)lane_rank(ma)] = T.rec[c];
                }
            }
            if (nearr) nbuf[nr + (int)lane_rank(mn)] = make_int2(nd.x, nd.y);
            if constexpr (CELLS == kCellsLocal) {
                if (loc) lid[nl + (int)lane_rank(ml)] = c;
            }
        }
        if (open) {
            const int q = top + 2 * (int)lane_rank(mo);
            stk[q] = nd.w;
            stk[q + 1] = nd.z;
        }
        tf += ca;
        tn += cn;
        tl += cl;
        nf += ca;
        nr += cn;
        nl += cl;
        top += 2 * co;
        __syncthreads();
        if (CELLS >= kCellsQuad ? nf > 0 : nf >= kGroup) flush_cells();
        if (nr >= kGroup) flush_near();
        if (nl >= kGroup) flush_local();
    }
    if (nf > 0) flush_cells();
    if (nl > 0) flush_local();
    if (nr > 0) flush_near();

    if constexpr (INSPECT) {
        if (lane == 0) {
            O.far_cnt[g] = tf;
            O.near_cnt[g] = tn;
            if (CELLS == kCellsLocal && O.loc_cnt) O.loc_cnt[g] = tl;
        }
    } else {
        // the group's own bodies, without the self pair
        S.zero();
        range_f32<1>(src, gn.x, gn.y, gn.x, gn.x + kGroup, TT, eps2, S);
        if constexpr (CELLS == kCellsLocal) {
            // sum the local expansion over the wave, evaluate it at this body
#pragma unroll
            for (int k = 0; k < 20; ++k) {
                float v = Lx.c[k];
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
                Lx.c[k] = v;
            }
            const float yx = TT.x[0] - zgx, yy = TT.y[0] - zgy, yz = TT.z[0] - zgz;
            const float *c = Lx.c;
            const float kx = __builtin_fmaf(c[4], yx, __builtin_fmaf(c[7], yy, c[8] * yz));
            const float ky = __builtin_fmaf(c[7], yx, __builtin_fmaf(c[5], yy, c[9] * yz));
            const float kz = __builtin_fmaf(c[8], yx, __builtin_fmaf(c[9], yy, c[6] * yz));
            // T(y, y): T (xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz) = c[10..19]
            const float xx = yx * yx, yy2 = yy * yy, zz = yz * yz, xy = yx * yy, xz = yx * yz, yz2 = yy * yz;
            const float tx = __builtin_fmaf(c[10], xx, __builtin_fmaf(c[15], yy2, __builtin_fmaf(c[17], zz,
                             2.0f * __builtin_fmaf(c[13], xy, __builtin_fmaf(c[14], xz, c[19] * yz2)))));
            const float ty = __builtin_fmaf(c[13], xx, __builtin_fmaf(c[11], yy2, __builtin_fmaf(c[18], zz,
                             2.0f * __builtin_fmaf(c[15], xy, __builtin_fmaf(c[19], xz, c[16] * yz2)))));
            const float tz = __builtin_fmaf(c[14], xx, __builtin_fmaf(c[16], yy2, __builtin_fmaf(c[12], zz,
                             2.0f * __builtin_fmaf(c[19], xy, __builtin_fmaf(c[17], xz, c[18] * yz2)))));
            S.ax[0] += c[1] + __builtin_fmaf(0.5f, tx, kx);
            S.ay[0] += c[2] + __builtin_fmaf(0.5f, ty, ky);
            S.az[0] += c[3] + __builtin_fmaf(0.5f, tz, kz);
            const float py = __builtin_fmaf(c[1], yx, __builtin_fmaf(c[2], yy, c[3] * yz));
            const float yky = __builtin_fmaf(yx, kx, __builtin_fmaf(yy, ky, yz * kz));
            const float ytyy = __builtin_fmaf(yx, tx, __builtin_fmaf(yy, ty, yz * tz));
            S.ph[0] += c[0] + __builtin_fmaf(1.0f / 6.0f, ytyy, __builtin_fmaf(0.5f, yky, py));
        }
        R[0].fold(S.ax[0]);
        R[1].fold(S.ay[0]);
        R[2].fold(S.az[0]);
        R[3].fold(S.ph[0]);
        if (i < gn.y) {
            double r[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) r[c] = R[c].get();
            if constexpr (MODE == M_F32)
                put_f32(O.acc_pot, i, r, (float)G);
            else
                put(O.acc_pot, i, r, G);
        }
    }
}

// Dispatch order of the local-expansion walk.  A group whose box is large
// (a few far-flung bodies, as in the halo of a Plummer sphere) finds few
// cells far enough for its expansion, evaluates the rest per target, and
// its walk costs several times the mean (at 2^20 on the colliding pair, up
// to 3.3 times).  Taken in ORB order, such groups start late and leave most
// of the chip idle behind them; started first, they overlap with the rest
// (measured 7-10% faster at theta 0.5-1.0).  The monopole and quadrupole
// walks, whose costs vary less, measured no gain and keep ORB order, which
// L2 locality favours.  k_order_bins puts each group's diag2 in one of 1024
// bins by its FP32 bit pattern (exponent and two mantissa bits);
// k_group_order, one workgroup, takes the bins from the top down until they
// hold 1/16 of the groups and writes a stable partition of the group
// indices: those groups, then the others, each in ORB order.  Only the order
// in which the workgroups run changes, never what a group computes.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBins = 1024;
constexpr int kOrderMinGroups = 8192;  // fewer groups run in about one round

// One thread per group; each workgroup also writes the histogram of its
// kOrderThreads groups' bins (a row of kOrderBins counts).
__global__ __launch_bounds__(kOrderThreads) void k_order_bins(TreeDev T, int ng)
{
    static_assert(kOrderBins == kOrderThreads, "one bin per thread");
    __shared__ int lh[kOrderBins];
    const int t = threadIdx.x;
    lh[t] = 0;
    __syncthreads();
    const int g = blockIdx.x * kOrderThreads + t;
    if (g < ng) {
        const unsigned b = min(__float_as_uint((float)T.comd[T.groups[g]].w) >> 21, (unsigned)(kOrderBins - 1));
        T.obin[g] = (unsigned short)b;
        atomicAdd(&lh[b], 1);
    }
    __syncthreads();
    T.ohist[(long)blockIdx.x * kOrderBins + t] = lh[t];
}

// Inclusive sum over the workgroup's threads (within each wave by shuffles,
// then over the waves' totals in LDS), and the workgroup's total if asked
// for; every thread must call it.
__device__ __forceinline__ int block_incl_sum(int *sc, int v, int *total = nullptr)
{
    constexpr int kWaves = kOrderThreads / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    if (lane == 63) sc[w] = v;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        const int s = sc[k];
        before += k < w ? s : 0;
        all += s;
    }
    __syncthreads();
    if (total) *total = all;
    return before + v;
}

// Chunks of kOrderChunk groups: loaded coalesced (kOrderPer per thread,
// strided), then read from LDS as one contiguous run per thread.
constexpr int kOrderPer = 16;
constexpr int kOrderChunk = kOrderPer * kOrderThreads;

__global__ __launch_bounds__(kOrderThreads) void k_group_order(TreeDev T, int ng)
{
    static_assert(kOrderBins == kOrderThreads, "one bin per thread");
    __shared__ int hist[kOrderBins];
    __shared__ int sc[kOrderThreads / 64];
    __shared__ unsigned short cb[kOrderChunk];
    __shared__ int cut, ftot;
    const unsigned short *__restrict__ bin = T.obin;
    const int t = threadIdx.x;
    {
        // bin t summed over k_order_bins' workgroup rows
        const int rows = (ng + kOrderThreads - 1) / kOrderThreads;
        int s = 0;
#pragma unroll 16
        for (int r = 0; r < rows; ++r) s += T.ohist[(long)r * kOrderBins + t];
        hist[t] = s;
    }
    if (t == 0) cut = 0;
    __syncthreads();
    // groups in bins >= kOrderBins - 1 - t, counted from the top bin down
    const int want = max(1, ng / 16);
    const int h = hist[kOrderBins - 1 - t];
    const int top = block_incl_sum(sc, h);
    if (top >= want && top - h < want) {
        cut = kOrderBins - 1 - t;
        ftot = top;
    }
    __syncthreads();
    const int c = cut, F = ftot;
    int done = 0;  // taken groups in the chunks before this one
    for (int c0 = 0; c0 < ng; c0 += kOrderChunk) {
#pragma unroll
        for (int k = 0; k < kOrderPer; ++k) {
            const int g = c0 + k * kOrderThreads + t;
            cb[k * kOrderThreads + t] = g < ng ? bin[g] : 0;
        }
        __syncthreads();
        const int r0 = t * kOrderPer;  // this thread's run in the chunk
        int first = 0;
#pragma unroll
        for (int k = 0; k < kOrderPer; ++k) first += c0 + r0 + k < ng && cb[r0 + k] >= c;
        int chunk_taken;
        const int incl = block_incl_sum(sc, first, &chunk_taken);
        int a = done + incl - first;
        int b = F + (c0 + r0) - a;  // the others before this run come after all taken groups
        for (int k = 0; k < kOrderPer; ++k) {
            const int g = c0 + r0 + k;
            if (g >= ng) break;
            if (cb[r0 + k] >= c)
                T.order[a++] = g;
            else
                T.order[b++] = g;
        }
        done += chunk_taken;
        __syncthreads();  // cb is reused by the next chunk
    }
}

__global__ void k_tree_export(TreeDev T, int nn, double *__restrict__ mom, float *__restrict__ box)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nn) return;
    const double4 s = T.sums[c], d = T.comd[c];
    const float4 lo = T.lo[c], hi = T.hi[c];
    if (mom) {
        mom[5L * c + 0] = s.x;
        mom[5L * c + 1] = d.x;
        mom[5L * c + 2] = d.y;
        mom[5L * c + 3] = d.z;
        mom[5L * c + 4] = d.w;
    }
    if (box) {
        box[6L * c + 0] = lo.x;
        box[6L * c + 1] = lo.y;
        box[6L * c + 2] = lo.z;
        box[6L * c + 3] = hi.x;
        box[6L * c + 4] = hi.y;
        box[6L * c + 5] = hi.z;
    }
}

// ---- host plan ------------------------------------------------------------------

int build_rec(HostTree &h, int b, int size, int leaf)
{
    const int id = (int)h.node.size();
    h.node.push_back(make_int4(b, b + size, -1, -1));
    h.height.push_back(0);
    if (size <= leaf) {
        h.leaves.push_back(id);
        return id;
    }
    const int L = (size + leaf - 1) / leaf;
    const int k = std::min(size, leaf * ((L + 1) / 2));
    const int l = build_rec(h, b, k, leaf);
    const int r = build_rec(h, b + k, size - k, leaf);
    h.node[id].z = l;
    h.node[id].w = r;
    h.height[id] = 1 + std::max(h.height[l], h.height[r]);
    return id;
}

void groups_rec(HostTree &h, int id)
{
    const int4 nd = h.node[id];
    if (nd.y - nd.x <= kGroup || nd.z < 0) {
        h.groups.push_back(id);
        return;
    }
    groups_rec(h, nd.z);
    groups_rec(h, nd.w);
}

// (node count, group count) of the plan for `size` bodies without building
// it: the recursion splits as build_rec does and meets at most two sizes per
// level, so with the memo it takes O(log(size / leaf)) steps.
std::pair<int64_t, int64_t> plan_counts(int size, int leaf, std::map<int, std::pair<int64_t, int64_t>> &memo)
{
    const auto it = memo.find(size);
    if (it != memo.end()) return it->second;
    std::pair<int64_t, int64_t> r(1, 1);
    if (size > leaf) {
        const int L = (size + leaf - 1) / leaf;
        const int k = std::min(size, leaf * ((L + 1) / 2));
        const auto a = plan_counts(k, leaf, memo), b = plan_counts(size - k, leaf, memo);
        r.first = 1 + a.first + b.first;
        r.second = size <= kGroup ? 1 : a.second + b.second;
    }
    memo.emplace(size, r);
    return r;
}

void plan(HostTree &h, int n, int leaf)
{
    h = HostTree();
    const size_t nl = (size_t)((n + (int64_t)leaf - 1) / leaf);
    h.node.reserve(2 * nl);
    h.height.reserve(2 * nl);
    h.leaves.reserve(nl);
    build_rec(h, 0, n, leaf);
    groups_rec(h, 0);
    // bucket the nodes by height (counting sort; leaves keep ORB order)
    const int H = h.height[0];
    h.height_off.assign(H + 2, 0);
    for (int v : h.height) ++h.height_off[v + 1];
    for (int k = 0; k <= H; ++k) h.height_off[k + 1] += h.height_off[k];
    h.by_height.assign(h.node.size(), 0);
    std::vector<int> pos(h.height_off.begin(), h.height_off.end() - 1);
    for (size_t id = 0; id < h.node.size(); ++id) {
        if (h.height[id] == 0) continue;
        h.by_height[pos[h.height[id]]++] = (int)id;
    }
    for (size_t k = 0; k < h.leaves.size(); ++k) h.by_height[k] = h.leaves[k];
}

struct TreeCache {
    int n = 0, leaf = 0, dev = -1;
    HostTree host;
    void *mem = nullptr;
    size_t bytes = 0;
    TreeDev d{};
    // re-ordering scratch of the tree leapfrog: one record array, the new
    // permutation and the composed order (allocated on first use)
    void *reo = nullptr;
    size_t reo_bytes = 0;
};
std::mutex g_tree_mu;
TreeCache g_tree;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Makes the device tables and node arrays for (n, leaf) current; returns the
// device view.  Called with g_tree_mu held.
int tree_prepare(int n, int leaf, hipStream_t s, TreeDev &out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return NBODY_E_HIP;
    }
    TreeCache &C = g_tree;
    if (C.mem && C.n == n && C.leaf == leaf && C.dev == dev) {
        out = C.d;
        return NBODY_OK;
    }
    HostTree h;
    plan(h, n, leaf);
    const size_t nn = h.node.size(), ng = h.groups.size();
    const size_t o_node = 0;
    const size_t o_byh = o_node + align256(nn * sizeof(int4));
    const size_t o_grp = o_byh + align256(nn * sizeof(int));
    const size_t o_sums = o_grp + align256(ng * sizeof(int));
    const size_t o_comd = o_sums + align256(nn * sizeof(double4));
    const size_t o_rec = o_comd + align256(nn * sizeof(double4));
    const size_t o_lo = o_rec + align256(nn * sizeof(float4));
    const size_t o_hi = o_lo + align256(nn * sizeof(float4));
    const size_t o_s2a = o_hi + align256(nn * sizeof(float4));
    const size_t o_s2b = o_s2a + align256(nn * sizeof(double4));
    const size_t o_pp = o_s2b + align256(nn * sizeof(double4));
    const size_t o_qr = o_pp + align256(nn * kPseudo * sizeof(float4));
    const size_t o_ord = o_qr + align256(nn * kQuadRec * sizeof(float4));
    const size_t o_obin = o_ord + align256(ng * sizeof(int));
    const size_t o_ohist = o_obin + align256(ng * sizeof(unsigned short));
    const size_t total = o_ohist + align256((ng + kOrderThreads - 1) / kOrderThreads * kOrderBins * sizeof(int));
    if (C.mem) {
        // work already enqueued may still read the old tables
        (void)hipDeviceSynchronize();
        (void)hipFree(C.mem);
        C.mem = nullptr;
        C.bytes = 0;
    }
    void *mem = nullptr;
    if (hipMalloc(&mem, total) != hipSuccess) {
        set_error("cannot allocate %zu bytes of tree tables", total);
        return NBODY_E_NOMEM;
    }
    char *base = (char *)mem;
    TreeDev d;
    d.node = (const int4 *)(base + o_node);
    d.by_height = (const int *)(base + o_byh);
    d.groups = (const int *)(base + o_grp);
    d.sums = (double4 *)(base + o_sums);
    d.comd = (double4 *)(base + o_comd);
    d.rec = (float4 *)(base + o_rec);
    d.lo = (float4 *)(base + o_lo);
    d.hi = (float4 *)(base + o_hi);
    d.s2a = (double4 *)(base + o_s2a);
    d.s2b = (double4 *)(base + o_s2b);
    d.pp = (float4 *)(base + o_pp);
    d.qr = (float4 *)(base + o_qr);
    d.order = (int *)(base + o_ord);
    d.obin = (unsigned short *)(base + o_obin);
    d.ohist = (int *)(base + o_ohist);
    // pageable copies complete on the host side before returning; the vectors
    // stay alive in the cache in any case
    C.host = std::move(h);
    hipError_t e = hipMemcpyAsync(base + o_node, C.host.node.data(), nn * sizeof(int4), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + o_byh, C.host.by_height.data(), nn * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + o_grp, C.host.groups.data(), ng * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(e, "tree table upload");
    }
    C.mem = mem;
    C.bytes = total;
    C.n = n;
    C.leaf = leaf;
    C.dev = dev;
    C.d = d;
    out = d;
    return NBODY_OK;
}

template <bool Q2>
hipError_t launch_moments_t(const float4 *pm, const TreeDev &d, const HostTree &h, int cells, hipStream_t s)
{
    const int nl = (int)h.leaves.size();
    hipLaunchKernelGGL(k_tree_leaves<Q2>, dim3((nl + 255) / 256), dim3(256), 0, s, pm, d, nl);
    hipError_t e = hipGetLastError();
    for (size_t k = 1; e == hipSuccess && k + 1 < h.height_off.size(); ++k) {
        const int first = h.height_off[k], count = h.height_off[k + 1] - first;
        hipLaunchKernelGGL(k_tree_inner<Q2>, dim3((count + 255) / 256), dim3(256), 0, s, d, first, count);
        e = hipGetLastError();
    }
    const int nn = (int)h.node.size();
    if (Q2 && e == hipSuccess && cells == kCellsPseudo) {
        hipLaunchKernelGGL(k_tree_pseudo, dim3((nn * kPseudo + 255) / 256), dim3(256), 0, s, d, nn);
        e = hipGetLastError();
    }
    if (Q2 && e == hipSuccess && (cells == kCellsQuad || cells == kCellsLocal)) {
        hipLaunchKernelGGL(k_tree_quad, dim3((nn + 255) / 256), dim3(256), 0, s, d, nn);
        e = hipGetLastError();
    }
    return e;
}

// The pseudo-particle kernel indexes (node, direction) pairs with an int.
bool pseudo_fits(const HostTree &h)
{
    if (h.node.size() * (size_t)kPseudo <= (size_t)INT32_MAX) return true;
    set_error("%zu tree nodes are too many for order-2 cells", h.node.size());
    return false;
}

// Monopole moments and boxes; for the other cell models also the second
// moments and the cells' records.
hipError_t launch_moments(const float4 *pm, const TreeDev &d, const HostTree &h, int cells, hipStream_t s)
{
    return cells != kCellsMono ? launch_moments_t<true>(pm, d, h, cells, s)
                               : launch_moments_t<false>(pm, d, h, cells, s);
}

template <int MODE, bool INSPECT, int CELLS>
hipError_t launch_walk(const float4 *pm, int n, const TreeDev &d, int ngroups, float eps2, double G,
                       double theta2, const WalkOut &o, hipStream_t s)
{
    const float4 *recs = CELLS == kCellsPseudo ? d.pp : (CELLS >= kCellsQuad ? d.qr : d.rec);
    // the local-expansion force walk over many groups runs the largest boxes
    // first (unless NBODY_TREE_ORDER=0); the other walks and inspection keep
    // ORB order
    const int *order = nullptr;
    const char *env = getenv("NBODY_TREE_ORDER");
    if (!INSPECT && CELLS == kCellsLocal && ngroups >= kOrderMinGroups && !(env && env[0] == '0')) {
        hipLaunchKernelGGL(k_order_bins, dim3((ngroups + kOrderThreads - 1) / kOrderThreads), dim3(kOrderThreads), 0,
                           s, d, ngroups);
        hipLaunchKernelGGL(k_group_order, dim3(1), dim3(kOrderThreads), 0, s, d, ngroups);
        order = d.order;
    }
    hipLaunchKernelGGL((k_tree_walk<MODE, INSPECT, CELLS>), dim3(ngroups), dim3(64), 0, s, pm, n, d, recs, eps2,
                       G, theta2, o, order);
    return hipGetLastError();
}

}  // namespace

int tree_shape(int n, int leaf, int64_t *num_nodes, int64_t *num_groups, int32_t *nodes_out)
{
    if (!nodes_out) {
        std::map<int, std::pair<int64_t, int64_t>> memo;
        const auto c = plan_counts(n, leaf, memo);
        if (num_nodes) *num_nodes = c.first;
        if (num_groups) *num_groups = c.second;
        return NBODY_OK;
    }
    HostTree h;
    plan(h, n, leaf);
    if (num_nodes) *num_nodes = (int64_t)h.node.size();
    if (num_groups) *num_groups = (int64_t)h.groups.size();
    if (nodes_out) std::memcpy(nodes_out, h.node.data(), h.node.size() * sizeof(int4));
    return NBODY_OK;
}

int tree_moments(const void *pm, int n, int leaf, double *mom, float *box, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_tree_mu);
    TreeDev d;
    int rc = tree_prepare(n, leaf, s, d);
    if (rc != NBODY_OK) return rc;
    const int nn = (int)g_tree.host.node.size();
    hipError_t e = launch_moments((const float4 *)pm, d, g_tree.host, 0, s);
    if (e == hipSuccess && (mom || box)) {
        hipLaunchKernelGGL(k_tree_export, dim3((nn + 255) / 256), dim3(256), 0, s, d, nn, mom, box);
        e = hipGetLastError();
    }
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "tree moments");
}

int tree_lists(const void *pm, int n, int leaf, double theta, int max_far, int max_near, int32_t *far_cnt,
               int32_t *near_cnt, int32_t *far_ids, int32_t *near_ids, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_tree_mu);
    TreeDev d;
    int rc = tree_prepare(n, leaf, s, d);
    if (rc != NBODY_OK) return rc;
    hipError_t e = launch_moments((const float4 *)pm, d, g_tree.host, 0, s);
    WalkOut o{};
    o.far_cnt = far_cnt;
    o.near_cnt = near_cnt;
    o.far_ids = far_ids;
    o.near_ids = near_ids;
    o.max_far = far_ids ? max_far : 0;
    o.max_near = near_ids ? max_near : 0;
    if (e == hipSuccess)
        e = launch_walk<M_F32, true, kCellsMono>((const float4 *)pm, n, d, (int)g_tree.host.groups.size(),
                                                 0.0f, 1.0, theta * theta, o, s);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "tree lists");
}

namespace {
template <int CELLS>
hipError_t walk_prec(int prec, const float4 *pm, int n, const TreeDev &d, int ng, float eps2, double G, double th2,
                     const WalkOut &o, hipStream_t s)
{
    switch (prec) {
    case NBODY_F32: return launch_walk<M_F32, false, CELLS>(pm, n, d, ng, eps2, G, th2, o, s);
    case NBODY_F32_KAHAN: return launch_walk<M_KAHAN, false, CELLS>(pm, n, d, ng, eps2, G, th2, o, s);
    default: return launch_walk<M_F64ACC, false, CELLS>(pm, n, d, ng, eps2, G, th2, o, s);
    }
}
}  // namespace

int tree_local_counts(const void *pm, int n, int leaf, double theta, int32_t *loc_cnt, int32_t *far_cnt,
                      int32_t *near_cnt, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_tree_mu);
    TreeDev d;
    int rc = tree_prepare(n, leaf, s, d);
    if (rc != NBODY_OK) return rc;
    hipError_t e = launch_moments((const float4 *)pm, d, g_tree.host, kCellsMono, s);
    WalkOut o{};
    o.far_cnt = far_cnt;
    o.near_cnt = near_cnt;
    o.loc_cnt = loc_cnt;
    if (e == hipSuccess)
        e = launch_walk<M_F32, true, kCellsLocal>((const float4 *)pm, n, d, (int)g_tree.host.groups.size(), 0.0f,
                                                  1.0, theta * theta, o, s);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "tree local counts");
}

int tree_accel(const void *pm, int n, int prec, double G, double eps, double theta, int leaf, int cells,
               void *out, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_tree_mu);
    TreeDev d;
    int rc = tree_prepare(n, leaf, s, d);
    if (rc != NBODY_OK) return rc;
    if (cells == kCellsPseudo && !pseudo_fits(g_tree.host)) return NBODY_E_INVAL;
    hipError_t e = launch_moments((const float4 *)pm, d, g_tree.host, cells, s);
    WalkOut o{};
    o.acc_pot = (float4 *)out;
    const int ng = (int)g_tree.host.groups.size();
    const float eps2 = (float)(eps * eps);
    const double th2 = theta * theta;
    if (e == hipSuccess) {
        if (cells == kCellsPseudo)
            e = walk_prec<kCellsPseudo>(prec, (const float4 *)pm, n, d, ng, eps2, G, th2, o, s);
        else if (cells == kCellsQuad)
            e = walk_prec<kCellsQuad>(prec, (const float4 *)pm, n, d, ng, eps2, G, th2, o, s);
        else if (cells == kCellsLocal)
            e = walk_prec<kCellsLocal>(prec, (const float4 *)pm, n, d, ng, eps2, G, th2, o, s);
        else
            e = walk_prec<kCellsMono>(prec, (const float4 *)pm, n, d, ng, eps2, G, th2, o, s);
    }
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "tree force");
}

std::mutex &tree_mutex() { return g_tree_mu; }

int tree_quad_prepare(const void *pm, int n, int leaf, hipStream_t s, TreeDev &d, const HostTree *&h)
{
    int rc = tree_prepare(n, leaf, s, d);
    if (rc != NBODY_OK) return rc;
    const hipError_t e = launch_moments((const float4 *)pm, d, g_tree.host, kCellsQuad, s);
    if (e != hipSuccess) return hip_fail(e, "tree moments");
    h = &g_tree.host;
    return NBODY_OK;
}

int tree_pseudo(const void *pm, int n, int leaf, void *out, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_tree_mu);
    TreeDev d;
    int rc = tree_prepare(n, leaf, s, d);
    if (rc != NBODY_OK) return rc;
    if (!pseudo_fits(g_tree.host)) return NBODY_E_INVAL;
    const size_t bytes = g_tree.host.node.size() * kPseudo * sizeof(float4);
    hipError_t e = launch_moments((const float4 *)pm, d, g_tree.host, kCellsPseudo, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d.pp, bytes, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "tree pseudo-particles");
}

int tree_quad(const void *pm, int n, int leaf, void *out, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_tree_mu);
    TreeDev d;
    int rc = tree_prepare(n, leaf, s, d);
    if (rc != NBODY_OK) return rc;
    const size_t bytes = g_tree.host.node.size() * kQuadRec * sizeof(float4);
    hipError_t e = launch_moments((const float4 *)pm, d, g_tree.host, kCellsQuad, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d.qr, bytes, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? NBODY_OK : hip_fail(e, "tree quadrupoles");
}

// ---- tree leapfrog ---------------------------------------------------------------
namespace {

__global__ __launch_bounds__(kBlock) void k_compose(const int32_t *__restrict__ order,
                                                    const int32_t *__restrict__ perm, int n,
                                                    int32_t *__restrict__ out)
{
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < n) out[p] = order[perm[p]];
}

// Puts the state into the ORB order of its current positions: x, v and a
// move with their bodies, and order[p] keeps naming the caller's index of
// the body at position p.
int reorder(void *pm, void *vel, void *acc, int32_t *order, int n, int leaf, hipStream_t s)
{
    const size_t rb = (size_t)n * 16, ib = (size_t)n * 4;
    const size_t need = rb + 2 * ((ib + 255) & ~size_t(255)) + 256;
    {
        std::lock_guard<std::mutex> lk(g_tree_mu);
        if (g_tree.reo_bytes < need) {
            if (g_tree.reo) {
                (void)hipDeviceSynchronize();
                (void)hipFree(g_tree.reo);
                g_tree.reo = nullptr;
                g_tree.reo_bytes = 0;
            }
            if (hipMalloc(&g_tree.reo, need) != hipSuccess) {
                set_error("cannot allocate %zu bytes of re-ordering scratch", need);
                return NBODY_E_NOMEM;
            }
            g_tree.reo_bytes = need;
        }
    }
    char *base = (char *)g_tree.reo;
    void *tmp = base;
    int32_t *perm = (int32_t *)(base + ((rb + 255) & ~size_t(255)));
    int32_t *ord = (int32_t *)((char *)perm + ((ib + 255) & ~size_t(255)));
    int rc = orb_order(pm, NBODY_F32, n, leaf, perm, s);
    if (rc != NBODY_OK) return rc;
    void *arr[3] = {pm, vel, acc};
    for (void *a : arr) {
        hipError_t e = launch_permute(a, tmp, perm, n, 16, false, s);
        if (e == hipSuccess) e = launch_copy(a, tmp, rb, s);
        if (e != hipSuccess) return hip_fail(e, "tree re-ordering");
    }
    if (order) {
        hipLaunchKernelGGL(k_compose, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, order, perm, n, ord);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(order, ord, ib, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "tree re-ordering");
    }
    return NBODY_OK;
}

}  // namespace

int tree_leapfrog(void *pm, void *vel, void *acc, int32_t *order, int n, int prec, double G, double eps,
                  double theta, int leaf, double dt, int nsteps, int reorder_every, unsigned flags,
                  double *energy, hipStream_t s)
{
    const double h = 0.5 * dt;
    double *ep = nullptr;
    if (energy) {
        ep = (double *)scratch(kSlotEnergy, sizeof(double) * 2 * step_blocks(n));
        if (!ep) {
            set_error("cannot allocate energy scratch");
            return NBODY_E_NOMEM;
        }
    }
    int eb = 0;
    if (reorder_every > 0) {
        const int rc = reorder(pm, vel, acc, order, n, leaf, s);
        if (rc != NBODY_OK) return rc;
    }
    const int cells = (flags & NBODY_TREE_LOCAL_CELLS)  ? kCellsLocal
                      : (flags & NBODY_TREE_QUAD_CELLS)   ? kCellsQuad
                      : (flags & NBODY_TREE_PSEUDO_CELLS) ? kCellsPseudo
                                                          : kCellsMono;
    if (!(flags & NBODY_ACC_VALID)) {
        const int rc = tree_accel(pm, n, prec, G, eps, theta, leaf, cells, acc, s);
        if (rc != NBODY_OK) return rc;
    }
    hipError_t e = launch_step(prec, pm, vel, acc, n, h, dt, false, nsteps > 0, ep, &eb, s);
    if (e == hipSuccess && energy) e = launch_energy_final(ep, eb, energy, s);
    if (e != hipSuccess) return hip_fail(e, "tree leapfrog step");
    for (int k = 0; k < nsteps; ++k) {
        if (reorder_every > 0 && (k + 1) % reorder_every == 0) {
            const int rc = reorder(pm, vel, acc, order, n, leaf, s);
            if (rc != NBODY_OK) return rc;
        }
        const int rc = tree_accel(pm, n, prec, G, eps, theta, leaf, cells, acc, s);
        if (rc != NBODY_OK) return rc;
        const bool last = (k == nsteps - 1);
        e = launch_step(prec, pm, vel, acc, n, h, dt, true, !last, ep, &eb, s);
        if (e == hipSuccess && energy) e = launch_energy_final(ep, eb, energy + 2 * (k + 1), s);
        if (e != hipSuccess) return hip_fail(e, "tree leapfrog step");
    }
    return NBODY_OK;
}

void tree_release()
{
    std::lock_guard<std::mutex> lk(g_tree_mu);
    if (g_tree.mem) (void)hipFree(g_tree.mem);
    if (g_tree.reo) (void)hipFree(g_tree.reo);
    g_tree = TreeCache();
}

}  // namespace nbi
