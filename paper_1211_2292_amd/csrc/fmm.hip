// Multi-level fast multipole method on the ORB nodes (gfx950).
//
// Section VI names the fast multipole method (its reference [20]) as the O(N)
// successor of the tree code.  Built here from the tree code's pieces: the
// ORB nodes with their FP64 moments and quadrupole records (tree.hip), the
// quadrupole cell's M2L into a third-order local expansion (m2l_f32), and
// the FP32 pair code of the direct sum (pair.h).  Definitions shared with the
// FP64 oracle (every node's lists are equal to the oracle's as sets):
// * MAC: target node A and source node B interact through M2L iff they share
//   no body and diag2_A + diag2_B < theta^2 |com_A - com_B|^2 (FP64).
// * Dual-tree traversal from (root, root): MAC -> B joins A's M2L list; two
//   leaves -> B joins A's P2P list; B a leaf, or A an inner node with
//   diag2_A >= diag2_B -> the pair passes to both children of A; otherwise
//   the pair is replaced by (A, B.left), (A, B.right).
// * A node's total local expansion = its own M2L sum + its parent's total
//   re-expanded about its centre of mass (exact for a cubic); every body of
//   a leaf evaluates its leaf's expansion and sums its P2P source leaves body
//   by body without the self pair.
//
// Device schedule:
// * Traversal, top-down by node depth.  For a target node A the pairs (A, .)
//   of the recursion are those inherited from its parent (the parent's
//   pass-down list) closed under source splits: one wave per node pops up to
//   64 pending sources per step from an LDS stack, one per lane, and
//   classifies them (ballot ranks give every output a fixed position).  Each
//   depth runs three kernels: count, scan (offsets, one workgroup), fill.
//   Lists live in library buffers; writes are bounds-checked and an overflow
//   flag makes the host grow the buffers and run again.
// * M2L: one wave per node, one source cell per lane, the twenty
//   coefficients summed over the wave in a fixed butterfly (FP32).
// * L2L: one thread per node, depth by depth, in FP64.
// * Leaves: one wave per leaf, 64 / P lanes per target (P the leaf size
//   rounded up to a power of two).  The P2P source leaves are staged in LDS
//   in batches of up to 512 bodies and swept with the direct kernel's pair
//   code (partials folded by the precision mode once per batch), then a
//   fixed butterfly over the target's lanes and the FP64 evaluation of the
//   leaf's expansion.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "pair.h"
#include "tree_shared.h"

namespace nbi {
namespace {

#define NB_CHECK_RC(expr)                \
    do {                                 \
        const int rc_ = (expr);          \
        if (rc_ != NBODY_OK) return rc_; \
    } while (0)

constexpr int kFmmStack = 64;     // bound on the tree height the traversal admits
constexpr int kWalkStack = 2048;  // LDS stack entries per walking wave (64 per source depth + refill)
constexpr int kTotWords = 3 + kFmmStack;  // list totals; node depth < tree height + 1 <= kFmmStack

struct FmmDev {
    const int4 *node;
    const double4 *comd;
    const float4 *qr;
    const int *parent;
    int nn;
    int *cnt;   // [3][nn]: M2L, P2P, pass-down counts per node
    int *lcnt;  // [3][nn]: the same counts at each node's position in depth order
    int *off;   // [3][nn]: M2L and P2P offsets (global), pass-down offsets (in the level's buffer)
    int *m2l, *p2p, *pass0, *pass1;
    long cap_m2l, cap_p2p, cap_pass;
    unsigned long long *tot;  // running M2L total, running P2P total, overflow flag, then the
                              // pass-down total of every depth
    float *own;               // [nn][20] own M2L sums
    double *loc;              // [nn][20] total expansions
};

__device__ __forceinline__ bool fmm_overlap(int4 a, int4 b) { return a.x < b.y && b.x < a.y; }

__device__ __forceinline__ unsigned fmm_rank(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// One wave per target node of one depth: the walk of its inherited
// sources.  The pending sources sit on an LDS stack; each step pops up to 64
// of them (one per lane) and classifies each: M2L, P2P, pass-down (to both
// children of A) or split (both children of B pushed).  Ballot ranks keep
// every output in a fixed order, so the count pass (FILL = false) and the
// fill pass (FILL = true, at the scanned offsets) produce the same lists.
template <bool FILL>
__global__ __launch_bounds__(64) void k_fmm_walk(FmmDev F, const int *__restrict__ ids, int first, int count,
                                                 int parity, double theta2)
{
    __shared__ int stk[kWalkStack];
    const int lane = threadIdx.x;
    const int t = blockIdx.x;
    if (t >= count) return;
    const int A = ids[t];
    const int4 na = F.node[A];
    const double4 ca = F.comd[A];
    const bool aleaf = na.z < 0;
    const int nn = F.nn;
    const int *in = nullptr;
    int nin = 1;
    if (A != 0) {
        const int P = F.parent[A];
        nin = F.cnt[2 * nn + P];
        const long base = F.off[2 * nn + P];
        if (base + nin > F.cap_pass) nin = (int)max(0L, F.cap_pass - base);  // the parent's depth overflowed
        in = (parity ? F.pass0 : F.pass1) + base;  // the previous depth's buffer
    }
    int *pass_out = parity ? F.pass1 : F.pass0;
    long om = 0, op = 0, opass = 0;
    if (FILL) {
        om = F.off[A];
        op = F.off[nn + A];
        opass = F.off[2 * nn + A];
    }
    int cm = 0, cp = 0, cq = 0, top = 0, next = 0;
    bool bad = false;
    for (;;) {
        if (top < 64 && next < nin) {  // refill from the inherited list
            const int k = min(64, nin - next);
            if (lane < k) stk[top + lane] = in ? in[next + lane] : 0;
            top += k;
            next += k;
        }
        if (top == 0) break;
        const int k = min(64, top);
        top -= k;
        __syncthreads();
        const bool act = lane < k;
        int B = act ? stk[top + lane] : 0;
        __syncthreads();
        if ((unsigned)B >= (unsigned)nn) B = 0;  // only after an overflow upstream
        bool m2l = false, p2p = false, pass = false, split = false;
        int4 nb = make_int4(0, 0, -1, -1);
        if (act) {
            nb = F.node[B];
            const double4 cb = F.comd[B];
            if (!fmm_overlap(na, nb)) {
                const double dx = ca.x - cb.x, dy = ca.y - cb.y, dz = ca.z - cb.z;
                const double dist2 = (dx * dx + dy * dy) + dz * dz;
                m2l = ca.w + cb.w < theta2 * dist2;
            }
            if (!m2l) {
                const bool bleaf = nb.z < 0;
                if (aleaf && bleaf)
                    p2p = true;
                else if (bleaf || (!aleaf && ca.w >= cb.w))
                    pass = true;
                else
                    split = true;
            }
        }
        const unsigned long long mm = __ballot(m2l), mp = __ballot(p2p), mq = __ballot(pass), ms = __ballot(split);
        if (FILL) {
            if (m2l) {
                const long q = om + cm + (long)fmm_rank(mm);
                if (q < F.cap_m2l) F.m2l[q] = B;
                else bad = true;
            }
            if (p2p) {  // a source leaf is stored as its first body
                const long q = op + cp + (long)fmm_rank(mp);
                if (q < F.cap_p2p) F.p2p[q] = nb.x;
                else bad = true;
            }
            if (pass) {
                const long q = opass + cq + (long)fmm_rank(mq);
                if (q < F.cap_pass) pass_out[q] = B;
                else bad = true;
            }
        }
        cm += __popcll(mm);
        cp += __popcll(mp);
        cq += __popcll(mq);
        const int ns = __popcll(ms);
        if (top + 2 * ns > kWalkStack) {  // cannot happen for trees the host admits
            bad = true;
            break;
        }
        if (split) {
            const int q = top + 2 * (int)fmm_rank(ms);
            stk[q] = nb.w;
            stk[q + 1] = nb.z;
        }
        top += 2 * ns;
        __syncthreads();
    }
    if (!FILL && lane == 0) {
        F.cnt[A] = cm;
        F.cnt[nn + A] = cp;
        F.cnt[2 * nn + A] = cq;
        F.lcnt[first + t] = cm;
        F.lcnt[nn + first + t] = cp;
        F.lcnt[2 * nn + first + t] = cq;
    }
    if (__ballot(bad) && lane == 0) atomicOr(&F.tot[2], 1ull);
}

// One workgroup: exclusive scans of the three counts over one depth's nodes
// (in the order of ids).  M2L and P2P offsets continue the running totals;
// pass-down offsets start at 0 in the depth's buffer.  Each thread sums a
// contiguous chunk, the 1024 chunk sums are scanned in LDS (Hillis-Steele),
// and each thread writes its chunk's offsets.
__global__ __launch_bounds__(1024) void k_fmm_scan(FmmDev F, const int *__restrict__ ids, int first, int count,
                                                   int depth)
{
    __shared__ long part[2][3][1024];
    const int tid = threadIdx.x;
    const int per = (count + 1023) / 1024;
    const int b = min(count, tid * per), e = min(count, b + per);
    const int nn = F.nn;
    const int *lc = F.lcnt + first;
    long s[3] = {0, 0, 0};
#pragma unroll 4
    for (int k = b; k < e; ++k)
        for (int q = 0; q < 3; ++q) s[q] += lc[q * nn + k];
    for (int q = 0; q < 3; ++q) part[0][q][tid] = s[q];
    __syncthreads();
    int cur = 0;
    for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan of the chunk sums
        for (int q = 0; q < 3; ++q)
            part[cur ^ 1][q][tid] = part[cur][q][tid] + (tid >= d ? part[cur][q][tid - d] : 0L);
        cur ^= 1;
        __syncthreads();
    }
    long o[3];
    for (int q = 0; q < 3; ++q) {
        const long base = q < 2 ? (long)F.tot[q] : 0L;
        o[q] = base + part[cur][q][tid] - s[q];
    }
    __syncthreads();  // every thread has read the running totals
    if (tid < 3) {
        const long run = (tid < 2 ? (long)F.tot[tid] : 0L) + part[cur][tid][1023];
        F.tot[tid < 2 ? tid : 3 + depth] = (unsigned long long)run;
        const long cap = tid == 0 ? F.cap_m2l : (tid == 1 ? F.cap_p2p : F.cap_pass);
        if (run > cap || run > (long)INT32_MAX) atomicOr(&F.tot[2], 1ull);
    }
    for (int k = b; k < e; ++k) {
        const int A = ids[k];
        for (int q = 0; q < 3; ++q) {
            F.off[q * nn + A] = (int)min(o[q], (long)INT32_MAX);
            o[q] += lc[q * nn + k];
        }
    }
}

// M2L: one wave per node.
__global__ __launch_bounds__(256) void k_fmm_m2l(FmmDev F, float eps2)
{
    const int A = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (A >= F.nn) return;
    const int c = F.cnt[A];
    const long o = F.off[A];
    const double4 ca = F.comd[A];
    const float zx = (float)ca.x, zy = (float)ca.y, zz = (float)ca.z;
    Local L;
#pragma unroll
    for (int k = 0; k < 20; ++k) L.c[k] = 0.0f;
    for (int k = lane; k < c; k += 64) {
        if (o + k >= F.cap_m2l) break;
        const int B = F.m2l[o + k];
        if ((unsigned)B < (unsigned)F.nn) m2l_f32(F.qr + (long)kQuadRec * B, zx, zy, zz, eps2, L);
    }
#pragma unroll
    for (int k = 0; k < 20; ++k) {
        float v = L.c[k];
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s);
        L.c[k] = v;
    }
    if (lane < 20) {
        float v = 0.0f;
#pragma unroll
        for (int k = 0; k < 20; ++k) v = lane == k ? L.c[k] : v;
        F.own[20L * A + lane] = v;
    }
}

// Full symmetric K and T of the 20 coefficients (P0, p, K: xx yy zz xy xz yz,
// T: xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz) contracted with d:
// kd = K d, td = T d (3x3), tdd = T(d, d).
__device__ __forceinline__ void fmm_contract(const double *c, const double d[3], double kd[3], double td[3][3],
                                             double tdd[3])
{
    const double K[3][3] = {{c[4], c[7], c[8]}, {c[7], c[5], c[9]}, {c[8], c[9], c[6]}};
    // T[k][l][m] by the stored index of the sorted triple
    auto T = [&](int k, int l, int m) -> double {
        int a = k, b = l, e = m, x;
        if (a > b) { x = a; a = b; b = x; }
        if (b > e) { x = b; b = e; e = x; }
        if (a > b) { x = a; a = b; b = x; }
        if (a == b && b == e) return c[10 + a];                       // xxx yyy zzz
        if (a == 0 && b == 0) return c[e == 1 ? 13 : 14];             // xxy xxz
        if (a == 0 && b == 1 && e == 1) return c[15];                 // xyy
        if (a == 1 && b == 1) return c[16];                           // yyz
        if (a == 0 && b == 2) return c[17];                           // xzz
        if (a == 1 && b == 2) return c[18];                           // yzz
        return c[19];                                                 // xyz
    };
    for (int k = 0; k < 3; ++k) {
        kd[k] = (K[k][0] * d[0] + K[k][1] * d[1]) + K[k][2] * d[2];
        for (int l = 0; l < 3; ++l) td[k][l] = (T(k, l, 0) * d[0] + T(k, l, 1) * d[1]) + T(k, l, 2) * d[2];
        tdd[k] = (td[k][0] * d[0] + td[k][1] * d[1]) + td[k][2] * d[2];
    }
}

// L2L, one thread per node of one depth: loc[A] = own[A] + the parent's
// total re-expanded about com_A (the root takes its own sum).
__global__ __launch_bounds__(256) void k_fmm_l2l(FmmDev F, const int *__restrict__ ids, int count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int A = ids[t];
    const int P = F.parent[A];
    double *out = F.loc + 20L * A;
    const float *own = F.own + 20L * A;
    if (P < 0) {
        for (int k = 0; k < 20; ++k) out[k] = (double)own[k];
        return;
    }
    const double *c = F.loc + 20L * P;
    const double4 ca = F.comd[A], cp = F.comd[P];
    const double d[3] = {ca.x - cp.x, ca.y - cp.y, ca.z - cp.z};
    double kd[3], td[3][3], tdd[3];
    fmm_contract(c, d, kd, td, tdd);
    const double pd = (c[1] * d[0] + c[2] * d[1]) + c[3] * d[2];
    const double dkd = (d[0] * kd[0] + d[1] * kd[1]) + d[2] * kd[2];
    const double dtdd = (d[0] * tdd[0] + d[1] * tdd[1]) + d[2] * tdd[2];
    out[0] = (c[0] + pd + 0.5 * dkd + dtdd / 6.0) + (double)own[0];
    for (int k = 0; k < 3; ++k) out[1 + k] = (c[1 + k] + kd[k] + 0.5 * tdd[k]) + (double)own[1 + k];
    out[4] = (c[4] + td[0][0]) + (double)own[4];
    out[5] = (c[5] + td[1][1]) + (double)own[5];
    out[6] = (c[6] + td[2][2]) + (double)own[6];
    out[7] = (c[7] + td[0][1]) + (double)own[7];
    out[8] = (c[8] + td[0][2]) + (double)own[8];
    out[9] = (c[9] + td[1][2]) + (double)own[9];
    for (int k = 10; k < 20; ++k) out[k] = c[k] + (double)own[k];
}

// Leaves: one wave per leaf; LPT lanes per target.  A P2P entry is the
// first body of a source leaf (every leaf holds `leaf` bodies except the
// last, which ends at n).  Lanes read the entries 64 at a time; every source
// body is then loaded straight from memory (the sources of one leaf are
// spatial neighbours, mostly cache hits) with the entry's base broadcast
// from its lane, several loads in flight per lane, and swept with the
// direct kernel's pair code.
template <int MODE, int LPT>
__global__ __launch_bounds__(64) void k_fmm_leaf(const float4 *__restrict__ src, FmmDev F,
                                                 const int *__restrict__ leaves, int nleaves, float eps2_in,
                                                 double G, float4 *__restrict__ out, int n, int leaf)
{
    constexpr int P = 64 / LPT;                  // target slots (>= the leaf size)
    constexpr int BPL = P >= LPT ? P / LPT : 1;  // bodies of one entry per lane
    constexpr int EPS = P >= LPT ? 1 : LPT / P;  // entries per step
    constexpr int UNR = BPL >= 8 ? 1 : 8 / BPL;  // steps per unrolled block (8 loads in flight)
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    if (w >= nleaves) return;
    const int A = leaves[w];
    const int4 na = F.node[A];
    const int nn = F.nn;
    const int u = lane % LPT;
    const int i = na.x + lane / LPT;
    const float eps2 = lane_copy(eps2_in);
    Targets<float, 1> T;
    {
        const float4 p = src[min(i, na.y - 1)];
        T.x[0] = p.x;
        T.y[0] = p.y;
        T.z[0] = p.z;
        T.i[0] = i;
    }
    Run<MODE> R[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) R[c].zero();
    const int cp = F.cnt[nn + A];
    const long op = F.off[nn + A];
    const int cpc = (int)min((long)cp, max(0L, F.cap_p2p - op));
    // lane's entry within a step and its body slot
    const int esub = EPS > 1 ? u / P : 0;
    const int b0 = EPS > 1 ? u % P : u;
    for (int base = 0; base < cpc; base += 64) {
        const int k = min(64, cpc - base);
        const int mybeg = lane < k ? F.p2p[op + base + lane] : 0;
        Sums<float, 1> S;
        S.zero();
        for (int e0 = 0; e0 < k; e0 += EPS * UNR) {
            float4 sv[UNR][BPL];
            int sj[UNR][BPL];
            bool ok[UNR][BPL];
#pragma unroll
            for (int r = 0; r < UNR; ++r) {
                const int e = e0 + r * EPS + esub;
                int bg;
                if constexpr (EPS > 1)
                    bg = __shfl(mybeg, min(e, 63));
                else
                    bg = __builtin_amdgcn_readlane(mybeg, min(e0 + r, 63));
                const int len = (unsigned)bg < (unsigned)n ? min(leaf, n - bg) : 0;
#pragma unroll
                for (int q = 0; q < BPL; ++q) {
                    const int body = b0 + q * LPT;
                    ok[r][q] = e < k && body < len;
                    sj[r][q] = bg + body;
                    sv[r][q] = src[ok[r][q] ? sj[r][q] : 0];
                }
            }
#pragma unroll
            for (int r = 0; r < UNR; ++r)
#pragma unroll
                for (int q = 0; q < BPL; ++q)
                    if (ok[r][q]) pair_f32<1, true>(sv[r][q], sj[r][q], T, eps2, S);
        }
        R[0].fold(S.ax[0]);
        R[1].fold(S.ay[0]);
        R[2].fold(S.az[0]);
        R[3].fold(S.ph[0]);
    }
    double r[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double v = R[c].get();
#pragma unroll
        for (int s = LPT / 2; s >= 1; s >>= 1) v += __shfl_xor(v, s);
        r[c] = v;
    }
    if (u != 0 || i >= na.y) return;
    // the leaf's expansion at this body, in FP64
    const double *c = F.loc + 20L * A;
    const double4 ca = F.comd[A];
    const double y[3] = {(double)T.x[0] - ca.x, (double)T.y[0] - ca.y, (double)T.z[0] - ca.z};
    double ky[3], ty[3][3], tyy[3];
    fmm_contract(c, y, ky, ty, tyy);
    r[0] += c[1] + ky[0] + 0.5 * tyy[0];
    r[1] += c[2] + ky[1] + 0.5 * tyy[1];
    r[2] += c[3] + ky[2] + 0.5 * tyy[2];
    const double py = (c[1] * y[0] + c[2] * y[1]) + c[3] * y[2];
    const double yky = (y[0] * ky[0] + y[1] * ky[1]) + y[2] * ky[2];
    const double ytyy = (y[0] * tyy[0] + y[1] * tyy[1]) + y[2] * tyy[2];
    r[3] += c[0] + py + 0.5 * yky + ytyy / 6.0;
    if constexpr (MODE == M_F32)
        put_f32(out, i, r, (float)G);
    else
        put(out, i, r, G);
}

__global__ void k_fmm_zero_tot(unsigned long long *tot, int count)
{
    for (int k = threadIdx.x; k < count; k += blockDim.x) tot[k] = 0ull;
}

// ---- host side -----------------------------------------------------------------
struct FmmPlan {
    int n = 0, leaf = 0, dev = -1, nn = 0, depth = 0;
    std::vector<int> parent, by_depth, depth_off;
    int *d_parent = nullptr, *d_by_depth = nullptr, *d_leaves = nullptr;
};

struct FmmBufs {
    int dev = -1, nn = 0;
    long cap_m2l = 0, cap_p2p = 0, cap_pass = 0;
    int *cnt = nullptr, *lcnt = nullptr, *off = nullptr, *m2l = nullptr, *p2p = nullptr, *pass0 = nullptr, *pass1 = nullptr;
    unsigned long long *tot = nullptr;
    float *own = nullptr;
    double *loc = nullptr;
};

std::mutex g_fmm_mu;
FmmPlan g_plan;
FmmBufs g_bufs;

void free_plan(FmmPlan &p)
{
    (void)hipFree(p.d_parent);
    (void)hipFree(p.d_by_depth);
    (void)hipFree(p.d_leaves);
    p = FmmPlan();
}

void free_bufs(FmmBufs &b)
{
    (void)hipFree(b.cnt);
    (void)hipFree(b.lcnt);
    (void)hipFree(b.off);
    (void)hipFree(b.m2l);
    (void)hipFree(b.p2p);
    (void)hipFree(b.pass0);
    (void)hipFree(b.pass1);
    (void)hipFree(b.tot);
    (void)hipFree(b.own);
    (void)hipFree(b.loc);
    b = FmmBufs();
}

int make_plan(const HostTree &h, int n, int leaf, int dev, hipStream_t s)
{
    FmmPlan &p = g_plan;
    if (p.d_parent && p.n == n && p.leaf == leaf && p.dev == dev) return NBODY_OK;
    if (p.d_parent) {
        (void)hipDeviceSynchronize();  // enqueued work may still read the old tables
        free_plan(p);
    }
    const int nn = (int)h.node.size();
    if (64 * (h.height[0] + 2) > kWalkStack || h.height[0] + 2 > kFmmStack) {
        set_error("tree height %d too large for the FMM traversal stack", h.height[0]);
        return NBODY_E_UNSUPPORTED;
    }
    p.parent.assign(nn, -1);
    std::vector<int> dep(nn, 0);
    for (int a = 0; a < nn; ++a) {  // preorder: parents come first
        const int4 nd = h.node[a];
        if (nd.z >= 0) {
            p.parent[nd.z] = p.parent[nd.w] = a;
            dep[nd.z] = dep[nd.w] = dep[a] + 1;
        }
    }
    p.depth = *std::max_element(dep.begin(), dep.end());
    p.depth_off.assign(p.depth + 2, 0);
    for (int v : dep) ++p.depth_off[v + 1];
    for (int k = 0; k <= p.depth; ++k) p.depth_off[k + 1] += p.depth_off[k];
    p.by_depth.assign(nn, 0);
    std::vector<int> pos(p.depth_off.begin(), p.depth_off.end() - 1);
    for (int a = 0; a < nn; ++a) p.by_depth[pos[dep[a]]++] = a;
    const size_t nl = h.leaves.size();
    if (hipMalloc(&p.d_parent, nn * sizeof(int)) != hipSuccess ||
        hipMalloc(&p.d_by_depth, nn * sizeof(int)) != hipSuccess ||
        hipMalloc(&p.d_leaves, nl * sizeof(int)) != hipSuccess) {
        free_plan(p);
        set_error("cannot allocate the FMM plan");
        return NBODY_E_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(p.d_parent, p.parent.data(), nn * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p.d_by_depth, p.by_depth.data(), nn * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p.d_leaves, h.leaves.data(), nl * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "FMM plan upload");
    }
    p.n = n;
    p.leaf = leaf;
    p.dev = dev;
    p.nn = nn;
    return NBODY_OK;
}

// Buffers for nn nodes with at least the given list capacities.
int make_bufs(int nn, int dev, long cap_m2l, long cap_p2p, long cap_pass)
{
    FmmBufs &b = g_bufs;
    if (b.cnt && b.dev == dev && b.nn >= nn && b.cap_m2l >= cap_m2l && b.cap_p2p >= cap_p2p &&
        b.cap_pass >= cap_pass)
        return NBODY_OK;
    cap_m2l = std::max(cap_m2l, b.dev == dev ? b.cap_m2l : 0L);
    cap_p2p = std::max(cap_p2p, b.dev == dev ? b.cap_p2p : 0L);
    cap_pass = std::max(cap_pass, b.dev == dev ? b.cap_pass : 0L);
    nn = std::max(nn, b.dev == dev ? b.nn : 0);
    if (b.cnt) {
        (void)hipDeviceSynchronize();
        free_bufs(b);
    }
    bool ok = hipMalloc(&b.cnt, 3 * (size_t)nn * sizeof(int)) == hipSuccess &&
              hipMalloc(&b.lcnt, 3 * (size_t)nn * sizeof(int)) == hipSuccess &&
              hipMalloc(&b.off, 3 * (size_t)nn * sizeof(int)) == hipSuccess &&
              hipMalloc(&b.m2l, (size_t)cap_m2l * sizeof(int)) == hipSuccess &&
              hipMalloc(&b.p2p, (size_t)cap_p2p * sizeof(int)) == hipSuccess &&
              hipMalloc(&b.pass0, (size_t)cap_pass * sizeof(int)) == hipSuccess &&
              hipMalloc(&b.pass1, (size_t)cap_pass * sizeof(int)) == hipSuccess &&
              hipMalloc(&b.tot, kTotWords * sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc(&b.own, 20 * (size_t)nn * sizeof(float)) == hipSuccess &&
              hipMalloc(&b.loc, 20 * (size_t)nn * sizeof(double)) == hipSuccess;
    if (!ok) {
        free_bufs(b);
        set_error("cannot allocate FMM lists (%ld M2L, %ld P2P, %ld pass-down entries)", cap_m2l, cap_p2p,
                  cap_pass);
        return NBODY_E_NOMEM;
    }
    b.dev = dev;
    b.nn = nn;
    b.cap_m2l = cap_m2l;
    b.cap_p2p = cap_p2p;
    b.cap_pass = cap_pass;
    return NBODY_OK;
}

FmmDev dev_view(const TreeDev &d, const FmmPlan &p, const FmmBufs &b)
{
    FmmDev F;
    F.node = d.node;
    F.comd = d.comd;
    F.qr = d.qr;
    F.parent = p.d_parent;
    F.nn = p.nn;
    F.cnt = b.cnt;
    F.lcnt = b.lcnt;
    F.off = b.off;
    F.m2l = b.m2l;
    F.p2p = b.p2p;
    F.pass0 = b.pass0;
    F.pass1 = b.pass1;
    F.cap_m2l = b.cap_m2l;
    F.cap_p2p = b.cap_p2p;
    F.cap_pass = b.cap_pass;
    F.tot = b.tot;
    F.own = b.own;
    F.loc = b.loc;
    return F;
}

// The traversal: count, scan and fill per depth.
hipError_t launch_traversal(const FmmDev &F, const FmmPlan &p, double theta2, hipStream_t s)
{
    hipLaunchKernelGGL(k_fmm_zero_tot, dim3(1), dim3(64), 0, s, F.tot, kTotWords);
    hipError_t e = hipGetLastError();
    for (int d = 0; d <= p.depth && e == hipSuccess; ++d) {
        const int first = p.depth_off[d], count = p.depth_off[d + 1] - first;
        const int *ids = p.d_by_depth + first;
        hipLaunchKernelGGL(k_fmm_walk<false>, dim3(count), dim3(64), 0, s, F, ids, first, count, d & 1, theta2);
        hipLaunchKernelGGL(k_fmm_scan, dim3(1), dim3(1024), 0, s, F, ids, first, count, d);
        hipLaunchKernelGGL(k_fmm_walk<true>, dim3(count), dim3(64), 0, s, F, ids, first, count, d & 1, theta2);
        e = hipGetLastError();
    }
    return e;
}

template <int MODE>
hipError_t launch_leaves_mode(const float4 *pm, const FmmDev &F, const FmmPlan &p, int nleaves, int n, int leaf,
                              float eps2, double G, float4 *out, hipStream_t s)
{
    int P2 = 1;
    while (P2 < leaf) P2 *= 2;
    const dim3 grid(nleaves), blk(64);
#define NB_FMM_LEAF(L) \
    hipLaunchKernelGGL((k_fmm_leaf<MODE, L>), grid, blk, 0, s, pm, F, p.d_leaves, nleaves, eps2, G, out, n, leaf)
    switch (64 / P2) {
    case 64: NB_FMM_LEAF(64); break;
    case 32: NB_FMM_LEAF(32); break;
    case 16: NB_FMM_LEAF(16); break;
    case 8: NB_FMM_LEAF(8); break;
    case 4: NB_FMM_LEAF(4); break;
    case 2: NB_FMM_LEAF(2); break;
    default: NB_FMM_LEAF(1); break;
    }
#undef NB_FMM_LEAF
    return hipGetLastError();
}

// Runs the traversal (and, with out != nullptr, the whole FMM) until the
// lists fit their buffers.  Called with the tree and FMM locks held.
int fmm_run(const void *pm, int n, int prec, double G, double eps, double theta, int leaf, void *out,
            hipStream_t s, TreeDev &d, const HostTree *&h)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return NBODY_E_HIP;
    }
    NB_CHECK_RC(tree_quad_prepare(pm, n, leaf, s, d, h));
    NB_CHECK_RC(make_plan(*h, n, leaf, dev, s));
    const FmmPlan &p = g_plan;
    const int nn = p.nn;
    const int nleaves = (int)h->leaves.size();
    long want_m2l = std::max(1024L, 64L * nn), want_p2p = std::max(1024L, 512L * nleaves);
    long want_pass = std::max(1024L, 16L * nn);
    if (g_bufs.dev == dev) {
        want_m2l = std::max(want_m2l, g_bufs.cap_m2l);
        want_p2p = std::max(want_p2p, g_bufs.cap_p2p);
        want_pass = std::max(want_pass, g_bufs.cap_pass);
    }
    for (int attempt = 0; attempt < 16; ++attempt) {
        NB_CHECK_RC(make_bufs(nn, dev, want_m2l, want_p2p, want_pass));
        const FmmDev F = dev_view(d, p, g_bufs);
        hipError_t e = launch_traversal(F, p, theta * theta, s);
        if (e == hipSuccess && out) {
            const float eps2 = (float)(eps * eps);
            hipLaunchKernelGGL(k_fmm_m2l, dim3((nn + 3) / 4), dim3(256), 0, s, F, eps2);
            e = hipGetLastError();
            for (int dd = 0; dd <= p.depth && e == hipSuccess; ++dd) {
                const int first = p.depth_off[dd], count = p.depth_off[dd + 1] - first;
                hipLaunchKernelGGL(k_fmm_l2l, dim3((count + 255) / 256), dim3(256), 0, s, F,
                                   p.d_by_depth + first, count);
                e = hipGetLastError();
            }
            if (e == hipSuccess) {
                const float4 *x = (const float4 *)pm;
                float4 *o = (float4 *)out;
                switch (prec) {
                case NBODY_F32: e = launch_leaves_mode<M_F32>(x, F, p, nleaves, n, leaf, eps2, G, o, s); break;
                case NBODY_F32_KAHAN: e = launch_leaves_mode<M_KAHAN>(x, F, p, nleaves, n, leaf, eps2, G, o, s); break;
                default: e = launch_leaves_mode<M_F64ACC>(x, F, p, nleaves, n, leaf, eps2, G, o, s); break;
                }
            }
        }
        if (e != hipSuccess) return hip_fail(e, "FMM kernels");
        unsigned long long tot[kTotWords];
        e = hipMemcpyAsync(tot, g_bufs.tot, sizeof tot, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "FMM list check");
        if (!tot[2]) return NBODY_OK;
        // Grow what overflowed and run again.  The totals are exact up to the
        // first depth whose pass-down list overflowed and short beyond it, so
        // every attempt makes at least one more depth exact.
        unsigned long long pass_max = 0;
        bool pass_over = false;
        for (int dd = 0; dd <= p.depth; ++dd) {
            pass_max = std::max(pass_max, tot[3 + dd]);
            pass_over = pass_over || tot[3 + dd] > (unsigned long long)g_bufs.cap_pass;
        }
        auto grow = [](long cap, unsigned long long need, bool doubled) {
            long w = std::max(cap, (long)std::min<unsigned long long>(need + need / 4 + 1024, 1ull << 40));
            return doubled ? std::max(w, 2 * cap) : w;
        };
        want_pass = grow(g_bufs.cap_pass, pass_max, pass_over);
        want_m2l = grow(g_bufs.cap_m2l, tot[0], false);
        want_p2p = grow(g_bufs.cap_p2p, tot[1], false);
        if (want_m2l > (long)INT32_MAX || want_p2p > (long)INT32_MAX || want_pass > (long)INT32_MAX) {
            set_error("FMM lists beyond 2^31 entries (M2L %llu, P2P %llu, pass-down %llu counted so far; "
                      "theta too small for this n and leaf)",
                      tot[0], tot[1], pass_max);
            return NBODY_E_UNSUPPORTED;
        }
    }
    set_error("FMM lists did not fit after repeated growth");
    return NBODY_E_NOMEM;
}

}  // namespace

int fmm_accel(const void *pm, int n, int prec, double G, double eps, double theta, int leaf, void *out,
              hipStream_t s)
{
    std::lock_guard<std::mutex> lt(tree_mutex());
    std::lock_guard<std::mutex> lf(g_fmm_mu);
    TreeDev d;
    const HostTree *h = nullptr;
    return fmm_run(pm, n, prec, G, eps, theta, leaf, out, s, d, h);
}

int fmm_lists(const void *pm, int n, int leaf, double theta, int32_t *m2l_cnt, int32_t *p2p_cnt, int32_t *m2l_ids,
              int64_t m2l_cap, int32_t *p2p_ids, int64_t p2p_cap, hipStream_t s)
{
    std::lock_guard<std::mutex> lt(tree_mutex());
    std::lock_guard<std::mutex> lf(g_fmm_mu);
    TreeDev d;
    const HostTree *h = nullptr;
    NB_CHECK_RC(fmm_run(pm, n, NBODY_F32, 1.0, 0.0, theta, leaf, nullptr, s, d, h));
    const int nn = g_plan.nn;
    std::vector<int> cnt(3 * (size_t)nn), off(3 * (size_t)nn);
    unsigned long long tot[4];
    hipError_t e = hipMemcpyAsync(cnt.data(), g_bufs.cnt, cnt.size() * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(off.data(), g_bufs.off, off.size() * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(tot, g_bufs.tot, sizeof tot, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "FMM list download");
    std::vector<int> mc(cnt.begin(), cnt.begin() + nn), pc(cnt.begin() + nn, cnt.begin() + 2 * nn);
    e = hipMemcpyAsync(m2l_cnt, mc.data(), nn * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(p2p_cnt, pc.data(), nn * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "FMM count upload");
    for (int which = 0; which < 2; ++which) {
        int32_t *dst = which ? p2p_ids : m2l_ids;
        if (!dst) continue;
        const long total = (long)tot[which];
        const int64_t cap = which ? p2p_cap : m2l_cap;
        if (total > cap) {
            set_error("%s list of %ld entries exceeds the capacity %lld", which ? "P2P" : "M2L", total,
                      (long long)cap);
            return NBODY_E_INVAL;
        }
        std::vector<int> all(std::max(total, 1L)), grouped(std::max(total, 1L));
        e = hipMemcpyAsync(all.data(), which ? g_bufs.p2p : g_bufs.m2l, total * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "FMM list download");
        long o = 0;
        for (int a = 0; a < nn; ++a) {  // node order, each node's entries in walk order
            const int c = cnt[(size_t)which * nn + a], b = off[(size_t)which * nn + a];
            std::memcpy(grouped.data() + o, all.data() + b, (size_t)c * sizeof(int));
            o += c;
        }
        if (which == 1)  // P2P entries hold the source leaf's first body: back to node ids
            for (long q = 0; q < total; ++q) grouped[q] = h->leaves[grouped[q] / leaf];
        e = hipMemcpyAsync(dst, grouped.data(), total * sizeof(int), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "FMM list upload");
    }
    return NBODY_OK;
}

void fmm_release()
{
    std::lock_guard<std::mutex> lf(g_fmm_mu);
    free_plan(g_plan);
    free_bufs(g_bufs);
}

}  // namespace nbi
