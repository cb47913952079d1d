// Multi-level fast multipole method on the ORB nodes (gfx950).
//
// Section VI names the fast multipole method (its reference [20]) as the O(N)
// successor of the tree code.  Built here from the tree code's pieces: the
// ORB nodes with their FP64 moments, boxes and quadrupole records
// (tree.hip), the quadrupole cell's evaluation at a body and its M2L into a
// third-order local expansion (tree_shared.h), and the FP32 pair code of the
// direct sum (pair.h).  Definitions shared with the FP64 oracle (every node's
// lists are equal to the oracle's as sets):
// * MAC: target node A and source node B interact through M2L iff they share
//   no body and diag2_A + diag2_B < theta^2 |com_A - com_B|^2 (FP64).
// * Dual-tree traversal from (root, root): MAC -> B joins A's M2L list; A a
//   leaf and B accepted by the tree code's opening test against A's box
//   (diag2_B < theta^2 D2, D2 the squared distance from com_B to the box) ->
//   B joins A's M2P list; two leaves -> B joins A's P2P list; B a leaf, or A
//   an inner node with diag2_A >= diag2_B -> the pair passes to both
//   children of A; otherwise the pair is replaced by (A, B.left),
//   (A, B.right).
// * A node's total local expansion = its own M2L sum + its parent's total
//   re-expanded about its centre of mass (exact for a cubic); every body of
//   a leaf evaluates its leaf's expansion, its M2P cells as quadrupole cells
//   and its P2P source leaves body by body without the self pair.
//
// Device schedule:
// * Traversal, top-down by node depth.  For a target node A the pairs (A, .)
//   of the recursion are those inherited from its parent (the parent's
//   pass-down list) closed under source splits: one wave per node pops up to
//   64 pending sources per step from an LDS stack, one per lane, and
//   classifies them (ballot ranks give every output a fixed position); at
//   the deep depths one wave walks two sibling nodes, gathering each source
//   once for both.  Each depth runs one walk that writes every node's lists into slots of a
//   per-depth capacity; when that layout would take more than its memory
//   budget, each depth instead runs a count walk, a two-kernel scan (block
//   sums, then offsets) and a fill walk into compact lists.  Writes are
//   bounds-checked and an overflow flag makes the host resize (from the
//   exact counts) and run again.
// * M2L: one wave per node, one source cell per lane, the twenty
//   coefficients summed over the wave in a fixed butterfly (FP32).
// * L2L: one thread per node, depth by depth, in FP64.
// * Leaves: one wave per leaf.  Each lane holds up to 8 of the leaf's
//   targets in registers and takes one source body (P2P) or cell (M2P) at a
//   time, so one load serves up to 8 pairs.  The lanes' FP32 partial sums are
//   folded by the precision mode in lane order through LDS, then each target
//   adds its leaf's expansion in FP64.
#include <algorithm>
#include <array>
#include <cstdlib>
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

// List kinds; per-node counts and offsets are stored [kind][nn].
constexpr int kM2L = 0, kP2P = 1, kM2P = 2, kPass = 3, kKinds = 4;
// tot: [0] the overflow flag; for the three interaction lists the running
// total before depth d at tot_at(kind, d); the pass-down total of depth d at
// tot_at(kPass, d).
constexpr int kRunStride = kFmmStack + 1;
constexpr int kTotWords = 1 + kKinds * kRunStride;
__host__ __device__ constexpr int tot_at(int kind, int d) { return 1 + kind * kRunStride + d; }

constexpr int kScanBlock = 1024;  // positions per scan block (256 threads x 4)

struct FmmDev {
    const int4 *node;
    const double4 *comd;
    const float4 *lo, *hi;
    const float4 *qr;
    const int *parent;
    int nn;
    int *cnt;   // [kKinds][nn] counts per node
    int *lcnt;  // [kKinds][nn] the same counts at each node's position in depth order
    int *off;   // [kKinds][nn] offsets (global; pass-down: in the depth's buffer)
    int *m2l;   // source node ids
    int *p2p;   // the first body of each source leaf
    int *m2p;   // source node ids
    int *pass0, *pass1;
    long cap_m2l, cap_p2p, cap_m2p, cap_pass;
    long *bsum;               // [blocks][kKinds] scan block sums
    unsigned long long *tot;  // see tot_at
    float *own;               // [nn][20] own M2L sums
    double *loc;              // [nn][20] total expansions
};

__device__ __forceinline__ long cap_of(const FmmDev &F, int kind)
{
    return kind == kM2L ? F.cap_m2l : (kind == kP2P ? F.cap_p2p : (kind == kM2P ? F.cap_m2p : F.cap_pass));
}

__device__ __forceinline__ bool fmm_overlap(int4 a, int4 b) { return a.x < b.y && b.x < a.y; }

__device__ __forceinline__ unsigned fmm_rank(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Bounds-checked store of one list entry: the entry's index in its list is
// done + its rank among the lanes of mask, stored at base + index if the
// index is below cap (the list's room); returns false when it does not fit.
__device__ __forceinline__ bool put_entry(int *list, long base, long done, long cap, unsigned long long mask,
                                          int value)
{
    const long q = done + (long)fmm_rank(mask);
    if (q >= cap) return false;
    list[base + q] = value;
    return true;
}

// Walk passes.  kWalkCount counts every list of every node; kWalkFill writes
// them at the offsets the scan derived from the counts; kWalkSlot writes
// them, in one pass, into per-node slots of a per-depth capacity (and
// records the exact counts, so that slots too small can be resized).
enum { kWalkCount = 0, kWalkFill = 1, kWalkSlot = 2 };

// Slot layout of one depth: list kind k of the node at position t of the
// depth starts at base[k] + t * cap[k] (the pass-down list in the depth's
// ping-pong buffer); prev_pass is the previous depth's pass-down capacity.
struct SlotDepth {
    long base[kKinds];
    int cap[kKinds];
    int prev_pass;
};

// One wave per target node of one depth: the walk of its inherited
// sources.  The pending sources sit on an LDS stack; each step pops up to 64
// of them (one per lane) and classifies each: M2L, M2P, P2P, pass-down (to
// both children of A) or split (both children of B pushed).  Ballot ranks
// keep every output in a fixed order, so every pass produces the same lists.
template <int WMODE>
__global__ __launch_bounds__(64) void k_fmm_walk(FmmDev F, const int *__restrict__ ids, int first, int count,
                                                 int parity, double theta2, SlotDepth sd)
{
    constexpr bool FILL = WMODE != kWalkCount;
    __shared__ int stk[kWalkStack];
    const int lane = threadIdx.x;
    const int t = blockIdx.x;
    if (t >= count) return;
    const int A = ids[t];
    const int4 na = F.node[A];
    const double4 ca = F.comd[A];
    const bool aleaf = na.z < 0;
    double bx0 = 0.0, by0 = 0.0, bz0 = 0.0, bx1 = 0.0, by1 = 0.0, bz1 = 0.0;  // A's box (M2P test)
    if (aleaf) {
        const float4 l = F.lo[A], h = F.hi[A];
        bx0 = l.x;
        by0 = l.y;
        bz0 = l.z;
        bx1 = h.x;
        by1 = h.y;
        bz1 = h.z;
    }
    const int nn = F.nn;
    const int *in = nullptr;
    int nin = 1;
    if (A != 0) {
        const int P = F.parent[A];
        nin = F.cnt[kPass * nn + P];
        const long base = F.off[kPass * nn + P];
        if (WMODE == kWalkSlot) nin = min(nin, sd.prev_pass);  // the parent's slot overflowed
        if (base + nin > F.cap_pass) nin = (int)max(0L, F.cap_pass - base);  // the parent's depth overflowed
        in = (parity ? F.pass0 : F.pass1) + base;  // the previous depth's buffer
    }
    int *pass_out = parity ? F.pass1 : F.pass0;
    long om = 0, op = 0, oc = 0, oq = 0;
    // room of each list: the slot in the one-pass layout, else all of the buffer
    long rm = F.cap_m2l, rp = F.cap_p2p, rc = F.cap_m2p, rq = F.cap_pass;
    if (WMODE == kWalkSlot) {
        om = sd.base[kM2L] + (long)t * sd.cap[kM2L];
        op = sd.base[kP2P] + (long)t * sd.cap[kP2P];
        oc = sd.base[kM2P] + (long)t * sd.cap[kM2P];
        oq = sd.base[kPass] + (long)t * sd.cap[kPass];
        rm = sd.cap[kM2L];
        rp = sd.cap[kP2P];
        rc = sd.cap[kM2P];
        rq = sd.cap[kPass];
    } else if (FILL) {
        om = F.off[kM2L * nn + A];
        op = F.off[kP2P * nn + A];
        oc = F.off[kM2P * nn + A];
        oq = F.off[kPass * nn + A];
        rm -= om;  // offsets are global: the room is the rest of the buffer
        rp -= op;
        rc -= oc;
        rq -= oq;
    }
    int cm = 0, cp = 0, cc = 0, cq = 0, top = 0, next = 0;
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
        bool m2l = false, m2p = false, p2p = false, pass = false, split = false;
        int4 nb = make_int4(0, 0, -1, -1);
        if (act) {
            nb = F.node[B];
            const double4 cb = F.comd[B];
            const bool apart = !fmm_overlap(na, nb);
            if (apart) {
                const double dx = ca.x - cb.x, dy = ca.y - cb.y, dz = ca.z - cb.z;
                const double dist2 = (dx * dx + dy * dy) + dz * dz;
                m2l = ca.w + cb.w < theta2 * dist2;
            }
            if (!m2l && aleaf && apart) {
                const double gx = box_gap(cb.x, bx0, bx1);
                const double gy = box_gap(cb.y, by0, by1);
                const double gz = box_gap(cb.z, bz0, bz1);
                const double D2 = (gx * gx + gy * gy) + gz * gz;
                m2p = cb.w < theta2 * D2;
            }
            if (!m2l && !m2p) {
                const bool bleaf = nb.z < 0;
                if (aleaf && bleaf)
                    p2p = true;
                else if (bleaf || (!aleaf && ca.w >= cb.w))
                    pass = true;
                else
                    split = true;
            }
        }
        const unsigned long long mm = __ballot(m2l), mc = __ballot(m2p), mp = __ballot(p2p), mq = __ballot(pass),
                                 ms = __ballot(split);
        if (FILL) {
            if (m2l && !put_entry(F.m2l, om, cm, rm, mm, B)) bad = true;
            if (m2p && !put_entry(F.m2p, oc, cc, rc, mc, B)) bad = true;
            if (p2p && !put_entry(F.p2p, op, cp, rp, mp, nb.x)) bad = true;  // a leaf as its first body
            if (pass && !put_entry(pass_out, oq, cq, rq, mq, B)) bad = true;
        }
        cm += __popcll(mm);
        cc += __popcll(mc);
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
    if (WMODE != kWalkFill && lane == 0) {
        const int c4[kKinds] = {cm, cp, cc, cq};
        const long o4[kKinds] = {om, op, oc, oq};
#pragma unroll
        for (int q = 0; q < kKinds; ++q) {
            F.cnt[q * nn + A] = c4[q];
            if (WMODE == kWalkCount)
                F.lcnt[q * nn + first + t] = c4[q];
            else
                F.off[q * nn + A] = (int)o4[q];
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&F.tot[0], 1ull);
}

// TPW target nodes per wave: positions TPW b .. TPW b + TPW - 1 of
// one depth.  Below the root every depth holds whole sibling pairs, adjacent
// in preorder, so targets 2j and 2j + 1 are the children of one parent and
// inherit the same list; each distinct inherited list is loaded once.  The
// stack holds the union of the targets' pending sources, each entry tagged
// with the targets that still need it (bit k for target k, in the four high
// bits of the entry; node ids stay below 2^28, which the host checks).  A
// popped source is gathered once and classified for each of its targets by
// the same tests as the one-target walk; it is split (children pushed,
// tagged with the targets that split it) if any target splits it.  Each
// target's lists are written at ballot ranks in pop order, so every pass
// produces the same lists for a target: the same entries as the one-target
// walk's, in another order.
constexpr unsigned kTagShift = 28, kIdMask = (1u << kTagShift) - 1;

template <int WMODE, int TPW>
__global__ __launch_bounds__(64) void k_fmm_walk_multi(FmmDev F, const int *__restrict__ ids, int first, int count,
                                                       int parity, double theta2, SlotDepth sd)
{
    constexpr bool FILL = WMODE != kWalkCount;
    __shared__ unsigned stk[kWalkStack];
    const int lane = threadIdx.x;
    const int nn = F.nn;
    int *pass_out = parity ? F.pass1 : F.pass0;
    const int *pass_in = parity ? F.pass0 : F.pass1;  // the previous depth's buffer
    int tpos[TPW], A[TPW], parent[TPW];
    int4 na[TPW];
    double4 ca[TPW];
    bool aleaf[TPW], live[TPW];
    double b0[TPW][3], b1[TPW][3];  // each target's box (M2P test)
    long o[TPW][kKinds], room[TPW][kKinds];
    int c[TPW][kKinds];
    // inherited lists: segment g is list seg_in[g] of seg_n[g] entries for the targets seg_tag[g]
    const int *seg_in[TPW];
    int seg_n[TPW];
    unsigned seg_tag[TPW];
    int nseg = 0;
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
        tpos[k] = TPW * blockIdx.x + k;
        live[k] = tpos[k] < count;
        A[k] = live[k] ? ids[tpos[k]] : ids[TPW * blockIdx.x];
        na[k] = F.node[A[k]];
        ca[k] = F.comd[A[k]];
        aleaf[k] = na[k].z < 0;
        const float4 l = F.lo[A[k]], h = F.hi[A[k]];
        b0[k][0] = l.x;
        b0[k][1] = l.y;
        b0[k][2] = l.z;
        b1[k][0] = h.x;
        b1[k][1] = h.y;
        b1[k][2] = h.z;
        parent[k] = A[k] == 0 ? -1 : F.parent[A[k]];
#pragma unroll
        for (int q = 0; q < kKinds; ++q) {
            c[k][q] = 0;
            if (WMODE == kWalkSlot) {
                o[k][q] = sd.base[q] + (long)tpos[k] * sd.cap[q];
                room[k][q] = sd.cap[q];
            } else if (FILL) {
                o[k][q] = F.off[q * nn + A[k]];
                room[k][q] = cap_of(F, q) - o[k][q];  // offsets are global: the rest of the buffer
            } else {
                o[k][q] = 0;
                room[k][q] = cap_of(F, q);
            }
        }
        if (!live[k]) continue;
        if (k > 0 && live[k - 1] && parent[k] >= 0 && parent[k] == parent[k - 1]) {
            seg_tag[nseg - 1] |= 1u << k;  // the sibling's list serves both
            continue;
        }
        if (A[k] == 0) {
            seg_in[nseg] = nullptr;
            seg_n[nseg] = 1;
        } else {
            int m = F.cnt[kPass * nn + parent[k]];
            const long base = F.off[kPass * nn + parent[k]];
            if (WMODE == kWalkSlot) m = min(m, sd.prev_pass);  // the parent's slot overflowed
            if (base + m > F.cap_pass) m = (int)max(0L, F.cap_pass - base);  // the parent's depth overflowed
            seg_in[nseg] = pass_in + base;
            seg_n[nseg] = m;
        }
        seg_tag[nseg] = 1u << k;
        ++nseg;
    }
    int seg = 0, next = 0, top = 0;
    bool bad = false;
    for (;;) {
        while (top < 64 && seg < nseg) {  // refill
            const int m = seg_n[seg];
            const int take = min(64, m - next);
            if (take > 0) {
                if (lane < take)
                    stk[top + lane] = (seg_in[seg] ? (unsigned)seg_in[seg][next + lane] : 0u) |
                                      (seg_tag[seg] << kTagShift);
                top += take;
                next += take;
            }
            if (next >= m) {
                ++seg;
                next = 0;
            }
        }
        if (top == 0) break;
        const int kpop = min(64, top);
        top -= kpop;
        __syncthreads();
        const bool act = lane < kpop;
        const unsigned e = act ? stk[top + lane] : 0u;
        __syncthreads();
        int B = (int)(e & kIdMask);
        const unsigned tag = e >> kTagShift;
        if ((unsigned)B >= (unsigned)nn) B = 0;  // only after an overflow upstream
        int4 nb = make_int4(0, 0, -1, -1);
        double4 cb = make_double4(0.0, 0.0, 0.0, 0.0);
        if (act) {
            nb = F.node[B];
            cb = F.comd[B];
        }
        unsigned split_tag = 0;
#pragma unroll
        for (int k = 0; k < TPW; ++k) {
            bool m2l = false, m2p = false, p2p = false, pass = false, split = false;
            if (act && (tag >> k & 1u)) {
                const bool apart = !fmm_overlap(na[k], nb);
                if (apart) {
                    const double dx = ca[k].x - cb.x, dy = ca[k].y - cb.y, dz = ca[k].z - cb.z;
                    const double dist2 = (dx * dx + dy * dy) + dz * dz;
                    m2l = ca[k].w + cb.w < theta2 * dist2;
                }
                if (!m2l && aleaf[k] && apart) {
                    const double gx = box_gap(cb.x, b0[k][0], b1[k][0]);
                    const double gy = box_gap(cb.y, b0[k][1], b1[k][1]);
                    const double gz = box_gap(cb.z, b0[k][2], b1[k][2]);
                    const double D2 = (gx * gx + gy * gy) + gz * gz;
                    m2p = cb.w < theta2 * D2;
                }
                if (!m2l && !m2p) {
                    const bool bleaf = nb.z < 0;
                    if (aleaf[k] && bleaf)
                        p2p = true;
                    else if (bleaf || (!aleaf[k] && ca[k].w >= cb.w))
                        pass = true;
                    else
                        split = true;
                }
            }
            const unsigned long long mm = __ballot(m2l), mc = __ballot(m2p), mp = __ballot(p2p),
                                     mq = __ballot(pass);
            if (FILL) {
                if (m2l && !put_entry(F.m2l, o[k][kM2L], c[k][kM2L], room[k][kM2L], mm, B)) bad = true;
                if (m2p && !put_entry(F.m2p, o[k][kM2P], c[k][kM2P], room[k][kM2P], mc, B)) bad = true;
                if (p2p && !put_entry(F.p2p, o[k][kP2P], c[k][kP2P], room[k][kP2P], mp, nb.x)) bad = true;
                if (pass && !put_entry(pass_out, o[k][kPass], c[k][kPass], room[k][kPass], mq, B)) bad = true;
            }
            c[k][kM2L] += __popcll(mm);
            c[k][kM2P] += __popcll(mc);
            c[k][kP2P] += __popcll(mp);
            c[k][kPass] += __popcll(mq);
            if (split) split_tag |= 1u << k;
        }
        const unsigned long long ms = __ballot(split_tag != 0);
        const int ns = __popcll(ms);
        if (top + 2 * ns > kWalkStack) {  // cannot happen for trees the host admits
            bad = true;
            break;
        }
        if (split_tag) {
            const int q = top + 2 * (int)fmm_rank(ms);
            stk[q] = (unsigned)nb.w | (split_tag << kTagShift);
            stk[q + 1] = (unsigned)nb.z | (split_tag << kTagShift);
        }
        top += 2 * ns;
        __syncthreads();
    }
    if (WMODE != kWalkFill && lane == 0) {
#pragma unroll
        for (int k = 0; k < TPW; ++k) {
            if (!live[k]) continue;
#pragma unroll
            for (int q = 0; q < kKinds; ++q) {
                F.cnt[q * nn + A[k]] = c[k][q];
                if (WMODE == kWalkCount)
                    F.lcnt[q * nn + first + tpos[k]] = c[k][q];
                else
                    F.off[q * nn + A[k]] = (int)o[k][q];
            }
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&F.tot[0], 1ull);
}

// Target nodes per wave at a depth of `count` nodes: the deep depths, with
// enough nodes to fill the chip more than once, walk 2 per wave (half the
// waves, each source gathered once for both); the others 1, for
// parallelism.  Measured at 2^20 (leaf 8, theta 0.5): the depths of 8192 to
// 131072 nodes took 239-1019 us against 311-1141 us with one target per
// wave, and 708-1299 us with 4 per wave from 32768 nodes on.
constexpr int kPairNodes = 8192;
int walk_tpw(int count, int nn)
{
    if (nn > (int)kIdMask) return 1;
    return count >= kPairNodes ? 2 : 1;
}

template <int WMODE>
void launch_walk_depth(int tpw, const FmmDev &F, const int *ids, int first, int count, int parity, double theta2,
                       const SlotDepth &sd, hipStream_t s)
{
    if (tpw == 2)
        hipLaunchKernelGGL((k_fmm_walk_multi<WMODE, 2>), dim3((count + 1) / 2), dim3(64), 0, s, F, ids, first, count,
                           parity, theta2, sd);
    else
        hipLaunchKernelGGL(k_fmm_walk<WMODE>, dim3(count), dim3(64), 0, s, F, ids, first, count, parity, theta2,
                           sd);
}

// Sum over the wave of four values (fixed butterfly).
__device__ __forceinline__ void wave_sum4(long (&s)[kKinds])
{
#pragma unroll
    for (int q = 0; q < kKinds; ++q)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s[q] += __shfl_xor(s[q], o);
}

// Scan, first kernel: the four count sums of each block of kScanBlock
// positions of one depth.
__global__ __launch_bounds__(256) void k_fmm_scan_part(FmmDev F, int first, int count)
{
    __shared__ long red[4][kKinds];
    const int tid = threadIdx.x, b = blockIdx.x, nn = F.nn;
    long s[kKinds] = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < kScanBlock / 256; ++r) {
        const int pos = b * kScanBlock + r * 256 + tid;
        if (pos < count)
#pragma unroll
            for (int q = 0; q < kKinds; ++q) s[q] += F.lcnt[q * nn + first + pos];
    }
    wave_sum4(s);
    if ((tid & 63) == 0)
#pragma unroll
        for (int q = 0; q < kKinds; ++q) red[tid >> 6][q] = s[q];
    __syncthreads();
    if (tid < kKinds) F.bsum[(long)b * kKinds + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// Scan, second kernel: block b adds the sums of the blocks before it to the
// running totals, scans its positions (4 contiguous per thread) and writes
// every node's offsets; the last block stores the totals for the next depth
// and raises the overflow flag when a list passes its capacity.
__global__ __launch_bounds__(256) void k_fmm_scan_fin(FmmDev F, const int *__restrict__ ids, int first, int count,
                                                      int depth, int nblk)
{
    __shared__ long wsum[4][kKinds];
    __shared__ long bbase[kKinds];
    const int tid = threadIdx.x, b = blockIdx.x, nn = F.nn;
    const int lane = tid & 63, wv = tid >> 6;
    if (wv == 0) {
        long s[kKinds] = {0, 0, 0, 0};
        for (int k = lane; k < b; k += 64)
#pragma unroll
            for (int q = 0; q < kKinds; ++q) s[q] += F.bsum[(long)k * kKinds + q];
        wave_sum4(s);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < kKinds; ++q) bbase[q] = (q < kPass ? (long)F.tot[tot_at(q, depth)] : 0L) + s[q];
    }
    const int p0 = b * kScanBlock + 4 * tid;
    int v[4][kKinds];
    long s[kKinds] = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < kKinds; ++q) {
            v[r][q] = p0 + r < count ? F.lcnt[q * nn + first + p0 + r] : 0;
            s[q] += v[r][q];
        }
    long inc[kKinds];
#pragma unroll
    for (int q = 0; q < kKinds; ++q) inc[q] = s[q];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1)
#pragma unroll
        for (int q = 0; q < kKinds; ++q) {
            const long y = __shfl_up(inc[q], d);
            if (lane >= d) inc[q] += y;
        }
    if (lane == 63)
#pragma unroll
        for (int q = 0; q < kKinds; ++q) wsum[wv][q] = inc[q];
    __syncthreads();
    long o[kKinds];
#pragma unroll
    for (int q = 0; q < kKinds; ++q) {
        long pre = bbase[q];
        for (int w = 0; w < wv; ++w) pre += wsum[w][q];
        o[q] = pre + inc[q] - s[q];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (p0 + r >= count) break;
        const int A = ids[p0 + r];
#pragma unroll
        for (int q = 0; q < kKinds; ++q) {
            F.off[q * nn + A] = (int)min(o[q], (long)INT32_MAX);
            o[q] += v[r][q];
        }
    }
    if (b == nblk - 1 && tid < kKinds) {
        const long run = bbase[tid] + (wsum[0][tid] + wsum[1][tid]) + (wsum[2][tid] + wsum[3][tid]);
        F.tot[tid < kPass ? tot_at(tid, depth + 1) : tot_at(kPass, depth)] = (unsigned long long)run;
        if (run > cap_of(F, tid) || run > (long)INT32_MAX) atomicOr(&F.tot[0], 1ull);
    }
}

// M2L: one wave per node.
__global__ __launch_bounds__(256) void k_fmm_m2l(FmmDev F, float eps2)
{
    const int A = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (A >= F.nn) return;
    const int c = F.cnt[kM2L * F.nn + A];
    const long o = F.off[kM2L * F.nn + A];
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

// Leaves: one wave per leaf.  The leaf's P = TPL * NTG target slots (its
// size rounded up to a power of two) form NTG groups of TPL targets; the
// LG = 64 / NTG lanes of a group hold its targets in registers and share its
// sources out, one per lane at a time:
// * P2P: up to 64 entries are read at once (a source leaf is stored as its
//   first body; every leaf holds `leaf` bodies except the last, which ends
//   at n); their (entry, body) pairs are numbered e * 2^lb + body and lane v
//   of a group takes v, v + LG, ... (the entry's first body read from the
//   lane that loaded it).  The leaf's own entry is swept apart with the self
//   pair masked.
// * M2P: lane v takes cells v, v + LG, ... as quadrupole cells.
// * Each lane's FP32 partial sums are folded by the precision mode over the
//   group's lanes in lane order (through LDS); each target then adds its
//   leaf's expansion in FP64 and is stored.
template <int MODE, int TPL, int NTG>
__global__ __launch_bounds__(64) void k_fmm_leaf(const float4 *__restrict__ src, FmmDev F,
                                                 const int *__restrict__ leaves, int nleaves, float eps2_in,
                                                 double G, float4 *__restrict__ out, int n, int leaf, int lb)
{
    constexpr int P = TPL * NTG;
    constexpr int LG = 64 / NTG;
    constexpr int UNR = TPL >= 8 ? 2 : (TPL >= 4 ? 4 : 8);  // source loads in flight per lane
    __shared__ float red[64][4 * TPL + 1];
    __shared__ double fin[P][4];
    const int w = blockIdx.x;
    if (w >= nleaves) return;
    const int lane = threadIdx.x;
    const int g = lane / LG, v = lane % LG;
    const int A = leaves[w];
    const int4 na = F.node[A];
    const int nn = F.nn;
    const float eps2 = lane_copy(eps2_in);
    Targets<float, TPL> T;
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int i = na.x + g * TPL + t;
        const float4 p = src[min(i, na.y - 1)];
        T.x[t] = p.x;
        T.y[t] = p.y;
        T.z[t] = p.z;
        T.i[t] = i;
    }
    Sums<float, TPL> S;
    S.zero();
    // P2P
    const int cp = F.cnt[kP2P * nn + A];
    const long op = F.off[kP2P * nn + A];
    const int cpc = (int)min((long)cp, max(0L, F.cap_p2p - op));
    const int bmask = (1 << lb) - 1;
    bool self = false;
    for (int base = 0; base < cpc; base += 64) {
        const int k = min(64, cpc - base);
        const int mybeg = lane < k ? F.p2p[op + base + lane] : -1;
        self = self || __ballot(mybeg == na.x) != 0ull;
        const int npairs = k << lb;
        for (int q0 = 0; q0 < npairs; q0 += LG * UNR) {
            float4 sv[UNR];
            int sj[UNR];
            bool ok[UNR];
#pragma unroll
            for (int r = 0; r < UNR; ++r) {
                const int q = q0 + r * LG + v;
                const int bg = __shfl(mybeg, (q >> lb) & 63);
                const int body = q & bmask;
                const int len = ((unsigned)bg < (unsigned)n && bg != na.x) ? min(leaf, n - bg) : 0;
                ok[r] = q < npairs && body < len;
                sj[r] = bg + body;
                sv[r] = src[ok[r] ? sj[r] : 0];
            }
#pragma unroll
            for (int r = 0; r < UNR; ++r)
                if (ok[r]) pair_f32<TPL, false>(sv[r], sj[r], T, eps2, S);
        }
    }
    if (self) {  // the leaf's own bodies, without the self pair
        for (int q = v; q < na.y - na.x; q += LG) pair_f32<TPL, true>(src[na.x + q], na.x + q, T, eps2, S);
    }
    // M2P
    const int cc = F.cnt[kM2P * nn + A];
    const long oc = F.off[kM2P * nn + A];
    const int ccc = (int)min((long)cc, max(0L, F.cap_m2p - oc));
    for (int k = v; k < ccc; k += LG) {
        const int B = F.m2p[oc + k];
        if ((unsigned)B < (unsigned)nn) {
            const float4 *rc = F.qr + (long)kQuadRec * B;
            quad_f32<TPL>(rc[0], rc[1], rc[2], T, eps2, S);
        }
    }
    // fold the group's lanes in lane order
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        red[lane][4 * t] = S.ax[t];
        red[lane][4 * t + 1] = S.ay[t];
        red[lane][4 * t + 2] = S.az[t];
        red[lane][4 * t + 3] = S.ph[t];
    }
    __syncthreads();
    for (int s = lane; s < 4 * P; s += 64) {
        const int slot = s >> 2, comp = s & 3;
        const int gg = slot / TPL, t = slot % TPL;
        Run<MODE> R;
        R.zero();
        for (int u = 0; u < LG; ++u) R.fold(red[gg * LG + u][4 * t + comp]);
        fin[slot][comp] = R.get();
    }
    __syncthreads();
    const int i = na.x + lane;
    if (lane >= P || i >= na.y) return;
    double r[4] = {fin[lane][0], fin[lane][1], fin[lane][2], fin[lane][3]};
    // the leaf's expansion at this body, in FP64
    const float4 pt = src[i];
    const double *c = F.loc + 20L * A;
    const double4 ca = F.comd[A];
    const double y[3] = {(double)pt.x - ca.x, (double)pt.y - ca.y, (double)pt.z - ca.z};
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

// Export of one list kind: node a's entries go, in walk order, to
// dst[dst_off[a] ...]; a P2P entry (a leaf's first body) becomes the leaf's
// node id when leaves != nullptr.  One wave per node.
__global__ __launch_bounds__(256) void k_fmm_export(const int *__restrict__ list, const int *__restrict__ cnt,
                                                    const int *__restrict__ off, const long *__restrict__ dst_off,
                                                    int nn, const int *__restrict__ leaves, int leaf,
                                                    int *__restrict__ dst)
{
    const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (a >= nn) return;
    const int c = cnt[a];
    const long o = off[a], t = dst_off[a];
    for (int k = lane; k < c; k += 64) {
        const int v = list[o + k];
        dst[t + k] = leaves ? leaves[v / leaf] : v;
    }
}

__global__ void k_fmm_zero_tot(unsigned long long *tot, int count)
{
    for (int k = threadIdx.x; k < count; k += blockDim.x) tot[k] = 0ull;
}

// ---- host side -----------------------------------------------------------------
struct FmmPlan {
    int n = 0, leaf = 0, dev = -1, nn = 0, depth = 0, max_level = 0;
    std::vector<int> parent, by_depth, depth_off;
    int *d_parent = nullptr, *d_by_depth = nullptr, *d_leaves = nullptr;
};

struct FmmBufs {
    int dev = -1, nn = 0, nblk = 0;
    long cap[kKinds] = {0, 0, 0, 0};
    int *cnt = nullptr, *lcnt = nullptr, *off = nullptr, *list[3] = {nullptr, nullptr, nullptr};
    int *pass0 = nullptr, *pass1 = nullptr;
    long *bsum = nullptr;
    unsigned long long *tot = nullptr;
    float *own = nullptr;
    double *loc = nullptr;
};

// One-pass slot layout for the current plan: per depth, the room of each
// list per node (grown from the exact counts whenever a walk overflowed).
struct SlotPlan {
    int nn = 0, dev = -1;
    std::vector<SlotDepth> depth;
    long total[kKinds] = {0, 0, 0, 0};  // slots per list kind (pass-down: the larger ping-pong half)
    bool disabled = false;              // the layout outgrew its memory budget: count, scan and fill
    long budget = 0;                    // entries the layout may take: an eighth of the device's memory,
                                        // or NBODY_FMM_SLOT_MB MiB if that is less
};

std::mutex g_fmm_mu;
FmmPlan g_plan;
FmmBufs g_bufs;
SlotPlan g_slots;

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
    for (int *l : b.list) (void)hipFree(l);
    (void)hipFree(b.pass0);
    (void)hipFree(b.pass1);
    (void)hipFree(b.bsum);
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
    p.max_level = 0;
    for (int k = 0; k <= p.depth; ++k) {
        p.max_level = std::max(p.max_level, p.depth_off[k + 1]);
        p.depth_off[k + 1] += p.depth_off[k];
    }
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

// Buffers for nn nodes (at most max_level on one depth) with at least the
// given list capacities (M2L, P2P, M2P, pass-down).
int make_bufs(int nn, int max_level, int dev, const long (&want)[kKinds])
{
    FmmBufs &b = g_bufs;
    const int nblk = std::max(1, (max_level + kScanBlock - 1) / kScanBlock);
    bool fits = b.cnt && b.dev == dev && b.nn >= nn && b.nblk >= nblk;
    for (int q = 0; q < kKinds; ++q) fits = fits && b.cap[q] >= want[q];
    if (fits) return NBODY_OK;
    long cap[kKinds];
    for (int q = 0; q < kKinds; ++q) cap[q] = std::max(want[q], b.dev == dev ? b.cap[q] : 0L);
    nn = std::max(nn, b.dev == dev ? b.nn : 0);
    const int nb = std::max(nblk, b.dev == dev ? b.nblk : 0);
    if (b.cnt) {
        (void)hipDeviceSynchronize();
        free_bufs(b);
    }
    const size_t per = kKinds * (size_t)nn * sizeof(int);
    bool ok = hipMalloc(&b.cnt, per) == hipSuccess && hipMalloc(&b.lcnt, per) == hipSuccess &&
              hipMalloc(&b.off, per) == hipSuccess;
    for (int q = 0; q < 3 && ok; ++q) ok = hipMalloc(&b.list[q], (size_t)cap[q] * sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc(&b.pass0, (size_t)cap[kPass] * sizeof(int)) == hipSuccess &&
         hipMalloc(&b.pass1, (size_t)cap[kPass] * sizeof(int)) == hipSuccess &&
         hipMalloc(&b.bsum, (size_t)nb * kKinds * sizeof(long)) == hipSuccess &&
         hipMalloc(&b.tot, kTotWords * sizeof(unsigned long long)) == hipSuccess &&
         hipMalloc(&b.own, 20 * (size_t)nn * sizeof(float)) == hipSuccess &&
         hipMalloc(&b.loc, 20 * (size_t)nn * sizeof(double)) == hipSuccess;
    if (!ok) {
        free_bufs(b);
        set_error("cannot allocate FMM lists (%ld M2L, %ld P2P, %ld M2P, %ld pass-down entries)", cap[kM2L],
                  cap[kP2P], cap[kM2P], cap[kPass]);
        return NBODY_E_NOMEM;
    }
    b.dev = dev;
    b.nn = nn;
    b.nblk = nb;
    for (int q = 0; q < kKinds; ++q) b.cap[q] = cap[q];
    return NBODY_OK;
}

FmmDev dev_view(const TreeDev &d, const FmmPlan &p, const FmmBufs &b)
{
    FmmDev F;
    F.node = d.node;
    F.comd = d.comd;
    F.lo = d.lo;
    F.hi = d.hi;
    F.qr = d.qr;
    F.parent = p.d_parent;
    F.nn = p.nn;
    F.cnt = b.cnt;
    F.lcnt = b.lcnt;
    F.off = b.off;
    F.m2l = b.list[kM2L];
    F.p2p = b.list[kP2P];
    F.m2p = b.list[kM2P];
    F.pass0 = b.pass0;
    F.pass1 = b.pass1;
    F.cap_m2l = b.cap[kM2L];
    F.cap_p2p = b.cap[kP2P];
    F.cap_m2p = b.cap[kM2P];
    F.cap_pass = b.cap[kPass];
    F.bsum = b.bsum;
    F.tot = b.tot;
    F.own = b.own;
    F.loc = b.loc;
    return F;
}

// The traversal: count, scan and fill per depth.
hipError_t launch_traversal(const FmmDev &F, const FmmPlan &p, double theta2, hipStream_t s)
{
    hipLaunchKernelGGL(k_fmm_zero_tot, dim3(1), dim3(256), 0, s, F.tot, kTotWords);
    hipError_t e = hipGetLastError();
    for (int d = 0; d <= p.depth && e == hipSuccess; ++d) {
        const int first = p.depth_off[d], count = p.depth_off[d + 1] - first;
        const int *ids = p.d_by_depth + first;
        const int nblk = (count + kScanBlock - 1) / kScanBlock;
        const int tpw = walk_tpw(count, F.nn);
        launch_walk_depth<kWalkCount>(tpw, F, ids, first, count, d & 1, theta2, SlotDepth{}, s);
        hipLaunchKernelGGL(k_fmm_scan_part, dim3(nblk), dim3(256), 0, s, F, first, count);
        hipLaunchKernelGGL(k_fmm_scan_fin, dim3(nblk), dim3(256), 0, s, F, ids, first, count, d, nblk);
        launch_walk_depth<kWalkFill>(tpw, F, ids, first, count, d & 1, theta2, SlotDepth{}, s);
        e = hipGetLastError();
    }
    return e;
}

// The one-pass traversal: one walk per depth into the slots of g_slots.
hipError_t launch_traversal_slots(const FmmDev &F, const FmmPlan &p, double theta2, hipStream_t s)
{
    hipLaunchKernelGGL(k_fmm_zero_tot, dim3(1), dim3(256), 0, s, F.tot, kTotWords);
    hipError_t e = hipGetLastError();
    for (int d = 0; d <= p.depth && e == hipSuccess; ++d) {
        const int first = p.depth_off[d], count = p.depth_off[d + 1] - first;
        const int tpw = walk_tpw(count, F.nn);
        launch_walk_depth<kWalkSlot>(tpw, F, p.d_by_depth + first, first, count, d & 1, theta2, g_slots.depth[d],
                                     s);
        e = hipGetLastError();
    }
    return e;
}

// Sets the slot layout from per-depth rooms: cap[d][k] entries per node.
void slots_layout(const FmmPlan &p, const std::vector<std::array<long, kKinds>> &cap)
{
    SlotPlan &S = g_slots;
    S.depth.assign(p.depth + 1, SlotDepth{});
    for (int k = 0; k < kKinds; ++k) S.total[k] = 0;
    for (int d = 0; d <= p.depth; ++d) {
        const long cnt = p.depth_off[d + 1] - p.depth_off[d];
        SlotDepth &sd = S.depth[d];
        for (int k = 0; k < kKinds; ++k) {
            sd.cap[k] = (int)cap[d][k];
            if (k == kPass) {
                sd.base[k] = 0;  // each depth starts its ping-pong half at 0
                S.total[k] = std::max(S.total[k], cnt * cap[d][k]);
            } else {
                sd.base[k] = S.total[k];
                S.total[k] += cnt * cap[d][k];
            }
        }
        sd.prev_pass = d > 0 ? (int)cap[d - 1][kPass] : 0;
    }
}

// Rooms for a first attempt: modest guesses where a depth has the nodes a
// list needs (inner nodes pass down, leaves take M2P and P2P), none elsewhere.
void slots_initial(const FmmPlan &p, const HostTree &h)
{
    std::vector<std::array<long, kKinds>> cap(p.depth + 1);
    for (int d = 0; d <= p.depth; ++d) {
        bool inner = false, leafy = false;
        for (int q = p.depth_off[d]; q < p.depth_off[d + 1]; ++q) (h.node[p.by_depth[q]].z < 0 ? leafy : inner) = true;
        cap[d] = {128, leafy ? 512 : 0, leafy ? 64 : 0, inner ? 512 : 0};
    }
    slots_layout(p, cap);
    g_slots.nn = p.nn;
    g_slots.dev = p.dev;
    g_slots.disabled = false;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) total_b = 0;
    g_slots.budget = (long)(total_b / 8 / sizeof(int));
    if (const char *mb = std::getenv("NBODY_FMM_SLOT_MB"))  // a smaller budget, in MiB
        g_slots.budget = std::min(g_slots.budget, std::max(0L, std::atol(mb)) * (1L << 20) / (long)sizeof(int));
}

// Entries the current slot layout needs (both pass-down halves).
long slots_need()
{
    long need = 0;
    for (int k = 0; k < kKinds; ++k) need += (k == kPass ? 2 : 1) * g_slots.total[k];
    return need;
}

// After an overflow: every room becomes at least the largest count of its
// depth (exact up to the first depth whose pass-down lists overflowed) plus
// an eighth.  Returns false when the layout would pass its memory budget.
bool slots_regrow(const FmmPlan &p, const std::vector<int> &cnt, long budget_entries)
{
    const int nn = p.nn;
    std::vector<std::array<long, kKinds>> cap(p.depth + 1);
    long need = 0;
    for (int d = 0; d <= p.depth; ++d) {
        for (int k = 0; k < kKinds; ++k) {
            long mx = 0;
            for (int q = p.depth_off[d]; q < p.depth_off[d + 1]; ++q)
                mx = std::max(mx, (long)cnt[(size_t)k * nn + p.by_depth[q]]);
            const long old = g_slots.depth[d].cap[k];
            cap[d][k] = mx > old ? mx + mx / 8 + 8 : old;
        }
    }
    const auto saved = g_slots.depth;
    long saved_total[kKinds];
    std::copy(g_slots.total, g_slots.total + kKinds, saved_total);
    slots_layout(p, cap);
    for (int k = 0; k < kKinds; ++k) need += (k == kPass ? 2 : 1) * g_slots.total[k];
    bool ok = need <= budget_entries;
    for (int k = 0; k < kKinds; ++k) ok = ok && g_slots.total[k] <= (long)INT32_MAX;
    if (!ok) {  // keep the old layout; the caller falls back to count, scan and fill
        g_slots.depth = saved;
        std::copy(saved_total, saved_total + kKinds, g_slots.total);
    }
    return ok;
}

template <int MODE>
hipError_t launch_leaves_mode(const float4 *pm, const FmmDev &F, const FmmPlan &p, int nleaves, int n, int leaf,
                              float eps2, double G, float4 *out, hipStream_t s)
{
    int lb = 0;
    while ((1 << lb) < leaf) ++lb;
    const dim3 grid(nleaves), blk(64);
#define NB_FMM_LEAF(TPL, NTG)                                                                                  \
    hipLaunchKernelGGL((k_fmm_leaf<MODE, TPL, NTG>), grid, blk, 0, s, pm, F, p.d_leaves, nleaves, eps2, G, out, \
                       n, leaf, lb)
    switch (lb) {
    case 0: NB_FMM_LEAF(1, 1); break;
    case 1: NB_FMM_LEAF(2, 1); break;
    case 2: NB_FMM_LEAF(4, 1); break;
    case 3: NB_FMM_LEAF(8, 1); break;
    case 4: NB_FMM_LEAF(8, 2); break;
    case 5: NB_FMM_LEAF(8, 4); break;
    default: NB_FMM_LEAF(8, 8); break;
    }
#undef NB_FMM_LEAF
    return hipGetLastError();
}

// Final list totals (M2L, P2P, M2P) after the deepest depth.
void list_totals(const unsigned long long *tot, int depth, unsigned long long (&out)[3])
{
    for (int q = 0; q < 3; ++q) out[q] = tot[tot_at(q, depth + 1)];
}

// Runs the traversal until the lists fit their buffers (one stream
// synchronisation per attempt), then, with out != nullptr, the evaluation.
// Called with the tree and FMM locks held.
int fmm_run(const void *pm, int n, int prec, double G, double eps, double theta, int leaf, void *out,
            hipStream_t s, TreeDev &d, const HostTree *&h)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return NBODY_E_HIP;
    }
    if (leaf > 64) {
        set_error("the FMM takes leaves of at most 64 bodies");
        return NBODY_E_INVAL;
    }
    NB_CHECK_RC(tree_quad_prepare(pm, n, leaf, s, d, h));
    NB_CHECK_RC(make_plan(*h, n, leaf, dev, s));
    const FmmPlan &p = g_plan;
    const int nn = p.nn;
    const int nleaves = (int)h->leaves.size();
    long want[kKinds] = {std::max(1024L, 64L * nn), std::max(1024L, 512L * nleaves), std::max(1024L, 16L * nleaves),
                         std::max(1024L, 16L * nn)};
    if (g_bufs.dev == dev)
        for (int q = 0; q < kKinds; ++q) want[q] = std::max(want[q], g_bufs.cap[q]);
    // One pass into per-node slots while the layout fits its budget;
    // otherwise count, scan and fill into compact lists.
    if (g_slots.nn != nn || g_slots.dev != dev || (int)g_slots.depth.size() != p.depth + 1) slots_initial(p, *h);
    bool slots = !g_slots.disabled && slots_need() <= g_slots.budget;
    // A pass-down list that overflowed truncates what the depths below it see,
    // so each attempt makes at least one more depth exact.
    for (int attempt = 0; attempt < p.depth + 16; ++attempt) {
        if (slots)
            for (int q = 0; q < kKinds; ++q) want[q] = std::max(want[q], std::max(1024L, g_slots.total[q]));
        NB_CHECK_RC(make_bufs(nn, p.max_level, dev, want));
        const FmmDev F = dev_view(d, p, g_bufs);
        hipError_t e = slots ? launch_traversal_slots(F, p, theta * theta, s) : launch_traversal(F, p, theta * theta, s);
        if (e != hipSuccess) return hip_fail(e, "FMM traversal");
        unsigned long long tot[kTotWords];
        e = hipMemcpyAsync(tot, g_bufs.tot, sizeof tot, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "FMM list check");
        if (!tot[0]) {  // the lists fit: evaluate
            if (!out) return NBODY_OK;
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
            return e == hipSuccess ? NBODY_OK : hip_fail(e, "FMM kernels");
        }
        if (slots) {  // resize the slots from the exact counts and run again
            std::vector<int> cnt(kKinds * (size_t)nn);
            e = hipMemcpyAsync(cnt.data(), g_bufs.cnt, cnt.size() * sizeof(int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "FMM count download");
            if (!slots_regrow(p, cnt, g_slots.budget)) {
                slots = false;
                g_slots.disabled = true;
            }
            continue;
        }
        // Grow what overflowed and run again.  The totals are exact up to the
        // first depth whose pass-down list overflowed and short beyond it, so
        // every attempt makes at least one more depth exact.
        unsigned long long pass_max = 0, lt[3];
        bool pass_over = false;
        for (int dd = 0; dd <= p.depth; ++dd) {
            pass_max = std::max(pass_max, tot[tot_at(kPass, dd)]);
            pass_over = pass_over || tot[tot_at(kPass, dd)] > (unsigned long long)g_bufs.cap[kPass];
        }
        list_totals(tot, p.depth, lt);
        auto grow = [](long cap, unsigned long long need, bool doubled) {
            long w = std::max(cap, (long)std::min<unsigned long long>(need + need / 4 + 1024, 1ull << 40));
            return doubled ? std::max(w, 2 * cap) : w;
        };
        want[kPass] = grow(g_bufs.cap[kPass], pass_max, pass_over);
        for (int q = 0; q < 3; ++q) want[q] = grow(g_bufs.cap[q], lt[q], false);
        for (int q = 0; q < kKinds; ++q)
            if (want[q] > (long)INT32_MAX) {
                set_error("FMM lists beyond 2^31 entries (M2L %llu, P2P %llu, M2P %llu, pass-down %llu counted so "
                          "far; theta too small for this n and leaf)",
                          lt[0], lt[1], lt[2], pass_max);
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

int fmm_lists(const void *pm, int n, int leaf, double theta, int32_t *const cnt_out[3], int32_t *const ids_out[3],
              const int64_t caps[3], hipStream_t s)
{
    std::lock_guard<std::mutex> lt(tree_mutex());
    std::lock_guard<std::mutex> lf(g_fmm_mu);
    TreeDev d;
    const HostTree *h = nullptr;
    NB_CHECK_RC(fmm_run(pm, n, NBODY_F32, 1.0, 0.0, theta, leaf, nullptr, s, d, h));
    const int nn = g_plan.nn;
    std::vector<int> cnt(kKinds * (size_t)nn), off(kKinds * (size_t)nn);
    hipError_t e = hipMemcpyAsync(cnt.data(), g_bufs.cnt, cnt.size() * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(off.data(), g_bufs.off, off.size() * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "FMM list download");
    long tl[3] = {0, 0, 0};  // list totals (M2L, P2P, M2P) from the per-node counts
    for (int q = 0; q < 3; ++q)
        for (int a = 0; a < nn; ++a) tl[q] += cnt[(size_t)q * nn + a];
    // the public order is (M2L, M2P, P2P)
    const int kind_of[3] = {kM2L, kM2P, kP2P};
    for (int w = 0; w < 3; ++w) {
        e = hipMemcpyAsync(cnt_out[w], cnt.data() + (size_t)kind_of[w] * nn, nn * sizeof(int), hipMemcpyHostToDevice,
                           s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "FMM count upload");
    }
    for (int w = 0; w < 3; ++w) {
        const int q = kind_of[w];
        int32_t *dst = ids_out[w];
        if (!dst) continue;
        const long total = (long)tl[q];
        if (total > caps[w]) {
            static const char *names[3] = {"M2L", "M2P", "P2P"};
            set_error("%s list of %ld entries exceeds the capacity %lld", names[w], total, (long long)caps[w]);
            return NBODY_E_INVAL;
        }
        std::vector<long> dst_off(nn);
        long o = 0;
        for (int a = 0; a < nn; ++a) {  // node order, each node's entries in walk order
            dst_off[a] = o;
            o += cnt[(size_t)q * nn + a];
        }
        long *d_off = nullptr;
        e = hipMalloc(&d_off, (size_t)nn * sizeof(long));
        if (e == hipSuccess) e = hipMemcpyAsync(d_off, dst_off.data(), (size_t)nn * sizeof(long), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_fmm_export, dim3((nn + 3) / 4), dim3(256), 0, s, g_bufs.list[q],
                               g_bufs.cnt + (size_t)q * nn, g_bufs.off + (size_t)q * nn, (const long *)d_off, nn,
                               q == kP2P ? (const int *)g_plan.d_leaves : nullptr, leaf, dst);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(d_off);
        if (e != hipSuccess) return hip_fail(e, "FMM list export");
    }
    return NBODY_OK;
}

void fmm_release()
{
    std::lock_guard<std::mutex> lf(g_fmm_mu);
    free_plan(g_plan);
    free_bufs(g_bufs);
    g_slots = SlotPlan();
}

}  // namespace nbi
