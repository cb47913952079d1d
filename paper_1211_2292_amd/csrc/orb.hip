// Orthogonal Recursive Bisection order on the device (gfx950).
//
// The paper (Section IV.B) divides space into non-overlapping sub-spaces
// holding about equal numbers of bodies by recursive bisection.  Here the
// recursion is carried down to leaves of at most `leaf` bodies and used as a
// body ordering on one device.  The split rule (see nbody.h) depends only on
// the set of bodies in a segment, and the segment sizes depend only on
// (n, leaf), so:
//   * the host computes the whole segment tree (sizes and left counts) once;
//   * the device only decides which bodies go left, by finding the k-th
//     smallest 64-bit key (total-order FP32 coordinate, original index) of
//     each segment exactly, with an 8-bit-digit radix select;
//   * bodies may be partitioned in any order (integer atomics hand out
//     slots), because every later decision depends on set membership only and
//     every leaf is finally sorted by original index.
// Phase A handles segments larger than kSmall bodies with multi-workgroup
// kernels over fixed-size chunks; phase B finishes every remaining segment
// (at most max(kSmall, leaf) <= kMaxBlockSeg bodies) inside one workgroup,
// in LDS, and writes the final order.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace nbi {

constexpr int kSmall = 2048;        // phase A splits segments larger than this
constexpr int kMaxBlockSeg = 4096;  // largest segment phase B accepts (and max leaf)
constexpr int kChunk = 4096;        // elements per phase-A workgroup
constexpr int kOrbBlock = 256;

namespace {

__device__ __forceinline__ uint32_t tkey(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float untkey(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k ^ 0x80000000u) : ~k);
}

// axis of largest FP32 extent fl32(max - min), ties to the lowest axis
__device__ __forceinline__ int pick_axis(const uint32_t *bb)
{
    float ext[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) ext[a] = untkey(bb[3 + a]) - untkey(bb[a]);
    int axis = 0;
    if (ext[1] > ext[axis]) axis = 1;
    if (ext[2] > ext[axis]) axis = 2;
    return axis;
}

__device__ __forceinline__ uint64_t body_key(const float *__restrict__ xyz, int n, int axis, int b)
{
    return ((uint64_t)tkey(xyz[(size_t)axis * n + b]) << 32) | (uint32_t)b;
}

template <typename V>
__global__ __launch_bounds__(kOrbBlock) void k_orb_coords(const V *__restrict__ pm, int n,
                                                          float *__restrict__ xyz,
                                                          int32_t *__restrict__ cur)
{
    const int i = blockIdx.x * kOrbBlock + threadIdx.x;
    if (i >= n) return;
    const V p = pm[i];
    xyz[i] = (float)p.x;
    xyz[(size_t)n + i] = (float)p.y;
    xyz[2 * (size_t)n + i] = (float)p.z;
    cur[i] = i;
}

// Per-segment state of one phase-A level.
struct SegState {
    uint32_t bb[6];    // min keys x,y,z then max keys x,y,z
    int axis;
    int krem;          // rank still to find inside the current prefix
    uint64_t prefix;   // digits of the k-th key found so far
    uint32_t lcnt, rcnt;
};

// seg table: (start, size, k) per segment; chunk table: (seg, begin, end)
__global__ __launch_bounds__(kOrbBlock) void k_orb_init(const int3 *__restrict__ segs, int nseg,
                                                        SegState *__restrict__ st,
                                                        uint32_t *__restrict__ hist)
{
    const int s = blockIdx.x;
    if (s >= nseg) return;
    if (threadIdx.x == 0) {
        SegState z;
        for (int a = 0; a < 3; ++a) {
            z.bb[a] = 0xFFFFFFFFu;
            z.bb[3 + a] = 0u;
        }
        z.axis = 0;
        z.krem = segs[s].z;
        z.prefix = 0;
        z.lcnt = z.rcnt = 0;
        st[s] = z;
    }
    hist[(size_t)s * 256 + threadIdx.x] = 0u;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

__global__ __launch_bounds__(kOrbBlock) void k_orb_bbox(const int3 *__restrict__ chunks,
                                                        const float *__restrict__ xyz, int n,
                                                        const int32_t *__restrict__ cur,
                                                        SegState *__restrict__ st)
{
    const int3 c = chunks[blockIdx.x];
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    for (int p = c.y + threadIdx.x; p < c.z; p += kOrbBlock) {
        const int b = cur[p];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint32_t k = tkey(xyz[(size_t)a * n + b]);
            lo[a] = min(lo[a], k);
            hi[a] = max(hi[a], k);
        }
    }
    __shared__ uint32_t red[kOrbBlock / 64][6];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
    }
    if (lane == 0)
        for (int a = 0; a < 3; ++a) {
            red[w][a] = lo[a];
            red[w][3 + a] = hi[a];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        uint32_t v = red[0][threadIdx.x];
        for (int k = 1; k < kOrbBlock / 64; ++k)
            v = threadIdx.x < 3 ? min(v, red[k][threadIdx.x]) : max(v, red[k][threadIdx.x]);
        if (threadIdx.x < 3)
            atomicMin(&st[c.x].bb[threadIdx.x], v);
        else
            atomicMax(&st[c.x].bb[threadIdx.x], v);
    }
}

__global__ __launch_bounds__(kOrbBlock) void k_orb_axis(int nseg, SegState *__restrict__ st)
{
    const int s = blockIdx.x * kOrbBlock + threadIdx.x;
    if (s < nseg) st[s].axis = pick_axis(st[s].bb);
}

// Histogram of digit `round` (8 bits, most significant first) of the keys
// that share the prefix found so far.
__global__ __launch_bounds__(kOrbBlock) void k_orb_hist(const int3 *__restrict__ chunks,
                                                        const float *__restrict__ xyz, int n,
                                                        const int32_t *__restrict__ cur,
                                                        const SegState *__restrict__ st,
                                                        uint32_t *__restrict__ hist, int round)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int3 c = chunks[blockIdx.x];
    const int axis = st[c.x].axis;
    const uint64_t prefix = st[c.x].prefix;
    const int shift = 56 - 8 * round;
    for (int p = c.y + threadIdx.x; p < c.z; p += kOrbBlock) {
        const uint64_t key = body_key(xyz, n, axis, cur[p]);
        if (round == 0 || (key >> (shift + 8)) == prefix) atomicAdd(&h[(key >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    const uint32_t v = h[threadIdx.x];
    if (v) atomicAdd(&hist[(size_t)c.x * 256 + threadIdx.x], v);
}

// One wave per segment: the bin holding rank krem, then clear the bins.
__global__ __launch_bounds__(64) void k_orb_pick(int nseg, SegState *__restrict__ st,
                                                 uint32_t *__restrict__ hist)
{
    const int s = blockIdx.x;
    if (s >= nseg) return;
    const int lane = threadIdx.x;
    uint32_t *hs = hist + (size_t)s * 256;
    uint32_t c[4], tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        c[q] = hs[4 * lane + q];
        tot += c[q];
    }
    // inclusive scan of the per-lane totals across the wave
    uint32_t inc = tot;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)inc, o);
        if (lane >= o) inc += y;
    }
    const uint32_t before = inc - tot;
    const uint32_t krem = (uint32_t)st[s].krem;
    // the lane whose range contains rank krem (1-based) decides
    if (before < krem && krem <= inc) {
        uint32_t acc = before;
        int bin = 4 * lane;
        for (int q = 0; q < 4; ++q) {
            if (acc + c[q] >= krem) {
                bin = 4 * lane + q;
                break;
            }
            acc += c[q];
        }
        st[s].prefix = (st[s].prefix << 8) | (uint64_t)bin;
        st[s].krem = (int)(krem - acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) hs[4 * lane + q] = 0u;
}

// Keys <= the k-th key go left.  Slots are handed out per workgroup with one
// atomic per side; the order inside a side is irrelevant to the result.
__global__ __launch_bounds__(kOrbBlock) void k_orb_partition(const int3 *__restrict__ chunks,
                                                             const int3 *__restrict__ segs,
                                                             const float *__restrict__ xyz, int n,
                                                             const int32_t *__restrict__ cur,
                                                             SegState *__restrict__ st,
                                                             int32_t *__restrict__ tmp)
{
    __shared__ uint32_t nl, nr, bl, br;
    if (threadIdx.x == 0) nl = nr = 0u;
    __syncthreads();
    const int3 c = chunks[blockIdx.x];
    const int axis = st[c.x].axis;
    const uint64_t kth = st[c.x].prefix;
    // count
    for (int p = c.y + threadIdx.x; p < c.z; p += kOrbBlock) {
        const uint64_t key = body_key(xyz, n, axis, cur[p]);
        if (key <= kth)
            atomicAdd(&nl, 1u);
        else
            atomicAdd(&nr, 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bl = atomicAdd(&st[c.x].lcnt, nl);
        br = atomicAdd(&st[c.x].rcnt, nr);
        nl = nr = 0u;
    }
    __syncthreads();
    const int3 sg = segs[c.x];
    // exactly k keys are <= the k-th key; the guards only keep a violated
    // precondition (non-finite coordinates) inside the segment
    for (int p = c.y + threadIdx.x; p < c.z; p += kOrbBlock) {
        const int b = cur[p];
        const uint64_t key = body_key(xyz, n, axis, b);
        if (key <= kth) {
            const uint32_t q = bl + atomicAdd(&nl, 1u);
            if (q < (uint32_t)sg.z) tmp[sg.x + q] = b;
        } else {
            const uint32_t q = br + atomicAdd(&nr, 1u);
            if (q < (uint32_t)(sg.y - sg.z)) tmp[sg.x + sg.z + q] = b;
        }
    }
}

__global__ __launch_bounds__(kOrbBlock) void k_orb_copyback(const int3 *__restrict__ chunks,
                                                            const int32_t *__restrict__ tmp,
                                                            int32_t *__restrict__ cur)
{
    const int3 c = chunks[blockIdx.x];
    for (int p = c.y + threadIdx.x; p < c.z; p += kOrbBlock) cur[p] = tmp[p];
}

// ---- phase B: one workgroup finishes one segment in LDS --------------------
__device__ __forceinline__ uint32_t block_reduce_u32(uint32_t v, bool is_min, uint32_t *scratch)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = is_min ? wave_min(v) : wave_max(v);
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    uint32_t r = scratch[0];
    for (int k = 1; k < kOrbBlock / 64; ++k) r = is_min ? min(r, scratch[k]) : max(r, scratch[k]);
    return r;
}

// Inclusive sum over the workgroup's threads (one 256-thread workgroup):
// within each wave by shuffles, then the totals of the waves before it.
__device__ __forceinline__ uint32_t block_incl_scan_u32(uint32_t v, uint32_t *scratch)
{
    static_assert(kOrbBlock == 256, "one bin per thread");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)v, o);
        if (lane >= o) v += y;
    }
    __syncthreads();
    if (lane == 63) scratch[w] = v;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before += scratch[k];
    return v + before;
}

// Finishes the recursion of a node of at most 64 bodies (positions
// [lo, lo + m) of idx) with one wave, one position per lane, every node of a
// level split at once.  keys: per-wave LDS of 3 x 64 total-order keys.  The
// k smallest keys of a node are found by ranking (keys and indices are
// distinct), then each leaf is ordered by original index.
constexpr int kWaveSeg = 64;

__device__ void orb_wave(int32_t *idx, uint32_t (*keys)[kWaveSeg], int lo, int m, int leaf,
                         const float *__restrict__ xyz, int n, int lane)
{
    int b = lane < m ? idx[lo + lane] : -1;
    uint32_t kx = 0, ky = 0, kz = 0;
    if (lane < m) {
        kx = tkey(xyz[b]);
        ky = tkey(xyz[(size_t)n + b]);
        kz = tkey(xyz[2 * (size_t)n + b]);
    }
    int slo = 0, sm = m;  // the node holding this lane's position (relative to lo)
    for (;;) {
        const bool split = lane < m && sm > leaf;
        if (!__any(split)) break;
        if (lane < m) {
            keys[0][lane] = kx;
            keys[1][lane] = ky;
            keys[2][lane] = kz;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int pos = lane;
        int k = sm;
        if (split) {
            uint32_t bb[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
            for (int f = slo; f < slo + sm; ++f)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const uint32_t v = keys[a][f];
                    bb[a] = min(bb[a], v);
                    bb[3 + a] = max(bb[3 + a], v);
                }
            const int axis = pick_axis(bb);
            const uint32_t mine = axis == 0 ? kx : (axis == 1 ? ky : kz);
            int r = 0;
            for (int f = slo; f < slo + sm; ++f) {
                const uint32_t v = keys[axis][f];
                const int bf = idx[lo + f];
                r += (v < mine) || (v == mine && bf < b);
            }
            pos = slo + r;
            const int L = (sm + leaf - 1) / leaf;
            k = min(sm, leaf * ((L + 1) / 2));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < m) {
            idx[lo + pos] = b;
            keys[0][pos] = kx;
            keys[1][pos] = ky;
            keys[2][pos] = kz;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < m) {
            b = idx[lo + lane];
            kx = keys[0][lane];
            ky = keys[1][lane];
            kz = keys[2][lane];
            if (split) {
                if (lane - slo < k) {
                    sm = k;
                } else {
                    slo += k;
                    sm -= k;
                }
            }
        }
    }
    // leaves: ascending original index
    int r = 0;
    if (lane < m)
        for (int f = slo; f < slo + sm; ++f) r += idx[lo + f] < b;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < m) idx[lo + slo + r] = b;
}

__global__ __launch_bounds__(kOrbBlock) void k_orb_block(const int2 *__restrict__ segs,
                                                         const float *__restrict__ xyz, int n,
                                                         const int32_t *__restrict__ cur, int leaf,
                                                         int32_t *__restrict__ perm)
{
    __shared__ int32_t idx[kMaxBlockSeg];
    __shared__ int32_t tmp[kMaxBlockSeg];
    __shared__ uint32_t akey[kMaxBlockSeg];  // the current node's keys along its split axis
    __shared__ uint32_t h[256];
    __shared__ uint32_t red[kOrbBlock / 64];
    __shared__ uint32_t wl[kOrbBlock / 64], wr[kOrbBlock / 64];
    __shared__ uint64_t kth_s;
    __shared__ uint32_t krem_s;
    constexpr int kMaxTask = kMaxBlockSeg / kWaveSeg * 2 + 2;
    __shared__ int2 task[kMaxTask];
    __shared__ uint32_t wkeys[kOrbBlock / 64][3][kWaveSeg];
    const int2 sg = segs[blockIdx.x];
    const int start = sg.x, size = sg.y;
    for (int e = threadIdx.x; e < size; e += kOrbBlock) idx[e] = cur[start + e];
    __syncthreads();
    int ntask = 0;  // same value in every thread: the loop below is uniform
    int stk_lo[24], stk_m[24], sp = 0;
    stk_lo[0] = 0;
    stk_m[0] = size;
    sp = 1;
    while (sp > 0) {
        --sp;
        const int lo = stk_lo[sp], m = stk_m[sp];
        if (m <= kWaveSeg && ntask < kMaxTask) {
            // finished by one wave below, all small nodes in parallel (past
            // the list's capacity the block-wide path below takes them)
            if (threadIdx.x == 0) task[ntask] = make_int2(lo, m);
            ++ntask;
            continue;
        }
        if (m <= leaf) {
            // leaf: ascending original index (rank of each element; distinct)
            for (int e = threadIdx.x; e < m; e += kOrbBlock) {
                const int v = idx[lo + e];
                int r = 0;
                for (int f = 0; f < m; ++f) r += idx[lo + f] < v;
                tmp[lo + r] = v;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < m; e += kOrbBlock) idx[lo + e] = tmp[lo + e];
            __syncthreads();
            continue;
        }
        // bounding box and axis
        uint32_t bb[6];
        for (int a = 0; a < 3; ++a) {
            uint32_t mn = 0xFFFFFFFFu, mx = 0u;
            for (int e = threadIdx.x; e < m; e += kOrbBlock) {
                const uint32_t k = tkey(xyz[(size_t)a * n + idx[lo + e]]);
                mn = min(mn, k);
                mx = max(mx, k);
            }
            bb[a] = block_reduce_u32(mn, true, red);
            bb[3 + a] = block_reduce_u32(mx, false, red);
        }
        const int axis = pick_axis(bb);
        const int L = (m + leaf - 1) / leaf;
        const int k = min(m, leaf * ((L + 1) / 2));
        // the split axis's keys, gathered once for the 8 rounds and the partition
        for (int e = threadIdx.x; e < m; e += kOrbBlock) akey[e] = tkey(xyz[(size_t)axis * n + idx[lo + e]]);
        // radix select of the k-th smallest key
        if (threadIdx.x == 0) {
            kth_s = 0;
            krem_s = (uint32_t)k;
        }
        for (int round = 0; round < 8; ++round) {
            __syncthreads();
            h[threadIdx.x] = 0u;
            const uint64_t prefix = kth_s;
            const uint32_t kr = krem_s;
            __syncthreads();
            const int shift = 56 - 8 * round;
            for (int e = threadIdx.x; e < m; e += kOrbBlock) {
                const uint64_t key = ((uint64_t)akey[e] << 32) | (uint32_t)idx[lo + e];
                if (round == 0 || (key >> (shift + 8)) == prefix) atomicAdd(&h[(key >> shift) & 0xFF], 1u);
            }
            __syncthreads();
            // the bin holding rank kr (1-based): the one thread whose
            // inclusive sum over the bins reaches kr first decides
            const uint32_t hv = h[threadIdx.x];
            const uint32_t inc = block_incl_scan_u32(hv, red);
            if (inc >= kr && inc - hv < kr) {
                kth_s = (prefix << 8) | (uint64_t)threadIdx.x;
                krem_s = kr - (inc - hv);
            }
        }
        __syncthreads();
        const uint64_t kth = kth_s;
        // partition: keys <= the k-th key go left, in position order within
        // each side (ballot ranks, then the waves before, then the chunks
        // before); the order inside a side does not change the result
        {
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
            int dl = 0, dr = 0;  // entries placed by the chunks before
            for (int e0 = 0; e0 < m; e0 += kOrbBlock) {
                const int e = e0 + threadIdx.x;
                const bool act = e < m;
                const int b = act ? idx[lo + e] : 0;
                const bool left = act && (((uint64_t)akey[act ? e : 0] << 32) | (uint32_t)b) <= kth;
                const bool right = act && !left;
                const unsigned long long bl = __ballot(left), br = __ballot(right);
                if (lane == 0) {
                    wl[w] = (uint32_t)__popcll(bl);
                    wr[w] = (uint32_t)__popcll(br);
                }
                __syncthreads();
                int pl = 0, pr = 0, cl = 0, cr = 0;
                for (int v = 0; v < kOrbBlock / 64; ++v) {
                    if (v < w) {
                        pl += (int)wl[v];
                        pr += (int)wr[v];
                    }
                    cl += (int)wl[v];
                    cr += (int)wr[v];
                }
                const int rl = __builtin_amdgcn_mbcnt_hi((unsigned)(bl >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bl, 0u));
                const int rr = __builtin_amdgcn_mbcnt_hi((unsigned)(br >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)br, 0u));
                if (left) {
                    const int q = dl + pl + rl;
                    if (q < k) tmp[lo + q] = b;
                }
                if (right) {
                    const int q = dr + pr + rr;
                    if (q < m - k) tmp[lo + k + q] = b;
                }
                dl += cl;
                dr += cr;
                __syncthreads();  // wl, wr are reused by the next chunk
            }
        }
        for (int e = threadIdx.x; e < m; e += kOrbBlock) idx[lo + e] = tmp[lo + e];
        __syncthreads();
        // right first so that the left child is processed next
        stk_lo[sp] = lo + k;
        stk_m[sp] = m - k;
        ++sp;
        stk_lo[sp] = lo;
        stk_m[sp] = k;
        ++sp;
    }
    __syncthreads();
    {
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int t = w; t < ntask; t += kOrbBlock / 64) {
            const int2 tk = task[t];
            orb_wave(idx, wkeys[w], tk.x, tk.y, leaf, xyz, n, lane);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < size; e += kOrbBlock) perm[start + e] = idx[e];
}

// ---- host side --------------------------------------------------------------
struct Level {
    std::vector<int3> segs;    // (start, size, k)
    std::vector<int3> chunks;  // (segment, begin, end)
};

void plan_tree(int n, int leaf, std::vector<Level> &levels, std::vector<int2> &finals)
{
    const int cut = std::max(kSmall, leaf);
    std::vector<int2> cur = {make_int2(0, n)};
    while (!cur.empty()) {
        Level lv;
        std::vector<int2> next;
        for (const int2 &s : cur) {
            if (s.y <= cut) {
                finals.push_back(s);
                continue;
            }
            const int L = (s.y + leaf - 1) / leaf;
            const int k = std::min(s.y, leaf * ((L + 1) / 2));
            const int id = (int)lv.segs.size();
            lv.segs.push_back(make_int3(s.x, s.y, k));
            for (int b = s.x; b < s.x + s.y; b += kChunk)
                lv.chunks.push_back(make_int3(id, b, std::min(b + kChunk, s.x + s.y)));
            next.push_back(make_int2(s.x, k));
            next.push_back(make_int2(s.x + k, s.y - k));
        }
        if (!lv.segs.empty()) levels.push_back(std::move(lv));
        cur.swap(next);
    }
}

std::mutex g_orb_mu;
void *g_pinned = nullptr;
size_t g_pinned_size = 0;
// An event belongs to one device: one per device, and the one recorded
// after the last upload (on whichever device) guards the shared buffer.
std::map<int, hipEvent_t> g_pinned_evs;
hipEvent_t g_pinned_last = nullptr;

}  // namespace

int orb_order(const void *pm, int prec, int n, int leaf, int32_t *perm, hipStream_t s)
{
    if (leaf > kMaxBlockSeg) {
        set_error("leaf %d larger than the supported %d", leaf, kMaxBlockSeg);
        return NBODY_E_UNSUPPORTED;
    }
    std::vector<Level> levels;
    std::vector<int2> finals;
    plan_tree(n, leaf, levels, finals);
    // one table upload: per level segs then chunks, then the final segments
    // sections start on 16-byte boundaries (int2 entries need 8-byte alignment)
    std::vector<char> tab;
    auto pad = [&tab]() { tab.resize((tab.size() + 15) & ~size_t(15), 0); };
    std::vector<std::pair<size_t, size_t>> off;  // byte offsets of segs, chunks per level
    size_t maxseg = 1;
    for (const Level &lv : levels) {
        const size_t a = tab.size();
        tab.insert(tab.end(), (const char *)lv.segs.data(), (const char *)(lv.segs.data() + lv.segs.size()));
        pad();
        const size_t b = tab.size();
        tab.insert(tab.end(), (const char *)lv.chunks.data(), (const char *)(lv.chunks.data() + lv.chunks.size()));
        pad();
        off.push_back({a, b});
        maxseg = std::max(maxseg, lv.segs.size());
    }
    const size_t foff = tab.size();
    tab.insert(tab.end(), (const char *)finals.data(), (const char *)(finals.data() + finals.size()));
    pad();
    const size_t nbytes = (size_t)n * 4;
    float *xyz = (float *)scratch(kSlotOrb0, 3 * nbytes);
    int32_t *cur = (int32_t *)scratch(kSlotOrb1, nbytes);
    int32_t *tmp = (int32_t *)scratch(kSlotOrb2, nbytes);
    char *dtab = (char *)scratch(kSlotOrb3, tab.size() + 16);
    char *state = (char *)scratch(kSlotOrb4, maxseg * (sizeof(SegState) + 256 * 4) + 64);
    if (!xyz || !cur || !tmp || !dtab || !state) {
        set_error("cannot allocate ORB scratch");
        return NBODY_E_NOMEM;
    }
    SegState *st = (SegState *)state;
    uint32_t *hist = (uint32_t *)(state + ((maxseg * sizeof(SegState) + 63) & ~size_t(63)));
    {
        // stage the tables through pinned host memory owned by the library;
        // the previous upload must have completed before the buffer is reused
        std::lock_guard<std::mutex> lk(g_orb_mu);
        if (g_pinned_last) (void)hipEventSynchronize(g_pinned_last);
        if (g_pinned_size < tab.size()) {
            if (g_pinned) (void)hipHostFree(g_pinned);
            g_pinned = nullptr;
            g_pinned_size = 0;
            if (hipHostMalloc(&g_pinned, std::max<size_t>(tab.size(), 4096), hipHostMallocDefault) != hipSuccess) {
                set_error("cannot allocate pinned ORB tables");
                return NBODY_E_NOMEM;
            }
            g_pinned_size = std::max<size_t>(tab.size(), 4096);
        }
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) {
            set_error("hipGetDevice failed");
            return NBODY_E_HIP;
        }
        hipEvent_t &ev = g_pinned_evs[dev];
        if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
            set_error("cannot create ORB event");
            return NBODY_E_HIP;
        }
        if (!tab.empty()) {
            std::memcpy(g_pinned, tab.data(), tab.size());
            hipError_t e = hipMemcpyAsync(dtab, g_pinned, tab.size(), hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "ORB table upload");
        }
        hipError_t e = hipEventRecord(ev, s);
        if (e != hipSuccess) return hip_fail(e, "ORB event");
        g_pinned_last = ev;
    }
    const int nb = (n + kOrbBlock - 1) / kOrbBlock;
    if (prec == NBODY_F64)
        hipLaunchKernelGGL(k_orb_coords<double4>, dim3(nb), dim3(kOrbBlock), 0, s, (const double4 *)pm, n, xyz, cur);
    else
        hipLaunchKernelGGL(k_orb_coords<float4>, dim3(nb), dim3(kOrbBlock), 0, s, (const float4 *)pm, n, xyz, cur);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ORB coordinates");
    for (size_t l = 0; l < levels.size(); ++l) {
        const int nseg = (int)levels[l].segs.size(), nch = (int)levels[l].chunks.size();
        const int3 *segs = (const int3 *)(dtab + off[l].first);
        const int3 *chunks = (const int3 *)(dtab + off[l].second);
        hipLaunchKernelGGL(k_orb_init, dim3(nseg), dim3(256), 0, s, segs, nseg, st, hist);
        hipLaunchKernelGGL(k_orb_bbox, dim3(nch), dim3(kOrbBlock), 0, s, chunks, xyz, n, cur, st);
        hipLaunchKernelGGL(k_orb_axis, dim3((nseg + kOrbBlock - 1) / kOrbBlock), dim3(kOrbBlock), 0, s, nseg, st);
        for (int r = 0; r < 8; ++r) {
            hipLaunchKernelGGL(k_orb_hist, dim3(nch), dim3(kOrbBlock), 0, s, chunks, xyz, n, cur, st, hist, r);
            hipLaunchKernelGGL(k_orb_pick, dim3(nseg), dim3(64), 0, s, nseg, st, hist);
        }
        hipLaunchKernelGGL(k_orb_partition, dim3(nch), dim3(kOrbBlock), 0, s, chunks, segs, xyz, n, cur, st, tmp);
        hipLaunchKernelGGL(k_orb_copyback, dim3(nch), dim3(kOrbBlock), 0, s, chunks, tmp, cur);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "ORB level");
    }
    hipLaunchKernelGGL(k_orb_block, dim3((unsigned)finals.size()), dim3(kOrbBlock), 0, s,
                       (const int2 *)(dtab + foff), xyz, n, cur, leaf, perm);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ORB leaves");
    return NBODY_OK;
}

void orb_release()
{
    std::lock_guard<std::mutex> lk(g_orb_mu);
    for (auto &kv : g_pinned_evs) {
        (void)hipEventSynchronize(kv.second);
        (void)hipEventDestroy(kv.second);
    }
    g_pinned_evs.clear();
    g_pinned_last = nullptr;
    if (g_pinned) (void)hipHostFree(g_pinned);
    g_pinned = nullptr;
    g_pinned_size = 0;
}

}  // namespace nbi
