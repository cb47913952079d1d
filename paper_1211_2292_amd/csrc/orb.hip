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
constexpr int kChunkPer = kChunk / kOrbBlock;  // elements per thread of a phase-A workgroup

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

// FP32 coordinates by original index (xyz), and their total-order keys in
// the current order (identity at the start).
template <typename V>
__global__ __launch_bounds__(kOrbBlock) void k_orb_coords(const V *__restrict__ pm, int n,
                                                          float *__restrict__ xyz,
                                                          uint32_t *__restrict__ keys,
                                                          int32_t *__restrict__ cur)
{
    const int i = blockIdx.x * kOrbBlock + threadIdx.x;
    if (i >= n) return;
    const V p = pm[i];
    const float f[3] = {(float)p.x, (float)p.y, (float)p.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        xyz[(size_t)a * n + i] = f[a];
        keys[(size_t)a * n + i] = tkey(f[a]);
    }
    cur[i] = i;
}

// Per-segment state of one phase-A level.
enum SegMode : int {
    kSelect = 0,  // radix select: histogram the next digit inside the prefix
    kFind = 1,    // one key holds the prefix: the next pass reads it whole
    kDone = 2,    // the k-th key is known
};
struct SegState {
    uint32_t bb[6];    // min keys x,y,z then max keys x,y,z
    int axis;
    int krem;          // rank still to find inside the current prefix
    uint64_t prefix;   // digits of the k-th key found so far
    uint64_t full;     // the k-th key, written by the kFind pass
    uint32_t lcnt, rcnt;
    uint32_t arrived;  // workgroups of the current launch done with the segment
    int mode;          // SegMode
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
        z.full = 0;
        z.lcnt = z.rcnt = 0;
        z.arrived = 0;
        z.mode = kSelect;
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

// Hand-off between the workgroups of one launch, with no cache-wide fence (a
// device-scope fence writes back and invalidates the XCD's whole L2 on this
// GPU, which costs more than the pass it would guard).  Every value that
// another workgroup reads is written by a device-scope atomic whose returned
// value the writing thread waits for (so the update has been performed at the
// device's coherence point before its workgroup arrives), and is read with
// device-scope loads.
template <typename T>
__device__ __forceinline__ T load_dev(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_dev(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// waits until v, returned by an atomic, has arrived
template <typename T>
__device__ __forceinline__ void performed(T v)
{
    asm volatile("" ::"v"(v));
}

// Called by every thread of a workgroup after its atomics for segment s: true
// in the workgroup that finishes the segment last.  No workgroup waits for
// another.
__device__ __forceinline__ bool last_of_segment(SegState *__restrict__ st, int s,
                                                const int3 *__restrict__ segs, int *flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t nch = (uint32_t)((segs[s].y + kChunk - 1) / kChunk);
        *flag = atomicAdd(&st[s].arrived, 1u) == nch - 1;
    }
    __syncthreads();
    return *flag != 0;
}

// Key bounding box of each segment; the workgroup that finishes a segment
// picks its split axis.  keys: the three axes' total-order keys in the
// current order (axis a at a * n).
__global__ __launch_bounds__(kOrbBlock) void k_orb_bbox(const int3 *__restrict__ chunks,
                                                        const int3 *__restrict__ segs,
                                                        const uint32_t *__restrict__ keys, int n,
                                                        SegState *__restrict__ st)
{
    const int3 c = chunks[blockIdx.x];
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    // a fixed number of elements per thread, so that all their loads are in
    // flight together
    // (positions past the chunk's end read its last element again: no branch
    // around the loads)
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) {
        const int p = min(c.y + u * kOrbBlock + (int)threadIdx.x, c.z - 1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint32_t k = keys[(size_t)a * n + p];
            lo[a] = min(lo[a], k);
            hi[a] = max(hi[a], k);
        }
    }
    __shared__ uint32_t red[kOrbBlock / 64][6];
    __shared__ int last;
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
        performed(threadIdx.x < 3 ? atomicMin(&st[c.x].bb[threadIdx.x], v)
                                  : atomicMax(&st[c.x].bb[threadIdx.x], v));
    }
    if (!last_of_segment(st, c.x, segs, &last)) return;
    if (threadIdx.x == 0) {
        uint32_t bb[6];
        for (int a = 0; a < 6; ++a) bb[a] = load_dev(&st[c.x].bb[a]);
        st[c.x].axis = pick_axis(bb);
        store_dev(&st[c.x].arrived, 0u);
    }
}

// One pass of the radix select of every segment, for digit `round` (8 bits,
// most significant first) of the 64-bit key (total-order key along the
// segment's axis, original index).  kSelect: count the digit of the keys
// inside the prefix found so far; the workgroup that finishes the segment
// picks the bin holding rank krem and clears the counts.  If that bin holds a
// single key, the next pass (kFind) only reads it whole.  keys: as for
// k_orb_bbox; cur: original index per position.
__global__ __launch_bounds__(kOrbBlock) void k_orb_hist(const int3 *__restrict__ chunks,
                                                        const int3 *__restrict__ segs,
                                                        const uint32_t *__restrict__ keys, int n,
                                                        const int32_t *__restrict__ cur,
                                                        SegState *__restrict__ st,
                                                        uint32_t *__restrict__ hist, int round)
{
    __shared__ uint32_t h[256];
    __shared__ uint32_t red[kOrbBlock / 64];
    __shared__ int last;
    const int3 c = chunks[blockIdx.x];
    // the state was written by earlier launches only
    const int mode = st[c.x].mode;
    if (mode == kDone) return;  // the whole segment returns: nobody arrives
    const int axis = st[c.x].axis;
    const uint64_t prefix = st[c.x].prefix;
    const int shift = 56 - 8 * round;
    const uint32_t *ka = keys + (size_t)axis * n;
    // the index (low 32 bits) matters from round 4 on, and to read the key whole
    const bool need_idx = round >= 4 || mode == kFind;
    // positions past the chunk's end read its last element (no branch around
    // the loads, so they are all in flight together) and are masked below
    uint64_t key[kChunkPer];
    if (need_idx) {
#pragma unroll
        for (int u = 0; u < kChunkPer; ++u) {
            const int p = min(c.y + u * kOrbBlock + (int)threadIdx.x, c.z - 1);
            key[u] = ((uint64_t)ka[p] << 32) | (uint32_t)cur[p];
        }
    } else {
#pragma unroll
        for (int u = 0; u < kChunkPer; ++u) {
            const int p = min(c.y + u * kOrbBlock + (int)threadIdx.x, c.z - 1);
            key[u] = (uint64_t)ka[p] << 32;
        }
    }
    if (mode == kFind) {
#pragma unroll
        for (int u = 0; u < kChunkPer; ++u) {
            const int p = c.y + u * kOrbBlock + threadIdx.x;
            if (p < c.z && (key[u] >> (shift + 8)) == prefix)
                performed(__hip_atomic_exchange(&st[c.x].full, key[u], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT));
        }
        if (!last_of_segment(st, c.x, segs, &last)) return;
        if (threadIdx.x == 0) {
            st[c.x].prefix = load_dev(&st[c.x].full);
            st[c.x].mode = kDone;
            store_dev(&st[c.x].arrived, 0u);
        }
        return;
    }
    h[threadIdx.x] = 0u;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) {
        const int p = c.y + u * kOrbBlock + threadIdx.x;
        if (p < c.z && (round == 0 || (key[u] >> (shift + 8)) == prefix))
            atomicAdd(&h[(key[u] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    uint32_t *hs = hist + (size_t)c.x * 256;
    const uint32_t v = h[threadIdx.x];
    if (v) performed(atomicAdd(&hs[threadIdx.x], v));
    if (!last_of_segment(st, c.x, segs, &last)) return;
    const uint32_t cnt = load_dev(&hs[threadIdx.x]);
    store_dev(&hs[threadIdx.x], 0u);
    const uint32_t inc = block_incl_scan_u32(cnt, red);
    const uint32_t krem = (uint32_t)st[c.x].krem;
    if (inc >= krem && inc - cnt < krem) {
        st[c.x].prefix = (prefix << 8) | (uint64_t)threadIdx.x;
        st[c.x].krem = (int)(krem - (inc - cnt));
        st[c.x].mode = (cnt == 1u && round < 7) ? kFind : kSelect;
    }
    if (threadIdx.x == 0) store_dev(&st[c.x].arrived, 0u);
}

// Keys <= the k-th key go left.  Each workgroup takes one run of slots per
// side with one atomic each and fills it in position order (ballot ranks);
// the order of the runs is irrelevant to the result.  The original indices
// go to tmp, the three axes' keys to keys_out, both in the new order.
__global__ __launch_bounds__(kOrbBlock) void k_orb_partition(const int3 *__restrict__ chunks,
                                                             const int3 *__restrict__ segs,
                                                             const uint32_t *__restrict__ keys,
                                                             uint32_t *__restrict__ keys_out, int n,
                                                             const int32_t *__restrict__ cur,
                                                             SegState *__restrict__ st,
                                                             int32_t *__restrict__ tmp)
{
    constexpr int kW = kOrbBlock / 64;
    __shared__ uint32_t cl[kChunkPer * kW], cr[kChunkPer * kW];
    __shared__ uint32_t bl, br;
    const int3 c = chunks[blockIdx.x];
    const int axis = st[c.x].axis;
    const uint64_t kth = st[c.x].prefix;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    const uint32_t *ka = keys + (size_t)axis * n;
    // this thread's bodies and their sides, loaded together
    int bod[kChunkPer];
    uint32_t rank[kChunkPer];
    bool lft[kChunkPer];
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) {
        const int p = c.y + u * kOrbBlock + threadIdx.x;
        const int q = min(p, c.z - 1);  // loads without a branch, masked below
        const int b = cur[q];
        lft[u] = (((uint64_t)ka[q] << 32) | (uint32_t)b) <= kth;
        bod[u] = p < c.z ? b : -1;
    }
    // rank inside the (step, wave) group by ballots, group totals in LDS
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) {
        const uint64_t ml = __ballot(bod[u] >= 0 && lft[u]);
        const uint64_t mr = __ballot(bod[u] >= 0 && !lft[u]);
        rank[u] = (uint32_t)__popcll((lft[u] ? ml : mr) & below);
        if (lane == 0) {
            cl[u * kW + w] = (uint32_t)__popcll(ml);
            cr[u * kW + w] = (uint32_t)__popcll(mr);
        }
    }
    __syncthreads();
    // exclusive scans over the kChunkPer * kW groups (position order), by wave 0
    static_assert(kChunkPer * kW == 64, "one group per lane of wave 0");
    if (w == 0) {
        const uint32_t a = cl[lane], b = cr[lane];
        uint32_t ia = a, ib = b;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t ya = (uint32_t)__shfl_up((int)ia, o), yb = (uint32_t)__shfl_up((int)ib, o);
            if (lane >= o) {
                ia += ya;
                ib += yb;
            }
        }
        cl[lane] = ia - a;
        cr[lane] = ib - b;
        if (lane == 63) {
            bl = atomicAdd(&st[c.x].lcnt, ia);
            br = atomicAdd(&st[c.x].rcnt, ib);
        }
    }
    __syncthreads();
    const int3 sg = segs[c.x];
    // exactly k keys are <= the k-th key; the guards only keep a violated
    // precondition (non-finite coordinates) inside the segment
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) {
        const int b = bod[u];
        if (b < 0) continue;
        const int p = c.y + u * kOrbBlock + threadIdx.x;
        int d;
        if (lft[u]) {
            const uint32_t q = bl + cl[u * kW + w] + rank[u];
            if (q >= (uint32_t)sg.z) continue;
            d = sg.x + (int)q;
        } else {
            const uint32_t q = br + cr[u * kW + w] + rank[u];
            if (q >= (uint32_t)(sg.y - sg.z)) continue;
            d = sg.x + sg.z + (int)q;
        }
        tmp[d] = b;
#pragma unroll
        for (int a = 0; a < 3; ++a) keys_out[(size_t)a * n + d] = keys[(size_t)a * n + p];
    }
}

// The clamp only keeps a broken invariant (a slot left unfilled) from turning
// into out-of-bounds reads later: every slot is filled.
__global__ __launch_bounds__(kOrbBlock) void k_orb_copyback(const int3 *__restrict__ chunks,
                                                            const int32_t *__restrict__ tmp, int n,
                                                            int32_t *__restrict__ cur)
{
    const int3 c = chunks[blockIdx.x];
    for (int p = c.y + threadIdx.x; p < c.z; p += kOrbBlock) cur[p] = (int32_t)min((uint32_t)tmp[p], (uint32_t)(n - 1));
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
    // xyz by original index, then two buffers of the three axes' keys in the
    // current order (each level reads one and writes the other)
    float *xyz = (float *)scratch(kSlotOrb0, 9 * nbytes);
    int32_t *cur = (int32_t *)scratch(kSlotOrb1, nbytes);
    int32_t *tmp = (int32_t *)scratch(kSlotOrb2, nbytes);
    char *dtab = (char *)scratch(kSlotOrb3, tab.size() + 16);
    char *state = (char *)scratch(kSlotOrb4, maxseg * (sizeof(SegState) + 256 * 4) + 64);
    if (!xyz || !cur || !tmp || !dtab || !state) {
        set_error("cannot allocate ORB scratch");
        return NBODY_E_NOMEM;
    }
    uint32_t *kbuf[2] = {(uint32_t *)(xyz + 3 * (size_t)n), (uint32_t *)(xyz + 6 * (size_t)n)};
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
        hipLaunchKernelGGL(k_orb_coords<double4>, dim3(nb), dim3(kOrbBlock), 0, s, (const double4 *)pm, n, xyz,
                           kbuf[0], cur);
    else
        hipLaunchKernelGGL(k_orb_coords<float4>, dim3(nb), dim3(kOrbBlock), 0, s, (const float4 *)pm, n, xyz,
                           kbuf[0], cur);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ORB coordinates");
    for (size_t l = 0; l < levels.size(); ++l) {
        const int nseg = (int)levels[l].segs.size(), nch = (int)levels[l].chunks.size();
        const int3 *segs = (const int3 *)(dtab + off[l].first);
        const int3 *chunks = (const int3 *)(dtab + off[l].second);
        const uint32_t *keys = kbuf[l & 1];
        hipLaunchKernelGGL(k_orb_init, dim3(nseg), dim3(256), 0, s, segs, nseg, st, hist);
        hipLaunchKernelGGL(k_orb_bbox, dim3(nch), dim3(kOrbBlock), 0, s, chunks, segs, keys, n, st);
        for (int r = 0; r < 8; ++r)
            hipLaunchKernelGGL(k_orb_hist, dim3(nch), dim3(kOrbBlock), 0, s, chunks, segs, keys, n, cur, st, hist, r);
        hipLaunchKernelGGL(k_orb_partition, dim3(nch), dim3(kOrbBlock), 0, s, chunks, segs, keys, kbuf[(l + 1) & 1],
                           n, cur, st, tmp);
        hipLaunchKernelGGL(k_orb_copyback, dim3(nch), dim3(kOrbBlock), 0, s, chunks, tmp, n, cur);
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
