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
//     each segment exactly, with a radix select;
//   * bodies may be partitioned in any order, because every later decision
//     depends on set membership only and every leaf is finally sorted by
//     original index.
// Phase A handles segments larger than kSmall bodies, one level of the tree
// per step, with multi-workgroup kernels over fixed-size chunks.  The three
// axes' keys travel with the index array (two buffers, read and written in
// turn), so every pass reads them coalesced.  A level is: four histogram
// passes over the coordinate's 8-bit digits (k_orb_hist; the workgroup that
// finishes a segment picks the bin, and once the bin holds a single key one
// pass reads it whole), one pass that settles ties between equal coordinates
// by index (k_orb_ties), and the partition (k_orb_partition), which also
// accumulates each part's key box for the next level.  Phase B (k_orb_block)
// finishes every remaining segment (at most max(kSmall, leaf) <=
// kMaxBlockSeg bodies) inside one workgroup: the segment's keys are loaded
// into LDS once, nodes above kWaveNode bodies are split by the workgroup,
// smaller ones by one wave each, nodes of at most 64 bodies by ranking
// inside the wave, and the final order is written.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace nbi {

constexpr int kSmall = 1024;        // phase A splits segments larger than this
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

// Total-order keys of the FP32 coordinates in the current order (identity at
// the start).
template <typename V>
__global__ __launch_bounds__(kOrbBlock) void k_orb_coords(const V *__restrict__ pm, int n,
                                                          uint32_t *__restrict__ keys,
                                                          int32_t *__restrict__ cur)
{
    const int i = blockIdx.x * kOrbBlock + threadIdx.x;
    if (i >= n) return;
    const V p = pm[i];
    const float f[3] = {(float)p.x, (float)p.y, (float)p.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) keys[(size_t)a * n + i] = tkey(f[a]);
    cur[i] = i;
}

// Radix select over the 64-bit key (coordinate key in the high half, index
// in the low half) in digits of kDigit bits, most significant first;
// digit_shift(r) is the lowest bit of digit r.
constexpr int kDigit = 8;
constexpr int kBins = 1 << kDigit;
__host__ __device__ constexpr int digit_shift(int round)
{
    return 64 - kDigit * (round + 1) > 0 ? 64 - kDigit * (round + 1) : 0;
}
// bits above the digit of `round`: the prefix found before it
__host__ __device__ constexpr int prefix_shift(int round)
{
    return round == 0 ? 64 : digit_shift(round - 1);
}
// The histogram, tie and partition passes run 512 threads per chunk: more
// waves per CU to hide their latency, without more workgroups per segment.
constexpr int kPassBlock = 512;
constexpr int kPassPer = kChunk / kPassBlock;
static_assert(kBins <= kPassBlock, "one bin per thread");
// The rounds over the coordinate's 32 bits run as histogram passes; the
// index bits, which only matter between equal coordinates, are settled by
// one pass over those bodies (k_orb_ties).
constexpr int kCoordRounds = 32 / kDigit;
static_assert(32 % kDigit == 0 && digit_shift(kCoordRounds - 1) == 32, "digits end at the coordinate");

// Per-segment state of one phase-A level.
enum SegMode : int {
    kSelect = 0,  // radix select: histogram the next digit inside the prefix
    kFind = 1,    // one key holds the prefix: the next pass reads it whole
    kDone = 2,    // the k-th key is known
};
struct SegState {
    uint32_t bb[6];    // min keys x,y,z then max keys x,y,z
    int krem;          // rank still to find inside the current prefix
    int mode;          // SegMode
    uint64_t prefix;   // digits of the k-th key found so far
    uint64_t full;     // the k-th key, written by the kFind pass
    uint64_t placed;   // partition: bodies placed (high half) and placed left (low half)
    uint32_t arrived;  // workgroups of the current pass done with the segment
    uint32_t ties;     // bodies whose coordinate equals the k-th key's (k_orb_ties)
};

__device__ __forceinline__ void init_state(SegState *st, int k)
{
    SegState z;
    for (int a = 0; a < 3; ++a) {
        z.bb[a] = 0xFFFFFFFFu;
        z.bb[3 + a] = 0u;
    }
    z.krem = k;
    z.mode = kSelect;
    z.prefix = 0;
    z.full = 0;
    z.placed = 0;
    z.arrived = 0;
    z.ties = 0;
    *st = z;
}

// the segment's split axis, from its key box (complete once the pass that
// accumulated it has ended)
__device__ __forceinline__ int seg_axis(const SegState *st)
{
    uint32_t bb[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) bb[a] = st->bb[a];
    return pick_axis(bb);
}

// Tables: segs (start, size, k) per segment of a level, chunks (segment,
// begin, end), kids (next-level segment of the left and of the right part,
// -1 where that part is finished by phase B).
// First level: its states, and every histogram row cleared (the passes
// leave them cleared after that).  One workgroup per row.
__global__ __launch_bounds__(kOrbBlock) void k_orb_init(const int3 *__restrict__ segs, int nseg,
                                                        SegState *__restrict__ st,
                                                        uint32_t *__restrict__ hist)
{
    const int s = blockIdx.x;
    if (s < nseg && threadIdx.x == 0) init_state(&st[s], segs[s].z);
    for (int j = threadIdx.x; j < kBins; j += kOrbBlock) hist[(size_t)s * kBins + j] = 0u;
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

// Inclusive sum over the workgroup's threads: within each wave by shuffles,
// then the totals of the waves before it (scratch: one entry per wave).
__device__ __forceinline__ uint32_t block_incl_scan_u32(uint32_t v, uint32_t *scratch)
{
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

__device__ __forceinline__ void box_atomics(uint32_t *bb, const uint32_t *v)
{
    if (threadIdx.x < 3)
        atomicMin(&bb[threadIdx.x], v[threadIdx.x]);
    else if (threadIdx.x < 6)
        atomicMax(&bb[threadIdx.x], v[threadIdx.x]);
}

// Key bounding box of each segment of the first level (the partition
// accumulates it for the later levels).  keys: the three axes' total-order
// keys in the current order (axis a at a * n).
__global__ __launch_bounds__(kOrbBlock) void k_orb_bbox(const int3 *__restrict__ chunks,
                                                        const uint32_t *__restrict__ keys, int n,
                                                        SegState *__restrict__ st)
{
    const int3 c = chunks[blockIdx.x];
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    // a fixed number of elements per thread, so that all their loads are in
    // flight together (positions past the chunk's end read its last element
    // again: no branch around the loads)
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
    __shared__ uint32_t tot[6];
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
        tot[threadIdx.x] = v;
    }
    __syncthreads();
    box_atomics(st[c.x].bb, tot);
}

// One pass of the radix select of every segment, for digit `round` of the
// 64-bit key (total-order key along the segment's axis, original index).
// kSelect: count the digit of the keys inside the prefix found so far; the
// workgroup that finishes the segment picks the bin holding rank krem and
// clears the counts.  If that bin holds a single key, the next pass (kFind)
// only reads it whole.  keys: as for k_orb_bbox; cur: original index per
// position.  The first pass also sets up the states of the next level
// (st_next), which the partition fills in.
__global__ __launch_bounds__(kPassBlock) void k_orb_hist(const int3 *__restrict__ chunks,
                                                        const int3 *__restrict__ segs,
                                                        const uint32_t *__restrict__ keys, int n,
                                                        const int32_t *__restrict__ cur,
                                                        SegState *__restrict__ st,
                                                        uint32_t *__restrict__ hist, int round,
                                                        const int3 *__restrict__ segs_next, int nseg_next,
                                                        SegState *__restrict__ st_next)
{
    __shared__ uint32_t h[kBins];
    __shared__ uint32_t red[kPassBlock / 64];
    __shared__ int last;
    if (round == 0 && threadIdx.x == 0)
        for (int s = blockIdx.x; s < nseg_next; s += gridDim.x) init_state(&st_next[s], segs_next[s].z);
    const int3 c = chunks[blockIdx.x];
    // the state was written by earlier launches only
    const int mode = st[c.x].mode;
    if (mode == kDone) return;  // the whole segment returns: nobody arrives
    const uint64_t prefix = st[c.x].prefix;
    const int shift = digit_shift(round), pshift = prefix_shift(round);
    const uint32_t dmask = (1u << (pshift - shift)) - 1u;
    const uint32_t *ka = keys + (size_t)seg_axis(&st[c.x]) * n;
    // the index (low 32 bits) matters once the digit reaches below bit 32, and
    // to read the key whole
    const bool need_idx = shift < 32 || mode == kFind;
    // positions past the chunk's end read its last element (no branch around
    // the loads, so they are all in flight together) and are masked below
    uint64_t key[kPassPer];
    if (need_idx) {
#pragma unroll
        for (int u = 0; u < kPassPer; ++u) {
            const int p = min(c.y + u * kPassBlock + (int)threadIdx.x, c.z - 1);
            key[u] = ((uint64_t)ka[p] << 32) | (uint32_t)cur[p];
        }
    } else {
#pragma unroll
        for (int u = 0; u < kPassPer; ++u) {
            const int p = min(c.y + u * kPassBlock + (int)threadIdx.x, c.z - 1);
            key[u] = (uint64_t)ka[p] << 32;
        }
    }
    // (round 0 has no prefix: a shift by 64 is not defined, so test it apart)
    if (mode == kFind) {
#pragma unroll
        for (int u = 0; u < kPassPer; ++u) {
            const int p = c.y + u * kPassBlock + threadIdx.x;
            if (p < c.z && (round == 0 || (key[u] >> pshift) == prefix))
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
    if (threadIdx.x < kBins) h[threadIdx.x] = 0u;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPassPer; ++u) {
        const int p = c.y + u * kPassBlock + threadIdx.x;
        if (p < c.z && (round == 0 || (key[u] >> pshift) == prefix))
            atomicAdd(&h[(uint32_t)(key[u] >> shift) & dmask], 1u);
    }
    __syncthreads();
    uint32_t *hs = hist + (size_t)c.x * kBins;
    if (threadIdx.x < kBins) {
        const uint32_t v = h[threadIdx.x];
        if (v) performed(atomicAdd(&hs[threadIdx.x], v));
    }
    if (!last_of_segment(st, c.x, segs, &last)) return;
    // the last workgroup: thread t < kBins holds bin t
    uint32_t cnt = 0;
    if (threadIdx.x < kBins) {
        cnt = load_dev(&hs[threadIdx.x]);
        store_dev(&hs[threadIdx.x], 0u);
    }
    const uint32_t inc = block_incl_scan_u32(cnt, red);
    const uint32_t krem = (uint32_t)st[c.x].krem;
    if (inc >= krem && inc - cnt < krem) {
        st[c.x].prefix = (round == 0 ? 0ull : prefix << (pshift - shift)) | (uint64_t)threadIdx.x;
        st[c.x].krem = (int)(krem - (inc - cnt));
        st[c.x].mode = (cnt == 1u && round < kCoordRounds - 1) ? kFind : kSelect;
    }
    if (threadIdx.x == 0) store_dev(&st[c.x].arrived, 0u);
}

// After the coordinate rounds: the k-th key's coordinate c is known, and its
// rank krem among the bodies with coordinate c.  Their original indices are
// gathered into cand (at the segment's own positions), and the workgroup that
// finishes the segment selects the krem-th smallest of them (radix select
// over the 32-bit index; a single body needs none).
__global__ __launch_bounds__(kPassBlock) void k_orb_ties(const int3 *__restrict__ chunks,
                                                        const int3 *__restrict__ segs,
                                                        const uint32_t *__restrict__ keys, int n,
                                                        const int32_t *__restrict__ cur,
                                                        SegState *__restrict__ st,
                                                        uint32_t *__restrict__ cand)
{
    __shared__ uint32_t h[256];
    __shared__ uint32_t red[kPassBlock / 64];
    __shared__ uint32_t sel_s, krem_s;
    __shared__ int last;
    const int3 c = chunks[blockIdx.x];
    if (st[c.x].mode == kDone) return;  // the whole segment returns: nobody arrives
    const uint32_t coord = (uint32_t)st[c.x].prefix;  // the prefix is the coordinate key here
    const int3 sg = segs[c.x];
    const uint32_t *ka = keys + (size_t)seg_axis(&st[c.x]) * n;
    const int lane = threadIdx.x & 63;
    uint32_t kv[kPassPer];
#pragma unroll
    for (int u = 0; u < kPassPer; ++u) kv[u] = ka[min(c.y + u * kPassBlock + (int)threadIdx.x, c.z - 1)];
#pragma unroll
    for (int u = 0; u < kPassPer; ++u) {
        const int p = c.y + u * kPassBlock + threadIdx.x;
        const bool hit = p < c.z && kv[u] == coord;
        const uint64_t mk = __ballot(hit);
        if (!mk) continue;
        // one slot run per wave and step
        uint32_t base = 0;
        if (lane == __ffsll((long long)mk) - 1) base = atomicAdd(&st[c.x].ties, (uint32_t)__popcll(mk));
        base = (uint32_t)__shfl((int)base, __ffsll((long long)mk) - 1);
        if (hit) {
            const uint32_t q = base + (uint32_t)__popcll(mk & ((1ull << lane) - 1ull));
            if (q < (uint32_t)sg.y)
                performed(__hip_atomic_exchange(&cand[sg.x + q], (uint32_t)cur[p], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT));
        }
    }
    if (!last_of_segment(st, c.x, segs, &last)) return;
    const uint32_t T = min(load_dev(&st[c.x].ties), (uint32_t)sg.y);
    const uint32_t *cs = cand + sg.x;
    uint32_t sel = 0;
    if (T == 1u) {
        sel = load_dev(&cs[0]);
    } else {
        if (threadIdx.x == 0) {
            sel_s = 0u;
            krem_s = (uint32_t)st[c.x].krem;
        }
        for (int round = 0; round < 4; ++round) {
            __syncthreads();
            if (threadIdx.x < 256) h[threadIdx.x] = 0u;
            const uint32_t prefix = sel_s, kr = krem_s;
            const int shift = 24 - 8 * round;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < T; i += kPassBlock) {
                const uint32_t v = load_dev(&cs[i]);
                if (round == 0 || (v >> (shift + 8)) == prefix) atomicAdd(&h[(v >> shift) & 0xFFu], 1u);
            }
            __syncthreads();
            const uint32_t hv = threadIdx.x < 256 ? h[threadIdx.x] : 0u;
            const uint32_t inc = block_incl_scan_u32(hv, red);
            if (inc >= kr && inc - hv < kr) {
                sel_s = (prefix << 8) | (uint32_t)threadIdx.x;
                krem_s = kr - (inc - hv);
            }
        }
        __syncthreads();
        sel = sel_s;
    }
    if (threadIdx.x == 0) {
        st[c.x].prefix = ((uint64_t)coord << 32) | sel;
        st[c.x].mode = kDone;
        store_dev(&st[c.x].arrived, 0u);
    }
}

// Keys <= the k-th key go left.  Each workgroup takes one run of slots per
// side (one 64-bit atomic gives both) and fills it in position order (ballot ranks);
// the order of the runs is irrelevant to the result.  The original indices
// go to cur_out and the three axes' keys to keys_out, both in the new order.
// Each side's key box is accumulated into its next-level state (if it has
// one).
__global__ __launch_bounds__(kPassBlock) void k_orb_partition(const int3 *__restrict__ chunks,
                                                             const int3 *__restrict__ segs,
                                                             const int2 *__restrict__ kids,
                                                             const uint32_t *__restrict__ keys,
                                                             uint32_t *__restrict__ keys_out, int n,
                                                             const int32_t *__restrict__ cur,
                                                             int32_t *__restrict__ cur_out,
                                                             SegState *__restrict__ st,
                                                             SegState *__restrict__ st_next)
{
    constexpr int kW = kPassBlock / 64;
    __shared__ uint32_t cl[kPassPer * kW], cr[kPassPer * kW];
    __shared__ uint32_t bl, br;
    __shared__ uint32_t box[kW][12];
    __shared__ uint32_t tot[12];
    const int3 c = chunks[blockIdx.x];
    const uint64_t kth = st[c.x].prefix;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    const uint32_t *ka = keys + (size_t)seg_axis(&st[c.x]) * n;
    // this thread's bodies and their sides, loaded together
    int bod[kPassPer];
    uint32_t rank[kPassPer];
    bool lft[kPassPer];
#pragma unroll
    for (int u = 0; u < kPassPer; ++u) {
        const int p = c.y + u * kPassBlock + threadIdx.x;
        const int q = min(p, c.z - 1);  // loads without a branch, masked below
        const int b = cur[q];
        lft[u] = (((uint64_t)ka[q] << 32) | (uint32_t)b) <= kth;
        bod[u] = p < c.z ? b : -1;
    }
    // rank inside the (step, wave) group by ballots, group totals in LDS
#pragma unroll
    for (int u = 0; u < kPassPer; ++u) {
        const uint64_t ml = __ballot(bod[u] >= 0 && lft[u]);
        const uint64_t mr = __ballot(bod[u] >= 0 && !lft[u]);
        rank[u] = (uint32_t)__popcll((lft[u] ? ml : mr) & below);
        if (lane == 0) {
            cl[u * kW + w] = (uint32_t)__popcll(ml);
            cr[u * kW + w] = (uint32_t)__popcll(mr);
        }
    }
    __syncthreads();
    // exclusive scans over the kPassPer * kW groups (position order), by wave 0
    static_assert(kPassPer * kW <= 64, "one group per lane of wave 0");
    if (w == 0) {
        const bool g = lane < kPassPer * kW;
        const uint32_t a = g ? cl[lane] : 0u, b = g ? cr[lane] : 0u;
        uint32_t ia = a, ib = b;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t ya = (uint32_t)__shfl_up((int)ia, o), yb = (uint32_t)__shfl_up((int)ib, o);
            if (lane >= o) {
                ia += ya;
                ib += yb;
            }
        }
        if (g) {
            cl[lane] = ia - a;
            cr[lane] = ib - b;
        }
        if (lane == 63) {
            // one atomic for both runs: the bodies placed before this
            // workgroup, and how many of them went left
            const unsigned long long was =
                atomicAdd(reinterpret_cast<unsigned long long *>(&st[c.x].placed),
                          ((unsigned long long)(ia + ib) << 32) | ia);
            bl = (uint32_t)was;
            br = (uint32_t)(was >> 32) - (uint32_t)was;
        }
    }
    __syncthreads();
    const int3 sg = segs[c.x];
    // box of each side: min keys x,y,z then max keys x,y,z; left then right
    uint32_t bx[12];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bx[a] = bx[6 + a] = 0xFFFFFFFFu;
        bx[3 + a] = bx[9 + a] = 0u;
    }
    // destinations; exactly k keys are <= the k-th key, and the guards only
    // keep a violated precondition (non-finite coordinates) inside the segment
    int dst[kPassPer];
#pragma unroll
    for (int u = 0; u < kPassPer; ++u) {
        const uint32_t q = (lft[u] ? bl + cl[u * kW + w] : br + cr[u * kW + w]) + rank[u];
        const bool fits = lft[u] ? q < (uint32_t)sg.z : q < (uint32_t)(sg.y - sg.z);
        dst[u] = bod[u] >= 0 && fits ? sg.x + (lft[u] ? 0 : sg.z) + (int)q : -1;
        if (dst[u] >= 0) cur_out[dst[u]] = bod[u];
    }
    // one axis at a time: all of the thread's loads first, then the stores
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        uint32_t kv[kPassPer];
#pragma unroll
        for (int u = 0; u < kPassPer; ++u) kv[u] = keys[(size_t)a * n + min(c.y + u * kPassBlock + (int)threadIdx.x, c.z - 1)];
#pragma unroll
        for (int u = 0; u < kPassPer; ++u) {
            if (dst[u] < 0) continue;
            keys_out[(size_t)a * n + dst[u]] = kv[u];
            const int o = lft[u] ? 0 : 6;
            bx[o + a] = min(bx[o + a], kv[u]);
            bx[o + 3 + a] = max(bx[o + 3 + a], kv[u]);
        }
    }
#pragma unroll
    for (int j = 0; j < 12; ++j) bx[j] = (j % 6) < 3 ? wave_min(bx[j]) : wave_max(bx[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < 12; ++j) box[w][j] = bx[j];
    __syncthreads();
    if (threadIdx.x < 12) {
        const int j = threadIdx.x;
        uint32_t v = box[0][j];
        for (int k = 1; k < kW; ++k) v = (j % 6) < 3 ? min(v, box[k][j]) : max(v, box[k][j]);
        tot[j] = v;
    }
    __syncthreads();
    const int2 kd = kids[c.x];
    if (kd.x >= 0) box_atomics(st_next[kd.x].bb, tot);
    if (kd.y >= 0) box_atomics(st_next[kd.y].bb, tot + 6);
}

// ---- phase B: one workgroup finishes one segment in LDS --------------------
// The segment's keys are loaded once, coalesced, from the key buffer that
// holds it (phase A leaves them in the segment's order) and stay in their
// slots; the recursion permutes slot numbers only.

// Box of a node (min keys x,y,z then max keys x,y,z), over the whole
// workgroup: two barriers for all six values.
__device__ __forceinline__ void block_box(uint32_t *bb, uint32_t (*red)[6])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 6; ++j) bb[j] = j < 3 ? wave_min(bb[j]) : wave_max(bb[j]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < 6; ++j) red[w][j] = bb[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        uint32_t v = red[0][j];
        for (int k = 1; k < kOrbBlock / 64; ++k) v = j < 3 ? min(v, red[k][j]) : max(v, red[k][j]);
        bb[j] = v;
    }
}

// Finishes the recursion of a node of at most 64 bodies (positions
// [lo, lo + m) of pos) with one wave, one position per lane, every node of a
// level split at once.  keys: per-wave LDS of 3 x 64 total-order keys.  The
// k smallest keys of a node are found by ranking (keys and indices are
// distinct), then each leaf is ordered by original index.
constexpr int kWaveSeg = 64;

__device__ void orb_wave(int32_t *pos, const uint32_t (*skey)[kSmall], const int32_t *gid,
                         uint32_t (*keys)[kWaveSeg], int32_t *wid, int lo, int m, int leaf, int lane)
{
    const int s = lane < m ? pos[lo + lane] : 0;  // this lane's slot
    const uint32_t kx = skey[0][s], ky = skey[1][s], kz = skey[2][s];
    const int b = gid[s];
    int slo = 0, sm = m;  // the node holding this lane's entry (relative to lo)
    int at = lane;        // this lane's entry's current position (relative to lo)
    if (lane < m) {
        keys[0][lane] = kx;
        keys[1][lane] = ky;
        keys[2][lane] = kz;
        wid[lane] = b;
    }
    for (;;) {
        const bool split = lane < m && sm > leaf;
        if (!__any(split)) break;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int to = at;
        int k = sm;
        if (split) {
            uint32_t bb[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
            // (unrolled so that several LDS reads are in flight per wait)
#pragma unroll 4
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
#pragma unroll 4
            for (int f = slo; f < slo + sm; ++f) {
                const uint32_t v = keys[axis][f];
                r += (v < mine) || (v == mine && wid[f] < b);
            }
            to = slo + r;
            const int L = (sm + leaf - 1) / leaf;
            k = min(sm, leaf * ((L + 1) / 2));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < m) {
            keys[0][to] = kx;
            keys[1][to] = ky;
            keys[2][to] = kz;
            wid[to] = b;
            at = to;
            if (split) {
                if (to - slo < k) {
                    sm = k;
                } else {
                    slo += k;
                    sm -= k;
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // leaves: ascending original index
    int r = 0;
    if (lane < m)
#pragma unroll 4
        for (int f = slo; f < slo + sm; ++f) r += wid[f] < b;
    if (lane < m) pos[lo + slo + r] = s;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Nodes of at most kWaveNode bodies are split by one wave each, several
// subtrees at once.
constexpr int kWaveNode = 256;
constexpr int kStack = 24;  // node stack entries (the recursion is at most 12 deep)

// One wave finishes the subtree of node [lo0, lo0 + m0) of pos: the same
// splits as the block-wide path (radix select of the k-th key with a
// 256-bin histogram hw of the wave's own, ballot-ranked partition through
// tmp), nodes of at most 64 bodies by orb_wave, leaves by rank.
__device__ void wave_subtree(int32_t *pos, int32_t *tmp, uint32_t *akey, const uint32_t (*skey)[kSmall],
                             const int32_t *gid, uint32_t *hw, uint32_t (*wk)[kWaveSeg], int32_t *wid, int2 *stk,
                             int lo0, int m0, int leaf, int lane)
{
    // node stack in LDS (stk: this wave's kStack entries); sp is uniform
    int sp = 1;
    if (lane == 0) stk[0] = make_int2(lo0, m0);
    wave_sync();
    while (sp > 0) {
        --sp;
        const int2 nd = stk[sp];
        const int lo = nd.x, m = nd.y;
        wave_sync();  // read before the pushes below overwrite the entry
        if (m <= kWaveSeg) {
            orb_wave(pos, skey, gid, wk, wid, lo, m, leaf, lane);
            wave_sync();
            continue;
        }
        if (m <= leaf) {
            // leaf: ranks by original index over a contiguous copy
            for (int e = lane; e < m; e += 64) akey[lo + e] = (uint32_t)gid[pos[lo + e]];
            wave_sync();
            for (int e = lane; e < m; e += 64) {
                const uint32_t v = akey[lo + e];
                int r = 0;
#pragma unroll 4
                for (int f = 0; f < m; ++f) r += akey[lo + f] < v;
                tmp[lo + r] = pos[lo + e];
            }
            wave_sync();
            for (int e = lane; e < m; e += 64) pos[lo + e] = tmp[lo + e];
            wave_sync();
            continue;
        }
        uint32_t bb[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
        for (int e = lane; e < m; e += 64) {
            const int s = pos[lo + e];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const uint32_t v = skey[a][s];
                bb[a] = min(bb[a], v);
                bb[3 + a] = max(bb[3 + a], v);
            }
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) bb[j] = j < 3 ? wave_min(bb[j]) : wave_max(bb[j]);
        const int axis = pick_axis(bb);
        const int L = (m + leaf - 1) / leaf;
        const int k = min(m, leaf * ((L + 1) / 2));
        for (int e = lane; e < m; e += 64) akey[lo + e] = skey[axis][pos[lo + e]];
        wave_sync();
        // radix select, 8 bits a round, with the single-key exit
        uint64_t prefix = 0;
        uint32_t kr = (uint32_t)k;
        bool one = false;
        for (int round = 0; round < 8; ++round) {
            const int shift = 56 - 8 * round;
            if (one) {
                // the one key whose digits above `shift` are the prefix
                uint64_t found = 0;
                bool hit = false;
                for (int e = lane; e < m; e += 64) {
                    const uint64_t key = ((uint64_t)akey[lo + e] << 32) | (uint32_t)gid[pos[lo + e]];
                    if ((key >> (shift + 8)) == prefix) {
                        found = key;
                        hit = true;
                    }
                }
                const uint64_t who = __ballot(hit);
                const int src = who ? __ffsll((long long)who) - 1 : 0;
                prefix = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(found >> 32), src) << 32) |
                         (uint32_t)__shfl((int)(uint32_t)found, src);
                break;
            }
            for (int j = lane; j < 256; j += 64) hw[j] = 0u;
            wave_sync();
            for (int e = lane; e < m; e += 64) {
                // the first four digits are the coordinate key's: no index needed
                uint64_t key = (uint64_t)akey[lo + e] << 32;
                if (round >= 4) key |= (uint32_t)gid[pos[lo + e]];
                if (round == 0 || (key >> (shift + 8)) == prefix) atomicAdd(&hw[(key >> shift) & 0xFF], 1u);
            }
            wave_sync();
            uint32_t c[4], tot = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = hw[4 * lane + q];
                tot += c[q];
            }
            uint32_t inc = tot;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = (uint32_t)__shfl_up((int)inc, o);
                if (lane >= o) inc += y;
            }
            const bool mine = inc >= kr && inc - tot < kr;
            int bin = 0;
            uint32_t nkr = 0, bc = 0;
            if (mine) {
                // the first of this lane's bins where the running count reaches kr
                uint32_t acc = inc - tot, before = 0;
                int jb = -1;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (jb < 0 && acc + c[j] >= kr) {
                        jb = j;
                        before = acc;
                        bc = c[j];
                    }
                    acc += c[j];
                }
                bin = 4 * lane + jb;
                nkr = kr - before;
            }
            const uint64_t who = __ballot(mine);
            const int src = who ? __ffsll((long long)who) - 1 : 0;
            bin = __shfl(bin, src);
            kr = (uint32_t)__shfl((int)nkr, src);
            one = __shfl((int)bc, src) == 1;
            prefix = (prefix << 8) | (uint64_t)bin;
            wave_sync();  // hw is cleared again by the next round
        }
        const uint64_t kth = prefix;
        // partition, 64 entries at a time, in position order within each side
        int dl = 0, dr = 0;
        for (int e0 = 0; e0 < m; e0 += 64) {
            const int e = e0 + lane;
            const bool act = e < m;
            const int s = act ? pos[lo + e] : 0;
            // (key, index) <= kth; the index only decides between equal keys
            const uint32_t hk = akey[lo + (act ? e : 0)], kh = (uint32_t)(kth >> 32);
            const bool left = act && (hk < kh || (hk == kh && (uint32_t)gid[s] <= (uint32_t)kth));
            const bool right = act && !left;
            const unsigned long long bl = __ballot(left), br = __ballot(right);
            const int rl = __builtin_amdgcn_mbcnt_hi((unsigned)(bl >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bl, 0u));
            const int rr = __builtin_amdgcn_mbcnt_hi((unsigned)(br >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)br, 0u));
            if (left && dl + rl < k) tmp[lo + dl + rl] = s;
            if (right && dr + rr < m - k) tmp[lo + k + dr + rr] = s;
            dl += __popcll(bl);
            dr += __popcll(br);
        }
        wave_sync();
        for (int e = lane; e < m; e += 64) pos[lo + e] = tmp[lo + e];
        // right first so that the left child is processed next
        if (lane == 0) {
            stk[sp] = make_int2(lo + k, m - k);
            stk[sp + 1] = make_int2(lo, k);
        }
        sp += 2;
        wave_sync();
    }
}

// Orders positions [lo, lo + m) of pos by original index (a leaf), through tmp.
__device__ __forceinline__ void block_leaf(int32_t *pos, int32_t *tmp, uint32_t *val, const int32_t *gid, int lo,
                                           int m)
{
    // ranks by original index over a contiguous copy (val)
    for (int e = threadIdx.x; e < m; e += kOrbBlock) val[lo + e] = (uint32_t)gid[pos[lo + e]];
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += kOrbBlock) {
        const uint32_t v = val[lo + e];
        int r = 0;
#pragma unroll 4
        for (int f = 0; f < m; ++f) r += val[lo + f] < v;
        tmp[lo + r] = pos[lo + e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += kOrbBlock) pos[lo + e] = tmp[lo + e];
    __syncthreads();
}

// segs: (start, size, which buffer pair holds it).  keys0/1: the three axes'
// keys in the order of cur0/1 (axis a at a * n).
__global__ __launch_bounds__(kOrbBlock) void k_orb_block(const int3 *__restrict__ segs,
                                                         const uint32_t *__restrict__ keys0,
                                                         const uint32_t *__restrict__ keys1,
                                                         const int32_t *__restrict__ cur0,
                                                         const int32_t *__restrict__ cur1, int n, int leaf,
                                                         int32_t *__restrict__ perm)
{
    // one buffer: keys by slot (3 x kSmall), original index by slot, slots in
    // the current order, partition target, the current node's keys along
    // its split axis; a segment that is one leaf only needs its indices
    __shared__ uint32_t lds[7 * kSmall];
    static_assert(7 * kSmall >= kMaxBlockSeg, "a one-leaf segment's indices fit");
    uint32_t (*skey)[kSmall] = reinterpret_cast<uint32_t (*)[kSmall]>(lds);
    int32_t *gid = reinterpret_cast<int32_t *>(lds + 3 * kSmall);
    int32_t *pos = reinterpret_cast<int32_t *>(lds + 4 * kSmall);
    int32_t *tmp = reinterpret_cast<int32_t *>(lds + 5 * kSmall);
    uint32_t *akey = lds + 6 * kSmall;
    __shared__ uint32_t h[256];
    __shared__ uint32_t red[kOrbBlock / 64];
    __shared__ uint32_t red6[kOrbBlock / 64][6];
    __shared__ uint32_t wl[kOrbBlock / 64], wr[kOrbBlock / 64];
    __shared__ uint64_t kth_s;
    __shared__ uint32_t krem_s, one_s;
    constexpr int kMaxTask = 64;
    __shared__ int2 task[kMaxTask];
    __shared__ uint32_t hw[kOrbBlock / 64][256];
    __shared__ uint32_t wkeys[kOrbBlock / 64][3][kWaveSeg];
    __shared__ int32_t wgid[kOrbBlock / 64][kWaveSeg];
    __shared__ int2 stk[kOrbBlock / 64 + 1][kStack];  // node stacks: the waves', then the block's
    const int3 sg = segs[blockIdx.x];
    const int start = sg.x, size = sg.y;
    const int32_t *cur = sg.z ? cur1 : cur0;
    const uint32_t *keys = sg.z ? keys1 : keys0;
    // the clamp only keeps a broken invariant (an unfilled slot) from turning
    // into out-of-bounds writes: every slot is filled
    if (size > kSmall) {
        // at most max(kSmall, leaf) bodies reach this kernel: a larger
        // segment is one leaf, written in ascending original index (ranks;
        // the indices are distinct)
        int32_t *big = reinterpret_cast<int32_t *>(lds);
        for (int e = threadIdx.x; e < size; e += kOrbBlock) big[e] = (int32_t)min((uint32_t)cur[start + e], (uint32_t)(n - 1));
        __syncthreads();
        for (int e = threadIdx.x; e < size; e += kOrbBlock) {
            const int v = big[e];
            int r = 0;
            for (int f = 0; f < size; ++f) r += big[f] < v;
            perm[start + r] = v;
        }
        return;
    }
    for (int e = threadIdx.x; e < size; e += kOrbBlock) {
        gid[e] = (int32_t)min((uint32_t)cur[start + e], (uint32_t)(n - 1));
        pos[e] = e;
#pragma unroll
        for (int a = 0; a < 3; ++a) skey[a][e] = keys[(size_t)a * n + start + e];
    }
    int2 *bstk = stk[kOrbBlock / 64];
    if (threadIdx.x == 0) bstk[0] = make_int2(0, size);
    __syncthreads();
    int ntask = 0;  // same value in every thread: the loop below is uniform
    int sp = 1;
    while (sp > 0) {
        --sp;
        const int2 nd = bstk[sp];
        const int lo = nd.x, m = nd.y;
        __syncthreads();  // read before the pushes below overwrite the entry
        if (m <= kWaveNode && ntask < kMaxTask) {
            // its subtree is finished by one wave below, several at once
            // (past the list's capacity the block-wide path takes them)
            if (threadIdx.x == 0) task[ntask] = make_int2(lo, m);
            ++ntask;
            continue;
        }
        if (m <= leaf) {
            block_leaf(pos, tmp, akey, gid, lo, m);
            continue;
        }
        // bounding box and axis
        uint32_t bb[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
        for (int e = threadIdx.x; e < m; e += kOrbBlock) {
            const int s = pos[lo + e];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const uint32_t v = skey[a][s];
                bb[a] = min(bb[a], v);
                bb[3 + a] = max(bb[3 + a], v);
            }
        }
        block_box(bb, red6);
        const int axis = pick_axis(bb);
        const int L = (m + leaf - 1) / leaf;
        const int k = min(m, leaf * ((L + 1) / 2));
        // the split axis's keys in node order, for the rounds and the partition
        for (int e = threadIdx.x; e < m; e += kOrbBlock) akey[e] = skey[axis][pos[lo + e]];
        // radix select of the k-th smallest key (total-order key, original
        // index), 8 bits a round; once the bin holding it holds it alone, one
        // pass reads it whole
        if (threadIdx.x == 0) {
            kth_s = 0;
            krem_s = (uint32_t)k;
            one_s = 0u;
        }
        for (int round = 0; round < 8; ++round) {
            __syncthreads();
            h[threadIdx.x] = 0u;
            const uint64_t prefix = kth_s;
            const uint32_t kr = krem_s;
            const int shift = 56 - 8 * round;
            if (one_s) {
                // the one key whose digits above `shift` are the prefix
                for (int e = threadIdx.x; e < m; e += kOrbBlock) {
                    const uint64_t key = ((uint64_t)akey[e] << 32) | (uint32_t)gid[pos[lo + e]];
                    if ((key >> (shift + 8)) == prefix) kth_s = key;
                }
                break;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < m; e += kOrbBlock) {
                // the first four digits are the coordinate key's: no index needed
                uint64_t key = (uint64_t)akey[e] << 32;
                if (round >= 4) key |= (uint32_t)gid[pos[lo + e]];
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
                one_s = hv == 1u;
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
                const int s = act ? pos[lo + e] : 0;
                // (key, index) <= kth; the index only decides between equal keys
                const uint32_t hk = akey[act ? e : 0], kh = (uint32_t)(kth >> 32);
                const bool left = act && (hk < kh || (hk == kh && (uint32_t)gid[s] <= (uint32_t)kth));
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
                    if (q < k) tmp[lo + q] = s;
                }
                if (right) {
                    const int q = dr + pr + rr;
                    if (q < m - k) tmp[lo + k + q] = s;
                }
                dl += cl;
                dr += cr;
                __syncthreads();  // wl, wr are reused by the next chunk
            }
        }
        for (int e = threadIdx.x; e < m; e += kOrbBlock) pos[lo + e] = tmp[lo + e];
        // right first so that the left child is processed next
        if (threadIdx.x == 0) {
            bstk[sp] = make_int2(lo + k, m - k);
            bstk[sp + 1] = make_int2(lo, k);
        }
        sp += 2;
        __syncthreads();
    }
    __syncthreads();
    {
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int t = w; t < ntask; t += kOrbBlock / 64) {
            const int2 tk = task[t];
            wave_subtree(pos, tmp, akey, skey, gid, hw[w], wkeys[w], wgid[w], stk[w], tk.x, tk.y, leaf, lane);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < size; e += kOrbBlock) perm[start + e] = gid[pos[e]];
}

// ---- host side --------------------------------------------------------------
struct Level {
    std::vector<int3> segs;    // (start, size, k)
    std::vector<int3> chunks;  // (segment, begin, end)
    std::vector<int2> kids;    // next-level segment of the left, right part (-1: phase B)
};

// Level l reads the index and key buffers l % 2 and writes (l + 1) % 2, so a
// segment at depth d sits in buffer d % 2: finals are (start, size, d % 2).
void plan_tree(int n, int leaf, std::vector<Level> &levels, std::vector<int3> &finals)
{
    const int cut = std::max(kSmall, leaf);
    std::vector<int2> cur = {make_int2(0, n)};
    for (int depth = 0; !cur.empty(); ++depth) {
        Level lv;
        std::vector<int2> next;
        int nid = 0;  // the next level numbers its segments in the order of `next`
        for (const int2 &s : cur) {
            if (s.y <= cut) {
                finals.push_back(make_int3(s.x, s.y, depth & 1));
                continue;
            }
            const int L = (s.y + leaf - 1) / leaf;
            const int k = std::min(s.y, leaf * ((L + 1) / 2));
            const int id = (int)lv.segs.size();
            lv.segs.push_back(make_int3(s.x, s.y, k));
            for (int b = s.x; b < s.x + s.y; b += kChunk)
                lv.chunks.push_back(make_int3(id, b, std::min(b + kChunk, s.x + s.y)));
            const int kl = k > cut ? nid++ : -1;
            const int kr = s.y - k > cut ? nid++ : -1;
            lv.kids.push_back(make_int2(kl, kr));
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
    std::vector<int3> finals;
    plan_tree(n, leaf, levels, finals);
    // one table upload: per level segs, chunks and kids, then the final
    // segments; sections start on 16-byte boundaries (int2 entries need
    // 8-byte alignment)
    std::vector<char> tab;
    auto pad = [&tab]() { tab.resize((tab.size() + 15) & ~size_t(15), 0); };
    auto put = [&tab, &pad](const void *p, size_t bytes) {
        const size_t at = tab.size();
        tab.insert(tab.end(), (const char *)p, (const char *)p + bytes);
        pad();
        return at;
    };
    struct Off {
        size_t segs, chunks, kids;
    };
    std::vector<Off> off;
    size_t maxseg = 1;
    for (const Level &lv : levels) {
        Off o;
        o.segs = put(lv.segs.data(), lv.segs.size() * sizeof(int3));
        o.chunks = put(lv.chunks.data(), lv.chunks.size() * sizeof(int3));
        o.kids = put(lv.kids.data(), lv.kids.size() * sizeof(int2));
        off.push_back(o);
        maxseg = std::max(maxseg, lv.segs.size());
    }
    const size_t foff = put(finals.data(), finals.size() * sizeof(int3));
    const size_t nbytes = (size_t)n * 4;
    // two buffers of the three axes' keys in the current order (each level
    // reads one and writes the other), then the tie pass's candidates
    uint32_t *kmem = (uint32_t *)scratch(kSlotOrb0, 7 * nbytes);
    // original index per position, same two-buffer scheme as the keys
    int32_t *cbuf[2] = {(int32_t *)scratch(kSlotOrb1, nbytes), (int32_t *)scratch(kSlotOrb2, nbytes)};
    char *dtab = (char *)scratch(kSlotOrb3, tab.size() + 16);
    // states of two levels (the partition fills in the next one's), then one
    // histogram row per segment
    const size_t stbytes = (maxseg * sizeof(SegState) + 63) & ~size_t(63);
    char *state = (char *)scratch(kSlotOrb4, 2 * stbytes + maxseg * kBins * 4 + 64);
    if (!kmem || !cbuf[0] || !cbuf[1] || !dtab || !state) {
        set_error("cannot allocate ORB scratch");
        return NBODY_E_NOMEM;
    }
    uint32_t *kbuf[2] = {kmem, kmem + 3 * (size_t)n};
    uint32_t *cand = kmem + 6 * (size_t)n;  // tied bodies' indices (k_orb_ties)
    SegState *st[2] = {(SegState *)state, (SegState *)(state + stbytes)};
    uint32_t *hist = (uint32_t *)(state + 2 * stbytes);
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
        hipLaunchKernelGGL(k_orb_coords<double4>, dim3(nb), dim3(kOrbBlock), 0, s, (const double4 *)pm, n,
                           kbuf[0], cbuf[0]);
    else
        hipLaunchKernelGGL(k_orb_coords<float4>, dim3(nb), dim3(kOrbBlock), 0, s, (const float4 *)pm, n,
                           kbuf[0], cbuf[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ORB coordinates");
    for (size_t l = 0; l < levels.size(); ++l) {
        const int nseg = (int)levels[l].segs.size(), nch = (int)levels[l].chunks.size();
        const int3 *segs = (const int3 *)(dtab + off[l].segs);
        const int3 *chunks = (const int3 *)(dtab + off[l].chunks);
        const int2 *kids = (const int2 *)(dtab + off[l].kids);
        const bool more = l + 1 < levels.size();
        const int3 *segs_next = more ? (const int3 *)(dtab + off[l + 1].segs) : nullptr;
        const int nseg_next = more ? (int)levels[l + 1].segs.size() : 0;
        const int i = (int)(l & 1), o = 1 - i;
        if (l == 0) {
            hipLaunchKernelGGL(k_orb_init, dim3((unsigned)maxseg), dim3(kOrbBlock), 0, s, segs, nseg, st[i], hist);
            hipLaunchKernelGGL(k_orb_bbox, dim3(nch), dim3(kOrbBlock), 0, s, chunks, kbuf[i], n, st[i]);
        }
        for (int r = 0; r < kCoordRounds; ++r)
            hipLaunchKernelGGL(k_orb_hist, dim3(nch), dim3(kPassBlock), 0, s, chunks, segs, kbuf[i], n, cbuf[i],
                               st[i], hist, r, segs_next, nseg_next, st[o]);
        hipLaunchKernelGGL(k_orb_ties, dim3(nch), dim3(kPassBlock), 0, s, chunks, segs, kbuf[i], n, cbuf[i], st[i],
                           cand);
        hipLaunchKernelGGL(k_orb_partition, dim3(nch), dim3(kPassBlock), 0, s, chunks, segs, kids, kbuf[i], kbuf[o],
                           n, cbuf[i], cbuf[o], st[i], st[o]);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "ORB level");
    }
    hipLaunchKernelGGL(k_orb_block, dim3((unsigned)finals.size()), dim3(kOrbBlock), 0, s,
                       (const int3 *)(dtab + foff), kbuf[0], kbuf[1], cbuf[0], cbuf[1], n, leaf, perm);
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
