// Internal declarations of the gfx950 n-body library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "nbody.h"

namespace nbi {

// Kernel shape of the force sweep.
//   tpl    targets held per lane (1, 2 or 4): a wave owns 64*tpl targets
//   jsplit number of independent source ranges per target (1..32); each
//          range is a separate workgroup row, reduced in fixed order after
//   jtile  sources per partial sum (multiple of 8); the partials are folded
//          into the running sum by the precision mode
//   variant 0: sources through scalar loads (SGPR operands);
//           1: sources staged in LDS (VGPR operands; FP32 force kernel only,
//              jtile a multiple of 256).  Both give identical results.
struct Tune {
    int tpl = 2;
    int jsplit = 1;
    int jtile = 512;
    int variant = 0;
};

constexpr int kBlock = 256;  // threads per workgroup: four independent waves
constexpr int kUnroll = 8;   // sources per unrolled step of the sweep

// Returns x in a vector register that the compiler treats as per-lane, so a
// loop invariant such as eps^2 is not kept as a scalar operand of the pair
// arithmetic: on gfx950 an FP32 VALU instruction that reads a scalar register
// issues at roughly half the rate of its all-vector-register form.
__device__ __forceinline__ float lane_copy(float x)
{
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

bool tune_valid(const Tune &t);

// ---- force (accel.hip) -----------------------------------------------------
// pm: float4/double4 records; out: target_count records; partial: scratch of
// jsplit * target_count double4 (F32 mode: float4) records when jsplit > 1.
// reduce = false leaves a split result in `partial` (out untouched) for a
// consumer that reduces it itself (launch_reduce_step).
hipError_t launch_accel(int prec, const void *pm, int n, double G, double eps, void *out,
                        int tbeg, int tcount, const Tune &t, void *partial, hipStream_t s,
                        bool reduce = true);
size_t accel_partial_bytes(int prec, int tcount, const Tune &t);

// Split partials of nbody_accel_noalloc: a file-scope device array in
// accel.hip of kStaticScratchBytes.  static_split_scratch() returns its
// address on the current device (looked up once per device), or nullptr with
// the error set.
constexpr size_t kStaticScratchBytes = NBODY_NOALLOC_SCRATCH;
void *static_split_scratch();

// Batched force over a work list of (system, first target) units sorted
// longest first.  units: int2[nunits] = (system, target offset within the
// system); offsets: int64 device copy [nsys+1]; counter: one zeroed uint32
// pair, left zeroed again by the kernel on exit.
hipError_t launch_batched(int prec, const void *pm, const int64_t *offsets, const int2 *units,
                          int nunits, double G, const float *eps_sys, double eps, void *out,
                          const Tune &t, unsigned *counter, int grid, hipStream_t s);

// ---- fused force + VJP (vjp.hip) -------------------------------------------
// partial: scratch of vjp_partial_bytes(n, t) when t.jsplit > 1.
hipError_t launch_vjp(int prec, const void *pm, const void *cot, int n, double G, double eps,
                      void *pos_cot, void *mass_cot, void *acc_out, const Tune &t, void *partial,
                      hipStream_t s);
// scale multiplies the cotangent; accumulate adds into pos_cot/mass_cot;
// phi = false ignores the phibar component of the cotangent records.
hipError_t launch_vjp_ex(int prec, const void *pm, const void *cot, int n, double G, double eps,
                         bool phi, double scale, bool accumulate, void *pos_cot, void *mass_cot,
                         void *acc_out, const Tune &t, void *partial, hipStream_t s);
size_t vjp_partial_bytes(int n, const Tune &t);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);

// ---- elementwise steps (step.hip) ------------------------------------------
// One pass between two force evaluations:
//   close: v += h a          (closing kick of the previous step)
//   energy partials of (v, phi) after the closing kick, if epart != nullptr
//   open:  v += h a; x += dt v  (opening kick and drift of the next step)
hipError_t launch_step(int prec, void *pm, void *vel, const void *acc, int n, double h, double dt,
                       bool close, bool open, double *epart, int *eblocks, hipStream_t s);
int step_blocks(int n);
// Split reduction of the force (js partial records per body, as left by
// launch_accel(..., reduce = false) for all n targets) fused with the step:
// acc receives the reduced force, then the kick/drift of launch_step runs.
hipError_t launch_reduce_step(int prec, const void *partial, int js, double G, void *pm, void *vel,
                              void *acc, int n, double h, double dt, bool close, bool open,
                              double *epart, int *eblocks, hipStream_t s);
hipError_t launch_energy_final(const double *epart, int nblocks, double *out, hipStream_t s);
hipError_t launch_permute(const void *src, void *dst, const int32_t *perm, int n, int rec_bytes,
                          bool inverse, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);

// Reverse leapfrog step by time reversal plus vbar += dt xbar, refreshing the
// scaled cotangent vsc = vbar / m (vjp.hip).
hipError_t launch_reverse_step(int prec, void *x, void *vh, const void *acc, const void *xbar,
                               void *vbar, void *vsc, int n, double hk, double dt, hipStream_t s);
// y += a x and ysc = y / m (m from the records pm) (vjp.hip).
hipError_t launch_adj_axpy(int prec, void *y, const void *x, double a, const void *pm, void *ysc,
                           int n, hipStream_t s);
// sc = cot / m; *nonpos |= (some m <= 0).  *nonpos must be zero before.
// dst = (0, 0, 0, src.w) per record (the potential part of a cotangent).
hipError_t launch_phibar_only(int prec, const void *src, int n, void *dst, hipStream_t s);
hipError_t launch_prescale(int prec, const void *cot, const void *pm, int n, void *sc, int *nonpos,
                           hipStream_t s);
// Adjoint VJP (phibar = 0, accumulate): mass-scaled form on sc unless
// *nonpos, then the general form on raw.
hipError_t launch_vjp_adj(int prec, const void *pm, const void *raw, const void *sc,
                          const int *nonpos, int n, double G, double eps, double scale,
                          void *pos_cot, void *mass_cot, void *acc_out, const Tune &t, void *partial,
                          hipStream_t s);
// Adjoint VJP and the elementwise step after it in as few launches as the
// shape allows (post 1: vbar += dt xbar; post 2: time reversal of x, vh;
// post 3: as post 1, and the force to acc).  Uses tpl = 1 when the source
// range is split.
hipError_t launch_vjp_adj_step(int prec, int post, void *pm, void *raw, void *sc, const int *nonpos,
                               int n, double G, double eps, double scale, void *pos_cot,
                               void *mass_cot, void *acc, void *vh, double hk, double dt,
                               const Tune &t, void *partial, hipStream_t s);

// ---- ORB (orb.hip) -----------------------------------------------------------
int orb_order(const void *pm, int prec, int n, int leaf, int32_t *perm, hipStream_t s);
void orb_release();

// ---- tree code (tree.hip) ----------------------------------------------------
int tree_shape(int n, int leaf, int64_t *num_nodes, int64_t *num_groups, int32_t *nodes_out);
int tree_moments(const void *pm, int n, int leaf, double *mom, float *box, hipStream_t s);
int tree_lists(const void *pm, int n, int leaf, double theta, int max_far, int max_near, int32_t *far_cnt,
               int32_t *near_cnt, int32_t *far_ids, int32_t *near_ids, hipStream_t s);
int tree_accel(const void *pm, int n, int prec, double G, double eps, double theta, int leaf, int cells,
               void *out, hipStream_t s);
int tree_pseudo(const void *pm, int n, int leaf, void *out, hipStream_t s);
int tree_quad(const void *pm, int n, int leaf, void *out, hipStream_t s);
int tree_local_counts(const void *pm, int n, int leaf, double theta, int32_t *loc_cnt, int32_t *far_cnt,
                      int32_t *near_cnt, hipStream_t s);
int tree_leapfrog(void *pm, void *vel, void *acc, int32_t *order, int n, int prec, double G, double eps,
                  double theta, int leaf, double dt, int nsteps, int reorder_every, unsigned flags,
                  double *energy, hipStream_t s);
void tree_release();

// ---- multi-level FMM (fmm.hip) ------------------------------------------------
// pm: n float4 records in ORB order (leaf as given).  fmm_accel writes n
// records (ORB order); synchronises s once to check the list buffers.
int fmm_accel(const void *pm, int n, int prec, double G, double eps, double theta, int leaf, void *out,
              hipStream_t s);
// fmm_lists: per-node counts and concatenated source ids of the (M2L, M2P,
// P2P) lists, grouped by target node (device outputs; ids_out entries may be
// NULL to count only).
int fmm_lists(const void *pm, int n, int leaf, double theta, int32_t *const cnt_out[3], int32_t *const ids_out[3],
              const int64_t caps[3], hipStream_t s);
void fmm_release();

// ---- bit-reversible fixed-point leapfrog (janus.hip) ---------------------------
// state: 2n longlong4 (X then V); the force kernel and the fused VJP run with
// G = 1 and the shape of janus_tune so their forces agree bit for bit.
Tune janus_tune(const Tune &vjp_default);
int janus_forward(const void *pm, const void *vel, int n, double G, double eps, double dt, int nsteps, int sx,
                  int sv, const Tune &t, void *state, void *pm_out, void *vel_out, void *acc, void *partial,
                  hipStream_t s);
int janus_decode(const void *state, const void *pm, int n, int sx, void *dec, hipStream_t s);
int janus_unstep(void *state, const void *acc, int n, double G, double dt, int sx, int sv, int kicks, int drift,
                 void *dec, hipStream_t s);

// ---- runtime helpers (runtime.hip) -----------------------------------------
void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
// Library scratch, one growable buffer per slot and device.
enum ScratchSlot { kSlotPartial = 0, kSlotEnergy, kSlotBatch, kSlotOrb0, kSlotOrb1, kSlotOrb2,
                   kSlotOrb3, kSlotOrb4, kSlotAdj0, kSlotAdj1, kSlotAdj2, kSlotAdj3, kSlotAdj4, kSlotTune,
                   kNumSlots };
void *scratch(int slot, size_t bytes);

}  // namespace nbi
