/*
 * nbody.h -- C ABI of the MI355X (gfx950) direct-sum n-body library.
 *
 * The library computes the hot path of the n-body simulation in Duy,
 * Yamazaki, Ikegami and Oyanagi, "Hybrid MPI-OpenMP Paradigm on SMP clusters:
 * MPEG-2 Encoder and n-body Simulation": the force calculation that the
 * paper's Section IV.B says takes upwards of 90% of the cycles, evaluated
 * exactly (every body against every other body, the limit of the tree code of
 * Section IV.A with every cell opened), and the position/velocity update
 * around it (Move_bodies in the Section IV.B pseudo-code).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers are DEVICE pointers unless the parameter says "host".  The
 *   caller owns every buffer passed in.  The library owns only internal
 *   scratch (released by nbody_release()).
 * - Body records are 4-vectors, array-of-structures:
 *     pos_mass  (x, y, z, m)        float4 (FP32 modes) or double4 (NBODY_F64)
 *     vel       (vx, vy, vz, unused)
 *     acc_pot   (ax, ay, az, phi)   the output of the force evaluation
 *   float4 buffers must be 16-byte aligned, double4 buffers 32-byte aligned.
 *   Buffers that a call writes must not share memory with the buffers it
 *   reads or with each other (arrays updated in place, such as the
 *   integrators' pos_mass, vel and acc_pot, are mutually disjoint); calls
 *   refuse such arguments with NBODY_E_INVAL.
 * - Law (Section IV; G and Plummer softening eps are parameters):
 *     a_i   =  G sum_{j != i} m_j (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^(3/2)
 *     phi_i = -G sum_{j != i} m_j / (|x_j - x_i|^2 + eps^2)^(1/2)
 *   The self pair j == i is excluded from both sums.  eps = 0 is allowed;
 *   then two distinct bodies at the same position give IEEE inf/NaN.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Every call is stream-ordered and asynchronous: it validates its
 *   arguments on the host, enqueues kernels and returns.  No call below
 *   synchronises the device except nbody_autotune(), nbody_release(), a
 *   tree call for a new (n, leaf) (it uploads the node table),
 *   nbody_janus_adjoint (its mass check), nbody_orb_order when
 *   NBODY_CHECK_INPUTS is set, and the FMM calls (one stream
 *   synchronisation each, to check their list buffers).
 * - Library scratch is one buffer per purpose and device, shared by all
 *   streams.  A call that needs more than any earlier one allocates a larger
 *   buffer (a power of two in size) and does not wait: the one it replaces
 *   may still be read by enqueued work or by a captured graph, so it stays
 *   allocated until nbody_release().  Calls that share library scratch (the
 *   same entry point on one device, or the entry points that share a
 *   purpose: force, VJP and the integrators' partial sums) must not run
 *   concurrently on different streams.
 * - A caller may capture calls into its own HIP graph after one eager call
 *   of the same shapes (which allocates the scratch and tables they use).
 *   The graph stays valid until a tree call changes (n, leaf) or
 *   nbody_release() runs.
 * - Return value: NBODY_OK (0) or a negative status.  On a validation error
 *   nothing has been enqueued.  nbody_last_error() gives a thread-local
 *   message for the last failing call.  The library never aborts or exits.
 * - Sizes: 1 <= n <= 2^31 - 4096.  Non-finite positions or masses are a
 *   precondition violation (results then unspecified).
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic of the force evaluation. */
typedef enum {
    NBODY_F64 = 0,        /* FP64 state, FP64 pair arithmetic and sums          */
    NBODY_F32 = 1,        /* FP32 pair arithmetic, FP32 per-tile partial sums,
                             plain FP32 sum across tiles                       */
    NBODY_F32_KAHAN = 2,  /* FP32 pair arithmetic, FP32 per-tile partial sums,
                             Kahan-compensated FP32 sum across tiles           */
    NBODY_F32_F64ACC = 3  /* FP32 pair arithmetic, FP32 per-tile partial sums,
                             FP64 sum across tiles                             */
} nbody_prec;

enum {
    NBODY_OK = 0,
    NBODY_E_INVAL = -1,       /* bad size, pointer, enum or non-finite scalar */
    NBODY_E_ALIGN = -2,       /* a vector buffer is not naturally aligned     */
    NBODY_E_NOMEM = -3,       /* library scratch could not be allocated       */
    NBODY_E_HIP = -4,         /* a HIP call failed (see nbody_last_error)     */
    NBODY_E_UNSUPPORTED = -5  /* valid but unsupported combination            */
};

/* Flags of nbody_leapfrog_kdk. */
#define NBODY_ACC_VALID 0x1u /* acc_pot already holds a(x) at the input state */
#define NBODY_GRAPH 0x2u     /* capture the step loop in a HIP graph, reuse it */
#define NBODY_ENERGY 0x4u    /* write FP64 energies to energy_out             */

/*
 * Orthogonal Recursive Bisection order (Section IV.B: divide space into
 * non-overlapping sub-spaces with about equal numbers of bodies), used here
 * as a body ordering on one device: leaves of at most `leaf` spatially close
 * bodies become contiguous.
 *   ORB(S): if |S| <= leaf, S by ascending original index.  Otherwise split
 *   on the axis of largest FP32 extent fl32(max - min) (ties: x, then y, then
 *   z); keys (IEEE total order of the FP32 coordinate, original index); the
 *   left part is the k = leaf * ceil(ceil(|S|/leaf) / 2) smallest keys; emit
 *   ORB(left) then ORB(right).  Coordinates of NBODY_F64 input are rounded to
 *   FP32 first.  The result is a pure function of the input (bit-exact).
 * pos_mass: n records (float4 or double4 by prec).  perm_out: int32[n],
 * perm_out[p] = original index of the body at position p.  Uses library
 * scratch of about 36 bytes per body.  Non-finite coordinates make the order
 * unspecified; with the environment variable NBODY_CHECK_INPUTS set (to
 * anything but "0") the call first checks every record, synchronises the
 * stream, and refuses non-finite coordinates or masses with NBODY_E_INVAL
 * (the message names the first such record).
 */
int nbody_orb_order(const void *pos_mass, int32_t prec, int64_t n, int32_t leaf,
                    int32_t *perm_out, void *stream);

/*
 * Gather or scatter of 16- or 32-byte records through a permutation:
 *   inverse == 0: dst[p] = src[perm[p]]   (apply an ORB order)
 *   inverse != 0: dst[perm[p]] = src[p]   (return results to input order)
 * rec_bytes is 16 or 32.  src and dst must not overlap.  perm should hold
 * every index of [0, n) once; an entry outside [0, n) is skipped (no record is
 * read or written for it), so the record it would have produced is left as
 * it was.
 */
int nbody_permute(const void *src, void *dst, const int32_t *perm, int64_t n,
                  int32_t rec_bytes, int32_t inverse, void *stream);

/*
 * Force and potential (the paper's Calculate_forces, Section IV.B, with every
 * body on every interaction list) for targets [target_begin,
 * target_begin + target_count) against all n sources.
 * acc_pot_out: target_count records, entry t for target target_begin + t;
 * it must not overlap pos_mass.  Deterministic: the same inputs and tuning
 * give bitwise the same output.
 */
int nbody_accel(const void *pos_mass, int64_t n, int32_t prec, double G, double eps,
                void *acc_pot_out, int64_t target_begin, int64_t target_count, void *stream);

/*
 * nbody_accel for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and validation as nbody_accel; it calls no hipMalloc, hipFree or
 * other allocating routine.  When the kernel shape splits the source range
 * (jsplit > 1) the per-split partial records (jsplit * target_count records
 * of 32 bytes; 16 in NBODY_F32) go to a file-scope device array of
 * NBODY_NOALLOC_SCRATCH bytes (64 MiB) that each GPU the library runs on
 * holds until the process ends.
 *   - If the partials of nbody_accel's shape fit, the same shape runs and the
 *     result equals nbody_accel's bit for bit.
 *   - If they do not fit and the shape was chosen by the library (default or
 *     autotuned), the split count is halved until they fit (one split needs
 *     no scratch): the partial sums are then grouped differently, within the
 *     same error bound.
 *   - If they do not fit and the shape was pinned with nbody_set_tuning, the
 *     call returns NBODY_E_INVAL before anything is enqueued, with the sizes
 *     in nbody_last_error().
 * Every call on a GPU shares that GPU's array: calls that overlap in time on
 * one GPU (different streams or threads) race and must be ordered by the
 * caller.  Nothing in the array needs clearing: each call writes every
 * record it reads.
 */
#define NBODY_NOALLOC_SCRATCH (64u << 20)
int nbody_accel_noalloc(const void *pos_mass, int64_t n, int32_t prec, double G, double eps,
                        void *acc_pot_out, int64_t target_begin, int64_t target_count,
                        void *stream);

/*
 * Fused force + vector-Jacobian product at one configuration (derivative of
 * the law above; the paper has no derivatives).  Given cotangents
 * acc_pot_cot = (abar, phibar) per body, writes
 *   pos_cot_out[k]  = xbar_k = sum_i (da_i/dx_k)^T abar_i + (dphi_i/dx_k) phibar_i
 *                     (record (x, y, z, 0))
 *   mass_cot_out[k] = mbar_k = sum_i abar_i . da_i/dm_k + phibar_i dphi_i/dm_k
 *                     (float or double by prec)
 *   acc_pot_out     = the forward force, if not NULL.
 * All outputs have n entries and must not overlap the inputs.
 */
int nbody_accel_vjp(const void *pos_mass, const void *acc_pot_cot, int64_t n, int32_t prec,
                    double G, double eps, void *pos_cot_out, void *mass_cot_out,
                    void *acc_pot_out, void *stream);

/*
 * nsteps of kick-drift-kick leapfrog with one force evaluation per step
 * (Move_bodies after Calculate_forces, Section IV.B), h = dt / 2:
 *   v += h a(x);  x += dt v;  a = a(x);  v += h a
 * pos_mass, vel, acc_pot are updated in place (acc_pot ends as a(x_final)).
 * Unless flags has NBODY_ACC_VALID, a(x) is evaluated first.
 * offsets_host (host, int64[nsys+1], NULL for one system): independent
 * systems stored back to back, offsets[0] = 0, offsets[nsys] = n,
 * nondecreasing; forces act only within a system.
 * NBODY_ENERGY: energy_out (device, double[(nsteps+1)*2]) receives
 * (K, U) = (1/2 sum m|v|^2, 1/2 sum m phi) in FP64 after each step, entry 0
 * at the input state (one system only).
 * NBODY_GRAPH: the whole step loop is captured once into a HIP graph keyed by
 * (pointers, sizes, scalars, flags) and replayed on later identical calls.
 */
int nbody_leapfrog_kdk(void *pos_mass, void *vel, void *acc_pot, int64_t n,
                       const int64_t *offsets_host, int32_t nsys, int32_t prec, double G,
                       double eps, double dt, int32_t nsteps, uint32_t flags,
                       double *energy_out, void *stream);

/*
 * The elementwise half of one leapfrog step, for callers that drive the loop
 * themselves (nbody_leapfrog_kdk is nbody_accel plus this):
 *   close != 0: v += h a             (closing kick with a = acc_pot)
 *   open  != 0: v += h a; x += dt v  (opening kick and drift)
 * Both may be set (closing kick of one step, then opening kick and drift of
 * the next, h = dt/2 for both).  pos_mass and vel are updated in place.
 */
int nbody_kick_drift(void *pos_mass, void *vel, const void *acc_pot, int64_t n, int32_t prec,
                     double h, double dt, int32_t close, int32_t open, void *stream);

/*
 * Force and potential of nsys independent systems stored back to back
 * (offsets_host as above) in one persistent launch over a longest-first
 * work list of (system, target tile) units.  eps_per_sys: device float[nsys]
 * or NULL to use `eps` for all.  Each system's result is bitwise the result
 * of nbody_accel on that system alone with the same tuning.
 */
int nbody_batched_accel(const void *pos_mass, const int64_t *offsets_host, int32_t nsys,
                        int32_t prec, double G, const float *eps_per_sys, double eps,
                        void *acc_pot_out, void *stream);

/*
 * FP64 energy diagnostics of one system: energy_out (device, double[2]) =
 * (K, U) with K = 1/2 sum m |v|^2 and U = 1/2 sum m phi (phi from acc_pot).
 * Deterministic fixed-order reduction.
 */
int nbody_energy(const void *pos_mass, const void *vel, const void *acc_pot, int64_t n,
                 int32_t prec, double *energy_out, void *stream);

/*
 * Leapfrog trajectory with checkpoints, and its adjoint.
 * nbody_trajectory_forward runs nsteps of nbody_leapfrog_kdk from
 * (pos_mass, vel) in place and stores (pos_mass, vel) every ckpt_every steps
 * into ckpt (device), slot c holding step c*ckpt_every for
 * c = 0..nsteps/ckpt_every: slot size 2 records per body.  nsteps must be a
 * multiple of ckpt_every.
 * nbody_trajectory_adjoint takes the cotangents (xbar_T, vbar_T) of the
 * final positions and velocities (records; w unused unless scheme includes
 * NBODY_ADJ_PHI, see below) and returns the
 * gradients with respect to the initial positions (pos_cot, record x,y,z),
 * velocities (vel_cot) and masses (mass_cot, float/double[n]), applying one
 * force VJP per position x_n with cotangent h vbar (first and last) or
 * 2h vbar (interior).  The positions come from
 *   NBODY_ADJ_RECOMPUTE: re-running each segment forward from its checkpoint
 *                        (exactly the forward positions; one extra force
 *                        evaluation per step), or
 *   NBODY_ADJ_REVERSE:   running the leapfrog backwards from the end of each
 *                        segment (x_n = x_{n+1} - dt v_{n+1/2}) with the force
 *                        returned by the fused VJP kernel, re-anchored at every
 *                        checkpoint (no extra force evaluation; positions
 *                        differ from the forward ones by rounding).
 * xbar_T / vbar_T are read only.
 */
int nbody_trajectory_forward(void *pos_mass, void *vel, int64_t n, int32_t prec, double G,
                             double eps, double dt, int32_t nsteps, int32_t ckpt_every,
                             void *ckpt, void *stream);
#define NBODY_ADJ_RECOMPUTE 0
#define NBODY_ADJ_REVERSE 1
/* OR-ed into scheme: the w components of xbar_T hold phibar_T, the cotangent
 * of the final potential phi(x_T) of the same softened law (one more
 * general-form VJP at x_T).  Without it the w components are ignored. */
#define NBODY_ADJ_PHI 0x10
int nbody_trajectory_adjoint(const void *ckpt, int64_t n, int32_t prec, double G, double eps,
                             double dt, int32_t nsteps, int32_t ckpt_every,
                             const void *xbar_T, const void *vbar_T, void *pos_cot,
                             void *vel_cot, void *mass_cot, int32_t scheme, void *stream);

/*
 * Tree code on the ORB cells (Section IV.A: a distant group of bodies acts as
 * one body of its total mass at its centre of mass; the distant cells are
 * found by a walk from the root, the force sums over them and the remaining
 * nearby bodies.  The cells are the nodes of the Section IV.B ORB recursion).
 *
 * Input: pos_mass, n float4 records (x, y, z, m), m >= 0, ALREADY IN ORB
 * ORDER for the same `leaf` (nbody_orb_order, then a gather such as
 * nbody_permute).  Node k of the tree is then the range of positions
 * [begin, end); a node of more than `leaf` bodies has the children
 * [begin, begin + k) and [begin + k, end), k = leaf * ceil(ceil(size/leaf)/2).
 * Nodes are numbered in preorder (node, left subtree, right subtree).
 * Targets are taken in groups, the maximal nodes of at most
 * NBODY_TREE_GROUP bodies, in ORB order.
 * Moments, in FP64 from the FP32 records: a leaf sums m and m*x over its
 * bodies in position order from 0 (each product rounded, then added), an inner
 * node adds left + right; com = S / M, or the box centre 0.5 (lo + hi) if
 * M = 0; lo/hi are the exact coordinate minima/maxima; diag2 = sum over
 * x, y, z of (hi - lo)^2.  Opening: cell c is accepted for group g iff c and
 * g share no body and diag2_c < theta^2 * D2, D2 the squared distance from
 * com_c to the box of g (per axis lo - com if com < lo, com - hi if com > hi,
 * else 0, summed x, y, z; all in FP64): the cell's size over its distance is
 * then below theta for every target of the group.  An accepted cell acts as
 * one body (com and M rounded to FP32) under the same softened law; a leaf
 * that is not accepted acts body by body; the group's own bodies act body by
 * body without the self pair.  theta = 0 accepts nothing: the exact direct
 * sum.  Decisions are bit-exact against an FP64 implementation of these
 * definitions.
 * 1 <= leaf <= NBODY_TREE_GROUP.  The first call for a new (n, leaf)
 * uploads the node table and synchronizes the stream; later calls are
 * asynchronous.  The tree tables are library scratch (about 430 bytes per
 * node) shared by all tree calls on a device: overlapping calls race.
 * With group local expansions (NBODY_CELLS_LOCAL) and 8192 groups or more,
 * the groups whose boxes are among the largest 1/16 (by a histogram of
 * diag2) are walked first, since their walks cost several times the mean;
 * the environment variable NBODY_TREE_ORDER=0 keeps ORB order.  The results
 * do not depend on the order.
 *
 * Cell models (the acceptance test and the interaction lists are the same
 * for all three):
 * NBODY_CELLS_MONOPOLE: an accepted cell acts as one body (above).
 * NBODY_CELLS_PSEUDO (order 2 by pseudo-particle multipoles: Makino,
 *   J. Comput. Phys. 151, 1999, the paper's reference [20], which Section
 *   VI cites for the O(N) fast multipole method): the cell acts as NBODY_TREE_PSEUDO point masses q_j at
 *   com + a s_j whose multipole expansion about com equals the cell's
 *   through the quadrupole term.  s_j: the unit vertices of the icosahedron,
 *   (0, u, v g), (u, v g, 0), (u g, 0, v) over sqrt(1 + g^2), g the golden
 *   ratio, (u, v) = (+,+), (+,-), (-,+), (-,-), j = 0..11 in that order;
 *   a = sqrt(diag2) / 2; q_j = M/12 + 5/(24 a^2) (3 s_j.S.s_j - trace S),
 *   S = sum m r r^T over the cell's bodies, r = x - com, in FP64
 *   (q_j = M/12 when a = 0).
 * NBODY_CELLS_QUADRUPOLE: the same expansion through l = 2 evaluated
 *   directly: with Q = 3 S - trace(S) I (FP64, rounded to FP32), d = x - com
 *   and s^2 = |d|^2 + eps^2, phi = -G (M/s + d.Q.d / (2 s^5)) and
 *   a = G (-M d/s^3 + Q d/s^5 - 5 (d.Q.d) d / (2 s^7)).  The same accuracy
 *   as the pseudo-particles for a fraction of the work.
 * NBODY_CELLS_LOCAL (the fast multipole method's M2L and L2P steps, at the
 *   level of the target groups): a cell c with diag2_c + diag2_g <
 *   theta^2 |com_c - z_g|^2 (z_g = the group's centre of mass, in FP64)
 *   enters the group's third-order Taylor expansion, about z_g, of the
 *   quadrupole cell's potential (one order above the cells', so that the
 *   force keeps their third-order error); each target evaluates that
 *   expansion at its own position.  Other cells are tested and evaluated as
 *   for NBODY_CELLS_QUADRUPOLE.  The local test bounds the combined
 *   size-to-distance ratio of cell and group by sqrt(2) theta.
 *
 * nbody_tree_shape (host only): node and group counts; nodes_out, if not
 *   NULL, receives int32[num_nodes][4] = (begin, end, left, right), -1
 *   children for a leaf.
 * nbody_tree_accel: acc_pot_out = n float4 (ax, ay, az, phi) in ORB order.
 *   prec: NBODY_F32, NBODY_F32_KAHAN or NBODY_F32_F64ACC (how the partial
 *   sums of each batch of cells or ranges are folded); NBODY_F64 is
 *   unsupported.  eps >= 0, theta >= 0 finite.
 * nbody_tree_accel_cells: the same with a cell model, NBODY_CELLS_*; other
 *   values are NBODY_E_INVAL.
 * nbody_tree_pseudo (inspection): pseudo_out = float4[num_nodes][12] =
 *   (x, y, z, q) of every node's pseudo-particles (positions and masses
 *   rounded to FP32).
 * nbody_tree_quad (inspection): quad_out = float4[num_nodes][3] =
 *   (com, M), (Qxx, Qyy, Qzz, Qxy), (Qxz, Qyz, 0, 0) in FP32.
 * nbody_tree_local_counts (inspection): per group, the numbers of cells in
 *   the local expansion (loc_count), of cells evaluated per target
 *   (far_count) and of rejected leaves outside the group (near_count) in
 *   the NBODY_CELLS_LOCAL walk.
 * nbody_tree_moments (inspection): moments_out double[num_nodes][5] =
 *   (M, com_x, com_y, com_z, diag2), box_out float[num_nodes][6] =
 *   (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z); either may be NULL.
 * nbody_tree_lists (inspection): for every group, the number of accepted
 *   cells (far_count[g]) and of rejected leaves outside the group
 *   (near_count[g]), and their node ids, in walk order, in
 *   far_ids[g * max_far + ...] and near_ids[g * max_near + ...] (NULL for
 *   counts only; lists longer than the maximum are cut, the counts are not).
 * Device pointers for all arrays except nodes_out.
 */
/*
 * nbody_tree_leapfrog: nsteps kick-drift-kick steps (as nbody_leapfrog_kdk)
 * with tree forces.  pos_mass, vel, acc_pot: n float4 records in the ORB
 * order of `leaf`.  reorder_every = K > 0 puts the state into the ORB order
 * of its current positions at entry and again before the force evaluation of
 * every K-th step (x, v and a move with their bodies), and composes
 * order[p] (int32[n], device, caller-initialized, e.g. to the identity) so
 * that it keeps naming the caller's index of the body at position p;
 * K = 0 never re-orders (order may be NULL).  flags: NBODY_ACC_VALID,
 * NBODY_ENERGY (energy_out as for nbody_leapfrog_kdk, with the tree
 * potential), NBODY_TREE_PSEUDO_CELLS, NBODY_TREE_QUAD_CELLS or
 * NBODY_TREE_LOCAL_CELLS (the cell model; monopole without any, two or more
 * are NBODY_E_INVAL).
 * Re-ordering uses library scratch of about 24 bytes per body.
 */
#define NBODY_TREE_GROUP 64
#define NBODY_TREE_PSEUDO 12
#define NBODY_CELLS_MONOPOLE 0
#define NBODY_CELLS_PSEUDO 2
#define NBODY_CELLS_QUADRUPOLE 3
#define NBODY_CELLS_LOCAL 4
#define NBODY_TREE_PSEUDO_CELLS 0x8u /* nbody_tree_leapfrog flags */
#define NBODY_TREE_QUAD_CELLS 0x20u
#define NBODY_TREE_LOCAL_CELLS 0x40u
int nbody_tree_shape(int64_t n, int32_t leaf, int64_t *num_nodes, int64_t *num_groups,
                     int32_t *nodes_out);
int nbody_tree_accel(const void *pos_mass, int64_t n, int32_t prec, double G, double eps,
                     double theta, int32_t leaf, void *acc_pot_out, void *stream);
int nbody_tree_accel_cells(const void *pos_mass, int64_t n, int32_t prec, double G, double eps,
                           double theta, int32_t leaf, int32_t cells, void *acc_pot_out,
                           void *stream);
int nbody_tree_pseudo(const void *pos_mass, int64_t n, int32_t leaf, void *pseudo_out,
                      void *stream);
int nbody_tree_quad(const void *pos_mass, int64_t n, int32_t leaf, void *quad_out, void *stream);
int nbody_tree_local_counts(const void *pos_mass, int64_t n, int32_t leaf, double theta,
                            int32_t *loc_count, int32_t *far_count, int32_t *near_count,
                            void *stream);
int nbody_tree_moments(const void *pos_mass, int64_t n, int32_t leaf, double *moments_out,
                       float *box_out, void *stream);
int nbody_tree_lists(const void *pos_mass, int64_t n, int32_t leaf, double theta,
                     int32_t max_far, int32_t max_near, int32_t *far_count, int32_t *near_count,
                     int32_t *far_ids, int32_t *near_ids, void *stream);
int nbody_tree_leapfrog(void *pos_mass, void *vel, void *acc_pot, int32_t *order, int64_t n,
                        int32_t prec, double G, double eps, double theta, int32_t leaf, double dt,
                        int32_t nsteps, int32_t reorder_every, uint32_t flags,
                        double *energy_out, void *stream);

/*
 * Multi-level fast multipole method on the ORB nodes: the O(N) method Section
 * VI names (citing its reference [20]) as the successor of the tree code.
 * Same node table, moments and quadrupole cells as the tree code (bodies in
 * ORB order with the same leaf size, 1 <= leaf <= NBODY_TREE_GROUP; FP32
 * modes only).
 *   MAC:       target node A and source node B interact through M2L iff they
 *              share no body and diag2_A + diag2_B < theta^2 |com_A - com_B|^2
 *              (FP64, as in the group local expansions).
 *   traversal: from (root, root): MAC -> B joins A's M2L list; A a leaf and
 *              B accepted by the tree code's opening test against A's box
 *              (diag2_B < theta^2 D2, D2 the squared distance from com_B to
 *              the box) -> B joins A's M2P list; both leaves -> B joins A's
 *              P2P list; B a leaf, or A an inner node with diag2_A >= diag2_B
 *              -> (A.left, B), (A.right, B); else (A, B.left), (A, B.right).
 *   M2L:       B's quadrupole potential as a third-order Taylor expansion
 *              about com_A (as NBODY_CELLS_LOCAL), FP32, summed over A's list.
 *   L2L:       a node's expansion = its own M2L sum + its parent's expansion
 *              re-expanded about its centre (exact for a cubic), FP64.
 *   L2P, M2P, P2P: every body of a leaf evaluates the leaf's expansion
 *              (FP64), its M2P cells as quadrupole cells (as
 *              NBODY_CELLS_QUAD) and its P2P source leaves body by body, with
 *              FP32 arithmetic; each lane's FP32 partial sums are folded by
 *              prec.
 * theta = 0 gives no M2L or M2P entry: the direct sum, at a P2P cost of
 * (n/leaf)^2 leaf pairs.  List buffers are library-owned and grow as needed;
 * each call synchronises its stream once to check them.  The traversal
 * writes each node's lists in one pass into slots sized for the largest
 * node of its depth (about five times the entries); when that would take
 * more than an eighth of the device's memory (or more than the environment
 * variable NBODY_FMM_SLOT_MB, in MiB, if set) it counts, scans and fills
 * compact lists instead.  Both give the same lists and results.
 * nbody_fmm_accel: acc_pot_out = n float4 (ax, ay, az, phi) in ORB order.
 * nbody_fmm_lists (inspection, synchronous): m2l_cnt, m2p_cnt, p2p_cnt =
 *   int32[num nodes] list lengths per target node; m2l_ids, m2p_ids, p2p_ids
 *   (may be NULL) the source node ids, target nodes in id order, each
 *   target's entries in the device walk's fixed order (as sets they are the
 *   recursion's lists); NBODY_E_INVAL if a list exceeds its capacity.  All
 *   arrays are device memory.
 */
int nbody_fmm_accel(const void *pos_mass, int64_t n, int32_t prec, double G, double eps, double theta,
                    int32_t leaf, void *acc_pot_out, void *stream);
int nbody_fmm_lists(const void *pos_mass, int64_t n, int32_t leaf, double theta, int32_t *m2l_cnt,
                    int32_t *m2p_cnt, int32_t *p2p_cnt, int32_t *m2l_ids, int64_t m2l_cap, int32_t *m2p_ids,
                    int64_t m2p_cap, int32_t *p2p_ids, int64_t p2p_cap, void *stream);

/*
 * Bit-reversible kick-drift-kick and its checkpoint-free adjoint (the
 * integer-state reading of the leapfrog of Section IV.B, after Rein and
 * Tamayo's JANUS integrator).  Positions and velocities are int64 fixed point
 * in units of 2^-shift_x and 2^-shift_v: kick V += round(h G 2^shift_v a),
 * drift X += round(V dt 2^(shift_x - shift_v)), rounded to nearest even in
 * FP64, forces of the positions decoded to FP32 (NBODY_F32_F64ACC sums).
 * Subtracting the same integers undoes a step exactly, so the adjoint rebuilds
 * every position bit for bit from the final state and stores nothing per step.
 * state: int64 [2n][4], rows [0, n) = (X, Y, Z, 0), rows [n, 2n) =
 * (VX, VY, VZ, 0); 32-byte aligned device memory.  |X|, |V| < 2^53 (not
 * checked).  shift_x, shift_v in [0, 60] (else NBODY_E_INVAL).  Both calls
 * use one kernel shape per n, independent of tuning pins and the tune cache:
 * the reverse pass must reproduce the forward's forces bit for bit.  They
 * use library scratch (force and VJP partials, three records per body):
 * overlapping calls on one device race.
 * nbody_janus_forward: encodes pos_mass/vel (float4, masses in w), runs
 *   nsteps, writes the final state, the decoded positions with the masses
 *   (pos_mass_out) and, if not NULL, the decoded velocities (vel_out).
 * nbody_janus_adjoint: gradients (pos_cot, vel_cot, mass_cot as for
 *   nbody_trajectory_adjoint) of a loss with cotangents xbar_T, vbar_T of
 *   the final decoded state, reversing `state` IN PLACE to the initial state
 *   (bit-exact); pos_mass supplies the masses (w).  Every mass must be
 *   positive (checked once, synchronizing the stream; else
 *   NBODY_E_UNSUPPORTED).  Rounding is treated as the identity in the
 *   derivative.
 */
int nbody_janus_forward(const void *pos_mass, const void *vel, int64_t n, double G, double eps,
                        double dt, int32_t nsteps, int32_t shift_x, int32_t shift_v,
                        void *state_out, void *pos_mass_out, void *vel_out, void *stream);
int nbody_janus_adjoint(void *state, const void *pos_mass, int64_t n, double G, double eps,
                        double dt, int32_t nsteps, int32_t shift_x, int32_t shift_v,
                        const void *xbar_T, const void *vbar_T, void *pos_cot, void *vel_cot,
                        void *mass_cot, void *stream);

/*
 * Tuning.  nbody_autotune times the candidate kernel shapes for one problem
 * (kernel 0 = nbody_accel at size n, 1 = nbody_batched_accel for the given
 * offsets, 2 = nbody_accel_vjp) on library-owned synthetic inputs,
 * synchronously, and records the fastest in the in-process table (and in the
 * JSON file named by the environment variable NBODY_TUNE_CACHE, if set).
 * The candidates are (tpl, jsplit, jtile) with variant 0; every candidate
 * performs the same arithmetic per pair, so tuning changes where partial sums
 * are folded, never the accuracy class of the result.
 * nbody_set_tuning pins a shape for later calls: tpl (targets per lane:
 * 1, 2, 4), jsplit (independent source ranges per target, 1..32, reduced in
 * fixed order; kernel 1 takes 1), jtile (sources per partial sum, multiple
 * of 8), variant (FP32 force kernel only, apart from 0: 0 = source records
 * through scalar loads; 1 = staged in LDS, jtile a multiple of 256, identical
 * results to 0, never chosen by nbody_autotune); kernel and prec as above;
 * tpl = jsplit = jtile = -1 clears it.
 * nbody_get_tuning reports the shape the library would use.
 */
int nbody_autotune(int32_t kernel, int32_t prec, int64_t n, const int64_t *offsets_host,
                   int32_t nsys, void *stream);
int nbody_set_tuning(int32_t kernel, int32_t prec, int32_t tpl, int32_t jsplit, int32_t jtile,
                     int32_t variant);
int nbody_get_tuning(int32_t kernel, int32_t prec, int64_t n, int32_t *tpl, int32_t *jsplit,
                     int32_t *jtile, int32_t *variant);

const char *nbody_status_string(int status);
const char *nbody_last_error(void);
/* Frees library scratch, cached graphs and work lists on every device. */
void nbody_release(void);
/* Library ABI version (major * 100 + minor). */
int nbody_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
