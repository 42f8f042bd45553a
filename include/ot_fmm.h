/*
 * ot_fmm.h -- C ABI of the MI355X (gfx950) FP64 fast-multipole cell-to-cell
 * gravity interaction kernels.
 *
 * The operation (paper Sec. 2.1: the gravity solver of Octo-Tiger is a fast
 * multipole method on an adaptive octree whose nodes are 8x8x8 sub-grids;
 * Sec. 2.2.1 and 2.3: every compute kernel works on one sub-grid and its
 * ghost layers; Sec. 2.2.4: kernels of many sub-grids can be aggregated into
 * one launch). For every target cell i of a target sub-grid and every
 * multi-index alpha with |alpha| <= 3 (20 coefficients):
 *
 *   L_alpha(i) = sum_{j in S(i)} sum_{|beta| <= 3-|alpha|}
 *                    (-1)^{|beta|}/beta! * M_beta(j) * d^{alpha+beta} G (X_i - X_j)
 *
 *   G(r) = -1/|r| (gravitational constant 1), X = centre of mass of a cell,
 *   M_beta = raw Cartesian moments of the cell's mass about X (no 1/beta!),
 *   S(i) = cells j of the 3x3x3 sub-grid neighbourhood of i's sub-grid (the
 *   24^3 halo block) with |j-i|_2 > 4 and |floor(j/2)-floor(i/2)|_2 <= 4 in
 *   integer cell coordinates, whose sub-grid is available.
 * L_alpha are Cartesian derivatives of the potential at X_i (the local Taylor
 * coefficients without the 1/alpha! factor).
 *
 * Conventions shared by every entry point
 *   - Component order of all 20-vectors: graded lexicographic, x most
 *     significant: 1; x,y,z; xx,xy,xz,yy,yz,zz; xxx,xxy,xxz,xyy,xyz,xzz,yyy,
 *     yyz,yzz,zzz. Arrays are structure-of-arrays: component-major.
 *   - All double pointers are DEVICE pointers (FP64, 8-byte aligned), owned by
 *     the caller. The library keeps no reference to them after a call returns,
 *     except inside a captured step graph (ot_fmm_step_graph_create).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). The
 *     compute calls only enqueue work; they never synchronize or allocate, and
 *     they may be captured into a hipGraph by the caller.
 *   - Outputs must not overlap inputs or each other (checked from the array
 *     extents: OT_FMM_EINVAL).
 *   - Return value: OT_FMM_OK or a negative error code. On OT_FMM_EINVAL
 *     nothing was enqueued. Details of the last error of the calling thread
 *     are available from ot_fmm_last_error(). Device faults surface at the
 *     caller's next synchronisation.
 *   - Results are bitwise reproducible run to run for a fixed schedule.
 */
#ifndef OT_FMM_H
#define OT_FMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OT_FMM_VERSION 100

enum {
    OT_FMM_OK = 0,
    OT_FMM_EINVAL = -1,       /* invalid argument; nothing enqueued */
    OT_FMM_EHIP = -2,         /* HIP runtime or launch error */
    OT_FMM_ENOMEM = -3,       /* device allocation failed (plan creation only) */
    OT_FMM_EUNSUPPORTED = -4, /* current device is not gfx950 / no device */
    OT_FMM_ETIMEDOUT = -5     /* ot_fmm_future_wait: not ready within the limit */
};

/* Schedules (how a target sub-grid's 512 cells are spread over wavefronts).
 * All keep one work-group per target sub-grid and one staged source z-plane
 * in LDS; lanes are the 8x8 target cells of one z-plane.
 * The adjoint takes two: sched = target_role | (source_role << 8)
 * (OT_FMM_SCHED_BWD); the target-role pass accepts every schedule, the
 * source-role pass AUTO, W8 or W8P2 (its accumulators do not fit 16
 * wavefronts). A byte left AUTO takes the plan's tuned choice, else W16 for
 * the target role and W8 for the source role. */
enum {
    OT_FMM_SCHED_AUTO = 0,  /* the plan's tuned choice (ot_fmm_autotune), else W16 */
    OT_FMM_SCHED_W8 = 1,    /* 8 wavefronts: one per target z-plane */
    OT_FMM_SCHED_W16 = 2,   /* 16 wavefronts: two per target z-plane, stencil rows split */
    OT_FMM_SCHED_W8P2 = 3,  /* 8 wavefronts, two passes over the source planes (target
                               planes 0-3, then 4-7), two wavefronts per target plane */
    /* flag, OR-ed into a schedule: persistent launch -- as many work-groups as
     * are resident at once, taking work-list entries (longest first) from
     * counters that a one-thread kernel zeroes just before, on the same
     * stream. The counters are never shared by launches that can overlap:
     * eager launches use one set per stream (up to 64 streams per plan),
     * launches recorded into a graph a set of their own (up to 960 per plan
     * over its life; the plan's own step graph returns its sets when it is
     * replaced). Beyond either limit the call returns OT_FMM_EINVAL. */
    OT_FMM_SCHED_PERSISTENT = 0x10,
    /* flag, OR-ed into a schedule: XCD-aware work order -- entries sorted
     * along a Morton curve of the lattice positions recovered from the
     * neighbour table, cut into one piece of equal work per XCD and
     * interleaved, so that the work-groups each XCD runs at once are spatial
     * neighbours sharing their staged blocks in that XCD's L2 (instead of
     * longest work first) */
    OT_FMM_SCHED_LOCAL = 0x20
};
#define OT_FMM_SCHED_BWD(target_role, source_role) ((target_role) | ((source_role) << 8))

/* ---------------------------------------------------------------------------
 * Single sub-grid forms (one 24^3 halo block = 3x3x3 sub-grids, all present).
 * Halo arrays: index x + 24 y + 576 z, x fastest. Output L[20][512] for the
 * central 8^3 cells (halo coordinates 8..15), index x + 8 y + 64 z.
 * ------------------------------------------------------------------------- */

/* Monopole kernel (paper Sec. 2.1 gravity FMM; only the mass moment):
 *   mass[13824], com[3][13824] -> L[20][512] with M_beta = 0 for |beta| > 0. */
int ot_fmm_monopole(const double* mass, const double* com, double* L, void* stream);

/* Multipole kernel: M[20][13824] raw moments, com[3][13824] -> L[20][512]. */
int ot_fmm_multipole(const double* M, const double* com, double* L, void* stream);

/* ---------------------------------------------------------------------------
 * Batched forms (paper Sec. 2.2.4: one launch over many sub-grids).
 *
 * A store holds S sub-grids: M[20][S*512], com[3][S*512]; cell c = x+8y+64z
 * of store sub-grid s lives at s*512 + c. T target sub-grids are given by
 *   tgt[T]       store id of each target (distinct),
 *   nbr[T][27]   store id of the sub-grid in each neighbour slot
 *                slot = sx + 3 sy + 9 sz, s in {0,1,2} <-> offset -1,0,+1;
 *                slot 13 must equal tgt[t]; -1 = not available (its pairs are
 *                dropped),
 *   shift[T][27][3] (may be NULL) periodic image shift of each neighbour in
 *                units of period[3]: the source centre used is
 *                com + shift * period.
 * The tables are HOST arrays; ot_fmm_plan_create validates them and keeps
 * device copies plus the inverse (source -> target) relations used by the
 * adjoint, the work order and the exact pair counts.
 * Outputs: L[20][T*512] (target t's cells at t*512 + c).
 * ------------------------------------------------------------------------- */
typedef struct ot_fmm_plan_s* ot_fmm_plan;

/* Validates the descriptor (EINVAL: S or T <= 0, tgt out of range or
 * repeated, nbr out of [-1, S), nbr[t][13] != tgt[t], shift without period,
 * two targets claiming the same (source, slot) relation) and allocates the
 * device tables (ENOMEM). Synchronous. The plan is bound to the current
 * device. */
int ot_fmm_plan_create(int32_t S, int32_t T, const int32_t* tgt, const int32_t* nbr,
                       const int8_t* shift, const double* period, ot_fmm_plan* out);
int ot_fmm_plan_destroy(ot_fmm_plan plan);

/* Exact number of interacting (target cell, source cell) pairs of the plan,
 * counted from the descriptor (the unit of the throughput metric). */
int ot_fmm_plan_pairs(ot_fmm_plan plan, int64_t* pairs);

/* Host-only (no device call): validates a descriptor exactly as
 * ot_fmm_plan_create does and returns its pair count; optionally the exact
 * pairs of each target (work[T]) and the launch order of the targets
 * (order[T]: longest work first, ties in target order). */
int ot_fmm_count_pairs(int32_t S, int32_t T, const int32_t* tgt, const int32_t* nbr, const int8_t* shift,
                       const double* period, int64_t* pairs, int64_t* work, int32_t* order);

/* Host-only: the other work orders of a plan built from this descriptor, for
 * a device with `nxcd` XCDs: fwd_local[T] (targets, XCD-aware),
 * rev_lpt[S] and rev_local[S] (store sub-grids of the adjoint's source-role
 * pass, longest work first / XCD-aware). Any output may be NULL. */
int ot_fmm_work_orders(int32_t S, int32_t T, const int32_t* tgt, const int32_t* nbr, const int8_t* shift,
                       const double* period, int32_t nxcd, int32_t* fwd_local, int32_t* rev_lpt,
                       int32_t* rev_local);

/* Host-only: the stencil tables the kernels use. slot_pairs[27] = pairs
 * between the 8^3 targets and the neighbour block in each slot;
 * offsets_per_target[2] = sources of one target of z parity 0 / 1;
 * rows_per_parity[2] = entries (dz, dy, x-interval) of the per-parity row
 * table the wavefronts walk.
 * EUNSUPPORTED if the mirrored row table does not reproduce the stencil of
 * every parity (the kernels then refuse to run). */
int ot_fmm_stencil_info(int64_t* slot_pairs, int32_t* offsets_per_target, int32_t* rows_per_parity);

/* Coarse substitutes for missing neighbours. Sec. 2.1 names the octree FMM
 * gravity solver without its formulas; what follows is a reading of the
 * interaction across a refinement boundary. For target t and a
 * slot s whose fine neighbour is missing (nbr[t][s] == -1), coarse[t][s] is
 * the node P of a coarse store and octant[t][s] = o the octant of P that
 * covers the missing block; -1 where there is none. Coarse cell
 * (cx, cy, cz) of the octant, cell (cx + 4 o_x) + 8 (cy + 4 o_y) +
 * 64 (cz + 4 o_z) of P, is the parent of the 2x2x2 missing fine cells
 * 8 s_k + 2 c_k + {0, 1} (halo coordinates); it stands in for them, with its
 * moments about its centre (shifted like the missing neighbour), for every
 * target cell i for which all 8 would be in S(i):
 *   L_a(i) += sum_{|b| <= 3-|a|} s_b M_b(J) G_{a+b}(X_i - X_J).
 * set_coarse: HOST tables [T][27] (EINVAL: node out of [-1, Sp), a
 * substitute for a present neighbour, octant out of [0, 8)); keeps device
 * copies (replacing earlier ones, after waiting for the device when there
 * were any); *pairs (may be NULL) = the included (target cell, coarse cell)
 * pairs. Synchronous; not to be called concurrently with other calls on the
 * same plan from other threads. */
int ot_fmm_plan_set_coarse(ot_fmm_plan plan, int32_t Sp, const int32_t* coarse, const int8_t* octant,
                           int64_t* pairs);

/* Adds the coarse contributions into L[20][T*512]: com[3][S*512] (the fine
 * centres of the targets), Mp[20][Sp*512], comp[3][Sp*512] the coarse store
 * (e.g. from ot_fmm_m2m); device pointers, 8-byte aligned, caller-owned.
 * EINVAL: no tables set, a null or misaligned pointer, L overlapping an input
 * (nothing enqueued). Enqueue only, on `stream`; targets without substitutes
 * are left untouched. */
int ot_fmm_coarse_fine(ot_fmm_plan plan, const double* com, const double* Mp, const double* comp, double* L,
                       void* stream);

/* The coarse substitutes under the full truncation (the reading of
 * ot_fmm_multipole_batched_full, for a step that uses it):
 *   L_a(i) += sum_{|b| <= 3} s_b M_b(J) G_{a+b}(X_i - X_J).
 * Same tables, arguments, accumulation and errors as ot_fmm_coarse_fine. */
int ot_fmm_coarse_fine_full(ot_fmm_plan plan, const double* com, const double* Mp, const double* comp,
                            double* L, void* stream);

/* Batched multipole forward: M[20][S*512], com[3][S*512] -> L[20][T*512]. */
int ot_fmm_multipole_batched(ot_fmm_plan plan, const double* M, const double* com, double* L,
                             int sched, void* stream);

/* Batched forward with the full truncation: every output |a| <= 3 keeps
 * every source moment |b| <= 3 (derivatives of G to order 6),
 *   L_a(i) = sum_{j in S(i)} sum_{|b| <= 3} s_b M_b(j) G_{a+b}(X_i - X_j),
 * the alternative to the total-order truncation |a| + |b| <= 3 of
 * ot_fmm_multipole_batched (Sec. 2.1 names the FMM without its truncation;
 * this is the other reading). Same plan, layouts, schedules (AUTO = W8P2 |
 * PERSISTENT | LOCAL, not autotuned) and
 * error rules as ot_fmm_multipole_batched; L is overwritten. */
int ot_fmm_multipole_batched_full(ot_fmm_plan plan, const double* M, const double* com, double* L,
                                  int sched, void* stream);

/* Adjoint of ot_fmm_multipole_batched_full (derivatives of G to order 7):
 * the same arrays, overwrite rules and errors as ot_fmm_multipole_backward;
 * schedules as there, AUTO = W8P2 | PERSISTENT | LOCAL for both passes, a target-role
 * shape of 16 wavefronts is EINVAL. */
int ot_fmm_multipole_backward_full(ot_fmm_plan plan, const double* M, const double* com,
                                   const double* gL, double* gM, double* gcom, int sched,
                                   void* stream);

/* Adjoint of the batched forward for the loss l = sum gL * L:
 *   gL[20][T*512] -> gM[20][S*512] = dl/dM, gcom[3][S*512] = dl/dcom.
 * gM and gcom are OVERWRITTEN; cells of store sub-grids that no target
 * references get 0. Gather form (no atomics): one pass over each store
 * sub-grid's source role, then one over each target's own cells. gM/gcom
 * must not alias M, com or gL. */
int ot_fmm_multipole_backward(ot_fmm_plan plan, const double* M, const double* com,
                              const double* gL, double* gM, double* gcom, int sched,
                              void* stream);

/* Training step in two passes instead of three: a forward that also saves
 * what the adjoint's target role needs, and a one-pass adjoint.
 *
 * ot_fmm_multipole_batched_save: L as ot_fmm_multipole_batched, and
 *   Cs[24][T*512], the target-side derivatives of L,
 *     C'_g(i) = sum_{j in S(i)} sum_{|b| <= 4-|g|} s_b M_b(j) G_{g+b}(X_i - X_j),
 *     1 <= |g| <= 4, so that dL_a(i)/dX_i,k (target role only) = C'_{a+e_k}(i);
 *   the 24 components with a z exponent below 2, in graded-lex order (x, y, z,
 *   xx, xy, xz, yy, yz, xxx, xxy, xxz, xyy, xyz, yyy, yyz, xxxx, xxxy, xxxz,
 *   xxyy, xxyz, xyyy, xyyz, yyyy, yyyz); the other 10 follow from Laplace's
 *   equation, C'_{g+zz} = -(C'_{g+xx} + C'_{g+yy}).
 * ot_fmm_multipole_backward_saved: gM, gcom exactly as
 *   ot_fmm_multipole_backward (overwritten), from gL and the Cs of the forward
 *   of the same M and com: one pass over the store sub-grids (source role),
 *   whose cells add their own target role from Cs.
 * Schedules: W8 or W8P2 with the PERSISTENT / LOCAL flags, or AUTO (the
 * choice of ot_fmm_autotune_saved, else W8P2 | PERSISTENT | LOCAL); 16
 * wavefronts are EINVAL. Errors and overlap rules as for the other batched
 * calls (Cs counts as an output of the forward and an input of the adjoint). */
int ot_fmm_multipole_batched_save(ot_fmm_plan plan, const double* M, const double* com, double* L,
                                  double* Cs, int sched, void* stream);
int ot_fmm_multipole_backward_saved(ot_fmm_plan plan, const double* M, const double* com,
                                    const double* gL, const double* Cs, double* gM, double* gcom,
                                    int sched, void* stream);

/* The same two-launch step for the full truncation (ot_fmm_multipole_batched_full
 * and its adjoint): Cs[24][T*512] holds C'_g(i) = sum_{j in S(i)} sum_{|b| <= 3}
 * s_b M_b(j) G_{g+b}(X_i - X_j), 1 <= |g| <= 4 (= dL_a(i)/dX_i,k under the full
 * truncation for g = a + e_k; its orders 1..3 equal L), the same 24 kept
 * components; derivatives of G to order 7. Schedules: W8 or W8P2 with the
 * flags, AUTO = W8P2 | PERSISTENT | LOCAL (not autotuned); errors and overlap
 * rules as for the total-order pair. */
int ot_fmm_multipole_batched_full_save(ot_fmm_plan plan, const double* M, const double* com, double* L,
                                       double* Cs, int sched, void* stream);
int ot_fmm_multipole_backward_full_saved(ot_fmm_plan plan, const double* M, const double* com,
                                         const double* gL, const double* Cs, double* gM, double* gcom,
                                         int sched, void* stream);

/* Forward with the angular-momentum correction of the force (Sec. 2.1 cites
 * Octo-Tiger's FMM, which conserves angular momentum, without its formulas;
 * this is a reading fixed by that conservation law). With the total-order
 * truncation the interaction energy
 *   E = 1/2 sum_i sum_a (M_a(i)/a!) L_a(i)
 * is invariant under rotations of positions and moments together, so the
 * forces F_i = -dE/dX_i and the cells' spin torques
 *   tau_i,m = -sum_{|g| <= 2} eps_mnl (M_{g+e_n}(i)/g!) L_{g+e_l}(i)
 * satisfy sum_i (X_i x F_i + tau_i) = 0 over a closed set. The force
 * evaluated from L (ot_fmm_evaluate) misses the terms of -dE/dX_i with
 * |a| + |b| = 3, and with it the balance fails; this call returns L as
 * ot_fmm_multipole_batched and those terms,
 *   dF_k(i) = -sum_{j in S(i)} sum_{|a|+|b| = 3} (M_a(i)/a!) s_b M_b(j) G_{a+b+e_k}(X_i - X_j),
 * dF[3][T*512] (overwritten): F_i = (force from L) + dF_i conserves linear
 * and total angular momentum to rounding. With the dipoles about the centres
 * of mass zero, dF holds the target's mass times the sources' octupoles and
 * the target's octupole times the sources' masses.
 * Schedules, errors and overlap rules as for ot_fmm_multipole_batched_save. */
int ot_fmm_multipole_batched_amc(ot_fmm_plan plan, const double* M, const double* com, double* L,
                                 double* dF, int sched, void* stream);

/* Times both passes of the two-pass step with every schedule (W8, W8P2, each
 * with the four flag combinations) on the given buffers and keeps the fastest
 * in the plan (used by AUTO); leaves the results of the chosen schedules in
 * L, Cs, gM and gcom. Synchronizes `stream`; not while capturing. */
int ot_fmm_autotune_saved(ot_fmm_plan plan, const double* M, const double* com, double* L,
                          double* Cs, const double* gL, double* gM, double* gcom, void* stream,
                          int* fwd_sched, int* bwd_sched);

/* Captures the two-pass step (forward with saved sums, one-pass adjoint)
 * into the plan's step graph (replacing any previous one), replayed by
 * ot_fmm_step_graph_launch. */
int ot_fmm_step_graph_create_saved(ot_fmm_plan plan, const double* M, const double* com, double* L,
                                   double* Cs, const double* gL, double* gM, double* gcom,
                                   int fwd_sched, int bwd_sched);

/* Times every schedule of the forward (and backward, if gL/gM/gcom are not
 * NULL) on the given buffers and stores the fastest in the plan; returns the
 * choices. Every shape is timed with each combination of the persistent and
 * XCD-aware flags, the forward and the two adjoint passes each on its own.
 * Synchronizes `stream`; do not call it while capturing. The buffers are
 * overwritten with valid results (L of the last forward timed, gM and gcom
 * of one backward with the chosen schedules). */
int ot_fmm_autotune(ot_fmm_plan plan, const double* M, const double* com, double* L,
                    const double* gL, double* gM, double* gcom, void* stream,
                    int* fwd_sched, int* bwd_sched);

/* Captures forward (+ backward when gL/gM/gcom are not NULL) with the given
 * schedules into a hipGraph owned by the plan (replacing any previous one).
 * The graph bakes in the pointers: re-create it when buffers move. */
int ot_fmm_step_graph_create(ot_fmm_plan plan, const double* M, const double* com, double* L,
                             const double* gL, double* gM, double* gcom, int fwd_sched,
                             int bwd_sched);
/* Replays the captured graph on `stream`. EINVAL if none was captured. */
int ot_fmm_step_graph_launch(ot_fmm_plan plan, void* stream);

/* Per-kernel timing of a plan's launches (tracing support): while enabled,
 * every forward / adjoint launch of the plan (not graph replays) is
 * bracketed by HIP events on its stream. ot_fmm_plan_kernel_times waits for
 * the recorded events, returns for each kernel -- [0] batched forward,
 * [1] adjoint source-role pass, [2] adjoint target-role pass, [3] forward
 * with saved sums, [4] one-pass adjoint, [5] forward with the
 * angular-momentum correction -- the summed duration in ms and the number of
 * launches, and resets the counters. */
#define OT_FMM_NKERNELS 6
int ot_fmm_plan_timing(ot_fmm_plan plan, int enable);
int ot_fmm_plan_kernel_times(ot_fmm_plan plan, double ms_total[OT_FMM_NKERNELS],
                             int64_t launches[OT_FMM_NKERNELS]);

/* ---------------------------------------------------------------------------
 * Tree passes around the interaction (paper Sec. 2.1 and 2.3: the FMM gravity
 * solver traverses the octree of sub-grids). A parent node p has 8 child nodes
 * children[p][o], o = ox + 2 oy + 4 oz (one octant each); parent cell
 * (X, Y, Z) of p covers the 2x2x2 child cells (2(X%4)+a, 2(Y%4)+b, 2(Z%4)+c),
 * a, b, c in {0, 1}, of child node o = (X/4) + 2(Y/4) + 4(Z/4). Parent and
 * child stores use the batched layout ([ncomp][nodes*512]).
 * ------------------------------------------------------------------------- */
typedef struct ot_fmm_tree_s* ot_fmm_tree;

/* children: HOST array [Sp][8] of child store ids in [0, Sc), each id at most
 * once, 8*Sp <= 2^26 (EINVAL otherwise). Keeps a device copy; synchronous;
 * bound to the current device (passes on another device return EINVAL).
 * All device pointers of the passes: 8-byte aligned (EINVAL otherwise);
 * the passes are asynchronous on `stream`, and outputs must not alias inputs. */
int ot_fmm_tree_create(int32_t Sp, int32_t Sc, const int32_t* children, ot_fmm_tree* out);
int ot_fmm_tree_destroy(ot_fmm_tree tree);

/* Upward pass (M2M; P2M when the children carry only masses): for every
 * parent cell, mass = sum of the 8 child masses, centre = their mass-weighted
 * mean (plain mean if the mass is 0), raw moments about it
 *   M_b(p) = sum_c sum_{g <= b} C(b, g) M_g(c) (X_c - X_p)^(b-g),
 * exact to order 3. Mc[20][Sc*512], comc[3][Sc*512] -> Mp[20][Sp*512],
 * comp[3][Sp*512] (overwritten). */
int ot_fmm_m2m(ot_fmm_tree tree, const double* Mc, const double* comc, double* Mp, double* comp,
               void* stream);

/* Downward pass (L2L): every child cell's coefficients are INCREMENTED by its
 * parent cell's local expansion re-expanded about the child centre,
 *   L_a(c) += sum_{|g| <= 3-|a|} L_{a+g}(p) (X_c - X_p)^g / g!,
 * exact for the cubic expansion. Lp[20][Sp*512], comp[3][Sp*512],
 * comc[3][Sc*512], Lc[20][Sc*512] (in/out; cells of child nodes not listed
 * in the tree are untouched). */
int ot_fmm_l2l(ot_fmm_tree tree, const double* Lp, const double* comp, const double* comc,
               double* Lc, void* stream);

/* Local evaluation per cell, from its moments M (about its centre) and local
 * coefficients L (about the same centre), with the expansion truncated at
 * order 3:  F_k = - sum_{|a|<=2} M_a/a! L_{a+e_k}  (force on the cell's mass),
 *           W   = 1/2 sum_{|a|<=3} M_a/a! L_a     (its share of the energy).
 * M, L [20][ncells] -> F[3][ncells], W[ncells]; 1 <= ncells <= 2^38. */
int ot_fmm_evaluate(int64_t ncells, const double* M, const double* L, double* F, double* W,
                    void* stream);

/* ---------------------------------------------------------------------------
 * Futures for asynchronous per-sub-grid launches, completed by event polling
 * (paper Sec. 3: the task scheduler polls GPU events between tasks and makes
 * the futures of completed events ready, which runs their continuations; one
 * thread polls at a time and the others skip; events not yet complete are
 * kept for the next poll; nothing ever blocks on the GPU).
 *
 * An executor owns `nstreams` HIP streams (created on first use, on the
 * device current then; default priority) and a task queue served by
 * `nworkers` threads (0: tasks run in the threads that call poll or wait).
 * Workers run tasks and poll between them while events are pending. All
 * calls are thread-safe. Futures must be released before their executor is
 * destroyed; ot_fmm_executor_destroy first waits (by polling) for every
 * registered event and runs the remaining tasks.
 * ------------------------------------------------------------------------- */
typedef struct ot_fmm_executor_s* ot_fmm_executor;
typedef struct ot_fmm_future_s* ot_fmm_future;
typedef void (*ot_fmm_callback)(void* user);

/* 1 <= nstreams <= 1024, 0 <= nworkers <= 256 (EINVAL otherwise). Makes no
 * HIP call. */
int ot_fmm_executor_create(int nstreams, int nworkers, ot_fmm_executor* out);
int ot_fmm_executor_destroy(ot_fmm_executor ex);

/* Stream i (0 <= i < nstreams) of the pool, as a hipStream_t. */
int ot_fmm_executor_stream(ot_fmm_executor ex, int i, void** stream);

/* A new future that becomes ready when all work enqueued on `stream` before
 * this call has completed (an event recorded on it). The caller owns one
 * reference (ot_fmm_future_release). */
int ot_fmm_executor_get_future(ot_fmm_executor ex, void* stream, ot_fmm_future* out);

/* ot_fmm_multipole (single 24^3 halo block, same arguments and layout) on the
 * next stream of the pool (round robin), plus its future. */
int ot_fmm_executor_multipole_async(ot_fmm_executor ex, const double* M, const double* com,
                                    double* L, ot_fmm_future* out);

/* Queues fn(user) on the executor's task queue. */
int ot_fmm_executor_post(ot_fmm_executor ex, ot_fmm_callback fn, void* user);

/* One poll: *completed = futures made ready, or -1 if another thread was
 * polling (the call then returns at once). Without workers it also runs the
 * queued tasks. `completed` may be NULL. */
int ot_fmm_executor_poll(ot_fmm_executor ex, int* completed);

/* Number of registered events not yet seen complete. */
int ot_fmm_executor_outstanding(ot_fmm_executor ex, int64_t* n);

/* A host-side future, made ready by ot_fmm_future_set_ready (once; EINVAL
 * for a second call or for an event-backed future). */
int ot_fmm_future_create(ot_fmm_executor ex, ot_fmm_future* out);
int ot_fmm_future_set_ready(ot_fmm_future f);

/* Runs fn(user) as a task once f is ready (queued at once if it already is). */
int ot_fmm_future_then(ot_fmm_future f, ot_fmm_callback fn, void* user);
int ot_fmm_future_is_ready(ot_fmm_future f, int* ready);

/* Waits until f is ready by running queued tasks and polling (never a
 * blocking GPU call). timeout_s < 0: no limit; otherwise ETIMEDOUT after
 * that many seconds. EHIP if the GPU work behind the future failed. */
int ot_fmm_future_wait(ot_fmm_future f, double timeout_s);
int ot_fmm_future_release(ot_fmm_future f);

/* ---------------------------------------------------------------------------
 * Allocation-free batched forward, for callers that cannot allocate device
 * memory or create a plan: code under hipGraph capture, tight serving loops,
 * harnesses that forbid hipMalloc.
 *
 * The result of ot_fmm_multipole_batched with the schedule
 * W16 | PERSISTENT (bitwise), without a plan. The descriptor (same meaning as
 * for ot_fmm_plan_create) is given in DEVICE arrays owned by the caller:
 * tgt[T] and nbr[T][27] (int32, 4-byte aligned), shift[T][27][3] (int8) or
 * NULL; period[3] is a HOST array (may be NULL when shift is NULL). M, com, L
 * as for ot_fmm_multipole_batched (L[20][T*512] overwritten).
 *
 * Scratch memory: the call's relation table and the work counters live in one
 * fixed library array per device (13.6 MiB, taken on the first call on a
 * device and held until the process ends); T <= OT_FMM_NOALLOC_MAX_T, EINVAL
 * beyond (nothing enqueued). The call allocates nothing and only enqueues
 * kernels on `stream` (it may be captured). Every call on a device shares
 * that array, which keeps the last call's contents: calls that can overlap on
 * one device (other streams or threads, replays of graphs holding a call) race
 * and must be ordered by the caller.
 *
 * Errors: host-side checks as for the other entry points (EINVAL, nothing
 * enqueued). The table entries are checked on the device: an entry out of
 * range (tgt outside [0, S), nbr outside [-1, S), nbr[t][13] != tgt[t]) is
 * dropped and counted, and then every element of L is set to NaN;
 * ot_fmm_noalloc_status returns the count. Unlike a plan, repeated target
 * ids are not rejected (the forward does not need them distinct).
 * ------------------------------------------------------------------------- */
#define OT_FMM_NOALLOC_MAX_T 32768
int ot_fmm_multipole_batched_noalloc(int32_t S, int32_t T, const int32_t* tgt, const int32_t* nbr,
                                     const int8_t* shift, const double* period, const double* M,
                                     const double* com, double* L, void* stream);

/* Descriptor check of the last allocation-free call on the current device:
 * waits for the device, then returns the number of invalid entries and the
 * first of them (t * 27 + slot; INT32_MAX when there is none). Synchronous. */
int ot_fmm_noalloc_status(int32_t* invalid, int32_t* first_invalid);

/* ---------------------------------------------------------------------------
 * Helpers
 * ------------------------------------------------------------------------- */
const char* ot_fmm_strerror(int code);
/* Detail of the last error on the calling thread ("" if none). */
const char* ot_fmm_last_error(void);
int ot_fmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OT_FMM_H */
