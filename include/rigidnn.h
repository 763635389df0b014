/*
 * rigidnn.h -- C ABI of the MI355X (gfx950) rigid-body pair library.
 *
 * The library evaluates the energy, forces and torques of every neighbouring
 * pair of composite-bead rigid bodies in two ways: the plain bead double sum
 * (paper section 2, first equation), and a learned map from the pair
 * configuration to the energy (paper section 2: the configuration of a pair
 * is the position and orientation of body j in the frame of body i) whose
 * gradient gives forces and torques (supplementary section 6).  It also
 * builds the pair list, integrates rigid-body motion and trains the network.
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller unless the
 *     comment says "host".  The library never frees them.
 *   - Arrays of per-body or per-pair vectors are structure-of-arrays: a
 *     "3 x n" FP64 array stores all x components, then all y, then all z.
 *   - Quaternions are (w, x, y, z), Hamilton product, unit norm, and map the
 *     body frame to the lab frame.  Bead templates are in the body frame with
 *     the centre of mass at the origin and principal axes along x, y, z.
 *   - A pair descriptor is 7 numbers (d_x, d_y, d_z, q_w, q_x, q_y, q_z):
 *     d = R_i^T minimg(x_j - x_i) is body j's centre in body i's frame and
 *     q = q_i^* q_j its orientation relative to body i (R(q) = R_i^T R_j).
 *   - Per-pair force/torque outputs are 9 numbers (F_j, tau_i, tau_j) in
 *     body i's frame: F_j is the force on body j (F_i = -F_j), tau_i and
 *     tau_j are torques about each body's own centre.
 *   - `stream` is a hipStream_t passed as void*.  Every call only enqueues
 *     work on it and returns; nothing synchronises the host.  The library
 *     allocates device memory only in rb_ctx_create.
 *   - Return value: RB_OK or a negative RB_ERR_* code; rb_last_error() then
 *     gives a message (thread local).  Conditions found on the device
 *     (pair-list overflow, non-finite forces) are written to the caller's
 *     int32 flag array, read when the caller chooses to synchronise.
 */
#ifndef RIGIDNN_H
#define RIGIDNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RB_OK 0
#define RB_ERR_INVALID_ARG (-1)
#define RB_ERR_CAPACITY (-2)
#define RB_ERR_HIP (-3)
#define RB_ERR_UNSUPPORTED (-4)
#define RB_ERR_NONFINITE (-5)   /* rb_flags_check: the device reported non-finite
                                   or overflowing forces, energies or orientations */

/* Device flag words (int32 array of RB_NFLAGS, 8-byte aligned, caller owned,
 * zero it once). */
#define RB_FLAG_REBUILD 0    /* 1: the pair list must be rebuilt before use     */
#define RB_FLAG_NPAIRS 1     /* pairs in the current list (<= capacity)         */
#define RB_FLAG_OVERFLOW 2   /* pairs found by the last build when > capacity   */
#define RB_FLAG_NREBUILDS 3  /* number of list builds done                      */
#define RB_FLAG_NBEAD 4      /* pairs routed to the bead sum (|d| < d_min)      */
#define RB_FLAG_NNN 5        /* pairs routed to the network                     */
#define RB_FLAG_NONFINITE 6  /* a non-finite per-pair force or energy was seen   */
#define RB_FLAG_NEVAL 7      /* running count of pairs evaluated by the per-body
                                force calls (bead and network); wraps at 2^31  */
#define RB_FLAG_NTESTS 8     /* flags[8..9] as one int64: running count of bead-
                                bead distance tests performed after culling    */
#define RB_FLAG_NSCREEN 10   /* pairs kept by rb_bead_screen (when its count_out
                                is &flags[NSCREEN]), or in the screened list of
                                rb_bead_pair_forces_screened or the candidate
                                list of rb_pair_descriptors_screened            */
#define RB_FLAG_RESCREEN 11  /* 1: the screened list must be rebuilt before use;
                                set by every pair-list build and by the
                                integrator's margin test                        */
#define RB_FLAG_NRESCREENS 12 /* number of screened-list builds done           */
#define RB_FLAG_FIXOVF 13    /* 1: a term added to the fixed-point accumulator
                                reached 2^28 in magnitude or was not finite, or
                                a per-body or global total reached 2^30 (the
                                accumulator holds totals below 2^31): forces,
                                torques, energy or virial may be invalid       */
#define RB_FLAG_QDRIFT 14    /* running count of body updates whose quaternion
                                norm had drifted from 1 by more than 1e-10
                                (|q|^2 - 1) before the integrator's
                                renormalisation; also counts non-finite q      */
#define RB_FLAG_ROUTE_WORK 16 /* words 16..17: one 64-bit working word of
                                rb_pair_descriptors (network count, bead count,
                                blocks done); word 18: candidate count of
                                rb_pair_descriptors_screened; zero between
                                calls                                          */
#define RB_FLAG_WAIT_TIMEOUT 19 /* 1: a kernel's internal wait between waves
                                gave up (an internal error: results invalid)   */
#define RB_FLAG_FB_WORK 20   /* words 20..21: working counters of the bead-sum
                                phase of rb_nn_pair_forces_routed (pair counter,
                                finishing ticket); zero between calls           */
#define RB_NFLAGS 24

#define RB_PREC_BF16 0       /* 128x128 layers on BF16 MFMA, FP32 accumulate     */
#define RB_PREC_FP32 1       /* every layer in FP32                              */

#define RB_BUILD_ALWAYS 0
#define RB_BUILD_IF_FLAGGED 1

#define RB_MLP_NPARAMS 50689 /* 7 -> 128 -> 128 -> 128 -> 128 -> 1               */

/* Fixed-point accumulator of per-body forces/torques and global sums:
 * int64 array of RB_ACC_LEN(n) = 6 n + 10 * RB_ACC_SLOTS words, layout
 * F_x[n] F_y[n] F_z[n] tau_x[n] tau_y[n] tau_z[n], then for each of the 10
 * global sums (E, W_xx, W_xy, W_xz, W_yx, ..., W_zz) RB_ACC_SLOTS partial
 * words that different workgroups add into (spreading the atomics over many
 * addresses); rb_accum_finalize adds the partials.  Every word is the value
 * times 2^32; integer addition is associative, so the result does not
 * depend on the order in which pairs are summed. */
#define RB_ACC_SCALE 4294967296.0
#define RB_ACC_SLOTS 64
#define RB_ACC_LEN(n) (6 * (int64_t)(n) + 10 * RB_ACC_SLOTS)

typedef struct rb_ctx rb_ctx;

/* Context: bead templates and the bead potential (Lennard-Jones 12-6,
 * energy-shifted at rc: u(r) - u(rc) for r < rc), and per-type mass and
 * principal inertia for the integrator.  Host inputs: n_beads[n_types],
 * beads[sum(n_beads) x 3] (xyz per bead, types concatenated), mass[n_types],
 * inertia[n_types x 3].  At most 8 types, at most 256 beads per type.
 * Allocates the device copies; rb_ctx_destroy frees them. */
int rb_ctx_create(rb_ctx **out, int32_t n_types, const int32_t *n_beads, const float *beads,
                  const double *mass, const double *inertia, float eps, float sigma, float rc);
int rb_ctx_destroy(rb_ctx *ctx);

/* Switches the context's bead potential to the half-power half-cosine form
 * of the paper (section 3): U(r) = (b - r)^p - 2A for r <= b and
 * -A (1 + cos(c (r - b))) for b < r < rc = b + pi / c, 0 beyond.  The printed
 * attractive branch, -A cos(c (r - b)), would jump by A at r = b and end at
 * +A; the form used joins both branches with zero slope and vanishes with
 * zero slope at rc.  The paper's parameters: A = 0.00035, b = 1.46375,
 * c = 3.3833, p = 2.5 (epsilon, sigma units).  Applies to every later bead
 * sum with this context; the pair-list cutoff must use this rc. */
int rb_ctx_set_hphc(rb_ctx *ctx, double A, double b, double c, double p);
const char *rb_last_error(void);

/* Host check of a flag array the caller has copied to host memory
 * (flags_host, RB_NFLAGS int32): RB_ERR_CAPACITY when the last pair-list
 * build overflowed its capacity, RB_ERR_NONFINITE when a non-finite pair
 * force or energy (RB_FLAG_NONFINITE), a fixed-point accumulator overflow
 * (RB_FLAG_FIXOVF), a quaternion norm drift (RB_FLAG_QDRIFT) or an
 * internal wait that gave up (RB_FLAG_WAIT_TIMEOUT) was
 * reported, RB_OK otherwise; rb_last_error() names the condition.  Touches
 * no device state. */
int rb_flags_check(const int32_t *flags_host);

/* ---- pair list: half list i < j of body pairs closer than r_list --------
 * Paper abstract: bead distances are computed only for bodies near each
 * other; a body pair can have a bead pair inside rc only when its centre
 * distance is below 2 r_max + rc, so r_list = 2 r_max + rc + skin.  Cell list
 * over a periodic orthorhombic box (host box[3]); requires box >= 2 r_list
 * per axis.  x: 3 x n FP64 positions (any periodic image).  Writes
 * pair_i/pair_j (capacity max_pairs): the exact set of pairs, each once with
 * pair_i < pair_j; for n <= 65536 the pairs of one body i are contiguous and
 * in a fixed cell order and the order of the bodies' runs is not specified;
 * above, the order is fixed (the same list for the same input);
 * flags[NPAIRS] = min(found, max_pairs) and
 * flags[OVERFLOW] = found if found > max_pairs (else 0).  Copies x into
 * x_ref (3 x n) for the skin test of rb_rigid_step.  With
 * RB_BUILD_IF_FLAGGED the kernels do nothing unless flags[REBUILD] is set,
 * which makes the call safe to capture in a graph; the call clears it.
 * For n <= 65536 the build is one launch whose workgroups wait for the one
 * that bins the bodies (a bounded wait: past it flags[WAIT_TIMEOUT] is set
 * and the list is invalid); flags[REBUILD] holds 2 while that launch runs.
 * ws: scratch of rb_pairlist_workspace_bytes(n, box, r_list) bytes. */
size_t rb_pairlist_workspace_bytes(int32_t n, const double *box, double r_list);
int rb_pairlist_build(int32_t n, const double *x, const double *box, double r_list,
                      int32_t *pair_i, int32_t *pair_j, int32_t max_pairs, double *x_ref,
                      int32_t *flags, int mode, void *ws, size_t ws_bytes, void *stream);

/* ---- descriptors and routing ---------------------------------------------
 * For the first flags[NPAIRS] pairs: desc (7 x max_pairs FP32) from FP64
 * state, and routing of each pair (paper section 2: the network replaces the
 * bead sum inside its training domain; the bead sum stays the reference
 * everywhere).  Without shells (ctx == NULL, type == NULL): pairs with
 * d_min <= |d| < d_max go to the network, pairs with |d| < d_min to the
 * bead sum, pairs at |d| >= d_max (where the switched network energy is
 * zero; d_max <= 0: no limit) to neither.  With shells (ctx and the bodies'
 * types, n int32): a lower bound G on the pair's closest bead-centre
 * distance is formed from two convex shells of each type's bead centres --
 * the bead-centre box (15-axis separating-axis gaps) and a capsule along the
 * longest body axis (segment distance minus radii), G the larger bound --
 * and, among the pairs with |d| < d_max, those with |d| < d_min or
 * G < gap_min (possibly closer than the training data's closest bead
 * distance) go to the bead sum, those with G >= gap_max (gap_max > 0; no
 * bead pair within gap_max, so zero bead energy when gap_max >= rc) to
 * neither, the rest to the network.  Routed pair indices go to idx_nn /
 * idx_bead (capacity max_pairs each, order not specified) with counts in
 * flags[NNN] / flags[NBEAD], written by the launch's last block (words
 * flags[RB_FLAG_ROUTE_WORK ..+1] count during the launch and are left
 * zero).  x: 3 x n, q: 4 x n.  RB_ERR_INVALID_ARG if max_pairs >= 2^27 or
 * flags is not 8-byte aligned. */
int rb_pair_descriptors(int32_t n, const double *x, const double *q, const double *box,
                        const int32_t *pair_i, const int32_t *pair_j, int32_t max_pairs,
                        float d_min, float d_max, float *desc, int32_t *idx_nn,
                        int32_t *idx_bead, int32_t *flags, const rb_ctx *ctx,
                        const int32_t *type, float gap_min, float gap_max, void *stream);

/* Two-level routing (the same routes, computed for fewer pairs): a call with
 * flags[RESCREEN] set does what rb_pair_descriptors does with shells and
 * also keeps, in cand_list (capacity max_pairs; flags[NSCREEN] their
 * number; word flags[RB_FLAG_ROUTE_WORK + 2] counts during the call and is
 * left zero), the listed pairs that can still be routed while no bead has
 * moved by margin / 2: centres closer than d_max + margin, and closer than
 * d_min + margin or with G below gap_max + margin; it copies x, q to x_sref
 * (3 x n) and q_sref (4 x n), clears flags[RESCREEN] and increments
 * flags[NRESCREENS].  A call with the flag clear writes desc for, and
 * routes, the pairs of cand_list only, each exactly as a full call would.
 * A listed pair left out has its centres at least d_max apart, or at least
 * d_min apart and no bead pair within gap_max (zero bead energy when
 * gap_max >= rc), until some bead has moved by margin / 2, which
 * rb_rigid_step and rb_rigid_step_fused test (given x_sref, q_sref and
 * half_margin = margin / 2) and report by setting flags[RESCREEN]; every
 * pair-list build sets it too.  A full call may route such a pair to the
 * network or the bead sum when its current bound is looser; this call then
 * leaves it out.  Set flags[RESCREEN] before the first call.  ctx and type
 * are required; gap_max > 0, 0 <= margin < 1e6. */
int rb_pair_descriptors_screened(int32_t n, const double *x, const double *q, const double *box,
                                 const int32_t *pair_i, const int32_t *pair_j, int32_t max_pairs,
                                 float d_min, float d_max, float *desc, int32_t *idx_nn,
                                 int32_t *idx_bead, int32_t *flags, const rb_ctx *ctx,
                                 const int32_t *type, float gap_min, float gap_max, float margin,
                                 int32_t *cand_list, double *x_sref, double *q_sref, void *stream);

/* ---- bead double sum (paper section 2, first equation) -------------------
 * Every bead pair closer than rc contributes; a body pair is skipped only
 * when the shells' lower bound on its closest bead distance (as in
 * rb_pair_descriptors) reaches rc, and a bead only when it lies farther than
 * rc from the other body's bead box, which cannot hold a partner within
 * rc.
 * Per-pair form, for labelling and checks: body i of type type_i at the
 * origin with identity orientation, body j of type type_j at desc's d with
 * orientation q/|q|.  out: 11 x n_pairs FP32 = E, F_j[3], tau_i[3], tau_j[3]
 * in body i's frame, and r_min = min(smallest bead-bead distance, rc).
 * flags (may be NULL): adds the distance tests performed to
 * flags[NTESTS]. */
int rb_bead_pair_eval(const rb_ctx *ctx, int64_t n_pairs, const float *desc, int32_t type_i,
                      int32_t type_j, float *out, int32_t *flags, void *stream);

/* Screen for the per-body form: of the pairs idx[0 .. *count_dev) of the
 * list (idx == NULL: 0 .. *count_dev, capped at max_count), keeps those whose
 * lower bound on the closest bead-centre distance is below rc (the shells'
 * bound of rb_pair_descriptors: bead-centre boxes, and for cylinder-like
 * types capsules and cylinders; the same test rb_bead_pair_forces applies);
 * every other pair has exactly zero bead energy, force and torque.  Writes
 * the kept pair ids to idx_out (capacity max_count, order not specified) and
 * their number to *count_out, to be passed to rb_bead_pair_forces.  tmp: two
 * int32 of caller memory that must be zero before the first call; each call
 * leaves them zero.  flags (may be NULL): the screened-out pairs are added to
 * flags[NEVAL] (rb_bead_pair_forces adds the kept ones). */
int rb_bead_screen(const rb_ctx *ctx, int32_t n, const double *x, const double *q, const int32_t *type,
                   const double *box, const int32_t *pair_i, const int32_t *pair_j, const int32_t *idx,
                   const int32_t *count_dev, int32_t max_count, int32_t *idx_out, int32_t *count_out,
                   int32_t *tmp, int32_t *flags, void *stream);

/* Per-body form for dynamics: the pairs idx[0 .. *count_dev) of the list
 * (idx == NULL: the pairs 0 .. *count_dev), count read on the device and
 * capped at max_count.  Geometry from FP64 state (x 3 x n, q 4 x n, type n),
 * bead sums in FP32.  Adds F, tau of both bodies, the pair energy and the
 * molecular virial W_ab += d_a F_j,b (lab frame) into acc (RB_ACC_LEN(n)). */
int rb_bead_pair_forces(const rb_ctx *ctx, int32_t n, const double *x, const double *q,
                        const int32_t *type, const double *box, const int32_t *pair_i,
                        const int32_t *pair_j, const int32_t *idx, const int32_t *count_dev,
                        int32_t max_count, int64_t *acc, int32_t *flags, void *stream);

/* Two-level form of rb_bead_pair_forces for dynamics over the whole list
 * (pairs 0 .. *count_dev, capped at max_count): the same sums, the same
 * accumulator outputs and the same flags[NEVAL] count (every listed pair),
 * but a launch visits only the listed pairs of a screened list unless
 * flags[RESCREEN] is set.  A launch with flags[RESCREEN] set evaluates the
 * whole list and rebuilds the screened list: screen_list (capacity
 * max_count) receives the pairs whose shells' bound is below rc + margin
 * (as in rb_bead_screen with rc widened by margin),
 * flags[NSCREEN] their number; x, q are copied to x_sref (3 x n) and q_sref
 * (4 x n); flags[RESCREEN] is cleared and flags[NRESCREENS] incremented.
 * A listed pair outside the screened list has no bead pair within rc while
 * every body's beads have moved by at most margin / 2 since then, which
 * rb_rigid_step and rb_rigid_step_fused test (given x_sref, q_sref and
 * half_margin = margin / 2) and report by setting flags[RESCREEN]; every
 * pair-list build sets it too.  Set flags[RESCREEN] before the first call.
 * tmp: four int32 of caller memory, zero before the first call (entries 0..2
 * are left zero, entry 3 holds state between calls).  Forces, torques,
 * energy and virial equal those of rb_bead_pair_forces on the same list bit
 * for bit (same per-pair arithmetic, fixed-point sums). */
int rb_bead_pair_forces_screened(const rb_ctx *ctx, int32_t n, const double *x, const double *q,
                                 const int32_t *type, const double *box, const int32_t *pair_i,
                                 const int32_t *pair_j, const int32_t *count_dev, int32_t max_count,
                                 double margin, int32_t *screen_list, double *x_sref, double *q_sref,
                                 int32_t *tmp, int64_t *acc, int32_t *flags, void *stream);

/* ---- accumulator -----------------------------------------------------------
 * rb_accum_zero clears acc with a fill kernel (graph safe); needed once,
 * before the first evaluation.
 * rb_accum_finalize converts acc into force[3 x n] and torque[3 x n] (FP32,
 * lab frame) and energy_virial[10] (FP64: E then W row-major, may be NULL),
 * and clears acc for the next evaluation.  flags (may be NULL): a total of
 * 2^30 or more in magnitude sets flags[RB_FLAG_FIXOVF]. */
int rb_accum_zero(int32_t n, int64_t *acc, void *stream);
int rb_accum_finalize(int32_t n, int64_t *acc, float *force, float *torque,
                      double *energy_virial, int32_t *flags, void *stream);

/* ---- energy network (paper section 2, g_NN_U; supplementary section 6) ---
 * params: RB_MLP_NPARAMS FP32 (16-byte aligned), layer by layer W_l (out x
 * in, row major) then b_l, dims 7 -> 128 -> 128 -> 128 -> 128 -> 1, SiLU on
 * the hidden layers.
 * norm (host, 16 floats): in_shift[7], in_scale[7], out_shift, out_scale;
 * the network sees u' = (u - in_shift) * in_scale and E = e' * out_scale +
 * out_shift.  precision: RB_PREC_BF16 (first and last layer FP32, the three
 * 128x128 layers BF16 MFMA with FP32 accumulation and BF16 activations) or
 * RB_PREC_FP32.  desc: 7 x n_pairs FP32. */
int rb_nn_pair_eval(const float *params, const float *norm, int precision, int64_t n_pairs,
                    const float *desc, float *energy, void *stream);

/* Input gradient by a hand-written reverse pass.  gE (n_pairs, NULL = all
 * ones) seeds the reverse pass.  Outputs (each may be NULL): energy
 * (n_pairs), dE_ddesc (7 x n_pairs, times gE), pair_ft (9 x n_pairs,
 * F_j, tau_i, tau_j in body i's frame, times gE): F_j = -dE/dd,
 * tau_j = -(w g_v - g_w v + v x g_v)/2 for q = (w, v) and g = dE/dq,
 * tau_i = -tau_j - d x F_j. */
int rb_nn_pair_grad(const float *params, const float *norm, int precision, int64_t n_pairs,
                    const float *desc, const float *gE, float *energy, float *dE_ddesc,
                    float *pair_ft, void *stream);

/* Network forces for dynamics: pairs idx[0 .. *count_dev) (idx == NULL: all
 * pairs up to *count_dev), desc from rb_pair_descriptors, q (4 x n FP64)
 * for the rotation to the lab frame.  The energy is multiplied by a C1
 * switch S(|d|) = 1 below sw_lo, smoothstep to 0 at sw_hi (sw_hi <= sw_lo
 * disables it), and forces/torques come from the switched energy.  Adds
 * into acc like rb_bead_pair_forces. */
int rb_nn_pair_forces(const float *params, const float *norm, int precision, int32_t n,
                      const double *q, const int32_t *pair_i, const int32_t *pair_j,
                      const float *desc, int32_t desc_stride, const int32_t *idx,
                      const int32_t *count_dev, int32_t max_count, float sw_lo, float sw_hi,
                      int64_t *acc, int32_t *flags, void *stream);

/* ---- symmetry-reduced descriptor of cube pairs -----------------------------
 * Paper, supplementary section 1: a pair of identical cubes reduced to six
 * numbers s = (p_x, p_y, p_z, alpha_1, alpha_2, alpha_3).  Body 1's axes are
 * relabelled and their signs chosen (signed permutation g, reflections
 * included) so that p = g d has p_x >= p_y >= p_z >= 0; with
 * M = g R(q) g^T, w is body 2's face normal with the largest x component,
 * alpha_1 = acos(w_x), alpha_2 = atan2(w_z, w_y); alpha_3 in [0, pi/2) is
 * the turn of body 2 about w: the angle in the y-z plane of Q v, Q the
 * smallest rotation taking w to (1, 0, 0) and v another face normal, modulo
 * pi/2.  Ties go to the lower axis index.  The network's seven inputs are
 * s = (p_x, p_y, p_z, w_y, w_z, cos 4 alpha_3, sin 4 alpha_3): the same
 * numbers through smooth functions (w_y = sin a1 cos a2, w_z = sin a1 sin a2),
 * free of the angles' polar singularity at w = (1, 0, 0) and of alpha_3's
 * cut.  For the pairs k = 0 .. count (count = *count_dev capped at
 * max_count, or n_pairs when count_dev is NULL), pair pid = idx[k] (or k) of
 * desc (7 x stride: d, q): sym (7 x max_count, or 7 x n_pairs without
 * count_dev) receives s, jac (49 x the same) the Jacobian ds_r/du_m at row
 * r * 7 + m (u = (d, q), q as four free components; R(q) taken as the
 * homogeneous form v -> q v q^*).  s still switches where the choices do
 * (ties in the sort or in the choice of w); the Jacobian is that of the
 * branch taken. */
int rb_cube_sym_descriptors(int64_t n_pairs, const float *desc, int64_t stride, const int32_t *idx,
                            const int32_t *count_dev, int64_t max_count, float *sym, float *jac,
                            void *stream);

/* rb_nn_pair_grad with the network taking the symmetry-reduced descriptor:
 * the network reads sym (7 x n_pairs), dE_ddesc receives dE/du =
 * J^T dE/ds (7 x n_pairs, with respect to desc's (d, q)), and pair_ft the
 * forces and torques from it as in rb_nn_pair_grad (desc: 7 x n_pairs). */
int rb_nn_pair_grad_sym(const float *params, const float *norm, int precision, int64_t n_pairs,
                        const float *desc, const float *sym, const float *jac, const float *gE,
                        float *energy, float *dE_ddesc, float *pair_ft, void *stream);

/* ---- four-number descriptor of cylinder pairs -----------------------------
 * Paper section 2 (a cylinder pair depends on four numbers thanks to the
 * cylindrical symmetry) and supplementary section 2: in body 1's frame with
 * z along its axis (oriented so that p_z >= 0) and x chosen so that p_y = 0,
 * body 2's centre is (p_r, 0, p_z) and its axis a unit vector a at spherical
 * angles (theta, phi).  The network's seven inputs are the smooth functions
 * s = (p_r^2, p_z^2, a_z^2, (p_r a_x)^2, p_r a_x a_z p_z, 0, 0), which are
 * also unchanged when body 2 is turned end over end and under the mirror
 * y -> -y of that frame; in the pair descriptor (d, q) they are polynomials
 * of d and the axis A = q e_z q^* (body z axis = cylinder axis).  Layout and
 * arguments as rb_cube_sym_descriptors; jac is the Jacobian of those
 * polynomials (q as four free components, homogeneous form). */
int rb_cyl_sym_descriptors(int64_t n_pairs, const float *desc, int64_t stride, const int32_t *idx,
                           const int32_t *count_dev, int64_t max_count, float *sym, float *jac,
                           void *stream);

/* rb_nn_pair_forces for cylinder pairs: the network sees the four-number form
 * of each pair's (d, q) (as rb_cyl_sym_descriptors defines it), computed
 * with its Jacobian inside the kernel; forces and torques from dE/du =
 * J^T dE/ds and the closed form of rb_nn_pair_grad.  The torque of each
 * cylinder about its own axis is zero.  Arguments as rb_nn_pair_forces. */
int rb_nn_pair_forces_cyl(const float *params, const float *norm, int precision, int32_t n,
                          const double *q, const int32_t *pair_i, const int32_t *pair_j,
                          const float *desc, int32_t desc_stride, const int32_t *idx,
                          const int32_t *count_dev, int32_t max_count, float sw_lo, float sw_hi,
                          int64_t *acc, int32_t *flags, void *stream);

/* rb_nn_pair_forces with the symmetry-reduced descriptor: sym and jac (row
 * stride max_count) hold the descriptor and Jacobian of launch row k, i.e.
 * of pair idx[k], as rb_cube_sym_descriptors writes them from the same idx
 * and count. */
int rb_nn_pair_forces_sym(const float *params, const float *norm, int precision, int32_t n,
                          const double *q, const int32_t *pair_i, const int32_t *pair_j,
                          const float *desc, int32_t desc_stride, const float *sym, const float *jac,
                          const int32_t *idx, const int32_t *count_dev, int32_t max_count, float sw_lo,
                          float sw_hi, int64_t *acc, int32_t *flags, void *stream);

/* ---- rigid-body velocity Verlet (FP64) -------------------------------------
 * State: x (3 x n), P (3 x n linear momentum), q (4 x n), L (3 x n angular
 * momentum in the body frame).  phase 1: half kick with force/torque (lab
 * frame, 3 x n FP32 each), drift, free rotation split as
 * R3(dt/2) R2(dt/2) R1(dt) R2(dt/2) R3(dt/2) (NO_SQUISH, Miller et al.,
 * J. Chem. Phys. 116, 8649, 2002), renormalise q; if x_ref != NULL and a
 * body moved more than half_skin from x_ref, sets flags[REBUILD]; if x_sref
 * != NULL (then q_sref too) and some bead of a body may have moved more than
 * half_margin since the state (x_sref, q_sref), i.e.
 * |x - x_sref| + 2 rho |vec(q_sref^* q)| > half_margin with rho the type's
 * largest bead radius, sets flags[RESCREEN] (the screened list of
 * rb_bead_pair_forces_screened); each body whose |q|^2 had drifted from 1
 * by more than 1e-10 before the renormalisation adds 1 to flags[QDRIFT]
 * (flags may be NULL only when x_ref and x_sref are).  phase 2:
 * second half kick; writes kinetic[2] = (translational, rotational) kinetic
 * energy (FP64 deterministic reduction).  ws: rb_rigid_workspace_bytes(n),
 * zero-filled before its first use.
 * Constant temperature (paper section 3, Nose-Hoover): nh != NULL is a
 * device array of 5 doubles, (xi, eta, s, Q, g kT), with xi = eta = 0,
 * s = 1 and the thermostat mass Q and g kT (g degrees of freedom, e.g.
 * 6 n - 3) set by the caller.  Phase 2 then follows the half kick with the
 * thermostat flow for dt on every momentum, as two halves U(dt/2), each
 * xi += (h/2)(2K - g kT)/Q, momenta *= exp(-xi h), eta += xi h,
 * xi += (h/2)(2K' - g kT)/Q (h = dt/2, K' the scaled kinetic energy),
 * written back to nh with the accumulated momentum factor s, which the next
 * phase 1 (given the same nh) applies to P and L before its half kick.
 * kinetic[] holds the energies before the thermostat.  Conserved:
 * K + U + Q xi^2 / 2 + g kT eta.  nh == NULL: constant energy. */
size_t rb_rigid_workspace_bytes(int32_t n);
int rb_rigid_step(const rb_ctx *ctx, int phase, int32_t n, double dt, double *x, double *P,
                  double *q, double *L, const int32_t *type, const float *force,
                  const float *torque, const double *x_ref, double half_skin, const double *x_sref,
                  const double *q_sref, double half_margin, double *kinetic, double *nh, int32_t *flags,
                  void *ws, size_t ws_bytes, void *stream);

/* Step boundary in one launch, for loops that keep the forces in the
 * accumulator: rb_accum_finalize (acc -> force, torque FP32, energy_virial
 * FP64 (may be NULL), acc cleared) + phase 2 (kinetic energy at the full
 * step) + phase 1 of the next step, with the same arithmetic in the same
 * order.  A run of K steps is phase 1, then (pair list, forces into acc,
 * rb_rigid_step_fused) K - 1 times, then pair list, forces, finalize,
 * phase 2.  The accumulator and quaternion checks of rb_accum_finalize and
 * phase 1 set flags[FIXOVF] and flags[QDRIFT] here too.
 * kinetic may be NULL: the kinetic energy of that step is then
 * not reduced (the grid-wide reduction is the launch's serial tail).  ws as
 * for phase 2, zero-filled before its first use. */
int rb_rigid_step_fused(const rb_ctx *ctx, int32_t n, double dt, double *x, double *P, double *q,
                        double *L, const int32_t *type, int64_t *acc, float *force, float *torque,
                        double *energy_virial, const double *x_ref, double half_skin,
                        const double *x_sref, const double *q_sref, double half_margin,
                        double *kinetic, int32_t *flags, void *ws, size_t ws_bytes, void *stream);

/* Allocation-free variant of rb_rigid_step_fused, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments without ws, the same
 * kernel and results bit for bit.  The kinetic partial sums and the
 * completion ticket live in a file-scope device array of the library
 * (262 656 bytes per device, held until the process ends); the call
 * allocates nothing, clears the ticket with a small kernel before the step
 * and needs n <= rb_rigid_step_fused_noalloc_max_bodies() (4 194 304),
 * else RB_ERR_INVALID_ARG.  Every call on one device shares that device's
 * array: calls that overlap on one device (different streams or host
 * threads without ordering) race and give wrong kinetic energies. */
size_t rb_rigid_step_fused_noalloc_max_bodies(void);
int rb_rigid_step_fused_noalloc(const rb_ctx *ctx, int32_t n, double dt, double *x, double *P, double *q,
                                double *L, const int32_t *type, int64_t *acc, float *force, float *torque,
                                double *energy_virial, const double *x_ref, double half_skin,
                                const double *x_sref, const double *q_sref, double half_margin,
                                double *kinetic, int32_t *flags, void *stream);

/* Forces of a routed list in one call: the network forces of the pairs
 * idx_nn[0 .. *nn_count) as rb_nn_pair_forces (form 0: (d, q) input) or
 * rb_nn_pair_forces_cyl (form 1: cylinder four-number form), and the bead
 * double sums of the pairs idx_bead[0 .. *bead_count) as rb_bead_pair_forces
 * (paper section 2: the bead sum takes the pairs outside the network's
 * domain), into the same accumulator and flags (flags[NEVAL] counts both).
 * With BF16 precision and templates whose staging fits the LDS of the
 * network kernel's weight image (36 x max_beads + total_beads float4 within
 * 104 976 bytes: up to 176 beads for a single type) one launch does both:
 * after its network tiles each block of the persistent grid claims
 * fallback pairs, one per wave and round, from a counter in flags (words
 * RB_FLAG_FB_WORK..+1, zero between calls, left zero); otherwise the two
 * kernels run one after the other.  The per-pair arithmetic is that of
 * the two calls it replaces, and so are the fixed-point sums.  ctx:
 * templates and bead potential; x (3 x n), q (4 x n), type (n), box[3] as
 * for the bead sums. */
int rb_nn_pair_forces_routed(const rb_ctx *ctx, const float *params, const float *norm, int precision, int form,
                             int32_t n, const double *x, const double *q, const int32_t *type, const double *box,
                             const int32_t *pair_i, const int32_t *pair_j, const float *desc, int32_t desc_stride,
                             const int32_t *idx_nn, const int32_t *nn_count_dev, const int32_t *idx_bead,
                             const int32_t *bead_count_dev, int32_t max_count, float sw_lo, float sw_hi,
                             int64_t *acc, int32_t *flags, void *stream);

/* ---- training step (energy loss, Adam) ------------------------------------
 * Paper section 2: the network g_NN_U is fitted by regression to pair
 * energies that the bead method computes for sampled pair configurations
 * (the same section: training data come from composite-body simulations;
 * supplementary section 1: fully connected feed-forward networks trained on
 * such samples); section 3 and supplementary section 6 then take forces and
 * torques from this energy network's gradient.  The optimiser is Adam
 * (Kingma and Ba, ICLR 2015); the paper does not name one.
 * One step on the batch idx[0 .. batch) of a data set (desc 7 x n_data
 * FP32, labels n_data FP32): forward with saved activations, loss
 * mean((e' - y')^2) in normalised units, reverse pass, weight gradients,
 * Adam (Kingma and Ba) on the FP32 master params with moments m, v and
 * 1-based step number t.  loss (device, 1 float) receives the batch loss
 * before the update; grad_out (RB_MLP_NPARAMS or NULL) the gradient.
 * ws: rb_nn_train_workspace_bytes(batch). */
size_t rb_nn_train_workspace_bytes(int32_t batch);
int rb_nn_train_step(float *params, float *adam_m, float *adam_v, int32_t t, const float *norm,
                     int precision, int32_t batch, const float *desc, int64_t n_data,
                     const float *labels, const int32_t *idx, float lr, float beta1, float beta2,
                     float eps, float *loss, float *grad_out, void *ws, size_t ws_bytes,
                     void *stream);

/* Training step with force and torque matching (on top of the energy loss):
 * loss[0] = mean((e' - y')^2) as rb_nn_train_step, loss[1] =
 * lam_f mean |F_j - F_j*|^2 + lam_t mean |tau_j - tau_j*|^2 with F_j, tau_j
 * the network's pair force and torque (body i's frame, from dE/du as
 * rb_nn_pair_grad gives them) and ft_labels (6 x n_data FP32: F_j*, tau_j*,
 * e.g. rb_bead_pair_eval's outputs 1..3 and 7..9).  The paper trains on
 * energies (section 2) and notes that forces fitted directly are more
 * accurate than gradients of an energy fit (supplementary section 6); this
 * step fits the energy's gradient to them.  The gradient of the matching
 * term is exact: it is the parameter gradient of the directional derivative
 * of E along v = dloss/dg, carried forward as tangents through every layer
 * and differentiated in reverse through both the primal and the tangent
 * chains (second derivative of SiLU where they meet); each sample adds a
 * tangent row to the weight-gradient GEMMs.  batch: positive multiple of
 * 32, at most 2^18.  ws: rb_nn_train_fm_workspace_bytes(batch). */
size_t rb_nn_train_fm_workspace_bytes(int32_t batch);
int rb_nn_train_step_fm(float *params, float *adam_m, float *adam_v, int32_t t, const float *norm,
                        int precision, int32_t batch, const float *desc, int64_t n_data,
                        const float *labels, const float *ft_labels, const int32_t *idx, float lam_f,
                        float lam_t, float lr, float beta1, float beta2, float eps, float *loss,
                        float *grad_out, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* RIGIDNN_H */
