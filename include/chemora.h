/* chemora.h -- C ABI of the MI355X (gfx950) BSSN right-hand-side library.
 *
 * The library evaluates the right-hand side of the BSSN form of the Einstein
 * equations with high-order finite differences on a Cartesian patch, and
 * advances a patch (or a batch of patches) by classic fourth-order or
 * third-order SSP Runge-Kutta steps, with the Hamiltonian and momentum
 * constraints as diagnostics and the algebraic constraints restorable (Chemora,
 * arXiv:1307.6488: the McLachlan BSSN evolution of section "Binary Black Hole
 * Simulations" -- derivative, advection and evaluation kernels, boundary
 * condition and time-integrator update -- and the per-point "numerical
 * kernel over a local grid section with ghost zones filled outside the
 * kernel" model of section "CaKernel Programming Abstractions").
 *
 * Conventions shared by every call
 *  - Every entry point returns a chemora_status (0 = OK, < 0 = error) and
 *    never aborts, except the queries documented as returning a value (a
 *    size, a count, a ghost width, a tile variant >= 0 or a negative
 *    status).  On error chemora_last_error() returns a thread-local,
 *    NUL-terminated message owned by the library (valid until the next call
 *    on the same thread).
 *  - All argument checks run on the host before any HIP call; a call that
 *    returns CHEMORA_EINVAL has enqueued no GPU work.
 *  - Device pointers are plain HIP device addresses (e.g. a torch tensor's
 *    data_ptr()); the caller owns and keeps them alive until the work has
 *    completed on `stream`.  `stream` is a hipStream_t passed as void*
 *    (NULL = the default stream).  Work is enqueued asynchronously; only
 *    chemora_check_finite, chemora_tune, chemora_plan_create,
 *    chemora_plan_create_rk3 and chemora_plan_destroy synchronise (each says
 *    so).  Device faults
 *    surface at the caller's next synchronisation.
 *  - CHEMORA_EDEVICE reports a failed HIP launch/runtime call.
 *
 * State layout (one patch): 24 grid functions (GFs), FP64, structure of
 * arrays.  Element (f, i, j, k) -- GF f, stored point (i, j, k) counted
 * from the first ghost point -- sits at u[f*sf + k*sz + j*sy + i].  Each axis
 * stores n[a] interior points plus `ghost` points on both sides; interior
 * point (0,0,0) is stored at (ghost, ghost, ghost) and sits at `origin`,
 * spacing h in all three directions.  Requirements:
 *     sy >= n[0] + 2g, and sy >= n[0] + 2g + 1 when n[0] is odd (the
 *     stencil staging moves pairs of doubles and may read one element of
 *     row padding), sz >= sy*(n[1] + 2g), sf >= sz*(n[2] + 2g),
 *     24*sf*8 + 64 bytes <= 4 GiB (32-bit byte offsets), every pointer
 *     8-byte aligned.  Row padding never affects a result, nor do the 3-D
 *     ghost corners with static or periodic boundaries (they may be read,
 *     never written; NaN there is harmless).  With the radiative boundary
 *     every ghost point, corners included, is an evolved point.
 * GF order: 0 chi | 1-6 gt_xx gt_xy gt_xz gt_yy gt_yz gt_zz | 7 K |
 *           8-13 At_xx..At_zz | 14-16 Gt^x Gt^y Gt^z | 17 alpha |
 *           18-20 beta^x beta^y beta^z | 21-23 B^x B^y B^z.
 */
#ifndef CHEMORA_H
#define CHEMORA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CHEMORA_OK = 0,
  CHEMORA_EINVAL = -1,        /* invalid argument (nothing enqueued)          */
  CHEMORA_EDEVICE = -2,       /* HIP runtime / launch failure                  */
  CHEMORA_ENOMEM = -3,        /* library-side allocation failed (plans only)   */
  CHEMORA_EUNSUPPORTED = -4,  /* valid but not built (e.g. order/precision)    */
  CHEMORA_ENOTFINITE = -5     /* chemora_check_finite found NaN/Inf            */
} chemora_status;

enum { CHEMORA_NGF = 24 };
enum { CHEMORA_LAPSE_ONE_PLUS_LOG = 0, CHEMORA_LAPSE_HARMONIC = 1, CHEMORA_LAPSE_FROZEN = 2 };
enum { CHEMORA_SHIFT_GAMMA_DRIVER = 0, CHEMORA_SHIFT_FROZEN = 1 };
enum { CHEMORA_BC_STATIC = 0, CHEMORA_BC_PERIODIC = 1, CHEMORA_BC_RADIATIVE = 2 };
enum { CHEMORA_PREC_FP64 = 0, CHEMORA_PREC_SPLIT = 1 };

/* Discretisation and gauge parameters.  This is the kernel descriptor of
 * section "Kernel Abstractions": the parameters a numerical kernel needs and
 * the extent of its stencil (fd_order, upwind and ko_radius fix how far a
 * point's neighbourhood reaches; ghost says how much of it is stored).  */
typedef struct chemora_params {
  int32_t fd_order;   /* 4 or 8: centred first/second/mixed derivatives      */
  int32_t ghost;      /* g >= chemora_required_ghost(fd_order, upwind, ko)   */
  int32_t upwind;     /* 1: lopsided advection stencils (offsets -1..3 at
                         order 4, -3..5 at order 8, mirrored for beta < 0);
                         0: centred advection                               */
  int32_t ko_radius;  /* Kreiss-Oliger radius r (0 = off), r <= g           */
  double eps_diss;    /* Kreiss-Oliger strength eps >= 0                     */
  int32_t lapse;      /* CHEMORA_LAPSE_*                                     */
  int32_t shift;      /* CHEMORA_SHIFT_*                                     */
  double eta;         /* Gamma-driver damping                                */
  int32_t bc;         /* CHEMORA_BC_*: ghost treatment inside the steps.
                         STATIC: ghosts hold their values; PERIODIC: images
                         of the interior; RADIATIVE: every ghost point
                         evolves by the outgoing-wave (Sommerfeld) condition
                         d_t u = -v (x^i/r) d_i u - v (u - u_inf)/r, r = |x|
                         from the coordinates (origin), at least h/2, with
                         second-order centred differences (one-sided into
                         the box at its faces), v = sqrt 2 for the 1+log
                         lapse and 1 otherwise, u_inf the flat-space value,
                         frozen gauge variables held -- the boundary step of
                         section "Binary Black Hole Simulations with
                         Chemora" (timer row "Boundary condition"), which
                         the paper does not spell out                       */
  int32_t precision;  /* CHEMORA_PREC_FP64, or CHEMORA_PREC_SPLIT (order 4
                         only, else EUNSUPPORTED): stencil inputs are FP64
                         differences rounded to FP32, combined with FP32
                         weights; the algebra is FP32; the state, the RK
                         combination and the 1/chi terms of D_i D_j alpha
                         and the Gt source stay FP64                        */
  double chi_split;   /* split precision: points with chi < chi_split (near
                         a puncture) evaluate the whole chi phase (d chi,
                         D~D~chi, R^chi, the chi RHS) in FP64 (>= 0, +inf
                         allowed; EINVAL otherwise; ignored for FP64)       */
} chemora_params;

/* One Cartesian patch: a grid section with its ghost zones, holding the 24
 * grid functions of the state (section "Grid Abstractions": a grid function
 * is one variable of the application over the grid; the grid geometry gives
 * its spacing and coordinates).  The library never allocates or frees u. */
typedef struct chemora_patch {
  int32_t n[3];       /* interior points nx, ny, nz (>= 1; >= ghost when the
                         boundary is periodic)                              */
  int32_t reserved;   /* must be 0                                            */
  int64_t sy, sz, sf; /* element strides of y, z and the GF index            */
  double h;           /* grid spacing (> 0)                                   */
  double origin[3];   /* coordinates of interior point (0,0,0): metadata,
                         except for the radiative boundary (finite there)  */
  double *u;          /* device pointer: 24 GFs, caller-owned                */
} chemora_patch;

/* Ghost width that one right-hand-side evaluation reads:
 * max(order/2, order/2+1 if upwind, ko_radius).  Returns < 0 for an
 * unsupported order. */
int chemora_required_ghost(int fd_order, int upwind, int ko_radius);

/* Right-hand side of all 24 BSSN equations at every interior point
 * (moving-puncture BSSN with 1+log / harmonic / frozen lapse and the
 * advective Gamma-driver shift, Kreiss-Oliger dissipation added to every
 * evolved variable).  Defined by section "Scientific Motivation" (the BSSN
 * form of the Einstein equations: thousands of terms per point, first,
 * second and mixed derivatives of the evolved variables) and section
 * "Binary Black Hole Simulations with Chemora" (the derivative, advection
 * and evaluation kernels of the McLachlan code, partially upwinded
 * stencils); it is the point-wise numerical kernel of section "Kernel
 * Abstractions", applied to every interior point of a grid section whose
 * ghost zones were filled outside the kernel.  Reads patch->u (ghosts
 * included: the caller provides them), writes the interior entries of
 * `rhs` (the patch's layout and strides; ghost and padding entries are not
 * written), and with the radiative boundary also every ghost entry (the
 * boundary condition's right-hand side).  `rhs` is caller-owned device memory and must not overlap the
 * patch state.  Asynchronous on `stream`.  EINVAL (bad params, strides,
 * NULL / misaligned / overlapping pointers) and EUNSUPPORTED are returned
 * before any GPU work; EDEVICE if the launch fails. */
int chemora_bssn_rhs(const chemora_params *params, const chemora_patch *patch, double *rhs,
                     void *stream);

/* Number of doubles of caller-provided scratch rk4_step needs: 3*24*sf
 * (two stage buffers and the RK accumulator). */
size_t chemora_rk4_scratch_elems(const chemora_patch *patch);

/* One classic RK4 step of size dt > 0 applied to patch->u in place: the
 * method-of-lines update the paper's framework applies after each
 * right-hand-side evaluation (section "Binary Black Hole Simulations with
 * Chemora", timer rows "Time integrator data copy" and "Boundary
 * condition"; the paper runs a third-order scheme, see chemora_rk3_step).
 * Four stage launches; each evaluates the right-hand side of its stage input
 * and applies the stage combination in the same pass (16 state transfers
 * per point and step).
 * BC static: ghost points of u are left untouched and are the ghosts of every
 * stage.  BC periodic: ghosts of every stage input and of the result are
 * refilled with periodic images of the interior.  BC radiative: the ghost
 * points are advanced by the same stages with the boundary condition's
 * right-hand side (one extra launch per stage).  `scratch` is a device
 * buffer of at least chemora_rk4_scratch_elems(patch) doubles that must not
 * overlap u; its content on entry is ignored and on return is unspecified. */
int chemora_rk4_step(const chemora_params *params, const chemora_patch *patch, double dt,
                     double *scratch, void *stream);

/* Most doubles of scratch chemora_rk4_step_noalloc holds per GPU (64 MiB):
 * patches with chemora_rk4_scratch_elems(patch) <= this, e.g. 42^3 interior
 * points with 3 ghosts and rows padded to 8 doubles. */
#define CHEMORA_NOALLOC_SCRATCH_ELEMS ((size_t)8 << 20)

/* chemora_rk4_step for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, and harnesses that forbid
 * allocation.  The same computation as chemora_rk4_step (bitwise, same tile
 * variant), with the three scratch states in a buffer the library holds per
 * GPU (a static device array of CHEMORA_NOALLOC_SCRATCH_ELEMS doubles,
 * loaded with the library and kept until the process ends) instead of a
 * caller's.  No hipMalloc, hipFree or other allocation, no memset: every
 * scratch value the step reads it has written first in the same call.
 * Errors: as chemora_rk4_step before any HIP call; EINVAL if
 * chemora_rk4_scratch_elems(patch) exceeds CHEMORA_NOALLOC_SCRATCH_ELEMS;
 * EDEVICE if the buffer's device address cannot be obtained.  All calls on
 * one GPU share its buffer: calls whose executions overlap on that GPU
 * (other streams, other host threads) race and give undefined results;
 * calls ordered on one stream are safe. */
int chemora_rk4_step_noalloc(const chemora_params *params, const chemora_patch *patch, double dt,
                             void *stream);

/* Stage s (1..4) of the step chemora_rk4_step performs, for callers that
 * interleave their own work between stages or time them one by one.
 * Calling s = 1, 2, 3, 4 in this order with the same dt and scratch is the
 * same computation as one chemora_rk4_step (bitwise); any other order is
 * undefined.  Stage 1 also prepares the stage buffers' ghosts (static BC). */
int chemora_rk4_stage(const chemora_params *params, const chemora_patch *patch, int stage, double dt,
                      double *scratch, void *stream);

/* Number of doubles of caller-provided scratch rk3_step needs: 2*24*sf (two
 * stage buffers). */
size_t chemora_rk3_scratch_elems(const chemora_patch *patch);

/* One third-order Runge-Kutta step of size dt > 0 applied to patch->u in
 * place -- the integrator of the paper's production runs (section "Binary
 * Black Hole Simulations"), taken as the strong-stability-preserving scheme
 * of Shu and Osher: S_A = u + dt k(u); S_B = 3/4 u + 1/4 S_A + dt/4 k(S_A);
 * u = 1/3 u + 2/3 S_B + 2dt/3 k(S_B).  Three launches, 8 state transfers per
 * point instead of RK4's 16.  Boundaries, scratch (at least
 * chemora_rk3_scratch_elems(patch) doubles, not overlapping u; content on
 * entry ignored, on return unspecified), tile variant and errors as for
 * chemora_rk4_step. */
int chemora_rk3_step(const chemora_params *params, const chemora_patch *patch, double dt,
                     double *scratch, void *stream);

/* Psi4, the Newman-Penrose Weyl scalar of outgoing gravitational radiation,
 * at every interior point: the paper's second GPU workload beside the
 * evolution (section "Binary Black Hole Simulations with Chemora", timer row
 * "Compute Psi4"), which it does not spell out.  From the 3+1 data in
 * vacuum -- gamma_ij = gt_ij / chi, K_ij = (At_ij + gt_ij K / 3) / chi --
 * the electric and magnetic parts of the Weyl tensor
 *   E_ij = R_ij - K_ik K^k_j + K K_ij,   B_ij = sym_ij eps_i^kl D_k K_lj
 * (R_ij the evolution's Ricci tensor, eps_ijk = sqrt(det gamma) [ijk]) are
 * projected on mbar = (e_theta - i e_phi)/sqrt 2 of the radial tetrad
 * obtained by Gram-Schmidt in gamma from (x, y, z), the theta-like vector
 * gamma^ad eps_dbc v1^b (x, y, z)^c and v1 = (-y, x, 0) (v1 = (0, 1, 0) on
 * the z axis, (0, 0, 1) replacing (x, y, z) at the origin):
 *   Psi4 = (E_ij - i B_ij) mbar^i mbar^j,
 * which is -d_t^2 h_+ + i d_t^2 h_x for an outgoing wave.  Coordinates come
 * from patch.origin and h (must be finite); centred first and second
 * derivatives of the patch's order.  psi4 holds two grid functions with the
 * patch's strides (2 * patch.sf doubles): the real part at psi4[0 .. sf),
 * the imaginary part at psi4[sf .. 2 sf); ghost entries are not written;
 * psi4 must not overlap the state.  Errors as chemora_bssn_rhs, EINVAL for
 * a NULL, misaligned or overlapping psi4 or a non-finite origin. */
int chemora_psi4(const chemora_params *params, const chemora_patch *patch, double *psi4, void *stream);

/* Momentum constraint M_i = gt^jk (d_j At_ki - Gt^l_jk At_li - Gt^l_ji At_kl)
 * - 3/(2 chi) gt^kl At_il d_k chi - 2/3 d_i K of the state at every interior
 * point -- the conformal form of the ADM momentum constraint, a diagnostic
 * like the Hamiltonian constraint (the paper's BBH runs monitor the
 * constraints, section "Binary Black Hole Simulations").  Centred first
 * derivatives of the patch's order.  M holds three grid functions with the
 * patch's strides (3 * patch.sf doubles, M_x at M[0 .. sf)); ghost entries
 * are not written; M must not overlap the state.  Errors as
 * chemora_bssn_rhs, EINVAL for a NULL, misaligned or overlapping M. */
int chemora_momentum_constraint(const chemora_params *params, const chemora_patch *patch, double *M,
                                void *stream);

/* Restores the algebraic constraints of the conformal variables, det(gt) = 1
 * and gt^ij At_ij = 0, at every interior point of patch->u in place:
 * gt_ij <- gt_ij / det(gt)^(1/3), then At_ij <- At_ij - gt_ij (gt^kl At_kl) / 3
 * with the rescaled metric.  Not part of the step (call it between steps, as
 * moving-puncture codes do; the paper leaves it to the evolution code it
 * accelerates).  Periodic BC: ghosts refilled with the images afterwards;
 * static BC: ghosts untouched.  One launch, 12 reads and 12 writes per point.
 * Errors as chemora_bssn_rhs. */
int chemora_enforce_constraints(const chemora_params *params, const chemora_patch *patch, void *stream);

/* Hamiltonian constraint H = chi gt^ij R_ij + 2/3 K^2 - At_ij At^ij of the
 * state at every interior point (a diagnostic, not part of the step; the
 * paper's BBH runs monitor the constraints, section "Binary Black Hole
 * Simulations").  H holds one grid function with the patch's strides
 * (patch.sf doubles); its ghost entries are not written.  Computed by the
 * stage kernel's own stencils and Ricci tensor (precision as params).
 * Errors as chemora_bssn_rhs. */
int chemora_hamiltonian(const chemora_params *params, const chemora_patch *patch, double *H, void *stream);

/* ---- autotuner: tile variants per size class -----------------------------
 * The stage kernel runs in one of several tile shapes ("variants": 0 = 64x4,
 * 1 = 64x8, 2 = 32x8, 3 = 32x16 points per work-group, x by y, one z plane;
 * 4 = 32x8x2 and 5 = 32x4x4, x by y by z, whose work-groups share the
 * z halo of their planes; order 8 builds 0 and 2).  In FP64 all variants compute bit-identical results; in
 * split precision they agree to FP32 rounding (their FP32 kernels are
 * compiled separately).  They differ in lane use on ragged extents, halo
 * overhead, staging depth and occupancy.  The choice is
 * kept per size class -- (GPU architecture, fd_order, upwind, staged reach,
 * precision, bucket of n[0]: <=32 <=64 <=96 <=128 >128, bucket of n[1]:
 * <=16 <=32 <=64 >64) -- in a process-wide table (thread-safe) that every
 * call and plan consults; a class without an entry uses variant 2 (32 x 8).
 * The paper tunes tile shapes with a model (section "Tile Size Selection");
 * here they are timed on the target GPU, as its autotuning sections
 * describe. */

/* Chooses the variant for patch's class: an entry already in the table (set,
 * tuned or loaded) is kept; otherwise every built variant is timed on RK4
 * stage-2 launches of this patch (reads patch.u and scratch, overwrites the
 * S_B and accumulator parts of scratch; scratch as for chemora_rk4_step):
 * one warm-up launch each, then three rounds that time every variant in
 * turn over two launches, and the variant with the fastest sample is
 * recorded.  cache_path (may be NULL): a JSON cache read
 * before and rewritten after (written to <path>.tmp, then renamed); entries
 * of this process win over the file's.  Synchronises `stream`.  *variant
 * (may be NULL) receives the choice.  Errors as chemora_rk4_step, EINVAL if
 * the cache cannot be written, EDEVICE on HIP failure. */
int chemora_tune(const chemora_params *params, const chemora_patch *patch, double *scratch,
                 const char *cache_path, void *stream, int32_t *variant);

/* Variant the library uses for patch's class (>= 0), or a negative status. */
int chemora_tile_variant(const chemora_params *params, const chemora_patch *patch);

/* Sets the variant of patch's class (EINVAL: unknown id; EUNSUPPORTED: not
 * built for params->fd_order).  Takes effect for later calls and plans. */
int chemora_set_tile_variant(const chemora_params *params, const chemora_patch *patch, int32_t variant);

/* Tile extent of a variant in x and y (either pointer may be NULL). */
int chemora_tile_variant_shape(int32_t variant, int32_t *tile_x, int32_t *tile_y);

/* Tile depth of a variant: the z planes one work-group evaluates (>= 1; the
 * tuner's z-sweep dimension), or a negative status for an unknown id. */
int chemora_tile_variant_depth(int32_t variant);

/* ---- batched form: many patches advanced together ------------------------
 * Section "Cactus-Carpet Computational Infrastructure": block-structured
 * grids with many patches (refinement levels, multi-block) per process;
 * section "Grid Abstractions": the grid hierarchy of such patches; section
 * "Stencils and Dynamic Tile Selection": the tile shape of each kernel
 * launch chosen for the grid it runs on.
 * A plan records a list of patches (each with its own spacing h, extents and
 * strides; all share params) and their RK4 scratch buffers.  One RK4 step of
 * every patch is captured once into a HIP graph: per RK stage one launch
 * per tile variant covers the tiles of all the plan's patches of that
 * variant, dispatched in one of two ways that compute the same bits:
 * persistent -- as many work-groups as the GPU holds at once, each pulling
 * tiles from a device-side queue of its own XCD (the XCD's contiguous
 * eighth of the tile list, so that neighbouring tiles share that XCD's L2)
 * and then from the other XCDs' queues until every tile is done; the queue
 * counters live in the plan and each launch leaves them zeroed for the
 * next, so the graph holds no memset -- or one work-group per tile in the
 * same XCD order.  By default (CHEMORA_DISPATCH_AUTO) plan creation times
 * a stage-2 pass both ways and keeps the faster; chemora_set_plan_dispatch
 * forces one.  Patch p advances with its own time
 * step dt_p = courant * h_p.  Patches are independent (each
 * keeps its own ghosts); no data moves between patches.  Replaying one plan
 * on two streams at once races on its queues. */
typedef struct chemora_plan chemora_plan;   /* opaque, library-owned */

/* How the stage launches of plans are dispatched. */
enum { CHEMORA_DISPATCH_PERSISTENT = 0, CHEMORA_DISPATCH_PER_TILE = 1, CHEMORA_DISPATCH_AUTO = 2 };

/* Sets the dispatch of plans created after this call, process-wide
 * (thread-safe): CHEMORA_DISPATCH_PERSISTENT, CHEMORA_DISPATCH_PER_TILE (one
 * work-group per tile, in the same XCD order) or CHEMORA_DISPATCH_AUTO (the
 * default: each plan times an RK4 stage-2 pass of its patches both ways at
 * creation -- overwriting the S_B and accumulator parts of their scratch
 * before the ghosts are prepared -- and keeps the faster).  Existing plans
 * keep theirs.  EINVAL for another value. */
int chemora_set_plan_dispatch(int32_t mode);

/* Dispatch a plan runs (CHEMORA_DISPATCH_PERSISTENT or _PER_TILE; never
 * AUTO), or EINVAL for a NULL plan. */
int chemora_plan_dispatch(const chemora_plan *plan);

/* Creates a plan.  patches[p].u and scratch[p] (chemora_rk4_scratch_elems
 * doubles) must stay allocated, and scratch must not be modified by the
 * caller, until chemora_plan_destroy.  With static ghosts the stage buffers'
 * ghosts are copied from u once, here, on `stream`.  Validation as for
 * chemora_rk4_step, per patch (EINVAL / EUNSUPPORTED before any HIP call);
 * courant must be finite and > 0; npatch >= 1.  Each patch runs with its
 * class's tile variant (see chemora_tune).  tune_cache_path NULL: the
 * variants chosen so far in this process (else the defaults).  Otherwise the
 * cache file is read if it exists, every class of the plan without an entry
 * is timed on its largest patch (chemora_tune; this synchronises `stream`
 * and overwrites that patch's scratch, before the ghosts are prepared), and the
 * file is rewritten with all entries.  An FP64 plan whose classes then use
 * more than one variant also times an RK4 stage-2 pass over all its patches
 * with that mix (one launch per variant group, one after another) and with
 * each built variant for every patch, and keeps the fastest assignment: the
 * FP64 variants are bit-identical, so only the time changes
 * (chemora_plan_patch_variant reports each patch's).  Device tables and the graph are
 * allocated here (ENOMEM or EDEVICE on failure, nothing leaked). */
int chemora_plan_create(const chemora_params *params, const chemora_patch *patches, double *const *scratch,
                        int32_t npatch, double courant, const char *tune_cache_path, void *stream,
                        chemora_plan **out);

/* The same plan with the third-order SSP Runge-Kutta step of
 * chemora_rk3_step captured instead of RK4 (3 launches per tile-variant
 * group and step).  Arguments, scratch size (chemora_rk4_scratch_elems:
 * the tuner uses all of it) and errors as chemora_plan_create. */
int chemora_plan_create_rk3(const chemora_params *params, const chemora_patch *patches, double *const *scratch,
                            int32_t npatch, double courant, const char *tune_cache_path, void *stream,
                            chemora_plan **out);

/* A synchronised plan: the patches form one grid hierarchy instead of being
 * independent -- the framework services the paper delegates to its driver
 * (section "Cactus-Carpet Computational Infrastructure": ghost-zone
 * synchronisation, mesh refinement, multi-block; section "Conclusion" names
 * them as the next step).  Patches sit on vertex-centred refinement levels
 * h_L = h_0 / 2^L (h_0 the largest spacing); every origin must lie on its
 * level's lattice through the first coarsest patch's origin.  Every patch
 * advances with the same dt (no subcycling) by RK4 (integrator 4) or the
 * SSP RK3 step (integrator 3).  After every stage the ghost points of every
 * stage output are refilled level by level, coarsest first: a ghost point
 * inside the interior of another patch of its level takes that value (the
 * lowest-numbered such patch); else, on a refined level, the order-p
 * Lagrange interpolation (p = fd_order, tensor product, per axis the
 * coincident coarse point or the p coarse points around a midpoint) from
 * the lowest-numbered patch of the next coarser level whose stored box holds
 * every tap; else (coarsest level only) it is an outer-boundary point with
 * the params' boundary treatment (static or radiative; periodic is
 * EUNSUPPORTED).  After the last stage, and once here before the first step,
 * coarse interior points that coincide with a finer level's interior point
 * take its value (finest level first), then the ghosts are refilled.  The
 * point maps are built here on the host; EINVAL if spacings or origins do
 * not form such a hierarchy or a refined patch's ghost point has no source.
 * Otherwise as chemora_plan_create (scratch, tuning, errors); dt must be
 * finite and > 0. */
int chemora_plan_create_synced(const chemora_params *params, const chemora_patch *patches,
                               double *const *scratch, int32_t npatch, double dt, int32_t integrator,
                               const char *tune_cache_path, void *stream, chemora_plan **out);

/* Advances every patch of the plan by nsteps steps of its integrator
 * (nsteps >= 0), by replaying the captured graph on `stream`: per step and
 * RK stage, the right-hand side and stage combination of every patch
 * (chemora_rk4_step's arithmetic, bitwise the same as per-patch calls with
 * the same tile variant).  Asynchronous; EINVAL for a NULL plan or
 * nsteps < 0, EDEVICE if a graph launch fails. */
int chemora_batch_step(chemora_plan *plan, int32_t nsteps, void *stream);

/* Total interior points of the plan's patches (0 for NULL). */
int64_t chemora_plan_points(const chemora_plan *plan);

/* Tile variant the plan runs patch p (0 <= p < npatch) with; EINVAL else. */
int chemora_plan_patch_variant(const chemora_plan *plan, int32_t p);

/* Releases the plan after synchronising the device (hipDeviceSynchronize:
 * its graph may still be running).  NULL is a no-op. */
int chemora_plan_destroy(chemora_plan *plan);

/* Counts NaN/Inf in the interior of all 24 GFs (ghost width from params),
 * waits for `stream` and stores the count in *bad_count (host pointer).
 * Returns CHEMORA_ENOTFINITE when the count is nonzero. */
int chemora_check_finite(const chemora_params *params, const chemora_patch *patch, int64_t *bad_count,
                         void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *chemora_last_error(void);

/* ABI version of this header (major*100 + minor): 103 (1.1 added
 * chemora_rk3_step, chemora_rk3_scratch_elems, chemora_plan_create_rk3,
 * chemora_enforce_constraints and chemora_momentum_constraint; 1.2 added
 * chemora_rk4_step_noalloc, chemora_psi4, chemora_plan_create_synced and
 * CHEMORA_BC_RADIATIVE; 1.3 added chemora_set_plan_dispatch and
 * chemora_plan_dispatch; nothing earlier changed). */
int chemora_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CHEMORA_H */
