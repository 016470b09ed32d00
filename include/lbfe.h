/*
 * lbfe.h -- C ABI of the MI355X (gfx950) D3Q27 free-energy lattice Boltzmann
 * library: the chemical-potential-based free-energy model with generalized
 * (sixth-order Hermite) equilibria and central-moment MRT collision of
 * Saito, Baba & Takada, arXiv:2504.03819.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns an int status: LBFE_OK (0) or a negative LBFE_E_*
 *    code.  No exception, abort or exit crosses this boundary; after an error
 *    lbfe_last_error(ctx) returns a human-readable reason (a string owned by
 *    the context, valid until the next call on it).
 *  - Grids are nx * ny * nz lattice nodes.  Scalar fields are double arrays
 *    laid out [z][y][x] (x fastest); vector fields are [3][z][y][x]; the
 *    population state is [27][z][y][x] with direction index
 *    i = 9 (cx+1) + 3 (cy+1) + (cz+1), rest i = 13, opposite 26 - i.
 *  - With walls_z = 1 the planes z = 0 and z = nz-1 are solid (halfway
 *    bounce-back and the wetting boundary of Sec. III C); every other node is
 *    fluid.  With walls_z = 0 the box is periodic in all three directions,
 *    and with solid_mask = 1 the solid nodes are those of a voxel mask
 *    (lbfe_set_solid) in that periodic box.
 *  - Pointers named *_dev are device pointers (HIP device memory on the
 *    context's device); all others are host pointers.  Every buffer is owned
 *    by the caller; the library never allocates or frees device memory: it
 *    works inside one caller-provided workspace (lbfe_bind_workspace).
 *  - All device work is enqueued on the HIP stream given to lbfe_create and
 *    is asynchronous unless a call says it synchronises.  One context per
 *    stream; calls on one context are not thread-safe.
 */
#ifndef LBFE_H
#define LBFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define LBFE_OK 0
#define LBFE_E_INVAL (-1)    /* invalid argument or parameter              */
#define LBFE_E_NOMEM (-2)    /* workspace missing or smaller than required */
#define LBFE_E_DEVICE (-3)   /* no usable GPU, or a HIP runtime error      */
#define LBFE_E_DIVERGED (-4) /* NaN/Inf, or density left the EOS domain    */
#define LBFE_E_STATE (-5)    /* call out of order (e.g. step before init)  */

/* ---- storage / arithmetic forms -------------------------------------- */
/* LBFE_FP64        populations stored and collided in double.
 * LBFE_FP32        populations stored in float, collision and forcing in
 *                  float; density sums, mu, grad mu and reductions in double.
 * LBFE_FP16_DEV    populations stored as half-precision deviations from the
 *                  rest-state weights, (f_i - w_i) / w_i; arithmetic as FP32.
 * LBFE_FP16_DEV_F0FP32  as FP16_DEV but the rest population is kept in float. */
#define LBFE_FP64 0
#define LBFE_FP32 1
#define LBFE_FP16_DEV 2
#define LBFE_FP16_DEV_F0FP32 3

/* ---- wetting modes, Eq. (38) ------------------------------------------ */
#define LBFE_WET_NEUTRAL 0 /* rho(x_s) = rho_ave(x_s)                      */
#define LBFE_WET_PHI 1     /* rho(x_s) = phi * rho_ave   (theta <= 90 deg) */
#define LBFE_WET_DELTA 2   /* rho(x_s) = rho_ave - drho  (theta >  90 deg) */

/* ---- field selectors for lbfe_field ------------------------------------ */
#define LBFE_FIELD_RHO 0 /* density, Eq. (11); solid nodes: Eqs. (37)-(38) */
#define LBFE_FIELD_U 1   /* velocity (3 comps), Eq. (11) incl. F/2; solid 0 */
#define LBFE_FIELD_MU 2  /* chemical potential, Eq. (32); solid: Eq. (36)  */
#define LBFE_FIELD_F 3   /* force (3 comps), Eq. (12); solid 0              */
#define LBFE_FIELD_Q 4   /* Q200, Q020, Q002 (3 comps), Eq. (27); solid 0   */
#define LBFE_FIELD_PM 5  /* modified pressure p_m = (1 + mu)/3, Eq. (12)    */

/* Parameters of one simulation (Sec. II B and Sec. III). */
typedef struct lbfe_params {
    int64_t nx, ny, nz;  /* lattice size, each >= 1 (nz >= 3 with walls),
                            nx*ny*nz < 2^31, nx*ny <= 2^28                */
    int32_t walls_z;     /* 0 periodic; 1 solid planes z = 0 and z = nz-1  */
    int32_t precision;   /* LBFE_FP64 / FP32 / FP16_DEV / FP16_DEV_F0FP32  */
    double a, b, R, T;   /* van der Waals EOS, Eqs. (29)-(32)              */
    double kappa;        /* interfacial coefficient kappa, Eq. (1)         */
    double nu;           /* kinematic viscosity; 1/omega_1 = rho nu/p_m+1/2 */
    double omega[11];    /* relaxation rates omega_0..omega_10, in [0, 2];
                            omega[1] is ignored (derived per node from nu) */
    int32_t corr4;       /* 1: fourth-order correction Eq. (28), 0: off    */
    int32_t wet_mode;    /* LBFE_WET_*                                     */
    double wet_value;    /* phi (> 0) or drho (>= 0) of Eq. (38)           */
    double rho_l, rho_v; /* coexistence pair for the wetting window; both 0
                            means: computed by lbfe_create (Maxwell at T) */
    int32_t check_every; /* lbfe_step checks the divergence flag every this
                            many steps (>= 1) and at the end               */
    int32_t adjoint;     /* 1: the workspace also holds adjoint buffers    */
    double wall_u[4];    /* tangential velocities (ux, uy) of the bottom
                            (z = 0) and top (z = nz-1) walls, moving-wall
                            test of Sec. III B: momentum-corrected halfway
                            bounce-back; |u| <= 0.3; nonzero needs
                            walls_z = 1; 0 = resting walls */
    int32_t solid_mask;  /* 1: the solid nodes come from a voxel mask given
                            by lbfe_set_solid (needs walls_z = 0 and resting
                            walls); 0: none or the wall planes */
    /* Schedule.  None of these changes a result bit; 0 lets lbfe_create
     * choose per grid, and lbfe_get_params reports the choice made. */
    int32_t step_path;   /* LBFE_PATH_*: how one step is split into kernels */
    int32_t tile_order;  /* LBFE_ORDER_*: how tiles are dealt to the XCDs   */
    int32_t chain_chunk; /* z-planes per workgroup of the stencil chain,
                            1..64                                          */
} lbfe_params;

/* ---- schedule choices (lbfe_params.step_path, .tile_order) ------------- */
/* LBFE_PATH_TWO_PASS  a moments pass over the stored populations, the
 *                     stencil chain, then collide + stream: the populations
 *                     are read twice per step.
 * LBFE_PATH_FUSED     the stencil chain, then one kernel that collides,
 *                     streams and forms the next step's density and momentum
 *                     (Eq. (11)): the populations are read once per step.
 *                     Not with a solid mask, and only when one z-plane of
 *                     the lattice is below 2 GiB (moving walls: the wall
 *                     term and the moments of the two wall-adjacent planes
 *                     are applied by a small pass after the kernel).
 * LBFE_PATH_STATE     the moment-representation state of the paper's rate
 *                     setting, every omega_k but omega_1 equal to 1 (Sec. II
 *                     B, stated after Eq. (26)): between the steps of one
 *                     lbfe_step call each node holds 16 post-collision
 *                     numbers instead of 27 populations; per step the
 *                     stencil chain, a collide pass and a moments pass each
 *                     rebuild the populations from those numbers.  The
 *                     first step of a call enters the state form from the
 *                     populations, the last leaves it, so between calls the
 *                     context holds populations as on the other paths.
 *                     FP64 and FP32 only, resting walls, no solid mask, and
 *                     a lattice z-plane below 2 GiB; lbfe_create rejects it
 *                     with LBFE_E_INVAL otherwise (other rates included).
 * LBFE_ORDER_ROUND_ROBIN  workgroups in launch order (the hardware deals them
 *                     to the 8 XCDs in turn).
 * LBFE_ORDER_XCD      each XCD takes one contiguous range of tiles, so
 *                     neighbouring tiles share that XCD's L2. */
#define LBFE_AUTO 0
#define LBFE_PATH_TWO_PASS 1
#define LBFE_PATH_FUSED 2
#define LBFE_PATH_STATE 3
#define LBFE_ORDER_ROUND_ROBIN 1
#define LBFE_ORDER_XCD 2

typedef struct lbfe_ctx lbfe_ctx;

/* Fill *p with the paper's defaults (Sec. III): a = 9/392, b = 2/21, R = 1,
 * T = 0.7 T_c, kappa = 0.02, nu = 0.15, all omega_k = 1, corr4 on,
 * periodic 32^3, neutral wetting, resting walls, FP64, check_every = 100,
 * adjoint off, schedule LBFE_AUTO. */
int lbfe_params_default(lbfe_params *p);

/* Coexistence pair of the vdW EOS at temperature T from equal chemical
 * potential and equal pressure (Maxwell's rule, Sec. III).  Host only.
 * E_INVAL if T is not strictly between 0.3 T_c and T_c. */
int lbfe_coexistence(double a, double b, double R, double T, double *rho_l, double *rho_v);

/* Validate *p, derive constants (coexistence pair if not given, wetting
 * window 0.05 rl + 0.95 rv .. 0.95 rl + 0.05 rv) and create a context bound
 * to the current HIP device and the given stream (hipStream_t as void*;
 * NULL = default stream).  Allocates no device memory.
 * E_INVAL on a bad parameter (checked before any device call), E_DEVICE
 * when no GPU is usable.  Schedule fields left at LBFE_AUTO are chosen per
 * grid: the fused step path for FP64 contexts of at least 2^24 nodes where
 * it is allowed, else the two-pass path; the XCD tile order from
 * 2^26 nodes and, without a solid mask, whenever nx or ny is not a power of
 * two; the chain chunk that minimises the busiest CU's plane iterations.
 * Asking for the fused path where it is not allowed is E_INVAL. */
int lbfe_create(const lbfe_params *p, void *hip_stream, lbfe_ctx **out);

/* Bytes of device workspace a context with these parameters needs. */
int lbfe_workspace_bytes(const lbfe_params *p, size_t *bytes);

/* Bind caller-owned device memory (256-byte aligned, >= the size from
 * lbfe_workspace_bytes) as the context's workspace.  The memory must outlive
 * the context; the library never frees it.  E_NOMEM if too small. */
int lbfe_bind_workspace(lbfe_ctx *ctx, void *workspace_dev, size_t bytes);

/* Copy the context's parameters, with derived rho_l/rho_v and the schedule
 * actually chosen (no LBFE_AUTO left), into *out. */
int lbfe_get_params(const lbfe_ctx *ctx, lbfe_params *out);

/* Solid voxel mask (params.solid_mask = 1): the halfway bounce-back of
 * Eq. (10) and the wetting boundary of Eqs. (36)-(38) at every solid node
 * x_s, which Sec. III C writes for a general x_s (curved or patterned
 * substrates; flat walls are the mask of the planes z = 0 and z = nz-1).
 * mask_dev: device uint8[nz][ny][nx], nonzero = solid, read during the call
 * (the library keeps its own per-node neighbour words; the caller may free
 * the mask afterwards).  Periodic wrap at the box faces.  Solid nodes hold
 * no populations; their rho is the wetting density (0 if no fluid
 * neighbour), their u, F, Q are 0.  Discards the state: call
 * lbfe_init_density (or lbfe_set_state / lbfe_set_populations) after it.
 * E_STATE if the context was created with solid_mask = 0 or has no
 * workspace; E_INVAL for a null mask. */
int lbfe_set_solid(lbfe_ctx *ctx, const uint8_t *mask_dev);

/* Initial state (Sec. III B, Eqs. (34)-(35) give the paper's droplets):
 * populations at the generalized equilibrium of Eq. (20) with density rho0,
 * velocity u0 (NULL = 0) and p_m from mu[rho0] (solid-node densities from
 * Eqs. (37)-(38) first).  rho0_dev: double[nz][ny][nx], entries at solid
 * nodes are ignored; u0_dev: double[3][nz][ny][nx] or NULL.  Synchronises
 * once to validate: E_INVAL if a fluid density is not finite or outside the
 * EOS domain 0 < rho < 1/b.  Resets the step counter to 0. */
int lbfe_init_density(lbfe_ctx *ctx, const double *rho0_dev, const double *u0_dev);

/* Advance nsteps time steps (Sec. II B): density and momentum, wall density
 * Eqs. (37)-(38), chemical potential Eq. (32) with Eq. (36) at walls, force
 * Eq. (12), Q corrections Eqs. (27)-(28), central-moment collision
 * Eqs. (21)-(26), inverse transform and streaming Eq. (10) with halfway
 * bounce-back.  Checks the divergence flag every check_every steps and at
 * the end (a synchronisation): E_DIVERGED, with the step in lbfe_last_error.
 * Each step runs as params.step_path says: a moments pass, the stencil
 * chain and a collide-stream pass (LBFE_PATH_TWO_PASS), or the stencil
 * chain and a collide-stream kernel that also forms the next step's density
 * and momentum (LBFE_PATH_FUSED, no moments pass), or through the moment
 * state (LBFE_PATH_STATE); all give bitwise identical states. */
int lbfe_step(lbfe_ctx *ctx, int64_t nsteps);

/* Timing variant of lbfe_step for benchmarks: the same launches, with HIP
 * events recorded on the context's stream around every kernel class;
 * kernel_ms[k] receives the summed milliseconds of class k over the nsteps
 * steps: 0 moments pass (with the wall density after it; on the fused path
 * only after the state was set from outside), 1 stencil chain (mu, force,
 * Q), 2 collide-stream (fused path: with the next step's moments), 3 wall
 * density after the step (fused path, walls only).  On the state path:
 * 0 the moments passes (with the populations at the end and the wall
 * density), 1 the chains, 2 the collide passes (the first from the
 * populations), 3 zero.  Synchronises after every step (host array). */
int lbfe_step_timed(lbfe_ctx *ctx, int64_t nsteps, double kernel_ms[4]);

/* Number of steps taken since lbfe_init_density / lbfe_set_state. */
int lbfe_step_count(const lbfe_ctx *ctx, int64_t *step);

/* Macroscopic fields of the current state f(t) (the quantities the next
 * step would use).  Each pointer may be NULL; rho_dev, mu_dev:
 * double[nz][ny][nx]; u_dev, F_dev: double[3][nz][ny][nx]. */
int lbfe_fields(lbfe_ctx *ctx, double *rho_dev, double *u_dev, double *mu_dev, double *F_dev);

/* One field of the current state by selector LBFE_FIELD_*; out_dev holds
 * 1 or 3 (U, F, Q) double planes of nz*ny*nx. */
int lbfe_field(lbfe_ctx *ctx, int which, double *out_dev);

/* Size in bytes of the raw population state at storage precision. */
int lbfe_state_bytes(const lbfe_ctx *ctx, size_t *bytes);
/* Raw state copy out / in (checkpoints).  set_state also sets the counter. */
int lbfe_get_state(lbfe_ctx *ctx, void *dst_dev);
int lbfe_set_state(lbfe_ctx *ctx, const void *src_dev, int64_t step);

/* Populations decoded to / encoded from double[27][nz][ny][nx] (solid-node
 * entries read as 0 and are ignored on input). */
int lbfe_get_populations(lbfe_ctx *ctx, double *f_dev);
int lbfe_set_populations(lbfe_ctx *ctx, const double *f_dev);

/* Deterministic FP64 reductions over fluid nodes of the current state:
 * out[0] = sum rho, out[1..3] = sum j (= sum_i f_i c_i), out[4..6] = sum F,
 * out[7] = max |u|.  Host array; synchronises. */
int lbfe_reduce(lbfe_ctx *ctx, double out[8]);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): lbfe_reduce with the result written asynchronously on the
 * context's stream to out_dev (8 doubles, caller-owned device memory, same
 * order), no host synchronisation, and the block partials in a static
 * device scratch of 4 MiB that each GPU the library runs on holds until the
 * process ends, instead of the workspace; it allocates nothing and calls no
 * allocating routine.  The same kernels and summation order as lbfe_reduce,
 * so the results are bit for bit the same.  Serves contexts of up to 2^24
 * fluid nodes (E_INVAL beyond, checked first).  All calls on one GPU share
 * its scratch: calls that overlap on one GPU (different streams or host
 * threads) race. */
int lbfe_reduce_into(lbfe_ctx *ctx, double *out_dev);

/* ---- discrete adjoint (needs params.adjoint = 1) ----------------------- *
 * Not part of the paper's method: the exact reverse-mode derivative of the
 * discrete step above (the map f(t) -> f(t+1) of Sec. II B with the wall
 * treatment of Eqs. (36)-(38)), taking the active branch of the wetting
 * window and limiter.  The adjoint state lambda(t) = dL/df(t) lives in the
 * workspace.  Reverse sweep: lbfe_adjoint_seed at the final time T, then for
 * t = T-1 .. 0 lbfe_adjoint_step with the forward state f(t) (raw state as
 * from lbfe_get_state, e.g. recomputed from a checkpoint), then
 * lbfe_adjoint_init_density for dL/drho0.  lbfe_adjoint_grads returns the
 * accumulated parameter gradients.  All of it is deterministic. */

/* lambda(T)_i(x) = dL/drho(x) at every fluid node and for every i (rho is
 * sum_i f_i); entries at solid nodes are ignored.  Resets the parameter
 * gradient accumulators.  dL_drho_dev: double[nz][ny][nx]. */
int lbfe_adjoint_seed(lbfe_ctx *ctx, const double *dL_drho_dev);

/* General seed: lambda(T) = dL/df(T) given as double[27][nz][ny][nx]
 * (direction-major like lbfe_get_populations; solid entries ignored).
 * Resets the parameter-gradient accumulators. */
int lbfe_adjoint_seed_populations(lbfe_ctx *ctx, const double *dL_df_dev);

/* Current adjoint state lambda(t) decoded to double[27][nz][ny][nx]
 * (zero at solid nodes). */
int lbfe_adjoint_get(lbfe_ctx *ctx, double *lambda_dev);

/* lambda(t) = (d step / d f(t))^T lambda(t+1), accumulating dL/dkappa,
 * dL/d(wet_value) and dL/dnu.  state_t_dev: f(t) at storage precision, or
 * NULL for the context's current state (e.g. f(t) just recomputed with
 * lbfe_step, which saves copying it out; E_STATE if there is none).  The
 * state is only read.  Overwrites the auxiliary fields of the context. */
int lbfe_adjoint_step(lbfe_ctx *ctx, const void *state_t_dev);

/* Forward auxiliary fields kept for the adjoint.  A checkpointed reverse
 * sweep recomputes f(t) with forward steps; each such step evaluates the
 * fields of its input state (rho with the wall densities, mu, j, F, Q, steps
 * S1-S5 of Sec. II B), which lbfe_adjoint_step would otherwise evaluate
 * again.  lbfe_aux_bytes: size of one record (depends only on the grid and
 * the storage form).  lbfe_step_aux: one step f(t) -> f(t+1) (unfused) that
 * leaves the fields of f(t) in aux_dev instead of the workspace; same
 * result as lbfe_step(ctx, 1), bit for bit, without the divergence check.
 * lbfe_adjoint_step_aux: lbfe_adjoint_step with the record of f(t) from
 * lbfe_step_aux; bit for bit the same lambda(t) and gradients, without the
 * recomputation.  aux_dev: caller-owned device memory of lbfe_aux_bytes,
 * 256-byte aligned (E_INVAL otherwise); it must be the record of exactly
 * state_t_dev. */
int lbfe_aux_bytes(const lbfe_ctx *ctx, size_t *bytes);
int lbfe_step_aux(lbfe_ctx *ctx, void *aux_dev);
int lbfe_adjoint_step_aux(lbfe_ctx *ctx, const void *state_t_dev, const void *aux_dev);

/* Pull lambda(0) back through the initialiser of lbfe_init_density given
 * the same rho0_dev and u0_dev (NULL = 0): dL/drho0 into dL_drho0_dev
 * (double[nz][ny][nx], zero at solid nodes); adds the initialiser's kappa and
 * wetting-value contributions to the accumulators. */
int lbfe_adjoint_init_density(lbfe_ctx *ctx, const double *rho0_dev, const double *u0_dev, double *dL_drho0_dev);

/* out[0] = dL/dkappa, out[1] = dL/d(wet_value), out[2] = dL/dnu,
 * out[3] = 0 (reserved).  Host array; synchronises. */
int lbfe_adjoint_grads(lbfe_ctx *ctx, double out[4]);

/* Reason for the last error on this context (never NULL). */
const char *lbfe_last_error(const lbfe_ctx *ctx);

/* Release the context (not the caller's workspace).  NULL is a no-op. */
int lbfe_destroy(lbfe_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBFE_H */
