/*
 * lbm.h - C ABI of the MI355X (gfx950) D2Q9 BGK solver for unconfined flow
 * past a circular cylinder, after Sahiti, Gurugubelli & Surasani, "Lattice
 * Boltzmann methodology for unconfined flows" (arXiv 2605.02185).
 *
 * Conventions (all entry points):
 *  - Lattice units throughout: dx = dt = 1, c = 1, c_s^2 = 1/3 (Sec. 2.1).
 *  - Directions k = 0..8 are the paper's Table 1 index minus one:
 *      k : 0  1  2  3  4  5  6  7  8     (rest, E, N, W, S, NE, NW, SW, SE)
 *      cx: 0  1  0 -1  0  1 -1 -1  1
 *      cy: 0  0  1  0 -1  1  1 -1 -1
 *  - Node (x, y) with x in [0, nx) along the flow, y in [0, ny) across it.
 *    Column x = 0 is the velocity inlet, x = nx-1 the outlet, rows y = 0 and
 *    y = ny-1 the bottom and top walls (wet-node placement, Sec. 2.4).
 *  - Field arrays are row-major [ny][nx]; population arrays are [9][ny][nx].
 *  - The library owns every device allocation it makes and frees it in the
 *    matching destroy call.  Pointers passed in are owned by the caller and
 *    are not retained after the call returns.
 *  - Device pointers are HIP device addresses on the device that was current
 *    when the context was created.  `stream` arguments are hipStream_t
 *    values passed as void*; NULL is the null stream.
 *  - Every function returns LBM_OK (0) or a negative lbm_status; the message
 *    of the last failure on the calling thread is lbm_last_error().  Nothing
 *    throws or exits across the ABI.
 *  - One context is used by one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARG = -1, /* a parameter or argument is out of its documented range */
  LBM_ERR_HIP = -2,         /* a HIP runtime call failed (message names it) */
  LBM_ERR_OOM = -3,         /* device allocation failed */
  LBM_ERR_DIVERGED = -4,    /* a fluid density became non-finite or left (0, 10) */
  LBM_ERR_RANGE = -5,       /* requested force steps are not (or no longer) stored */
  LBM_ERR_STATE = -6        /* call not valid in the context's current state */
} lbm_status;

/* Top/bottom treatments of Sec. 2.3 (the four the paper compares). */
typedef enum {
  LBM_WALL_FREE_SLIP = 0, /* Eq. 7: specular reflection of the missing populations */
  LBM_WALL_PERIODIC = 1,  /* Eq. 8, realised as wrap-around streaming in y */
  LBM_WALL_NEBB = 2,      /* Eqs. 9-10: Zou-He wet-node wall moving at (U_w, 0) */
  LBM_WALL_MOVING_BB = 3  /* Eq. 11: bounce-back of a wall moving at (U_w, 0) */
} lbm_wall;

/* Outlet of Eq. 13 (zeroth-order extrapolation from column nx-2). */
typedef enum {
  LBM_OUTLET_COPY_ALL = 0,    /* all nine populations (Eq. 13 as printed) */
  LBM_OUTLET_COPY_UNKNOWN = 1 /* only the populations no streaming fills: W, NW, SW, and at the two
                               * outlet corners also those from beyond the wall row (N, NE at the
                               * bottom, S, SE at the top) */
} lbm_outlet;

/* Cylinder wall treatment (Sec. 2.4). */
typedef enum {
  LBM_BOUNCE_HALFWAY = 0, /* half-way bounce-back on the staircase disk (the paper's choice) */
  LBM_BOUNCE_INTERP = 1,  /* link-wise interpolated bounce-back (Bouzidi, Firdaouss & Lallemand)
                           * with the wall fraction q of each link from the circle */
  LBM_BOUNCE_FULLWAY = 2  /* full-way bounce-back (Sec. 3.1): solid nodes stream like fluid ones
                           * and their collision reverses every population, so what reaches the
                           * wall returns to its fluid node one step later; solid nodes start at
                           * rest (f = w) and the momentum of each link is booked in the step
                           * its population enters the wall */
} lbm_bounce;

/* Collision operator. */
typedef enum {
  LBM_COLLISION_BGK = 0, /* single relaxation time 1/tau (Eq. 2) */
  LBM_COLLISION_MRT = 1  /* multiple relaxation times in moment space (Eq. 6, Sec. 2.1) */
} lbm_collision;

typedef struct {
  int32_t struct_size;   /* sizeof(lbm_params); set by lbm_params_init */
  int32_t nx, ny;        /* lattice size, both >= 3 */
  int32_t diameter;      /* cylinder diameter D in lattice units; 0 = no cylinder */
  int32_t cx2, cy2;      /* cylinder centre in doubled coordinates (2 x_c, 2 y_c) */
  double u_in;           /* inlet velocity U, 0 <= U < 1/sqrt(3) */
  double re;             /* Reynolds number, used when tau <= 0 */
  double tau;            /* BGK relaxation time; <= 0 derives it by Eqs. 16-17 */
  int32_t wall;          /* lbm_wall for both the top and the bottom row */
  int32_t outlet_mode;   /* lbm_outlet */
  double u_wall_top;     /* wall tangential velocity (NEBB, moving BB); NaN = u_in */
  double u_wall_bottom;  /* same for the bottom row; NaN = u_in */
  int32_t x_periodic;    /* 1: periodic in x, no inlet/outlet (test boxes) */
  int32_t collision;     /* lbm_collision */
  double perturb_amp;    /* initial v = amp * U * sin(2 pi y/(ny-1)) */
  int64_t hist_capacity; /* force steps kept on the device (ring buffer) */
  /* MRT only: diag(S) of Eq. 6 over the moments (rho, e, epsilon, j_x, q_x,
   * j_y, q_y, p_xx, p_xy).  Entries 0, 3 and 5 belong to conserved moments
   * and have no effect; entries 7 and 8 (the shear rates) <= 0 mean 1/tau,
   * so that tau sets the viscosity through Eq. 5 as for BGK. */
  double s_rates[9];
  int32_t bounce;        /* lbm_bounce */
  int32_t reserved1;
} lbm_params;

/* Defaults: D = 0, centre 21*D doubled (10.5 D), U = 0.1, Re = 100, tau
 * derived, free-slip walls, copy-all outlet, BGK, the rates of Sec. 2.1
 * (1, 1.1, 1.1, 1, 1.1, 1, 1.1, 1/tau, 1/tau) for MRT, perturbation 1e-3,
 * history of 1<<20 steps.  nx and ny are set to 0 and must be filled in. */
void lbm_params_init(lbm_params* p);

/* Host-only check of a parameter set (no GPU needed).  Rejects nx or ny < 3,
 * tau <= 1/2, U outside [0, 1/sqrt(3)), an unknown wall, outlet or collision
 * mode, an MRT rate of a non-conserved moment outside (0, 2), an unknown
 * bounce-back mode, a
 * cylinder with a solid node outside [3, nx-4] x [3, ny-4] (so that two fluid
 * nodes separate it from every edge row and column), and hist_capacity < 1. */
lbm_status lbm_validate_params(const lbm_params* p);

/* tau actually used: p->tau if > 0, else 3 U D / Re + 1/2 (Eqs. 16-17). */
double lbm_params_tau(const lbm_params* p);

/* Host-only geometry of the staircase disk (Sec. 2.5, Fig. 4): node (x, y)
 * is solid iff (2x - cx2)^2 + (2y - cy2)^2 <= D^2.  Outputs may be NULL:
 * solid_mask [ny][nx] 0/1, the number of solid nodes, of fluid nodes with a
 * solid neighbour, and of fluid-to-solid links over all 8 directions. */
lbm_status lbm_geometry(const lbm_params* p, uint8_t* solid_mask, int64_t* n_solid,
                        int64_t* n_boundary_nodes, int64_t* n_links);

typedef struct lbm_ctx lbm_ctx;

/* Validate p, allocate the device state on the current device and initialise
 * it to the equilibrium of rho = 1, u = (U, amp U sin(2 pi y/(ny-1))) (Eq. 3).
 * All later work of the context is ordered on `stream`. */
lbm_status lbm_create(const lbm_params* p, void* stream, lbm_ctx** out);

/* Release every device allocation of the context (synchronises its stream). */
void lbm_destroy(lbm_ctx* ctx);

/* Advance n >= 0 time steps.  One step is, per node, the pull of the
 * post-collision populations of the neighbours (streaming, Eq. 2),
 * bounce-back at the cylinder (half-way or full-way, Sec. 3.1, or
 * interpolated, Sec. 2.4), the boundary corrections of
 * Sec. 2.3 and the inlet, then the collision (BGK, Eqs. 2-4, or MRT, Eq. 6); the force on the
 * cylinder is taken by momentum exchange (Eq. 14) in the same pass.
 * Stream-ordered and asynchronous; a divergence is reported by the next
 * lbm_sync / lbm_forces / lbm_fields / lbm_get_populations call. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Wait for the context's stream; LBM_ERR_DIVERGED if a step went bad. */
lbm_status lbm_sync(lbm_ctx* ctx);

/* Steps completed so far. */
lbm_status lbm_get_step(lbm_ctx* ctx, int64_t* step);

/* First step that diverged (1-based), or 0 if none (synchronises). */
lbm_status lbm_diverged_step(lbm_ctx* ctx, int64_t* step);

/* Force on the cylinder by momentum exchange (Eq. 14), accumulated in FP64,
 * and its coefficients (Eq. 15 with rho_in = 1 and the nominal D).  Step k
 * (1-based) is the force exchanged while streaming from time k-1 to k.
 * Copies steps [first, first+count) into the host arrays fx, fy, cd, cl (any
 * may be NULL).  LBM_ERR_RANGE if a step was not yet run or has left the
 * ring of hist_capacity steps.  cd/cl need D > 0 and U > 0. */
lbm_status lbm_forces(lbm_ctx* ctx, int64_t first, int64_t count, double* fx, double* fy,
                      double* cd, double* cl);

/* Density and velocity (Eq. 4) of the current state into caller arrays
 * [ny][nx] (host memory if on_device == 0, device memory otherwise).  Solid
 * nodes report rho = 1, u = 0.  Any pointer may be NULL. */
lbm_status lbm_fields(lbm_ctx* ctx, float* rho, float* ux, float* uy, int on_device);

/* State exchange, layout [9][ny][nx].  The state between steps is the set of
 * post-collision populations f*(x, t) (what streams next).  The device holds
 * them in FP32 as deviations f*_k - w_k from the rest equilibrium; these
 * calls exchange the unshifted f*_k.  dtype 0 = float32 (rounded once),
 * 1 = float64 (holds the stored state exactly, so a float64 get/set round
 * trip restores the state bit for bit).  Setting the state keeps the step
 * counter and force history; the next step streams the given populations. */
lbm_status lbm_get_populations(lbm_ctx* ctx, void* buf, int dtype, int on_device);
lbm_status lbm_set_populations(lbm_ctx* ctx, const void* buf, int dtype, int on_device);

/* Shedding statistics of a coefficient history (host-only): periods from the
 * upward crossings of cl through its mean (linear interpolation between
 * steps), St = D/(T U) with T the mean period over the last `periods`
 * periods, cl amplitude = (max-min)/2 and mean cd over those periods.
 * LBM_ERR_RANGE if fewer than periods+1 crossings exist. */
typedef struct {
  double mean_cd, cl_amp, st, period;
} lbm_shedding;
lbm_status lbm_shedding_stats(const double* cd, const double* cl, int64_t n, double d, double u,
                              int32_t periods, lbm_shedding* out);

/* Kernel selection for measurement and autotuning.  Valid variants are
 * 1..lbm_num_variants(); variant 0 selects the context's default.  The result
 * is bit-identical for every variant.  Variants named "tS_*" (S = 2, 3, 4)
 * advance S time steps per launch and keep the intermediate populations in
 * registers, so one launch reads and writes each population once for S node
 * updates; the steps left over (a remainder of n, or steps between learned-
 * closure evaluations that do not fill a launch) run the one-step kernel.
 * The default of a new context is "t4_h10u_s10" from 2^21 nodes,
 * "t3_h16u_s2"
 * from 2^20, "t2_h8_u1" from 2^18 and the one-step "v1_ty1_xcd" (cached
 * stores, each XCD on its own band of rows) below ("_hH": interior segments
 * of H rows, "_hHu": whose output rows are stored as they are made; "_sN":
 * segments that need the boundary code run in pieces of N rows; "_uN":
 * pieces of N rows that load all their rows before any update).
 * lbm_get_variant reports the variant in use. */
int32_t lbm_num_variants(void);
lbm_status lbm_set_variant(lbm_ctx* ctx, int32_t variant);
int32_t lbm_get_variant(const lbm_ctx* ctx);
const char* lbm_variant_name(int32_t variant);

/* Step scheduling.  With graphs enabled (the default) lbm_step replays HIP
 * graphs that each hold 96 steps plus the force-history reduction, captured
 * once per context on an internal stream and launched on the context's
 * stream; the remainder of n runs as plain launches.  Results are identical
 * bit for bit either way. */
lbm_status lbm_set_graphs(lbm_ctx* ctx, int enable);

/* Measurement utility: copies nbytes (a multiple of 16) from src to dst, both
 * device buffers, with a plain streaming kernel (16 B per thread, one
 * launch), ordered on `stream`.  Its duration gives the achievable
 * copy bandwidth that the step kernel's HBM traffic is compared with. */
lbm_status lbm_copy_probe(void* dst, const void* src, int64_t nbytes, void* stream);

/* Autotuner: times every kernel variant for `steps` steps on a scratch copy
 * of the context's lattice (the context's own state is not touched), selects
 * the fastest for the context and returns it in *best (may be NULL).
 * `cache_path` (may be NULL) names a text file of "key variant" lines; a hit
 * skips the timing, a miss appends the result. */
lbm_status lbm_autotune(lbm_ctx* ctx, int32_t steps, const char* cache_path, int32_t* best);

/* ------------------------------------------------------------------ ensemble
 * An ensemble advances many independent lattices (e.g. cylinder channels of
 * different D, Re and size) together: every launch (of one step, or of three
 * or four with a multi-step variant) covers a flattened list of the tiles or
 * wave tasks of all active cases, and 96-step chunks are replayed as HIP
 * graphs.  Each case evolves bit for bit as it would in its own context.
 * Cases are identified by their index in the `cases` array. */
typedef struct lbm_batch lbm_batch;

/* `cases[n]` as for lbm_create; `budgets` (may be NULL = unlimited) gives the
 * number of steps after which each case stops (retires) while the others go
 * on.  The kernel variant (tile shape, nodes per lane, steps per launch) is
 * chosen by the autotuner: every variant lbm_batch_set_variant accepts is
 * timed over 48 steps on a scratch ensemble of the same cases (allocated and
 * freed inside this call) and the fastest is kept; lbm_batch_variant reports
 * it.  `tune_cache` (may be NULL) names a text file of "key variant" lines:
 * a hit skips the timing, a miss appends the choice. */
lbm_status lbm_batch_create(const lbm_params* cases, const int64_t* budgets, int32_t n, void* stream,
                            const char* tune_cache, lbm_batch** out);
void lbm_batch_destroy(lbm_batch* b);

/* Advance every case still within its budget by up to n steps. */
lbm_status lbm_batch_step(lbm_batch* b, int64_t n);

/* Wait for the stream; LBM_ERR_DIVERGED if any case diverged (which ones:
 * lbm_batch_case_info). */
lbm_status lbm_batch_sync(lbm_batch* b);

/* Steps taken and first diverged step (0 = none) of case `c` (synchronises). */
lbm_status lbm_batch_case_info(lbm_batch* b, int32_t c, int64_t* steps, int64_t* diverged_step);

/* As lbm_forces / lbm_fields / lbm_get_populations, for case `c`.  A case's
 * divergence does not make these fail for the other cases. */
lbm_status lbm_batch_forces(lbm_batch* b, int32_t c, int64_t first, int64_t count, double* fx, double* fy,
                            double* cd, double* cl);
lbm_status lbm_batch_fields(lbm_batch* b, int32_t c, float* rho, float* ux, float* uy, int on_device);
lbm_status lbm_batch_get_populations(lbm_batch* b, int32_t c, void* buf, int dtype, int on_device);

/* As lbm_set_populations, for case `c`: the case's next step streams the
 * given post-collision populations ([9][ny][nx] of that case, float32 or
 * float64 as dtype, host or device memory).  Its step counter and force
 * history are kept; the other cases are untouched. */
lbm_status lbm_batch_set_populations(lbm_batch* b, int32_t c, const void* buf, int dtype, int on_device);

/* Kernel variant in use (1-based, as lbm_variant_name). */
int32_t lbm_batch_variant(const lbm_batch* b);

/* Select the ensemble's kernel variant (synchronises the ensemble's stream;
 * also done by the autotuner).  Allowed: the one-step variants without a
 * remapped block order, and the multi-step variants "t3_h8_s2", "t3_h8_s4",
 * "t4_h8_s2", "t4_h8_s4", "t4_h8_s8", "t4_h16u_s8", "t4_h10u_s10" and
 * "t3_h16u_s2", which
 * advance every active case by
 * their 3 or 4 steps per launch (the steps a case has left before the active
 * set changes, when fewer, run one per launch on "v1_ty1_nt").  Every
 * variant gives each case the same bits as running it alone.  Returns
 * LBM_ERR_INVALID_ARG for any other variant. */
lbm_status lbm_batch_set_variant(lbm_batch* b, int32_t variant);

/* ------------------------------------------------------ learned closure
 * A small network (36 -> 64 -> 64 -> 3, exact-erf GELU after both hidden
 * layers) that predicts, on the open top, bottom and outlet boundaries of a
 * truncated domain, the populations streaming in from outside as a residual
 * on top of the plain treatment (free-slip walls, Eq. 7; extrapolated
 * missing populations at the outlet, Eq. 13).  The paper has no such part:
 * it truncates the domain far from the body (Sec. 1) and this closure aims
 * to let a much smaller window reproduce the full domain's forces.
 *
 * Boundary nodes of an nx x ny lattice are numbered 0 .. nb-1 with
 * nb = 2(nx-2) + (ny-2): the top row (y = ny-1, x = 1..nx-2), the bottom row
 * (y = 0, x = 1..nx-2), then the outlet column (x = nx-1, y = 1..ny-2).
 * Features of a node (36): for the node and its two inward neighbours along
 * the boundary normal, the nine stored deviations f*_k - w_k, rho - 1 and
 * the two velocity components, all in a frame turned so that the outward
 * normal is +y (bottom mirrored, outlet rotated a quarter turn).  Outputs
 * (3): the residuals of the canonical S, SW and SE populations.
 *
 * Weights are a flat FP32 vector of LBM_MLP_PARAMS values, W row-major
 * (input x output): W1[36][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3].
 * The matrix products run on the matrix cores with bfloat16 operands
 * (round to nearest even) and FP32 accumulation; bias, GELU, loss and Adam
 * run in FP32 on FP32 master weights. */
#define LBM_MLP_PARAMS 6723
typedef struct lbm_mlp lbm_mlp;

/* `init` (host, LBM_MLP_PARAMS floats) or NULL for all zeros. */
lbm_status lbm_mlp_create(const float* init, void* stream, lbm_mlp** out);
void lbm_mlp_destroy(lbm_mlp* m);
lbm_status lbm_mlp_get_params(lbm_mlp* m, float* out);
lbm_status lbm_mlp_set_params(lbm_mlp* m, const float* in);

/* Optional z-scoring inside the network's kernels (norm NULL = off): norm
 * (host, 75 floats) = feature mean[36], feature 1/std[36], output scale[3].
 * When on, forward/train/gradient read raw features x and raw targets t:
 * the network sees (x - mean)/std and is fitted to t/scale, and forward
 * returns outputs times scale. */
lbm_status lbm_mlp_set_norm(lbm_mlp* m, const float* norm);

/* Training-input noise: train steps add independent N(0, amplitude^2) noise
 * to every z-scored input (counter-based SplitMix64 + Box-Muller, keyed by
 * seed, step, row and feature).  0 (the default) switches it off; gradients
 * from lbm_mlp_gradient never use it.  Definition: the k-th train step
 * (k = 0, 1, ... since lbm_mlp_create) has key K = seed * 0x100000001B3 + k
 * (mod 2^64); feature c of dataset row i draws r = SplitMix64's output for
 * the state K ^ (64 i + c) (Steele, Lea & Flood 2014: add 0x9E3779B97F4A7C15,
 * then the two xor-shift-multiply rounds), u1 = ((r >> 40) + 1) / (2^24 + 1),
 * u2 = ((r >> 16) mod 2^24) / 2^24, and the variate sqrt(-2 ln u1) cos(2 pi
 * u2) (Box & Muller 1958), evaluated in FP32. */
lbm_status lbm_mlp_set_noise(lbm_mlp* m, float amplitude, uint64_t seed);

/* y[M][3] = network(x[M][36]); device pointers. */
lbm_status lbm_mlp_forward(lbm_mlp* m, const float* x, int64_t M, float* y);

/* One training step on the mini-batch of rows idx[0..B) of x[.][36] and
 * t[.][3] (device; idx NULL = rows 0..B-1): forward, mean squared error,
 * backward, gradient summed over the batch in a fixed order, one Adam step
 * (beta 0.9/0.999, eps 1e-8) with learning rate lr.  *loss (host, may be
 * NULL; non-NULL synchronises) receives the batch loss before the update.
 * B <= 65536. */
lbm_status lbm_mlp_train_step(lbm_mlp* m, const float* x, const float* t, const int32_t* idx, int64_t B,
                              float lr, double* loss);

/* Gradient of the mean squared error on rows [0, B) without updating
 * (host output of LBM_MLP_PARAMS floats); for checking against a reference. */
lbm_status lbm_mlp_gradient(lbm_mlp* m, const float* x, const float* t, int64_t B, float* grad, double* loss);

/* Per-column mean and standard deviation (population) of x[M][ncols]
 * (device), into host arrays; 1 <= ncols <= 65536.  FP64 sums. */
lbm_status lbm_column_moments(const float* x, int64_t M, int32_t ncols, double* mean, double* std, void* stream);

/* For callers that cannot allocate device memory (code running under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same as lbm_column_moments, with the same kernel and the same results bit
 * for bit, but its per-column sums go to a static device array of the
 * library (2 x 4096 doubles = 64 KiB, held on each device it runs on until
 * the process ends) instead of a device allocation per call; it calls no
 * hipMalloc or hipFree.  ncols must lie in [1, 4096] (LBM_ERR_INVALID_ARG
 * otherwise).  Every call on one device shares that device's array, so
 * calls that overlap on one device (other threads, other streams) race;
 * calls in sequence are safe, as each fully rewrites what it reads.
 * Synchronises `stream`. */
lbm_status lbm_column_moments_noalloc(const float* x, int64_t M, int32_t ncols, double* mean, double* std,
                                      void* stream);

/* Training data from a full-domain context: for a wnx x wny window whose
 * node (0, 0) sits at node (ox, oy) of `full`, and n boundary-node indices
 * nodes[] of that window (device), writes the features feat[n][36] and the
 * residual targets target[n][3] (population streaming in from outside the
 * window in `full`, minus the value the plain treatment computes from
 * inside the window, minus bias[node][.] when `bias`, a device array
 * [nb][3] of the window, is not NULL), from full's current state.  The
 * window and its outside neighbours must lie inside `full`. */
lbm_status lbm_sample_boundary(lbm_ctx* full, int32_t ox, int32_t oy, int32_t wnx, int32_t wny,
                               const int32_t* nodes, int64_t n, const float* bias, float* feat, float* target);

/* Switch the context to the learned closure: before every step (or every
 * `interval` steps, lbm_closure_set_interval) the network is evaluated on
 * all boundary nodes from the current state, and its residuals,
 * out_scale * output, are added to the plain values of the missing
 * populations on the boundaries selected by the bit mask `boundaries` (1
 * top, 2 bottom, 4 outlet; the others keep their plain treatment) from one
 * interval later on: an evaluation before step t feeds steps t + interval
 * to t + 2 interval - 1, and the first interval after enabling runs plain.
 * The lag lets the network run on a second stream alongside the launch that
 * starts at step t instead of before it.
 * norm (host): feature mean[36], feature 1/std[36], out_scale[3].  Needs
 * free-slip walls, the copy-unknown outlet and no x-periodicity; the network
 * object must outlive the context's use of it.  A network whose last layer
 * is zero reproduces the plain run bit for bit. */
lbm_status lbm_closure_enable(lbm_ctx* ctx, lbm_mlp* m, const float* norm, int32_t boundaries);
lbm_status lbm_closure_disable(lbm_ctx* ctx);

/* Low-pass of the applied residual per node: r <- r + beta (prediction - r)
 * at each evaluation, starting from r = 0 when the closure is enabled; beta = 1 (the
 * default) applies each prediction as is.  Row nodes within `taper` nodes of
 * the inlet or the outlet column keep the plain treatment (default 0). */
lbm_status lbm_closure_set_filter(lbm_ctx* ctx, float beta, int32_t taper);

/* Guards of the closed loop (all off by default): the network's output is
 * clamped to [-limit, limit] (in units of out_scale, i.e. of the training
 * targets' spread; limit 0 = no clamp) before it becomes a residual; outlet
 * nodes within `outlet_taper` nodes of the top and bottom rows keep the
 * plain treatment; with outlet_neutral != 0 the three outlet residuals of a
 * node are shifted by their mean so that they add no mass (nor x-momentum)
 * to it.  LBM_ERR_INVALID_ARG for a negative limit or taper. */
lbm_status lbm_closure_set_guard(lbm_ctx* ctx, float limit, int32_t outlet_taper, int32_t outlet_neutral);

/* Evaluate the network only every `interval` steps (a divisor of 96: 1, 2,
 * 3, 4, 6, 8, 12, 16, 24, 32, 48 or 96; default 1), before the steps whose
 * index since lbm_create is a multiple of `interval`; its residuals apply
 * during the following interval, the previous ones in between.  A launch
 * of the variant's two, three or four steps runs wherever no evaluation
 * falls strictly inside it (else single steps), the residuals in use
 * entering every step of the launch; the results are the same bit for bit
 * as with one step per launch, with or without graph replay.  beta applies
 * per evaluation. */
lbm_status lbm_closure_set_interval(lbm_ctx* ctx, int32_t interval);

/* A fixed part of the residual per boundary node (host [nb][3], copied;
 * NULL removes it): the closure then applies out_scale * output + bias[node]
 * (the clamp of lbm_closure_set_guard acts on the output alone).  Meant for
 * the time-mean residual of each node in the training data, which leaves
 * the network the fluctuations around it. */
lbm_status lbm_closure_set_bias(lbm_ctx* ctx, const float* bias);

/* Residuals the closure computes from the current state, host [nb][3]
 * (the prediction alone, without the low-pass; the residuals in use are not
 * touched). */
lbm_status lbm_closure_residuals(lbm_ctx* ctx, float* out);

/* Thread-local message of the last failure ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
