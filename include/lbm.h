/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann library for
 * quasi-static linear elasticity in 2D on periodic lattices.
 *
 * Method: Boolakee, Geier, De Lorenzis, "A new lattice Boltzmann scheme for
 * linear elastic solids: periodic problems" (arXiv 2208.14870).  The library
 * solves the damped Navier-Cauchy problem of Sec. 2.1 (Eq. linelasdamp,
 * kappa du/dt = mu lap u + K grad div u + b, with the periodicity of
 * Eq. periodicity and u0 = 0) by pseudo-time stepping of the single-
 * distribution D2Q8 scheme of Algorithm 1 until the steady-state residual
 * falls below a tolerance (Sec. 2.1: ||du/dt|| < TOL "in some norm").
 *
 * Units.  Everything is in lattice units: dx = dt = 1, kappa = 1, U = 1.
 * Material parameters are the lattice Lame parameters lambda~, mu~ (Eq.
 * scaling_example: mu~ = dt mu / (kappa dx^2)); the body force is the per-step
 * force g = b (Sec. 3.3.2, g^(2) = L U^-1 b~ with diffusive scaling).
 *
 * Data layout.  Every field passed across this ABI is an FP64 array in
 * device memory of shape [ny][nx] (x fastest), one array per component.
 * Node (i, j) sits at (i + 1/2, j + 1/2) (Sec. 6.1).  Population arrays are
 * [8][ny][nx] in the one-index order of the velocity table of Sec. 5:
 * 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1).
 *
 * Streams and ownership.  All device work is enqueued on the HIP stream given
 * at creation (NULL = the null stream).  Device pointers passed in are read
 * in stream order; the caller keeps them alive until the stream has
 * synchronised.  Workspaces and arenas are caller-owned device memory; the
 * library never frees caller memory.  Handles are not thread-safe; distinct
 * handles are independent.  No exception or abort crosses the ABI: every call
 * returns a status and lbm_last_error() describes the last failure.
 *
 * Numerics.  LBM_FP64 stores and computes in FP64.  LBM_FP32 stores the
 * populations in FP32 and computes in FP32.  LBM_FP16 stores the populations
 * in FP16 scaled by a per-lattice power of two (the problem is linear and the
 * rest equilibrium of the scheme is zero) and computes in FP32.  Residuals,
 * displacements and error norms are always produced in FP64.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_solver lbm_solver;
typedef struct lbm_batch lbm_batch;

/* Storage precision of the populations. */
enum lbm_precision { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16 = 2 };

/* Status codes: 0 ok, > 0 informational, < 0 error.  The informational
 * codes of lbm_set_body_force are bits and may be combined (2 | 4 = 6). */
enum lbm_status {
    LBM_OK = 0,
    LBM_NOT_CONVERGED = 1,   /* solve stopped at max_steps above tolerance            */
    LBM_W_MEAN_REMOVED = 2,  /* force accepted with its non-zero mean subtracted: the
                                mean of u is conserved, so a load with a mean has no
                                steady state (Sec. 7.2)                                */
    LBM_W_STAGGERED_LOAD = 4, /* force accepted, but it has a component at k = (pi, 0)
                                or (0, pi) (sum (-1)^x gx or sum (-1)^y gy is not at
                                rounding level, even nx or ny): the staggered first
                                moment then oscillates for good, so the iteration
                                from f = 0 does not reach a steady state            */
    LBM_E_ARG = -1,          /* invalid argument (null pointer, size, tolerance)       */
    LBM_E_MATERIAL = -2,     /* mu <= 0, lambda + mu <= 0, non-finite, or theta,
                                omega outside the admissible range                    */
    LBM_E_WORKSPACE = -3,    /* workspace / arena too small, or no room for a lattice */
    LBM_E_HIP = -4,          /* a HIP runtime call failed                              */
    LBM_E_DIVERGED = -5,     /* residual or populations became non-finite, or the
                                update norm kept rising (lbm_set_divergence_guard)    */
    LBM_E_STATE = -6         /* call not valid in the current state (e.g. no force)   */
};

/* ------------------------------------------------------------------------ */
/* Single lattice                                                             */
/* ------------------------------------------------------------------------ */

/* Bytes of device workspace an nx x ny lattice needs at `precision`: two
 * population buffers, the force, the FP64 displacement of the last residual
 * check and reduction scratch.  With `with_polish` != 0 (FP32/FP16 only) the
 * workspace also holds the FP64 state the solver switches to for the final
 * polishing phase (lbm_set_polish).  Returns 0 for invalid sizes. */
size_t lbm_workspace_bytes(int nx, int ny, int precision, int with_polish);

/* Create a solver for a periodic nx x ny lattice (nx, ny >= 1; N = 1 or 2 are
 * valid, neighbours then coincide).  `workspace` is caller-owned device memory
 * of at least lbm_workspace_bytes(nx, ny, precision, with_polish) bytes,
 * 256-byte aligned; `stream` is a hipStream_t (NULL = null stream).  The state
 * starts at f = 0 (equilibrium for u0 = 0, Sec. 6.2).  The force must be set
 * before stepping.  On success *out receives the handle (free with
 * lbm_destroy).  Errors: LBM_E_ARG, LBM_E_WORKSPACE, LBM_E_HIP. */
int lbm_create(int nx, int ny, int precision, int with_polish, void *workspace,
               size_t workspace_bytes, void *stream, lbm_solver **out);

/* In-place streaming (one population buffer instead of two: the "AA" access
 * pattern of optimised lattice Boltzmann codes).  An even step reads each
 * site's own populations and writes the post-collision values into the
 * opposite directions' slots of the same site; an odd step reads those slots
 * at the neighbours and pushes the new post-collision values to the
 * neighbours' own slots.  Every step reads and writes each population once
 * and every memory location is touched by one site only, so one buffer
 * suffices and the bytes per site-update are those of lbm_step; the
 * population footprint halves (about twice the lattice per GPU).  Results are
 * identical to the two-buffer solver bit for bit, with one qualification for
 * FP16 storage: lbm_solve_to_tol may rescale the half storage one step earlier
 * or later than the two-buffer solver, which changes the rounding of
 * subnormal halves only.  Same
 * handle and entry points, with these differences: no LDS tile kernel, no
 * stochastic rounding, no polish phase, and lbm_solve_to_tol evaluates its
 * residual with a launch that does not step (the state cannot step back in
 * place).
 * Workspace: lbm_workspace_bytes_inplace (0 for invalid sizes) runs one step
 * per launch.  Temporal blocking in place (up to k = 2..8 steps per launch
 * through the register wavefront, LBM_FUSED_WAVEFRONT) needs room for copies
 * of the columns and rows that neighbouring waves overwrite during a launch:
 * a ring of columns per strip and 2 x depth rows per segment, taken by a short
 * copy launch before each blocked launch.  lbm_workspace_bytes_inplace_blocked
 * (nx, ny, precision, k, segment_rows) is the workspace with that room for
 * launches of up to k steps with segments of segment_rows rows (0: the default
 * of lbm_set_time_blocking; FP32 8192^2 at k = 8: about a quarter of the
 * population buffer more; 0 for invalid arguments).
 * lbm_create_inplace takes whatever lies beyond lbm_workspace_bytes_inplace
 * as that room and defaults to the deepest k (8 down to 2) whose default shape
 * fits, else to one step per launch.  A blocked launch reads the layout it
 * finds (odd depths start from the even-step layout, even depths from the
 * odd-step one) and always leaves the odd-step layout, so a sequence of n
 * steps runs launches of up to k steps with the parity each start needs and a
 * single step where none fits.  Results are identical to single steps bit for
 * bit. */
size_t lbm_workspace_bytes_inplace(int nx, int ny, int precision);
size_t lbm_workspace_bytes_inplace_blocked(int nx, int ny, int precision, int steps_per_launch,
                                           int segment_rows);
int lbm_create_inplace(int nx, int ny, int precision, void *workspace, size_t workspace_bytes,
                       void *stream, lbm_solver **out);

/* Release the handle (never frees the workspace).  Waits for the stream. */
int lbm_destroy(lbm_solver *s);

/* Material in lattice units.  Sets the relaxation rates of Table "scheme":
 * tau_11 = mu/theta, tau_s = 2K/(1+theta), tau_d = 2 mu/(1-theta),
 * K = lambda + mu, omega = 1/(tau + 1/2) (Eq. relaxation_rate), with
 * theta = 1/3 and omega_12 = omega_21 = omega_22 = 1 unless changed by
 * lbm_set_rates.  Requires mu > 0 and lambda + mu > 0 (then every omega lies
 * in (0, 2), the long-wave stability bound of Eq. stability); finite-k
 * stability is not checked here.  Errors: LBM_E_MATERIAL. */
int lbm_set_material(lbm_solver *s, double lame_lambda, double lame_mu);

/* Optional: the free parameters of the collision (Sec. 3.3.2 remarks,
 * App. C): theta in (0, 1) (third-order equilibrium constant) and the rates
 * omega_12, omega_21, omega_22 in (0, 2).  Defaults 1/3, 1, 1, 1 (the fast
 * path).  Re-derives the rates of the current material.  Errors:
 * LBM_E_MATERIAL. */
int lbm_set_rates(lbm_solver *s, double theta, double omega12, double omega21, double omega22);

/* Body force g (per-step force in lattice units), FP64 device arrays
 * [ny][nx].  The force's FP64 statistics are formed first (a two-stage
 * reduction in a fixed order); a non-finite force returns LBM_E_ARG and leaves
 * the previous force in place.  Otherwise the force is copied into the
 * workspace (in the arithmetic type) with its FP64 mean subtracted from a
 * component whose |mean| exceeds 1e-12 * rms of the force (LBM_W_MEAN_REMOVED;
 * a smaller mean is at the rounding level of the sum and is left as given).
 * Returns the OR of LBM_W_MEAN_REMOVED and LBM_W_STAGGERED_LOAD (see the
 * status codes), or LBM_OK.  Blocking.  Errors: LBM_E_ARG, LBM_E_HIP. */
int lbm_set_body_force(lbm_solver *s, const double *gx, const double *gy);

/* Body force with the leading-order correction of the improved scheme
 * (Sec. 4, Eqs. force_correction_x/y; used in Sec. 7.3.2 and 7.3.3): the
 * library takes in
 *   gx' = gx - (D1 d_xx gx + D2 d_xy gy + D3 d_yy gx),
 *   gy' = gy - (D3' d_xx gy + D2' d_xy gx + D1' d_yy gy)
 * in place of (gx, gy), with D1..D3 the constants of the leading-order error
 * (lbm_leading_error_constants) of the solver's current material and rates
 * (D' = the y row's, equal to D when omega_12 = omega_21).  Set the material
 * and rates first: a later change does not update the correction.
 * gx, gy: FP64 device arrays [ny][nx] as for lbm_set_body_force.
 * d2g: NULL, or an FP64 device array [6][ny][nx] with the planes d_xx gx,
 * d_xy gx, d_yy gx, d_xx gy, d_xy gy, d_yy gy (second derivatives of the
 * per-step force in lattice units, e.g. analytic ones as the paper assumes);
 * NULL takes the second-order central differences of g on the periodic
 * lattice, d_xx g = g(x+1) - 2 g(x) + g(x-1), d_xy g = (g(x+1,y+1) -
 * g(x-1,y+1) - g(x+1,y-1) + g(x-1,y-1)) / 4, which changes the result only at
 * O(k^4) relative.  The corrected force is then treated exactly as by
 * lbm_set_body_force (statistics, mean removal, warnings).  Caller keeps
 * ownership; read in stream order, blocking.  Errors: LBM_E_ARG, LBM_E_STATE
 * (no material), LBM_E_MATERIAL (constants not finite), LBM_E_HIP. */
int lbm_set_body_force_corrected(lbm_solver *s, const double *gx, const double *gy,
                                 const double *d2g);

/* Constants of the leading-order error (Sec. 4, Eq. leadingCoefficients,
 * App. B) for a material (lattice units) and the free rates, host only (no
 * GPU call):  out[0..4] = C1..C5, out[5..7] = D1..D3 (x row; the y row is the
 * same call with omega12 and omega21 exchanged), out[8] = R1, out[9] = R2
 * (Eq. rss_estimate).  Sign: the coefficients of r_x^(4) in Eq. ux_order2.
 * App. B's printed constants are the negatives of these, and three of its
 * terms differ (the tau terms of D1 and D2 are over (1-theta^2)(1-nu^2); the
 * E^3 term of C2 is over 8 theta (1-theta^2)(1-nu^2)^3): these values are the
 * ones the exact scheme has.  Errors: LBM_E_ARG (NULL out), LBM_E_MATERIAL
 * (inadmissible material, theta outside (0, 1), omega outside (0, 2), or a
 * constant not finite). */
int lbm_leading_error_constants(double lame_lambda, double lame_mu, double theta,
                                double omega12, double omega21, double omega22, double out[10]);

/* Rates of the fourth-order special case (Sec. 7.3.3, App. C), host only:
 * out[0] = omega_12 = omega_21 from App. C's tau_12 (which cancels C5),
 * out[1] = omega_22 from the root of C1 = 0 (App. C's printed tau_22 does not
 * cancel C1).  Use with lbm_set_rates(theta, out[0], out[0], out[1]) and
 * lbm_set_body_force_corrected; fourth order holds for loads without mixed
 * derivatives.  Finite-k stability is not checked (Sec. 7.3.3: these rates
 * are unstable for many materials).  Errors: LBM_E_ARG, LBM_E_MATERIAL
 * (inadmissible material, no root, or a rate outside (0, 2)). */
int lbm_fourth_order_rates(double lame_lambda, double lame_mu, double theta, double out[2]);

/* f := 0 (u0 = 0 initialisation at equilibrium, Sec. 6.2), step count := 0,
 * back to the creation precision. */
int lbm_reset(lbm_solver *s);

/* Advance nsteps >= 0 steps of Algorithm 1 (asynchronous on the stream). */
int lbm_step(lbm_solver *s, long long nsteps);

/* Advance nsteps >= 2 steps and return (host double *residual) the steady-state
 * residual of the last two: r(n - 1) = ||u(n - 1) - u(n - 2)||_2 / ||u(n - 1)||_2
 * (Sec. 7.1 grid norm, FP64, R10), n = the step count after the call.  With two
 * buffers and the LDS tile kernel the check rides on the last fused launch.
 * Half storage is rescaled after the check as in lbm_solve_to_tol.  Blocking.
 * Errors: LBM_E_ARG, LBM_E_STATE, LBM_E_DIVERGED (residual not finite),
 * LBM_E_HIP. */
int lbm_step_checked(lbm_solver *s, long long nsteps, double *residual);

/* Pseudo-time stepping to steady state (blocking).  Steps and evaluates
 * r(n) = ||u(n) - u(n-1)||_2 / ||u(n)||_2 (FP64 sums over all nodes and both
 * components; 0 if both vanish) after every `check_every` >= 1 steps of this
 * call, and stops at the first check with r <= tol (LBM_OK) or after
 * max_steps steps of this call (LBM_NOT_CONVERGED).  The state left behind is
 * f(n) with n = *steps_done steps taken by this call; *residual = the last
 * r evaluated (NaN if none).  With a polish threshold set (lbm_set_polish), an
 * FP32/FP16 solver switches to FP64 storage once r <= r_switch or r stops
 * decreasing, resets the two undamped modes that narrow storage leaves
 * rounding noise in to the values of the exact trajectory, and continues in
 * FP64: the staggered first moments at k = (pi,0), (0,pi), which oscillate
 * with period two about -G/2 (G = sum (-1)^x gx, likewise in y) with the
 * amplitude set by the initial state, and the mean first moments (the initial
 * sums plus steps * sum g).  The FP64 phase therefore follows the FP64
 * solver's trajectory: a load with a staggered component (LBM_W_STAGGERED_LOAD)
 * stays unconverged in both.  Small lattices (see lbm_set_small_solve) run the
 * whole call in one workgroup on the device with the same steps, states and
 * outcome.  Errors: LBM_E_ARG, LBM_E_STATE (no force), LBM_E_DIVERGED
 * (non-finite residual, or the rise rule of lbm_set_divergence_guard; the
 * state f(n) of that check step is left readable), LBM_E_HIP. */
int lbm_solve_to_tol(lbm_solver *s, double tol, long long max_steps, int check_every,
                     long long *steps_done, double *residual);

/* Enable the FP64 polishing phase of lbm_solve_to_tol for FP32/FP16
 * storage: switch when r <= r_switch (0 disables).  Needs a workspace made
 * with with_polish != 0.  Errors: LBM_E_STATE. */
int lbm_set_polish(lbm_solver *s, double r_switch);

/* Whole solves of small lattices on the device (lbm_solve_to_tol).  A residual
 * check every K steps makes a small lattice's solve launch-bound, so a
 * two-buffer lattice of at most 1152 FP64 or 2304 FP32 sites (1152 for FP32
 * with a polish switch) runs as one workgroup that keeps both population
 * buffers in LDS, evaluates the residual of Sec. 2.1 at the check steps and
 * stops on the device by the rules of lbm_solve_to_tol, at most
 * `steps_per_launch` steps per launch (the host resumes it, and performs the
 * FP64 switch where the device finds it due).  States and stop steps equal those of the
 * launch-per-check solve (the residual's FP64 sums run in another order).
 * steps_per_launch = 0 turns this off; the default is 65536.  Errors: LBM_E_ARG
 * (negative). */
int lbm_set_small_solve(lbm_solver *s, long long steps_per_launch);

/* Divergence guard of lbm_solve_to_tol (both the launch-per-check and the
 * one-workgroup paths).  With a material outside the stability region of
 * Sec. 5 (e.g. nu = -0.4, E = 0.082, Sec. 7.3.5) the unstable modes grow
 * geometrically, and with them the update norm d(n) = ||u(n) - u(n-1)||_2 (the
 * residual's numerator), long before any value overflows; in a stable solve d
 * decays.  The solve stops with LBM_E_DIVERGED when d rose at each of `checks`
 * consecutive checks and is at least twice the largest d of the 32 checks
 * before that run of rises (a decaying oscillation climbs from its dips, but
 * not above its earlier peaks); a non-finite residual always stops it.  The
 * state of the check step that fired (f(n), n = *steps_done) is left
 * readable.  checks = 0 turns the rise rule off; default 8.  The rule restarts
 * at the FP64 switch of the polish phase.  Errors: LBM_E_ARG (negative). */
int lbm_set_divergence_guard(lbm_solver *s, int checks);

/* Current storage precision (changes to LBM_FP64 after a polish switch). */
int lbm_current_precision(const lbm_solver *s);

/* Steps taken since creation or the last reset. */
long long lbm_steps_done(const lbm_solver *s);

/* Displacement u(n) = (mbar_10, mbar_01) = (m10 + gx/2, m01 + gy/2) of the
 * current state (Table "solution"; Sec. 7.1), FP64 device arrays [ny][nx]. */
int lbm_get_displacement(lbm_solver *s, double *ux, double *uy);

/* Cauchy stress of the current state in lattice units from the bared
 * second-order moments (Eq. compute_bared, Table "solution" without the
 * 1/eps factor): sxx = -(mb_s + mb_d)/2, syy = -(mb_s - mb_d)/2,
 * sxy = -mb_11, mb_a = (1 - omega_a/2) m_a.  FP64 device arrays. */
int lbm_get_stress(lbm_solver *s, double *sxx, double *syy, double *sxy);

/* Error norms of the current displacement against a reference field
 * (FP64 device arrays [ny][nx]); out[4] (host) = { sum |e_i|_2^2,
 * sum |ref_i|_2^2, max |e_i|_inf, max |ref_i|_inf } with e = u - ref: the
 * grid norms of Sec. 7.1 before the dx weighting.  Blocking. */
int lbm_error_norms(lbm_solver *s, const double *ux_ref, const double *uy_ref, double out[4]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the error
 * norms of lbm_error_norms for displacement fields given directly (ux, uy,
 * e.g. from lbm_get_displacement), with no solver handle.  Allocates nothing
 * and does not wait: two kernels on `stream` (a hipStream_t, NULL = null
 * stream) write out[4] (caller-owned FP64 device memory) = { sum |e_i|_2^2,
 * sum |ref_i|_2^2, max |e_i|_inf, max |ref_i|_inf }, e = u - ref, the same
 * values lbm_error_norms returns for the same fields.  The reduction's partials
 * live in a static device array of 32 KiB per GPU (held until the process
 * ends), shared by every call on that GPU: calls that overlap on one GPU race.
 * Limit: nx * ny <= 2^31 (LBM_E_ARG beyond; the scratch does not grow with the
 * lattice).  Errors: LBM_E_ARG (sizes, NULL pointers), LBM_E_HIP; messages
 * through lbm_last_error(NULL). */
int lbm_error_norms_noalloc(int nx, int ny, const double *ux, const double *uy,
                            const double *ux_ref, const double *uy_ref, double *out,
                            void *stream);

/* Checkpoint / restart: the pre-collision populations f(n) as FP64 device
 * arrays [8][ny][nx] (paper order, unscaled).  set leaves the step count
 * unchanged and is blocking (it records the mean first moments of the given
 * state for the polish switch).  With half storage, set first picks the
 * power-of-two scale so that the state's max |f| maps to 2^12 (never finer
 * than the force's steady-state bound), so that no state overflows the half
 * range; LBM_E_ARG for a non-finite state.  State, force and material may be
 * set in any order before the first step: a force or material set later that
 * needs a coarser scale rescales the stored state by that power of two; after
 * the first step a new force or material only coarsens the scale (rescaling
 * the live state), so plain steps do not overflow before the next checked
 * rescale.  lbm_reset returns to the scale of a freshly created solver. */
int lbm_get_populations(lbm_solver *s, double *f);
int lbm_set_populations(lbm_solver *s, const double *f);

/* Launch shape of the step kernel: tile width 2^bx_log2 threads (0..8; the
 * tile height is 256 >> bx_log2 threads times rows_per_thread in {1, 2, 4})
 * and blocks_per_cu: 0 launches one workgroup per tile, k > 0 launches a
 * persistent grid of k workgroups per compute unit that walks the tiles.
 * Results do not depend on the shape.  Used by the autotuner. */
int lbm_set_tile(lbm_solver *s, int bx_log2, int rows_per_thread, int blocks_per_cu);

/* Temporal blocking: with steps_per_launch = k in 2..8, plain steps run k at a
 * time through one fused kernel, so populations cross HBM once per k steps.
 * Results are identical to single steps.  Residual-check steps, remainders
 * and the general-rates variant run one step per launch (with the tile kernel
 * a check rides on the last fused launch).  Overrides the tile shape of
 * lbm_set_tile while active.  Default by storage type and size: FP32 and FP16
 * 8 above 2^17 sites, else 4; FP64 5 below 458752 sites (the tile kernel),
 * else 8 (the wavefront; also after a polish switch).  The fused kernel follows the default of
 * lbm_set_fused_kernel for k until the caller picks one.  In place: the
 * in-place wavefront (see lbm_create_inplace), one column per lane for FP64
 * and for FP16 above four steps, two otherwise on even widths; segments of
 * 256 rows, halved down to 32 while the lattice would give fewer than 4096
 * waves, until the caller picks a segment height.  Errors: LBM_E_ARG (k
 * outside 1..8), LBM_E_WORKSPACE (in place, k >= 2 and the halo room of the
 * workspace is too small for k). */
int lbm_set_time_blocking(lbm_solver *s, int steps_per_launch);

/* Tile height of the LDS tile kernel (the tile is 64 columns wide): rows in
 * {8, 12, 16, 24}, where a kernel exists for the storage type and steps per
 * launch (FP64 8; FP32 16 and 24 at any depth, 8 up to four steps; FP16 16 at
 * any depth, 12 up to four); 0 restores the default of lbm_set_time_blocking.
 * A later change of the steps per launch keeps the choice where a kernel
 * exists for it.  Results do not depend on it.  Errors: LBM_E_ARG. */
int lbm_set_tile_rows(lbm_solver *s, int rows);

/* Fused kernel kinds (both give identical results). */
enum lbm_fused_kernel {
    /* LDS tile: a workgroup advances a 64-wide tile plus a ring of k-1 sites
     * in LDS, then narrower rings down to the tile.  Tile rows: FP64 8; FP32
     * 16 (8 for k <= 4 on lattices of up to 2^21 sites); FP16 12 for k <= 4,
     * 16 above. */
    LBM_FUSED_TILE = 0,
    /* Register wavefront: a wave owns a strip of columns (one per lane, or
     * two per lane for FP32/FP16 on even widths) with a ring of k columns per
     * side (with two per lane: 4 for k <= 4, k rounded up to even above) and
     * marches along y through segments of `segment_rows` rows, keeping the
     * rows of every intermediate step that the next one still reads in
     * registers (x neighbours through cross-lane moves); no LDS. */
    LBM_FUSED_WAVEFRONT = 1
};

/* Select the fused kernel for steps_per_launch >= 2.  segment_rows (1..2^20)
 * is used by LBM_FUSED_WAVEFRONT only: each strip is split into segments of
 * that many rows, each recomputing 2k halo rows.  Default (until this is
 * called, and again after a polish switch), measured: the wavefront for FP64
 * lattices from 458752 sites (about 677^2), FP32 from 2^20 (two columns per
 * lane from 2^25 on even widths) and FP16 from 2^24, with segments as long as
 * leaves one wave per SIMD over the lattice's strips (16 to 128 rows); the
 * tile kernel otherwise.  The tile kernel addresses a plane
 * with 32-bit byte offsets, so a lattice whose planes hold 2^32 bytes or more
 * in the arithmetic type (above 2^30 FP32/FP16 or 2^29 FP64 sites) defaults
 * to the wavefront whatever its width.  In place the wavefront is the only
 * fused kernel; its segment height sets the rows copied per launch.  Errors:
 * LBM_E_ARG, LBM_E_STATE (LBM_FUSED_TILE in place), LBM_E_WORKSPACE (in
 * place, the segment height needs more halo room than the workspace has). */
int lbm_set_fused_kernel(lbm_solver *s, int kind, int segment_rows);

/* Optional, half storage (LBM_FP16) with two buffers: on = 1 rounds every
 * stored population (HBM and the fused kernel's LDS copies) stochastically
 * instead of to nearest: up with probability equal to the discarded fraction
 * of a half ulp (13 random bits), so that changes below half an ulp are not
 * lost and slow modes do not stall.  The random bits are a fixed function of
 * (site, population, step count since lbm_reset, seed): fused and single-step
 * launches (tile and wavefront) give identical bits, and reruns repeat.  Not
 * available in place or in a batch.  Errors: LBM_E_STATE (not half storage,
 * or in place). */
int lbm_set_stochastic_rounding(lbm_solver *s, int on, unsigned int seed);

/* Current launch configuration of plain steps: out[0] steps per launch;
 * out[1] the fused kernel (LBM_FUSED_TILE, LBM_FUSED_WAVEFRONT, or -1 for one
 * step per launch); out[2] its tile rows (tile), segment rows (wavefront) or
 * rows per thread (one step per launch); out[3] threads per workgroup.
 * out is a host array of 4 ints.  Errors: LBM_E_ARG. */
int lbm_get_launch_config(const lbm_solver *s, int out[4]);

/* Columns per lane of the register wavefront when plain steps run through it
 * (1 or 2: a wave's strip is 64 or 128 columns, of which 2 x ring are
 * recomputed neighbours), 0 otherwise.  Errors: LBM_E_ARG. */
int lbm_get_wave_columns(const lbm_solver *s);

/* Diagnostic: nsteps of streaming alone (no collision), for bit-exact checks
 * of the periodic index arithmetic (Eq. streaming, Sec. 6.1). */
int lbm_debug_stream_only(lbm_solver *s, long long nsteps);

/* Message for the last failed call on this handle (never NULL).  With a NULL
 * handle: the last failure of lbm_create / lbm_batch_create in this thread. */
const char *lbm_last_error(const lbm_solver *s);

/* ------------------------------------------------------------------------ */
/* Batches: many independent lattices of uneven size and material stepped    */
/* together, one persistent launch per step over a (lattice, tile) work list. */
/* ------------------------------------------------------------------------ */
/* Plain fused steps of some lattices run through a wavefront launch over a
 * list of their (lattice, strip, segment) waves, one column per lane, beside
 * the tile launch of the others.  By default (see
 * lbm_batch_set_wavefront_sites) these are, per storage type, all of its
 * lattices once they hold at least 2^22 (FP64), 2^23 (FP32) or 2^24 (FP16)
 * sites together, and otherwise those a single solver would step through the
 * register wavefront (FP32 from 2^20 sites, FP64 from 458752, FP16 from
 * 2^24).  A precision with lattices on the list defaults to eight steps per
 * launch.  Residual checks run through the tile kernel for every lattice.
 * Results are identical either way (each equals single steps). */

/* Bytes of arena one lattice occupies in a batch at `precision` (with
 * `with_polish`: plus its FP64 polish state).  Used for admission. */
size_t lbm_batch_slot_bytes(int nx, int ny, int precision, int with_polish);

/* Create a batch over a caller-owned device arena (256-byte aligned) that
 * holds the lattices and the batch bookkeeping; up to max_slots lattices.
 * Errors: LBM_E_ARG, LBM_E_WORKSPACE, LBM_E_HIP. */
int lbm_batch_create(int max_slots, void *arena, size_t arena_bytes, void *stream,
                     lbm_batch **out);
int lbm_batch_destroy(lbm_batch *b);

/* Add a lattice: material (lattice units), FP64 device force arrays [ny][nx],
 * storage precision, optional polish reservation.  The lattice starts at f = 0
 * and joins the next step.  *slot receives its id.  The force is read
 * asynchronously on the batch's stream: keep the arrays valid until that
 * stream has run the call's work (the next lbm_batch_step returns after it;
 * reuse ordered on the same stream is safe).  Adds and removals do not wait
 * for the GPU: the work list is rebuilt once, before the next step.  The
 * force is mean-projected on the device by the rule of lbm_set_body_force (the
 * statistics are formed on the stream before the copy, so a solo solver and a
 * batch slot hold the same force bit for bit); since the call does not wait,
 * its warnings are read with lbm_batch_force_warnings.  LBM_E_WORKSPACE if the
 * arena or the work list has no room (nothing changed). */
int lbm_batch_add(lbm_batch *b, int nx, int ny, int precision, int with_polish,
                  double lame_lambda, double lame_mu, const double *gx, const double *gy,
                  int *slot);

/* Warning bits of a slot's force, as lbm_set_body_force returns them
 * (LBM_W_MEAN_REMOVED | LBM_W_STAGGERED_LOAD, or 0).  Blocking when the slot
 * was added since the last step (it reads the force statistics back).
 * Errors: LBM_E_ARG (no such slot), LBM_E_HIP. */
int lbm_batch_force_warnings(lbm_batch *b, int slot);

/* Remove a lattice and return its memory to the arena (no wait: later work on
 * that memory is ordered on the batch's stream after the launches reading it). */
int lbm_batch_remove(lbm_batch *b, int slot);

/* Advance every active lattice by nsteps >= 1.  With check != 0 the last two
 * steps also evaluate each lattice's residual r(n) (as in lbm_solve_to_tol)
 * at its step count after the call; read them with lbm_batch_residuals.
 * Chunks are replayed from captured HIP graphs.  Asynchronous. */
int lbm_batch_step(lbm_batch *b, long long nsteps, int check);

/* Blocking: residual of the last checked chunk and step count per slot,
 * written for slots 0..max_slots-1 (NaN / -1 for unused slots). */
int lbm_batch_residuals(lbm_batch *b, double *r_host, long long *steps_host);

/* Divergence flags per slot (host int array of max_slots): 1 when a slot's
 * residual, over the checks read by lbm_batch_residuals (each check counted
 * once), became non-finite or its update norm tripped the rise rule of
 * lbm_set_divergence_guard; 0 otherwise and for unused slots.  The rule
 * restarts at lbm_batch_promote.  Not blocking. */
int lbm_batch_diverged(lbm_batch *b, int *flags_host);

/* Rise rule of the batch's divergence guard (see lbm_set_divergence_guard):
 * checks in a row, 0 = off; default 8.  Errors: LBM_E_ARG. */
int lbm_batch_set_divergence_guard(lbm_batch *b, int checks);

/* Switch a FP32/FP16 lattice to FP64 storage (polish phase); needs its
 * polish reservation.  Resets the undamped modes as lbm_solve_to_tol's
 * switch does.  Stream-ordered, no host wait (except right after the slot's
 * lbm_batch_add, whose force statistics it then reads back); the work list is
 * rebuilt before the next launch.  Errors: LBM_E_ARG, LBM_E_STATE (no polish
 * reservation). */
int lbm_batch_promote(lbm_batch *b, int slot);

/* Current displacement of one lattice (FP64 device arrays [ny][nx]). */
int lbm_batch_get_displacement(lbm_batch *b, int slot, double *ux, double *uy);

/* Launch shape for all lattices of the batch (see lbm_set_tile; bx_log2 in
 * 3..8). */
int lbm_batch_set_tile(lbm_batch *b, int bx_log2, int rows_per_thread, int blocks_per_cu);

/* Temporal blocking for all lattices of the batch (see lbm_set_time_blocking,
 * 1..8).  Until set, a storage type with lattices on the wavefront list runs
 * eight steps per launch, and otherwise takes the tile kernel's default for
 * the total sites of its lattices in the batch (FP64 5, FP32 / FP16 8 above
 * 2^17 sites).  Errors: LBM_E_ARG. */
int lbm_batch_set_time_blocking(lbm_batch *b, int steps_per_launch);

/* Which lattices of one storage type (precision LBM_FP64, LBM_FP32 or
 * LBM_FP16) take their plain fused steps through the wavefront list: those
 * with nx * ny >= min_sites (0: all of them), or with -1 the default rule
 * above (the batch autotuner times it against all and none).  Applies to the
 * plain fused launches only (two or more steps per launch).  Errors:
 * LBM_E_ARG. */
int lbm_batch_set_wavefront_sites(lbm_batch *b, int precision, long long min_sites);

/* Temporal blocking for the lattices of one storage type only (precision
 * LBM_FP64, LBM_FP32 or LBM_FP16; steps_per_launch 1..8).  Lattices of each
 * type run their own launch sequence, so the types may differ.  Errors:
 * LBM_E_ARG. */
int lbm_batch_set_time_blocking_for(lbm_batch *b, int precision, int steps_per_launch);

/* Number of active lattices, and arena bytes in use / free (largest hole). */
int lbm_batch_info(const lbm_batch *b, int *active, size_t *used_bytes, size_t *largest_free);

const char *lbm_batch_last_error(const lbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
