/*
 * teuk.h -- C ABI of libteuk.so, an MI355X (gfx950) implementation of the
 * two-step Lax-Wendroff time evolution of the homogeneous (2+1)D Teukolsky
 * equation for one azimuthal mode m on a Kerr background.
 *
 * Source of the operation: Choudhary, Navada, Ginjupalli & Khanna,
 * "An exploration of OpenCL on multiple hardware platforms for a numerical
 * relativity application" (arXiv:1010.3816), Sec. 3: Eq. (1) (Teukolsky
 * master equation, Boyer-Lindquist coordinates), the decomposition
 * Psi = sum_m exp(i m phi) r^3 Phi_m, the first-order system in (Phi, Pi),
 * the two-step Lax-Wendroff scheme Eqs. (lw1) and (lw2), and the boundary
 * conditions stated after them (angular: d_theta Phi = 0 at the poles for
 * even |m|, Phi = 0 for odd |m|; radial: Phi = Pi = 0 at both r* ends).
 *
 * Units: M = 1.  Grid: r*_i = rstar_min + i dr, i = 0..nr-1,
 * dr = (rstar_max - rstar_min)/(nr - 1); theta_j = (j + 1/2) pi/ntheta.
 * Field arrays: complex128 (interleaved re, im doubles; torch.complex128),
 * shape [ntheta][nr], r* fastest, dense (row stride nr).
 *
 * Conventions for every entry point:
 *  - return value: TEUK_OK (0) or a negative TEUK_E_* code; the message of
 *    the last failure on the calling thread is in teuk_last_error().
 *  - "d_" pointers are device pointers on the grid's device, "h_" pointers
 *    are host pointers.  Device work is enqueued on the stream given to
 *    teuk_init_grid and is asynchronous unless stated otherwise.
 *  - argument errors are detected on the host before any device work is
 *    enqueued; the grid is then left unchanged.
 *  - the library never allocates device memory: all device storage lives
 *    in the caller's workspace (teuk_workspace_bytes) and in the caller's
 *    arrays, which the caller keeps alive while work using them is queued.
 *  - a grid handle is not thread-safe; distinct handles are independent.
 */
#ifndef TEUK_H
#define TEUK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TEUK_OK 0
#define TEUK_E_INVALID_ARG (-1) /* an argument is out of range or NULL       */
#define TEUK_E_HIP (-2)         /* a HIP runtime call failed                 */
#define TEUK_E_NONFINITE (-3)   /* the state holds a NaN or an infinity      */
#define TEUK_E_WORKSPACE (-4)   /* workspace too small or misaligned         */
#define TEUK_E_STATE (-5)       /* call not valid in the grid's current state */
#define TEUK_E_UNSTABLE_DT (-6) /* strict mode: dt would let the run blow up  */

#define TEUK_COEF_KERR 0 /* coefficients of Eq. (1) for (a, s, m)           */
#define TEUK_COEF_USER 1 /* caller-supplied coefficient tables              */

#define TEUK_NCOEF 9 /* b, Re c, Im c, Re Ct, Im Ct, A2, A1, Re V0, Im V0   */

typedef struct teuk_grid teuk_grid;

/* Problem description.  The coefficients of the first-order system
 *   d_t Phi + b Phi'         = Pi
 *   d_t Pi - b Pi' + c Phi'  = -Ct Pi + A2 Phi_thth + A1 Phi_th - V0 Phi
 * (' = d/dr*) follow from Eq. (1) with Pi = d_t Phi + b Phi' and
 * b = (r^2 + a^2)/Sigma, Sigma^2 = (r^2 + a^2)^2 - a^2 Delta sin^2 theta. */
typedef struct teuk_params {
    double a;                    /* spin, 0 <= a < 1                              */
    int32_t s;                   /* spin weight, |s| <= 2                         */
    int32_t m;                   /* azimuthal mode number                         */
    int64_t nr;                  /* radial points, 3 <= nr <= 2^24                */
    int64_t ntheta;              /* angular rows, 2 <= ntheta <= 2^20             */
    double rstar_min, rstar_max; /* r* range, rstar_min < rstar_max               */
    double dt;                   /* time step; <= 0: the policy step (below)      */
    int32_t coef_mode;           /* TEUK_COEF_KERR or TEUK_COEF_USER              */
    int32_t n_extract;           /* number of extraction points, 0..4096          */
    const double* extract_rstar; /* h_, n_extract entries, in [rstar_min, rstar_max] */
    const double* extract_theta; /* h_, n_extract entries, in [0, pi]             */
    int64_t stable_steps;        /* horizon of the time-step policy and check     */
} teuk_params;
/* The time step (KERR mode; the explicit scheme's fastest angular mode grows
 * by |g|^2 = 1 + (w dt)^4/4 per step, see teuk_suggest_dt):
 *  - dt <= 0 selects the policy step teuk_suggest_dt(p, N, 10, 0.5): half the
 *    r* spacing, or less so that the fastest angular mode grows at most 10x
 *    over N = stable_steps steps (10,000 if stable_steps <= 0).  The grid's
 *    step is then teuk_get_dt.  It depends on a; gradients with respect to a
 *    treat the step as fixed.
 *  - dt > 0 with stable_steps > 0 (strict mode): TEUK_E_UNSTABLE_DT if dt is
 *    above teuk_suggest_dt(p, stable_steps, 10, 1.0), i.e. the fastest
 *    angular mode would grow more than 10x over stable_steps steps or the r*
 *    Courant number would exceed 1.  The check comes before any other use of
 *    the arguments.
 *  - dt > 0 with stable_steps <= 0: used as given.
 * USER mode needs dt > 0 and ignores stable_steps. */

/* Bytes of device workspace a grid with these parameters needs (0 and an
 * error message if the parameters are invalid).  The workspace must be
 * 256-byte aligned. */
size_t teuk_workspace_bytes(const teuk_params* p);

/* Create a grid.  Solves r*(r) on the host, builds the 1-D radial and angular
 * coefficient tables of Eq. (1) (KERR mode) and uploads them into the
 * workspace on `hip_stream` (a hipStream_t; NULL = default stream).  The
 * call returns after the upload has completed.  The state is zero until
 * teuk_set_initial_data.  *out receives the handle, owned by the caller
 * (teuk_free).  The workspace must stay allocated until teuk_free. */
int teuk_init_grid(const teuk_params* p, void* hip_stream, void* d_workspace, size_t workspace_bytes,
                   teuk_grid** out);

/* USER mode only: copy caller coefficient tables into the workspace.
 * d_ci: [TEUK_NCOEF][ntheta][nr] doubles at r*_i; d_ch: [TEUK_NCOEF][ntheta][nr-1]
 * at r*_{i+1/2}; order as in TEUK_NCOEF.  The arrays may be freed once the
 * stream has passed this call. */
int teuk_set_coefficients(teuk_grid* g, const double* d_ci, const double* d_ch);

/* Set the state to (d_phi, d_pi) (complex128 [ntheta][nr], read only), the
 * initial data of the evolution of Sec. 3.2 (the paper does not state its
 * initial data; any caller data are taken), applying the radial boundary
 * condition of Sec. 3.2 (Phi = Pi = 0 on columns 0 and nr-1) so that the data
 * lie in the space the steps act on, and reset the step counter to 0. */
int teuk_set_initial_data(teuk_grid* g, const void* d_phi, const void* d_pi);

/* Advance the state by n >= 0 Lax-Wendroff steps, Eqs. (lw1)-(lw2), each
 * followed by the boundary conditions.  If d_series is not NULL it receives
 * complex128 [n][n_extract]: entry [k][e] is Phi bilinearly interpolated at
 * extraction point e after step k+1 of this call. */
int teuk_step_n(teuk_grid* g, int64_t n, void* d_series);

/* ---- Inhomogeneous variant (a source term) ----------------------------
 * The Teukolsky equation of a particle-driven problem (an extreme-mass-ratio
 * inspiral, Sec. 1) has a source on its right-hand side; the paper does not
 * give the source model.  Here the source of the first-order system is a
 * caller-supplied separable term in the Pi equation,
 *   d_t Pi - b Pi' + c Phi' = -Ct Pi + A2 Phi_thth + A1 Phi_th - V0 Phi + f(t) g(r*, theta),
 * taken as part of S and evaluated where and when S is in each stage: with
 * f(t_n) and g at r*_{i+1/2} in Eq. (lw1), with f(t_n + dt/2) and g at r*_i
 * in Eq. (lw2).  (Several separable terms add: the evolution is affine.) */

/* Device bytes for teuk_set_source (256-byte aligned, caller-allocated). */
size_t teuk_source_workspace_bytes(const teuk_grid* g);

/* Attach the source profile g: d_gi complex128 [ntheta][nr] at r*_i and
 * d_gh complex128 [ntheta][nr-1] at r*_{i+1/2} (copied into d_src_workspace
 * on the grid's stream; the arrays may be freed once the stream has passed
 * this call; the workspace must stay allocated while the source is used).
 * Both NULL: detach the source.  TEUK_E_INVALID_ARG if only one is NULL,
 * TEUK_E_WORKSPACE if the workspace is missing, misaligned or too small. */
int teuk_set_source(teuk_grid* g, void* d_src_workspace, size_t bytes, const void* d_gi, const void* d_gh);

/* As teuk_step_n with the source term: h_f holds 4n doubles, for step k of
 * the call (t_k its start) Re f(t_k), Im f(t_k), Re f(t_k + dt/2),
 * Im f(t_k + dt/2); the caller keeps the absolute time.  TEUK_E_STATE
 * without teuk_set_source; TEUK_E_INVALID_ARG for a NULL or non-finite h_f. */
int teuk_step_n_source(teuk_grid* g, int64_t n, void* d_series, const double* h_f);

/* The waveform samples of Sec. 3 (the purpose of the evolution is the
 * gravitational waveform; the paper does not say how the field is sampled,
 * and bilinear interpolation of Phi in (r*, theta) between the bracketing
 * columns and cell-centred rows is the reading used here): the current Phi at
 * n points (h_rstar, h_theta: host arrays, r* in range, theta in [0, pi];
 * outside the first and last row centres the angular ghost rows of the pole
 * condition of Sec. 3.2 are used) into d_out (complex128 [n]).  Synchronises
 * the grid's stream. */
int teuk_extract(teuk_grid* g, int32_t n, const double* h_rstar, const double* h_theta, void* d_out);

/* Allocation-free variant of teuk_extract, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): same arguments, same results bit for
 * bit.  The point records are staged in a static device array of the
 * library (192 KiB per device, held until the process ends) instead of the
 * grid's workspace; the call allocates nothing.  n is at most 4096
 * (TEUK_E_INVALID_ARG above).  The array is shared by every call on one
 * device: the call synchronises the grid's stream before it returns, so
 * calls from one thread follow each other, but calls that overlap on one
 * device (other threads or streams) race for it. */
int teuk_extract_noalloc(teuk_grid* g, int32_t n, const double* h_rstar, const double* h_theta, void* d_out);

/* Copy the current state (Phi, Pi of Sec. 3.2 after teuk_steps_taken steps)
 * into caller arrays (complex128 [ntheta][nr]); asynchronous. */
int teuk_get_state(teuk_grid* g, void* d_phi, void* d_pi);

/* Synchronous check of the current state: TEUK_OK if every value is finite,
 * TEUK_E_NONFINITE otherwise. */
int teuk_check_finite(teuk_grid* g);

/* Failure detection inside the step loop (the explicit scheme of Eqs.
 * (lw1)-(lw2) blows up when dt is too large for the angular terms; a blown-up
 * state is all the paper's boundary updates would carry forward).  every >= 1:
 * teuk_step_n and teuk_step_n_store check the state on the device after
 * every `every` steps (at the first pass boundary at or after each multiple,
 * counted from the call's start) and after the call's last step; the first
 * check that finds a NaN or an infinity records its step count on the
 * device, and the call, which then synchronises the grid's stream once at
 * its end, returns TEUK_E_NONFINITE naming that step (the steps are taken
 * regardless; teuk_steps_taken counts them).  Each check reads the state
 * once (32 bytes per point).  every = 0 (default): no checks, the calls stay
 * asynchronous.  TEUK_E_INVALID_ARG for every < 0. */
int teuk_set_finite_check(teuk_grid* g, int64_t every);

/* Steps taken since the last teuk_set_initial_data, and the time step. */
int64_t teuk_steps_taken(const teuk_grid* g);
double teuk_get_dt(const teuk_grid* g);

/* Launch shape of the step kernels: rows of theta per wavefront tile
 * (1..ntheta) and wavefronts per workgroup (1, 2, 4 or 8).  The default cuts
 * the rows so that the tiles just fill a whole number of rounds of the
 * device's resident wavefronts (two per SIMD), taking the fewest rounds that
 * keep a tile within 64 rows (so a grid that fits one round gets the
 * shortest tiles that do, down to one row); 4 wavefronts per workgroup, or 1
 * when the grid has fewer tiles than the device has SIMDs.  Results do not
 * depend on it (every point's arithmetic is the same).  It applies to the
 * sweeps, not to the small-grid block pass (teuk_set_block_launch). */
int teuk_set_tile(teuk_grid* g, int32_t rows_per_tile, int32_t waves_per_block);
int teuk_get_tile(const teuk_grid* g, int32_t* rows_per_tile, int32_t* waves_per_block);

/* Steps per pass over the state: 1 or 2 (default).  With 2, teuk_step_n
 * advances pairs of steps in one kernel pass (temporal blocking: the
 * intermediate state stays in registers, halving the state traffic per
 * step) and an odd last step alone; the per-point arithmetic is that of
 * single steps, so results are identical.  teuk_step_n_store keeps the
 * intermediate state of a pass in its window slot; its first step runs
 * alone (it also copies its input).  Runs whose extraction points share a
 * tile of the two-step kernel run one step per pass.  The tile rows of
 * teuk_set_tile apply; at most 4 wavefronts per workgroup are used.  Where
 * the small-grid block pass is on (teuk_set_block_launch), teuk_step_n takes
 * it instead of these passes.  TEUK_E_INVALID_ARG for other values. */
int teuk_set_steps_per_pass(teuk_grid* g, int32_t steps_per_pass);
int teuk_get_steps_per_pass(const teuk_grid* g, int32_t* steps_per_pass);

/* Small grids: the block pass's launch.  The block pass (grids with
 * ntheta <= 64 and Kerr coefficients) keeps `cols` consecutive columns by all
 * rows of the state in one workgroup's LDS, one point per thread
 * (cols x ntheta <= 1024 threads, 4 <= cols <= 64), and takes `steps` steps
 * per launch (Sec. 3.2, Eqs. (lw1)-(lw2), the same per-point arithmetic as
 * the sweeps, so results are identical); each step consumes one halo column
 * at each side, and the cols - 2 x steps middle columns are written back, so
 * 1 <= steps <= (cols - 2) / 2; steps = 0 turns it off (the sweeps), and
 * cols = 0 keeps the grid's columns (or takes min(64, 1024 / ntheta) if none
 * are set).  teuk_step_n uses it when on, except for a series of more than 8
 * extraction points; teuk_step_n_store and the source-term and adjoint calls
 * keep the sweeps.  Default: among workgroups of up to 256, 512 and 1024
 * threads, the most steps (at least 4) whose workgroups fit the device one
 * per compute unit, the pair scored by the per-step time measured on small
 * grids; off where none fits (400 x 32 on 256 compute units: 16 columns,
 * 7 steps; 6400 x 64: off).  TEUK_E_INVALID_ARG for values out of range or a
 * grid the pass does not take.  The getter reports cols = 0 when unset. */
int teuk_set_block_launch(teuk_grid* g, int32_t steps, int32_t cols);
int teuk_get_block_launch(const teuk_grid* g, int32_t* steps, int32_t* cols);

/* Cache policy of the stores that write the next state (teuk_step_n and its
 * variants, teuk_step_n_tangent) and the next cotangents
 * (teuk_adjoint_step_n): with TEUK_CACHE_KEEP they are ordinary stores,
 * whose lines stay in the device's last-level cache (256 MB on MI355X), so
 * the next pass reads them from there; with TEUK_CACHE_STREAM they are
 * non-temporal, which leaves the cache to the pass's input.  TEUK_CACHE_AUTO
 * (the default) keeps them when two states (the input and the output of a
 * pass) take at most 192 MiB.  Window slots and step tangents are always
 * streamed.  Results do not depend on the policy, only the speed does.
 * TEUK_E_INVALID_ARG for other values.  teuk_get_cache_policy returns the
 * policy and, in *keeps, whether states are currently kept (either may be
 * NULL). */
#define TEUK_CACHE_AUTO 0
#define TEUK_CACHE_KEEP 1
#define TEUK_CACHE_STREAM 2
int teuk_set_cache_policy(teuk_grid* g, int32_t policy);
int teuk_get_cache_policy(const teuk_grid* g, int32_t* policy, int32_t* keeps);

/* Host-only: the Boyer-Lindquist radius r (M = 1) at tortoise coordinate
 * rstar for spin a (the inverse of r*(r) of Sec. 3.2 as read here: r* = r +
 * 2r+/(r+ - r-) ln((r - r+)/2) - 2r-/(r+ - r-) ln((r - r-)/2)), e.g. for the
 * factor r^3 between Phi and Psi.  TEUK_E_INVALID_ARG for a outside [0, 1),
 * a non-finite rstar or a NULL h_r. */
int teuk_radius(double a, double rstar, double* h_r);

/* Host-only: a time step for n_steps steps of this problem.  Returns
 * min(courant * dr, dt_g), where dt_g bounds the growth of the fastest
 * angular mode of the explicit scheme over n_steps to `growth` (for modes
 * smooth in r* the two stages act as the midpoint rule, amplification
 * 1 + z + z^2/2, |.|^2 = 1 + (w dt)^4/4).  The fastest angular frequency w is
 * bounded by Gershgorin's theorem on the discrete theta operator of each
 * column. */
int teuk_suggest_dt(const teuk_params* p, int64_t n_steps, double growth, double courant, double* h_dt);

/* ---- Forward states kept for the adjoint ------------------------------ */

/* Bytes of a window holding n states (one slot per state, layout internal
 * to the library; 256-byte aligned, caller-allocated). */
size_t teuk_window_bytes(const teuk_grid* g, int64_t n);

/* As teuk_step_n, and also leave the state before step k (k = 0..n-1) in
 * window slot k: the steps write their outputs straight into the next slot,
 * so keeping the states costs no extra pass.  The grid's own state ends at
 * step n as with teuk_step_n.  d_window must not overlap the workspace; it
 * may be reused by later calls once the stream has passed the adjoint call
 * that reads it. */
int teuk_step_n_store(teuk_grid* g, int64_t n, void* d_series, void* d_window);

/* ---- Adjoint (gradients of a loss of the extraction series) ------------
 * The Lax-Wendroff step with its boundary conditions is a complex-linear
 * map u^{k+1} = A u^k; for a real loss L with the gradient convention
 * dL/dRe + i dL/dIm, cotangents propagate by the conjugate transpose A^H,
 * and the spin enters through the coefficients of Eq. (1) (and r(r*; a)),
 * dL/da = sum_k Re <lambda^{k+1}, (dA/da) u^k>. */

#define TEUK_ADJ_PROJECT_INITIAL 1 /* zero the radial boundary columns of the result,
                                      giving the gradient w.r.t. the arguments of
                                      teuk_set_initial_data */
#define TEUK_ADJ_TANGENT_WINDOW 2  /* the window holds the step tangents T_k written by
                                      teuk_step_n_tangent instead of the states u^k */

/* Device bytes for teuk_enable_adjoint (256-byte aligned, caller-allocated). */
size_t teuk_adjoint_workspace_bytes(teuk_grid* g);

/* Build the a-derivative tables (dual numbers on the host) and attach the
 * adjoint workspace.  KERR mode only.  Synchronous. */
int teuk_enable_adjoint(teuk_grid* g, void* d_adj_workspace, size_t bytes);

/* Launch shape of the adjoint kernels: theta rows per wavefront tile (1 ..
 * ntheta) and wavefronts per workgroup (1, 2 or 4, default 4; a workgroup
 * takes consecutive tiles of the strip-major tile list, and at most
 * 1 + the chunks per strip of them).  Default rows, at most 16: for the
 * spin-gradient (and one-step) kernel the fewest whose tiles fit 7/8 of one
 * round of two wavefronts per SIMD, leaving the rest to a recompute running
 * beside it; for the two-step cotangent kernel the fewest that fit the whole
 * round.  Setting the tile sets both; get returns the spin-gradient kernel's.
 * The cotangents do not depend on it; dL/da is summed per tile, so its last
 * bits may.  TEUK_E_INVALID_ARG outside these ranges. */
int teuk_set_adjoint_tile(teuk_grid* g, int32_t rows_per_tile, int32_t waves_per_block);
int teuk_get_adjoint_tile(const teuk_grid* g, int32_t* rows_per_tile, int32_t* waves_per_block);

/* Copy window slot k (a state of teuk_step_n_store, or a tangent of
 * teuk_step_n_tangent) into caller arrays (complex128 [ntheta][nr]).  The
 * caller keeps k below the window's slot count; the call cannot check it. */
int teuk_get_window_slot(teuk_grid* g, const void* d_window, int64_t k, void* d_phi, void* d_pi);

/* As teuk_step_n without extraction (n >= 0 steps), and also leave in window
 * slot k (k = 0..n-1) the derivative of step k with respect to the spin at
 * fixed input, T_k = (dA/da) u^{s0+k}, where s0 is the step count before the
 * call: dA/da differentiates the coefficients of Eq. (1) (and r(r*; a)) in
 * both stages of Eqs. (lw1)-(lw2), T_k is zero on the radial boundary
 * columns.  Then dL/da = sum_k Re <lambda^{s0+k+1}, T_k>, which
 * teuk_adjoint_step_n forms with TEUK_ADJ_TANGENT_WINDOW from cotangents it
 * computes anyway, so the reverse sweep needs no forward state.  The states
 * u^{s0+k} equal those of teuk_step_n bit for bit.  Needs teuk_enable_adjoint
 * (TEUK_E_STATE otherwise); d_window as for teuk_step_n_store. */
int teuk_step_n_tangent(teuk_grid* g, int64_t n, void* d_window);

/* Reverse of one segment of n forward steps whose input states are in
 * d_window (as written by teuk_step_n_store; slot k = state s0+k), or whose
 * step tangents are (teuk_step_n_tangent, flag TEUK_ADJ_TANGENT_WINDOW).
 *   d_lam_phi, d_lam_pi  (complex128 [ntheta][nr], in/out): in, the
 *       cotangent of state s0+n from everything after the segment; out, the
 *       cotangent of state s0 including the segment's samples.
 *   d_dL_dseries (complex128 [n][n_extract], or NULL = 0): gradient of L
 *       with respect to the series written by the forward call.
 *   flags: TEUK_ADJ_PROJECT_INITIAL, TEUK_ADJ_TANGENT_WINDOW or both (or 0).
 *   h_dL_da_accum: += this segment's part of dL/da (the call synchronises).
 *       NULL: dL/da is not computed; the cotangents of the linear step do
 *       not depend on the forward states, so d_window may then be NULL (it
 *       is not read) and the call returns without synchronising.
 * Segments are processed last to first; the result of one is the input of
 * the previous one. */
int teuk_adjoint_step_n(teuk_grid* g, int64_t n, void* d_lam_phi, void* d_lam_pi, const void* d_dL_dseries,
                        const void* d_window, int32_t flags, double* h_dL_da_accum);

/* As teuk_adjoint_step_n with the spin gradient, but this segment's part of
 * dL/da is added to the device double *d_dL_da_accum on the grid's stream
 * (accumulators of consecutive calls add in call order) and the call does
 * not synchronise: a reverse pass over many segments keeps the device busy
 * and reads the sum once.  The accumulator must stay allocated until the
 * stream has passed the call.  TEUK_E_INVALID_ARG for a NULL accumulator. */
int teuk_adjoint_step_n_async(teuk_grid* g, int64_t n, void* d_lam_phi, void* d_lam_pi, const void* d_dL_dseries,
                              const void* d_window, int32_t flags, double* d_dL_da_accum);

/* ---- Forward-mode spin derivative ---------------------------------------
 * For the one scalar parameter a, the derivative of the evolution can run
 * forward beside it: v = du/da obeys the tangent-linear step of
 * Eqs. (lw1)-(lw2),
 *     v^{k+1} = A v^k + (dA/da) u^k     (T_k of teuk_step_n_tangent),
 * and the samples of v are ds/da, so for a loss of the series
 * dL/da = sum_k Re <dL/ds_k, ds_k/da> with no reverse sweep and no stored
 * states.  teuk_spin_tangent_workspace_bytes: the bytes of the two buffers
 * of v.  teuk_enable_spin_tangent: needs teuk_enable_adjoint first (it holds
 * the a-derivative tables; TEUK_E_STATE otherwise); d_workspace as the grid
 * workspace (TEUK_E_WORKSPACE if too small or misaligned); sets v = 0.
 * teuk_set_spin_tangent: v from caller arrays (complex128 [ntheta][nr],
 * radial boundary columns ignored, as teuk_set_initial_data), or v = 0 for
 * two NULL pointers; teuk_set_initial_data does not touch v.
 * teuk_get_spin_tangent: the current v into caller arrays. */
size_t teuk_spin_tangent_workspace_bytes(const teuk_grid* g);
int teuk_enable_spin_tangent(teuk_grid* g, void* d_workspace, size_t bytes);
int teuk_set_spin_tangent(teuk_grid* g, const void* d_vphi, const void* d_vpi);
int teuk_get_spin_tangent(teuk_grid* g, void* d_vphi, void* d_vpi);

/* n >= 0 steps of u and v together, one kernel pass per step (the tiles of
 * teuk_set_adjoint_tile).  d_series and d_tseries (complex128
 * [n][n_extract], or NULL): the samples of u and of v after each step, as
 * teuk_step_n writes its series.  The states u equal those of teuk_step_n
 * bit for bit; teuk_set_finite_check applies (to u).  Asynchronous unless
 * the finite check is on.  TEUK_E_STATE before teuk_enable_spin_tangent. */
int teuk_step_n_spin_tangent(teuk_grid* g, int64_t n, void* d_series, void* d_tseries);

/* dL/da from the samples of v: adds sum over the n rows and n_extract
 * points of Re(conj(g) t), with g = d_dL_dseries (the gradient of L with
 * respect to the series of u, complex128 [n][n_extract], PyTorch's complex
 * convention) and t = d_tseries (the series of v of the same call), to the
 * device double *d_dL_da_accum, on the grid's stream without synchronising
 * (one workgroup, a fixed summation order).  TEUK_E_INVALID_ARG for NULL
 * pointers (the series may be NULL when n * n_extract is 0). */
int teuk_spin_gradient(teuk_grid* g, int64_t n, const void* d_dL_dseries, const void* d_tseries,
                       double* d_dL_da_accum);

/* ---- Batched evolutions ------------------------------------------------
 * Many independent grids (each its own a, s, m, nr, ntheta, r* range, dt
 * and extraction points; TEUK_COEF_KERR) advanced together: one persistent
 * launch per pass walks a single work list of all members' tiles, and runs
 * of two launches are replayed from a captured HIP graph.  Every member's
 * arithmetic is identical to that of a single grid.  The azimuthal modes of
 * one field are one use (Sec. 3.2: the m-modes evolve independently): a
 * batch of modes m = -m_max .. m_max sampled with teuk_batch_extract gives
 * the Phi_m whose sum e^{i m phi} r^3 Phi_m is the field Psi at an
 * observer. */
typedef struct teuk_batch teuk_batch;

/* Device bytes for a batch of `count` members (0 if a member is invalid). */
size_t teuk_batch_workspace_bytes(const teuk_params* members, int32_t count);

/* Create a batch: builds every member's tables (synchronous).  The state of
 * every member is zero until teuk_batch_set_initial_data. */
int teuk_batch_init(const teuk_params* members, int32_t count, void* hip_stream, void* d_workspace, size_t bytes,
                    teuk_batch** out);

/* As teuk_set_initial_data / teuk_get_state for one member. */
int teuk_batch_set_initial_data(teuk_batch* b, int32_t member, const void* d_phi, const void* d_pi);
int teuk_batch_get_state(teuk_batch* b, int32_t member, void* d_phi, void* d_pi);

/* Advance every member by n >= 0 steps. */
int teuk_batch_step_n(teuk_batch* b, int64_t n);

/* Bilinear samples of Phi of every member's current state at its extraction
 * points (as teuk_extract), all in one launch: d_out is complex128
 * [teuk_batch_n_extract(b)], the points of member 0 first, each member's in
 * the order of its extract_rstar/extract_theta.  Asynchronous on the batch
 * stream.  TEUK_E_STATE if no member has extraction points. */
int teuk_batch_extract(teuk_batch* b, void* d_out);
int32_t teuk_batch_n_extract(const teuk_batch* b);

/* The field from its azimuthal modes (Sec. 3.2: Psi = e^{i m phi} r^3 Phi
 * for each mode, and the modes add): for every sample k and observer o,
 *   psi[k][o] = r_o^3 * sum_j e^{i m_j phi_o} samples[k][j][o],
 * modes summed in the given order.  h_m: the n_modes (<= 64) mode numbers;
 * h_phi, h_r: the n_obs (<= 64) observers' azimuth and Boyer-Lindquist
 * radius (teuk_radius).  d_samples: complex128 [n_samples][n_modes][n_obs]
 * (the layout of teuk_batch_extract over a batch of one member per mode,
 * each with the same observers); d_psi: complex128 [n_samples][n_obs].
 * Asynchronous on hip_stream.  TEUK_E_INVALID_ARG for sizes out of range,
 * NULL pointers or an observer with r <= 0. */
int teuk_assemble_modes(int64_t n_samples, int32_t n_modes, const int32_t* h_m, int32_t n_obs, const double* h_phi,
                        const double* h_r, const void* d_samples, void* d_psi, void* hip_stream);

/* Launch shape: theta rows per tile, wavefronts per workgroup (1, 2, 4, 8)
 * and workgroups of the persistent launch.  Waits for queued work.  The
 * default is 64 rows (each member's rows at most), 4 wavefronts and
 * 4 x CUs workgroups (four wavefronts per SIMD). */
int teuk_batch_set_launch(teuk_batch* b, int32_t rows_per_tile, int32_t waves_per_block, int32_t n_blocks);
/* A batch writes its members' next states with cache-keeping stores (see
 * teuk_set_cache_policy) when all their states, two per member, take at most
 * 192 MiB; otherwise it streams them. */
/* Steps per launch of the batch: 1 or 2 (default; see teuk_set_steps_per_pass).
 * Member results do not depend on it.  Synchronises the batch's stream. */
int teuk_batch_set_steps_per_pass(teuk_batch* b, int32_t steps_per_pass);
int teuk_batch_get_launch(const teuk_batch* b, int32_t* rows_per_tile, int32_t* waves_per_block,
                          int32_t* n_blocks);

/* Grid points over all members (updates per batched step). */
int64_t teuk_batch_total_points(const teuk_batch* b);

/* Release the batch and its members (host memory only). */
int teuk_batch_free(teuk_batch* b);

/* Release the handle (host memory only; the workspace stays the caller's).
 * Waits for work queued on the grid's stream. */
int teuk_free(teuk_grid* g);

/* Message of the last failed call on this thread ("" if none). */
const char* teuk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TEUK_H */
