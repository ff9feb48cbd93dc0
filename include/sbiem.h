/*
 * sbiem.h - C ABI of the MI355X spectral boundary-integral (sBIEM) hot path
 * for a mildly non-planar 1-D fault in a 2-D in-plane elastic medium
 * (Romanet & Ozawa, "Fully dynamic earthquake cycle simulations on a
 * non-planar fault using the spectral boundary integral element method").
 *
 * What one time step computes (section 3, "Model and algorithm"):
 *   - the elastic shear traction tau^el (section 2.3, eq. Ct and the
 *     truncated form of section 3.1) and the small-slope normal traction
 *     sigma^el driven by curvature x slip (section 2.4), each a static term
 *     plus a per-wavenumber truncated time convolution of the slip-rate
 *     spectra with the closed-form kernels C^T_II and C^N_II, truncation
 *     window T_w(k) of section 3.1, midpoint weights;
 *   - the rate-and-state (aging law) momentum balance solved per element for
 *     the slip rate, inside the two-pass predictor-corrector step of
 *     section 3.3.
 *
 * Conventions used throughout:
 *   - N elements at x_i = i L / N on a periodic fault of length L (metres);
 *     N must be a power of two with 8 <= N <= 2^22.
 *   - Wavenumber index n = 0..N/2, k_n = 2 pi n / L; the forward transform is
 *     F_n = sum_i f_i exp(-i k_n x_i) (the sign fixed by the Fourier pairs of
 *     appendix B).
 *   - Shear traction and slip are positive in the same sense; the normal
 *     traction sigma is compression-positive; the normal elastic traction
 *     uses the multiplier -i sgn(k) mu (Nyquist bin dropped).
 *   - The momentum balance carries radiation damping -mu V / (2 c_s)
 *     (section 2.3: the S-wave inertia term contains it).
 *   - Loading is backslip at the plate rate V_pl: the elastic terms act on
 *     slip - V_pl t and V - V_pl, so uniform sliding at V_pl is a steady
 *     state.  The slip-rate history before the first step is V_pl.
 *   - All arrays passed through this ABI are host memory, FP64, length N,
 *     element-major, owned by the caller; inputs are copied before return and
 *     outputs are fully written before return (host-pointer calls synchronise
 *     the plan's stream).  A plan owns all of its device memory.
 *   - Return value: SBIEM_OK (0) or a negative status; sbiem_last_error()
 *     gives a message.  A plan is not thread-safe; distinct plans are
 *     independent.
 */
#ifndef SBIEM_H
#define SBIEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBIEM_ABI_VERSION 3

typedef struct sbiem_plan sbiem_plan;
typedef struct sbiem_batch sbiem_batch;

enum sbiem_status {
  SBIEM_OK = 0,
  SBIEM_EINVAL = -1,    /* invalid argument or call order                       */
  SBIEM_ENOMEM = -2,    /* device or host allocation failed                     */
  SBIEM_EDEVICE = -3,   /* HIP runtime error / no usable gfx950 device          */
  SBIEM_ENEWTON = -4,   /* momentum balance did not converge (section 3.2)      */
  SBIEM_ESTATE = -5,    /* state variable became non-positive (section 3.2)     */
  SBIEM_EOPEN = -6,     /* normal traction not compressive (section 3.2)        */
  SBIEM_ENOTREADY = -7  /* friction, state or time step not set yet             */
};

/* Precision of the history convolution and the FFTs.  Slip, slip rate,
 * state, the spectral slip accumulators and the friction solve are FP64 in
 * both modes.  SBIEM_FP32CONV keeps the slip-rate history in FP32 and
 * evaluates the kernel weights on the fly from an interpolated table. */
enum sbiem_precision { SBIEM_FP64 = 0, SBIEM_FP32CONV = 1 };

/* State update of each pass (section 3.3).  PAPER: theta_p = theta_0 +
 * dt * thetadot_c (the paper's explicit update).  EXP: exact integration of
 * the aging law at the pass's constant rate V_c,
 * theta_p = Dc/V_c + (theta_0 - Dc/V_c) exp(-V_c dt / Dc); it stays positive
 * where the explicit update is unstable (V dt / Dc > 2). */
enum sbiem_theta_mode { SBIEM_THETA_PAPER = 0, SBIEM_THETA_EXP = 1 };

/* Convolution weights of the history intervals (section 3.1; the paper
 * names only "the midpoint method").  MIDPOINT (rule R1): the weight of lag
 * j (interval [j dt, (j+1) dt] back from the evaluation time) is
 * dt C(c_s |k| (j + 1/2) dt).  INTERVAL (rule R2): the exact integral of the
 * kernel over the interval, clipped at the window end T_w,
 * [P(c_s |k| min((j+1) dt, T_w)) - P(c_s |k| j dt)] / (c_s |k|), with P the
 * closed-form primitive of the kernel (sbiem_kernel_primitive_eval); this is
 * the rule of variable steps. */
enum sbiem_rule { SBIEM_RULE_MIDPOINT = 0, SBIEM_RULE_INTERVAL = 1 };

/* Outcomes recorded by sbiem_adapt for each attempted step. */
enum sbiem_adapt_outcome {
  SBIEM_ADAPT_ACCEPT = 0,  /* eps <= eps0: kept (the two-half-step solution) */
  SBIEM_ADAPT_REJECT = 1,  /* eps > eps0: taken again with a smaller dt      */
  SBIEM_ADAPT_FAIL = 2,    /* a step failed: taken again with dt/2           */
  SBIEM_ADAPT_FLOOR = 3,   /* eps > eps0 at dt_min: kept anyway              */
  SBIEM_ADAPT_STOP = 4     /* a step failed at dt_min: the run stops         */
};

/* ABI version of the loaded library (SBIEM_ABI_VERSION it was built with). */
int sbiem_abi_version(void);

/* Human-readable name of a status code (static string). */
const char* sbiem_status_string(int status);

/* Create a plan for one fault.
 *   N       number of elements (power of two, 8..2^22)
 *   L       periodic fault length [m] (> 0)
 *   mu      shear modulus [Pa] (> 0)
 *   nu      Poisson's ratio; only checked for consistency with the wave
 *           speeds: 0 < nu < 0.5 and |nu - nu(c_s, c_p)| <= 1e-3, where
 *           c_p^2/c_s^2 = 2(1-nu)/(1-2nu).  The kernels use r = c_s^2/c_p^2.
 *   cs, cp  shear and dilatational wave speeds [m/s], 0 < cs < cp
 *   h       fault profile h(x_i) [m], length N, copied; NULL = planar.
 *           The curvature kappa = h'' (section 2.2, small-slope
 *           approximation) is computed spectrally on the host in extended
 *           (long double) precision: kappa = IDFT(-k_n^2 DFT(h)), Nyquist
 *           term kept, then rounded to FP64 and uploaded.
 * Selects a device (the current HIP device) and allocates the per-element
 * buffers.  Errors: EINVAL (bad arguments, non-finite h), EDEVICE, ENOMEM.
 * On error *out is NULL. */
int sbiem_plan_create(sbiem_plan** out, int64_t N, double L, double mu, double nu,
                      double cs, double cp, const double* h);

/* Release a plan and all its device memory (NULL is a no-op). */
int sbiem_plan_destroy(sbiem_plan* p);

/* Message of the last failing call on p; with p == NULL, the last failing
 * call of this thread that had no plan (e.g. sbiem_plan_create).  The string
 * is owned by the library and valid until the next call on the same plan. */
const char* sbiem_last_error(const sbiem_plan* p);

/* Choose SBIEM_FP64 (default) or SBIEM_FP32CONV.  Must precede
 * sbiem_set_dt / the first step; EINVAL afterwards. */
int sbiem_set_precision(sbiem_plan* p, int mode);

/* Choose SBIEM_THETA_PAPER (default) or SBIEM_THETA_EXP; may change
 * between steps. */
int sbiem_set_theta_mode(sbiem_plan* p, int mode);

/* Iteration limit of the double-precision Newton phase of each element's
 * momentum balance (section 3.3; default 100, 0 restores it; at most 1000).
 * A solve that has not converged within the limit fails the step with
 * SBIEM_ENEWTON (section 3.2's "Newton-Raphson did not converge"); small
 * limits force that failure from the host.  May change between steps.
 * Errors: EINVAL (out of range). */
int sbiem_set_newton_limit(sbiem_plan* p, int max_iterations);

/* Weight rule of the history convolution (SBIEM_RULE_MIDPOINT default, or
 * SBIEM_RULE_INTERVAL).  Must precede sbiem_set_dt / the first step
 * (EINVAL afterwards); adaptive plans always use the INTERVAL rule.  FP32
 * plans on the INTERVAL rule run on the variable-step engine (see
 * sbiem_set_adaptive), whose weights are evaluated per step; FP64 plans take
 * exact per-lag weights from the host.  The learned closure needs the
 * MIDPOINT rule.  Errors: EINVAL. */
int sbiem_set_rule(sbiem_plan* p, int rule);

/* Cut-off wavenumbers of the truncation window (section 3.1), given as
 * k_c L for the shear and for the normal kernel (the paper uses one value,
 * 200, for both and suggests separate ones because the normal kernel
 * converges more slowly): T_w^X(k) = (L/c_s) min(1, k_c^X / |k|).  A mode
 * keeps the history of the longer window; each kind's weights are zero past
 * its own.  Must precede sbiem_set_dt (EINVAL afterwards); values in
 * [1, 1e6].  The learned closure needs equal values. */
int sbiem_set_cutoffs(sbiem_plan* p, double kcL_shear, double kcL_normal);

/* Variable time steps (section 3.2) on (1) or off (0).  Must precede
 * sbiem_set_dt, whose dt then becomes the smallest step dt_min (the paper
 * takes beta_min dx / c_s with beta_min = 0.25).  The slip-rate history is
 * then a list of committed intervals of any length >= dt_min: each mode
 * keeps ceil(T_w / dt_min) + 2 of them in its ring (the two more that a
 * rejected attempt may overwrite), the interval times in a per-fault log,
 * and every step weighs each stored interval by the exact kernel integral
 * over its lag span (INTERVAL rule).  Steps run launch by launch (no graph,
 * no overlap of the next step's convolution).  Not with the learned
 * closure or in batches.  Errors: EINVAL. */
int sbiem_set_adaptive(sbiem_plan* p, int on);

/* One two-pass step of length dt >= dt_min (section 3.3) on an adaptive
 * plan (or an FP32 INTERVAL-rule plan), against its non-uniform history.
 * Synchronous; failures as sbiem_step (state left at the start of the
 * step).  sbiem_step and sbiem_run on such plans take steps of the dt they
 * are given the same way.  Errors: EINVAL (dt < dt_min, other plans),
 * ENOTREADY, ENEWTON / ESTATE / EOPEN. */
int sbiem_step_var(sbiem_plan* p, double dt);

/* Step-size control of section 3.2 on an adaptive plan.  Each attempt takes
 * one step of dt and, from the same state, two steps of dt/2;
 * eps = max over elements of |ln V_1 - ln V_2| and |ln theta_1 - ln theta_2|
 * (reading: the paper names neither the variable nor the norm).
 *   eps <= eps0: accepted with the two-half-step solution; the next dt is
 *     min(dt_max, 5 dt, max(dt_min, 0.9 (eps0/eps)^(1/3) dt)) (5 dt when
 *     eps = 0);
 *   eps > eps0: taken again with max(dt_min, 0.9 (eps0/eps)^(1/3) dt);
 *   a failed step (ENEWTON, ESTATE, EOPEN): taken again with
 *     max(dt_min, dt/2);
 *   at dt_min an error above eps0 is accepted (FLOOR) and a failure stops
 *     the run: its status is returned, the state is that of the last
 *     accepted step.
 * Runs until max_accepted steps are accepted or the time reaches t_end
 * (the last step is not shortened to hit it).  *dt_io: first dt to try on
 * entry, next dt to try on return.  log (may be NULL): host array of
 * log_cap records of 4 doubles (t at the attempt's start, dt, eps or -1
 * for a failed attempt, outcome from sbiem_adapt_outcome); *log_len (may be
 * NULL) receives the number of attempts (records past log_cap are counted,
 * not written).  eps0 > 0, dt_max >= dt_min.  On SBIEM_FP32CONV plans the
 * spectral slip of the static term, integrated from FP32 rate spectra, is
 * recomputed from the FP64 slip after every 32nd accepted step (counted
 * from sbiem_set_state), so its rounding does not accumulate over long
 * runs.  Errors: EINVAL, ENOTREADY, the stopping step's status. */
int sbiem_adapt(sbiem_plan* p, double eps0, double dt_max, double t_end, int64_t max_accepted,
                double* dt_io, double* log, int64_t log_cap, int64_t* log_len);

/* sbiem_adapt for event-driven runs (seismic cycles, section 6): the same
 * controller, and the run also ends after the first accepted step whose
 * maximum slip rate lies on the other side of v_cross [m/s] than the
 * maximum slip rate before it (v_cross <= 0: no such stop; the first
 * comparison is with the state the call starts from).  log records hold
 * 5 doubles: those of sbiem_adapt, then the maximum slip rate of the
 * attempt's two-half-step solution (-1 for a failed attempt).  *crossed
 * (may be NULL) is 1 if the run ended at such a crossing, else 0.  Errors
 * as sbiem_adapt; EINVAL for a non-finite v_cross. */
int sbiem_adapt_until(sbiem_plan* p, double eps0, double dt_max, double t_end,
                      int64_t max_accepted, double v_cross, double* dt_io, double* log,
                      int64_t log_cap, int64_t* log_len, int* crossed);

/* Rate-and-state friction and loading (section 3, eq. momentum; aging law).
 *   a, b         [N] direct and evolution effects (a > 0)
 *   Dc, V_ref, f0  critical slip [m], reference velocity [m/s] (the law's
 *                "V0"), reference friction
 *   sigma_load   [N] normal load [Pa], compression positive
 *   tau_load     [N] shear load [Pa] at t = 0; grows as tau_load_rate * t
 *   V_pl         plate rate [m/s] of the backslip loading (may be 0)
 * Errors: EINVAL (non-finite values, a <= 0, Dc <= 0, V_ref <= 0). */
int sbiem_set_friction(sbiem_plan* p, const double* a, const double* b, double Dc,
                       double V_ref, double f0, const double* sigma_load,
                       const double* tau_load, double tau_load_rate, double V_pl);

/* Constrained elements (the fault-benchmark section holds the periodic line
 * outside the fault at null slip rate): mask [N], nonzero = constrained.
 * A constrained element slides at exactly V_pl (zero slip rate in the
 * loading frame of eq. momentum): no friction solve, no failure, state and
 * thetadot frozen (thetadot = 0), V = V_pl.  NULL or an all-zero mask frees
 * every element.  Needs sbiem_set_friction first (ENOTREADY); a later
 * set_friction frees every element.  Both calls clear the state when a mask
 * was or is in force: sbiem_set_state must follow (ENOTREADY until then). */
int sbiem_set_constrained(sbiem_plan* p, const uint8_t* mask);

/* Set slip [m], slip rate [m/s] (> 0) and state [s] (> 0) at time t and
 * clear the slip-rate history (rates before t are V_pl).  thetadot is set
 * from the aging law, 1 - theta V / Dc, so set_friction must come first
 * (else ENOTREADY).  At constrained elements the V given is replaced by V_pl
 * (any finite value is accepted there) and thetadot is 0.  Clears a pending
 * failure. */
int sbiem_set_state(sbiem_plan* p, const double* slip, const double* V,
                    const double* theta, double t);

/* Read the state after the last committed step.  Any output pointer may be
 * NULL.  tau_el and sigma_el are the elastic tractions of the last pass
 * (without radiation damping and without the loads); zero before the first
 * step. */
int sbiem_get_state(sbiem_plan* p, double* slip, double* V, double* theta,
                    double* tau_el, double* sigma_el, double* t);

/* The plan's curvature kappa = h'' [1/m], length N, as the kernels use it
 * (the FP64 rounding of the extended-precision spectral second derivative
 * computed by sbiem_plan_create). */
int sbiem_get_curvature(const sbiem_plan* p, double* kappa);

/* Fix the time step dt [s] (> 0): computes the windows M_n (section 3.1:
 * T_w(k) = (L/c_s) min(1, k_c/|k|), k_c = 200/L, M_n = ceil(T_w/dt) with a
 * 1e-9 relative guard), the midpoint weights w_{n,j} = dt C(c_s|k_n|(j+1/2)dt)
 * and allocates the zeroed history ring.  Clears the history.  Called
 * implicitly by the first sbiem_step/sbiem_run. */
int sbiem_set_dt(sbiem_plan* p, double dt);

/* Window lengths M_n for n = 1..N/2 (M[0] is mode 1) at time step dt,
 * computed on the host: the longer of the shear and normal windows
 * (sbiem_set_cutoffs); does not change the plan. */
int sbiem_window_lengths(const sbiem_plan* p, double dt, int64_t* M);

/* Stress-only evaluation of the spectral-time functional (section 3.1):
 * the elastic tractions at t_nt of a slip history slip_hist
 * [(nt+1) * N], oldest snapshot first, snapshot m at t_m = m dt.  The rate of
 * interval [t_l, t_{l+1}] is the first difference of the snapshots; the
 * static terms act on the last snapshot; no backslip (V_pl = 0), no
 * radiation damping.  Uses the plan's precision; does not touch the
 * stepping state.  Errors: EINVAL (nt < 0, dt <= 0). */
int sbiem_stress(sbiem_plan* p, const double* slip_hist, int64_t nt, double dt,
                 double* tau_out, double* sigma_out);

/* One two-pass step of length dt (section 3.3).  dt must equal the plan's
 * dt once set, except on adaptive and FP32 INTERVAL-rule plans, which take
 * any dt >= dt_min (sbiem_step_var).  Synchronous: returns
 * ENEWTON / ESTATE / EOPEN if the step failed, leaving the state at the
 * start of the step (section 3.2).  ENOTREADY without friction and state. */
int sbiem_step(sbiem_plan* p, double dt);

/* nsteps steps launched back to back without host synchronisation (a
 * captured HIP graph replayed), then one synchronisation.  The first
 * failing step stops the run: the state is left at the start of that step
 * and its status returned; sbiem_steps_done tells how far it got. */
int sbiem_run(sbiem_plan* p, double dt, int64_t nsteps);

/* Number of committed steps since the last set_state / set_dt. */
int sbiem_steps_done(const sbiem_plan* p, int64_t* nsteps);

/* Failure report of the last step/run: number of failing elements of the
 * failing pass and the first failing element index (-1 if none). */
int sbiem_failures(const sbiem_plan* p, int64_t* count, int64_t* first_index);

/* Run the plan's work on this HIP stream (hipStream_t passed as void*,
 * e.g. torch.cuda.current_stream().cuda_stream).  Default: the null
 * stream.  Invalidates captured graphs. */
int sbiem_set_stream(sbiem_plan* p, void* hip_stream);

/* Process-wide device allocator used for plan and batch memory allocated
 * after this call (e.g. a caching allocator).  alloc returns NULL on
 * failure; both NULL restores hipMalloc/hipFree. */
int sbiem_set_allocator(void* (*alloc)(size_t bytes, void* ctx),
                        void (*release)(void* ptr, void* ctx), void* ctx);

/* Host evaluation (extended precision) of the kernels of sections 2.3/2.4
 * and their derivatives at dimensionless times T[i] = c_s |k| t >= 0.
 * Any output may be NULL.  Used to build the weight tables; exported for
 * verification. */
int sbiem_kernel_eval(double cs, double cp, const double* T, int64_t n, double* CT,
                      double* CN, double* dCT, double* dCN);

/* Host evaluation (extended precision) of the kernel primitives
 * P^X(T) = integral of C^X over [0, T] at T[i] >= 0 (closed form from
 * elementary primitives of the terms of sections 2.3 and 2.4); any output
 * may be NULL.  Used for the INTERVAL-rule weights; exported for
 * verification. */
int sbiem_kernel_primitive_eval(double cs, double cp, const double* T, int64_t n, double* PT,
                                double* PN);

/* Slip/curvature scaling diagnostic (section 5: the scaled slip gradient
 * (1/(f du)) d(du)/dy equals -kappa away from the fault's edges).  For a
 * slip profile du [N] on the periodic grid x_i = i L/N (host arrays,
 * natural order) writes ratio[i] = (du[i+1] - du[i-1]) / (2 dx f du[i]),
 * dx = L/N, indices mod N (second-order centred difference; along-fault
 * distance is x to first order in the slope), NaN where |du[i]| <=
 * slip_floor.  Compare with -kappa from sbiem_get_curvature.  Host only;
 * no plan.  Errors: EINVAL (N < 3, L <= 0, f = 0 or non-finite, NULL,
 * slip_floor < 0). */
int sbiem_slip_scaling(int64_t N, double L, double f, const double* slip, double slip_floor,
                       double* ratio);

/* Per-launch timing of the history-convolution kernel with HIP events on
 * the stream it runs on.  While on, sbiem_run launches one step in every 33
 * directly, its convolution bracketed by two events, and replays the other
 * steps from the step graph (results are identical either way).
 * On the variable-step engine (sbiem_step_var, sbiem_adapt,
 * sbiem_adapt_until) every convolution launch is timed instead, by events
 * that the launch itself stamps with its start and end.
 * sbiem_profile returns the accumulated milliseconds and launch count, the
 * algorithmic bytes one launch reads and writes (ring records of lags
 * 2..M_n-1, partial sums; on the variable-step engine the average over
 * the evented launches of the records inside each mode's window at the
 * launch's time, the interval-log entries they use and the partial sums)
 * and resets the counters. */
int sbiem_set_profiling(sbiem_plan* p, int on);
int sbiem_profile(sbiem_plan* p, double* conv_ms, int64_t* conv_launches,
                  double* conv_bytes_per_launch);

/* Ensembles: independent faults of uneven N stepped together (one launch
 * per phase for all faults, graph-captured).  The plans keep their own
 * state and must share precision; each must have friction, state and dt
 * set.  A batch holds references to the plans (destroy the batch first). */
int sbiem_batch_create(sbiem_batch** out, sbiem_plan* const* plans, int64_t n);
int sbiem_batch_destroy(sbiem_batch* b);
/* nsteps steps of every member; returns the first failing member's status
 * (other members keep stepping; each failed member stops at the start of its
 * failing step). */
int sbiem_batch_run(sbiem_batch* b, int64_t nsteps);
int sbiem_batch_set_profiling(sbiem_batch* b, int on);
int sbiem_batch_profile(sbiem_batch* b, double* conv_ms, int64_t* conv_launches,
                        double* conv_bytes_per_launch);

/* Autotuning of the history-convolution launch for this plan's (or batch's)
 * workload: whole steps are replayed with each candidate number of
 * convolution workgroups (the full resident grid, and grids that leave one
 * workgroup fewer on 64, 128, 192 or all 256 CUs so that the element and
 * mode launches of the step run beside it), each with the convolution or the
 * first element launch enqueued first after the previous step's commit and,
 * with the learned closure on, with its network launched after the
 * convolution or before the first element launch, steps_per_trial steps
 * each (rounded up to the 16-step graph, plus one settling graph); the
 * fastest is tried once more with the convolution's record loads on the
 * default cache policy instead of the non-temporal one, and the faster of the
 * two is kept until the plan's tables are rebuilt (sbiem_set_dt,
 * sbiem_set_precision, sbiem_set_closure).  Unless a member's tile was set
 * with sbiem_set_conv_tile, all of this is repeated for each FP32 tile
 * shape (256, 320, 512 and 1024 ring records per tile; the ring itself does
 * not change) and the fastest tile is kept with its grid and order.  The trial
 * steps are ordinary steps: results do not depend on the launch shape or
 * order, and a tile change alters only the FP32 summation order of the
 * history sums; the state advances by about (steps_per_trial + 16) times the
 * number of candidates (at most 11, 21 with the closure, per tile).
 * *conv_workgroups (may be NULL) receives the chosen grid
 * (sbiem_get_conv_tile the tile).  FP64 plans have nothing to tune (OK).
 * Errors as sbiem_run; a plan used by a batch is tuned through the batch. */
int sbiem_tune(sbiem_plan* p, double dt, int64_t steps_per_trial, int32_t* conv_workgroups);

/* FP32 convolution tile: records = 256, 512 or 1024 ring records per
 * wavefront tile (16 rows of 64 records in flight per wave either way, so a
 * workgroup task stays 8192 records), 320 (five rows, four tiles per wave:
 * 20 rows in flight, tasks of 10240 records), or 0 for the default by window length
 * (512; 256 under the learned closure, whose kept windows are short).
 * records = 64 selects packed rows: every 64-record row of every mode in
 * order, 16 to a wave and 128 to a task, so no row lies past a mode's end
 * (sbiem_tune does not try it: slower on every workload measured).  A
 * non-zero tile is kept by sbiem_tune.  The tiling is the summation order
 * of the FP32 history sums, so runs on different tiles agree to FP32
 * rounding, runs on one tile bit for bit.  Applies to FP32 fixed-step plans
 * (others keep 256 FP64 slots); takes effect at once (pending sums are
 * recomputed).  Errors: EINVAL (other sizes, a plan used by a batch). */
int sbiem_set_conv_tile(sbiem_plan* p, int records);
/* The tile in use (records per tile). */
int sbiem_get_conv_tile(const sbiem_plan* p, int* records);
int sbiem_batch_tune(sbiem_batch* b, int64_t steps_per_trial, int32_t* conv_workgroups);

/* ---------------------------------------------------------------------------
 * Learned tail closure.  Not part of the paper: it shortens the history
 * window of section 3.1 and predicts the part of the convolution that falls
 * beyond the cut.  With cut c, a mode n keeps M'_n = ceil(c M_n) lags when
 * 18 <= M'_n < M_n (other modes keep their whole window); the tail
 *   tail^X_n = sum_{j=M'_n}^{M_n-1} w^X_{n,j} H^X_n(lag j),  X = shear, normal,
 * is predicted by one network per kind: input (33 values) T_cut/100 with
 * T_cut = c_s |k_n| M'_n dt, then the 16 oldest kept values
 * H(lag M'_n-16+k), k = 0..15, as (Re, Im) pairs divided by their RMS r;
 * output y (2 values), a correction to the constant extrapolation of the
 * oldest kept value a_15 = H(lag M'_n-1) over the discarded lags:
 *   tail = D^X_n a_15 + (y_0 + i y_1) r / (c_s |k_n|),
 *   D^X_n = sum_{j=M'_n}^{M_n-1} w^X_{n,j}  (computed by the library).
 * A zero network therefore gives the constant extrapolation.  Layers
 * 33 -> 64 -> 64 -> 2, GELU (erf form) after the first two.
 * Parameters: SBIEM_CLOSURE_PARAMS floats in the order W1[33][64], b1[64],
 * W2[64][64], b2[64], W3[64][2], b3[2] (row = input), h1 = gelu(x W1 + b1),
 * h2 = gelu(h1 W2 + b2), y = h2 W3 + b3.  Inference uses bfloat16 weights and
 * layer inputs with float32 accumulation (matrix cores) and evaluates erf by
 * Abramowitz & Stegun 7.1.26 (error < 1.5e-7); training float32 with erf.
 * ------------------------------------------------------------------------- */
#define SBIEM_CLOSURE_PARAMS 6466

/* Enable the closure on a SBIEM_FP32CONV plan with the shear and normal
 * networks (host, SBIEM_CLOSURE_PARAMS floats each, copied) and cut
 * 0 < c < 1 (0.25: a quarter of each window); both NULL disables it.  With a
 * time step already set, the tables and ring are rebuilt as by
 * sbiem_set_dt: the state is kept and the history restarts.  EINVAL for
 * FP64 plans, non-finite parameters or a plan used by a batch. */
int sbiem_set_closure(sbiem_plan* p, const float* params_shear, const float* params_normal,
                      double cut);

/* Training pairs from the current history of a plain SBIEM_FP32CONV plan
 * (whole windows, state and dt set): for every mode n = 1..N/2 that cut c
 * would close and both kinds (0 shear, 1 normal), the network input
 * X[kind][n][33], the target Y[kind][n][2] = (exact tail - D a_15) c_s |k_n| / r
 * (complex as two floats; the tail uses the FP32 convolution weights) and
 * the scale R[kind][n] = r.  Rows of modes that stay open, and rows with
 * r = 0, are zero.  X, Y, R: host, 2 (N/2+1) rows, written. */
int sbiem_closure_sample(sbiem_plan* p, double cut, float* X, float* Y, double* R);

/* Evaluate one network on n inputs X[n][33] (host) with the matrix-core
 * inference kernel; Y[n][2] (host) written. */
int sbiem_closure_eval(const float* params, const float* X, int64_t n, float* Y);

/* Adam training of one network on the device (float32): `steps` updates on
 * minibatches of `batch` rows of (X[n][33], Y[n][2]); update k uses rows
 * (t_k batch + i) mod n, i < batch, with t_k the number of updates so far
 * (*adam_t on entry plus k).  Loss: mean over the batch of sum_o (y_o - Y_o)^2.
 * Adam with beta1 0.9, beta2 0.999, eps 1e-8 and step size lr.  params,
 * adam_m, adam_v (SBIEM_CLOSURE_PARAMS floats each) and adam_t are updated
 * in place; losses[steps] (may be NULL) receives each update's loss. */
int sbiem_closure_train(const float* X, const float* Y, int64_t n, int64_t batch, int64_t steps,
                        double lr, float* params, float* adam_m, float* adam_v, int64_t* adam_t,
                        double* losses);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc): the same
 * Adam updates as sbiem_closure_train, with every array in the caller's
 * device memory and the per-block gradient rows in a fixed workspace that
 * the library holds on each GPU it runs on (about 3.3 MB, kept until the
 * process ends).  It calls no allocator.
 *   X[n][33], Y[n][2]     device, the pairs (read)
 *   params, adam_m, adam_v  device, SBIEM_CLOSURE_PARAMS floats each (updated)
 *   adam_t                host, the update count (updated)
 *   losses                device, [steps] doubles, or NULL
 *   hip_stream            hipStream_t the updates are enqueued on (NULL: the
 *                         null stream); the call returns once they are
 *                         enqueued, the caller synchronises.
 * 1 <= batch <= SBIEM_CLOSURE_TRAIN_MAX_BATCH, else EINVAL.  Calls that
 * overlap on one GPU (two streams, two threads) share its workspace and race;
 * calls in sequence on one stream do not.  Errors: EINVAL, EDEVICE. */
#define SBIEM_CLOSURE_TRAIN_MAX_BATCH 4096
int sbiem_closure_train_noalloc(const float* X, const float* Y, int64_t n, int64_t batch,
                                int64_t steps, double lr, float* params, float* adam_m,
                                float* adam_v, int64_t* adam_t, double* losses, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SBIEM_H */
