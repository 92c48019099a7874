/*
 * lw.h -- C ABI of the MI355X (gfx950) Lienard-Wiechert library (liblw.so).
 *
 * The library evaluates, for every (observation point, point charge) pair,
 * the retarded time of Eq. (ret_t), t' = t - R(t')/c, on the charge's
 * trajectory, then the Lienard-Wiechert potentials of Eqs. (V), (A) and the
 * fields of Eqs. (E) / (ECoulomb) / (Eradiation) and (B), and sums them over
 * charges (arXiv 2107.12437, Secs. 2.1-2.2).  It also runs the
 * self-consistent Lorentz-oscillator loop of Algorithm 1 (Secs. 2.3, 3.2):
 * dipoles driven by the retarded fields of the other dipoles' charges,
 * integrated with RK4 from a device-resident history.
 *
 * Conventions
 *   - SI units throughout.  Physical constants are CODATA 2018.
 *   - "d_" arguments are device pointers (HIP device memory), "h_" arguments
 *     are host pointers.  The caller owns every buffer it passes; the library
 *     never frees or retains caller memory past the call (it keeps only its
 *     own workspace, owned by the context).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every call enqueues
 *     its work on that stream and returns without waiting, except where a
 *     function says it synchronises.
 *   - Errors are returned as lw_status codes; no C++ exception crosses the
 *     ABI.  lw_last_error() gives a message for the last failure on the
 *     calling thread.  Argument errors are detected on the host before any
 *     launch; errors found by a kernel (a dipole charge above the speed limit,
 *     a non-finite state, history overrun) are latched in the context and
 *     returned by lw_sync_status().
 *   - A context may be used from one host thread at a time.  Calls that share a
 *     context must run on one stream (they share the context's workspace).
 */
#ifndef LW_H
#define LW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------ */
/* status                                                                    */
/* ------------------------------------------------------------------------ */
typedef int32_t lw_status;
enum {
    LW_OK = 0,
    LW_E_INVALID = 1,       /* bad argument (size, pointer, non-finite or unnormalised input)   */
    LW_E_SUPERLUMINAL = 2,  /* a trajectory reaches |v| >= c within the requested times         */
    LW_E_DT_TOO_LARGE = 3,  /* c*dt >= the smallest dipole separation under LW_DT_STRICT
                               (Sec. 3.2: radiation must not reach another dipole in one step) */
    LW_E_VELOCITY = 4,      /* a dipole charge exceeded max_vel (Sec. 3.2, default c/100)      */
    LW_E_NOCONV = 5,        /* retarded-time solve hit max_iter (fields: per-point flag bit 2)  */
    LW_E_HIP = 6,           /* a HIP runtime call failed                                        */
    LW_E_NOMEM = 7,         /* device or host allocation failed                                 */
    LW_E_NONFINITE = 8,     /* an oscillator state became NaN or Inf                            */
    LW_E_HISTORY = 9,       /* a retarded time fell outside the stored history window           */
    LW_E_STATE = 10         /* a resumed run's state was written for other dipoles or depth     */
};

/* Message for the last failed call on this thread ("" if none). */
const char *lw_last_error(void);

/* ------------------------------------------------------------------------ */
/* context                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct lw_ctx lw_ctx;

/* Creates a context on HIP device `device` (made current for the calls on the
 * context).  The context owns device workspace, pinned staging memory and the
 * tuning table; all are released by lw_destroy. */
lw_status lw_create(lw_ctx **out, int32_t device);
lw_status lw_destroy(lw_ctx *ctx);

/* Waits for `stream`, then returns (and clears) the first error latched by a
 * kernel of this context since the previous call; LW_OK if none. */
lw_status lw_sync_status(lw_ctx *ctx, void *stream);

/* Launch-shape tuning of lw_fields (on by default; LW_AUTOTUNE=0 in the
 * environment turns it off at lw_create).  While on, the first lw_fields call
 * of each shape class (precision, field kind, charge and time counts, point
 * count rounded up to a power of two, the set of trajectory kinds present, the
 * output groups) times every candidate workgroup size and
 * times-per-workgroup on its own inputs and keeps the fastest: that call
 * synchronises `stream` and writes d_out several times, the last time with the
 * result.  Choices persist in the context, and across processes in the file
 * named by LW_TUNE_CACHE when set. */
lw_status lw_set_autotune(lw_ctx *ctx, int32_t enable);

/* ------------------------------------------------------------------------ */
/* point charges with prescribed trajectories (Sec. 3.1)                     */
/* ------------------------------------------------------------------------ */
enum {
    LW_STATIONARY = 0,       /* r(t) = c0                                                      */
    LW_UNIFORM_VELOCITY = 1, /* r(t) = c0 + v t                                                */
    LW_LINEAR_OSC = 2,       /* r(t) = c0 + amp cos(omega t + phase) e1                        */
    LW_CIRCULAR = 3,         /* r(t) = c0 + amp (cos(omega t + phase) e1 + sin(... ) e2), e1 . e2 = 0 */
    LW_ACCEL = 4             /* r(t) = c0 for t < 0, c0 + accel t^2 e1 / 2 for t >= 0          */
};

/* One point charge: its value q and parametric x(t), y(t), z(t) with exact
 * derivatives (the paper's Charge subclasses, Sec. 3.1).  e1 and e2 must be
 * unit vectors where the kind uses them.  Layout: 8-byte aligned, 144 bytes. */
typedef struct {
    int32_t kind;
    int32_t pad_;
    double q;          /* C            */
    double c0[3];      /* m            */
    double e1[3];
    double e2[3];
    double amp;        /* m            */
    double omega;      /* rad/s        */
    double phase;      /* rad          */
    double accel;      /* m/s^2        */
    double v[3];       /* m/s          */
} lw_traj;

enum { LW_FP64 = 0, LW_MIXED = 1 };
enum { LW_FIELD_TOTAL = 0, LW_FIELD_COULOMB = 1, LW_FIELD_RADIATION = 2 };
enum { LW_FLAG_MASKED = 1u, LW_FLAG_NOCONV = 2u };
/* Output components (lw_opts.outputs): rows of the output in this order. */
enum { LW_OUT_PHI = 1, LW_OUT_A = 2, LW_OUT_E = 4, LW_OUT_B = 8, LW_OUT_S = 16 };

typedef struct {
    int32_t precision;   /* LW_FP64: FP64 throughout.  LW_MIXED: FP64 retarded time and
                            kinematics, FP32 field expressions summed over charges in FP64,
                            FP32 outputs.                                                   */
    int32_t field_kind;  /* E and B as the total field of Eq. (E) or its Coulomb or
                            radiation part (Eqs. (ECoulomb), (Eradiation)); Phi and A
                            are unaffected                                                  */
    int32_t max_iter;    /* cap on retarded-time iterations per pair (0: 100)               */
    int32_t outputs;     /* LW_OUT_* bits selecting the output rows, in the order Phi (1 row),
                            A (3), E (3), B (3), S (3); S = E x B / mu0 is the Poynting
                            vector (W/m^2) of the summed fields (Sec. 2.2).  0: Phi | A |
                            E | B, the 10 rows of Eqs. (V), (A), (E), (B)                   */
    double mask_radius;  /* (point, time) with a retarded distance below this to any charge
                            gets NaN outputs and LW_FLAG_MASKED (m; < 0: 1e-10)             */
} lw_opts;

/* Potentials and fields of n_charges point charges at n_pts points and n_times
 * times (Secs. 2.1-2.2; the paper's calculate_V / calculate_A / calculate_E /
 * calculate_B fused over outputs and times).
 *   h_charges  host array of n_charges trajectories (n_charges >= 1)
 *   d_pts      device FP64, SoA [3][n_pts]: x[], then y[], then z[]
 *   h_times    host FP64 [n_times] observation times (s)
 *   d_out      device, SoA [n_times][n_rows][n_pts]: the rows opts->outputs
 *              selects, in the order Phi; Ax, Ay, Az; Ex, Ey, Ez; Bx, By, Bz;
 *              Sx, Sy, Sz (V, V s/m, V/m, T, W/m^2); by default the first 10;
 *              FP64 for LW_FP64, FP32 for LW_MIXED (S is formed from the FP64
 *              sums of E and B and rounded once)
 *   d_flags    device uint32 [n_pts] or NULL: LW_FLAG_* OR-ed over times
 * Returns LW_E_SUPERLUMINAL if a charge moves at >= c at or before a requested
 * time.  n_pts == 0 or n_times == 0 is a no-op.  Asynchronous. */
lw_status lw_fields(lw_ctx *ctx, const lw_traj *h_charges, int32_t n_charges, const double *d_pts,
                    int64_t n_pts, const double *h_times, int32_t n_times, const lw_opts *opts,
                    void *d_out, uint32_t *d_flags, void *stream);

/* Largest scratch of lw_fields_noalloc, in bytes: the charges (144 bytes each), the
 * times (8 bytes each) and one 272-byte record per (time, charge), each part
 * rounded up to 256 bytes.  For example 64 times x 238 charges fit. */
#define LW_NOALLOC_SCRATCH_BYTES (4u << 20)

/* lw_fields without any allocation, for callers that cannot allocate device or
 * pinned host memory during the call (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, outputs
 * and errors as lw_fields, with these differences:
 *   - The charges, times and per-(time, charge) records go to a fixed scratch
 *     array of LW_NOALLOC_SCRATCH_BYTES on each GPU (static device memory of
 *     the library, held until the process ends), not to the context's
 *     workspace.  A call that needs more returns LW_E_INVALID before any work.
 *   - h_charges and h_times are copied from pageable host memory on `stream`;
 *     the call returns once the copies have read them.
 *   - The launch shape is the context's default (no tuning, no timing).
 * Every call on one GPU shares that GPU's scratch: calls that may overlap on
 * one GPU (different streams, or threads without ordering) race and give wrong
 * results; calls on one stream are ordered and safe.  The context is used only
 * for its device and launch shape.  Asynchronous. */
lw_status lw_fields_noalloc(lw_ctx *ctx, const lw_traj *h_charges, int32_t n_charges, const double *d_pts,
                            int64_t n_pts, const double *h_times, int32_t n_times, const lw_opts *opts,
                            void *d_out, uint32_t *d_flags, void *stream);

/* Vector-Jacobian product of lw_fields with respect to the trajectory
 * parameters: d_grad[c][k] = sum over points p, times t and outputs j of
 * d_cot[t][j][p] * d out[t][j][p] / d theta_{c,k}, for the parameters
 *   k = 0 q, 1..3 c0, 4 amp, 5 omega, 6 phase, 7 accel, 8..10 v
 * of charge c (those a kind does not use get 0).  The derivative follows the
 * retarded time through the implicit-function theorem on Eq. (ret_t) and the
 * trajectory's own derivatives (the jerk enters through d a / d t').
 *   d_cot   device, [n_times][n_rows][n_pts], FP32 if opts->precision is
 *           LW_MIXED, FP64 otherwise: the layout of lw_fields' output for the
 *           same opts->outputs, which may not include LW_OUT_S (LW_E_INVALID);
 *           (point, time) entries with a non-finite cotangent, and pairs
 *           closer than the mask radius, contribute nothing
 *   d_grad  device FP64 [n_charges][11], overwritten
 * The forward quantities are recomputed in FP64 whatever the precision.
 * With opts->outputs = LW_OUT_E (objectives of E alone, such as |E|^2) the
 * kernel reads and reverses only E, which is faster; the gradient is the same
 * bits as with all outputs and zero cotangents for Phi, A and B.
 * Sums run in a fixed order: the result is bitwise reproducible.  Asynchronous. */
lw_status lw_fields_vjp(lw_ctx *ctx, const lw_traj *h_charges, int32_t n_charges, const double *d_pts,
                        int64_t n_pts, const double *h_times, int32_t n_times, const lw_opts *opts,
                        const void *d_cot, double *d_grad, void *stream);

/* Debugging: a histogram of the retarded-time solves (Eq. (ret_t)) of lw_fields
 * calls, by the iterations each (point, time, charge) pair's solve took.
 * Bins (uint64 counts):
 *   0..30                 that many iterations (0: the closed forms of the
 *                         stationary and uniformly moving charges; the mixed
 *                         path counts its FP32 steps and its FP64 step)
 *   31                    31 or more
 *   LW_ITER_BIN_FALLBACK  mixed-path solves that fell back to the safeguarded
 *                         FP64 solver (counted here instead of 0..31)
 *   LW_ITER_BIN_NOCONV    solves flagged as not converged (also counted in
 *                         their iteration bin)
 * lw_set_iteration_histogram(ctx, 1) allocates and clears the context's
 * histogram; while it is on, lw_fields launches a counting instance of the
 * grid kernel (one time per lane, 256 lanes, no launch tuning; same outputs,
 * slower) that adds every pair of the call.  0 turns counting off and keeps
 * the counts.  lw_fields_noalloc and lw_fields_vjp never count.
 * lw_iteration_histogram synchronises `stream`, copies the n_bins counts to
 * h_bins (n_bins <= LW_ITER_BINS) and, if reset is nonzero, clears them.
 * LW_E_INVALID if counting was never turned on for the context. */
enum { LW_ITER_BINS = 34, LW_ITER_BIN_FALLBACK = 32, LW_ITER_BIN_NOCONV = 33 };
lw_status lw_set_iteration_histogram(lw_ctx *ctx, int32_t enable);
lw_status lw_iteration_histogram(lw_ctx *ctx, uint64_t *h_bins, int32_t n_bins, int32_t reset, void *stream);

/* ------------------------------------------------------------------------ */
/* Lorentz oscillators (Secs. 2.3, 3.2; Algorithm 1)                         */
/* ------------------------------------------------------------------------ */

/* One oscillator (the paper's Dipole): two charges +q (mass m1) and -q (mass
 * m2) about the centre of mass R(t), displaced along the unit axis p by
 * r_dip = (d/q) p (Eqs. (r_1), (r_2)); d0 is the signed initial moment along p
 * (C m).  The centre of mass is fixed at `origin`, or moves (Sec. 4.3, moving
 * dipoles) as R(t) = origin + motion_amp cos(motion_omega t + motion_phase)
 * for all t, before t = 0 as well; its drive field is taken at R(t) and its
 * charges ride on R(t).  Layout: 128 bytes. */
typedef struct {
    double origin[3];
    double axis[3];
    double omega0;     /* rad/s */
    double q;          /* C, > 0 */
    double m1, m2;     /* kg    */
    double d0;         /* C m   */
    double motion_amp[3];   /* m; all 0: fixed origin                    */
    double motion_omega;    /* rad/s, nonzero when motion_amp is;
                               motion_omega |motion_amp| < c / 10         */
    double motion_phase;    /* rad                                        */
} lw_dipole;

enum { LW_DT_STRICT = 0, LW_DT_EXTRAPOLATE = 1 };

typedef struct {
    int32_t precision;   /* LW_FP64: FP64 throughout.  LW_MIXED: each source dipole's field
                            at a target in FP32, its two charges' nearly cancelling
                            monopole terms differenced without cancellation; retarded
                            times, state and sums stay FP64 (lw_dipole_run_vjp: FP64
                            only)                                                         */
    int32_t dt_policy;   /* LW_DT_STRICT: require c*dt < smallest separation (Sec. 3.2).
                            LW_DT_EXTRAPOLATE: allow it; a source read beyond its newest
                            stored step is a second-order Taylor step from that sample     */
    int64_t out_stride;  /* outputs every out_stride steps (>= 1)                            */
    double max_vel;      /* charge speed limit, m/s (<= 0: c/100)                            */
    int32_t ring_depth;  /* stored steps per dipole (0: automatic, power of two)             */
    int32_t stepped_min_n; /* instances of at least this many dipoles (or whose history does
                              not fit in LDS) advance one launch per step with one workgroup
                              per dipole; smaller ones run whole in one workgroup
                              (0: 16; LW_STEPPED_TUNE: the fastest threshold for the run's
                              shape class, timed on trial runs of its dipoles at the first
                              call (which then synchronises the stream) and cached like the
                              grid shapes; other negative values: only when the history
                              does not fit)                                              */
} lw_run_opts;

enum { LW_STEPPED_TUNE = -2 };

/* Runs `steps` RK4 steps of Eq. (LO_equation) for n_inst independent
 * instances; instance k holds dipoles [h_inst_off[k], h_inst_off[k+1]) of
 * h_dip.  Each dipole is driven by the component along its axis of the total
 * field at its origin of the other dipoles' charges in its instance, read at
 * their retarded times from the stored history (linear interpolation between
 * steps; static at d0 before t = 0).  All dipoles advance together.  The
 * paper's run() followed by its extraction of the collective decay rates and
 * frequency shift (Secs. 2.4, 3.2).
 * Outputs (device FP64, [steps/out_stride + 1][n_dip], row k = step k*stride):
 *   d_moment  moment d along the axis (required)
 *   d_dot     d d/dt                    (nullable)
 *   d_energy  energy of Eq. (dipoleE)   (nullable)
 *   d_drive   drive field E_d           (nullable)
 *   d_wabs    work done on the dipole by its drive field since t = 0, the
 *             integral of E_d d_dot (nullable)
 *   d_wrad    energy radiated since t = 0, the integral of the Larmor power
 *             |d_ddot|^2 / (6 pi eps0 c^3) (nullable)
 *   (both by the trapezoid rule over steps; the sum over the dipoles of an
 *   instance of energy - wabs + wrad is the conserved W_total of Sec. 2.5)
 * and, for two-dipole instances (host, nullable; when either is given the call
 * synchronises `stream`, returns the run's latched errors as lw_sync_status
 * does, and fits the moments copied back as lw_pair_modes does, with the first
 * dipole's omega0 as reference and a transient of max(2000 steps, three light
 * times of the separation) skipped):
 *   h_gamma   [n_inst][2]: gamma+ and gamma-, the energy decay rates of the
 *             in-phase and anti-phase modes (s^-1)
 *   h_domega  [n_inst]: delta_omega = (omega+ - omega-)/2 (rad/s)
 *   NaN for other instances, for a mode the run does not excite (delta_omega
 *   then falls back as in lw_pair_modes) and for runs too short to fit.
 * Small instances run concurrently with the stepped ones on a second stream of
 * the context that is joined back into `stream` before the call's work ends.
 * Asynchronous unless h_gamma or h_domega is given: speed-limit, non-finite
 * and history errors are reported by lw_sync_status(). */
lw_status lw_dipole_run(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                        int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts,
                        double *d_moment, double *d_dot, double *d_energy, double *d_drive,
                        double *d_wabs, double *d_wrad, double *h_gamma, double *h_domega, void *stream);

/* Run state of an oscillator run, for checkpoints and resumed runs: the step
 * count, every dipole's history ring (the stored (d, d_dot, d_ddot) of the
 * last `ring` steps), E_d at the last step and the two energy sums, FP64 on
 * the device.  *n_doubles receives its size in doubles for these arguments
 * (the history depth follows from the geometry, dt and opts->ring_depth, as in
 * lw_dipole_run).  Host only; the same argument checks as lw_dipole_run. */
lw_status lw_dipole_state_size(const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off, int32_t n_inst,
                               double dt, const lw_run_opts *opts, int64_t *n_doubles);

/* lw_dipole_run with a run state (Algorithm 1 continued across calls):
 *   d_state  device FP64, n_state doubles, at least lw_dipole_state_size's
 *            (LW_E_INVALID otherwise); owned by the caller.
 *   resume   0: the run starts at t = 0, as lw_dipole_run.  Nonzero: it
 *            continues the run whose state d_state holds, at that state's step
 *            n0: output row 0 is the state at n0 and row k the state at
 *            n0 + k out_stride, and `steps` more steps are taken.
 * Either way d_state holds the run's state after its last step when the call's
 * work ends, so a run split into calls gives the outputs of one call.  The
 * dipoles, instances, dt and options must be those the state was written
 * with; a state of another size or depth is reported as LW_E_STATE by
 * lw_sync_status().  Asynchronous, like lw_dipole_run. */
lw_status lw_dipole_run_state(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                              int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts,
                              double *d_moment, double *d_dot, double *d_energy, double *d_drive,
                              double *d_wabs, double *d_wrad, double *d_state, int64_t n_state, int32_t resume,
                              void *stream);

/* Gradient of a detector objective with respect to the oscillator positions,
 * by a backward-in-time discrete adjoint of the run.  The run is that of
 * lw_dipole_run (same arguments; out_stride is ignored); the objective is
 *   J = (1/n_snap) sum_k sum_p |E(r_p, t_k)|^2
 * with E the total field (Eq. (E)) of every oscillator charge of every instance
 * at detector point r_p and time t_k, read from the stored history at its
 * retarded time.  The adjoint transposes each RK4 step and the delay coupling:
 * every drive pair's retarded time is differentiated by the implicit-function
 * theorem against the interpolated history, and the cotangents owed to earlier
 * source times accumulate in an adjoint history read back as the sweep reaches
 * them.
 *   ckpt_every   0 (or >= steps): the forward history is kept whole in device
 *                memory (24 bytes per dipole per step).  K > 0: checkpointed:
 *                the forward run keeps its run state (as lw_dipole_run_state)
 *                every K steps, and the backward sweep recomputes each segment
 *                of K steps from its state, last segment first, so the device
 *                holds the states and two windows of K steps plus the
 *                retarded look-back instead of the whole run.  A second stream
 *                of the context recomputes the next segment while the current
 *                one is swept, so the extra forward run mostly overlaps.  The
 *                result equals the whole-history one to rounding.  Negative:
 *                LW_E_INVALID; so is a K whose window would exceed 2^26 steps.
 * Moving origins and LW_MIXED are rejected (LW_E_INVALID).
 *   d_det_pts    device FP64 SoA [3][n_det]
 *   h_snap_times host FP64 [n_snap], each in [0, steps dt]
 *   d_grad_pos   device FP64 [n_dip][3]: dJ/d origin, overwritten
 *   h_J          host: J
 * Instances may hold at most 1024 dipoles.  Synchronises `stream` and returns
 * the run's latched errors (as lw_sync_status).  The position sums use device
 * atomics: results agree to rounding between runs, not bitwise. */
lw_status lw_dipole_run_vjp(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                            int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts, const double *d_det_pts,
                            int64_t n_det, const double *h_snap_times, int32_t n_snap, int32_t ckpt_every,
                            double *d_grad_pos, double *h_J, void *stream);

/* Collective decay rates and frequency shift of two-dipole instances from a
 * finished run's moments (Sec. 2.4, Eq. (KE)): the sum and difference of the
 * two moments are the in-phase and anti-phase normal modes; each is fitted,
 * after skipping `skip_steps` steps, by order-2 linear prediction with a lag of
 * a quarter period of omega_ref, giving its complex frequency.
 *   h_moment  host FP64 [n_rows][n_dip] (the d_moment output copied back)
 *   h_out     host FP64 [n_inst][5]: gamma+, gamma-, omega+, omega-,
 *             delta_omega = (omega+ - omega-)/2.  A mode whose RMS is below
 *             1e-6 of the other's is NaN, and delta_omega then falls back to
 *             omega+ - omega_ref (or omega_ref - omega-).  Instances that do
 *             not hold exactly two dipoles get NaN.
 * Host only; synchronous. */
lw_status lw_pair_modes(const double *h_moment, int64_t n_rows, int32_t n_dip, const int32_t *h_inst_off,
                        int32_t n_inst, double dt, int64_t out_stride, const double *h_omega_ref,
                        const int64_t *h_skip_steps, double *h_out);

/* Free-space energy decay rate gamma_0 = q^2 omega0^2 / (6 pi eps0 c^3 m)
 * (Sec. 2.3) of an oscillator with reduced mass m. */
double lw_gamma0(double q, double m, double omega0);

/* Coupling of two identical dipoles (axes p1, p2, resonance omega0) at
 * separation R from the free-space dyadic Green's function of App. A,
 * G = k^2 e^{ikR}/(4 pi R) [(1 + (ikR - 1)/(kR)^2) I + (3 - 3ikR - (kR)^2)/(kR)^2 R^R^]
 * at k = omega0/c, with gamma_0 from Im G(r, r) = k^3/(6 pi):
 *   out[0] = delta_12 / gamma_0 = -Re(p1.G.p2) / (2 Im G(r, r))   (Eq. (qed_delta))
 *   out[1] = gamma_12 / gamma_0 =  Im(p1.G.p2) / Im G(r, r)        (Eq. (qed_gamma_ab))
 * so that gamma_+- = gamma_0 (1 +- out[1]) (Eq. (gamma_super_sub)).
 * R, p1, p2: host, 3 doubles (p1, p2 unit).  Host only; LW_E_INVALID on bad
 * arguments. */
lw_status lw_gf_pair(const double *R, const double *p1, const double *p2, double omega0, double *out);

/* Exact classical normal modes of two identical oscillators (charge q, reduced
 * mass m, resonance omega0, common unit axis p) at separation R, without the
 * Markov approximation of the Green's-function rates: the roots omega near
 * omega0 of Eq. (LO_equation) with the other dipole's field as drive,
 *   omega0^2 - omega^2 - i gamma_0 omega = +-(q^2 / (m eps0)) p.G(omega).p,
 * for the in-phase (+) and antiphase (-) modes, by complex Newton from
 * omega0 - i gamma_0/2.  out[0] = gamma_+ = -2 Im omega_+, out[1] = gamma_-,
 * out[2] = Re omega_+, out[3] = Re omega_-, out[4] = (Re omega_+ - Re omega_-)/2.
 * Host only; LW_E_INVALID on bad arguments, LW_E_NOCONV if Newton fails. */
lw_status lw_exact_modes(const double *R, const double *p, double q, double m, double omega0, double *out);

#ifdef __cplusplus
}
#endif
#endif /* LW_H */
