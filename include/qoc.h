/*
 * qoc.h -- C ABI of the MI355X library for the multiple-shooting quantum
 * optimal-control objective and its adjoint gradient (arxiv 2407.13950).
 *
 * The calls follow the paper's problem statement (Sec. 3): build the system,
 * set the controls alpha and the window initial states W^1..W^{M-1}, evaluate
 * the penalty objective P (eq. penalty-fcn), evaluate its gradient with respect
 * to alpha (eq. grad-int, exact in the time-discrete setting) and to the real
 * and imaginary parts of every W^m (eq. dP-dW with the factor 2 of App. B).
 *
 * Conventions shared by every call
 *   - Return value: QOC_OK (0) or a negative QOC_E* code; qoc_last_error()
 *     gives a message for the calling thread.  No exception crosses the ABI.
 *   - Ownership: the caller owns every buffer it passes.  Inputs are copied
 *     (asynchronously, on the context's stream) before the call returns or
 *     before any later work on that stream; the library keeps no caller pointer.
 *   - Memory kind: each buffer argument comes with a QOC_HOST or QOC_DEVICE flag.
 *     Device pointers must be HIP device (or managed) allocations of the
 *     context's device.  Host outputs make the call synchronous; device outputs
 *     are written on the context's stream and the call returns without waiting.
 *   - Layouts: complex numbers are interleaved (re, im) doubles.  A state
 *     matrix is N x E, column-major (column c occupies entries c*N .. c*N+N-1),
 *     N = L^q levels, E = 2^q essential states.  Rows enumerate the tensor-
 *     product basis with qubit 0 as the most significant digit; essential state
 *     e sits at the row whose levels are the binary digits of e.
 *   - A context is not thread-safe; use one context per optimisation run or
 *     serialise calls.  Distinct contexts may be used from distinct threads.
 */
#ifndef QOC_H
#define QOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QOC_OK 0
#define QOC_EINVAL (-1)       /* invalid argument, shape or non-finite input      */
#define QOC_ENOMEM (-2)       /* device allocation failed                          */
#define QOC_EDEVICE (-3)      /* HIP runtime or kernel launch error                 */
#define QOC_ENOTCONV (-4)     /* fixed-point solve cannot meet its tolerance        */
#define QOC_EUNSUPPORTED (-5) /* no kernel instance for this (qubits, levels) pair  */
#define QOC_ESTATE (-6)       /* call out of order (e.g. gradient before controls)  */

#define QOC_HOST 0
#define QOC_DEVICE 1

/* Propagation precision.  Reductions (penalty, infidelity) and the gradient
 * accumulation are FP64 in both modes. */
#define QOC_FP64 0   /* states and adjoints propagated in double                 */
#define QOC_FP32 1   /* states and adjoints propagated in float (complex FP32)   */

typedef struct qoc_ctx qoc_ctx;

/* System description (copied by qoc_create).
 *
 * Hamiltonian (Sec. 2, eqs. sys-ham and ctrl-ham):
 *   H(t) = H_d + H_J + sum_j [ 2 pi d_j(t) a_j + conj(2 pi d_j(t)) a_j^+ ],
 *   H_d  = sum_j [ detuning_j l_j + anharmonicity_j/2 l_j (l_j - 1) ]
 *        + sum_{j<q-1} cross_kerr_j l_j l_{j+1}             (rad/ns),
 *   H_J  = sum_{j<q-1} dipole_j (a_{j+1}^+ a_j + a_{j+1} a_j^+)   (rad/ns; the
 *          dipole coupling of eq. sys-ham on the nearest neighbours of the chain),
 * a_j the lowering operator of qubit j truncated to n_levels levels.
 * Controls (eq. dj-ctrl and the B-spline expansion of Sec. 2):
 *   d_j(t) = sum_f exp(i carrier_freq[j*n_carriers+f] t) sum_s (alpha1_jfs + i alpha2_jfs) B_s(t)
 * with quadratic cardinal B-splines B_s(t) = B(t/dtau + 1/2 - s), dtau = T/(n_splines-2),
 * s = 0..n_splines-1 (alpha in GHz, t in ns).  alpha is indexed
 * ((j*n_carriers + f)*2 + part)*n_splines + s, part 0 = alpha1, part 1 = alpha2.
 * Time stepping: n_steps implicit-midpoint steps of dt = T/n_steps with H at the
 * step midpoint (Sec. 5); window m = 1..M covers steps floor((m-1) n_steps/M) ..
 * floor(m n_steps/M) - 1 (equal durations up to one step, Sec. 3).
 * Objective (eqs. mod-infid, penalty-fcn), n replaced by E:
 *   P = |U^M|_F^2/E - |<V, U^M>_F|^2/E^2 + mu/2 sum_{m<M} |U^m(t_m) - W^m|_F^2. */
typedef struct qoc_system_desc {
  int32_t n_qubits;             /* q, 1..6                                            */
  int32_t n_levels;             /* L >= 2 levels per qubit (guard levels included)    */
  const double *detuning;       /* [q] rad/ns, host                                   */
  const double *anharmonicity;  /* [q] rad/ns, host                                   */
  const double *cross_kerr;     /* [q-1] rad/ns, host; NULL = 0                       */
  int32_t n_carriers;           /* carriers per qubit, >= 1                           */
  const double *carrier_freq;   /* [q*n_carriers] rad/ns, host                        */
  int32_t n_splines;            /* B-spline coefficients per carrier, >= 3            */
  double T;                     /* gate duration in ns, > 0                           */
  int64_t n_steps;              /* N_T >= n_windows                                   */
  int32_t n_windows;            /* M >= 1                                             */
  double mu;                    /* penalty coefficient, >= 0                          */
  const double *target;         /* [2*E*E] unitary E x E target, column-major, host   */
  int32_t precision;            /* QOC_FP64 or QOC_FP32                               */
  int32_t fixed_point_iters;    /* 0: derived per evaluation from a contraction bound;
                                   >0: forced count, no bound check.  Counts Jacobi
                                   iterations for odd n_levels and red-black half
                                   sweeps (half an iteration's work each) for even  */
  double solve_tol;             /* per-step fixed-point error target; 0: default      */
  int32_t checkpoint_every;     /* >0: store states every this many steps per window
                                   and re-sync the reverse reconstruction there; 0: none */
  int32_t device;               /* HIP device ordinal                                 */
  const double *dipole;         /* [q-1] rad/ns, host; NULL (or all zero) = no dipole
                                   coupling.  The coupling keeps the digit-sum parity,
                                   so the fixed point treats it Jacobi-style within a
                                   colour; its count bound includes the term.         */
} qoc_system_desc;

/* Read-only facts about a context. */
typedef struct qoc_info {
  int32_t N, E, d;              /* levels, essential states, control count            */
  int32_t n_windows;
  int64_t n_window_doubles;     /* 2*(M-1)*N*E: doubles in W and grad_W               */
  int32_t n_terms;              /* 4 + M: doubles written to `terms`                  */
  int32_t lane_digits;          /* register layout: qubits spread over lanes          */
  int32_t columns_per_wave;
  int64_t device_bytes;         /* device memory held by the context                  */
} qoc_info;

/* Build the system on `desc->device`, allocate its device buffers.  Ownership
 * of *out passes to the caller (release with qoc_destroy).  Errors: QOC_EINVAL
 * (bad sizes, non-finite parameters, non-unitary target), QOC_EUNSUPPORTED,
 * QOC_ENOMEM, QOC_EDEVICE. */
int qoc_create(const qoc_system_desc *desc, qoc_ctx **out);
int qoc_destroy(qoc_ctx *ctx);
int qoc_get_info(const qoc_ctx *ctx, qoc_info *out);

/* Stream for all later work of this context (a hipStream_t; NULL = the null
 * stream).  The caller keeps the stream alive while the context uses it. */
int qoc_set_stream(qoc_ctx *ctx, void *hip_stream);

/* Schedule of the backward (adjoint) sweep, App. B: a choice of how the work is
 * spread over wavefronts, not of what is computed.  Two schedules give the same
 * result up to the rounding order of the per-step inner products.
 *   QOC_BWD_AUTO        the library's rule (the default): the layout's multi-
 *                       wavefront schedule (THREE_WAVES for layouts with one column
 *                       per wavefront, TWO_WAVES for the others) when the sweep has
 *                       at most 1024 (FP32) or 256 (FP64) (window, column group)
 *                       items, else ONE_WAVE;
 *   QOC_BWD_ONE_WAVE    one wavefront per item reconstructs the state and
 *                       propagates the adjoint (in the two halves of the wavefront
 *                       for layouts with two or more columns per wavefront) and
 *                       takes the per-step inner products;
 *   QOC_BWD_TWO_WAVES   two wavefronts per item.  One column per wavefront: the
 *                       state and the adjoint in one wavefront each, the state
 *                       handed over through LDS each step.  Two or more: the solves
 *                       of both halves in one wavefront, the inner products in the
 *                       other, one step behind, from LDS records;
 *   QOC_BWD_THREE_WAVES (one column per wavefront only, else QOC_EUNSUPPORTED)
 *                       state, adjoint and inner products in one wavefront each,
 *                       the inner products one step behind, so that a step costs
 *                       the solving wavefronts one solve.
 * More wavefronts shorten a window's chain of steps (long windows on an otherwise
 * idle GPU); one spends the fewest instructions per item-step.  The setting belongs
 * to the context and is used by its single and batched calls alike, so a batched
 * result still equals the single call's bit for bit.  qoc_get_schedule writes the
 * schedule in force with AUTO resolved.  Errors: QOC_EINVAL (NULL context or
 * output, unknown value). */
#define QOC_BWD_AUTO 0
#define QOC_BWD_ONE_WAVE 1
#define QOC_BWD_TWO_WAVES 2
#define QOC_BWD_THREE_WAVES 3
int qoc_set_schedule(qoc_ctx *ctx, int32_t backward);
int qoc_get_schedule(const qoc_ctx *ctx, int32_t *backward);


/* Controls alpha [d] (eq. dj-ctrl and the B-spline expansion).  Copied. */
int qoc_set_controls(qoc_ctx *ctx, const double *alpha, int64_t d, int32_t where);

/* Window initial states W^1..W^{M-1}: n_doubles = 2*(M-1)*N*E doubles, window-
 * major, each a column-major N x E complex matrix (eqs. sch-ic, con0).  W^0 = I
 * (the essential columns of the identity) is implied.  Copied.  With M = 1 pass
 * n_doubles = 0. */
int qoc_set_window_states(qoc_ctx *ctx, const double *W, int64_t n_doubles, int32_t where);

/* Objective P (eq. penalty-fcn).  P: 1 double; terms (nullable): 4 + M doubles
 *   [J_V(U^M), mu/2 sum |C^m|^2, |U^M|_F^2, Re gamma, Im gamma, |C^1|_F^2 .. |C^{M-1}|_F^2]
 * with C^m = U^m(t_m) - W^m (eq. constraint) and gamma = <V, U^M>_F.  Requires
 * controls and (for M > 1) window states.  QOC_ENOTCONV (host outputs only)
 * when the contraction bound of the implicit solve exceeded its limit. */
int qoc_objective(qoc_ctx *ctx, double *P, double *terms, int32_t where);

/* Objective and gradient in one call (forward sweep, FP64 boundary reductions,
 * backward adjoint sweep; Sec. 3.1).  grad_alpha: d doubles, dP/dalpha
 * (eq. grad-int, exact for the discrete scheme).  grad_W: 2*(M-1)*N*E doubles in
 * the layout of W; the re slot holds dP/dRe W^m, the im slot dP/dIm W^m
 * (= mu (W^m - U^m(t_m)) - 2 Lambda^{m+1}(t_m), App. B).  All outputs share `where`.
 * P, terms and grad_W may be NULL. */
int qoc_gradient(qoc_ctx *ctx, double *P, double *terms, double *grad_alpha, double *grad_W, int32_t where);

/* Adjoint sweep only (Sec. 3.1): dP/dalpha and dP/dW for the controls and
 * window states of the most recent successful qoc_objective call on this
 * context, reusing its forward sweep.  QOC_ESTATE when no objective has been
 * evaluated since the last qoc_set_controls / qoc_set_window_states.  Outputs
 * as in qoc_gradient. */
int qoc_backward(qoc_ctx *ctx, double *grad_alpha, double *grad_W, int32_t where);

/* Roll-out (Sec. 3.2): one propagation over [0, T] from W^0 = I under the
 * current controls.  W_out (nullable): the states at t_1..t_{M-1} in the layout
 * of W; U_out (nullable): U(T), 2*N*E doubles.  Both share `where`. */
int qoc_rollout(qoc_ctx *ctx, double *W_out, double *U_out, int32_t where);

/* ---- Batched evaluation of several contexts (many systems, one launch per phase).
 *
 * A batch object owns the device tables that describe one batched launch
 * sequence; create one per stream that runs batches.  qoc_batch_run evaluates
 * every listed context with its current controls and window states: all
 * (context, window, column group) propagation items of all contexts form one
 * forward launch and one backward launch, ordered longest first; the small FP64
 * kernels run as one launch each over all contexts.  Each context's results
 * stay in its own buffers (read them with qoc_read_results).  All contexts must
 * share the batch's device and one precision and appear at most once; a context
 * must not be used on another stream while the batch runs.  want_grad (nullable:
 * all) selects objective-only (0) or objective+gradient (1) per context.  Each
 * context's stream becomes `hip_stream`.  The call is asynchronous.  Errors:
 * QOC_EINVAL (mixed precision/device, duplicates, more contexts or items than
 * the batch was created for), QOC_ESTATE (a context without controls/states).
 * Results agree with the single-context calls bit for bit (same kernels, same
 * reduction order).  When a call's backward items are of more than one schedule
 * (qoc_set_schedule), those of two and of three wavefronts run on two streams the
 * batch owns, forked from hip_stream and joined back to it within the call's work,
 * so the caller sees ordinary stream order.  max_items bounds the forward items and, separately, the
 * backward items (window x backward column group) of one call. */
typedef struct qoc_batch qoc_batch;
int qoc_batch_create(int32_t device, int32_t max_contexts, int64_t max_items, qoc_batch **out);
int qoc_batch_destroy(qoc_batch *b);
int qoc_batch_run(qoc_batch *b, qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad, void *hip_stream);

/* Per-context outcome of the last qoc_batch_run on b (the fixed-point bound check
 * of Sec. 5's implicit solve, done per context as in qoc_objective): status[i] is
 * QOC_OK or QOC_ENOTCONV for the i-th context of that run, so that one failed
 * evaluation can be reported without failing the others.  qoc_batch_run moves each
 * context's flag into the batch (a later qoc_synchronize on the context no longer
 * reports it).  Waits for the run's work to complete.  n must equal the run's
 * context count.  Valid until the next qoc_batch_run on b.  Errors: QOC_EINVAL
 * (NULL, wrong n), QOC_ESTATE (b has not run). */
int qoc_batch_status(qoc_batch *b, int32_t *status, int32_t n);

/* The batched objective+gradient of n contexts in one call (Sec. 3.1 evaluated for
 * many systems at once): a batch sized for these contexts runs them on the stream of
 * ctxs[0] (every context's stream becomes that stream), as qoc_batch_run does, and the
 * call waits for the work to finish.  want_grad (nullable: all) as in qoc_batch_run.
 * Read each context's results with qoc_read_results.  Returns QOC_ENOTCONV when any
 * context exceeded the fixed-point bound (the message lists them; the others' results
 * are valid), and the errors of qoc_batch_create / qoc_batch_run.  Allocates and frees
 * the batch's tables on every call: callers that evaluate repeatedly keep a qoc_batch. */
int qoc_batch_gradient(qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad);

/* qoc_batch_run without a batch object, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * same batched evaluation of n contexts (same kernels, same item order, results equal to
 * qoc_batch_run's bit for bit), with its tables -- the systems, the propagation item lists
 * and the small-kernel block table -- in a static device array of 4 MiB per GPU that the
 * library holds until the process ends, and in static host memory.  The call allocates
 * nothing (no hipMalloc, hipFree or pinned memory; contexts are created beforehand).
 * Limits and behaviour:
 *   - the tables must fit in 4 MiB (about twenty 4-qubit, 128-window contexts, or the
 *     64-evaluation 2/3/4-qubit mix); a larger call returns QOC_EINVAL before any work;
 *   - every kind of backward item runs on hip_stream, one after another (there are no
 *     streams of a batch to fork onto); each context's stream becomes hip_stream;
 *   - the call waits until its tables are on the device (a copy from the static host
 *     image, ordered after earlier work on hip_stream), then launches asynchronously;
 *   - all calls on one GPU share the array: calls that overlap on one GPU (different
 *     streams, or threads) race; calls in stream order on one stream do not;
 *   - the fixed-point bound flags stay in the contexts (qoc_synchronize reports them).
 * Arguments and other errors as qoc_batch_run. */
int qoc_batch_run_noalloc(qoc_ctx *const *ctxs, int32_t n, const int32_t *want_grad, void *hip_stream);

/* Results of the last evaluation of ctx (single or batched) into caller buffers
 * (all nullable; layouts as in qoc_gradient; gradients only after a gradient
 * evaluation, else QOC_ESTATE).  Device outputs are copied on the context's
 * stream without waiting; host outputs synchronise. */
int qoc_read_results(qoc_ctx *ctx, double *P, double *terms, double *grad_alpha, double *grad_W, int32_t where);

/* Per-phase kernel timing with HIP events recorded on the context's stream.
 * Phases: 0 controls (+ iteration count), 1 forward sweep, 2 boundary reductions,
 * 3 backward (adjoint) sweep, 4 gradient series reduction + B-spline projection,
 * 5 window-state gradient; 6 = whole evaluation.  qoc_enable_timing(ctx, 1)
 * starts a fresh record (up to 4096 evaluations are kept; later ones are not
 * timed); qoc_get_timings synchronises the stream and returns the mean duration
 * per phase over the recorded calls that ran it (qoc_objective runs phases
 * 0-2, qoc_backward 3-5, qoc_gradient 0-5; "whole evaluation" is each call's span). */
typedef struct qoc_timings {
  int32_t n_calls;              /* evaluations recorded                              */
  int32_t n_grad_calls;         /* of which gradient evaluations                     */
  double mean_ms[8];            /* mean kernel time per phase, ms                    */
  int32_t fixed_point_iters;    /* count used by the last evaluation (Jacobi
                                   iterations, or half sweeps for even n_levels)     */
} qoc_timings;
int qoc_enable_timing(qoc_ctx *ctx, int32_t on);
int qoc_get_timings(qoc_ctx *ctx, qoc_timings *out);

/* ---- Optimisation driver: the quadratic-penalty method of Sec. 3 with the
 * settings of Sec. 5 (L-BFGS, box constraints, Tikhonov and energy terms, scaled
 * window states, roll-out-estimate stopping rule), run over the calls above.
 *
 * Variables x = [alpha (d doubles), sigma * W (2*(M-1)*N*E doubles, layout of W)]
 * (W scaled by sigma as in Sec. 5).  The driver minimises
 *   F(x) = P(alpha, W) + gamma_tik/2 |alpha|^2 + gamma_energy * Ee(alpha),
 *   Ee(alpha) = dt * sum_k sum_j |d_j(t_{k+1/2})|^2   (GHz^2 ns, d_j as in eq. dj-ctrl),
 * subject to |alpha_i| <= amp_bound / (sqrt(2) * n_carriers): then
 * |d_j(t)| <= amp_bound for all t (the B-splines sum to one).
 * Iteration (both sides of the parity tests implement exactly this):
 *   active set: alpha_i at a bound with the gradient pointing outwards;
 *   gr = gradient with active entries zeroed;
 *   p = -H gr by the L-BFGS two-loop recursion over the last `memory` pairs
 *     (s, y) with H0 = (s.y / y.y) I of the newest pair; active entries of p
 *     zeroed; p = -gr when the history is empty or p is not a descent direction
 *     (the history is then cleared);
 *   backtracking from t0 = 1 (t0 = 1 / max(1, |gr|_2) without history), halving
 *     up to 30 times: x_t = clip(x + t p), accepted when
 *     F(x_t) <= F(x) + 1e-4 * g.(x_t - x);
 *   the pair (s, y) = (x_t - x, g_t - g) is kept when s.y > 1e-12 |s| |y|.
 * Stops when the roll-out infidelity estimate (eq. rollout-infid-est, with
 * n = E) of the current iterate is below tol_estimate, when |gr|_inf <
 * tol_grad, or when no step is accepted.  Trial points cost one objective
 * evaluation; an accepted point adds one adjoint sweep (qoc_backward).  All
 * vectors live in device memory of the context's device. */
typedef struct qoc_opt qoc_opt;
typedef struct qoc_opt_desc {
  double sigma;                 /* window-state scale, > 0 (Sec. 5: 0.05 .. 0.15)    */
  double gamma_tik;             /* Tikhonov coefficient, >= 0 (Sec. 5: 1e-3 / d)     */
  double gamma_energy;          /* energy coefficient, >= 0 (Sec. 5: 1e-3)           */
  double amp_bound;             /* pulse amplitude bound in GHz, > 0 (Sec. 5: 0.025) */
  int32_t memory;               /* L-BFGS pairs kept, 1..64                          */
  double tol_estimate;          /* stop below this roll-out estimate (Sec. 5: 1e-3)  */
  double tol_grad;              /* stop below this |gr|_inf (0: never)               */
} qoc_opt_desc;

typedef struct qoc_opt_status {
  int32_t iterations;           /* accepted steps so far                             */
  int32_t evaluations;          /* objective evaluations (trial points)              */
  int32_t backward_sweeps;      /* adjoint sweeps                                    */
  int32_t stop;                 /* 0 running, 1 estimate below tol, 2 gradient below
                                   tol, 3 no step accepted                           */
  double F, P, J, penalty, energy, tikhonov;   /* at the current iterate             */
  double estimate;              /* roll-out infidelity estimate at the iterate       */
  double grad_inf;              /* |gr|_inf at the iterate                           */
  double last_step;             /* accepted step length t of the last iteration      */
} qoc_opt_status;

/* Start an optimisation on ctx (which then belongs to it until qoc_opt_destroy;
 * the context's stream is used).  alpha0: d doubles (clipped to the box); W0:
 * 2*(M-1)*N*E doubles, unscaled (Sec. 5 starts from the roll-out states;
 * NULL = roll out alpha0 on the GPU); both on `where`.  Evaluates F and its
 * gradient at the start point.  Errors: QOC_EINVAL, QOC_ENOMEM, QOC_ENOTCONV. */
int qoc_opt_create(qoc_ctx *ctx, const qoc_opt_desc *desc, const double *alpha0, const double *W0, int32_t where,
                   qoc_opt **out);
int qoc_opt_destroy(qoc_opt *opt);
/* Up to n_iters iterations (fewer when a stop condition holds); status
 * (nullable) describes the current iterate afterwards. */
int qoc_opt_run(qoc_opt *opt, int32_t n_iters, qoc_opt_status *status);
/* The current iterate: alpha (d doubles) and W (unscaled, 2*(M-1)*N*E doubles);
 * both nullable, on `where`. */
int qoc_opt_get(qoc_opt *opt, double *alpha, double *W, int32_t where);

/* Block until this context's queued work is done; returns QOC_ENOTCONV if a
 * previous evaluation flagged a fixed-point bound violation (then clears it). */
int qoc_synchronize(qoc_ctx *ctx);

/* Message for the last failing call on this thread (never NULL). */
const char *qoc_last_error(void);
const char *qoc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* QOC_H */
