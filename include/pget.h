/*
 * pget.h — C ABI of the MI355X (gfx950) library for the Levenberg-Marquardt
 * reconstruction of emission and attenuation maps in passive gamma emission
 * tomography (arXiv 2604.26745, "Robust Model-Based Iteration for Passive
 * Gamma Emission Tomography").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Maps (emission f, the paper's lambda; attenuation mu) are N x N,
 *    row-major, pixel (r, c) centred at (c - (N-1)/2, r - (N-1)/2), pixel
 *    size 1.  Sinograms are n_angles x n_bins, row-major.
 *  - All array arguments are DEVICE pointers (hipMalloc'd or torch CUDA
 *    tensors), contiguous, 4-byte aligned, FP32 (IEEE binary32).  Inputs must
 *    not alias outputs unless stated.
 *  - Every call is asynchronous on `stream`; argument errors are returned
 *    synchronously and nothing is enqueued.  Device-side failures of the
 *    solver are reported in the report's `status` after the stream syncs.
 *  - The caller owns every data buffer and the workspace; the library owns
 *    only the plan's small tables (angle table, collimator taps, ray clip
 *    bounds).  `ws` must be at least pget_workspace_bytes(plan, op, batch)
 *    bytes of device memory, 256-byte aligned; its contents on entry are
 *    ignored and on exit are unspecified.
 *  - A plan may be used from several threads only with distinct workspaces
 *    and streams.
 *  - No entry point throws; every failure is a negative pget_status.
 */
#ifndef PGET_H
#define PGET_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PGET_OK = 0,
    PGET_ERR_INVALID_ARG = -1, /* bad pointer, size or parameter            */
    PGET_ERR_HIP = -2,         /* a HIP runtime call failed                  */
    PGET_ERR_WORKSPACE = -3,   /* workspace missing or too small             */
    PGET_ERR_NONFINITE = -4,   /* NaN/Inf met in the solver (report status)  */
    PGET_ERR_UNSUPPORTED = -5  /* geometry outside what the kernels handle   */
} pget_status;

/*
 * Storage of the Jacobian's two large internal streams: the per-sample
 * weights written by the linearisation and the map pair (search direction)
 * staged for J v.  PGET_FP32 keeps them in binary32; PGET_BF16 rounds them
 * to bfloat16 (round to nearest even), halving their memory traffic and the
 * LDS footprint of J v.  The ray march that gives the forward map, the
 * residual and the objective always reads the maps in FP32, so with
 * PGET_BF16 the solver runs an inexact-Jacobian LM (gradient, CG operator and
 * predicted decrease carry the rounding) whose gain ratio still uses the
 * exact objective.  Every sum is accumulated in FP32 and every reduction of
 * the solver in FP64 either way; maps and sinograms at the API are FP32.
 */
typedef enum { PGET_FP32 = 0, PGET_BF16 = 1 } pget_storage;

/*
 * Parallel-beam geometry of one slice (Sec. 2.1, eq. fwd_model and its
 * discrete form eq. d_fwd_model).  Angle a is theta_a = angle0 + a*arc/n_angles;
 * omega = (cos theta, sin theta) points toward the detector, bin j sits at
 * s_j = (j - (n_bins-1)/2)*bin_size along omega_perp = (-sin, cos), and each
 * ray is sampled at t_i = (i - (n_t-1)/2)*step, n_t = 2*ceil((N/sqrt2+1)/step).
 * The maps are sampled bilinearly (zero outside the grid), a sample is
 * attenuated by half its own attenuation plus all samples nearer the detector,
 * the ray sum is weighted by step, and the collimator response r_{m,n} is a
 * Gaussian across bins with standard deviation psf_sigma bins, truncated at
 * psf_radius bins (negative: ceil(3 sigma)), normalised, zero-padded.
 * atten_scale is the constant correction c of eq. d_fwd_model.
 */
typedef struct {
    int32_t n;          /* N, 2 <= N <= 512                                  */
    int32_t n_angles;   /* 1 .. 1024                                         */
    int32_t n_bins;     /* 1 .. 8192                                         */
    int32_t psf_radius; /* taps per side; < 0 -> ceil(3*psf_sigma); <= 32   */
    double angle0;      /* radians                                           */
    double arc;         /* radians, e.g. 2*pi for a full turn                */
    double bin_size;    /* >= 1, pixels (at most 3x3 gather candidates)     */
    double step;        /* >= 1, pixels                                      */
    double psf_sigma;   /* >= 0, bins; 0 = no blur                           */
    double atten_scale; /* > 0                                               */
} pget_geometry;

typedef struct pget_plan pget_plan;

/* Operation codes for pget_workspace_bytes. */
enum { PGET_OP_FORWARD = 0, PGET_OP_JVP = 1, PGET_OP_VJP = 2, PGET_OP_LM = 3 };

/*
 * Build the geometry tables of one slice shape on the current HIP device.
 * *out receives an opaque plan to release with pget_plan_destroy.
 * The plan holds, per ray, the range of its samples inside the support and
 * their offset in the compacted per-sample arrays of a workspace (a ray's
 * in-support samples contiguous; with a full turn and an even angle count
 * the mirror ray right after it).
 * Errors: INVALID_ARG (null pointer, size out of range), UNSUPPORTED
 * (storage other than FP32 / BF16; more than 2^29 in-support samples per
 * slice, since the adjoint forms 32-bit byte offsets into a slice's weights;
 * detector rows that overflow the kernels' LDS rows; a device index beyond
 * the library's per-device tables), HIP (device allocation of the tables
 * failed).
 */
pget_status pget_plan_create(const pget_geometry* geom, pget_storage storage, pget_plan** out);
void pget_plan_destroy(pget_plan* plan);

/* Derived sizes: samples per ray n_t, the collimator half width, and the
 * number of lattice samples (angle, bin, sample) whose bilinear footprint
 * meets the map -- the work unit of one operator pass. */
int32_t pget_plan_n_samples(const pget_plan* plan);
int32_t pget_plan_psf_half_width(const pget_plan* plan);
int64_t pget_plan_support_samples(const pget_plan* plan);

/*
 * Band staging for maps whose bordered pair does not fit in LDS (FP32 above
 * 138^2, BF16 above about 196^2 at 1.5 bins per pixel; up to 8 bands of
 * rows).  Off by default: the Jacobian product reads such a map from a
 * bordered copy in HBM in one pass.  On, it walks the map in the plan's
 * bands of rows: blocks of at least 6 angle slots (large batches) stage each
 * band in LDS, smaller ones read the same bands from the HBM copy; each
 * ray's per-band sums are added in band order, so every launch shape gives
 * the same bits.  It pays for plans solved in large batches and costs small
 * ones.  Switching changes the plan's results at the FP32 rounding level and
 * drops its captured solver graphs and tuned shapes; call it between solves
 * (slot pools created before the switch keep the setting they were created
 * with; workspace sizes do not change).  A plan whose map fits in LDS, or
 * needs more than 8 bands, ignores it.
 * Errors: INVALID_ARG (null plan), UNSUPPORTED (a depth response set on the
 * plan would no longer fit an angle slot per block; the setting is
 * unchanged).  pget_plan_jvp_bands: the bands the product walks (1: none).
 */
pget_status pget_plan_set_band_staging(pget_plan* plan, int32_t enable);
int32_t pget_plan_jvp_bands(const pget_plan* plan);

/*
 * Depth factor of the attenuation path (the vertical correction c_{m,n} >= 1
 * of the discrete model, Sec. 2.1 eq. d_fwd_model: an emitter farther from
 * the detector reaches it along a steeper path through the medium).  The
 * transmission of sample i of every ray becomes exp(-atten_scale * d[i] *
 * B_i), and the Jacobian products follow.  `depth` is a host array of
 * pget_plan_n_samples(plan) values, sample 0 farthest from the detector
 * (t_i = (i - (n_t - 1)/2) * step along the direction toward the detector);
 * each must be finite and > 0.  NULL restores d = 1.  The values are copied
 * to the device (a small allocation owned by the plan) before the call
 * returns; calls enqueued afterwards use them, and no call of this plan may
 * be in flight meanwhile.  Errors: INVALID_ARG (null plan, wrong count, bad
 * value), HIP (allocation or copy failed).
 */
pget_status pget_plan_set_depth_factor(pget_plan* plan, const double* depth, int32_t n);

/*
 * Depth-dependent collimator response (the response r_{m,n} of the discrete
 * model, Sec. 2.1 eq. d_fwd_model, which for a deep collimator widens with
 * the emitter's distance from the detector).  The response to sample i of
 * every ray becomes (1 - alpha[i]) * kappa + alpha[i] * far_taps: the plan's
 * Gaussian taps kappa blended toward a second response, at offsets -K..K
 * bins from the ray's own bin.  `alpha` is a host array of
 * pget_plan_n_samples(plan) values in [0, 1], sample 0 farthest from the
 * detector; `far_taps` a host array of n_taps = 2K + 1 finite values (K =
 * pget_plan_psf_half_width(plan)), symmetric (far_taps[k] == far_taps[2K -
 * k], as the adjoint applies the same taps).  NULL alpha restores the
 * depth-independent response.  Forward, Jacobian products and every solver
 * follow.  The workspace of every operation grows (one more float per
 * lattice sample, a second plane of the per-ray sums): query
 * pget_workspace_bytes / pget_workspace_bytes_multi again after the call.
 * Values are copied to the device (a small allocation owned by the plan)
 * before the call returns; no call of this plan may be in flight meanwhile.
 * Errors: INVALID_ARG (null plan, wrong counts, alpha outside [0, 1], taps
 * not finite or not symmetric), UNSUPPORTED (BF16 storage, or the extra
 * rows of sums do not fit in the kernels' LDS for this shape), HIP
 * (allocation or copy failed).
 */
pget_status pget_plan_set_depth_response(pget_plan* plan, const double* alpha, int32_t n, const double* far_taps,
                                         int32_t n_taps);

/*
 * Device workspace needed by `op` for `batch` slices of this plan's shape
 * (batch >= 1; forward/jvp/vjp use batch 1).  0 on a bad argument.
 */
size_t pget_workspace_bytes(const pget_plan* plan, int32_t op, int32_t batch);

/*
 * y = A(f, mu): the attenuated ray transform with collimator response
 * (Sec. 2.1, eq. fwd_model / eq. d_fwd_model).  f, mu: N x N; y: n_angles x
 * n_bins.  ws: pget_workspace_bytes(plan, PGET_OP_FORWARD, 1).
 */
pget_status pget_forward(const pget_plan* plan, const float* f, const float* mu, float* y,
                         void* ws, hipStream_t stream);

/*
 * pget_forward without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels and the same result bit for bit.
 * The bordered copy of the map pair that the ray march reads when the pair
 * does not fit in LDS (N > 136: (N + 2)^2 * 8 bytes) lives in a static
 * device array of 2.25 MiB that the library holds on each device until the
 * process ends; sizes beyond it return PGET_ERR_UNSUPPORTED (no plan within
 * the N <= 512 limit reaches it).  Calls on one device share that array:
 * calls that overlap in time on one device (several streams or threads)
 * race and must be serialised by the caller.  The current device must be
 * the plan's (else PGET_ERR_INVALID_ARG).  Nothing is allocated, freed or
 * set with memset.
 */
pget_status pget_forward_noalloc(const pget_plan* plan, const float* f, const float* mu, float* y,
                                 hipStream_t stream);

/*
 * jv = J(f, mu) [vf, vmu] = D_lambda F[vf] + D_mu F[vmu] with
 * D_lambda F[v] = F(v, mu) and D_mu F[v] = -F(lambda * B v, mu) (Sec. 2.1,
 * eq. frechet), in the same discretisation as pget_forward.  y_or_null, if
 * not NULL, also receives A(f, mu).  ws: PGET_OP_JVP.
 */
pget_status pget_jvp(const pget_plan* plan, const float* f, const float* mu, const float* vf,
                     const float* vmu, float* jv, float* y_or_null, void* ws, hipStream_t stream);

/*
 * [gf, gmu] = J(f, mu)^T w, the exact transpose of pget_jvp (the adjoint
 * F'^* used for the gradient F'^*[r_k] in Sec. 3.1).  Computed as a gather
 * per pixel over (angle, bin, sample); no atomics, deterministic.
 * w: n_angles x n_bins; gf, gmu: N x N.  ws: PGET_OP_VJP.
 */
pget_status pget_vjp(const pget_plan* plan, const float* f, const float* mu, const float* w,
                     float* gf, float* gmu, void* ws, hipStream_t stream);

/*
 * Solver parameters (Sec. 2.2, eqs. lma_objective, LMA-step; Sec. 3.1).
 * Objective Phi(u) = 0.5 ||A(u) - y||^2 + 0.5 alpha_f ||grad f||^2
 *                    + 0.5 alpha_mu ||grad mu||^2   (forward differences,
 * Neumann boundary: the paper's priors P1, P2 are replaced by this gradient
 * penalty).  Each outer iteration solves (J^T J + beta D + R) x = -g with
 * n_cg conjugate-gradient steps from x = 0, D = diag(d_f I, d_mu I),
 * R = diag(alpha_f L, alpha_mu L), L = grad^T grad; clamps u + x into the box
 * [f_lo, f_hi] x [mu_lo, mu_hi]; accepts iff the gain ratio
 * rho = (Phi(u) - Phi(u')) / (m(0) - m(s)) > eta (eq. rho_agreement; rho is
 * -inf when the predicted decrease is <= 0); and updates beta by Nielsen's
 * rule.  beta0 <= 0 selects beta0 = tau * ||J 1||^2 / ||1||^2.
 * alpha_decay > 1 divides both alphas by alpha_decay^min(k, alpha_decay_until)
 * at outer iteration k (the continuation of Sec. 3.1); 1 disables it.
 * tol > 0 stops after an accepted step with ared <= tol*Phi or
 * ||s|| <= tol*||u||.  replay (test use): per outer iteration 1 = accept,
 * 0 = reject, instead of the rho test; NULL for the normal rule.
 * w_f, w_mu (> 0; 0 means 1) precondition CG by W = diag(w_f I, w_mu I),
 * the metric of variables scaled by their typical magnitudes, e.g. the
 * squares of the upper bounds (the paper solves the constrained step by a
 * scaled gradient projection, Sec. 2.2); 1, 1 is plain CG.  active_set = 1
 * holds every variable that lies on a bound with its gradient pointing out
 * of the box at zero step and runs CG on the free ones; 0 leaves every
 * variable free (the clamp alone keeps the trial point in the box).
 * cg_rr then reports r^T W r.
 * prior_w, prior_ref: the geometry prior (the paper's P1, P2, Sec. 2.2,
 * penalising emission and attenuation outside the possible rod locations),
 * Phi += 0.5 sum_m prior_w[m] (u[m] - prior_ref[m])^2 over the 2 N^2
 * elements of u = (f, mu) (f block first, row-major, like the maps).  Device
 * pointers owned by the caller, read on the stream until the solve ends;
 * prior_w = NULL: no prior; prior_ref = NULL: zero reference.  Weights must
 * be >= 0 (not checked: the solver reads them on the device); they are
 * divided by the same continuation factor as the alphas.
 * step selects the solver of the damped step.  PGET_STEP_CG: n_cg CG steps
 * on the normal equations as above, then the clamp into the box.
 * PGET_STEP_SGP: the paper's scaled gradient projection (Sec. 2.2, after
 * Bonettini, Zanella and Zanni) of the box-constrained step: n_cg
 * iterations, each y = P_box(s - alpha W grad q(s)), d = y - s, an Armijo
 * backtracking factor lambda (1, 0.4, 0.16, ...; sufficient decrease 1e-4,
 * exact for the quadratic q), s += lambda d, and the next alpha from the two
 * scaled Barzilai-Borwein rules with alternation (threshold 0.5, memory 3,
 * alpha in [1e-10, 1e5], alpha_0 = 1); W = diag(w_f I, w_mu I) is the
 * scaling, active_set is ignored, and cg_rr reports q(s) after each
 * iteration.  One normal-operator product per iteration either way.  All
 * slices of one batched or mixed call that share a plan must use the same
 * step solver.
 * trace_u, trace_t (optional, for step-by-step checks against a reference
 * implementation): device buffers of max_outer x 2 N^2 floats owned by the
 * caller; outer iteration k writes the iterate u_k it linearises at (f
 * block then mu block) to trace_u + k 2 N^2 and its trial point
 * u'_k = clamp(u_k + x_k) to trace_t + k 2 N^2 (with a hook, before the
 * proposal is evaluated).  Iterations not run leave their rows untouched.
 */
typedef struct {
    int32_t max_outer;        /* >= 1                                        */
    int32_t n_cg;             /* >= 1                                        */
    double alpha_f, alpha_mu; /* >= 0                                        */
    double alpha_decay;       /* >= 1                                        */
    int32_t alpha_decay_until;
    double beta0, tau;
    double eta;               /* acceptance threshold, e.g. 1e-3             */
    double d_f, d_mu;         /* > 0                                         */
    double f_lo, f_hi, mu_lo, mu_hi;
    double tol;
    const int8_t* replay;     /* host pointer, max_outer entries, or NULL    */
    double w_f, w_mu;         /* CG preconditioner, > 0 (0 -> 1)             */
    int32_t active_set;       /* 0 or 1                                      */
    const float* prior_w;     /* device, 2 N^2, or NULL                      */
    const float* prior_ref;   /* device, 2 N^2, or NULL                      */
    float* trace_u;           /* device, max_outer x 2 N^2, or NULL          */
    float* trace_t;           /* device, max_outer x 2 N^2, or NULL          */
    int32_t step;             /* PGET_STEP_CG (0) or PGET_STEP_SGP (1)       */
} pget_lm_params;

/* Solvers of the damped step (pget_lm_params.step). */
enum { PGET_STEP_CG = 0, PGET_STEP_SGP = 1 };

/*
 * Per-solve report.  Every pointer is caller-owned and may be NULL (not
 * written) or point to host or device memory of the given length; it is
 * written asynchronously on the stream.  After the stream syncs:
 *   status        PGET_OK, or PGET_ERR_NONFINITE if Phi or a step went
 *                 non-finite (the iterate is left at its last finite value).
 *   iters_run     outer iterations executed (<= max_outer).
 *   phi[k]        Phi at the start of outer iteration k; phi[iters_run] is
 *                 Phi of the returned maps.       [max_outer + 1]
 *   rho, beta, pred, ared, gnorm [k]               [max_outer]
 *   accepted[k], hook_accepted[k]                  [max_outer]
 *   cg_rr[k * n_cg + m]  r^T r after CG step m     [max_outer * n_cg]
 *   hook_rho[k], hook_pred[k]  rho(s~) and m(0) - m(s~) of the hook's
 *                 proposal after iteration k (the two sides of the
 *                 safeguard, with pred[k] = m(0) - m(s_k)); NaN where no
 *                 proposal was evaluated.                [max_outer]
 *   beta_final    damping after the last iteration.
 * The scalar fields are written through `scalars` (device or host memory,
 * 4 doubles: status, iters_run, beta_final, stop_reason) when not NULL;
 * stop_reason: 0 max_outer, 1 tolerance, 2 damping overflow, 3 non-finite.
 */
typedef struct {
    double* scalars;
    double* phi;
    double* rho;
    double* beta;
    double* pred;
    double* ared;
    double* gnorm;
    int8_t* accepted;
    int8_t* hook_accepted;
    double* cg_rr;
    double* hook_rho;
    double* hook_pred;
} pget_lm_report;

/*
 * The learned refinement of Alg. 2 (Deep Gauss-Newton step), called on the
 * host after each ACCEPTED LM step with device pointers to the previous
 * iterate u_k = (f, mu) and the LM step s_k = (s_f, s_mu); it must enqueue
 * work on `stream` that writes its proposal u~ into (f_tilde, mu_tilde) and
 * return 0, or return nonzero to skip.  The proposal is kept iff
 * rho(u~ - u_k) > eta and m(u~ - u_k) <= m(s_k) (Prop. 3.2, Alg. 2).
 */
typedef int (*pget_refine_fn)(void* user, const float* f, const float* mu, const float* s_f,
                              const float* s_mu, float* f_tilde, float* mu_tilde,
                              hipStream_t stream);

/*
 * Levenberg-Marquardt reconstruction of one slice.  f_inout, mu_inout hold
 * the initial guess on entry and the result on exit (N x N each); y is the
 * measured sinogram.  Without a hook the whole solve is enqueued with no
 * host synchronisation; with a hook the host waits for each accept decision.
 * ws: PGET_OP_LM with batch 1.
 */
pget_status pget_lm_solve(const pget_plan* plan, const float* y, float* f_inout, float* mu_inout,
                          const pget_lm_params* params, pget_refine_fn hook, void* hook_user,
                          const pget_lm_report* report, void* ws, hipStream_t stream);

/*
 * n_slices >= 1 (else PGET_ERR_INVALID_ARG) independent reconstructions of
 * the same plan shape solved
 * together (every kernel launch covers all slices).  y, f_inout, mu_inout
 * are arrays of n_slices device pointers (host arrays of pointers);
 * params and reports are arrays of n_slices entries (reports may be NULL).
 * Each slice's result is the one pget_lm_solve gives for it alone, bit for
 * bit: every order of additions (per-angle partials of the squared norms,
 * fixed-order sums of partials, the adjoint's fine angle groups) depends on
 * the plan only, never on the batch.
 * ws: PGET_OP_LM with batch n_slices.
 */
pget_status pget_lm_solve_batched(const pget_plan* plan, int32_t n_slices, const float* const* y,
                                  float* const* f_inout, float* const* mu_inout,
                                  const pget_lm_params* params, const pget_lm_report* reports,
                                  void* ws, hipStream_t stream);

/*
 * Kernel timing for measurement tools.  pget_timing_enable(classes, capacity)
 * brackets every later launch of the kernel classes in the bit mask `classes`
 * (1 << PGET_KC_*) with HIP events on the launch's own stream, up to
 * `capacity` launches in total (0 disables and frees the events).
 * pget_timing_read waits for the recorded events of one class and returns the
 * summed device time in milliseconds and the number of launches.  Not
 * thread-safe; meant for benchmarks and profilers.
 */
enum {
    PGET_KC_MARCH = 0,   /* ray march: forward / linearisation / trial point */
    PGET_KC_JVP = 1,     /* Jacobian product from the stored weights          */
    PGET_KC_VJP = 2,     /* adjoint gather (CG solve, pget_vjp)               */
    PGET_KC_VECTOR = 3,  /* element-wise CG / step kernels                    */
    PGET_KC_CONTROL = 4, /* per-slice decisions, packing, blur                */
    PGET_KC_GRADIENT = 5 /* adjoint gather of the gradient (skipped when the
                            iterate did not change)                           */
};
pget_status pget_timing_enable(int32_t classes, int32_t capacity);
pget_status pget_timing_read(int32_t kernel_class, double* total_ms, int64_t* launches);

/*
 * Replay of the solver's kernel sequence as a HIP graph (default on).  The
 * sequence of a solve without hook is captured once per (plan, workspace,
 * batch, max_outer, n_cg) and replayed on later calls with the same key;
 * inputs and parameters are uploaded before each replay.  Graphs are not used
 * while kernel timing is enabled or when a hook is given.  enable = 0 turns
 * replay off (every call launches its kernels directly).  Results are the same
 * either way, bit for bit.
 */
pget_status pget_set_graphs(int32_t enable);

/*
 * Slices of different shapes solved together (mixed grid sizes): slice s
 * uses plans[s]; slices sharing a plan form one group solved as a batch, and
 * the groups run concurrently on the device (one graph launch when graphs are
 * on).  Arguments as for pget_lm_solve_batched, per slice; within a group all
 * slices must share max_outer and n_cg.  ws must hold
 * pget_workspace_bytes_multi(n_slices, plans) bytes; ws_bytes is its size.
 * Each slice's result is the one pget_lm_solve gives for it alone, bit for
 * bit (as for pget_lm_solve_batched).
 */
size_t pget_workspace_bytes_multi(int32_t n_slices, const pget_plan* const* plans);
pget_status pget_lm_solve_multi(int32_t n_slices, const pget_plan* const* plans, const float* const* y,
                                float* const* f_inout, float* const* mu_inout,
                                const pget_lm_params* params, const pget_lm_report* reports, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/*
 * Autotuner of launch shapes: times the candidate shapes of the Jacobian
 * product (angle slots per block: 1, 2, 4, ...) and of the adjoint gather
 * (blocks per pixel tile, each running a run of the plan's fine angle
 * groups) for `batch` slices of this plan's shape on zero-filled data, and
 * keeps the fastest pair in the plan for later solves of that batch size.
 * ws: at least pget_workspace_bytes(plan, PGET_OP_LM, batch) bytes (its
 * contents are overwritten).  Synchronises `stream`.  No shape changes any
 * result bit: the fine angle groups, whose partial images are added in
 * order, are fixed by the plan.
 * pget_tuned_shape reports the shape a solve of `batch` slices will use
 * (vjp_groups: gather blocks per tile and slice) and returns 1 if it came
 * from the autotuner, 0 if from the default heuristic.
 */
pget_status pget_autotune(pget_plan* plan, int32_t batch, void* ws, size_t ws_bytes, hipStream_t stream);
int32_t pget_tuned_shape(const pget_plan* plan, int32_t batch, int32_t* japb, int32_t* vjp_groups);

/*
 * Fix the launch shapes of solves of `batch` slices by hand, as the
 * autotuner would: japb angle slots per Jacobian-product block (1 ..
 * the plan's limit; 0 keeps the default) and fine_per_block fine angle groups
 * per gather block (a multiple of the plan's super group or all of them,
 * else one; 0 keeps the default).  With band staging on
 * (pget_plan_set_band_staging), product blocks of at least 6 angle slots
 * stage the map in bands of rows and smaller ones read the same bands from
 * the HBM copy: like every shape, this changes no result bit.  Errors:
 * INVALID_ARG (null plan, batch < 1, negative values, japb above the
 * plan's limit).
 */
pget_status pget_set_shape(pget_plan* plan, int32_t batch, int32_t japb, int32_t fine_per_block);

/*
 * Slot pools: continuous batching at outer-iteration boundaries (Sec. 2.2's
 * outer LM iteration is the unit of admission and retirement).  A pool
 * keeps `capacity` slots of one plan's shape, each holding one slice's
 * whole LM state on the device; slots at different outer iterations run in
 * the same launches.  pget_lm_pool_load puts a slice into a free slot;
 * pget_lm_pool_step runs ONE outer iteration of every loaded, unfinished
 * slot (its initial damping at its first iteration) and writes, to
 * `finished` (capacity int32, host or device memory of the caller, written
 * asynchronously), 1 for every slot whose solve has stopped (max_outer,
 * tolerance, damping overflow, non-finite) or that is free, else 0;
 * pget_lm_pool_fetch copies a slot's maps and report out and frees the slot
 * (fetching an unfinished slot cancels its solve at the iteration boundary:
 * the maps are its current iterate).  Each slice's result is the one
 * pget_lm_solve gives for it alone, bit for bit, whatever the other slots
 * hold.  Rules: params->step must equal the pool's `step` (PGET_STEP_*),
 * params->n_cg must equal the pool's n_cg and
 * params->max_outer be at most the pool's; no hook; every call of a pool on
 * one stream (or ordered by the caller); a pool is not thread-safe.  The
 * step is captured as a HIP graph on its first call and replayed (unless
 * graphs are off or timing is on).  ws: pget_lm_pool_workspace_bytes bytes,
 * owned by the caller, alive until pget_lm_pool_destroy; the pool object
 * itself holds only host-side bookkeeping.  Errors: INVALID_ARG (bad slot,
 * slot busy on load or free on fetch, parameters), WORKSPACE, HIP.
 */
typedef struct pget_lm_pool pget_lm_pool;
size_t pget_lm_pool_workspace_bytes(const pget_plan* plan, int32_t capacity, int32_t max_outer, int32_t n_cg);
pget_status pget_lm_pool_create(const pget_plan* plan, int32_t capacity, int32_t max_outer, int32_t n_cg,
                                int32_t step, void* ws, size_t ws_bytes, hipStream_t stream, pget_lm_pool** out);
void pget_lm_pool_destroy(pget_lm_pool* pool);
pget_status pget_lm_pool_load(pget_lm_pool* pool, int32_t slot, const float* y, const float* f0, const float* mu0,
                              const pget_lm_params* params, hipStream_t stream);
pget_status pget_lm_pool_step(pget_lm_pool* pool, int32_t* finished, hipStream_t stream);
pget_status pget_lm_pool_fetch(pget_lm_pool* pool, int32_t slot, float* f_out, float* mu_out,
                               const pget_lm_report* report, hipStream_t stream);

/* Human-readable name of a status code (static string). */
const char* pget_status_string(pget_status status);

#ifdef __cplusplus
}
#endif

#endif /* PGET_H */
