/*
 * gbs.h -- click-pattern probabilities of a lossy Gaussian boson sampler on
 * one AMD Instinct MI355X (gfx950).  C ABI; no PyTorch or HIP types.
 *
 * Method: A. S. Popova and A. N. Rubtsov, "Cracking the Quantum Advantage
 * threshold for Gaussian Boson Sampling".  The probability that exactly the
 * detectors in C fire is computed two ways:
 *   - exactly, as the signed sum over the 2^n subsets of C of vacuum
 *     probabilities (Methods, Probability of any sample: "2^n determinants");
 *   - approximately at order j, by the paper's scheme (Results, Approximation
 *     scheme; Methods, Moments calculation and Approximation method):
 *     photon-number sectors of the sub-ensemble, their click-count moments up
 *     to order j from clusters of <= j modes, an exp-polynomial fitted per
 *     sector, and the sum over sectors of the fitted all-click point.
 *
 * State conventions: a_out = U a_in; input j is a single-mode squeezed vacuum
 * with parameter r_j (0 = vacuum), squeezed along x; output mode i then passes
 * a pure-loss channel of transmission eta_i; hbar = 1, vacuum covariance I/2,
 * quadratures ordered xxpp (mode i owns rows i and M+i).  At eta = 1 the state
 * is the paper's exp(-a+ X a+)|0> with X = (1/2) U diag(tanh r) U^T (Methods,
 * Model; the paper's U is the transpose of this one).
 *
 * Ownership: the caller owns every array passed in.  gbs_set_model and
 * gbs_set_covariance copy their inputs to the device.  Calls without the _dev
 * suffix take host pointers and return when the results are in host memory.
 * Calls with the _dev suffix take device pointers, enqueue work on the
 * context's stream and return without synchronising; the caller keeps the
 * buffers alive until that stream has passed them.
 *
 * Errors: every call returns GBS_OK (0), a negative error code, or
 * GBS_W_PATTERN (1) when some pattern's status is non-zero.  Argument errors
 * are detected before any device work and write no output.  The message of the
 * last failing call is available from gbs_last_error.  A pattern whose numerics
 * fail gets a NaN result and a non-zero status bit; nothing is substituted.
 *
 * Threading: one context per host thread.  Calls on one context are not
 * re-entrant.
 */
#ifndef GBS_H
#define GBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gbs_ctx gbs_ctx;
typedef struct gbs_plan gbs_plan;

enum {
    GBS_OK = 0,
    GBS_E_INVAL = -1,  /* bad argument (sizes, CSR rows, order, precision)       */
    GBS_E_NOTPD = -2,  /* covariance + I/2 not positive definite                 */
    GBS_E_NOMEM = -3,  /* device allocation failed                               */
    GBS_E_HIP = -4,    /* HIP runtime error (message has the HIP error string)   */
    GBS_E_STATE = -5,  /* no model set, plan from another ctx or for another M   */
    GBS_W_PATTERN = 1  /* success, but some status[p] != 0                       */
};

/*
 * Precision.  GBS_PREC_FP64: every step in fp64 (double-double where stated).
 * GBS_PREC_MIXED (approximate path, forward only, orders 1-3): the cluster
 * eliminations run in fp32 on an fp32 copy of M(w); the model, the
 * eigen-decomposition, the contour plan, M(w) itself, G_0(w), the sums over
 * clusters, the sector transform and the fits stay fp64.  The sector transform
 * extracts small moments from contour values whose fp32 rounding is set by the
 * largest ones, so the error grows with a row's dynamic range.  Every row's
 * rounding error is therefore bounded (gbs_plan_info); a row whose bound
 * exceeds the tier's target of 1e-5 in log p, or whose fits fail, is run again
 * in fp64 within the same call, on the device, and flagged GBS_PS_ESCALATED,
 * so that every row meets the target against fp64.  (Measured: the fp32
 * eliminations leave |d log p| of median 3e-6 / 3e-5 / 1e-4 at 20 / 70 / 100
 * modes, and the bound, which holds on every measured row, escalates nearly
 * every row of these workloads: on this GPU the fp32 vector rate equals the
 * fp64 rate, so the tier saves registers and on-chip memory, not arithmetic.)
 * Where no fp32 kernel exists the tier is accepted and the work runs at the
 * higher precision, every row flagged GBS_PS_ESCALATED: the exact path (fp32
 * terms would meet 1e-6 only where kappa_IE <= 10, far below the measured
 * 5e5 .. 1e11 of 20-mode rows; it runs in double-double), order 4 (fp64), and
 * the gradient (forward and adjoint in fp64).  The plain comparison kernel
 * takes GBS_PREC_FP64 only (GBS_E_INVAL otherwise).
 */
enum { GBS_PREC_FP64 = 0, GBS_PREC_MIXED = 1 };

/*
 * Per-pattern status bits.  FIT_NOCONV, PIVOT, CANCEL and BADROW mean the row
 * has no result: its output is NaN.  CONTOUR and ESCALATED are informational:
 * the result is returned and the bit says how it was obtained.
 *
 * GBS_PS_CONTOUR (Methods, Partition function: the sectors come from a sum
 * over a discrete set of points of the generating function) is set when
 *   (a) the contour cannot resolve the sectors that carry the estimate: their
 *       tilted weights tau_kappa (the contour's total is 1), averaged with
 *       their shares of the estimate as sum_kappa w_kappa / tau_kappa, fall
 *       below 1e-6, so that the transform's rounding floor (about 1e-16 of
 *       the total) reaches 1e-10 of the estimate.  Such a row is first run
 *       again, on the device within the same call, on a contour whose tilted
 *       mean photon number is the mean of those sectors (not on a frozen
 *       plan, whose radii stay fixed); the bit is set when the re-tilted
 *       radius still leaves them unresolved, which happens when it hits the
 *       cap 0.98 R_b (the lossless 70-mode device with 50 clicks: every row
 *       resolved at orders 1 and 2, 3 of 16 flagged at orders 3 and 4; on the
 *       144-mode workload the 301 of 4096 rows whose radius is capped keep at
 *       least 0.24 of the tilted weight above n photons and are not
 *       flagged); or
 *   (b) a frozen plan's radius no longer suits the current model:
 *       rho max|alpha - 1| reached 1 or the aliasing factor
 *       (rho max|alpha - 1|)^K exceeds 1e-14.  The row is then planned afresh
 *       for this call (new rho and K).
 */
enum {
    GBS_PS_OK = 0,
    GBS_PS_FIT_NOCONV = 1, /* a sector fit carrying >1e-10 of the estimate did not converge */
    GBS_PS_CONTOUR = 2,    /* the contour deviated from its accuracy rule (see above)        */
    GBS_PS_PIVOT = 4,      /* a determinant pivot left its valid half-plane                   */
    GBS_PS_ESCALATED = 8,  /* ran at higher precision than asked (mixed -> fp64 / dd)         */
    GBS_PS_CANCEL = 16,    /* exact sum not resolved: |sum| below its rounding bound          */
    GBS_PS_BADROW = 32     /* device-side CSR check failed (gbs_prob_exact_dev): no result    */
};

/* Create a context on HIP device `hip_device`.  hip_stream: a hipStream_t to
 * enqueue on (cast to void*), or NULL for a stream owned by the context. */
int gbs_create(gbs_ctx **out, int hip_device, void *hip_stream);
int gbs_destroy(gbs_ctx *ctx);
/* Message of the last failing call on ctx (valid until the next call). */
const char *gbs_last_error(const gbs_ctx *ctx);

/* Model build (Methods, Model, with output loss added): M modes, U row-major
 * M x M as separate real and imaginary planes, r[M] >= 0, eta[M] in [0, 1].
 * Builds sigma = D O diag(e^{-2r}, e^{2r}) O^T D / 2 + (I - D^2)/2 with
 * O = [[Re U, -Im U], [Im U, Re U]] and D = diag(sqrt eta, sqrt eta), then
 * Q = sigma + I/2, its Cholesky factor, Q^{-1} and log det Q, all in
 * double-double, on the device.  1 <= M <= 512.  Host pointers. */
int gbs_set_model(gbs_ctx *ctx, int M, const double *U_re, const double *U_im,
                  const double *r, const double *eta);
/* Stream-ordered model build from device arrays (same layout as
 * gbs_set_model); no host synchronisation.  A covariance that is not positive
 * definite is reported per row (status GBS_PS_PIVOT) by the next call. */
int gbs_set_model_dev(gbs_ctx *ctx, int M, const double *U_re_dev, const double *U_im_dev,
                      const double *r_dev, const double *eta_dev);
/* Same from a covariance matrix sigma ((2M)^2, row-major, xxpp, vacuum I/2);
 * sigma + I/2 must be positive definite.  The gradient call needs the model
 * form and returns GBS_E_STATE after gbs_set_covariance. */
int gbs_set_covariance(gbs_ctx *ctx, int M, const double *sigma);
/* Copy the device model back: q_inv (2M)^2 fp64 (high part), logdet_q. */
int gbs_get_model(gbs_ctx *ctx, double *q_inv, double *logdet_q);

/*
 * Click patterns are CSR rows: offsets[P+1] (offsets[0] = 0, non-decreasing),
 * modes[offsets[P]]; each row lists the clicked output modes, strictly
 * ascending, in [0, M).  Every other mode is a no-click.
 *
 * gbs_prob_exact: exact probability (Methods, Probability of any sample; the
 * click projector of Methods, Model):
 *     p(C) = det(Q)^{-1/2} sum_{Z subset C} (-1)^{n-|Z|} det((Q^{-1})_{ZZ})^{-1/2}
 * The 2^n terms and their signed sum are evaluated in double-double, so p is
 * accurate to ~1e-16 relative even when the sum cancels by 1e11.  Rows may hold
 * at most 30 clicks (2^30 terms; a row of 30 clicks takes of the order of a
 * second).  Outputs (host arrays of length P): p, logp (nullable),
 * kappa = sum|terms| / |sum| (nullable), status.  A row whose sum cancels by
 * more than 1e20 gets NaN and GBS_PS_CANCEL.  prec: GBS_PREC_FP64, or
 * GBS_PREC_MIXED (the same double-double run, every row flagged
 * GBS_PS_ESCALATED; see Precision above).
 */
int gbs_prob_exact(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int prec,
                   double *p, double *logp, double *kappa, int32_t *status);
/*
 * The same from device arrays, stream-ordered (no host synchronisation): CSR
 * offsets_dev[P+1], modes_dev[offsets[P]] and outputs p_dev[P], status_dev[P],
 * logp_dev[P] and kappa_dev[P] (both nullable), all device pointers.
 * max_clicks (0..30) bounds the clicks of every row and sizes the launch; the
 * rows are checked on the device: a row with more clicks, a mode outside
 * [0, M) or modes not strictly ascending gets NaN and GBS_PS_BADROW.  The
 * call returns GBS_OK once the work is enqueued (the per-row status is in
 * status_dev).  Partial sums live in a context-owned device buffer of
 * 24 P 2^min(max(max_clicks - 9, 0), 12) bytes, grown on demand (the call then
 * waits for the stream before it frees the old one).
 */
int gbs_prob_exact_dev(gbs_ctx *ctx, int P, const int32_t *offsets_dev, const int32_t *modes_dev, int max_clicks,
                       double *p_dev, double *logp_dev, double *kappa_dev, int32_t *status_dev);
/*
 * gbs_prob_exact_dev for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): same arguments, results and errors, but no hipMalloc, hipFree
 * or other allocating call.  The partial sums live in a fixed device array of
 * 24 MiB per GPU (2^20 work items), set up when the first context is created
 * on that GPU and held until the process ends; a batch needing more than
 * P 2^min(max(max_clicks - 9, 0), 12) = 2^20 work items is GBS_E_INVAL.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other contexts, other host threads) race and give wrong results.
 */
int gbs_prob_exact_dev_noalloc(gbs_ctx *ctx, int P, const int32_t *offsets_dev, const int32_t *modes_dev,
                               int max_clicks, double *p_dev, double *logp_dev, double *kappa_dev,
                               int32_t *status_dev);

/*
 * gbs_prob_approx: the paper's order-j estimate (1 <= order <= 4), returned as
 * log p_hat (p_hat reaches 1e-35 and below).  For each row:
 *   1. A = (Q^{-1})_CC, eigen-decomposed (A = V diag(alpha) V^T);
 *      log P_vac(Cbar) = -(log det Q + log det A) / 2 (eq. 3, second factor);
 *   2. contour radius rho: the tilted mean photon number equals max(n, the
 *      untilted mean), capped at 0.98 of the convergence radius
 *      1/max|alpha-1|; K points, K the smallest r 2^k (r odd <= 15, k >= 1) with
 *      (rho/R)^K <= 1e-16 and K >= 2n+32, K <= 2048;
 *   3. at each contour point w: M(w) = ((1-w)I + wA)^{-1} and, for every cluster
 *      T of <= j clicked modes, G_T(w) = det(A)^{1/2} det((1-w)I+wA)^{-1/2}
 *      det(M(w)_TT)^{-1/2} (Methods, Partition function and Moments
 *      calculation), summed per cluster size;
 *   4. sector moments by a discrete Fourier transform over the contour;
 *   5. per sector kappa >= n, the exp-polynomial of degree min(j, n-1) matching
 *      the moments (Methods, Approximation method) and its all-click value;
 *   6. log p_hat = log P_vac(Cbar) + log sum_kappa S_0[kappa] q_kappa(n).
 * Rows may hold at most 128 clicks at orders 1 and 2 and at most 64 at orders
 * 3 and 4 (more is GBS_E_INVAL); order 4 runs in fp64 (GBS_PREC_MIXED there:
 * fp64, every row flagged GBS_PS_ESCALATED).  Rows above 40 clicks read their eigenvectors from
 * device memory (L2) instead of on-chip memory, and beyond 64 clicks (orders 1
 * and 2) keep only the diagonal blocks of M(w) on chip (slower per contour
 * point, same results).  Outputs: logp[P], status[P].
 */
int gbs_prob_approx(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int order,
                    int prec, double *logp, int32_t *status);

/*
 * The same estimate (same eigen-decomposition, contour plan, sector transform
 * and fits) with a plain contour kernel in place of the tuned one: one
 * workgroup per row, contour points in sequence, M(w) by plain dot products,
 * and every cluster determinant by its own unpivoted LDL^T.  For speed-up
 * comparisons and as an independent check of gbs_prob_approx.  Rows may hold
 * at most 40 clicks; arguments, outputs and errors as gbs_prob_approx.
 */
int gbs_prob_approx_plain(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes,
                          int order, int prec, double *logp, int32_t *status);

/*
 * gbs_click_distribution: the order-j estimate (1 <= order <= 4) of the whole
 * device's click distribution p(n), n = 0..M, the probability that exactly n
 * of the M detectors click, and of its photon-number sector curves p_k(n)
 * (Results, Calculation of p(n) and of sectors p_k(n); Fig. 2).  The steps of
 * gbs_prob_approx with C = every mode (no conditioning): the sector moments
 * from clusters of <= j modes, and per sector k an exp-polynomial fitted on its
 * support n = 1..min(k, M) (k photons click at most k detectors), whose whole
 * curve is kept: p_k(n) = S_0[k] q_k(n), p(n) = sum_k p_k(n), p(0) = S_0[0].
 * The contour runs at radius 1 (capped at 0.98 of the convergence radius), so
 * every sector comes at its own weight with rounding ~1e-16 of the largest;
 * sectors below 1e-14 of the largest are left out.  The values are therefore
 * accurate in absolute terms (~1e-10), not relative to tiny p(n).
 * M <= 40 modes, fp64.  ks[nk]: the sectors whose curves are wanted (host);
 * outputs (host): p_n[M+1], p_k[nk][M+1] (row i for ks[i]; zero for a sector
 * outside the contour's range), status[1] (GBS_PS_FIT_NOCONV if fits carrying
 * more than 1e-10 of the weight failed; the call then returns GBS_W_PATTERN).
 */
int gbs_click_distribution(gbs_ctx *ctx, int order, int nk, const int32_t *ks, double *p_n, double *p_k,
                           int32_t *status);

/*
 * Plans: the per-batch layout (rows sorted by cost, device copies of the CSR,
 * workspace) built once and reused.  gbs_plan_create copies the host CSR.
 * The plan holds the contour radius and size per row from the first run on;
 * set freeze = 1 in gbs_plan_freeze to keep them fixed for later runs (finite
 * differences, fit loops).
 */
int gbs_plan_create(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int order,
                    int prec, gbs_plan **out);
int gbs_plan_destroy(gbs_plan *plan);
int gbs_plan_freeze(gbs_plan *plan, int freeze);
/* Stream-ordered forward on a plan: logp_dev[P], status_dev[P] device arrays
 * (status_dev nullable), results in the caller's row order. */
int gbs_prob_approx_dev(gbs_ctx *ctx, gbs_plan *plan, double *logp_dev, int32_t *status_dev);

/*
 * gbs_grad: gradient of L = sum_p dL_dlogp[p] * log p_hat_p (order-j estimate)
 * with respect to r[M] and eta[M] of the model set by gbs_set_model, by a
 * hand-written adjoint of steps 1-6 (d log det X = tr(X^{-1} dX) at every
 * determinant, implicit differentiation of each sector fit), with the contour
 * radius and size held at their forward values.  Orders 1 to 4, the row
 * limits of gbs_prob_approx; at order 4 each quadruple's c_T M_TT^{-1} comes
 * from the bordered inverse of its triple (y = M3^{-1} r_d by back-substitution
 * through the elimination's factors).  fp64 (GBS_PREC_MIXED, or a mixed-tier
 * plan: fp64 forward and adjoint, every row flagged GBS_PS_ESCALATED).  Host
 * pointers; logp (nullable) receives the forward values.
 */
int gbs_grad(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int order, int prec,
             const double *dL_dlogp, double *logp, double *grad_r, double *grad_eta,
             int32_t *status);
/* Stream-ordered gradient on a plan: all pointers are device arrays. */
int gbs_grad_dev(gbs_ctx *ctx, gbs_plan *plan, const double *dL_dlogp_dev, double *logp_dev,
                 double *grad_r_dev, double *grad_eta_dev, int32_t *status_dev);

/*
 * Launch choices of a plan, params[4]: [0] third modes per cluster work unit of
 * the forward contour kernel (order 3; at order 4 also the fourth modes per
 * quadruple unit, at most 15 of them), [1] the same for the adjoint, [2]
 * contour points per forward work item (4, 8, 16, 32 or 64), [3] most contour
 * points per pass of the forward kernel (1, 2, 4 or 8).  Defaults 3, 3, 8, 8.
 * They change the speed, not the results (up to the order of floating-point
 * sums).  gbs_plan_set_params returns GBS_E_INVAL for values outside these sets.
 */
int gbs_plan_get_params(gbs_plan *plan, int32_t *params);
int gbs_plan_set_params(gbs_plan *plan, const int32_t *params);

/*
 * Autotuner: times candidate launch choices (coordinate descent over third
 * modes per unit 2, 3, 4, 6, 8, 12 for the forward and 2, 3, 4, 6 for the
 * adjoint, points per item 4, 8, 16 and per pass 2, 4, 8; two runs each, the
 * faster counts) on a stratified
 * sample of the plan's rows (every s-th row in cost order, s = max(1, P/1024))
 * with the context's current model, and stores the fastest in the plan.  what:
 * bit 0 the forward choices, bit 1 the adjoint's (needs a model set from
 * parameters).  params (nullable) receives the chosen values.  Synchronous;
 * allocates a temporary plan for the sample.
 */
int gbs_plan_tune(gbs_ctx *ctx, gbs_plan *plan, int what, int32_t *params);

/* Per-row diagnostics of the last run on a plan (host arrays of length P,
 * each nullable): contour radius, convergence radius, K, sectors fitted, and
 * the estimated rounding error of log p_hat in the precision the row ran in:
 * each tilted moment carries the rounding of its contour values (relative
 * 2e-16 in fp64, 2e-7 for fp32 cluster eliminations; through the transform at
 * most that times the mean modulus of the values over the contour), pushed
 * through each sector fit's sensitivity (d log q / d m = -H^{-1} m) and summed
 * with the sectors' shares of the estimate. */
int gbs_plan_info(gbs_plan *plan, double *rho, double *rconv, int32_t *K, int32_t *nsectors, double *err);

/*
 * Deterministic gradients (on != 0; off by default).  The adjoint adds
 * cluster terms into Z(w) and rows' terms into the adjoint of Q^-1 with
 * atomic floating-point adds, whose order, and so the last bits of the
 * gradient, vary from run to run (~1e-14 relative).  With the switch on, the
 * terms are added as 64-bit integers, llrint(term x scale), whose sum does not
 * depend on the order, and converted back: the results are bitwise
 * reproducible (same plan, model, weights and GPU type).  The scales are
 * powers of two that leave room for every term of an entry (one per cluster
 * holding its modes; one per row for Q^-1's adjoint) below the largest term
 * of its kind: for Q^-1's adjoint a first pass over the rows finds it; for
 * Z(w), separately for its diagonal and its pair blocks, each point adds at
 * the scales its predecessor's terms set and is run again at exact scales
 * when its own largest terms do not fit them (an item's first point first
 * takes a pass that only finds them).  Each term is rounded at its scale,
 * which costs precision where there are many clusters and their sums
 * cancel: measured against the floating-point sums, in units of the largest
 * gradient component, about 1e-15 at orders 1 and 2, 1e-12 for 40-click rows
 * and 4e-11 for 60-click rows at order 3, 1e-13 for 14-click rows and 1e-8
 * for 45-click rows at order 4 (where the floating-point path's own
 * run-to-run spread is 2e-10).  The cost: about 10 % on a forward + gradient
 * step of 15-40-click rows at order 3.  Affects gbs_grad and gbs_grad_dev on
 * this context.  Errors: GBS_E_INVAL for a NULL context.
 */
int gbs_set_deterministic(gbs_ctx *ctx, int on);

/*
 * gbs_mcmc_step_dev: one Metropolis-Hastings step (Metropolis et al. 1953,
 * Hastings 1970) of P chains of click patterns whose target is the order-j
 * estimate p_hat of the plan's order (Discussion: the approximate
 * probabilities as the basis of a Markov chain Monte Carlo sampler).  Chain p
 * is row p of the plan (made by gbs_plan_create from the chains' initial
 * patterns, not frozen) and keeps its number of clicks n_p.  Per step and
 * chain, from three uniforms u in [0, 1): the clicked mode at position
 * floor(u[3p] n_p) of the row is swapped for the k-th unclicked mode in
 * increasing order, k = floor(u[3p+1] (M - n_p)) (a symmetric proposal; rows
 * with n_p = 0 or M do not move); log p_hat of every proposal is computed on
 * the plan (the plan's copy of the rows is overwritten with the proposals);
 * the proposal is accepted when its log p_hat is >= the current one or
 * u[3p+2] < exp(difference), rejected when its estimate failed (NaN).
 * Device arrays, stream-ordered: u_dev[3P] (caller-drawn uniforms),
 * modes_dev[offsets[P]] the chains' current rows (the plan's offsets,
 * strictly ascending modes; in/out), logp_dev[P] their log p_hat (in/out; from
 * gbs_prob_approx_dev on the initial rows), accepted_dev[P] (nullable; 1 where
 * the chain moved, 0 where not, -1 where its row is malformed: modes not
 * strictly ascending in [0, M); such a chain never moves).  Errors: GBS_E_STATE for a frozen plan or a plan of
 * another context or model size, GBS_E_INVAL for NULL arrays.
 */
int gbs_mcmc_step_dev(gbs_ctx *ctx, gbs_plan *plan, const double *u_dev, int32_t *modes_dev, double *logp_dev,
                      int32_t *accepted_dev);

/*
 * gbs_mcmc_da_step_dev: one two-stage (delayed-acceptance) Metropolis-Hastings
 * step (Christen & Fox 2005) of P chains whose target is the exact p, with the
 * order-j estimate as the proposal filter (Discussion: the approximation as
 * the proposal distribution of a Markov chain Monte Carlo sampler).  The
 * swap proposal is that of gbs_mcmc_step_dev; the first stage accepts it with
 * min(1, p_hat(new) / p_hat(old)), and only proposals that pass get an exact
 * evaluation (the exact path of gbs_prob_exact_dev, on the packed rows), which
 * accepts them with min(1, [p(new) p_hat(old)] / [p(old) p_hat(new)]): the
 * chains' stationary distribution is the exact p restricted to n_p clicks.
 * Device arrays, stream-ordered: u_dev[4P] (caller-drawn uniforms: swap,
 * swap, first stage, second stage), modes_dev (as gbs_mcmc_step_dev; in/out),
 * logp_hat_dev[P] and logp_exact_dev[P] the current rows' log p_hat and exact
 * log p (in/out; from gbs_prob_approx_dev and gbs_prob_exact_dev on the
 * initial rows), accepted_dev[P] (nullable; 1 moved, 0 rejected by the
 * estimate, 2 rejected by the exact correction, -1 malformed row).  A chain
 * whose current values are not both finite takes any proposal whose two
 * values are.  Rows of at most 30 clicks (the exact path).  The plan holds the
 * chains' workspace (allocated on the first call: 4P + 1 + offsets[P] ints and
 * 2P doubles); the exact path's partial sums are the context's, grown on
 * demand.  Errors: as gbs_mcmc_step_dev, and GBS_E_INVAL for rows above 30
 * clicks.
 */
int gbs_mcmc_da_step_dev(gbs_ctx *ctx, gbs_plan *plan, const double *u_dev, int32_t *modes_dev,
                         double *logp_hat_dev, double *logp_exact_dev, int32_t *accepted_dev);

/* Per-kernel timing.  With on = 1, every later launch on the context is
 * bracketed by HIP events recorded on the context's stream.  gbs_timing
 * synchronises the stream, writes the summed milliseconds per kernel group
 * since the last call into ms[GBS_TIMING_GROUPS] and the launch counts into
 * count[GBS_TIMING_GROUPS] (0 model build, 1 row set-up, 2 work-queue build,
 * 3 contour/cluster, 4 DFT and fit, 5 exact subsets, 6 adjoint of the fit and
 * DFT, 7 adjoint of the contour/cluster step, 8 adjoint per row and its
 * scatter into the mode pairs, 9 adjoint of the model build, 10 the second
 * pass of a forward call: re-tilted and escalated rows, their contour and
 * fits), then clears the record.  Either array may be NULL. */
#define GBS_TIMING_GROUPS 11
int gbs_set_timing(gbs_ctx *ctx, int on);
int gbs_timing(gbs_ctx *ctx, double *ms, int32_t *count);

/* The context's stream (hipStream_t) as void*. */
void *gbs_stream(gbs_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* GBS_H */
