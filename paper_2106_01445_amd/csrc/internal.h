// Internal declarations shared by the kernels and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "dd.h"
#include "../../include/gbs.h"

#define GBS_MAX_M 512          // modes supported by the model build
#define GBS_MAX_N_APPROX 128   // clicks per row on the approximate path (orders 1, 2)
#define GBS_MAX_N_ORDER3 64    // clicks per row at order 3
#define GBS_MAX_N_ORDER4 64    // clicks per row at order 4 (M(w) in LDS)
#define GBS_NSMALL 40          // rows up to this many clicks keep V and M(w) in LDS (contour)
#define GBS_RSLOTS 3           // R slots per adjoint work item of such a row (column units)
#define GBS_MAX_N_EXACT 30     // clicks per row on the exact path
#define GBS_KMAX 2048          // contour size cap
#define GBS_QCAP (GBS_KMAX / 2 + 1)
#define GBS_QCHUNK 8           // contour points per work item (default)
#define GBS_QCHUNK_MIN 4       // smallest tunable value (sizes the item lists)
#define GBS_QCHUNK_MAX 64      // largest tunable value
// Work-queue counters of a plan: [0..7] the forward and backward queues,
// [8..15] heads, [16..23] lengths and [24..31] offsets of the backward queues
// of the larger rows, one per XCD
#define GBS_NXCD 8
// contour points per adjoint work item: rows up to GBS_NSMALL clicks, larger rows
#define GBS_ADJ_CHUNK 64
#ifndef GBS_ADJ_CHUNK_BIG
#define GBS_ADJ_CHUNK_BIG 64
#endif
#define GBS_NCOUNTER (8 + 3 * GBS_NXCD)
#define GBS_CLUSTER_SEG 3      // triples per cluster work unit at order 3 (default)

struct alignas(16) cplx {
    double re, im;
};

// Model held on the device.  Q and Q^{-1} in double-double (hi and lo planes),
// row-major (2M)^2, xxpp.
struct DevModel {
    int M = 0;
    bool have = false;
    bool from_params = false;       // set_model (true) or set_covariance (false)
    double *q_hi = nullptr, *q_lo = nullptr;
    double *qi_hi = nullptr, *qi_lo = nullptr;
    double *chol_hi = nullptr, *chol_lo = nullptr;  // Cholesky factor L (lower), then scratch
    double *params = nullptr;       // U_re, U_im (M^2 each), r, eta (M each) on the device
    double *scal = nullptr;         // [0] log det Q, [1..2] det(Q)^{-1/2} as dd, [3] flag (non-PD)
    double *expd = nullptr;         // e^{-2r}, e^{2r} as dd (4M doubles) and sqrt(eta) dd (4M)
};

struct TimedLaunch {
    int group;
    hipEvent_t a, b;
};

struct gbs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    DevModel model;
    int num_cu = 0;
    int lds_per_block = 65536;  // largest LDS allocation of one workgroup (bytes)
    bool timing = false;
    bool deterministic = false;  // gradients summed in a fixed order (gbs_set_deterministic)
    std::vector<TimedLaunch> timeline;
    std::vector<hipEvent_t> event_pool;
    // per-kernel launch facts, queried once: a launch then makes no call besides
    // the kernel itself, so a step can be recorded into a HIP graph
    std::map<const void *, int> lds_limit, lds_static;
    std::map<std::pair<const void *, int>, int> occupancy;
    // partial sums of gbs_prob_exact_dev (grown on demand, freed with the context)
    double *ex_part = nullptr;
    long long ex_part_items = 0;
};

// Cached kernel queries (see gbs_ctx).
int func_static_lds(gbs_ctx *ctx, const void *f, int *bytes);
int func_lds_limit(gbs_ctx *ctx, const void *f, int bytes);
int func_occupancy(gbs_ctx *ctx, const void *f, int threads, int lds, int *blocks);

// Bracket a group of launches with events when timing is on (no-ops otherwise).
int timer_begin(gbs_ctx *ctx, int group);
void timer_end(gbs_ctx *ctx, int slot);
enum { TG_MODEL = 0, TG_PREP = 1, TG_ITEMS = 2, TG_CONTOUR = 3, TG_FIT = 4, TG_EXACT = 5,
       TG_ADJ_FIT = 6, TG_ADJ_CLUSTER = 7, TG_ADJ_ROWS = 8, TG_ADJ_MODEL = 9, TG_PASS2 = 10 };

// Per-row scalar results of the approximate path's set-up step.  status holds
// the failure bits (the row has no result); flags the informational bits that
// are reported with a valid result (GBS_PS_CONTOUR, GBS_PS_ESCALATED).
struct RowPlan {
    double rho, rconv, log_g_rho, logdet_a, log_pvac, log_rho;
    double err;   // estimated rounding error of log p_hat (sector transform and fits)
    double kbar;  // tilted mean photon number of the contour (the re-tilt sets it to the
                  // mean photon number of the sectors that carry the estimate)
    int K, status, nsec, flags;
};

// status bits that mean "no result" (the output is NaN); the others are
// informational
#define GBS_PS_FAILED (GBS_PS_FIT_NOCONV | GBS_PS_PIVOT | GBS_PS_CANCEL)
// internal flag (never reported): the row's contour is tilted afresh towards
// the sectors that carry its estimate and the row is run again
#define GBS_ROW_RETILT (1 << 8)
#define GBS_PS_PUBLIC 0xff

struct gbs_plan {
    gbs_ctx *ctx = nullptr;
    int M = 0;                            // modes of the model the plan was made for
    int P = 0, order = 0, prec = 0, max_n = 0;
    int nbig = 0;                         // rows with more than GBS_NSMALL clicks: perm[0..nbig)
    // tunable launch choices (gbs_plan_tune): cluster segment length of the
    // forward and adjoint work units, contour points per forward work item,
    // largest number of contour points per pass of the forward kernel
    int seg_fwd = GBS_CLUSTER_SEG, seg_adj = GBS_CLUSTER_SEG, qchunk = GBS_QCHUNK, gmax = 8;
    int max_n_small = 0;                  // largest click count among the other rows
    bool frozen = false;
    bool whole = false;                   // one row of every mode: contour at rho = 1 (click distribution)
    bool have_run = false;
    std::vector<int32_t> h_offsets, h_modes, h_perm, h_n;
    // device
    int32_t *d_offsets = nullptr, *d_modes = nullptr, *d_perm = nullptr;
    long long *d_voff = nullptr;          // offset of row p's eigenvectors in d_v
    double *d_alpha = nullptr;            // 2n per row, offset 2*offsets[p]
    double *d_v = nullptr;                // (2n)^2 per row
    RowPlan *d_rows = nullptr;            // P
    cplx *d_sw = nullptr;                 // (order+1) * QCAP per row: sums over clusters
    int32_t *d_items = nullptr;           // work items (row, chunk), 2 ints each
    int32_t *d_counter = nullptr;         // work queues: [0] end, [1] head (rows <= GBS_NSMALL),
                                          // [4] end, [5] head (larger rows); [2,3], [6,7] adjoint
    double *d_wbig = nullptr;             // 2 (2n)^2 per row: eigen-decomposition, then adjoint scratch
    cplx *d_mscr = nullptr;               // per-workgroup M(w) scratch of the larger rows
    int mscr_blocks = 0;                  // workgroups d_mscr serves
    int32_t *d_cluster_items = nullptr;   // per click count n: packed cluster units (a, b, c0, c1),
                                          // the forward's list, then the adjoint's
    int32_t *d_cluster_off = nullptr;     // [n] -> offset, count (2 ints); forward, then adjoint
                                          // at + 2 (max_n + 1)
    double *d_logp = nullptr;             // P (scratch when caller passes none)
    // two-stage chains: flags, lengths, exact status (P each), packed offsets
    // (P + 1) and rows (nnz); the exact path's p and log p (P each)
    int32_t *d_da = nullptr;
    double *d_da_x = nullptr;
    // deterministic gradients: the largest term into Psi (bit pattern), its scale
    unsigned long long *d_det = nullptr;
    int32_t *d_status = nullptr;          // P
    size_t v_total = 0;
    int max_items = 0;
    int n_cluster_items = 0;
    // gradient workspace (allocated by the first gradient call)
    bool have_adj = false;
    cplx *d_asw = nullptr;                // cotangents of the cluster sums, like d_sw
    int32_t *d_aitems = nullptr;          // backward work items (row, chunk)
    long long *d_roff = nullptr;          // per item: offset of its R in d_rscr
    int32_t *d_ritem0 = nullptr;          // per row: first backward item
    int32_t *d_axq = nullptr;             // backward items of the larger rows by XCD queue
    double *d_rscr = nullptr;             // per item: upper triangle of R
    double *d_qibar = nullptr;            // (2M)^2: Psi (adjoint of Q^{-1}), then sigma_bar
    double *d_qitmp = nullptr;            // (2M)^2 scratch
    double *d_grad = nullptr;             // 2M: grad r, grad eta
    double *d_dl = nullptr;               // P
    cplx *d_ascr = nullptr;               // per-workgroup adjoint scratch of the larger rows
    int ascr_blocks = 0;
    long long ascr_stride = 0;            // complex entries per workgroup
};

// error helpers ------------------------------------------------------------
int set_err(gbs_ctx *ctx, int code, const std::string &msg);
#define HIP_TRY(ctx, call)                                                          \
    do {                                                                            \
        hipError_t _e = (call);                                                     \
        if (_e != hipSuccess)                                                       \
            return set_err((ctx), -4, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

// kernels' host launchers ----------------------------------------------------
int model_build_dev(gbs_ctx *ctx, const double *sigma_dev, bool sync);
int approx_forward(gbs_ctx *ctx, gbs_plan *plan, double *logp_dev, int32_t *status_dev);
// status_dev[p] |= bits for every row (stream-ordered; NULL status: nothing)
int status_or(gbs_ctx *ctx, int P, int32_t *status_dev, int bits);
int exact_run(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, double *p,
              double *logp, double *kappa, int32_t *status);
int exact_lgs(int maxn);
int exact_scratch_init(int device);
double *exact_scratch(int device);
long long exact_noalloc_items();
int exact_launch(gbs_ctx *ctx, int P, const int32_t *d_off, const int32_t *d_modes, int maxn, double *d_part,
                 double *p_dev, double *logp_dev, double *kappa_dev, int32_t *status_dev);
int approx_backward(gbs_ctx *ctx, gbs_plan *plan, const double *dl_dev, const int32_t *status_dev,
                    double *grad_r_dev, double *grad_eta_dev);
int eig_rows(gbs_ctx *ctx, gbs_plan *plan);
int plain_contour(gbs_ctx *ctx, gbs_plan *plan);
int click_distribution_run(gbs_ctx *ctx, gbs_plan *pl, int nk, const int *ks_dev, double *pn_dev, double *pk_dev,
                           int32_t *status_dev);
int approx_forward_plain(gbs_ctx *ctx, gbs_plan *plan, double *logp_dev, int32_t *status_dev);
int plan_units(gbs_ctx *ctx, gbs_plan *plan);
