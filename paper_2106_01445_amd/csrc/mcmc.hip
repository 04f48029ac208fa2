// Metropolis-Hastings sampling of click patterns (Discussion: the approximate
// probabilities as the basis of a Markov chain Monte Carlo sampler;
// Metropolis et al. 1953, Hastings 1970): with the order-j estimate as the
// target (below), and two-stage chains with the exact p as the target and the
// estimate screening the proposals (further below).
//
// Every chain keeps its number of clicks n.  One step, for all chains at once:
//   1. proposal (k_mh_propose, one thread per chain): the clicked mode at
//      position i = floor(u0 n) of the row is replaced by the k-th unclicked
//      mode in increasing order, k = floor(u1 (M - n)); the row is kept
//      ascending.  The move is symmetric (each of the n (M - n) swaps has the
//      same probability in both directions), so the acceptance ratio is the
//      ratio of the targets;
//   2. log p_hat of every proposal: the plan's forward (approx_forward) on the
//      proposals, written into the plan's own mode array;
//   3. acceptance (k_mh_accept): accept when log p_hat(proposal) >=
//      log p_hat(current) or u2 < exp(difference); a proposal whose estimate
//      failed (NaN) is rejected.  Accepted rows and their log p_hat replace the
//      chain's state.
// Rows with n = 0 or n = M have no move: the proposal is the current row.  A
// chain whose row is malformed (modes not strictly ascending in [0, M)) is
// not moved and reports -1 in accepted; its slot of the plan is evaluated on
// the row 0..n-1 so that no kernel reads outside the model.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace {

// a chain's row is usable when its modes are strictly ascending in [0, M)
__device__ __forceinline__ bool row_ok(const int32_t *row, int n, int M)
{
    for (int i = 0; i < n; ++i)
        if (row[i] < 0 || row[i] >= M || (i > 0 && row[i] <= row[i - 1])) return false;
    return true;
}

// (us uniforms per chain, the first two for the swap)
__global__ void k_mh_propose(int P, int M, const int32_t *__restrict__ offsets, const int32_t *__restrict__ cur,
                             const double *__restrict__ u, int us, int32_t *__restrict__ prop)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int o = offsets[p], n = offsets[p + 1] - o;
    if (n == 0 || n == M || !row_ok(cur + o, n, M)) {
        // (no move; a malformed row is replaced by 0..n-1 for the evaluation
        // and the chain is not moved)
        const bool ok = row_ok(cur + o, n, M);
        for (int i = 0; i < n; ++i) prop[o + i] = ok ? cur[o + i] : i;
        return;
    }
    // (uniforms outside [0, 1), NaN included, are clamped into range)
    const double u0 = fmin(fmax(u[us * p], 0.0), 1.0), u1 = fmin(fmax(u[us * p + 1], 0.0), 1.0);
    const int i = max(0, min(n - 1, (int)(u0 * n)));
    const int k = max(0, min(M - n - 1, (int)(u1 * (M - n))));
    // the k-th mode (from 0) that the row does not hold
    int m = 0, seen = -1, j = 0;
    for (m = 0; m < M; ++m) {
        while (j < n && cur[o + j] < m) ++j;
        if (j < n && cur[o + j] == m) continue;
        if (++seen == k) break;
    }
    // the row without position i, with m inserted in order
    int w = o;
    bool put = false;
    for (int r = 0; r < n; ++r) {
        if (r == i) continue;
        const int v = cur[o + r];
        if (!put && m < v) {
            prop[w++] = m;
            put = true;
        }
        prop[w++] = v;
    }
    if (!put) prop[w++] = m;
}

__global__ void k_mh_accept(int P, int M, const int32_t *__restrict__ offsets, const int32_t *__restrict__ prop,
                            const double *__restrict__ lp_prop, const int32_t *__restrict__ st_prop,
                            const double *__restrict__ u, int32_t *__restrict__ cur, double *__restrict__ lp_cur,
                            int32_t *__restrict__ accepted)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int o = offsets[p], n = offsets[p + 1] - o;
    if (!row_ok(cur + o, n, M)) {
        if (accepted) accepted[p] = -1;
        return;
    }
    const double d = lp_prop[p] - lp_cur[p];
    const bool ok = (st_prop[p] & GBS_PS_FAILED) == 0 && !isnan(lp_prop[p]);
    // (a chain whose current value is NaN moves to any proposal with a value)
    const bool acc = ok && (isnan(lp_cur[p]) || d >= 0.0 || u[3 * p + 2] < exp(d));
    if (acc) {
        for (int i = 0; i < n; ++i) cur[o + i] = prop[o + i];
        lp_cur[p] = lp_prop[p];
    }
    if (accepted) accepted[p] = acc ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Two-stage (delayed-acceptance) steps, Christen & Fox 2005: the order-j
// estimate screens each proposal (first stage, as above), the exact
// probability corrects the proposals that pass (second stage: accept with
// min(1, [p(new) p_hat(old)] / [p(old) p_hat(new)])), so that the chains'
// stationary distribution is the exact p (restricted to n clicks) while only
// the screened proposals pay for an exact evaluation.  Four uniforms per
// chain: the swap (two), the first stage, the second.  A chain whose current
// values are not both finite takes any proposal whose two values are.
// ---------------------------------------------------------------------------
__global__ void k_da_stage1(int P, int M, const int32_t *__restrict__ offsets, const double *__restrict__ lh_prop,
                            const int32_t *__restrict__ st_prop, const double *__restrict__ u,
                            const int32_t *__restrict__ cur, const double *__restrict__ lh_cur,
                            const double *__restrict__ le_cur, int32_t *__restrict__ flag, int32_t *__restrict__ len)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int o = offsets[p], n = offsets[p + 1] - o;
    if (!row_ok(cur + o, n, M)) {
        flag[p] = -1;
        len[p] = 0;
        return;
    }
    const double h1 = lh_prop[p], dh = h1 - lh_cur[p];
    const bool bad_cur = !(isfinite(lh_cur[p]) && isfinite(le_cur[p]));
    const bool pass = (st_prop[p] & GBS_PS_FAILED) == 0 && !isnan(h1) &&
                      (bad_cur || dh >= 0.0 || u[4 * p + 2] < exp(dh));
    flag[p] = pass ? 1 : 0;
    len[p] = pass ? n : 0;
}

// exclusive prefix sum of len[0..P) into off[0..P] (one workgroup of 1024:
// each thread sums a contiguous run, the run totals are scanned in LDS)
__global__ __launch_bounds__(1024) void k_da_scan(int P, const int32_t *__restrict__ len, int32_t *__restrict__ off)
{
    __shared__ int part[1024];
    const int t = threadIdx.x, per = (P + 1023) / 1024;
    const int b = min(P, t * per), e = min(P, b + per);
    int s = 0;
    for (int i = b; i < e; ++i) s += len[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int acc = part[t] - s;
    for (int i = b; i < e; ++i) {
        off[i] = acc;
        acc += len[i];
    }
    if (t == 1023) off[P] = part[1023];
}

// the screened proposals' rows, packed (the other chains' rows empty)
__global__ void k_da_gather(int P, const int32_t *__restrict__ offsets, const int32_t *__restrict__ prop,
                            const int32_t *__restrict__ flag, const int32_t *__restrict__ off,
                            int32_t *__restrict__ dst)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || flag[p] != 1) return;
    const int o = offsets[p], n = offsets[p + 1] - o, d = off[p];
    for (int i = 0; i < n; ++i) dst[d + i] = prop[o + i];
}

__global__ void k_da_stage2(int P, const int32_t *__restrict__ offsets, const int32_t *__restrict__ prop,
                            const double *__restrict__ lh_prop, const double *__restrict__ le_prop,
                            const int32_t *__restrict__ st_ex, const double *__restrict__ u,
                            const int32_t *__restrict__ flag, int32_t *__restrict__ cur, double *__restrict__ lh_cur,
                            double *__restrict__ le_cur, int32_t *__restrict__ accepted)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int f = flag[p];
    int code = f < 0 ? -1 : 0;
    if (f == 1) {
        const double h1 = lh_prop[p], e1 = le_prop[p];
        const bool ok = (st_ex[p] & GBS_PS_FAILED) == 0 && !isnan(e1);
        const bool bad_cur = !(isfinite(lh_cur[p]) && isfinite(le_cur[p]));
        bool acc;
        if (bad_cur) {
            acc = ok && isfinite(h1) && isfinite(e1);
        } else {
            const double r = (e1 - le_cur[p]) - (h1 - lh_cur[p]);
            acc = ok && (r >= 0.0 || u[4 * p + 3] < exp(r));
        }
        code = acc ? 1 : 2;
        if (acc) {
            const int o = offsets[p], n = offsets[p + 1] - o;
            for (int i = 0; i < n; ++i) cur[o + i] = prop[o + i];
            lh_cur[p] = h1;
            le_cur[p] = e1;
        }
    }
    if (accepted) accepted[p] = code;
}

}  // namespace

int mcmc_step(gbs_ctx *ctx, gbs_plan *pl, const double *u, int32_t *modes, double *logp, int32_t *accepted)
{
    if (pl->P == 0) return 0;
    const int P = pl->P, blocks = (P + 255) / 256;
    hipLaunchKernelGGL(k_mh_propose, dim3(blocks), dim3(256), 0, ctx->stream, P, pl->M, pl->d_offsets, modes, u, 3,
                       pl->d_modes);
    HIP_TRY(ctx, hipGetLastError());
    if (int rc = approx_forward(ctx, pl, pl->d_logp, pl->d_status)) return rc;
    hipLaunchKernelGGL(k_mh_accept, dim3(blocks), dim3(256), 0, ctx->stream, P, pl->M, pl->d_offsets, pl->d_modes,
                       pl->d_logp, pl->d_status, u, modes, logp, accepted);
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}

// One two-stage step of every chain of a plan, in the plan's workspace
// pl->d_da (flags, lengths, exact status, packed offsets and rows) and
// pl->d_da_x (the exact path's p and log p), allocated by the caller.
int mcmc_da_step(gbs_ctx *ctx, gbs_plan *pl, const double *u, int32_t *modes, double *logp_hat, double *logp_exact,
                 int32_t *accepted)
{
    const int P = pl->P;
    if (P == 0) return 0;
    int32_t *flag = pl->d_da, *len = flag + P, *st_ex = len + P, *off = st_ex + P, *pk = off + P + 1;
    double *px = pl->d_da_x, *lx = px + P;
    const int blocks = (P + 255) / 256;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(k_mh_propose, dim3(blocks), dim3(256), 0, st, P, pl->M, pl->d_offsets, modes, u, 4,
                       pl->d_modes);
    HIP_TRY(ctx, hipGetLastError());
    if (int rc = approx_forward(ctx, pl, pl->d_logp, pl->d_status)) return rc;
    hipLaunchKernelGGL(k_da_stage1, dim3(blocks), dim3(256), 0, st, P, pl->M, pl->d_offsets, pl->d_logp,
                       pl->d_status, u, modes, logp_hat, logp_exact, flag, len);
    hipLaunchKernelGGL(k_da_scan, dim3(1), dim3(1024), 0, st, P, len, off);
    hipLaunchKernelGGL(k_da_gather, dim3(blocks), dim3(256), 0, st, P, pl->d_offsets, pl->d_modes, flag, off, pk);
    HIP_TRY(ctx, hipGetLastError());
    if (int rc = gbs_prob_exact_dev(ctx, P, off, pk, pl->max_n, px, lx, nullptr, st_ex)) return rc;
    hipLaunchKernelGGL(k_da_stage2, dim3(blocks), dim3(256), 0, st, P, pl->d_offsets, pl->d_modes, pl->d_logp, lx,
                       st_ex, u, flag, modes, logp_hat, logp_exact, accepted);
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}
