// Metropolis-Hastings sampling of click patterns with the order-j estimate as
// the target (Discussion: the approximate probabilities as the basis of a
// Markov chain Monte Carlo sampler; Metropolis et al. 1953, Hastings 1970).
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

__global__ void k_mh_propose(int P, int M, const int32_t *__restrict__ offsets, const int32_t *__restrict__ cur,
                             const double *__restrict__ u, int32_t *__restrict__ prop)
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
    const double u0 = fmin(fmax(u[3 * p], 0.0), 1.0), u1 = fmin(fmax(u[3 * p + 1], 0.0), 1.0);
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

}  // namespace

int mcmc_step(gbs_ctx *ctx, gbs_plan *pl, const double *u, int32_t *modes, double *logp, int32_t *accepted)
{
    if (pl->P == 0) return 0;
    const int P = pl->P, blocks = (P + 255) / 256;
    hipLaunchKernelGGL(k_mh_propose, dim3(blocks), dim3(256), 0, ctx->stream, P, pl->M, pl->d_offsets, modes, u,
                       pl->d_modes);
    HIP_TRY(ctx, hipGetLastError());
    if (int rc = approx_forward(ctx, pl, pl->d_logp, pl->d_status)) return rc;
    hipLaunchKernelGGL(k_mh_accept, dim3(blocks), dim3(256), 0, ctx->stream, P, pl->M, pl->d_offsets, pl->d_modes,
                       pl->d_logp, pl->d_status, u, modes, logp, accepted);
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}
