// C ABI of the click-probability library (declared in include/gbs.h).
// Argument validation, device buffers, plans; the kernels live in model.hip,
// approx.hip, exact.hip and grad.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "../../include/gbs.h"
#include "internal.h"

int model_alloc(gbs_ctx *ctx, int M);
void model_release(gbs_ctx *ctx);

int set_err(gbs_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

static hipEvent_t pool_event(gbs_ctx *ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int func_static_lds(gbs_ctx *ctx, const void *f, int *bytes)
{
    auto it = ctx->lds_static.find(f);
    if (it == ctx->lds_static.end()) {
        hipFuncAttributes fa;
        HIP_TRY(ctx, hipFuncGetAttributes(&fa, f));
        it = ctx->lds_static.emplace(f, (int)fa.sharedSizeBytes).first;
    }
    *bytes = it->second;
    return 0;
}

int func_lds_limit(gbs_ctx *ctx, const void *f, int bytes)
{
    auto it = ctx->lds_limit.find(f);
    if (it != ctx->lds_limit.end() && it->second >= bytes) return 0;
    HIP_TRY(ctx, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    ctx->lds_limit[f] = bytes;
    return 0;
}

int func_occupancy(gbs_ctx *ctx, const void *f, int threads, int lds, int *blocks)
{
    const auto key = std::make_pair(f, lds * 2048 + threads / 64);
    auto it = ctx->occupancy.find(key);
    if (it == ctx->occupancy.end()) {
        int occ = 0;
        HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, threads, lds));
        it = ctx->occupancy.emplace(key, occ < 1 ? 1 : occ).first;
    }
    *blocks = it->second;
    return 0;
}

int timer_begin(gbs_ctx *ctx, int group)
{
    if (!ctx->timing) return -1;
    hipEvent_t a = pool_event(ctx), b = pool_event(ctx);
    if (!a || !b) return -1;
    (void)hipEventRecord(a, ctx->stream);
    ctx->timeline.push_back(TimedLaunch{group, a, b});
    return (int)ctx->timeline.size() - 1;
}

void timer_end(gbs_ctx *ctx, int slot)
{
    if (slot < 0) return;
    (void)hipEventRecord(ctx->timeline[slot].b, ctx->stream);
}

namespace {

int check_csr(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int M,
              int max_n)
{
    if (P < 0) return set_err(ctx, GBS_E_INVAL, "P must be >= 0");
    if (P > 0 && !offsets) return set_err(ctx, GBS_E_INVAL, "offsets is NULL");
    if (P == 0) return GBS_OK;
    if (offsets[0] != 0) return set_err(ctx, GBS_E_INVAL, "offsets[0] must be 0");
    if (offsets[P] > 0 && !modes) return set_err(ctx, GBS_E_INVAL, "modes is NULL");
    for (int p = 0; p < P; ++p) {
        int n = offsets[p + 1] - offsets[p];
        if (n < 0)
            return set_err(ctx, GBS_E_INVAL, "offsets must be non-decreasing (row " +
                                                 std::to_string(p) + ")");
        if (n > max_n)
            return set_err(ctx, GBS_E_INVAL, "row " + std::to_string(p) + " has " +
                                                 std::to_string(n) + " clicks; at most " +
                                                 std::to_string(max_n) + " supported");
        for (int i = offsets[p]; i < offsets[p + 1]; ++i) {
            if (modes[i] < 0 || modes[i] >= M)
                return set_err(ctx, GBS_E_INVAL, "row " + std::to_string(p) +
                                                     ": mode out of range [0, M)");
            if (i > offsets[p] && modes[i] <= modes[i - 1])
                return set_err(ctx, GBS_E_INVAL, "row " + std::to_string(p) +
                                                     ": modes must be strictly ascending");
        }
    }
    return GBS_OK;
}

void plan_free_dev(gbs_plan *pl)
{
    void *ptrs[] = {pl->d_offsets, pl->d_modes, pl->d_perm, pl->d_voff, pl->d_alpha,
                    pl->d_v, pl->d_rows, pl->d_sw, pl->d_items, pl->d_counter,
                    pl->d_cluster_items, pl->d_cluster_off, pl->d_logp, pl->d_status,
                    pl->d_asw, pl->d_aitems, pl->d_roff, pl->d_ritem0, pl->d_axq, pl->d_rscr,
                    pl->d_qibar, pl->d_qitmp, pl->d_grad, pl->d_dl, pl->d_wbig, pl->d_mscr,
                    pl->d_ascr, pl->d_da, pl->d_da_x, pl->d_det};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

// Cluster work units for rows with n clicks (orders 2 and 3), one packed int
// each: a | b << 8 | c0 << 16 | c1 << 24.  A unit is the pair a < b plus the
// triples (a, b, c) for c in [c0, c1); the unit with c0 = b + 1 also carries the
// pair itself.  At order 3 the range c > b is cut into segments of
// GBS_CLUSTER_SEG, so that no thread of a slot group waits for one long pair;
// units are listed by decreasing length, then (b, c0, a) for the forward
// (neighbouring lanes read neighbouring blocks of M(w)) or (b - a, c0 - b, a)
// for the adjoint (neighbouring lanes hold distinct a, b and c, so their
// scatters into Z(w) never meet in one instruction), so that a strided
// assignment to threads is balanced.
void cluster_units(int n, int order, int seg, bool adjoint, std::vector<int32_t> &out)
{
    struct U { int a, b, c0, c1; };
    std::vector<U> u;
    for (int b = 1; b < n; ++b)
        for (int a = 0; a < b; ++a) {
            if (order < 3 || b == n - 1) {
                u.push_back({a, b, b + 1, b + 1});
                continue;
            }
            for (int c0 = b + 1; c0 < n; c0 += seg)
                u.push_back({a, b, c0, std::min(c0 + seg, n)});
        }
    std::stable_sort(u.begin(), u.end(), [adjoint](const U &x, const U &y) {
        if (x.c1 - x.c0 != y.c1 - y.c0) return x.c1 - x.c0 > y.c1 - y.c0;
        if (adjoint) {
            if (x.b - x.a != y.b - y.a) return x.b - x.a < y.b - y.a;
            if (x.c0 - x.b != y.c0 - y.b) return x.c0 - x.b < y.c0 - y.b;
            return x.a < y.a;
        }
        if (x.b != y.b) return x.b < y.b;
        if (x.c0 != y.c0) return x.c0 < y.c0;
        return x.a < y.a;
    });
    for (const U &x : u)
        out.push_back((int32_t)((unsigned)x.a | (unsigned)x.b << 8 | (unsigned)x.c0 << 16 |
                                (unsigned)x.c1 << 24));
}

// Quadruple work units of a row with n <= 40 clicks: (a, b, c; d0 .. d0+len-1)
// for a < b < c < d, len <= min(seg, 15), packed a | b << 6 | c << 12 |
// d0 << 18 | len << 24, ordered by decreasing length, then (b, c, d0, a), so
// that neighbouring lanes hold consecutive a of the same (b, c, d0).
void quad_units(int n, int seg, std::vector<int32_t> &out)
{
    struct U { int a, b, c, d0, len; };
    std::vector<U> u;
    const int sg = std::min(seg, 15);
    for (int c = 2; c < n - 1; ++c)
        for (int b = 1; b < c; ++b)
            for (int a = 0; a < b; ++a)
                for (int d0 = c + 1; d0 < n; d0 += sg) u.push_back({a, b, c, d0, std::min(sg, n - d0)});
    std::stable_sort(u.begin(), u.end(), [](const U &x, const U &y) {
        if (x.len != y.len) return x.len > y.len;
        if (x.b != y.b) return x.b < y.b;
        if (x.c != y.c) return x.c < y.c;
        if (x.d0 != y.d0) return x.d0 < y.d0;
        return x.a < y.a;
    });
    for (const U &x : u)
        out.push_back((int32_t)((unsigned)x.a | (unsigned)x.b << 6 | (unsigned)x.c << 12 | (unsigned)x.d0 << 18 |
                                (unsigned)x.len << 24));
}

template <class T>
int dev_alloc(gbs_ctx *ctx, T **p, size_t count)
{
    if (count == 0) count = 1;
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return set_err(ctx, GBS_E_NOMEM, "device allocation of " +
                                             std::to_string(count * sizeof(T)) + " bytes failed");
    }
    return 0;
}

}  // namespace

// (Re)build the cluster work units of a plan for its segment lengths: the
// forward list, the adjoint list, then (order 4) the quadruple list; offsets
// [n] -> (offset, count) for the forward at d_cluster_off, for the adjoint at
// d_cluster_off + 2 (max_n + 1), for the quadruples at d_cluster_off +
// 4 (max_n + 1).
int plan_units(gbs_ctx *ctx, gbs_plan *pl)
{
    const int nm = pl->max_n;
    std::vector<int32_t> citems, coff(6 * (nm + 1), 0);
    for (int pass = 0; pass < 3; ++pass)
        for (int n = 0; n <= nm; ++n) {
            int32_t *o = coff.data() + 2 * (nm + 1) * pass + 2 * n;
            o[0] = (int32_t)citems.size();
            if (pass < 2 && pl->order >= 2)
                cluster_units(n, pl->order, pass ? pl->seg_adj : pl->seg_fwd, pass == 1, citems);
            if (pass == 2 && pl->order >= 4) quad_units(n, pl->seg_fwd, citems);
            o[1] = (int32_t)citems.size() - o[0];
        }
    pl->n_cluster_items = (int)citems.size();
    if (pl->d_cluster_items) (void)hipFree(pl->d_cluster_items);
    if (pl->d_cluster_off) (void)hipFree(pl->d_cluster_off);
    pl->d_cluster_items = nullptr;
    pl->d_cluster_off = nullptr;
    int e = dev_alloc(ctx, &pl->d_cluster_items, citems.size());
    e = e ? e : dev_alloc(ctx, &pl->d_cluster_off, coff.size());
    if (e) return e;
    HIP_TRY(ctx, hipMemcpyAsync(pl->d_cluster_items, citems.data(), citems.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(pl->d_cluster_off, coff.data(), coff.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return 0;
}

long long adj_pair_scratch(int n);

// Gradient workspace of a plan, allocated on first use.
int adj_workspace(gbs_ctx *ctx, gbs_plan *pl)
{
    if (pl->have_adj) return 0;
    const int P = pl->P, M = pl->M, order = pl->order;
    const int chunks_s = (GBS_QCAP + GBS_ADJ_CHUNK - 1) / GBS_ADJ_CHUNK;
    const int chunks_b = (GBS_QCAP + GBS_ADJ_CHUNK_BIG - 1) / GBS_ADJ_CHUNK_BIG;
    const int chunks = pl->nbig > 0 ? std::max(chunks_s, chunks_b) : chunks_s;
    size_t rtot = 0;
    for (int p = 0; p < P; ++p) {
        const size_t N = 2 * (size_t)pl->h_n[p];
        rtot += (N * (N + 1) / 2) * (pl->h_n[p] > GBS_NSMALL ? chunks_b : chunks_s * GBS_RSLOTS);
    }
    const size_t D = 2 * (size_t)M;
    int e = 0;
    e = e ? e : dev_alloc(ctx, &pl->d_asw, (size_t)P * (order + 1) * GBS_QCAP);
    e = e ? e : dev_alloc(ctx, &pl->d_aitems, 2 * (size_t)P * chunks);
    e = e ? e : dev_alloc(ctx, &pl->d_roff, (size_t)P * chunks);
    e = e ? e : dev_alloc(ctx, &pl->d_ritem0, (size_t)P);
    e = e ? e : dev_alloc(ctx, &pl->d_axq, (size_t)P * chunks);
    e = e ? e : dev_alloc(ctx, &pl->d_rscr, rtot);
    e = e ? e : dev_alloc(ctx, &pl->d_qibar, D * D);
    e = e ? e : dev_alloc(ctx, &pl->d_qitmp, D * D);
    e = e ? e : dev_alloc(ctx, &pl->d_det, 2);
    if (!pl->d_grad) e = e ? e : dev_alloc(ctx, &pl->d_grad, D);
    if (pl->nbig > 0) {
        // larger rows, per workgroup: at order 2 the pair blocks of Z(w) as
        // 16 x 16 planes; otherwise M(w), the pair blocks of Z(w) at order 1 and
        // Z V
        const long long nb = pl->max_n, npb = nb * (nb - 1) / 2;
        pl->ascr_stride = order == 2 ? adj_pair_scratch((int)nb)
                                     : 3 * nb + 4 * npb + (order <= 1 ? 4 * npb : 0) + 2 * nb * (32 * ((2 * nb + 31) / 32));
        pl->ascr_blocks = 2 * ctx->num_cu;
        e = e ? e : dev_alloc(ctx, &pl->d_ascr, (size_t)pl->ascr_blocks * pl->ascr_stride);
    }
    if (e) return e;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    pl->have_adj = true;
    return 0;
}

extern "C" {

int gbs_create(gbs_ctx **out, int hip_device, void *hip_stream)
{
    if (!out) return GBS_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return GBS_E_HIP;
    if (hip_device < 0 || hip_device >= ndev) return GBS_E_INVAL;
    gbs_ctx *ctx = new (std::nothrow) gbs_ctx();
    if (!ctx) return GBS_E_NOMEM;
    ctx->device = hip_device;
    if (hipSetDevice(hip_device) != hipSuccess) {
        delete ctx;
        return GBS_E_HIP;
    }
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&ctx->stream) != hipSuccess) {
            delete ctx;
            return GBS_E_HIP;
        }
        ctx->own_stream = true;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) {
        ctx->num_cu = prop.multiProcessorCount;
        ctx->lds_per_block = (int)prop.sharedMemPerBlock;
    }
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, hip_device) == hipSuccess &&
        optin > ctx->lds_per_block)
        ctx->lds_per_block = optin;
    if (ctx->num_cu <= 0) ctx->num_cu = 256;
    // the device address of the fixed scratch of gbs_prob_exact_dev_noalloc
    // (once per device; this device is current)
    if (exact_scratch_init(hip_device) != 0) {
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return GBS_E_HIP;
    }
    *out = ctx;
    return GBS_OK;
}

int gbs_destroy(gbs_ctx *ctx)
{
    if (!ctx) return GBS_E_INVAL;
    (void)hipSetDevice(ctx->device);
    model_release(ctx);
    for (const TimedLaunch &t : ctx->timeline) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->ex_part) (void)hipFree(ctx->ex_part);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return GBS_OK;
}

const char *gbs_last_error(const gbs_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void *gbs_stream(gbs_ctx *ctx) { return ctx ? (void *)ctx->stream : nullptr; }

int gbs_set_model(gbs_ctx *ctx, int M, const double *U_re, const double *U_im, const double *r,
                  const double *eta)
{
    if (!ctx) return GBS_E_INVAL;
    if (M < 1 || M > GBS_MAX_M) return set_err(ctx, GBS_E_INVAL, "M must be in [1, 512]");
    if (!U_re || !U_im || !r || !eta) return set_err(ctx, GBS_E_INVAL, "NULL model array");
    for (int i = 0; i < M; ++i) {
        if (!(r[i] >= 0.0) || !std::isfinite(r[i]))
            return set_err(ctx, GBS_E_INVAL, "r must be finite and >= 0");
        if (!(eta[i] >= 0.0 && eta[i] <= 1.0))
            return set_err(ctx, GBS_E_INVAL, "eta must lie in [0, 1]");
    }
    for (long i = 0; i < (long)M * M; ++i)
        if (!std::isfinite(U_re[i]) || !std::isfinite(U_im[i]))
            return set_err(ctx, GBS_E_INVAL, "U must be finite");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int rc = model_alloc(ctx, M);
    if (rc) return rc;
    DevModel &m = ctx->model;
    size_t MM = (size_t)M * M;
    HIP_TRY(ctx, hipMemcpyAsync(m.params, U_re, MM * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(m.params + MM, U_im, MM * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(m.params + 2 * MM, r, M * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(m.params + 2 * MM + M, eta, M * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    m.from_params = true;
    return model_build_dev(ctx, nullptr, true);
}

int gbs_set_model_dev(gbs_ctx *ctx, int M, const double *U_re_dev, const double *U_im_dev,
                      const double *r_dev, const double *eta_dev)
{
    if (!ctx) return GBS_E_INVAL;
    if (M < 1 || M > GBS_MAX_M) return set_err(ctx, GBS_E_INVAL, "M must be in [1, 512]");
    if (!U_re_dev || !U_im_dev || !r_dev || !eta_dev) return set_err(ctx, GBS_E_INVAL, "NULL model array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int rc = model_alloc(ctx, M);
    if (rc) return rc;
    DevModel &m = ctx->model;
    size_t MM = (size_t)M * M;
    HIP_TRY(ctx, hipMemcpyAsync(m.params, U_re_dev, MM * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(m.params + MM, U_im_dev, MM * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(m.params + 2 * MM, r_dev, M * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(m.params + 2 * MM + M, eta_dev, M * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    m.from_params = true;
    return model_build_dev(ctx, nullptr, false);
}

int gbs_set_timing(gbs_ctx *ctx, int on)
{
    if (!ctx) return GBS_E_INVAL;
    ctx->timing = on != 0;
    return GBS_OK;
}

int gbs_timing(gbs_ctx *ctx, double *ms, int32_t *count)
{
    if (!ctx) return GBS_E_INVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    double acc[GBS_TIMING_GROUPS] = {};
    int32_t cnt[GBS_TIMING_GROUPS] = {};
    for (const TimedLaunch &t : ctx->timeline) {
        float e = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&e, t.a, t.b));
        acc[t.group] += e;
        cnt[t.group] += 1;
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    ctx->timeline.clear();
    for (int i = 0; i < GBS_TIMING_GROUPS; ++i) {
        if (ms) ms[i] = acc[i];
        if (count) count[i] = cnt[i];
    }
    return GBS_OK;
}

int gbs_set_covariance(gbs_ctx *ctx, int M, const double *sigma)
{
    if (!ctx) return GBS_E_INVAL;
    if (M < 1 || M > GBS_MAX_M) return set_err(ctx, GBS_E_INVAL, "M must be in [1, 512]");
    if (!sigma) return set_err(ctx, GBS_E_INVAL, "sigma is NULL");
    long D = 2L * M;
    for (long i = 0; i < D; ++i)
        for (long j = 0; j < D; ++j) {
            if (!std::isfinite(sigma[i * D + j])) return set_err(ctx, GBS_E_INVAL, "sigma must be finite");
            if (sigma[i * D + j] != sigma[j * D + i]) return set_err(ctx, GBS_E_INVAL, "sigma must be symmetric");
        }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int rc = model_alloc(ctx, M);
    if (rc) return rc;
    double *d_sigma = nullptr;
    rc = dev_alloc(ctx, &d_sigma, D * D);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(d_sigma, sigma, D * D * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(d_sigma);
        return set_err(ctx, GBS_E_HIP, hipGetErrorString(e));
    }
    ctx->model.from_params = false;
    rc = model_build_dev(ctx, d_sigma, true);
    (void)hipFree(d_sigma);
    return rc;
}

int gbs_get_model(gbs_ctx *ctx, double *q_inv, double *logdet_q)
{
    if (!ctx) return GBS_E_INVAL;
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    long D = 2L * ctx->model.M;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (q_inv)
        HIP_TRY(ctx, hipMemcpyAsync(q_inv, ctx->model.qi_hi, D * D * sizeof(double),
                                    hipMemcpyDeviceToHost, ctx->stream));
    if (logdet_q)
        HIP_TRY(ctx, hipMemcpyAsync(logdet_q, ctx->model.scal, sizeof(double),
                                    hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return GBS_OK;
}

int gbs_plan_create(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int order,
                    int prec, gbs_plan **out)
{
    if (!ctx || !out) return GBS_E_INVAL;
    *out = nullptr;
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    if (order < 1 || order > 4) return set_err(ctx, GBS_E_INVAL, "order must be 1, 2, 3 or 4");
    if (prec != GBS_PREC_FP64 && prec != GBS_PREC_MIXED)
        return set_err(ctx, GBS_E_INVAL, "prec must be GBS_PREC_FP64 or GBS_PREC_MIXED");
    int rc = check_csr(ctx, P, offsets, modes, ctx->model.M,
                       order == 4 ? GBS_MAX_N_ORDER4 : order == 3 ? GBS_MAX_N_ORDER3 : GBS_MAX_N_APPROX);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    gbs_plan *pl = new (std::nothrow) gbs_plan();
    if (!pl) return set_err(ctx, GBS_E_NOMEM, "host allocation failed");
    pl->ctx = ctx;
    pl->M = ctx->model.M;
    pl->P = P;
    pl->order = order;
    pl->prec = prec;
    int nnz = P > 0 ? offsets[P] : 0;
    pl->h_offsets.assign(offsets, offsets + P + 1);
    if (P == 0) pl->h_offsets.assign(1, 0);
    pl->h_modes.assign(modes, modes + nnz);
    pl->h_n.resize(P);
    std::vector<long long> voff(P);
    long long vt = 0;
    for (int p = 0; p < P; ++p) {
        int n = offsets[p + 1] - offsets[p];
        pl->h_n[p] = n;
        pl->max_n = std::max(pl->max_n, n);
        if (n > GBS_NSMALL) pl->nbig += 1;
        else pl->max_n_small = std::max(pl->max_n_small, n);
        voff[p] = vt;
        vt += 4LL * n * n;
    }
    pl->v_total = (size_t)vt;
    // rows by decreasing cost (click count), stable
    pl->h_perm.resize(P);
    std::iota(pl->h_perm.begin(), pl->h_perm.end(), 0);
    std::stable_sort(pl->h_perm.begin(), pl->h_perm.end(),
                     [&](int a, int b) { return pl->h_n[a] > pl->h_n[b]; });
    long long max_items = (long long)P * ((GBS_QCAP + GBS_QCHUNK_MIN - 1) / GBS_QCHUNK_MIN);
    pl->max_items = (int)max_items;
    int e = 0;
    e = e ? e : dev_alloc(ctx, &pl->d_offsets, P + 1);
    e = e ? e : dev_alloc(ctx, &pl->d_modes, nnz);
    e = e ? e : dev_alloc(ctx, &pl->d_perm, P);
    e = e ? e : dev_alloc(ctx, &pl->d_voff, P);
    e = e ? e : dev_alloc(ctx, &pl->d_alpha, 2 * (size_t)nnz);
    e = e ? e : dev_alloc(ctx, &pl->d_v, pl->v_total);
    e = e ? e : dev_alloc(ctx, &pl->d_rows, P);
    e = e ? e : dev_alloc(ctx, &pl->d_sw, (size_t)P * (order + 1) * GBS_QCAP);
    e = e ? e : dev_alloc(ctx, &pl->d_items, 2 * (size_t)max_items);
    e = e ? e : dev_alloc(ctx, &pl->d_counter, GBS_NCOUNTER);
    e = e ? e : dev_alloc(ctx, &pl->d_wbig, 2 * pl->v_total);
    if (pl->nbig > 0) {
        // M(w) of rows whose blocks do not fit in LDS: one copy per workgroup
        const long long ms = 2LL * pl->max_n * pl->max_n + 5LL * pl->max_n;
        if (16 * ms + 16 * 64 > (long long)ctx->lds_per_block - 8 * 1024) {
            pl->mscr_blocks = 2 * ctx->num_cu;
            e = e ? e : dev_alloc(ctx, &pl->d_mscr, (size_t)pl->mscr_blocks * ms);
        }
    }
    e = e ? e : dev_alloc(ctx, &pl->d_logp, P);
    e = e ? e : dev_alloc(ctx, &pl->d_status, P);
    if (e) {
        plan_free_dev(pl);
        delete pl;
        return e;
    }
    hipStream_t st = ctx->stream;
    auto cp = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    hipError_t he = hipSuccess;
    if (he == hipSuccess) he = cp(pl->d_offsets, pl->h_offsets.data(), (P + 1) * sizeof(int32_t));
    if (he == hipSuccess) he = cp(pl->d_modes, pl->h_modes.data(), nnz * sizeof(int32_t));
    if (he == hipSuccess) he = cp(pl->d_perm, pl->h_perm.data(), P * sizeof(int32_t));
    if (he == hipSuccess) he = cp(pl->d_voff, voff.data(), P * sizeof(long long));
    // (rows start unplanned, K = 0: a frozen plan re-plans a row that never got
    // a contour)
    if (he == hipSuccess && P > 0) he = hipMemsetAsync(pl->d_rows, 0, P * sizeof(RowPlan), st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) {
        plan_free_dev(pl);
        delete pl;
        return set_err(ctx, GBS_E_HIP, hipGetErrorString(he));
    }
    if ((rc = plan_units(ctx, pl))) {
        plan_free_dev(pl);
        delete pl;
        return rc;
    }
    *out = pl;
    return GBS_OK;
}

int gbs_plan_destroy(gbs_plan *pl)
{
    if (!pl) return GBS_E_INVAL;
    if (pl->ctx) (void)hipSetDevice(pl->ctx->device);
    plan_free_dev(pl);
    delete pl;
    return GBS_OK;
}

int gbs_plan_freeze(gbs_plan *pl, int freeze)
{
    if (!pl) return GBS_E_INVAL;
    if (freeze && !pl->have_run)
        return set_err(pl->ctx, GBS_E_STATE, "plan has not run yet; nothing to freeze");
    pl->frozen = freeze != 0;
    return GBS_OK;
}

int gbs_prob_approx_dev(gbs_ctx *ctx, gbs_plan *pl, double *logp_dev, int32_t *status_dev)
{
    if (!ctx || !pl) return GBS_E_INVAL;
    if (pl->ctx != ctx) return set_err(ctx, GBS_E_STATE, "plan belongs to another context");
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    if (ctx->model.M != pl->M) return set_err(ctx, GBS_E_STATE, "plan was made for a model of another size M");
    if (pl->P > 0 && !logp_dev) return set_err(ctx, GBS_E_INVAL, "logp_dev is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int rc = approx_forward(ctx, pl, logp_dev, status_dev);
    if (rc == 0) pl->have_run = true;
    return rc;
}

int gbs_prob_approx(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int order,
                    int prec, double *logp, int32_t *status)
{
    if (!ctx) return GBS_E_INVAL;
    if (P > 0 && (!logp || !status)) return set_err(ctx, GBS_E_INVAL, "NULL output array");
    gbs_plan *pl = nullptr;
    int rc = gbs_plan_create(ctx, P, offsets, modes, order, prec, &pl);
    if (rc) return rc;
    rc = gbs_prob_approx_dev(ctx, pl, pl->d_logp, pl->d_status);
    if (rc == 0 && P > 0) {
        hipError_t e = hipMemcpyAsync(logp, pl->d_logp, P * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(status, pl->d_status, P * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) rc = set_err(ctx, GBS_E_HIP, hipGetErrorString(e));
    }
    gbs_plan_destroy(pl);
    if (rc) return rc;
    for (int p = 0; p < P; ++p)
        if (status[p] != 0) return GBS_W_PATTERN;
    return GBS_OK;
}

int gbs_prob_approx_plain(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int order,
                    int prec, double *logp, int32_t *status)
{
    if (!ctx) return GBS_E_INVAL;
    if (P > 0 && (!logp || !status)) return set_err(ctx, GBS_E_INVAL, "NULL output array");
    gbs_plan *pl = nullptr;
    int rc = gbs_plan_create(ctx, P, offsets, modes, order, prec, &pl);
    if (rc) return rc;
    rc = pl->max_n > GBS_NSMALL
             ? set_err(ctx, GBS_E_INVAL, "the plain kernel takes rows of at most 40 clicks")
         : prec != GBS_PREC_FP64
             ? set_err(ctx, GBS_E_INVAL, "the plain kernel runs in fp64 only")
             : approx_forward_plain(ctx, pl, pl->d_logp, pl->d_status);
    if (rc == 0 && P > 0) {
        hipError_t e = hipMemcpyAsync(logp, pl->d_logp, P * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(status, pl->d_status, P * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) rc = set_err(ctx, GBS_E_HIP, hipGetErrorString(e));
    }
    gbs_plan_destroy(pl);
    if (rc) return rc;
    for (int p = 0; p < P; ++p)
        if (status[p] != 0) return GBS_W_PATTERN;
    return GBS_OK;
}

int gbs_plan_get_params(gbs_plan *pl, int32_t *params)
{
    if (!pl || !params) return GBS_E_INVAL;
    params[0] = pl->seg_fwd;
    params[1] = pl->seg_adj;
    params[2] = pl->qchunk;
    params[3] = pl->gmax;
    return GBS_OK;
}

int gbs_plan_set_params(gbs_plan *pl, const int32_t *params)
{
    if (!pl || !params) return GBS_E_INVAL;
    gbs_ctx *ctx = pl->ctx;
    const int sf = params[0], sa = params[1], qc = params[2], gm = params[3];
    if (sf < 1 || sf > 64 || sa < 1 || sa > 64)
        return set_err(ctx, GBS_E_INVAL, "segment lengths must be in [1, 64]");
    if (qc < GBS_QCHUNK_MIN || qc > GBS_QCHUNK_MAX || (qc & (qc - 1)))
        return set_err(ctx, GBS_E_INVAL, "contour points per item must be 4, 8, 16, 32 or 64");
    if (gm < 1 || gm > 8 || (gm & (gm - 1)))
        return set_err(ctx, GBS_E_INVAL, "points per pass must be 1, 2, 4 or 8");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const bool units = sf != pl->seg_fwd || sa != pl->seg_adj;
    pl->seg_fwd = sf;
    pl->seg_adj = sa;
    pl->qchunk = qc;
    pl->gmax = gm;
    return units ? plan_units(ctx, pl) : GBS_OK;
}

namespace {

// device time (ms) of one forward, or one adjoint after a forward, on a plan;
// the smaller of two runs
int time_pass(gbs_ctx *ctx, gbs_plan *pl, bool adjoint, const double *dl, double *g, double *ms)
{
    hipEvent_t a, b;
    HIP_TRY(ctx, hipEventCreate(&a));
    HIP_TRY(ctx, hipEventCreate(&b));
    double best = 1e300;
    int rc = 0;
    for (int rep = 0; rep < 2 && !rc; ++rep) {
        if (adjoint && (rc = approx_forward(ctx, pl, pl->d_logp, pl->d_status))) break;
        (void)hipEventRecord(a, ctx->stream);
        rc = adjoint ? approx_backward(ctx, pl, dl, pl->d_status, g, g + ctx->model.M)
                     : approx_forward(ctx, pl, pl->d_logp, pl->d_status);
        (void)hipEventRecord(b, ctx->stream);
        if (!rc && hipEventSynchronize(b) != hipSuccess) rc = set_err(ctx, GBS_E_HIP, "event wait failed");
        float e = 0.f;
        if (!rc && hipEventElapsedTime(&e, a, b) == hipSuccess) best = std::min(best, (double)e);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = best;
    return rc;
}

}  // namespace

int gbs_plan_tune(gbs_ctx *ctx, gbs_plan *pl, int what, int32_t *params_out)
{
    if (!ctx || !pl) return GBS_E_INVAL;
    if (pl->ctx != ctx) return set_err(ctx, GBS_E_STATE, "plan belongs to another context");
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    if (ctx->model.M != pl->M) return set_err(ctx, GBS_E_STATE, "plan was made for a model of another size M");
    if ((what & 2) && !ctx->model.from_params)
        return set_err(ctx, GBS_E_STATE, "tuning the gradient needs a model set by gbs_set_model");
    if (pl->P == 0 || !(what & 3)) return params_out ? gbs_plan_get_params(pl, params_out) : GBS_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // a stratified sample of the rows (every s-th row in cost order, at least 512 rows)
    const int s = std::max(1, pl->P / 1024);
    std::vector<int32_t> off(1, 0), mod;
    for (int k = 0; k < pl->P; k += s) {
        const int p = pl->h_perm[k];
        for (int i = pl->h_offsets[p]; i < pl->h_offsets[p + 1]; ++i) mod.push_back(pl->h_modes[i]);
        off.push_back((int32_t)mod.size());
    }
    const int Ps = (int)off.size() - 1;
    gbs_plan *sub = nullptr;
    int rc = gbs_plan_create(ctx, Ps, off.data(), mod.data(), pl->order, pl->prec, &sub);
    if (rc) return rc;
    const bool timing = ctx->timing;
    ctx->timing = false;
    double *dl = nullptr, *g = nullptr;
    int32_t cur[4], best[4];
    gbs_plan_get_params(pl, cur);
    std::copy(cur, cur + 4, best);
    auto measure = [&](const int32_t *prm, bool adjoint, double *ms) {
        int r = gbs_plan_set_params(sub, prm);
        return r ? r : time_pass(ctx, sub, adjoint, dl, g, ms);
    };
    if (what & 2) {
        rc = dev_alloc(ctx, &dl, Ps);
        rc = rc ? rc : dev_alloc(ctx, &g, 2 * (size_t)ctx->model.M);
        if (!rc) {
            std::vector<double> ones(Ps, 1.0);
            if (hipMemcpy(dl, ones.data(), Ps * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
                rc = set_err(ctx, GBS_E_HIP, "upload failed");
        }
    }
    // warm-up (plan of the sample, gradient workspace)
    double ms = 0.0;
    if (!rc) rc = measure(best, (what & 2) != 0, &ms);
    // coordinate descent over the candidate values, one choice at a time
    struct Axis { int index; std::vector<int> values; bool adjoint; };
    std::vector<Axis> axes;
    if (what & 1) {
        if (pl->order >= 3) axes.push_back({0, {2, 3, 4, 6, 8, 12}, false});
        axes.push_back({2, {4, 8, 16}, false});
        axes.push_back({3, {2, 4, 8}, false});
    }
    if ((what & 2) && pl->order >= 3) axes.push_back({1, {2, 3, 4, 6}, true});
    for (const Axis &ax : axes) {
        if (rc) break;
        double tbest = 1e300;
        int vbest = best[ax.index];
        for (int v : ax.values) {
            int32_t prm[4];
            std::copy(best, best + 4, prm);
            prm[ax.index] = v;
            double t = 0.0;
            if ((rc = measure(prm, ax.adjoint, &t))) break;
            if (t < tbest) {
                tbest = t;
                vbest = v;
            }
        }
        best[ax.index] = vbest;
    }
    if (dl) (void)hipFree(dl);
    if (g) (void)hipFree(g);
    gbs_plan_destroy(sub);
    ctx->timing = timing;
    if (rc) return rc;
    rc = gbs_plan_set_params(pl, best);
    if (rc) return rc;
    if (params_out) std::copy(best, best + 4, params_out);
    return GBS_OK;
}

int gbs_plan_info(gbs_plan *pl, double *rho, double *rconv, int32_t *K, int32_t *nsectors, double *err)
{
    if (!pl) return GBS_E_INVAL;
    gbs_ctx *ctx = pl->ctx;
    std::vector<RowPlan> rows(pl->P);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (pl->P > 0) {
        HIP_TRY(ctx, hipMemcpyAsync(rows.data(), pl->d_rows, pl->P * sizeof(RowPlan),
                                    hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    for (int p = 0; p < pl->P; ++p) {
        if (rho) rho[p] = rows[p].rho;
        if (rconv) rconv[p] = rows[p].rconv;
        if (K) K[p] = rows[p].K;
        if (nsectors) nsectors[p] = rows[p].nsec;
        if (err) err[p] = rows[p].err;
    }
    return GBS_OK;
}

int gbs_prob_exact(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int prec,
                   double *p, double *logp, double *kappa, int32_t *status)
{
    if (!ctx) return GBS_E_INVAL;
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    if (prec != GBS_PREC_FP64 && prec != GBS_PREC_MIXED)
        return set_err(ctx, GBS_E_INVAL, "prec must be GBS_PREC_FP64 or GBS_PREC_MIXED");
    if (P > 0 && (!p || !status)) return set_err(ctx, GBS_E_INVAL, "NULL output array");
    int rc = check_csr(ctx, P, offsets, modes, ctx->model.M, GBS_MAX_N_EXACT);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    rc = exact_run(ctx, P, offsets, modes, p, logp, kappa, status);
    if (rc) return rc;
    // the mixed tier: fp32 terms would reach 1e-6 only for kappa_IE <= 10, so
    // every row runs in the double-double tier and says so
    if (prec == GBS_PREC_MIXED)
        for (int i = 0; i < P; ++i) status[i] |= GBS_PS_ESCALATED;
    for (int i = 0; i < P; ++i)
        if (status[i] != 0) return GBS_W_PATTERN;
    return GBS_OK;
}

int gbs_prob_exact_dev(gbs_ctx *ctx, int P, const int32_t *offsets_dev, const int32_t *modes_dev, int max_clicks,
                       double *p_dev, double *logp_dev, double *kappa_dev, int32_t *status_dev)
{
    if (!ctx) return GBS_E_INVAL;
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    if (P < 0) return set_err(ctx, GBS_E_INVAL, "P must be >= 0");
    if (max_clicks < 0 || max_clicks > GBS_MAX_N_EXACT)
        return set_err(ctx, GBS_E_INVAL, "max_clicks must be in [0, " + std::to_string(GBS_MAX_N_EXACT) + "]");
    if (P == 0) return GBS_OK;
    if (!offsets_dev || !modes_dev || !p_dev || !status_dev) return set_err(ctx, GBS_E_INVAL, "NULL device array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const long long need = (long long)P << exact_lgs(max_clicks);
    if (need > ctx->ex_part_items) {
        // (grown on demand: the previous launches on the stream may still read
        // the old buffer, so wait for them before it is released)
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->ex_part) (void)hipFree(ctx->ex_part);
        ctx->ex_part = nullptr;
        ctx->ex_part_items = 0;
        if (int rc = dev_alloc(ctx, &ctx->ex_part, 3 * (size_t)need)) return rc;
        ctx->ex_part_items = need;
    }
    return exact_launch(ctx, P, offsets_dev, modes_dev, max_clicks, ctx->ex_part, p_dev, logp_dev, kappa_dev,
                        status_dev);
}

int gbs_prob_exact_dev_noalloc(gbs_ctx *ctx, int P, const int32_t *offsets_dev, const int32_t *modes_dev,
                               int max_clicks, double *p_dev, double *logp_dev, double *kappa_dev,
                               int32_t *status_dev)
{
    if (!ctx) return GBS_E_INVAL;
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    if (P < 0) return set_err(ctx, GBS_E_INVAL, "P must be >= 0");
    if (max_clicks < 0 || max_clicks > GBS_MAX_N_EXACT)
        return set_err(ctx, GBS_E_INVAL, "max_clicks must be in [0, " + std::to_string(GBS_MAX_N_EXACT) + "]");
    if (P == 0) return GBS_OK;
    if (!offsets_dev || !modes_dev || !p_dev || !status_dev) return set_err(ctx, GBS_E_INVAL, "NULL device array");
    const long long need = (long long)P << exact_lgs(max_clicks);
    if (need > exact_noalloc_items())
        return set_err(ctx, GBS_E_INVAL, "P * 2^min(max(max_clicks - 9, 0), 12) = " + std::to_string(need) +
                                             " work items exceed the fixed scratch of " +
                                             std::to_string(exact_noalloc_items()));
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    double *part = exact_scratch(ctx->device);
    if (!part) return set_err(ctx, GBS_E_STATE, "fixed scratch of this device not initialised");
    return exact_launch(ctx, P, offsets_dev, modes_dev, max_clicks, part, p_dev, logp_dev, kappa_dev, status_dev);
}

int gbs_grad_dev(gbs_ctx *ctx, gbs_plan *pl, const double *dl_dev, double *logp_dev,
                 double *grad_r_dev, double *grad_eta_dev, int32_t *status_dev)
{
    if (!ctx || !pl) return GBS_E_INVAL;
    if (pl->ctx != ctx) return set_err(ctx, GBS_E_STATE, "plan belongs to another context");
    if (!ctx->model.have || !ctx->model.from_params)
        return set_err(ctx, GBS_E_STATE, "gradient needs a model set by gbs_set_model");
    if (ctx->model.M != pl->M) return set_err(ctx, GBS_E_STATE, "plan was made for a model of another size M");
    if (!dl_dev || !grad_r_dev || !grad_eta_dev) return set_err(ctx, GBS_E_INVAL, "NULL device array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    double *lp = logp_dev ? logp_dev : pl->d_logp;
    int32_t *stt = status_dev ? status_dev : pl->d_status;
    // the adjoint exists in fp64 only: a mixed-tier plan runs forward and
    // adjoint in fp64 here, and every row reports GBS_PS_ESCALATED
    const bool esc_all = pl->prec != GBS_PREC_FP64;
    const int prec = pl->prec;
    pl->prec = GBS_PREC_FP64;
    int rc = approx_forward(ctx, pl, lp, stt);
    if (rc == 0) {
        pl->have_run = true;
        rc = approx_backward(ctx, pl, dl_dev, stt, grad_r_dev, grad_eta_dev);
    }
    pl->prec = prec;
    if (rc == 0 && esc_all) rc = status_or(ctx, pl->P, stt, GBS_PS_ESCALATED);
    return rc;
}

}  // extern "C"

// mcmc.hip: one Metropolis-Hastings step of the chains held in modes (CSR rows
// of the plan's offsets), their log p_hat in logp; proposals evaluated on the
// plan
int mcmc_step(gbs_ctx *ctx, gbs_plan *plan, const double *u, int32_t *modes, double *logp, int32_t *accepted);
int mcmc_da_step(gbs_ctx *ctx, gbs_plan *plan, const double *u, int32_t *modes, double *logp_hat, double *logp_exact,
                 int32_t *accepted);

extern "C" {

int gbs_mcmc_step_dev(gbs_ctx *ctx, gbs_plan *pl, const double *u_dev, int32_t *modes_dev, double *logp_dev,
                      int32_t *accepted_dev)
{
    if (!ctx || !pl) return GBS_E_INVAL;
    if (pl->ctx != ctx) return set_err(ctx, GBS_E_STATE, "plan belongs to another context");
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    if (ctx->model.M != pl->M) return set_err(ctx, GBS_E_STATE, "plan was made for a model of another size M");
    if (pl->frozen) return set_err(ctx, GBS_E_STATE, "the chains need a plan that is not frozen (new rows every step)");
    if (pl->whole) return set_err(ctx, GBS_E_INVAL, "not a plan of click patterns");
    if (pl->P > 0 && (!u_dev || !modes_dev || !logp_dev)) return set_err(ctx, GBS_E_INVAL, "NULL device array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    return mcmc_step(ctx, pl, u_dev, modes_dev, logp_dev, accepted_dev);
}

int gbs_mcmc_da_step_dev(gbs_ctx *ctx, gbs_plan *pl, const double *u_dev, int32_t *modes_dev, double *logp_hat_dev,
                         double *logp_exact_dev, int32_t *accepted_dev)
{
    if (!ctx || !pl) return GBS_E_INVAL;
    if (pl->ctx != ctx) return set_err(ctx, GBS_E_STATE, "plan belongs to another context");
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    if (ctx->model.M != pl->M) return set_err(ctx, GBS_E_STATE, "plan was made for a model of another size M");
    if (pl->frozen) return set_err(ctx, GBS_E_STATE, "the chains need a plan that is not frozen (new rows every step)");
    if (pl->whole) return set_err(ctx, GBS_E_INVAL, "not a plan of click patterns");
    if (pl->max_n > GBS_MAX_N_EXACT)
        return set_err(ctx, GBS_E_INVAL, "the exact correction takes rows of at most " +
                                             std::to_string(GBS_MAX_N_EXACT) + " clicks");
    if (pl->P > 0 && (!u_dev || !modes_dev || !logp_hat_dev || !logp_exact_dev))
        return set_err(ctx, GBS_E_INVAL, "NULL device array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (pl->P > 0) {
        // the chains' workspace, on the first call
        const size_t P = pl->P, nnz = pl->h_offsets[pl->P];
        if (!pl->d_da)
            if (int e = dev_alloc(ctx, &pl->d_da, 4 * P + 1 + nnz)) return e;
        if (!pl->d_da_x)
            if (int e = dev_alloc(ctx, &pl->d_da_x, 2 * P)) return e;
    }
    return mcmc_da_step(ctx, pl, u_dev, modes_dev, logp_hat_dev, logp_exact_dev, accepted_dev);
}

int gbs_set_deterministic(gbs_ctx *ctx, int on)
{
    if (!ctx) return GBS_E_INVAL;
    ctx->deterministic = on != 0;
    return GBS_OK;
}

int gbs_click_distribution(gbs_ctx *ctx, int order, int nk, const int32_t *ks, double *p_n, double *p_k,
                           int32_t *status)
{
    if (!ctx) return GBS_E_INVAL;
    if (!ctx->model.have) return set_err(ctx, GBS_E_STATE, "no model set");
    const int M = ctx->model.M;
    if (M > GBS_NSMALL) return set_err(ctx, GBS_E_INVAL, "the click distribution takes at most 40 modes");
    if (nk < 0 || (nk > 0 && (!ks || !p_k)) || !p_n || !status)
        return set_err(ctx, GBS_E_INVAL, "NULL or negative argument");
    std::vector<int32_t> off = {0, M}, mod(M);
    std::iota(mod.begin(), mod.end(), 0);
    gbs_plan *pl = nullptr;
    int rc = gbs_plan_create(ctx, 1, off.data(), mod.data(), order, GBS_PREC_FP64, &pl);
    if (rc) return rc;
    pl->whole = true;
    int *dks = nullptr;
    double *dpn = nullptr, *dpk = nullptr;
    int32_t *dst = nullptr;
    rc = dev_alloc(ctx, &dks, nk > 0 ? nk : 1);
    if (!rc) rc = dev_alloc(ctx, &dpn, M + 1);
    if (!rc) rc = dev_alloc(ctx, &dpk, nk > 0 ? (size_t)nk * (M + 1) : 1);
    if (!rc) rc = dev_alloc(ctx, &dst, 1);
    hipStream_t st = ctx->stream;
    if (!rc && nk > 0 &&
        hipMemcpyAsync(dks, ks, nk * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = set_err(ctx, GBS_E_HIP, "copy of ks failed");
    if (!rc) rc = click_distribution_run(ctx, pl, nk, dks, dpn, dpk, dst);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(p_n, dpn, (M + 1) * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && nk > 0)
            e = hipMemcpyAsync(p_k, dpk, (size_t)nk * (M + 1) * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(status, dst, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = set_err(ctx, GBS_E_HIP, hipGetErrorString(e));
    }
    if (dks) (void)hipFree(dks);
    if (dpn) (void)hipFree(dpn);
    if (dpk) (void)hipFree(dpk);
    if (dst) (void)hipFree(dst);
    gbs_plan_destroy(pl);
    if (rc) return rc;
    return *status != 0 ? GBS_W_PATTERN : GBS_OK;
}

int gbs_grad(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, int order, int prec,
             const double *dL_dlogp, double *logp, double *grad_r, double *grad_eta, int32_t *status)
{
    if (!ctx) return GBS_E_INVAL;
    if (!dL_dlogp || !grad_r || !grad_eta || (P > 0 && !status))
        return set_err(ctx, GBS_E_INVAL, "NULL array");
    if (!ctx->model.have || !ctx->model.from_params)
        return set_err(ctx, GBS_E_STATE, "gradient needs a model set by gbs_set_model");
    gbs_plan *pl = nullptr;
    int rc = gbs_plan_create(ctx, P, offsets, modes, order, prec, &pl);
    if (rc) return rc;
    int M = ctx->model.M;
    rc = dev_alloc(ctx, &pl->d_dl, P > 0 ? P : 1);
    if (!rc) rc = dev_alloc(ctx, &pl->d_grad, 2 * (size_t)M);
    hipStream_t st = ctx->stream;
    if (!rc && P > 0 &&
        hipMemcpyAsync(pl->d_dl, dL_dlogp, P * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = set_err(ctx, GBS_E_HIP, "copy of dL_dlogp failed");
    if (!rc) rc = gbs_grad_dev(ctx, pl, pl->d_dl, pl->d_logp, pl->d_grad, pl->d_grad + M, pl->d_status);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(grad_r, pl->d_grad, M * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(grad_eta, pl->d_grad + M, M * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && logp && P > 0)
            e = hipMemcpyAsync(logp, pl->d_logp, P * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && P > 0)
            e = hipMemcpyAsync(status, pl->d_status, P * sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = set_err(ctx, GBS_E_HIP, hipGetErrorString(e));
    }
    gbs_plan_destroy(pl);
    if (rc) return rc;
    for (int i = 0; i < P; ++i)
        if (status[i] != 0) return GBS_W_PATTERN;
    return GBS_OK;
}

}  // extern "C"
