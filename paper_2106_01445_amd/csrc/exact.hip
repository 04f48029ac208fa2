// Exact click probabilities (Methods, Probability of any sample; the click
// projector of Methods, Model), in double-double on one MI355X.
//
//   p(C) = det(Q)^{-1/2} sum_{Z subset C} (-1)^{n-|Z|} det(A_Z)^{-1/2},  A = (Q^{-1})_CC
//
// Each determinant is a product of 2x2 Schur-complement determinants taken one
// mode at a time, so the subsets form a binary include/exclude tree over the
// clicked modes and every tree edge that includes a mode costs one rank-2
// update of the remaining matrix.  Work split:
//   - the first h = max(0, n-9) modes: 2^h included/excluded assignments z0,
//     dealt to at most 2^EX_LGI work items (one wavefront each) per row, each
//     item taking a contiguous range of z0 in turn; for each z0 the wave
//     conditions A on the included prefix modes by successive Schur steps in
//     LDS;
//   - the next m = R-3 modes (R = n-h <= 9): breadth-first expansion in LDS,
//     level by level, ending with 2^m <= 64 nodes, one per lane;
//   - the last 3 modes: each lane evaluates its node's 8 subsets in registers.
// All matrices are kept as packed symmetric double-double (hi/lo planes) with
// the two quadratures of a mode interleaved.  Signed sums are double-double,
// reduced in a fixed order; kappa = sum|terms| / |sum| is returned.
#include <algorithm>
#include <mutex>

#include "internal.h"

#define EX_R 9          // modes handled inside one prefix assignment
#define EX_BUF 1344     // packed dd entries of the 64 nodes x 21 of the last level
#define EX_LGI 12       // at most 2^12 work items per row

// packed dd entries per LDS buffer for rows of up to maxn clicks: the last
// expansion level, or the matrix of all maxn modes
__host__ __device__ __forceinline__ int ex_buf(int maxn)
{
    const int k = maxn * (2 * maxn + 1);
    return k > EX_BUF ? k : EX_BUF;
}
__host__ __device__ __forceinline__ int ex_lds_bytes(int maxn)
{
    // two buffers (hi and lo planes) and the packed index tables (two shorts)
    return 4 * 8 * ex_buf(maxn) + 2 * 2 * ex_buf(maxn);
}

namespace {

__device__ __forceinline__ int pk(int r, int c) { return r >= c ? r * (r + 1) / 2 + c : c * (c + 1) / 2 + r; }

struct Sym2 {  // symmetric 2x2 dd block
    dd a, b, c;  // [[a, b], [b, c]]
};

__device__ __forceinline__ dd det2(const Sym2 &s) { return dd_sub(dd_mul(s.a, s.c), dd_mul(s.b, s.b)); }

__device__ __forceinline__ Sym2 inv2(const Sym2 &s, dd det)
{
    dd id = dd_recip(det);
    return Sym2{dd_mul(s.c, id), dd_neg(dd_mul(s.b, id)), dd_mul(s.a, id)};
}

struct Gen2 {  // general 2x2 dd block [[p, q], [r, s]]
    dd p, q, r, s;
};

// inv (sym) * X (general)
__device__ __forceinline__ Gen2 mul_sg(const Sym2 &i, const Gen2 &x)
{
    return Gen2{dd_add(dd_mul(i.a, x.p), dd_mul(i.b, x.r)), dd_add(dd_mul(i.a, x.q), dd_mul(i.b, x.s)),
                dd_add(dd_mul(i.b, x.p), dd_mul(i.c, x.r)), dd_add(dd_mul(i.b, x.q), dd_mul(i.c, x.s))};
}
// Y^T * G  (general^T * general), symmetric result when G = inv * Y
__device__ __forceinline__ Sym2 tmul_sym(const Gen2 &y, const Gen2 &g)
{
    return Sym2{dd_add(dd_mul(y.p, g.p), dd_mul(y.r, g.r)), dd_add(dd_mul(y.p, g.q), dd_mul(y.r, g.s)),
                dd_add(dd_mul(y.q, g.q), dd_mul(y.s, g.s))};
}
__device__ __forceinline__ Gen2 tmul_gen(const Gen2 &y, const Gen2 &g)
{
    return Gen2{dd_add(dd_mul(y.p, g.p), dd_mul(y.r, g.r)), dd_add(dd_mul(y.p, g.q), dd_mul(y.r, g.s)),
                dd_add(dd_mul(y.q, g.p), dd_mul(y.s, g.r)), dd_add(dd_mul(y.q, g.q), dd_mul(y.s, g.s))};
}
__device__ __forceinline__ Sym2 sub_s(const Sym2 &a, const Sym2 &b)
{
    return Sym2{dd_sub(a.a, b.a), dd_sub(a.b, b.b), dd_sub(a.c, b.c)};
}
__device__ __forceinline__ Gen2 sub_g(const Gen2 &a, const Gen2 &b)
{
    return Gen2{dd_sub(a.p, b.p), dd_sub(a.q, b.q), dd_sub(a.r, b.r), dd_sub(a.s, b.s)};
}

struct Buf {
    double *hi, *lo;
    __device__ __forceinline__ dd get(int i) const { return dd{hi[i], lo[i]}; }
    __device__ __forceinline__ void put(int i, dd v) const
    {
        hi[i] = v.hi;
        lo[i] = v.lo;
    }
};

__device__ __forceinline__ Sym2 sblk(const Buf &b, int base, int j)
{
    return Sym2{b.get(base + pk(2 * j, 2 * j)), b.get(base + pk(2 * j + 1, 2 * j)),
                b.get(base + pk(2 * j + 1, 2 * j + 1))};
}
// block (rows of mode i, cols of mode j), i < j
__device__ __forceinline__ Gen2 gblk(const Buf &b, int base, int i, int j)
{
    return Gen2{b.get(base + pk(2 * i, 2 * j)), b.get(base + pk(2 * i, 2 * j + 1)),
                b.get(base + pk(2 * i + 1, 2 * j)), b.get(base + pk(2 * i + 1, 2 * j + 1))};
}

// Leaf: the 2^S subsets of the last S (1..3) modes of one node's matrix.
// Adds sign * acc * det(S_T)^{-1/2} into tot and acc*|...| into ab, where the
// sign of subset T is (-1)^(base_par + |T|).
template <int S>
__device__ void leaf(const Buf &b, int base, dd acc, int base_par, dd &tot, double &ab)
{
    auto add = [&](dd f, int t) {
        dd v = dd_mul(acc, f);
        tot = ((base_par + t) & 1) ? dd_sub(tot, v) : dd_add(tot, v);
        ab += fabs(v.hi);
    };
    add(dd_make(1.0), 0);
    const Sym2 sx = sblk(b, base, 0);
    const dd dx = det2(sx);
    const dd rx = dd_rsqrt(dx);
    add(rx, 1);
    if (S == 1) return;
    const Sym2 sy = sblk(b, base, 1);
    const dd dy = det2(sy);
    const dd ry = dd_rsqrt(dy);
    add(ry, 1);
    const Sym2 ix = inv2(sx, dx);
    const Gen2 xy = gblk(b, base, 0, 1);
    const Gen2 gy = mul_sg(ix, xy);
    const Sym2 syx = sub_s(sy, tmul_sym(xy, gy));      // S_yy | x
    const dd dyx = det2(syx);
    add(dd_mul(rx, dd_rsqrt(dyx)), 2);
    if (S == 2) return;
    const Sym2 sz = sblk(b, base, 2);
    add(dd_rsqrt(det2(sz)), 1);
    const Gen2 xz = gblk(b, base, 0, 2);
    const Gen2 yz = gblk(b, base, 1, 2);
    const Gen2 gz = mul_sg(ix, xz);
    const Sym2 szx = sub_s(sz, tmul_sym(xz, gz));      // S_zz | x
    add(dd_mul(rx, dd_rsqrt(det2(szx))), 2);
    const Sym2 iy = inv2(sy, dy);
    const Sym2 szy = sub_s(sz, tmul_sym(yz, mul_sg(iy, yz)));  // S_zz | y
    add(dd_mul(ry, dd_rsqrt(det2(szy))), 2);
    const Gen2 yzx = sub_g(yz, tmul_gen(xy, gz));     // S_yz | x
    const Sym2 iyx = inv2(syx, dyx);
    const Sym2 szxy = sub_s(szx, tmul_sym(yzx, mul_sg(iyx, yzx)));  // S_zz | x,y
    add(dd_mul(dd_mul(rx, dd_rsqrt(dyx)), dd_rsqrt(det2(szxy))), 3);
}

// One elimination step: Schur complement of the first mode of the k-mode
// matrix at src+sbase, written (k-1 modes) to dst+dbase; lanes split entries.
__device__ __forceinline__ void schur_first(const Buf &src, int sbase, const Buf &dst, int dbase, int k,
                                            const Sym2 &inv, int e, const short *lr, const short *lc)
{
    const int r = lr[e], c = lc[e];
    const int R = r + 2, Cc = c + 2;
    const dd a0 = src.get(sbase + pk(R, 0)), a1 = src.get(sbase + pk(R, 1));
    const dd b0 = src.get(sbase + pk(0, Cc)), b1 = src.get(sbase + pk(1, Cc));
    const dd t0 = dd_add(dd_mul(inv.a, b0), dd_mul(inv.b, b1));
    const dd t1 = dd_add(dd_mul(inv.b, b0), dd_mul(inv.c, b1));
    dst.put(dbase + e, dd_sub(src.get(sbase + pk(R, Cc)), dd_add(dd_mul(a0, t0), dd_mul(a1, t1))));
}

__device__ __forceinline__ dd wave_dd_sum(dd v)
{
    for (int m = 32; m > 0; m >>= 1) {
        dd o = dd{__shfl_xor(v.hi, m), __shfl_xor(v.lo, m)};
        v = dd_add(v, o);
    }
    return v;
}

// One work item: row p = item >> lgS, part i = item & (S - 1) of its 2^h prefix
// assignments (rows of more than maxn clicks, or with modes outside [0, M) or
// not ascending, are left to k_exact_final, which flags them).
__global__ __launch_bounds__(64) void k_exact(int M, const double *__restrict__ qi_hi,
                                              const double *__restrict__ qi_lo,
                                              const int *__restrict__ offsets,
                                              const int *__restrict__ modes, int lgS, int maxn,
                                              double *__restrict__ part)
{
    extern __shared__ __attribute__((aligned(16))) double exsh[];
    __shared__ double nacc_h[2][64], nacc_l[2][64];
    __shared__ int npar[2][64];
    __shared__ double ninv_h[3][32], ninv_l[3][32];
    __shared__ int gidx[2 * GBS_MAX_N_EXACT];
    __shared__ int s_bad;
    const int BUF = ex_buf(maxn);
    double *bh0 = exsh, *bh1 = bh0 + BUF, *bl0 = bh1 + BUF, *bl1 = bl0 + BUF;
    short *lr = (short *)(bl1 + BUF), *lc = lr + BUF;
    const int lane = threadIdx.x;
    const long long item = blockIdx.x;
    const int p = (int)(item >> lgS), ip = (int)(item & ((1LL << lgS) - 1));
    const int o = offsets[p], n = offsets[p + 1] - o;
    if (n <= 0 || n > maxn) return;
    const int D = 2 * M;
    const int h = n > EX_R ? n - EX_R : 0;
    const int R = n - h;
    const int lgI = h < EX_LGI ? h : EX_LGI;   // this row's items: 2^lgI
    if (ip >= (1 << lgI)) return;
    const int lgC = h - lgI;                    // prefix assignments per item: 2^lgC
    if (lane == 0) {
        int bad = 0;
        for (int i = 0; i < n; ++i) {
            const int m = modes[o + i];
            if (m < 0 || m >= M || (i > 0 && m <= modes[o + i - 1])) bad = 1;
        }
        s_bad = bad;
    }
    // packed-index -> (row, col) tables for up to 2 maxn rows
    for (int r = lane; r < 2 * maxn; r += 64)
        for (int c = 0; c <= r; ++c) {
            int e = r * (r + 1) / 2 + c;
            if (e < BUF) {
                lr[e] = (short)r;
                lc[e] = (short)c;
            }
        }
    __syncthreads();
    if (s_bad) return;
    dd rtot = dd_make(0.0);
    double rab = 0.0;
    for (int zi = 0; zi < (1 << lgC); ++zi) {
        const int z0 = (ip << lgC) | zi;
        // local mode list: included prefix modes, then the last R modes
        int kz = 0;
        if (lane == 0) {
            for (int i = 0; i < h; ++i)
                if (z0 >> i & 1) gidx[kz++] = modes[o + i];
            for (int i = h; i < n; ++i) gidx[kz++] = modes[o + i];
        }
        __syncthreads();
        const int nz0 = __popc(z0);
        int k = nz0 + R;
        Buf B0{bh0, bl0}, B1{bh1, bl1};
        for (int e = lane; e < k * (2 * k + 1); e += 64) {
            int r = lr[e], c = lc[e];
            int gr = gidx[r >> 1] + ((r & 1) ? M : 0);
            int gc = gidx[c >> 1] + ((c & 1) ? M : 0);
            B0.put(e, dd{qi_hi[(long)gr * D + gc], qi_lo[(long)gr * D + gc]});
        }
        __syncthreads();
        // condition on the included prefix modes
        dd acc = dd_make(1.0);
        int cur = 0;
        for (int s = 0; s < nz0; ++s) {
            Buf src = cur ? B1 : B0, dst = cur ? B0 : B1;
            const Sym2 s00 = sblk(src, 0, 0);
            const dd det = det2(s00);
            const Sym2 inv = inv2(s00, det);
            acc = dd_mul(acc, dd_rsqrt(det));
            const int cnt = (k - 1) * (2 * k - 1);
            for (int e = lane; e < cnt; e += 64) schur_first(src, 0, dst, 0, k, inv, e, lr, lc);
            __syncthreads();
            cur ^= 1;
            --k;
        }
        // breadth-first expansion of the next m modes
        const int sl = R < 3 ? R : 3;
        const int m = R - sl;
        if (lane == 0) {
            nacc_h[0][0] = acc.hi;
            nacc_l[0][0] = acc.lo;
            npar[0][0] = nz0 & 1;
        }
        int nc = 0;  // node-info buffer
        __syncthreads();
        for (int lev = 0; lev < m; ++lev) {
            Buf src = cur ? B1 : B0, dst = cur ? B0 : B1;
            const int nodes = 1 << lev;
            const int cs = k * (2 * k + 1);            // packed size per parent
            const int cd = (k - 1) * (2 * k - 1);      // packed size per child
            // children node info: 2i exclude, 2i+1 include
            for (int i = lane; i < nodes; i += 64) {
                const Sym2 s00 = sblk(src, i * cs, 0);
                const dd det = det2(s00);
                const Sym2 inv = inv2(s00, det);
                ninv_h[0][i] = inv.a.hi; ninv_l[0][i] = inv.a.lo;
                ninv_h[1][i] = inv.b.hi; ninv_l[1][i] = inv.b.lo;
                ninv_h[2][i] = inv.c.hi; ninv_l[2][i] = inv.c.lo;
                dd a = dd{nacc_h[nc][i], nacc_l[nc][i]};
                const int par = npar[nc][i];
                nacc_h[nc ^ 1][2 * i] = a.hi;
                nacc_l[nc ^ 1][2 * i] = a.lo;
                npar[nc ^ 1][2 * i] = par;
                dd ai = dd_mul(a, dd_rsqrt(det));
                nacc_h[nc ^ 1][2 * i + 1] = ai.hi;
                nacc_l[nc ^ 1][2 * i + 1] = ai.lo;
                npar[nc ^ 1][2 * i + 1] = par ^ 1;
            }
            __syncthreads();
            for (int e = lane; e < 2 * nodes * cd; e += 64) {
                const int child = e / cd, idx = e - child * cd;
                const int parent = child >> 1;
                if (child & 1) {
                    const Sym2 inv{dd{ninv_h[0][parent], ninv_l[0][parent]},
                                   dd{ninv_h[1][parent], ninv_l[1][parent]},
                                   dd{ninv_h[2][parent], ninv_l[2][parent]}};
                    schur_first(src, parent * cs, dst, child * cd, k, inv, idx, lr, lc);
                } else {
                    const int r = lr[idx] + 2, c = lc[idx] + 2;
                    dst.put(child * cd + idx, src.get(parent * cs + pk(r, c)));
                }
            }
            __syncthreads();
            cur ^= 1;
            nc ^= 1;
            --k;
        }
        // leaves: one node per lane
        dd tot = dd_make(0.0);
        double ab = 0.0;
        const int leaves = 1 << m;
        if (lane < leaves) {
            Buf src = cur ? B1 : B0;
            const int cs = k * (2 * k + 1);
            dd a = dd{nacc_h[nc][lane], nacc_l[nc][lane]};
            const int par = (n + npar[nc][lane]) & 1;
            if (sl == 3) leaf<3>(src, lane * cs, a, par, tot, ab);
            else if (sl == 2) leaf<2>(src, lane * cs, a, par, tot, ab);
            else if (sl == 1) leaf<1>(src, lane * cs, a, par, tot, ab);
            else {
                tot = (par & 1) ? dd_neg(a) : a;  // n = 0: the empty set only
                ab = fabs(a.hi);
            }
        }
        tot = wave_dd_sum(tot);
        for (int mm = 32; mm > 0; mm >>= 1) ab += __shfl_xor(ab, mm);
        rtot = dd_add(rtot, tot);
        rab += ab;
        __syncthreads();
    }
    if (lane == 0) {
        part[3 * item] = rtot.hi;
        part[3 * item + 1] = rtot.lo;
        part[3 * item + 2] = rab;
    }
}

// Per row: the CSR check, the fixed-order sum of the item partials, times
// det(Q)^{-1/2}.  Outputs: p, status (required), logp, kappa (nullable).
__global__ void k_exact_final(int P, int M, const int *__restrict__ offsets, const int *__restrict__ modes,
                              int lgS, int maxn, const double *__restrict__ part,
                              const double *__restrict__ scal, double *__restrict__ p_out,
                              double *__restrict__ logp_out, double *__restrict__ kappa_out,
                              int *__restrict__ status_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int o = offsets[p], n = offsets[p + 1] - o;
    bool bad = n < 0 || n > maxn;
    for (int i = 0; i < n && !bad; ++i) {
        const int m = modes[o + i];
        bad = m < 0 || m >= M || (i > 0 && m <= modes[o + i - 1]);
    }
    if (bad) {
        p_out[p] = NAN;
        if (logp_out) logp_out[p] = NAN;
        if (kappa_out) kappa_out[p] = NAN;
        status_out[p] = GBS_PS_BADROW;
        return;
    }
    const int h = n > EX_R ? n - EX_R : 0;
    const int ni = 1 << (h < EX_LGI ? h : EX_LGI);
    const long long i0 = (long long)p << lgS;
    dd s = dd_make(0.0);
    double ab = 0.0;
    for (int i = 0; i < ni; ++i) {
        s = dd_add(s, dd{part[3 * (i0 + i)], part[3 * (i0 + i) + 1]});
        ab += part[3 * (i0 + i) + 2];
    }
    if (n == 0) {
        s = dd_make(1.0);
        ab = 1.0;
    }
    const dd rq = dd{scal[1], scal[2]};
    const dd pr = dd_mul(s, rq);
    const double kappa = s.hi != 0.0 ? ab / fabs(s.hi) : INFINITY;
    int st = 0;
    // double-double terms carry ~1e-30 relative error; the sum is resolved to
    // 1e-10 unless it cancels by more than 1e20
    if (!(kappa < 1e20) || !(pr.hi > 0.0)) st = GBS_PS_CANCEL;
    p_out[p] = st ? NAN : pr.hi;
    if (logp_out) logp_out[p] = st ? NAN : log(pr.hi) + pr.lo / pr.hi;
    if (kappa_out) kappa_out[p] = kappa;
    status_out[p] = st;
}

}  // namespace

// work items of a batch whose rows hold at most maxn clicks: P << exact_lgs(maxn)
int exact_lgs(int maxn)
{
    const int h = maxn > EX_R ? maxn - EX_R : 0;
    return h < EX_LGI ? h : EX_LGI;
}

// The exact path on device CSR: partials in d_part (3 doubles per work item,
// at least P << exact_lgs(maxn) items), results into the device outputs.
int exact_launch(gbs_ctx *ctx, int P, const int32_t *d_off, const int32_t *d_modes, int maxn, double *d_part,
                 double *p_dev, double *logp_dev, double *kappa_dev, int32_t *status_dev)
{
    if (P == 0) return 0;
    DevModel &m = ctx->model;
    hipStream_t st = ctx->stream;
    const int lgS = exact_lgs(maxn);
    const long long nitems = (long long)P << lgS;
    if (nitems > 0x7fffffffLL) return set_err(ctx, GBS_E_INVAL, "exact: too many work items (rows x 2^12)");
    const int lds = ex_lds_bytes(maxn);
    if (int rc = func_lds_limit(ctx, (const void *)k_exact, lds)) return rc;
    const int ts = timer_begin(ctx, TG_EXACT);
    if (maxn > 0)
        hipLaunchKernelGGL(k_exact, dim3((unsigned)nitems), dim3(64), lds, st, m.M, m.qi_hi, m.qi_lo, d_off,
                           d_modes, lgS, maxn, d_part);
    hipLaunchKernelGGL(k_exact_final, dim3((P + 127) / 128), dim3(128), 0, st, P, m.M, d_off, d_modes, lgS, maxn,
                       d_part, m.scal, p_dev, logp_dev, kappa_dev, status_dev);
    timer_end(ctx, ts);
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------------------
// Fixed scratch for gbs_prob_exact_dev_noalloc: the partial sums of up to
// EX_NOALLOC_ITEMS work items (3 doubles each, 24 MiB), one copy per GPU that
// the library runs on, held until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): its device address is taken once per device, with that device
// current, and kept in scratch_ptr.
// ---------------------------------------------------------------------------
#define EX_NOALLOC_ITEMS (1 << 20)
#define EX_MAX_DEVICES 64
static __device__ __align__(256) double scratch[3 * EX_NOALLOC_ITEMS];

namespace {
std::mutex scratch_mu;
double *scratch_ptr[EX_MAX_DEVICES] = {};
}  // namespace

// Once per device (the caller has made it current): the device address of
// `scratch`.  Returns a HIP error code.
int exact_scratch_init(int device)
{
    if (device < 0 || device >= EX_MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_ptr[device]) return 0;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    scratch_ptr[device] = (double *)ptr;
    return 0;
}

long long exact_noalloc_items() { return EX_NOALLOC_ITEMS; }

double *exact_scratch(int device)
{
    if (device < 0 || device >= EX_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    return scratch_ptr[device];
}

// Host CSR (already checked): copies in, one launch, copies out.
int exact_run(gbs_ctx *ctx, int P, const int32_t *offsets, const int32_t *modes, double *p,
              double *logp, double *kappa, int32_t *status)
{
    if (P == 0) return 0;
    hipStream_t st = ctx->stream;
    int maxn = 0;
    for (int r = 0; r < P; ++r) maxn = std::max(maxn, offsets[r + 1] - offsets[r]);
    const long long nitems = (long long)P << exact_lgs(maxn);
    const int nnz = offsets[P];
    int32_t *d_off = nullptr, *d_modes = nullptr, *d_st = nullptr;
    double *d_part = nullptr, *d_out = nullptr;
    auto cleanup = [&]() {
        void *ptrs[] = {d_off, d_modes, d_st, d_part, d_out};
        for (void *q : ptrs)
            if (q) (void)hipFree(q);
    };
    if (hipMalloc((void **)&d_off, (P + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&d_modes, std::max(nnz, 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&d_st, P * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&d_part, std::max(nitems, 1LL) * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&d_out, (size_t)P * 3 * sizeof(double)) != hipSuccess) {
        cleanup();
        return set_err(ctx, GBS_E_NOMEM, "exact: device allocation failed");
    }
    hipError_t e = hipMemcpyAsync(d_off, offsets, (P + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nnz)
        e = hipMemcpyAsync(d_modes, modes, nnz * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        cleanup();
        return set_err(ctx, GBS_E_HIP, std::string("exact: ") + hipGetErrorString(e));
    }
    int rc = exact_launch(ctx, P, d_off, d_modes, maxn, d_part, d_out, d_out + P, d_out + 2 * P, d_st);
    std::vector<double> out((size_t)P * 3);
    if (!rc) {
        e = hipMemcpyAsync(out.data(), d_out, out.size() * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(status, d_st, P * sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = set_err(ctx, GBS_E_HIP, std::string("exact: ") + hipGetErrorString(e));
    }
    cleanup();
    if (rc) return rc;
    for (int r = 0; r < P; ++r) {
        p[r] = out[r];
        if (logp) logp[r] = out[P + r];
        if (kappa) kappa[r] = out[2 * (size_t)P + r];
    }
    return 0;
}
