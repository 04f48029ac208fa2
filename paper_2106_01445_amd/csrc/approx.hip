// Order-j estimate of click-pattern probabilities (Results, Approximation
// scheme; Methods, Partition function, Moments calculation, Approximation
// method), fp64, one MI355X.
//
// Pipeline per batch (all on one stream, no host synchronisation):
//   k_eig          (eig.hip) one workgroup per row: A = (Q^{-1})_CC gathered,
//                  A = V diag(alpha) V^T, log det A, log P_vac(Cbar), contour
//                  radius rho and size K
//   k_build_items  one workgroup: (row, chunk of contour points) work items in
//                  decreasing-cost row order, queue counters reset
//   k_contour      persistent workgroups pulling items from an atomic queue;
//                  per contour point w: d = 1/(1 + w(alpha-1)),
//                  M(w) = V diag(d) V^T as 2x2 mode blocks in LDS, and the sums
//                  over clusters T (|T| <= j) of det(M_TT)^{-1/2}, evaluated by
//                  2x2-block elimination with one principal square root per
//                  block (each block's determinant lies off the negative axis);
//                  the results, times G_0(w)/G_0(rho), go to HBM
//   k_dft_fit      one workgroup per row: sector moments by a direct DFT over the
//                  contour, one max-entropy fit per sector, log-sum over sectors
#include "contour_common.h"


namespace {

// ---------------------------------------------------------------------------
// k_build_items: work items (row, chunk) in the plan's cost order.  The rows
// perm[0..nbig) (the large ones) come first: their items form the queue
// counter[4] (length) / counter[5] (head); the rest form counter[0] (end) /
// counter[1] (head, starting at counter[4]).  With only_flags, only the rows
// carrying one of those flags from the previous fit get items (the fp64 rerun
// of the mixed precision tier, and the re-tilted rows).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_build_items(int P, int nbig, int qchunk,
                                                      const int *__restrict__ offsets,
                                                      const int *__restrict__ perm,
                                                      const RowPlan *__restrict__ rows,
                                                      int *__restrict__ items,
                                                      int *__restrict__ counter, int only_flags = 0)
{
    __shared__ int part[1024];
    __shared__ int s_big;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (P + nt - 1) / nt;
    const int b = tid * per, e = min(P, b + per);
    auto nch = [&](int i) {
        int p = perm[i];
        int n = offsets[p + 1] - offsets[p];
        const RowPlan &rp = rows[p];
        if (n == 0 || rp.status != 0 || rp.K <= 0) return 0;
        if (only_flags && !(rp.flags & only_flags)) return 0;
        return (rp.K / 2 + 1 + qchunk - 1) / qchunk;
    };
    if (tid == 0) s_big = 0;
    int s = 0, sb = 0;
    for (int i = b; i < e; ++i) {
        const int c = nch(i);
        s += c;
        if (i < nbig) sb += c;
    }
    part[tid] = s;
    __syncthreads();
    if (sb) atomicAdd(&s_big, sb);
    if (tid == 0) {
        int acc = 0;
        for (int t = 0; t < nt; ++t) {
            int v = part[t];
            part[t] = acc;
            acc += v;
        }
        counter[0] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        counter[1] = s_big;
        counter[4] = s_big;
        counter[5] = 0;
    }
    int off = part[tid];
    for (int i = b; i < e; ++i) {
        int c = nch(i), p = perm[i];
        for (int k = 0; k < c; ++k) {
            items[2 * (off + k)] = p;
            items[2 * (off + k) + 1] = k;
        }
        off += c;
    }
}

// ---------------------------------------------------------------------------
// k_contour: cluster sums at contour points.
//
// A work item is (row, chunk of GBS_QCHUNK contour points).  The row's
// eigenvectors stay in LDS for the whole item; G contour points are processed
// per pass, G the largest power of two <= 8 whose G copies of M(w) fit in LDS
// next to V.  Per pass: z_k = 1 + w(alpha_k - 1), d_k = 1/z_k and z_k^{-1/2} for
// every slot; M(w) = V diag(d) V^T as 2x2 mode blocks; then the clusters, with
// the threads split into G slot groups of whole wavefronts.
//
// LDS layout of M(w): the diagonal blocks (a,a) and the blocks (a,b), a < b,
// column-major (index b(b-1)/2 + a), each of the 3 or 4 entries in its own
// array.  The clusters come as work units (pair (a,b) and a segment [c0, c1) of
// third modes c > b, listed longest first); the threads of a slot group take
// units in turn.  Neighbouring lanes mostly hold consecutive a of the same b
// and segment, so the reads of the triple loop are broadcasts (blocks (b,c),
// (c,c)) or consecutive across lanes (block (a,c)).
// ---------------------------------------------------------------------------
// (RERUN: the same kernel for the second pass of a call, under its own name so
// that traces keep the two passes apart)
template <int ORDER, bool BIG, class C, bool RERUN = false>
__global__ __launch_bounds__(CONT_THREADS) void k_contour(
    int lds_bytes, int qchunk, int gmax, const int *__restrict__ offsets,
    const long long *__restrict__ voff,
    const double *__restrict__ alpha, const double *__restrict__ vt,
    const RowPlan *__restrict__ rows, const int *__restrict__ items, const int *__restrict__ q_end,
    int *__restrict__ q_head, const int *__restrict__ units, const int *__restrict__ unit_off,
    const int *__restrict__ unit4_off, cplx *__restrict__ mscr, long long mscr_stride, cplx *__restrict__ sw)
{
    extern __shared__ __attribute__((aligned(16))) double sh[];
    __shared__ int s_item;
    __shared__ cplx s_wq[GBS_QCHUNK_MAX];                    // the item's contour points
    cplx *red = (cplx *)sh;                                  // [waves][4]
    cplx *ghat = red + (CONT_THREADS / 64) * 4;              // [CONT_MAXG]
    double *dyn = (double *)(ghat + CONT_MAXG);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int total = *q_end;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(q_head, 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= total) break;
        const int p = items[2 * item], ch = items[2 * item + 1];
        const int o = offsets[p], n = offsets[p + 1] - o, N = 2 * n;
        const RowPlan rp = rows[p];
        const long long vo = voff[p];
        const int mstride = cont_mbytes<C>(n) / 16;  // one slot, in complex fp64 units
        const double *Vt;                       // eigenvector k contiguous, row stride vs
        double *al;                             // N
        cplx *slots;                            // G x (2n^2 + 5n) complex
        int G = 1;
        if (BIG) {
            // eigenvectors read from HBM (L2); M(w) in LDS when it fits, else in
            // this workgroup's HBM scratch
            Vt = vt + vo;
            al = dyn;
            // (order 2: only d, rz and the diagonal blocks are stored, in LDS)
            slots = ORDER == 2 || cont_fixed() + 8 * N + cont_mbytes<C>(n) <= lds_bytes
                        ? (cplx *)(al + N)
                        : mscr + blockIdx.x * mscr_stride;
        } else {
            // V and each slot's d zero-padded to whole tiles (no operand masks)
            const int tp = cont_tp(n), vsp = tp + 1;
            double *vl = dyn;
            al = vl + tp * vsp;
            slots = (cplx *)(al + N);
            G = gmax;
            while (G > 1 && cont_fixed() + cont_vbytes(n) + G * cont_mbytes<C>(n) > lds_bytes) G >>= 1;
            for (int idx = tid; idx < tp * vsp; idx += CONT_THREADS) {
                const int k = idx / vsp, i = idx - k * vsp;
                vl[idx] = k < N && i < N ? vt[vo + k * N + i] : 0.0;
            }
            for (int idx = tid; idx < G * (tp - N); idx += CONT_THREADS) {
                const int sl = idx / (tp - N), k = N + idx - sl * (tp - N);
                slots[sl * mstride + k] = cmk(0.0, 0.0);
            }
            Vt = vl;
        }
        for (int i = tid; i < N; i += CONT_THREADS) al[i] = alpha[2 * o + i];
        const int vs = BIG ? N : cont_tp(n) + 1;
        const int Q = rp.K / 2 + 1;
        const int q0 = ch * qchunk, q1 = min(q0 + qchunk, Q);
        const int np = n * (n - 1) / 2;
        // the item's contour points w_q = rho e^{2 pi i q / K}
        if (tid < q1 - q0) {
            s_wq[tid] = cscale(unit_root(q0 + tid, rp.K), rp.rho);
        }
        __syncthreads();
        // (every pass ends with a barrier, so the next pass may write its slots
        // at once)
        for (int qb = q0; qb < q1; qb += G) {
            const int g = min(G, q1 - qb);
            // d_k = 1/z_k and z_k^{-1/2}, z_k = 1 + w(alpha_k - 1); Re z_k > 0 inside
            // the convergence radius, so the principal root is the branch that is
            // continuous from w = 0
            for (int idx = tid; idx < g * N; idx += CONT_THREADS) {
                const int sl = idx / N, k = idx - sl * N;
                const cplx w = s_wq[qb - q0 + sl];
                const double am1 = al[k] - 1.0;
                const cplx z = cmk(fma(w.re, am1, 1.0), w.im * am1);
                const cplx rz = crsqrt_p(z);
                const SlotMT<C> m = slot_view<C>(slots + sl * mstride, n);
                m.d[k] = cmul(rz, rz);
                m.rz[k] = rz;
            }
            __syncthreads();
            if (wid < g) {
                // G_0(w)/G_0(rho) = exp(log det A/2 - log G_0(rho)) prod_k z_k^{-1/2},
                // slot wid's product over the lanes of wavefront wid
                const SlotMT<C> m = slot_view<C>(slots + wid * mstride, n);
                cplx pr = cmk(1.0, 0.0);
                for (int k = lane; k < N; k += 64) pr = cmul(pr, m.rz[k]);
                pr = cmul(warp_cprod(pr), cmk(exp(0.5 * rp.logdet_a - rp.log_g_rho), 0.0));
                if (lane == 0) ghat[wid] = pr;
            }
            // M(w) = V diag(d) V^T: at order >= 2 every 2x2 mode block, as the upper
            // 16x16 tiles of the 2n x 2n matrix on the matrix cores (one wavefront
            // per (slot, tile)); at order 1 only the diagonal blocks
            static_assert(GBS_MAX_N_APPROX <= 16 * (CONT_THREADS / 64), "one diagonal mode block per wavefront");
            cplx s2f = cmk(0.0, 0.0);  // pair sums of the fused order-2 path below
            if (ORDER == 2 && BIG) {
                // Order 2, V read from L2: M(w) is never stored whole.  For a 16 x 16
                // block (I, J) of modes the four quadrant products x_a x_b, x_a p_b,
                // p_a x_b and p_a p_b land in the same accumulator positions, so each
                // lane holds the whole 2x2 block of its pairs (a, b) (row a = 16 I +
                // 4e + l/16, column b = 16 J + l%16).  The diagonal blocks (I = I)
                // come first, for the diagonal 2x2 blocks M_aa that every pair needs
                // (stored in LDS); their pairs follow from registers.
                const SlotMT<C> m = slot_view<C>(slots, n);
                const int TM = (n + 15) / 16, KS = (N + 3) >> 2;
                const int lq = lane >> 4, l16 = lane & 15;
                auto quad = [&](int I, int J, dbl4 (&q)[4][2]) {
#pragma unroll
                    for (int h = 0; h < 4; ++h) q[h][0] = q[h][1] = dbl4{0.0, 0.0, 0.0, 0.0};
                    const int ia = 16 * I + l16, jb = 16 * J + l16;
#pragma unroll 2
                    for (int ks = 0; ks < KS; ++ks) {
                        const int k = ks * 4 + lq;
                        const bool kok = k < N, aok = kok && ia < n, bok = kok && jb < n;
                        const cplx dl = m.d[kok ? k : 0];
                        const double axl = Vt[aok ? k * N + ia : 0], apl = Vt[aok ? k * N + n + ia : 0];
                        const double bxl = Vt[bok ? k * N + jb : 0], bpl = Vt[bok ? k * N + n + jb : 0];
                        const double ax = aok ? axl : 0.0, ap = aok ? apl : 0.0;
                        const double bx = bok ? bxl : 0.0, bp = bok ? bpl : 0.0;
                        const double axr = ax * dl.re, axi = ax * dl.im, apr = ap * dl.re, api = ap * dl.im;
                        q[0][0] = mfma4(axr, bx, q[0][0]);
                        q[0][1] = mfma4(axi, bx, q[0][1]);
                        q[1][0] = mfma4(axr, bp, q[1][0]);
                        q[1][1] = mfma4(axi, bp, q[1][1]);
                        q[2][0] = mfma4(apr, bx, q[2][0]);
                        q[2][1] = mfma4(api, bx, q[2][1]);
                        q[3][0] = mfma4(apr, bp, q[3][0]);
                        q[3][1] = mfma4(api, bp, q[3][1]);
                    }
                };
                auto pairs = [&](int I, int J, const dbl4 (&q)[4][2]) {
                    const int b = 16 * J + l16;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int a = 16 * I + 4 * e + lq;
                        if (a < b && b < n) {
                            const C b00 = from_d<C>(cmk(q[0][0][e], q[0][1][e]));
                            const C b01 = from_d<C>(cmk(q[1][0][e], q[1][1][e]));
                            const C b10 = from_d<C>(cmk(q[2][0][e], q[2][1][e]));
                            const C b11 = from_d<C>(cmk(q[3][0][e], q[3][1][e]));
                            const C a00 = m.d0[a], a01 = m.d1[a], a11 = m.d2[a];
                            const C deta = cfnma(a01, a01, cmul(a00, a11));
                            const C ra = crsqrt_p(deta);
                            const C ideta = cmul(ra, ra);
                            const C ia00 = cmul(a11, ideta), ia11 = cmul(a00, ideta);
                            const C ia01 = cneg(cmul(a01, ideta));
                            const C G00 = cfma(ia00, b00, cmul(ia01, b10));
                            const C G01 = cfma(ia00, b01, cmul(ia01, b11));
                            const C G10 = cfma(ia01, b00, cmul(ia11, b10));
                            const C G11 = cfma(ia01, b01, cmul(ia11, b11));
                            const C sb00 = csub(m.d0[b], cfma(b00, G00, cmul(b10, G10)));
                            const C sb01 = csub(m.d1[b], cfma(b00, G01, cmul(b10, G11)));
                            const C sb11 = csub(m.d2[b], cfma(b01, G01, cmul(b11, G11)));
                            const C rb = crsqrt_p(cfnma(sb01, sb01, cmul(sb00, sb11)));
                            s2f = cadd(s2f, to_d(cmul(ra, rb)));
                        }
                    }
                };
                dbl4 qd[4][2];
                if (wid < TM) {
                    quad(wid, wid, qd);
                    const int b = 16 * wid + l16;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (4 * e + lq == l16 && b < n) {
                            m.d0[b] = from_d<C>(cmk(qd[0][0][e], qd[0][1][e]));
                            m.d1[b] = from_d<C>(cmk(qd[1][0][e], qd[1][1][e]));
                            m.d2[b] = from_d<C>(cmk(qd[3][0][e], qd[3][1][e]));
                        }
                }
                __syncthreads();
                if (wid < TM) pairs(wid, wid, qd);
                for (int u = wid; u < TM * (TM - 1) / 2; u += CONT_THREADS / 64) {
                    int I, J;
                    upper_tile(u, I, J);
                    dbl4 q[4][2];
                    quad(I, J + 1, q);
                    pairs(I, J + 1, q);
                }
            } else if (ORDER >= 2) {
                // BIG: V comes from L2, so 2x2 blocks of tiles share each operand fetch
                constexpr int BS = BIG ? 2 : 1;
                const int T = (N + 16 * BS - 1) / (16 * BS), ntile = T * (T + 1) / 2;
                // (dealt from the last wavefront down: wavefronts 0..g-1 form
                // the G_0(w) products first)
                for (int c = CONT_THREADS / 64 - 1 - wid; c < g * ntile; c += CONT_THREADS / 64) {
                    const int sl = c / ntile;
                    int it, jt;
                    upper_tile(c - sl * ntile, it, jt);
                    const SlotMT<C> m = slot_view<C>(slots + sl * mstride, n);
                    m_block_mfma<BS, C, false, !BIG>(n, it, jt, Vt, vs, m.d, m.d0, lane);
                }
            } else {
                for (int idx = tid; idx < g * n; idx += CONT_THREADS) {
                    const int sl = idx / n, a = idx - sl * n;
                    const SlotMT<C> m = slot_view<C>(slots + sl * mstride, n);
                    cplx m00 = cmk(0, 0), m01 = cmk(0, 0), m11 = cmk(0, 0);
#pragma unroll 1
                    for (int k = 0; k < N; ++k) {
                        const double v0 = Vt[k * vs + a], v1 = Vt[k * vs + n + a];
                        const cplx d = m.d[k];
                        const double p00 = v0 * v0, p01 = v0 * v1, p11 = v1 * v1;
                        m00.re = fma(p00, d.re, m00.re); m00.im = fma(p00, d.im, m00.im);
                        m01.re = fma(p01, d.re, m01.re); m01.im = fma(p01, d.im, m01.im);
                        m11.re = fma(p11, d.re, m11.re); m11.im = fma(p11, d.im, m11.im);
                    }
                    m.d0[a] = from_d<C>(m00);
                    m.d1[a] = from_d<C>(m01);
                    m.d2[a] = from_d<C>(m11);
                }
            }
            __syncthreads();
            // clusters: slot groups of SG threads (whole wavefronts)
            const int SG = CONT_THREADS / G;
            const int sl = tid / SG, lt = tid - sl * SG;
            cplx s1 = cmk(0, 0), s2 = cmk(0, 0), s3 = cmk(0, 0), s4 = cmk(0, 0);
            if (sl < g) {
                const SlotMT<C> m = slot_view<C>(slots + sl * mstride, n);
                for (int a = lt; a < n; a += SG) {
                    const C a00 = m.d0[a], a01 = m.d1[a], a11 = m.d2[a];
                    s1 = cadd(s1, to_d(crsqrt_p(cfnma(a01, a01, cmul(a00, a11)))));
                }
                if (ORDER == 2 && BIG) s2 = s2f;
                if (ORDER >= 2 && !(ORDER == 2 && BIG)) {
                    const int *un = units + unit_off[2 * n];
                    const int nu = unit_off[2 * n + 1];
                    int unext = lt < nu ? un[lt] : 0;
#pragma unroll 1
                    for (int ui = lt; ui < nu; ui += SG) {
                        const unsigned u = (unsigned)unext;
                        if (ui + SG < nu) unext = un[ui + SG];
                        const int a = u & 255, b = (u >> 8) & 255, c0 = (u >> 16) & 255, c1 = u >> 24;
                        const int pi = b * (b - 1) / 2 + a;
                        const C a00 = m.d0[a], a01 = m.d1[a], a11 = m.d2[a];
                        const C b00 = m.o0[pi], b01 = m.o1[pi], b10 = m.o2[pi], b11 = m.o3[pi];
                        const C bb00 = m.d0[b], bb01 = m.d1[b], bb11 = m.d2[b];
                        const C deta = cfnma(a01, a01, cmul(a00, a11));
                        const C ra = crsqrt_p(deta);
                        const C ideta = cmul(ra, ra);
                        const C ia00 = cmul(a11, ideta), ia11 = cmul(a00, ideta);
                        const C ia01 = cneg(cmul(a01, ideta));
                        // G = Maa^{-1} Mab ; Sb = Mbb - Mab^T G
                        const C G00 = cfma(ia00, b00, cmul(ia01, b10));
                        const C G01 = cfma(ia00, b01, cmul(ia01, b11));
                        const C G10 = cfma(ia01, b00, cmul(ia11, b10));
                        const C G11 = cfma(ia01, b01, cmul(ia11, b11));
                        const C sb00 = csub(bb00, cfma(b00, G00, cmul(b10, G10)));
                        const C sb01 = csub(bb01, cfma(b00, G01, cmul(b10, G11)));
                        const C sb11 = csub(bb11, cfma(b01, G01, cmul(b11, G11)));
                        const C detb = cfnma(sb01, sb01, cmul(sb00, sb11));
                        const C rb = crsqrt_p(detb);
                        const C rab = cmul(ra, rb);
                        if (c0 == b + 1) s2 = cadd(s2, to_d(rab));
                        if (ORDER >= 3) {
                            const C idetb = cmul(rb, rb);
                            const C ib00 = cmul(sb11, idetb), ib11 = cmul(sb00, idetb);
                            const C ib01 = cneg(cmul(sb01, idetb));
                            cplx s3p = cmk(0, 0);
                            // (column offsets stepped along c: (c + 1) c / 2 = c (c - 1) / 2 + c)
                            int cb = c0 * (c0 - 1) / 2;
#pragma unroll 1
                            for (int c = c0; c < c1; cb += c, ++c) {
                                const int iac = cb + a, ibc = cb + b;
                                // Sc = Mcc - Xa^T Maa^{-1} Xa - Y^T Sb^{-1} Y, Y = Xb - G^T Xa,
                                // evaluated so that each intermediate dies early (the
                                // blocks are all read first, so that their LDS reads overlap)
                                const C x00 = m.o0[iac], x01 = m.o1[iac], x10 = m.o2[iac], x11 = m.o3[iac];
                                const C y00 = m.o0[ibc], y01 = m.o1[ibc], y10 = m.o2[ibc], y11 = m.o3[ibc];
                                C sc00 = m.d0[c], sc01 = m.d1[c], sc11 = m.d2[c];
                                {
                                    const C Z00 = cfma(ia00, x00, cmul(ia01, x10));
                                    const C Z10 = cfma(ia01, x00, cmul(ia11, x10));
                                    sc00 = csub(sc00, cfma(x00, Z00, cmul(x10, Z10)));
                                    const C Z01 = cfma(ia00, x01, cmul(ia01, x11));
                                    const C Z11 = cfma(ia01, x01, cmul(ia11, x11));
                                    sc01 = csub(sc01, cfma(x00, Z01, cmul(x10, Z11)));
                                    sc11 = csub(sc11, cfma(x01, Z01, cmul(x11, Z11)));
                                }
                                const C Y00 = csub(y00, cfma(G00, x00, cmul(G10, x10)));
                                const C Y01 = csub(y01, cfma(G00, x01, cmul(G10, x11)));
                                const C Y10 = csub(y10, cfma(G01, x00, cmul(G11, x10)));
                                const C Y11 = csub(y11, cfma(G01, x01, cmul(G11, x11)));
                                {
                                    const C W00 = cfma(ib00, Y00, cmul(ib01, Y10));
                                    const C W10 = cfma(ib01, Y00, cmul(ib11, Y10));
                                    sc00 = csub(sc00, cfma(Y00, W00, cmul(Y10, W10)));
                                    const C W01 = cfma(ib00, Y01, cmul(ib01, Y11));
                                    const C W11 = cfma(ib01, Y01, cmul(ib11, Y11));
                                    sc01 = csub(sc01, cfma(Y00, W01, cmul(Y10, W11)));
                                    sc11 = csub(sc11, cfma(Y01, W01, cmul(Y11, W11)));
                                }
                                s3p = cadd(s3p, to_d(crsqrt_p(cfnma(sc01, sc01, cmul(sc00, sc11)))));
                            }
                            s3 = cfma(to_d(rab), s3p, s3);
                        }
                    }
                }
                if (ORDER >= 4) {
                    // quadruples (a, b, c, d): units (a, b, c; d0..d0+len-1).  With the
                    // pair P = {a, b} eliminated (Maa^{-1}, G, Sb^{-1}) and then c (its
                    // Schur complement Sc), each d costs the 2x2 Schur complement
                    //   Sd = Mdd - r^T P^{-1} r - u^T Sc^{-1} u,  r = [Mad; Mbd],
                    //   u = Mcd - [Mac; Mbc]^T P^{-1} r,
                    // where s^T P^{-1} r = (Maa^{-1} xs)^T x + Ys^T Sb^{-1} Y for
                    // s = [xs; ys], Y = y - G^T x, Ys = ys - G^T xs; and
                    // det M_TT = det Maa det Sb det Sc det Sd
                    const int *un4 = units + unit4_off[2 * n];
                    const int nu4 = unit4_off[2 * n + 1];
#pragma unroll 1
                    for (int ui = lt; ui < nu4; ui += SG) {
                        const unsigned u = (unsigned)un4[ui];
                        const int a = u & 63, b = (u >> 6) & 63, c = (u >> 12) & 63, d0 = (u >> 18) & 63,
                                  d1 = d0 + (int)(u >> 24);
                        const int pi = b * (b - 1) / 2 + a;
                        const C a00 = m.d0[a], a01 = m.d1[a], a11 = m.d2[a];
                        const C b00 = m.o0[pi], b01 = m.o1[pi], b10 = m.o2[pi], b11 = m.o3[pi];
                        const C ra = crsqrt_p(cfnma(a01, a01, cmul(a00, a11)));
                        const C ideta = cmul(ra, ra);
                        const C ia00 = cmul(a11, ideta), ia11 = cmul(a00, ideta);
                        const C ia01 = cneg(cmul(a01, ideta));
                        const C G00 = cfma(ia00, b00, cmul(ia01, b10));
                        const C G01 = cfma(ia00, b01, cmul(ia01, b11));
                        const C G10 = cfma(ia01, b00, cmul(ia11, b10));
                        const C G11 = cfma(ia01, b01, cmul(ia11, b11));
                        const C sb00 = csub(m.d0[b], cfma(b00, G00, cmul(b10, G10)));
                        const C sb01 = csub(m.d1[b], cfma(b00, G01, cmul(b10, G11)));
                        const C sb11 = csub(m.d2[b], cfma(b01, G01, cmul(b11, G11)));
                        const C rb = crsqrt_p(cfnma(sb01, sb01, cmul(sb00, sb11)));
                        const C idetb = cmul(rb, rb);
                        const C ib00 = cmul(sb11, idetb), ib11 = cmul(sb00, idetb);
                        const C ib01 = cneg(cmul(sb01, idetb));
                        // c: xc = Mac, Zc = Maa^{-1} xc, Yc = Mbc - G^T xc, Wc = Sb^{-1} Yc
                        const int cb = c * (c - 1) / 2;
                        const C xc00 = m.o0[cb + a], xc01 = m.o1[cb + a], xc10 = m.o2[cb + a], xc11 = m.o3[cb + a];
                        const C Zc00 = cfma(ia00, xc00, cmul(ia01, xc10)), Zc10 = cfma(ia01, xc00, cmul(ia11, xc10));
                        const C Zc01 = cfma(ia00, xc01, cmul(ia01, xc11)), Zc11 = cfma(ia01, xc01, cmul(ia11, xc11));
                        const C Yc00 = csub(m.o0[cb + b], cfma(G00, xc00, cmul(G10, xc10)));
                        const C Yc01 = csub(m.o1[cb + b], cfma(G00, xc01, cmul(G10, xc11)));
                        const C Yc10 = csub(m.o2[cb + b], cfma(G01, xc00, cmul(G11, xc10)));
                        const C Yc11 = csub(m.o3[cb + b], cfma(G01, xc01, cmul(G11, xc11)));
                        const C Wc00 = cfma(ib00, Yc00, cmul(ib01, Yc10)), Wc10 = cfma(ib01, Yc00, cmul(ib11, Yc10));
                        const C Wc01 = cfma(ib00, Yc01, cmul(ib01, Yc11)), Wc11 = cfma(ib01, Yc01, cmul(ib11, Yc11));
                        const C sc00 = csub(m.d0[c], cfma(xc00, Zc00, cfma(xc10, Zc10, cfma(Yc00, Wc00, cmul(Yc10, Wc10)))));
                        const C sc01 = csub(m.d1[c], cfma(xc00, Zc01, cfma(xc10, Zc11, cfma(Yc00, Wc01, cmul(Yc10, Wc11)))));
                        const C sc11 = csub(m.d2[c], cfma(xc01, Zc01, cfma(xc11, Zc11, cfma(Yc01, Wc01, cmul(Yc11, Wc11)))));
                        const C rc = crsqrt_p(cfnma(sc01, sc01, cmul(sc00, sc11)));
                        const C idetc = cmul(rc, rc);
                        const C ic00 = cmul(sc11, idetc), ic11 = cmul(sc00, idetc);
                        const C ic01 = cneg(cmul(sc01, idetc));
                        cplx s4p = cmk(0, 0);
#pragma unroll 1
                        for (int d = d0; d < d1; ++d) {
                            const int db = d * (d - 1) / 2;
                            const int iad = db + a, ibd = db + b, icd = db + c;
                            const C x00 = m.o0[iad], x01 = m.o1[iad], x10 = m.o2[iad], x11 = m.o3[iad];
                            const C Y00 = csub(m.o0[ibd], cfma(G00, x00, cmul(G10, x10)));
                            const C Y01 = csub(m.o1[ibd], cfma(G00, x01, cmul(G10, x11)));
                            const C Y10 = csub(m.o2[ibd], cfma(G01, x00, cmul(G11, x10)));
                            const C Y11 = csub(m.o3[ibd], cfma(G01, x01, cmul(G11, x11)));
                            const C W00 = cfma(ib00, Y00, cmul(ib01, Y10)), W10 = cfma(ib01, Y00, cmul(ib11, Y10));
                            const C W01 = cfma(ib00, Y01, cmul(ib01, Y11)), W11 = cfma(ib01, Y01, cmul(ib11, Y11));
                            C q00, q01, q11;
                            {
                                const C Z00 = cfma(ia00, x00, cmul(ia01, x10)), Z10 = cfma(ia01, x00, cmul(ia11, x10));
                                const C Z01 = cfma(ia00, x01, cmul(ia01, x11)), Z11 = cfma(ia01, x01, cmul(ia11, x11));
                                q00 = csub(m.d0[d], cfma(x00, Z00, cfma(x10, Z10, cfma(Y00, W00, cmul(Y10, W10)))));
                                q01 = csub(m.d1[d], cfma(x00, Z01, cfma(x10, Z11, cfma(Y00, W01, cmul(Y10, W11)))));
                                q11 = csub(m.d2[d], cfma(x01, Z01, cfma(x11, Z11, cfma(Y01, W01, cmul(Y11, W11)))));
                            }
                            // u[i][j] = Mcd[i][j] - sum_k (Zc[k][i] x[k][j] + Yc[k][i] W[k][j])
                            const C u00 = csub(m.o0[icd], cfma(Zc00, x00, cfma(Zc10, x10, cfma(Yc00, W00, cmul(Yc10, W10)))));
                            const C u01 = csub(m.o1[icd], cfma(Zc00, x01, cfma(Zc10, x11, cfma(Yc00, W01, cmul(Yc10, W11)))));
                            const C u10 = csub(m.o2[icd], cfma(Zc01, x00, cfma(Zc11, x10, cfma(Yc01, W00, cmul(Yc11, W10)))));
                            const C u11 = csub(m.o3[icd], cfma(Zc01, x01, cfma(Zc11, x11, cfma(Yc01, W01, cmul(Yc11, W11)))));
                            // v = Sc^{-1} u; Sd = q - u^T v
                            const C v00 = cfma(ic00, u00, cmul(ic01, u10)), v10 = cfma(ic01, u00, cmul(ic11, u10));
                            const C v01 = cfma(ic00, u01, cmul(ic01, u11)), v11 = cfma(ic01, u01, cmul(ic11, u11));
                            q00 = csub(q00, cfma(u00, v00, cmul(u10, v10)));
                            q01 = csub(q01, cfma(u00, v01, cmul(u10, v11)));
                            q11 = csub(q11, cfma(u01, v01, cmul(u11, v11)));
                            s4p = cadd(s4p, to_d(crsqrt_p(cfnma(q01, q01, cmul(q00, q11)))));
                        }
                        s4 = cfma(to_d(cmul(cmul(ra, rb), rc)), s4p, s4);
                    }
                }
            }
            s1 = warp_csum(s1);
            s2 = warp_csum(s2);
            s3 = warp_csum(s3);
            if (ORDER >= 4) s4 = warp_csum(s4);
            if (lane == 0) {
                red[4 * wid + 1] = s1;
                red[4 * wid + 2] = s2;
                red[4 * wid + 3] = s3;
                if (ORDER >= 4) red[4 * wid] = s4;  // (slot 0 is free: t = 4 takes it)
            }

            __syncthreads();
            if (tid < g * (ORDER + 1)) {
                const int s = tid / (ORDER + 1), t = tid - s * (ORDER + 1);
                cplx acc = cmk(1.0, 0.0);
                if (t > 0) {
                    acc = cmk(0.0, 0.0);
                    const int w0 = s * (SG / 64), w1 = w0 + SG / 64;
                    for (int w = w0; w < w1; ++w) acc = cadd(acc, red[4 * w + (t & 3)]);
                }
                sw[((long)p * (ORDER + 1) + t) * GBS_QCAP + qb + s] = cmul(ghat[s], acc);
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// k_dft_fit: sector moments, fits, log-sum, and the estimated rounding error of
// the result.
//
// Rounding estimate.  A contour value S_t(w_q) carries a relative rounding
// error of about u_t (u_0 = ROUND_FP64 for the fp64 G_0; u_t = u_clu for the
// cluster sums), so each tilted moment tau_t[kappa] carries at most
// d_t = u_t mean_q |S_t(w_q)| (the transform's triangle inequality).  In a
// fitted sector, m_t = tau_t binv_t / tau_0 and d log q / d m = -u with
// u = H^{-1} m, so
//   |d log(term)| <= d_0 / tau_0 (1 + sum_t |u_t m_t|) + sum_t |u_t| binv_t d_t / tau_0,
// and the row's estimate is the sum over sectors weighted by their shares of
// the estimate.
//   pass 0: every row; a row whose estimate exceeds esc_bound (> 0 only in
//           mixed precision) is marked GBS_PS_ESCALATED, to be run again in
//           fp64 (pass 1, only the marked rows).  A row whose estimate sits in
//           sectors the contour does not resolve (their tilted weights, as a
//           harmonic mean weighted by their shares of the estimate, below
//           1e-6) is marked for a re-tilt when allow_retilt: k_retilt centres
//           its contour on the estimate's mean photon number kbar and pass 1
//           runs it again; where that is not possible it is flagged
//           GBS_PS_CONTOUR.
// ---------------------------------------------------------------------------
template <int ORDER, int PASS = 0>
__global__ __launch_bounds__(FIT_THREADS) void k_dft_fit(const int *__restrict__ offsets,
                                                         RowPlan *__restrict__ rows,
                                                         const cplx *__restrict__ sw,
                                                         double *__restrict__ logp,
                                                         int *__restrict__ status, double u_clu,
                                                         double esc_bound, int allow_retilt)
{
    constexpr int pass = PASS;
    extern __shared__ __attribute__((aligned(16))) double sh[];
    __shared__ double red[FIT_THREADS], red2[FIT_THREADS];
    const int p = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int n = offsets[p + 1] - offsets[p];
    RowPlan rp = rows[p];
    if (pass == 1 && !(rp.flags & (GBS_PS_ESCALATED | GBS_ROW_RETILT))) return;
    if (n == 0) {
        if (tid == 0) {
            logp[p] = rp.log_pvac;
            if (status) status[p] = 0;
            rows[p].err = 0.0;
        }
        return;
    }
    if (rp.status != 0) {
        if (tid == 0) {
            logp[p] = NAN;
            if (status) status[p] = rp.status | (rp.flags & GBS_PS_PUBLIC);
        }
        return;
    }
    const int K = rp.K, Q = K / 2 + 1, jp = min(ORDER, n - 1);
    const DftShape dsh = dft_shape(K);
    cplx *X = (cplx *)sh;            // K
    cplx *W = X + K;                 // K/2
    for (int m = tid; m < K / 2; m += nt) {
        const cplx u = unit_root(m, K);
        W[m] = cmk(u.re, -u.im);
    }
    // tilted sector moments tau_t[kappa] = Re FFT(S_t(w_q))[kappa] / K, where the
    // points q > K/2 are the conjugates of K - q (real coefficients)
    // (loops over t and j unrolled: every index into tau is static)
    constexpr int NT = ORDER >= 4 ? 5 : 4;  // moments held per sector
    double tau[FIT_KPT][NT];
    const double invK = 1.0 / K;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t <= ORDER && t <= jp) {
            const cplx *src = sw + ((long)p * (ORDER + 1) + t) * GBS_QCAP;
            for (int q = tid; q < K; q += nt) {
                const cplx v = q < Q ? src[q] : cmk(src[K - q].re, -src[K - q].im);
                const int rq = dft_pos(dsh, q);
                X[rq] = v;
            }
            __syncthreads();
            dft_lds(X, W, dsh);
#pragma unroll
            for (int j = 0; j < FIT_KPT; ++j) {
                const int kap = n + tid + nt * j;
                tau[j][t] = kap < K ? X[kap].re * invK : 0.0;
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int j = 0; j < FIT_KPT; ++j) tau[j][t] = 0.0;
        }
    }
    double tmax = 0.0;
    for (int j = 0; j < FIT_KPT; ++j)
        if (n + tid + nt * j < K) tmax = fmax(tmax, tau[j][0]);
    tmax = block_max(tmax, red);
    const double thr = 1e-14 * tmax;
    // rounding of the tilted moments: tau_t[kappa] = (1/K) sum_q S_t(w_q)
    // e^{-2 pi i q kappa / K}, so contour values with relative errors u_t
    // leave at most u_t (1/K) sum_q |S_t(w_q)| in each moment
    double dt[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        double s0 = 0.0;
        if (t <= ORDER && t <= jp) {
            const cplx *src = sw + ((long)p * (ORDER + 1) + (t <= ORDER ? t : 0)) * GBS_QCAP;
            double a = 0.0;
            for (int q = tid; q < Q; q += nt)
                a += (q == 0 || q == K / 2 ? 1.0 : 2.0) * sqrt(src[q].re * src[q].re + src[q].im * src[q].im);
            s0 = block_sum(a, red) / K;
        }
        dt[t] = (t == 0 ? ROUND_FP64 : u_clu) * s0;
    }
    double fm = -INFINITY, fs = 0.0, um = -INFINITY, us = 0.0;
    int nsec = 0;
    // log-sums of term_kappa * rounding estimate of log(term_kappa)
    double em = -INFINITY, es = 0.0, eh = -INFINITY, esh = 0.0, ek = -INFINITY, esk = 0.0;
    double lower = -INFINITY;  // log of a lower bound of the total (after pass 0)
    // Pass 0 fits each thread's first sector; its block log-sum is a lower
    // bound L of the estimate.  Later sectors whose upper bound S_0[kappa]
    // (q <= 1) is below 1e-17 L are skipped: they change the sum by < 1e-14.
#pragma unroll
    for (int j = 0; j < FIT_KPT; ++j) {
        if (j == 1) {
            double mx = block_max(fm, red);
            double sm = block_sum(fm == -INFINITY ? 0.0 : fs * exp(fm - mx), red);
            lower = sm > 0.0 ? mx + log(sm) : -INFINITY;
        }
        const int kap = n + tid + nt * j;
        if (kap >= K) continue;
        const double t0 = tau[j][0];
        if (!(t0 >= thr) || !(t0 > 0.0)) continue;
        const double lw = log(t0) + rp.log_g_rho - kap * rp.log_rho;
        if (lw < lower + log(1e-17)) continue;
        const SectorFitT<ORDER >= 4 ? 4 : 3> f =
            fit_sector<ORDER >= 4 ? 4 : 3>(n, 0, jp, t0, tau[j][1], tau[j][2], tau[j][3], ORDER >= 4 ? tau[j][NT - 1] : 0.0);
        if (f.bad) {
            lse_add(um, us, lw);
        } else {
            lse_add(fm, fs, lw + f.lq);
            ++nsec;
            double u[4];
            fit_sensitivity<ORDER >= 4 ? 4 : 3>(n, f, u);
            const double binv[4] = {1.0 / (n - 1.0), 2.0 / ((n - 1.0) * (n - 2.0)),
                                    6.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0)),
                                    24.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0) * (n - 4.0))};
            double um0 = 1.0, e1 = 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t < f.jr) {
                    um0 += fabs(u[t] * f.m[t]);
                    e1 += fabs(u[t]) * binv[t] * dt[t + 1];
                }
            const double e = (dt[0] * um0 + e1) / t0;
            lse_add(em, es, lw + f.lq + log(e));
            lse_add(eh, esh, lw + f.lq - log(t0));
            lse_add(ek, esk, lw + f.lq + log((double)kap));
        }
    }
    // block log-sum-exp of the fitted and the unresolved sectors
    double fmx = block_max(fm, red);
    double fsum = block_sum(fm == -INFINITY ? 0.0 : fs * exp(fm - fmx), red);
    double umx = block_max(um, red2);
    double usum = block_sum(um == -INFINITY ? 0.0 : us * exp(um - umx), red2);
    double ns = block_sum((double)nsec, red);
    const double emx = block_max(em, red2);
    const double esum = block_sum(em == -INFINITY ? 0.0 : es * exp(em - emx), red2);
    const double ehx = block_max(eh, red2);
    const double ehsum = block_sum(eh == -INFINITY ? 0.0 : esh * exp(eh - ehx), red2);
    const double ekx = block_max(ek, red2);
    const double eksum = block_sum(ek == -INFINITY ? 0.0 : esk * exp(ek - ekx), red2);
    if (tid == 0) {
        double tot = fmx + log(fsum);
        double unres = umx + log(usum);
        int stt = 0;
        double out = rp.log_pvac + tot;
        if (fsum > 0.0 && usum > 0.0 && unres > tot + log(1e-10)) {
            stt = GBS_PS_FIT_NOCONV;
            out = NAN;
        }
        if (!(fsum > 0.0)) out = -INFINITY;
        // estimated rounding error of log p_hat in this precision; the
        // contour cannot resolve the sectors that carry the estimate when their
        // tilted weights, averaged with their shares of the estimate (the
        // harmonic mean sum_kappa w_kappa / tau_kappa), fall below 1e-6: the
        // transform's rounding floor (~1e-16 of the contour's tilted weight)
        // then reaches 1e-10 of the estimate
        const double err = fsum > 0.0 && esum > 0.0 ? exp(emx + log(esum) - tot) : 0.0;
        int flags = rp.flags & ~GBS_ROW_RETILT;
        if (fsum > 0.0 && ehsum > 0.0 && ehx + log(ehsum) - tot > log(1e6)) {
            // the estimate's sectors lie far out in the tilted distribution: on
            // the first pass, tilt the contour afresh towards their mean photon
            // number and run the row again; otherwise report it
            const double kbar = eksum > 0.0 ? exp(ekx + log(eksum) - tot) : 0.0;
            const bool moves = kbar > 1.02 * rp.kbar ? rp.rho < 0.97 * rp.rconv : kbar < rp.kbar / 1.02;
            if (pass == 0 && allow_retilt && moves) {
                flags |= GBS_ROW_RETILT;
                rows[p].kbar = kbar;
                if (esc_bound > 0.0) flags |= GBS_PS_ESCALATED;  // (the rerun is fp64)
            } else {
                flags |= GBS_PS_CONTOUR;
            }
        }
        // (mixed precision: rows over the bound, and rows whose fits failed)
        if (pass == 0 && esc_bound > 0.0 && (!(err <= esc_bound) || stt != 0)) flags |= GBS_PS_ESCALATED;
        logp[p] = out;
        if (status) status[p] = stt | (flags & GBS_PS_PUBLIC);
        rows[p].nsec = (int)ns;
        rows[p].flags = flags;
        rows[p].err = err;
    }
}

// ---------------------------------------------------------------------------
// k_dist_fit: the whole device's click distribution (one row, C = every mode,
// n = M): per sector k (0 <= k < K) the tilted moments by the FFT, the
// exp-polynomial fitted on the sector's support n' = 1..min(k, n) (k photons
// click at most k detectors; k = 0 is the vacuum, n' = 0), and its whole curve:
// p_k(n') = S_0[k] q_k(n'), p(n') = sum_k p_k(n') (LDS accumulators, one block).
// Sectors below the transform's noise floor (1e-14 of the largest tilted
// weight) are left out; a sector whose fit fails sets GBS_PS_FIT_NOCONV when
// its weight exceeds 1e-10 of the total.
// ---------------------------------------------------------------------------
template <int ORDER>
__global__ __launch_bounds__(FIT_THREADS) void k_dist_fit(const int *__restrict__ offsets,
                                                          const RowPlan *__restrict__ rows,
                                                          const cplx *__restrict__ sw, int nk,
                                                          const int *__restrict__ ks, double *__restrict__ p_n,
                                                          double *__restrict__ p_k, int *__restrict__ status)
{
    extern __shared__ __attribute__((aligned(16))) double sh[];
    __shared__ double red[FIT_THREADS];
    __shared__ double pacc[2 * GBS_NSMALL + 2];
    __shared__ double s_fail;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n = offsets[1] - offsets[0];
    const RowPlan rp = rows[0];
    for (int i = tid; i <= n; i += nt) pacc[i] = 0.0;
    for (int i = tid; i < nk * (n + 1); i += nt) p_k[i] = 0.0;
    if (tid == 0) s_fail = 0.0;
    if (n == 0 || rp.status != 0) {
        for (int i = tid; i <= n; i += nt) p_n[i] = n == 0 ? 1.0 : NAN;
        if (tid == 0) *status = rp.status;
        return;
    }
    const int K = rp.K, Q = K / 2 + 1, jp = min(ORDER, n - 1);
    const DftShape dsh = dft_shape(K);
    cplx *X = (cplx *)sh;
    cplx *W = X + K;
    for (int m = tid; m < K / 2; m += nt) {
        const cplx u = unit_root(m, K);
        W[m] = cmk(u.re, -u.im);
    }
    constexpr int NT = ORDER >= 4 ? 5 : 4;
    double tau[FIT_KPT][NT];
    const double invK = 1.0 / K;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t <= ORDER && t <= jp) {
            const cplx *src = sw + (long)t * GBS_QCAP;  // (the row's planes: row 0)
            for (int q = tid; q < K; q += nt) {
                const cplx v = q < Q ? src[q] : cmk(src[K - q].re, -src[K - q].im);
                X[dft_pos(dsh, q)] = v;
            }
            __syncthreads();
            dft_lds(X, W, dsh);
#pragma unroll
            for (int j = 0; j < FIT_KPT; ++j) {
                const int kap = tid + nt * j;
                tau[j][t] = kap < K ? X[kap].re * invK : 0.0;
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int j = 0; j < FIT_KPT; ++j) tau[j][t] = 0.0;
        }
    }
    double tmax = 0.0;
#pragma unroll
    for (int j = 0; j < FIT_KPT; ++j)
        if (tid + nt * j < K) tmax = fmax(tmax, tau[j][0]);
    tmax = block_max(tmax, red);
    const double thr = 1e-14 * tmax;
    const double binv[4] = {1.0 / (n - 1.0), 2.0 / ((n - 1.0) * (n - 2.0)),
                            6.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0)),
                            24.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0) * (n - 4.0))};
#pragma unroll
    for (int j = 0; j < FIT_KPT; ++j) {
        const int kap = tid + nt * j;
        if (kap >= K) continue;
        const double t0 = tau[j][0];
        if (!(t0 >= thr) || !(t0 > 0.0)) continue;
        const double w0 = exp(log(t0) + rp.log_pvac + rp.log_g_rho - kap * rp.log_rho);  // S_0[k]
        int slot = -1;
        for (int i = 0; i < nk; ++i)
            if (ks[i] == kap) slot = i;
        if (kap == 0) {
            atomicAdd(&pacc[0], w0);
            if (slot >= 0) p_k[slot * (n + 1)] = w0;
            continue;
        }
        const int s = min(kap, n), v0 = n - s;
        if (s == 1) {
            atomicAdd(&pacc[1], w0);
            if (slot >= 0) p_k[slot * (n + 1) + 1] = w0;
            continue;
        }
        const SectorFitT<ORDER >= 4 ? 4 : 3> f = fit_sector<ORDER >= 4 ? 4 : 3>(
            n, v0, min(jp, s - 1), t0, tau[j][1], tau[j][2], tau[j][3], ORDER >= 4 ? tau[j][NT - 1] : 0.0);
        if (f.bad) {
            atomicAdd(&s_fail, w0);
            continue;
        }
        if (f.jr == 0) {
            // no usable moment (m_1 <= 0): every detector the sector can reach fires
            atomicAdd(&pacc[s], w0);
            if (slot >= 0) p_k[slot * (n + 1) + s] = w0;
            continue;
        }
        // q(n') = exp(lq - c . phi(v)), v = n - n' (lq = minus the log-partition sum)
        for (int v = v0; v < n; ++v) {
            const double ph[4] = {v * binv[0], 0.5 * v * (v - 1.0) * binv[1],
                                  v * (v - 1.0) * (v - 2.0) / 6.0 * binv[2],
                                  v * (v - 1.0) * (v - 2.0) * (v - 3.0) / 24.0 * binv[3]};
            double z = f.lq;
#pragma unroll
            for (int t = 0; t < (ORDER >= 4 ? 4 : 3); ++t)
                if (t < f.jr) z -= f.c[t] * ph[t];
            const double pv = w0 * exp(z);
            atomicAdd(&pacc[n - v], pv);
            if (slot >= 0) p_k[slot * (n + 1) + n - v] = pv;
        }
    }
    __syncthreads();
    double tot = 0.0;
    for (int i = 0; i <= n; ++i) tot += pacc[i];
    for (int i = tid; i <= n; i += nt) p_n[i] = pacc[i];
    if (tid == 0) *status = s_fail > 1e-10 * tot ? GBS_PS_FIT_NOCONV : 0;
}

// ---------------------------------------------------------------------------
// k_retilt: the rows marked for a re-tilt get a contour whose tilted mean
// photon number is kbar (radius, size and log G_0(rho) from their spectrum),
// one thread per row.
// ---------------------------------------------------------------------------
__global__ void k_retilt(int P, const int *__restrict__ offsets, const double *__restrict__ alpha,
                         RowPlan *__restrict__ rows)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    RowPlan rp = rows[p];
    if (!(rp.flags & GBS_ROW_RETILT) || rp.status != 0) return;
    const int o = offsets[p], n = offsets[p + 1] - o;
    const int flags = rp.flags;
    const double logdet_q = -2.0 * rp.log_pvac - rp.logdet_a;
    const double dev = rp.rconv < 1e299 ? 1.0 / rp.rconv : 0.0;
    row_plan(rp, n, alpha + 2 * o, 1, logdet_q, rp.logdet_a, 1.0, dev, false, 0, false, rp.kbar);
    rp.flags = flags;
    rows[p] = rp;
}

template <int ORDER, bool BIG, class C, bool RERUN = false>
int launch_contour(gbs_ctx *ctx, gbs_plan *pl, int nmax)
{
    hipStream_t st = ctx->stream;
    const void *fn = (const void *)k_contour<ORDER, BIG, C, RERUN>;
    int lds_static = 0;
    if (int rc = func_static_lds(ctx, fn, &lds_static)) return rc;
    const int lds_cap = ctx->lds_per_block - lds_static;
    int lds_c;
    if (BIG) {
        // the largest row's M(w) in LDS if it fits, else only alpha (M in HBM);
        // order 2 keeps only d, rz and the diagonal blocks
        lds_c = cont_fixed() + 8 * 2 * nmax + cont_mbytes<C>(nmax);
        if (lds_c > lds_cap) lds_c = cont_fixed() + 8 * 2 * nmax;
        if (ORDER == 2) lds_c = cont_fixed() + 8 * 2 * nmax + 16 * (cont_tp(nmax) + 5 * nmax);
    } else {
        // the whole 160 KB when the largest row needs it, else enough for eight
        // contour points of the largest row (two workgroups may then share a CU)
        lds_c = cont_fixed() + cont_vbytes(nmax) + pl->gmax * cont_mbytes<C>(nmax);
        if (lds_c > lds_cap) lds_c = lds_cap;
        if (cont_fixed() + cont_vbytes(nmax) + cont_mbytes<C>(nmax) > lds_c)
            return set_err(ctx, GBS_E_INVAL, "row too large for the contour kernel's LDS");
    }
    int occ = 1;
    if (int rc = func_lds_limit(ctx, fn, lds_c)) return rc;
    if (int rc = func_occupancy(ctx, fn, CONT_THREADS, lds_c, &occ)) return rc;
    int grid = occ * ctx->num_cu;
    cplx *mscr = nullptr;
    long long mstride = 0;
    if (BIG) {
        mstride = cont_mbytes<C>(nmax) / 16;
        if (pl->d_mscr) {
            if (grid > pl->mscr_blocks) grid = pl->mscr_blocks;
            mscr = pl->d_mscr;
        }
    }
    const int *q_end = pl->d_counter + (BIG ? 4 : 0);
    int *q_head = pl->d_counter + (BIG ? 5 : 1);
    hipLaunchKernelGGL((k_contour<ORDER, BIG, C, RERUN>), dim3(grid), dim3(CONT_THREADS), lds_c, st, lds_c,
                       pl->qchunk, pl->gmax, pl->d_offsets, pl->d_voff, pl->d_alpha, pl->d_v, pl->d_rows, pl->d_items,
                       q_end, q_head, pl->d_cluster_items, pl->d_cluster_off,
                       pl->order >= 4 ? pl->d_cluster_off + 4 * (pl->max_n + 1) : nullptr, mscr, mstride,
                       pl->d_sw);
    return 0;
}

// Forward on a plan: row set-up, work items, the contour kernels (rows above
// 40 clicks and the others), the fits; then, on the device, a second pass for
// the rows the fit marked: escalated rows of the mixed tier (fp64 rerun) and
// rows whose contour is re-tilted (new radius, rerun) -- not on a frozen plan,
// whose radii stay as they are.  Order 4 runs in fp64 only (the plan
// enforces it).
template <int ORDER>
int launch_order(gbs_ctx *ctx, gbs_plan *pl, double *logp, int32_t *status)
{
    hipStream_t st = ctx->stream;
    const int P = pl->P, nbig = pl->nbig;
    const int nsmall_max = pl->max_n_small;
    int ts = timer_begin(ctx, TG_PREP);
    int rc = eig_rows(ctx, pl);
    if (rc) return rc;
    timer_end(ctx, ts);
    ts = timer_begin(ctx, TG_ITEMS);
    hipLaunchKernelGGL(k_build_items, dim3(1), dim3(1024), 0, st, P, nbig, pl->qchunk, pl->d_offsets,
                       pl->d_perm,
                       pl->d_rows, pl->d_items, pl->d_counter);
    timer_end(ctx, ts);
    ts = timer_begin(ctx, TG_CONTOUR);
    const bool mixed = pl->prec == GBS_PREC_MIXED;
    if constexpr (ORDER < 4) {
        if (mixed) {
            // cluster eliminations in fp32 (M(w) stored in fp32), sums in fp64
            if (nbig > 0 && (rc = launch_contour<ORDER, true, cplxf>(ctx, pl, pl->max_n))) return rc;
            if (nbig < P && (rc = launch_contour<ORDER, false, cplxf>(ctx, pl, nsmall_max))) return rc;
        }
    } else if (mixed) {
        return set_err(ctx, GBS_E_INVAL, "order 4 runs in fp64");
    }
    if (!mixed) {
        if (nbig > 0 && (rc = launch_contour<ORDER, true, cplx>(ctx, pl, pl->max_n))) return rc;
        if (nbig < P && (rc = launch_contour<ORDER, false, cplx>(ctx, pl, nsmall_max))) return rc;
    }
    timer_end(ctx, ts);
    size_t lds_f = sizeof(cplx) * (GBS_KMAX + GBS_KMAX / 2);
    if ((rc = func_lds_limit(ctx, (const void *)k_dft_fit<ORDER>, (int)lds_f))) return rc;
    const int retilt = !pl->frozen && !pl->whole;
    ts = timer_begin(ctx, TG_FIT);
    hipLaunchKernelGGL(k_dft_fit<ORDER>, dim3(P), dim3(FIT_THREADS), lds_f, st, pl->d_offsets,
                       pl->d_rows, pl->d_sw, logp, status, mixed ? ROUND_FP32 : ROUND_FP64,
                       mixed ? MIXED_BOUND : 0.0, retilt);
    timer_end(ctx, ts);
    if (mixed || retilt) {
        if ((rc = func_lds_limit(ctx, (const void *)k_dft_fit<ORDER, 1>, (int)lds_f))) return rc;
        ts = timer_begin(ctx, TG_PASS2);
        hipLaunchKernelGGL(k_retilt, dim3((P + 255) / 256), dim3(256), 0, st, P, pl->d_offsets, pl->d_alpha,
                           pl->d_rows);
        hipLaunchKernelGGL(k_build_items, dim3(1), dim3(1024), 0, st, P, nbig, pl->qchunk, pl->d_offsets,
                           pl->d_perm, pl->d_rows, pl->d_items, pl->d_counter, GBS_PS_ESCALATED | GBS_ROW_RETILT);
        if (nbig > 0 && (rc = launch_contour<ORDER, true, cplx, true>(ctx, pl, pl->max_n))) return rc;
        if (nbig < P && (rc = launch_contour<ORDER, false, cplx, true>(ctx, pl, nsmall_max))) return rc;
        hipLaunchKernelGGL((k_dft_fit<ORDER, 1>), dim3(P), dim3(FIT_THREADS), lds_f, st, pl->d_offsets,
                           pl->d_rows, pl->d_sw, logp, status, ROUND_FP64, 0.0, 0);
        timer_end(ctx, ts);
    }
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}

// The whole device's click distribution: the plan's single row is every mode.
template <int ORDER>
int dist_order(gbs_ctx *ctx, gbs_plan *pl, int nk, const int *ks, double *p_n, double *p_k, int32_t *status)
{
    hipStream_t st = ctx->stream;
    int rc = eig_rows(ctx, pl);
    if (rc) return rc;
    hipLaunchKernelGGL(k_build_items, dim3(1), dim3(1024), 0, st, pl->P, 0, pl->qchunk, pl->d_offsets, pl->d_perm,
                       pl->d_rows, pl->d_items, pl->d_counter);
    if ((rc = launch_contour<ORDER, false, cplx>(ctx, pl, pl->max_n_small))) return rc;
    size_t lds_f = sizeof(cplx) * (GBS_KMAX + GBS_KMAX / 2);
    if ((rc = func_lds_limit(ctx, (const void *)k_dist_fit<ORDER>, (int)lds_f))) return rc;
    hipLaunchKernelGGL(k_dist_fit<ORDER>, dim3(1), dim3(FIT_THREADS), lds_f, st, pl->d_offsets, pl->d_rows,
                       pl->d_sw, nk, ks, p_n, p_k, status);
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}

// The plain comparison kernel (plain.hip) in place of the contour kernels.

template <int ORDER>
int launch_plain(gbs_ctx *ctx, gbs_plan *pl, double *logp, int32_t *status)
{
    hipStream_t st = ctx->stream;
    int ts = timer_begin(ctx, TG_PREP);
    int rc = eig_rows(ctx, pl);
    if (rc) return rc;
    timer_end(ctx, ts);
    ts = timer_begin(ctx, TG_CONTOUR);
    if ((rc = plain_contour(ctx, pl))) return rc;
    timer_end(ctx, ts);
    size_t lds_f = sizeof(cplx) * (GBS_KMAX + GBS_KMAX / 2);
    if ((rc = func_lds_limit(ctx, (const void *)k_dft_fit<ORDER>, (int)lds_f))) return rc;
    ts = timer_begin(ctx, TG_FIT);
    hipLaunchKernelGGL(k_dft_fit<ORDER>, dim3(pl->P), dim3(FIT_THREADS), lds_f, st, pl->d_offsets,
                       pl->d_rows, pl->d_sw, logp, status, ROUND_FP64, 0.0, 0);
    timer_end(ctx, ts);
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}

}  // namespace

int approx_forward_plain(gbs_ctx *ctx, gbs_plan *pl, double *logp_dev, int32_t *status_dev)
{
    if (pl->P == 0) return 0;
    switch (pl->order) {
    case 1: return launch_plain<1>(ctx, pl, logp_dev, status_dev);
    case 2: return launch_plain<2>(ctx, pl, logp_dev, status_dev);
    case 3: return launch_plain<3>(ctx, pl, logp_dev, status_dev);
    case 4: return launch_plain<4>(ctx, pl, logp_dev, status_dev);
    default: return set_err(ctx, -1, "order must be 1, 2, 3 or 4");
    }
}

namespace {
__global__ void k_status_or(int P, int32_t *__restrict__ status, int bits)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) status[p] |= bits;
}
}  // namespace

int status_or(gbs_ctx *ctx, int P, int32_t *status_dev, int bits)
{
    if (P == 0 || !status_dev) return 0;
    hipLaunchKernelGGL(k_status_or, dim3((P + 255) / 256), dim3(256), 0, ctx->stream, P, status_dev, bits);
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}

namespace {
int forward_order(gbs_ctx *ctx, gbs_plan *pl, double *logp_dev, int32_t *status_dev)
{
    switch (pl->order) {
    case 1: return launch_order<1>(ctx, pl, logp_dev, status_dev);
    case 2: return launch_order<2>(ctx, pl, logp_dev, status_dev);
    case 3: return launch_order<3>(ctx, pl, logp_dev, status_dev);
    case 4: return launch_order<4>(ctx, pl, logp_dev, status_dev);
    default: return set_err(ctx, -1, "order must be 1, 2, 3 or 4");
    }
}
}  // namespace

// Order 4 has no fp32 cluster kernels: asked for the mixed tier, it runs in
// fp64 and every row reports GBS_PS_ESCALATED.
int approx_forward(gbs_ctx *ctx, gbs_plan *pl, double *logp_dev, int32_t *status_dev)
{
    if (pl->P == 0) return 0;
    const bool esc_all = pl->order == 4 && pl->prec == GBS_PREC_MIXED;
    if (esc_all) pl->prec = GBS_PREC_FP64;
    int rc = forward_order(ctx, pl, logp_dev, status_dev);
    if (esc_all) {
        pl->prec = GBS_PREC_MIXED;
        if (rc == 0) rc = status_or(ctx, pl->P, status_dev, GBS_PS_ESCALATED);
    }
    return rc;
}

int click_distribution_run(gbs_ctx *ctx, gbs_plan *pl, int nk, const int *ks_dev, double *pn_dev, double *pk_dev,
                           int32_t *status_dev)
{
    if (pl->P != 1 || pl->nbig > 0) return set_err(ctx, GBS_E_INVAL, "one row of at most 40 modes");
    switch (pl->order) {
    case 1: return dist_order<1>(ctx, pl, nk, ks_dev, pn_dev, pk_dev, status_dev);
    case 2: return dist_order<2>(ctx, pl, nk, ks_dev, pn_dev, pk_dev, status_dev);
    case 3: return dist_order<3>(ctx, pl, nk, ks_dev, pn_dev, pk_dev, status_dev);
    case 4: return dist_order<4>(ctx, pl, nk, ks_dev, pn_dev, pk_dev, status_dev);
    default: return set_err(ctx, GBS_E_INVAL, "order must be 1, 2, 3 or 4");
    }
}
