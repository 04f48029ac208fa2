"""Benchmark: click-pattern probabilities at 70 modes on one MI355X.

Workload (synthetic, seeded): 70 modes, 35 squeezed inputs r ~ U[1.0, 1.6],
eta = 0.4, a Haar-random 70x70 interferometer, 10^4 click patterns with 15-40
clicks, the order-3 estimate.  One step = one pass of the whole path over the
batch with every input already in HBM: model build from device arrays, per-row
set-up (A = (Q^{-1})_CC, eigen-decomposition, contour plan), the persistent
contour/cluster kernel, the sector DFT and fits, and the log-sum.

Prints one JSON line.  value = click-pattern probabilities per second; the
subset-determinant rate, the roofline of the dominant kernel (contour/cluster,
FP64 vector ALU), the exact path at 20 modes and the CPU oracle baseline ride
along in the same line.
"""
import argparse
import json
import os
import sys
import time
from math import comb

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "subset dets/s and click-pattern probs/s at 70 modes; fwd+grad; rel err vs FP64"
PEAK_FP64_VALU_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def contour_point_flops(n: int, order: int) -> float:
    """Algorithmic real flops per contour point of a row with n clicks: M(w) as
    the symmetric V diag(d) V^T (4 flops per entry per term), d_k and the log of
    G_0 (20 per quadrature), and the cluster determinants by 2x2-block
    elimination (26, 180, 262 flops for 1, 2, 3 modes)."""
    N = 2 * n
    f = 8.0 * n * n * (2 * n + 1) + 20.0 * N
    per = {1: 26.0, 2: 180.0, 3: 262.0}
    for t in range(1, order + 1):
        f += per[t] * comb(n, t)
    return f


def adjoint_point_flops(n: int, order: int) -> float:
    """Algorithmic real flops per contour point of the adjoint: M(w) again, the
    cluster determinants again with their inverses scattered into Z(w) (56, 280,
    620 flops for 1, 2, 3 modes), and V^T Z V (4 N^3 for Z V, 2 N^2 (N+1) for
    the upper triangle of V^T (Z V)), N = 2n."""
    N = 2 * n
    f = 8.0 * n * n * (2 * n + 1) + 20.0 * N + 4.0 * N ** 3 + 2.0 * N * N * (N + 1)
    per = {1: 56.0, 2: 280.0, 3: 620.0}
    for t in range(1, order + 1):
        f += per[t] * comb(n, t)
    return f


def _oracle_row(args):
    """One oracle evaluation in a worker process (BLAS pinned to one thread)."""
    Q, C, order = args
    from threadpoolctl import threadpool_limits
    from oracle import approx
    with threadpool_limits(limits=1):
        return approx.prob_approx(Q, list(C), order)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, gpu_logp, budget_s: float = 12.0):
    """The oracle as it stands on a bounded sample of rows spread over the
    click-count range: first on one core, then on all the host cores this
    process may use (a process pool, at most 16 workers, one row per task);
    rows/s of each, the host, and the GPU's error on the rows evaluated."""
    import concurrent.futures as cf
    from threadpoolctl import threadpool_limits
    from oracle import approx, model
    from workloads import csr_rows
    rows = csr_rows(wl.offsets, wl.modes)
    ns = np.diff(wl.offsets)
    order = np.argsort(ns, kind="stable")
    pick = [int(order[int(q * (len(order) - 1))]) for q in np.linspace(0.0, 1.0, 21)]
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    done, errs = [], []
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        for i in pick:
            ref = approx.prob_approx(Q, list(rows[i]), wl.order)
            done.append(i)
            errs.append(abs(gpu_logp[i] - ref))
            if time.perf_counter() - t0 > budget_s:
                break
    dt1 = time.perf_counter() - t0
    cores = min(16, len(os.sched_getaffinity(0)))
    # all cores: the same spread of rows, repeated to give every worker work
    tasks = [(Q, rows[i], wl.order) for i in pick] * max(1, (2 * cores + 20) // 21)
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(_oracle_row, tasks))
    dtn = time.perf_counter() - t0
    errs += [abs(gpu_logp[i] - res[k]) for k, i in enumerate(pick)]
    return ({"value": len(tasks) / dtn, "unit": "click-pattern probs/s", "cores": cores, "kind": "oracle",
             "single_core_value": len(done) / dt1, "cpu": _cpu_model(), "host_cpus": os.cpu_count(),
             "sample": f"{len(tasks)} rows of the same batch ({len(pick)} rows spread over 15-40 clicks, "
                       f"repeated), power-series sector weights, numpy fp64, BLAS pinned to 1 thread per "
                       f"worker, {cores} worker processes; {dtn:.1f} s (one core: {len(done)} rows in "
                       f"{dt1:.1f} s)"},
            {"rows": len(pick), "max_abs_dlogp": float(max(errs)),
             "max_rel_err_p": float(np.expm1(max(errs)))})


def exact_leg(ctx, steps: int = 3):
    """Exact path on the 20-mode batch (4096 rows, 6-14 clicks): device time of
    the subset kernel, terms/s and rows/s."""
    from workloads import make_workload
    wl = make_workload(2)
    ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    ctx.gbs_prob_exact(wl.offsets, wl.modes)           # warm-up
    ctx.gbs_timing()
    ctx.gbs_set_timing(True)
    for _ in range(steps):
        out = ctx.gbs_prob_exact(wl.offsets, wl.modes)
    t = ctx.gbs_timing()
    ctx.gbs_set_timing(False)
    ms = t["exact"][0] / max(1, t["exact"][1])
    ns = np.diff(wl.offsets).astype(np.float64)
    terms = float(np.sum(2.0 ** ns))
    return {"workload": "m20_exact", "rows": wl.P, "ms": ms,
            "probs_per_s": wl.P / (ms * 1e-3), "subset_dets_per_s": terms / (ms * 1e-3),
            "max_kappa": float(out["kappa"].max()), "status_nonzero": int(np.sum(out["status"] != 0))}


def big_leg(ctx, torch, cfg: int, name: str, mixed: bool = False):
    """One forward and one forward + adjoint pass (after a warm-up) on the 100-
    or 144-mode batch (rows up to 60 / 110 clicks: eigenvectors and M(w) in HBM);
    device timings per kernel group."""
    from workloads import make_workload
    wl = make_workload(cfg)
    dev = torch.device("cuda:0")
    ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    ure = torch.tensor(np.ascontiguousarray(wl.U.real), device=dev)
    uim = torch.tensor(np.ascontiguousarray(wl.U.imag), device=dev)
    r = torch.tensor(wl.r, device=dev)
    eta = torch.tensor(wl.eta, device=dev)
    logp = torch.empty(wl.P, dtype=torch.float64, device=dev)
    st = torch.empty(wl.P, dtype=torch.int32, device=dev)
    dl = torch.ones(wl.P, dtype=torch.float64, device=dev)
    gr = torch.empty(wl.M, dtype=torch.float64, device=dev)
    ge = torch.empty(wl.M, dtype=torch.float64, device=dev)
    plan = ctx.gbs_plan_create(wl.offsets, wl.modes, wl.order)
    out = {"workload": name, "modes": wl.M, "patterns": wl.P, "order": wl.order,
           "clicks": f"{int(np.diff(wl.offsets).min())}-{int(np.diff(wl.offsets).max())}"}
    for key, grad in (("forward", False), ("forward+adjoint", True)):
        def fn():
            ctx.gbs_set_model_dev(ure, uim, r, eta)
            if grad:
                ctx.gbs_grad_dev(plan, dl, logp, gr, ge, st)
            else:
                ctx.gbs_prob_approx_dev(plan, logp, st)
        fn()
        torch.cuda.synchronize()
        ctx.gbs_timing()
        ctx.gbs_set_timing(True)
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        tim = ctx.gbs_timing()
        ctx.gbs_set_timing(False)
        out[key] = {"ms": ms, "probs_per_s": wl.P / (ms * 1e-3),
                    "status_nonzero": int((st != 0).sum().item()),
                    "kernel_ms": {k: round(v[0], 3) for k, v in tim.items() if v[1]}}
    plan.close()
    if mixed:
        out["forward_mixed"] = mixed_leg(ctx, torch, wl, (ure, uim, r, eta), logp.cpu().numpy(),
                                         out["forward"]["ms"])
    return out


def mixed_leg(ctx, torch, wl, model_dev, fp64_logp, fp64_ms):
    """The forward with fp32 cluster eliminations (GBS_PREC_MIXED, rows whose
    estimated error exceeds 1e-6 rerun in fp64 on the device): model build +
    forward time after a warm-up, its speed-up over the fp64 forward, the share
    of escalated rows, |log p_mixed - log p_fp64| and the rows' error estimates."""
    import paper_2106_01445_amd as g
    dev = torch.device("cuda:0")
    pm = ctx.gbs_plan_create(wl.offsets, wl.modes, wl.order, prec=g.GBS_PREC_MIXED)
    lm = torch.empty(wl.P, dtype=torch.float64, device=dev)
    st = torch.empty(wl.P, dtype=torch.int32, device=dev)
    for rep in range(2):
        ctx.gbs_set_model_dev(*model_dev)
        if rep:
            torch.cuda.synchronize()
            ctx.gbs_timing()
            ctx.gbs_set_timing(True)
            t0 = time.perf_counter()
        ctx.gbs_prob_approx_dev(pm, lm, st)
        torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    tim = ctx.gbs_timing()
    ctx.gbs_set_timing(False)
    sv = st.cpu().numpy()
    esc = (sv & g.gbs.GBS_PS_ESCALATED) != 0
    err = pm.info()["err"]
    pm.close()
    d = np.abs(lm.cpu().numpy() - fp64_logp)
    return {"ms": ms, "probs_per_s": wl.P / (ms * 1e-3), "speedup_vs_fp64_forward": fp64_ms / ms,
            "escalated_rows": int(esc.sum()), "escalated_fraction": float(esc.mean()),
            "other_status_nonzero": int(np.sum((sv & ~g.gbs.GBS_PS_ESCALATED) != 0)),
            "kernel_ms": {k: round(v[0], 3) for k, v in tim.items() if v[1]},
            "abs_dlogp_vs_fp64": {"median": float(np.median(d)), "p99": float(np.quantile(d, 0.99)),
                                  "max": float(d.max()),
                                  "max_not_escalated": float(d[~esc].max()) if (~esc).any() else 0.0},
            "err_estimate_not_escalated": {"median": float(np.median(err[~esc])) if (~esc).any() else 0.0,
                                           "max": float(err[~esc].max()) if (~esc).any() else 0.0}}


def plain_leg(ctx, wl, tuned_logp, tuned_fwd_kernel_ms):
    """The same forward through the plain comparison kernel (one workgroup per
    row, contour points in sequence, own LDL^T per cluster): device time per
    kernel group, and the speed-up of the tuned forward over it."""
    ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    ctx.gbs_timing()
    ctx.gbs_set_timing(True)
    out = ctx.gbs_prob_approx_plain(wl.offsets, wl.modes, wl.order)
    tim = ctx.gbs_timing()
    ctx.gbs_set_timing(False)
    km = {k: round(v[0], 3) for k, v in tim.items() if v[1]}
    ms = sum(km.values())
    return {"kernel_ms": km, "ms": ms, "probs_per_s": wl.P / (ms * 1e-3),
            "speedup_of_tuned_forward": ms / tuned_fwd_kernel_ms,
            "max_abs_dlogp_vs_tuned": float(np.max(np.abs(out["logp"] - tuned_logp)))}


def order4_leg(ctx, torch):
    """The paper's fourth-order scheme (forward) on the same 70-mode batch:
    quadruple clusters and four-moment fits, launch choices tuned first; one
    timed pass (model build + forward) after a warm-up, device timings per
    kernel group, subset determinants per second, and the two rows with the
    fewest clicks against the oracle."""
    from workloads import make_workload, csr_rows
    from oracle import approx, model
    wl = make_workload(3)
    dev = torch.device("cuda:0")
    ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    ure = torch.tensor(np.ascontiguousarray(wl.U.real), device=dev)
    uim = torch.tensor(np.ascontiguousarray(wl.U.imag), device=dev)
    r = torch.tensor(wl.r, device=dev)
    eta = torch.tensor(wl.eta, device=dev)
    logp = torch.empty(wl.P, dtype=torch.float64, device=dev)
    st = torch.empty(wl.P, dtype=torch.int32, device=dev)
    plan = ctx.gbs_plan_create(wl.offsets, wl.modes, 4)
    prm = plan.tune(1)

    def fn():
        ctx.gbs_set_model_dev(ure, uim, r, eta)
        ctx.gbs_prob_approx_dev(plan, logp, st)
    fn()
    torch.cuda.synchronize()
    ctx.gbs_timing()
    ctx.gbs_set_timing(True)
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    tim = ctx.gbs_timing()
    ctx.gbs_set_timing(False)
    ns = np.diff(wl.offsets)
    npts = (plan.info()["K"] // 2 + 1).astype(np.float64)
    dets = float(sum(npts[i] * sum(comb(int(ns[i]), t) for t in range(1, 5)) for i in range(wl.P)))
    lp = logp.cpu().numpy()
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    rows = csr_rows(wl.offsets, wl.modes)
    idx = [int(i) for i in np.argsort(ns, kind="stable")[:2]]
    err = max(abs(lp[i] - approx.prob_approx(Q, list(rows[i]), 4)) for i in idx)
    plan.close()
    km = {k: round(v[0], 3) for k, v in tim.items() if v[1]}
    # the same scheme with its adjoint on 512 rows of the batch (forward + gradient)
    sub = wl.subset(range(512))
    ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    ctx.gbs_grad(sub.offsets, sub.modes, 4, np.ones(sub.P))
    t0 = time.perf_counter()
    gout = ctx.gbs_grad(sub.offsets, sub.modes, 4, np.ones(sub.P))
    ms_grad = (time.perf_counter() - t0) * 1e3
    # the paper's headline case: 50 clicks of a lossless 70-mode device (every
    # second input squeezed at r = 1.6), rows above 40 clicks
    from workloads import accuracy_workload
    hw = accuracy_workload(70, 1.6, 50, P=256)
    ctx.gbs_set_model(hw.U, hw.r, hw.eta)
    ctx.gbs_prob_approx(hw.offsets, hw.modes, 4)
    t0 = time.perf_counter()
    hout = ctx.gbs_prob_approx(hw.offsets, hw.modes, 4)
    ms_head = (time.perf_counter() - t0) * 1e3
    return {"workload": "m70_order4", "modes": wl.M, "patterns": wl.P, "order": 4,
            "forward_adjoint_512_rows": {"ms_host_call": ms_grad, "status_nonzero": int(np.sum(gout["status"] != 0))},
            "headline_lossless_50_clicks": {"patterns": hw.P, "ms_host_call": ms_head,
                                            "probs_per_s": hw.P / (ms_head * 1e-3),
                                            "status_nonzero": int(np.sum(hout["status"] != 0)),
                                            "median_log10_p_hat": float(np.median(hout["logp"]) / np.log(10))},
            "clicks": f"{int(ns.min())}-{int(ns.max())}", "pass": "model build + forward",
            "ms": ms, "probs_per_s": wl.P / (ms * 1e-3), "subset_dets_per_s": dets / (ms * 1e-3),
            "status_nonzero": int((st != 0).sum().item()), "kernel_ms": km,
            "tuned_params": {"seg_forward": int(prm[0]), "points_per_item": int(prm[2]),
                             "points_per_pass": int(prm[3])},
            "max_abs_dlogp_vs_oracle_2_rows": float(err)}


def mcmc_leg(ctx, torch, stream):
    """Metropolis-Hastings chains of click patterns (Discussion: the
    approximate probabilities as the target of a Markov chain Monte Carlo
    sampler): 4096 chains on the 70-mode device, started from the batch's
    first 4096 patterns (15-40 clicks, fixed per chain), target the order-3 and
    the order-4 estimate; one step = a swap proposal for every chain, its
    log p_hat on the device, acceptance (gbs_mcmc_step_dev), uniforms drawn
    on the library's stream; 4 steps timed after one."""
    from workloads import make_workload
    wl = make_workload(3, P=4096)
    ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    dev = torch.device("cuda:0")
    out = {"workload": "m70_mcmc", "chains": wl.P, "clicks": "15-40 (fixed per chain)"}
    gen = torch.Generator(device=dev)
    gen.manual_seed(2106)
    for order in (3, 4):
        plan = ctx.gbs_plan_create(wl.offsets, wl.modes, order)
        with torch.cuda.stream(stream):
            modes = torch.tensor(wl.modes, dtype=torch.int32, device=dev)
            lp = torch.empty(wl.P, dtype=torch.float64, device=dev)
            acc = torch.empty(wl.P, dtype=torch.int32, device=dev)
            tot = torch.zeros((), dtype=torch.int64, device=dev)
            u = torch.empty(3 * wl.P, dtype=torch.float64, device=dev)
        ctx.gbs_prob_approx_dev(plan, lp)
        steps = 4
        for s in range(steps + 1):
            if s == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                u.uniform_(0.0, 1.0, generator=gen)
            ctx.gbs_mcmc_step_dev(plan, u, modes, lp, acc)
            if s >= 1:
                with torch.cuda.stream(stream):
                    tot += acc.sum()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        out[f"order{order}"] = {"ms_per_step": ms, "chain_steps_per_s": wl.P / (ms * 1e-3),
                                "acceptance": float(tot.item()) / (steps * wl.P),
                                "finite_logp": bool(torch.isfinite(lp).all().item())}
        plan.close()
    out["two_stage_m20"] = two_stage_leg(ctx, torch, stream)
    return out


def two_stage_leg(ctx, torch, stream):
    """Two-stage chains (gbs_mcmc_da_step_dev: the order-3 estimate screens
    each swap proposal, the exact probability corrects the survivors, target
    the exact p): 4096 chains on the 20-mode device, started from its batch's
    first 4096 patterns (6-14 clicks); 4 steps timed after one; the shares of
    proposals rejected by the estimate and by the exact correction."""
    from workloads import make_workload
    wl = make_workload(2)
    ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(2107)
    plan = ctx.gbs_plan_create(wl.offsets, wl.modes, 3)
    nmax = int(np.diff(wl.offsets).max())
    with torch.cuda.stream(stream):
        off = torch.tensor(wl.offsets, dtype=torch.int32, device=dev)
        modes = torch.tensor(wl.modes, dtype=torch.int32, device=dev)
        lh = torch.empty(wl.P, dtype=torch.float64, device=dev)
        le = torch.empty(wl.P, dtype=torch.float64, device=dev)
        pe = torch.empty(wl.P, dtype=torch.float64, device=dev)
        st = torch.empty(wl.P, dtype=torch.int32, device=dev)
        acc = torch.empty(wl.P, dtype=torch.int32, device=dev)
        cnt = torch.zeros(3, dtype=torch.int64, device=dev)
        u = torch.empty(4 * wl.P, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    ctx.gbs_prob_approx_dev(plan, lh)
    ctx.gbs_prob_exact_dev(off, modes, nmax, pe, le, None, st)
    steps = 4
    for s in range(steps + 1):
        if s == 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            u.uniform_(0.0, 1.0, generator=gen)
        ctx.gbs_mcmc_da_step_dev(plan, u, modes, lh, le, acc)
        if s >= 1:
            with torch.cuda.stream(stream):
                for c in range(3):
                    cnt[c] += (acc == c).sum()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    c = cnt.cpu().numpy() / (steps * wl.P)
    plan.close()
    return {"chains": wl.P, "clicks": "6-14 (fixed per chain)", "screen_order": 3, "ms_per_step": ms,
            "chain_steps_per_s": wl.P / (ms * 1e-3), "moved": float(c[1]),
            "rejected_by_estimate": float(c[0]), "rejected_by_exact": float(c[2]),
            "finite": bool((torch.isfinite(lh).all() & torch.isfinite(le).all()).item())}


def accuracy_leg(ctx):
    """The accuracy study of the paper's Numerical accuracy paragraph (Fig. 4)
    on synthetic Haar interferometers: the relative deviation
    Delta_p = |p_hat - p| / p of the order-2, -3 and -4 estimates from the exact
    (double-double) probability, mean and standard deviation over 100 random
    outcomes per point: against the number of modes (r = 1.6, 18 clicks,
    m = 26, 36, 54) and against the squeezing (30 modes, 20 clicks)."""
    from workloads import accuracy_workload
    pts = [(m, 1.6, 18) for m in (26, 36, 54)] + [(30, r, 20) for r in (0.8, 1.2, 1.6, 2.0)]
    res = []
    t0 = time.perf_counter()
    for m, r, n in pts:
        wl = accuracy_workload(m, r, n)
        ctx.gbs_set_model(wl.U, wl.r, wl.eta)
        ex = ctx.gbs_prob_exact(wl.offsets, wl.modes)
        rec = {"modes": m, "r": r, "clicks": n, "outcomes": wl.P,
               "exact_status_nonzero": int(np.sum(ex["status"] != 0))}
        for order in (2, 3, 4):
            ap = ctx.gbs_prob_approx(wl.offsets, wl.modes, order)
            d = np.abs(np.expm1(ap["logp"] - ex["logp"]))
            rec[f"order{order}"] = {"mean_delta_p": float(d.mean()), "std_delta_p": float(d.std())}
        res.append(rec)
    # Fig. 3b: the 30-mode device of Fig. 2 (15 inputs at r = 1.4, lossless)
    # with every detector clicked; exact p by 2^30 double-double terms
    from workloads import csr_from_lists, device30_model
    U, r, eta = device30_model()
    ctx.gbs_set_model(U, r, eta)
    off, mod = csr_from_lists([list(range(30))])
    t1 = time.perf_counter()
    ex = ctx.gbs_prob_exact(off, mod)
    fig = {"modes": 30, "r": 1.4, "clicks": 30, "exact_p": float(ex["p"][0]), "exact_status": int(ex["status"][0]),
           "kappa": float(ex["kappa"][0]), "exact_s": time.perf_counter() - t1}
    for order in (2, 3, 4):
        ap = ctx.gbs_prob_approx(off, mod, order)
        fig[f"order{order}"] = {"p_hat": float(np.exp(ap["logp"][0])), "status": int(ap["status"][0]),
                                "delta_p": float(abs(np.expm1(ap["logp"][0] - ex["logp"][0])))}
    return {"points": res, "fig3b_all_clicked": fig, "s": time.perf_counter() - t0}


def distribution_leg(ctx):
    """The whole device's click distribution p(n) and the sector curves p_k(n)
    of the paper's Fig. 2 device (30 modes, 15 inputs at r = 1.4, Haar U,
    lossless) at orders 2-4: wall time per call, sum p, mean clicks against the
    exact mean, the most likely n, p(30), and for k = 20, 50, 80, 110, 140, 170
    the peak position and weight of p_k(n)."""
    from workloads import device30_model
    from oracle import model
    U, r, eta = device30_model()
    ctx.gbs_set_model(U, r, eta)
    Q = model.q_matrix(model.covariance(U, r, eta))
    mean = sum(1.0 - model.vacuum_prob(Q, [l]) for l in range(30))
    ks = (20, 50, 80, 110, 140, 170)
    out = {"workload": "device30_r1.4", "modes": 30, "squeezed_inputs": 15, "r": 1.4, "eta": 1.0,
           "exact_mean_clicks": mean}
    for order in (2, 3, 4):
        ctx.gbs_click_distribution(order, ks)
        t0 = time.perf_counter()
        d = ctx.gbs_click_distribution(order, ks)
        ms = (time.perf_counter() - t0) * 1e3
        p = d["p_n"]
        out[f"order{order}"] = {
            "ms": ms, "status": d["status"], "sum_p": float(p.sum()),
            "mean_clicks": float(np.arange(31) @ p), "argmax_n": int(np.argmax(p)),
            "p_30": float(p[30]),
            "sectors": {str(k): {"argmax_n": int(np.argmax(d["p_k"][i])), "weight": float(d["p_k"][i].sum())}
                        for i, k in enumerate(ks)}}
    return out


def source_sha(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def load_counters(srcs, kernel: str):
    """Counter figures per launch of `kernel` from the committed summary
    (profiles/counters_m70_order3.json: HBM bytes from FETCH_SIZE/WRITE_SIZE,
    executed fp64 VALU and MFMA flops from SQ_INSTS_VALU_FLOPS_FP64 and
    SQ_INSTS_VALU_MFMA_MOPS_F64, each calibrated on a kernel of known count), if
    they were taken on the current kernel sources (hash match); else None."""
    path = os.path.join(ROOT, "profiles", "counters_m70_order3.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha") != source_sha(srcs):
        return None
    return rec.get("kernels", {}).get(kernel)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-exact", action="store_true", help="skip the 20-mode exact leg")
    ap.add_argument("--no-big", action="store_true", help="skip the 100- and 144-mode legs")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain comparison kernel")
    ap.add_argument("--no-order4", action="store_true", help="skip the fourth-order leg")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the accuracy-study leg")
    ap.add_argument("--no-mcmc", action="store_true", help="skip the Metropolis-Hastings leg")
    ap.add_argument("--no-dist", action="store_true", help="skip the click-distribution leg")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch choices")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 3 times (calibrates the "
                         "HBM byte counters against a kernel of known traffic)")
    ap.add_argument("--flop-probe", action="store_true",
                    help="only run kernels of known fp64 operation counts (an elementwise product "
                         "of 2^27 doubles, 3 times; a 4096^3 fp64 matrix product, 3 times): "
                         "calibrates the fp64 instruction counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: there is no multi-GPU path "
              "(rows are independent: a batch would shard over GPUs by cost, with one all-reduce of the 2M gradient entries)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 8, "copy_probe_bytes_written": b.numel() * 8,
                          "dispatches": 3}), flush=True)
        return
    if args.flop_probe:
        a = torch.rand(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.rand_like(a)
        c = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, b, out=c)
        x = torch.rand(4096, 4096, dtype=torch.float64, device="cuda:0")
        y = torch.rand_like(x)
        for _ in range(3):
            z = x @ y
        torch.cuda.synchronize()
        print(json.dumps({"elementwise_mul_f64_per_dispatch": a.numel(),
                          "matmul_f64_flops_per_dispatch": 2 * 4096 ** 3, "dispatches": 3,
                          "check": float(z[0, 0])}), flush=True)
        return
    import paper_2106_01445_amd as g
    from workloads import make_workload

    wl = make_workload(3)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)          # default priority
    ctx = g.Context(0, stream=stream.cuda_stream)
    ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    ure = torch.tensor(np.ascontiguousarray(wl.U.real), dtype=torch.float64, device=dev)
    uim = torch.tensor(np.ascontiguousarray(wl.U.imag), dtype=torch.float64, device=dev)
    r = torch.tensor(wl.r, dtype=torch.float64, device=dev)
    eta = torch.tensor(wl.eta, dtype=torch.float64, device=dev)
    logp = torch.empty(wl.P, dtype=torch.float64, device=dev)
    status = torch.empty(wl.P, dtype=torch.int32, device=dev)
    plan = ctx.gbs_plan_create(wl.offsets, wl.modes, wl.order)

    dl = torch.ones(wl.P, dtype=torch.float64, device=dev)       # d/dtheta of sum_p log p_hat
    gr = torch.empty(wl.M, dtype=torch.float64, device=dev)
    ge = torch.empty(wl.M, dtype=torch.float64, device=dev)

    def fwd():
        ctx.gbs_set_model_dev(ure, uim, r, eta)
        ctx.gbs_prob_approx_dev(plan, logp, status)

    def fwd_grad():
        ctx.gbs_set_model_dev(ure, uim, r, eta)
        ctx.gbs_grad_dev(plan, dl, logp, gr, ge, status)

    def timed(fn, steps):
        ctx.gbs_timing()
        ctx.gbs_set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tim = ctx.gbs_timing()
        ctx.gbs_set_timing(False)
        return (t1 - t0) * 1e3 / steps, tim

    for _ in range(args.warmup):
        fwd_grad()
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    if np.any(st & g.gbs.GBS_PS_FAILED):
        raise RuntimeError(f"{int(np.sum((st & g.gbs.GBS_PS_FAILED) != 0))} rows without a result")
    if not np.all(np.isfinite(gr.cpu().numpy())) or not np.all(np.isfinite(ge.cpu().numpy())):
        raise RuntimeError("non-finite gradient")
    info = plan.info()
    tuning = None
    if not args.no_tune:
        # default launch choices first, then the autotuner's
        ms_fwd0, _ = timed(fwd, args.steps)
        ms_step0, _ = timed(fwd_grad, args.steps)
        t0 = time.perf_counter()
        prm = plan.tune(3)
        t_tune = time.perf_counter() - t0
        fwd_grad()
        torch.cuda.synchronize()
        tuning = {"params": {"seg_forward": int(prm[0]), "seg_adjoint": int(prm[1]),
                             "points_per_item": int(prm[2]), "points_per_pass": int(prm[3])},
                  "tune_s": t_tune, "default_ms_per_step": ms_step0, "default_forward_ms": ms_fwd0}
    ms_fwd, tim_fwd = timed(fwd, args.steps)
    ms_step, tim = timed(fwd_grad, args.steps)
    lp = logp.cpu().numpy()
    # the same step recorded once into a HIP graph on the library's stream and replayed
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        fwd_grad()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / args.steps
    graph_match = bool(np.array_equal(logp.cpu().numpy(), lp))
    # the same step with bitwise-reproducible gradients (gbs_set_deterministic):
    # its time, two calls compared bit for bit, and its distance from the
    # floating-point gradient in units of the largest component
    g_fp = torch.cat([gr, ge]).cpu().numpy()
    ctx.gbs_set_deterministic(True)
    try:
        ms_det, _ = timed(fwd_grad, args.steps)
        g_d1 = torch.cat([gr, ge]).cpu().numpy()
        fwd_grad()
        torch.cuda.synchronize()
        g_d2 = torch.cat([gr, ge]).cpu().numpy()
    finally:
        ctx.gbs_set_deterministic(False)
    deterministic = {"ms_per_step": ms_det, "vs_default_step": ms_det / ms_step,
                     "bitwise_repeat": bool(np.array_equal(g_d1, g_d2)),
                     "max_dev_vs_floating_point": float(np.max(np.abs(g_d1 - g_fp)) / np.max(np.abs(g_fp)))}

    ns = np.diff(wl.offsets)
    npts = (info["K"] // 2 + 1).astype(np.float64)
    dets = float(sum(npts[i] * sum(comb(int(ns[i]), t) for t in range(1, wl.order + 1))
                     for i in range(wl.P)))
    fl_fwd = float(sum(npts[i] * contour_point_flops(int(ns[i]), wl.order) for i in range(wl.P)))
    fl_adj = float(sum(npts[i] * adjoint_point_flops(int(ns[i]), wl.order) for i in range(wl.P)))
    per = {k: v[0] / max(1, v[1]) for k, v in tim.items() if v[1]}
    rates = {}
    for key, fl, kname in (("contour_clusters", fl_fwd, "k_contour (forward contour points x clusters)"),
                           ("adjoint_contour_clusters", fl_adj, "k_adj_contour (adjoint contour points x clusters)")):
        ms = per.get(key, 0.0)
        if ms > 0:
            rates[key] = {"kernel": kname, "ms": ms, "flops": fl, "tflops": fl / (ms * 1e-3) / 1e12}
    dom = max(rates.values(), key=lambda d: d["ms"])
    src = [os.path.join(ROOT, "paper_2106_01445_amd", "csrc", f)
           for f in ("approx.hip", "grad.hip", "contour_common.h", "cplx.h", "internal.h")]
    cnt = load_counters(src, dom["kernel"].split()[0])
    roof = {"bound": "alu", "kernel": dom["kernel"],
            "achieved": round(dom["tflops"], 3), "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(dom["tflops"] / PEAK_FP64_VALU_TFLOPS, 4),
            "traffic": (cnt or {}).get("bytes_per_launch"),
            "kernel_ms": round(dom["ms"], 3), "flops_per_launch": dom["flops"],
            "all_kernels": {k: {"ms": round(v["ms"], 3), "tflops": round(v["tflops"], 3),
                                "frac": round(v["tflops"] / PEAK_FP64_VALU_TFLOPS, 4)}
                            for k, v in rates.items()}}
    roof["traffic_source"] = ("committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary "
                              "(profiles/counters_m70_order3.md), taken on these kernel sources"
                              if cnt and cnt.get("bytes_per_launch") is not None else
                              "none: the committed counter summary was taken on other kernel sources")
    if cnt and cnt.get("valu_fp64_flops") is not None:
        # executed fp64 work of the same launch, from the committed counters
        # (taken on these kernel sources), over this run's kernel time
        ex = cnt["valu_fp64_flops"] + cnt["mfma_fp64_flops"]
        roof["executed"] = {
            "valu_fp64_tflops": round(cnt["valu_fp64_flops"] / (dom["ms"] * 1e-3) / 1e12, 3),
            "mfma_fp64_tflops": round(cnt["mfma_fp64_flops"] / (dom["ms"] * 1e-3) / 1e12, 3),
            "executed_over_algorithmic": round(ex / dom["flops"], 3),
            "source": "profiles/counters_m70_order3.md"}
    out = {
        "metric": METRIC,
        "value": wl.P / (ms_step * 1e-3),
        "unit": "click-pattern probs/s (forward + gradient)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "m70_order3", "modes": 70, "squeezed_inputs": 35,
                   "r": "U[1.0,1.6]", "eta": 0.4, "patterns": wl.P, "clicks": "15-40",
                   "order": wl.order, "pass": "model build + forward + adjoint (d sum log p / d r, eta)"},
        "forward": {"ms_per_step": ms_fwd, "probs_per_s": wl.P / (ms_fwd * 1e-3),
                    "subset_dets_per_s": dets / (ms_fwd * 1e-3),
                    "kernel_ms": {k: round(v[0] / max(1, v[1]), 3) for k, v in tim_fwd.items() if v[1]}},
        "autotune": tuning,
        "graph": {"ms_per_step": ms_graph, "probs_per_s": wl.P / (ms_graph * 1e-3),
                  "logp_identical_to_eager": graph_match},
        "deterministic_gradients": deterministic,
        "subset_dets_per_step": dets,
        "subset_dets_per_s_fwd_grad": dets / (ms_step * 1e-3),
        "kernel_ms_per_step": {k: round(v, 3) for k, v in per.items()},
        "contour_points_per_step": int(npts.sum()),
        "status_counts": {"contour_flag": int(np.sum((st & g.gbs.GBS_PS_CONTOUR) != 0)),
                          "failed": int(np.sum((st & g.gbs.GBS_PS_FAILED) != 0))},
        "err_estimate_log_p": {"median": float(np.median(info["err"])), "max": float(np.max(info["err"]))},
        "roofline": roof,
    }
    out["forward_mixed"] = mixed_leg(ctx, torch, wl, (ure, uim, r, eta), lp, ms_fwd)
    if not args.no_plain:
        fwd_kernel_ms = sum(v[0] / max(1, v[1]) for k, v in tim_fwd.items() if v[1] and k != "model")
        out["plain_forward"] = plain_leg(ctx, wl, lp, fwd_kernel_ms)
    if not args.no_order4:
        out["m70_order4"] = order4_leg(ctx, torch)
    if not args.no_mcmc:
        out["mcmc"] = mcmc_leg(ctx, torch, stream)
    if not args.no_accuracy:
        out["accuracy_study"] = accuracy_leg(ctx)
    if not args.no_dist:
        out["click_distribution"] = distribution_leg(ctx)
    if not args.no_exact:
        out["exact_m20"] = exact_leg(ctx)
    if not args.no_big:
        out["m100_order3"] = big_leg(ctx, torch, 4, "m100_order3", mixed=True)
        out["m144_order2_grad"] = big_leg(ctx, torch, 5, "m144_order2_grad")
    if not args.no_cpu:
        cb, err = cpu_baseline(wl, lp)
        out["cpu_baseline"] = cb
        out["rel_err_vs_fp64_oracle"] = err
    print(json.dumps(out), flush=True)
    plan.close()
    ctx.close()


if __name__ == "__main__":
    main()
