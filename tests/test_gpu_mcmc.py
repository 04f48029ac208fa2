"""Metropolis-Hastings chains of click patterns on the GPU (Discussion: the
approximate probabilities as the target of a Markov chain Monte Carlo
sampler), through gbs_mcmc_step_dev, against the oracle's step
(oracle/mcmc.py) and against the exact stationary distribution."""
import itertools

import numpy as np
import pytest

from oracle import approx, exact, exact128, mcmc, model
from workloads import SEED_ROOT, csr_from_lists, csr_rows, make_workload, small_model

from paper_2106_01445_amd import gbs as g

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    import torch
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def test_mcmc_step_matches_oracle_step(gpu_ctx):
    """20 modes, order 3, 64 chains of 6-14 clicks: one step with drawn
    uniforms, then one step that accepts every proposal (u2 = 0).  The chains'
    new rows equal the oracle's wherever the acceptance decision is not
    within 1e-8 of its threshold (the two sides' log p_hat differ by ~1e-11),
    and after the all-accepting step every row is the oracle's proposal."""
    import torch
    wl = make_workload(2, P=64)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    rows = [list(r) for r in csr_rows(wl.offsets, wl.modes)]
    plan = gpu_ctx.gbs_plan_create(wl.offsets, wl.modes, 3)
    modes = _dev(wl.modes, torch.int32)
    lp = torch.empty(wl.P, dtype=torch.float64, device="cuda")
    gpu_ctx.gbs_prob_approx_dev(plan, lp)
    torch.cuda.synchronize()
    lp0 = lp.cpu().numpy()
    acc = torch.empty(wl.P, dtype=torch.int32, device="cuda")
    rng = np.random.default_rng([SEED_ROOT, 140])
    u = rng.random(3 * wl.P)
    gpu_ctx.gbs_mcmc_step_dev(plan, _dev(u, torch.float64), modes, lp, acc)
    torch.cuda.synchronize()
    got = [list(r) for r in csr_rows(wl.offsets, modes.cpu().numpy())]
    cache = {}

    def oracle_lp(c):
        if tuple(c) not in cache:
            cache[tuple(c)] = approx.prob_approx(Q, list(c), 3)
        return cache[tuple(c)]

    new, _, oacc, props = mcmc.mh_step(rows, wl.M, u, lp0, oracle_lp)
    a = acc.cpu().numpy()
    checked = 0
    for p in range(wl.P):
        d = oracle_lp(props[p]) - lp0[p]
        if d < 0 and abs(np.log(u[3 * p + 2]) - d) < 1e-8:
            continue
        checked += 1
        assert a[p] == oacc[p] and got[p] == new[p], (p, a[p], oacc[p], got[p], new[p])
    assert checked >= 60 and 0 < a.sum() < wl.P
    # every proposal accepted: the rows are the oracle's proposals from `got`
    u = rng.random(3 * wl.P)
    u[2::3] = 0.0
    lpn = lp.cpu().numpy()
    gpu_ctx.gbs_mcmc_step_dev(plan, _dev(u, torch.float64), modes, lp, acc)
    torch.cuda.synchronize()
    got2 = [list(r) for r in csr_rows(wl.offsets, modes.cpu().numpy())]
    assert np.all(acc.cpu().numpy() == 1)
    for p in range(wl.P):
        assert got2[p] == mcmc.propose(got[p], wl.M, u[3 * p], u[3 * p + 1])
    ref = np.array([oracle_lp(got2[p]) for p in range(0, wl.P, 8)])
    assert np.max(np.abs(lp.cpu().numpy()[::8] - ref)) < 1e-9
    assert np.all(np.isfinite(lpn))
    plan.close()


def test_mcmc_stationary_distribution(gpu_ctx):
    """8 lossy modes, 3 clicks, order 2 (= exact: j >= n - 1), 4096 chains from
    uniformly drawn patterns, 150 steps: over the last 100 steps the chains'
    visits to the 56 three-click patterns match the exact p restricted to three
    clicks, normalised (total variation < 0.02; statistical spread ~0.005)."""
    import torch
    M, n, B = 8, 3, 4096
    U, r, eta = small_model(M, 43, r_range=(0.6, 1.3), eta_range=(0.4, 0.9))
    gpu_ctx.gbs_set_model(U, r, eta)
    Q = model.q_matrix(model.covariance(U, r, eta))
    pats = [tuple(c) for c in itertools.combinations(range(M), n)]
    p = np.array([exact.prob_exact_direct(Q, list(c))[0] for c in pats])
    p /= p.sum()
    rng = np.random.default_rng([SEED_ROOT, 141])
    rows = [sorted(rng.choice(M, n, replace=False).tolist()) for _ in range(B)]
    off, mod = csr_from_lists(rows)
    plan = gpu_ctx.gbs_plan_create(off, mod, 2)
    modes = _dev(mod, torch.int32)
    lp = torch.empty(B, dtype=torch.float64, device="cuda")
    gpu_ctx.gbs_prob_approx_dev(plan, lp)
    index = {c: i for i, c in enumerate(pats)}
    counts = np.zeros(len(pats))
    u = torch.empty(3 * B, dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(141)
    torch.cuda.synchronize()
    for step in range(150):
        # (torch's stream draws the uniforms, the library's stream steps the
        # chains: synchronise between them)
        u.uniform_(0.0, 1.0, generator=gen)
        torch.cuda.synchronize()
        gpu_ctx.gbs_mcmc_step_dev(plan, u, modes, lp)
        torch.cuda.synchronize()
        if step >= 50:
            for row in modes.cpu().numpy().reshape(B, n):
                counts[index[tuple(row)]] += 1
    f = counts / counts.sum()
    tv = 0.5 * np.abs(f - p).sum()
    assert tv < 0.02, tv
    plan.close()


def test_mcmc_errors(gpu_ctx):
    """A frozen plan (its radii would not suit the new rows) and NULL arrays are
    refused."""
    import torch
    U, r, eta = small_model(8, 44)
    gpu_ctx.gbs_set_model(U, r, eta)
    off, mod = csr_from_lists([[0, 2, 5], [1, 3, 4]])
    plan = gpu_ctx.gbs_plan_create(off, mod, 2)
    modes = _dev(mod, torch.int32)
    lp = torch.empty(2, dtype=torch.float64, device="cuda")
    gpu_ctx.gbs_prob_approx_dev(plan, lp)
    u = torch.zeros(6, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(g.GBSError):
        gpu_ctx.gbs_mcmc_step_dev(plan, None, modes, lp)
    plan.freeze(True)
    with pytest.raises(g.GBSError) as e:
        gpu_ctx.gbs_mcmc_step_dev(plan, u, modes, lp)
    assert e.value.code == g.GBS_E_STATE
    plan.close()


def _init_values(gpu_ctx, plan, off, mod, nmax):
    """log p_hat and exact log p of the plan's rows, on the device."""
    import torch
    P = len(off) - 1
    lh = torch.empty(P, dtype=torch.float64, device="cuda")
    gpu_ctx.gbs_prob_approx_dev(plan, lh)
    pe = torch.empty(P, dtype=torch.float64, device="cuda")
    le = torch.empty(P, dtype=torch.float64, device="cuda")
    st = torch.empty(P, dtype=torch.int32, device="cuda")
    gpu_ctx.gbs_prob_exact_dev(_dev(off, torch.int32), _dev(mod, torch.int32), nmax, pe, le, None, st)
    torch.cuda.synchronize()
    assert int((st & g.GBS_PS_FAILED).sum()) == 0
    return lh, le


def test_two_stage_step_matches_oracle_step(gpu_ctx):
    """20 modes, 48 chains of 5-9 clicks, order-2 screen, exact target: one
    two-stage step with drawn uniforms.  Every chain's code (moved, rejected by
    the estimate, rejected by the exact correction) and new row equal the
    oracle's step (oracle/mcmc.py da_step with the oracle's estimate and its
    binary128 exact p) wherever neither decision is within 1e-8 of its
    threshold, and the moved chains' values equal the oracle's (1e-9 estimate,
    1e-10 exact)."""
    import torch
    M, P = 20, 48
    U, r, eta = small_model(M, 45, r_range=(0.5, 1.4), eta_range=(0.4, 0.9))
    gpu_ctx.gbs_set_model(U, r, eta)
    Q = model.q_matrix(model.covariance(U, r, eta))
    rng = np.random.default_rng([SEED_ROOT, 142])
    rows = [sorted(rng.choice(M, int(rng.integers(5, 10)), replace=False).tolist()) for _ in range(P)]
    off, mod = csr_from_lists(rows)
    plan = gpu_ctx.gbs_plan_create(off, mod, 2)
    lh, le = _init_values(gpu_ctx, plan, off, mod, 9)
    lh0, le0 = lh.cpu().numpy(), le.cpu().numpy()
    modes = _dev(mod, torch.int32)
    acc = torch.empty(P, dtype=torch.int32, device="cuda")
    u = rng.random(4 * P)
    gpu_ctx.gbs_mcmc_da_step_dev(plan, _dev(u, torch.float64), modes, lh, le, acc)
    torch.cuda.synchronize()
    got = [list(x) for x in csr_rows(off, modes.cpu().numpy())]
    codes = acc.cpu().numpy()
    hat = lambda c: approx.prob_approx(Q, list(c), 2)
    ex = lambda c: float(exact128.exact(M, U, r, eta, [0, len(c)], list(c))["logp"][0])
    new, nh, ne, ocodes, props = mcmc.da_step(rows, M, u, lh0, le0, hat, ex)
    checked = 0
    for p in range(P):
        dh = hat(props[p]) - lh0[p]
        if dh < 0 and abs(np.log(u[4 * p + 2]) - dh) < 1e-8:
            continue
        if ocodes[p] != 0:
            rr = (ex(props[p]) - le0[p]) - dh
            if rr < 0 and abs(np.log(u[4 * p + 3]) - rr) < 1e-8:
                continue
        checked += 1
        assert codes[p] == ocodes[p] and got[p] == new[p], (p, codes[p], ocodes[p], got[p], new[p])
        if codes[p] == 1:
            assert abs(lh.cpu().numpy()[p] - nh[p]) < 1e-9 and abs(le.cpu().numpy()[p] - ne[p]) < 1e-10
    assert checked >= 44 and {0, 1} <= set(codes.tolist())
    plan.close()


def test_two_stage_stationary_distribution_is_exact(gpu_ctx):
    """8 lossy modes, 3 clicks, screened by the order-1 estimate (whose
    normalised distribution is 0.05 from the exact p in total variation),
    4096 chains, 150 steps: over the last 100 steps the visits match the exact
    p restricted to three clicks (total variation < 0.02; spread ~0.005) and
    not the estimate's distribution (> 0.03 from it)."""
    import torch
    M, n, B = 8, 3, 4096
    U, r, eta = small_model(M, 43, r_range=(0.6, 1.3), eta_range=(0.4, 0.9))
    gpu_ctx.gbs_set_model(U, r, eta)
    Q = model.q_matrix(model.covariance(U, r, eta))
    pats = [tuple(c) for c in itertools.combinations(range(M), n)]
    p = np.array([exact.prob_exact_direct(Q, list(c))[0] for c in pats]); p /= p.sum()
    q = np.array([np.exp(approx.prob_approx(Q, list(c), 1)) for c in pats]); q /= q.sum()
    rng = np.random.default_rng([SEED_ROOT, 143])
    rows = [sorted(rng.choice(M, n, replace=False).tolist()) for _ in range(B)]
    off, mod = csr_from_lists(rows)
    plan = gpu_ctx.gbs_plan_create(off, mod, 1)
    lh, le = _init_values(gpu_ctx, plan, off, mod, n)
    modes = _dev(mod, torch.int32)
    index = {c: i for i, c in enumerate(pats)}
    counts = np.zeros(len(pats))
    u = torch.empty(4 * B, dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(143)
    for step in range(150):
        u.uniform_(0.0, 1.0, generator=gen)
        torch.cuda.synchronize()
        gpu_ctx.gbs_mcmc_da_step_dev(plan, u, modes, lh, le)
        torch.cuda.synchronize()
        if step >= 50:
            for row in modes.cpu().numpy().reshape(B, n):
                counts[index[tuple(row)]] += 1
    f = counts / counts.sum()
    assert 0.5 * np.abs(f - p).sum() < 0.02, 0.5 * np.abs(f - p).sum()
    assert 0.5 * np.abs(f - q).sum() > 0.03, 0.5 * np.abs(f - q).sum()
    plan.close()


def test_two_stage_errors(gpu_ctx):
    """Rows above 30 clicks (beyond the exact path) and NULL arrays are refused
    before anything runs."""
    import torch
    M = 40
    U, r, eta = small_model(M, 46)
    gpu_ctx.gbs_set_model(U, r, eta)
    off, mod = csr_from_lists([list(range(31)), [0, 5, 9]])
    plan = gpu_ctx.gbs_plan_create(off, mod, 2)
    modes = _dev(mod, torch.int32)
    v = torch.zeros(2, dtype=torch.float64, device="cuda")
    u = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(g.GBSError) as e:
        gpu_ctx.gbs_mcmc_da_step_dev(plan, u, modes, v, v.clone())
    assert e.value.code == g.GBS_E_INVAL
    plan.close()
    off, mod = csr_from_lists([[0, 5, 9], [1, 2, 3]])
    plan = gpu_ctx.gbs_plan_create(off, mod, 2)
    with pytest.raises(g.GBSError):
        gpu_ctx.gbs_mcmc_da_step_dev(plan, u, _dev(mod, torch.int32), None, v.clone())
    plan.close()
