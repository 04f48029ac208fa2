"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself: a
closed form, an invariant, a brute force on a tiny input, or a higher-precision
evaluation.  Citations are to the paper (Popova & Rubtsov) by section.
"""
import itertools
from math import comb, factorial

import mpmath as mp
import numpy as np
import pytest

from oracle import approx, exact, exact128, fit, fock, grad, model, sectors
from workloads import SEED_ROOT, csr_from_lists, haar_unitary, small_model


def single_mode(r, eta):
    U = np.eye(1, dtype=complex)
    return model.q_matrix(model.covariance(U, np.array([r]), np.array([eta])))


# ---------------------------------------------------------------- P1 single mode
@pytest.mark.parametrize("r", [0.3, 1.0, 1.6])
@pytest.mark.parametrize("eta", [1.0, 0.55, 0.2])
def test_single_mode_vacuum_closed_form(r, eta):
    """Methods, Model: the single-mode series has norm (1-4|x|^2)^{-1/2} with
    x = tanh(r)/2, so P_vac = 1/cosh r; with loss eta the vacuum probability is
    (1 + eta(2-eta) sinh^2 r)^{-1/2}."""
    Q = single_mode(r, eta)
    pv = model.vacuum_prob(Q, [0])
    assert pv == pytest.approx((1 + eta * (2 - eta) * np.sinh(r) ** 2) ** -0.5, rel=1e-14)
    if eta == 1.0:
        assert pv == pytest.approx(1 / np.cosh(r), rel=1e-14)


@pytest.mark.parametrize("r,eta", [(0.8, 1.0), (1.2, 0.6)])
def test_single_mode_photon_distribution(r, eta):
    """Methods, Model: |x> = sum_l (-x)^l sqrt((2l)!)/l! |2l>, normalised, gives
    P(2l) = C(2l, l) (tanh r / 2)^{2l} / cosh r; loss thins it binomially.  The
    sector series of the oracle (no clusters, clicked set = the mode) must give
    the same distribution."""
    L = 60
    Lsrc = 600          # the lossless tail above L still thins down below L
    lossless = np.zeros(Lsrc)
    for l in range(Lsrc // 2):
        lossless[2 * l] = float(mp.binomial(2 * l, l) * (mp.tanh(r) / 2) ** (2 * l) / mp.cosh(r))
    thinned = np.zeros(L)
    for k in range(Lsrc):
        for m in range(min(k, L - 1) + 1):
            thinned[m] += lossless[k] * float(mp.binomial(k, m)) * eta ** m * (1 - eta) ** (k - m)
    Q = single_mode(r, eta)
    W = exact.conditional_W(Q, [0])
    g = sectors.cluster_sector_weights(W, [()], L)[0]
    assert np.allclose(g[:40], thinned[:40], rtol=1e-12, atol=1e-16)


def test_single_mode_series_norm_factor4():
    """Methods, Model and Partition function: Z_X for a 1x1 X must equal the
    series sum_l |x|^{2l}(2l)!/(l!)^2 -- this fixes the factor 4 that the printed
    matrix formula omits."""
    x = 0.3
    series = float(mp.nsum(lambda l: x ** (2 * l) * mp.factorial(2 * l) / mp.factorial(l) ** 2,
                           [0, mp.inf]))
    assert model.partition_function(np.array([[x]])) == pytest.approx(series, rel=1e-13)


# ---------------------------------------------------------------- P2, P3, P4
def test_probabilities_sum_to_one():
    """Click patterns partition the outcomes: sum over all 2^M patterns is 1."""
    U, r, eta = small_model(5, 1)
    Q = model.q_matrix(model.covariance(U, r, eta))
    probs = exact.all_pattern_probs(Q)
    assert sum(probs.values()) == pytest.approx(1.0, abs=1e-13)
    assert min(probs.values()) > 0


def test_eta_zero_gives_no_clicks():
    U, r, _ = small_model(4, 2)
    Q = model.q_matrix(model.covariance(U, r, np.zeros(4)))
    probs = exact.all_pattern_probs(Q)
    assert probs[()] == pytest.approx(1.0, abs=1e-14)
    assert max(abs(v) for k, v in probs.items() if k) < 1e-14


def test_product_state_closed_form_fp64_and_binary128():
    """U = I: the modes are independent, p(C) = prod_{C}(1 - P0_i) prod_{Cbar} P0_i
    with the single-mode closed form.  At n = 14 the signed sum cancels by ~3^14,
    so the binary128 oracle must hit the closed form to ~1e-20."""
    M = 20
    rng = np.random.default_rng([SEED_ROOT, 97, 0])
    r = rng.uniform(0.5, 1.5, M)
    eta = rng.uniform(0.3, 0.9, M)
    U = np.eye(M, dtype=complex)
    C = sorted(rng.choice(M, 14, replace=False).tolist())
    with mp.workdps(40):
        p0 = [1 / mp.sqrt(1 + mp.mpf(e) * (2 - mp.mpf(e)) * mp.sinh(mp.mpf(x)) ** 2)
              for x, e in zip(r, eta)]
        ref = mp.mpf(1)
        for i in range(M):
            ref *= (1 - p0[i]) if i in C else p0[i]
    off, mod = csr_from_lists([C])
    out = exact128.exact(M, U, r, eta, off, mod)
    with mp.workdps(40):
        got = mp.mpf(out["p_hi"][0]) + mp.mpf(out["p_lo"][0])
        rel = float(abs(got - ref) / ref)
    assert rel < 1e-20
    assert out["kappa"][0] > 1e5          # the sum does cancel
    Q = model.q_matrix(model.covariance(U, r, eta))
    pf, kap = exact.prob_exact_conditional(Q, C)
    assert pf == pytest.approx(float(ref), rel=kap * 1e-14)


# ---------------------------------------------------------------- P5 X form
def test_covariance_matches_paper_X_form():
    """Methods, Model / Partition function / Probability of any sample: at
    eta = 1 the vacuum probability of a set S equals Z_{X'}/Z_X with X' the
    submatrix of the paper's X on the other modes (eq. 3, second factor)."""
    M = 6
    U, r, _ = small_model(M, 3)
    Q = model.q_matrix(model.covariance(U, r, np.ones(M)))
    X = model.takagi_X(U, r)
    zx = model.partition_function(X)
    rng = np.random.default_rng(0)
    for _ in range(6):
        S = sorted(rng.choice(M, rng.integers(1, M), replace=False).tolist())
        rest = [m for m in range(M) if m not in S]
        ratio = model.partition_function(X[np.ix_(rest, rest)]) / zx
        assert model.vacuum_prob(Q, S) == pytest.approx(ratio, rel=1e-12)


# ---------------------------------------------------------------- P6 exact forms
def test_exact_forms_agree():
    U, r, eta = small_model(7, 4)
    Q = model.q_matrix(model.covariance(U, r, eta))
    rows = [[0, 2, 5], [1, 3, 4, 6], [0, 1, 2, 3, 4, 5, 6], [4]]
    off, mod = csr_from_lists(rows)
    q128 = exact128.exact(7, U, r, eta, off, mod)
    for i, C in enumerate(rows):
        d, kap = exact.prob_exact_direct(Q, C)
        c, _ = exact.prob_exact_conditional(Q, C)
        t, _ = exact.prob_exact_torontonian(Q, C)
        ref = q128["p_hi"][i] + q128["p_lo"][i]
        for v in (d, c, t):
            assert v == pytest.approx(ref, rel=max(kap, 10) * 1e-14)


def test_binary128_covariance_route_matches_model_route():
    """The covariance entry point (sigma given) must give the same binary128
    probabilities as the (U, r, eta) route to the rounding of sigma."""
    U, r, eta = small_model(6, 5)
    sig = model.covariance(U, r, eta)
    off, mod = csr_from_lists([[0, 3], [1, 2, 4, 5]])
    a = exact128.exact(6, U, r, eta, off, mod)
    b = exact128.exact(6, None, r, eta, off, mod, sigma=sig)
    assert np.allclose(a["p_hi"], b["p_hi"], rtol=1e-12)


# ---------------------------------------------------------------- P7 Fock
@pytest.fixture(scope="module")
def fock_case():
    U, r, eta = small_model(3, 6, r_range=(0.2, 0.5), eta_range=(0.5, 0.9))
    P, defect = fock.photon_distribution(U, r, eta, 40)
    Q = model.q_matrix(model.covariance(U, r, eta))
    return U, r, eta, P, defect, Q


def test_fock_truncation_small(fock_case):
    assert abs(fock_case[4]) < 1e-12


def test_fock_matches_exact_click_probabilities(fock_case):
    """Methods, Model: the Fock expansion of exp(-a+ X a+)|0> with output loss
    gives the same click probabilities as the covariance inclusion-exclusion."""
    _, _, _, P, _, Q = fock_case
    for k in range(4):
        for C in itertools.combinations(range(3), k):
            assert fock.click_prob(P, C) == pytest.approx(
                exact.prob_exact_direct(Q, C)[0], rel=1e-10, abs=1e-15)


def test_fock_matches_sector_weights(fock_case):
    """Methods, Partition function and Moments calculation: the sector weights
    of the sub-ensemble (photon-number distribution with the unclicked modes,
    and the cluster's modes, empty) from the power series equal the Fock sums."""
    _, _, _, P, _, Q = fock_case
    C = [0, 2]
    W = exact.conditional_W(Q, C)
    clusters = [(), (0,), (1,), (0, 1)]
    g = sectors.cluster_sector_weights(W, clusters, 25)
    for i, T in enumerate(clusters):
        assert np.allclose(g[i], fock.sector_weights(P, C, T, 25), rtol=1e-9, atol=1e-14)
    ac = sectors.sector_allclick_exact(W, 25)
    assert np.allclose(ac, fock.allclick_sectors(P, C, 25), rtol=1e-9, atol=1e-14)


# ---------------------------------------------------------------- P8, P9
def test_sector_sum_is_vacuum_probability_and_mp_agrees():
    """G_T(1) = sum_kappa g_T[kappa] = det(W_T)^{-1/2} (all photon numbers, T
    empty); the fp64 series agrees with a 40-digit evaluation."""
    U, r, eta = small_model(8, 7)
    Q = model.q_matrix(model.covariance(U, r, eta))
    C = [0, 2, 3, 6, 7]
    W = exact.conditional_W(Q, C)
    n = len(C)
    L = 400
    for T in [(), (1,), (0, 3), (1, 2, 4)]:
        g = sectors.cluster_sector_weights(W, [T], L)[0]
        it = np.array(list(T) + [a + n for a in T], dtype=int)
        ref = 1.0 if not T else 1 / np.sqrt(np.linalg.det(W[np.ix_(it, it)]))
        assert g.sum() == pytest.approx(ref, rel=1e-12)
        gm = sectors.cluster_sector_weights_mp(W, T, 30)
        assert np.allclose(g[:30], [float(x) for x in gm], rtol=1e-11, atol=1e-300)


def test_sector_resolved_inclusion_exclusion_sums_to_exact():
    """Results, Calculation of sectors: p = sum over photon-number sectors of the
    all-click sector probability (eq. 2 per sector, times the eq. 3 weight)."""
    U, r, eta = small_model(6, 8)
    Q = model.q_matrix(model.covariance(U, r, eta))
    C = [0, 1, 3, 5]
    W = exact.conditional_W(Q, C)
    Cbar = [m for m in range(6) if m not in C]
    tot = sectors.sector_allclick_exact(W, 600).sum() * model.vacuum_prob(Q, Cbar)
    assert tot == pytest.approx(exact.prob_exact_direct(Q, C)[0], rel=1e-10)


# ---------------------------------------------------------------- P10, P11, P13
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_order_n_minus_1_is_exact(n):
    """Results, Approximation scheme: with as many moments as free points of the
    click distribution (j = n-1 on n' = 1..n) the fitted curve is the true one,
    so the estimate equals the exact probability (n = 5: the fourth-order fit)."""
    U, r, eta = small_model(6, 9)
    Q = model.q_matrix(model.covariance(U, r, eta))
    C = list(range(0, 2 * n, 2))[:n] if n <= 3 else [0, 1, 3, 4] if n == 4 else [0, 1, 2, 4, 5]
    lp = approx.prob_approx(Q, C, order=max(1, n - 1))
    assert lp == pytest.approx(np.log(exact.prob_exact_direct(Q, C)[0]), abs=1e-10)


def test_fit_recovers_exp_polynomial():
    """Methods, Approximation method: if the sector distribution is itself the
    exponential of a degree-j polynomial, matching j moments recovers it."""
    n = 12
    v = np.arange(n)                       # v = n - n' empty modes
    c_true = np.array([2.0, -0.7, 0.4])
    phi = fit.basis(n, 3)                  # columns n' = 1..n  <->  v = n-1..0
    logits = -c_true @ phi
    q = np.exp(logits - logits.max())
    q /= q.sum()
    m = phi @ q
    lq, ok, _ = fit.maxent_last_point(m, n)
    assert ok
    assert lq == pytest.approx(np.log(q[-1]), abs=1e-12)   # n' = n is the last column


def test_fit_reproduces_moments():
    rng = np.random.default_rng(1)
    for n in (5, 9, 20):
        p = rng.dirichlet(np.ones(n))
        phi = fit.basis(n, 3)
        m = phi @ p
        lq, ok, _ = fit.maxent_last_point(m, n)
        assert ok and np.isfinite(lq)


def test_approximation_improves_with_order():
    """Results, Approximation scheme and Fig. 3: more moments reproduce the
    sector shape better (lossless, half the inputs squeezed, all detectors
    clicked).  Qualitative: orders 2 and 3 beat order 1; order n-1 is exact."""
    for seed in range(3):
        rng = np.random.default_rng([SEED_ROOT, 98, seed])
        M = 6
        U = haar_unitary(M, rng)
        r = np.zeros(M)
        r[: M // 2] = 1.4
        Q = model.q_matrix(model.covariance(U, r, np.ones(M)))
        C = list(range(M))
        le = np.log(exact.prob_exact_conditional(Q, C)[0])
        d = {j: abs(np.expm1(approx.prob_approx(Q, C, j) - le)) for j in (1, 2, 3, M - 1)}
        assert d[2] < d[1] and d[3] < d[1]
        assert d[M - 1] < 1e-10


# ---------------------------------------------------------------- P12
def test_mean_clicks_from_vacuum_probabilities():
    """Methods, Moments calculation: the mean number of clicks is
    sum_l (1 - Z_{X_l}/Z_X) = sum_l (1 - P_vac(l))."""
    U, r, eta = small_model(5, 10)
    Q = model.q_matrix(model.covariance(U, r, eta))
    probs = exact.all_pattern_probs(Q)
    mean = sum(len(C) * p for C, p in probs.items())
    assert mean == pytest.approx(sum(1 - model.vacuum_prob(Q, [l]) for l in range(5)), rel=1e-12)


# ---------------------------------------------------------------- P14 FD machinery
def test_central_fd_on_closed_form():
    """d/dr log P_vac of one lossy mode: -eta(2-eta) sinh r cosh r /
    (1 + eta(2-eta) sinh^2 r)."""
    eta = 0.6

    def f(x):
        return float(np.log(model.vacuum_prob(single_mode(x[0], eta), [0])))

    r0 = 1.1
    g = grad.central_fd(f, np.array([r0]), [0])[0]
    a = eta * (2 - eta)
    ref = -a * np.sinh(r0) * np.cosh(r0) / (1 + a * np.sinh(r0) ** 2)
    assert g == pytest.approx(ref, rel=1e-8)


def test_haar_unitary_is_unitary():
    U = haar_unitary(12, np.random.default_rng(3))
    assert np.allclose(U @ U.conj().T, np.eye(12), atol=1e-13)


# ---------------------------------------------------------------- whole-device p(n)
@pytest.mark.parametrize("M,order", [(4, 3), (5, 4)])
def test_click_distribution_order_m_minus_1_is_exact(M, order):
    """Results, Calculation of p(n) and of sectors p_k(n): with C = every mode,
    j = M-1 moments fix every sector's curve on its support, so the estimated
    p(n) equals the brute-force sum of exact pattern probabilities."""
    import itertools
    U, r, eta = small_model(M, 31)
    Q = model.q_matrix(model.covariance(U, r, eta))
    p, _, _ = approx.click_distribution(Q, order)
    pb = np.zeros(M + 1)
    for bits in itertools.product([0, 1], repeat=M):
        C = [i for i in range(M) if bits[i]]
        pb[len(C)] += exact.prob_exact_direct(Q, C)[0] if C else model.vacuum_prob(Q, list(range(M)))
    assert np.max(np.abs(p - pb)) < 1e-13


@pytest.mark.parametrize("order", [1, 2, 3])
def test_click_distribution_norm_and_mean(order):
    """Every order: the sectors' weights sum to 1 and each fit matches its first
    moment, so sum_n p(n) = 1 and sum_n n p(n) = sum_l (1 - P_vac(l)) (Methods,
    Moments calculation) hold exactly."""
    U, r, eta = small_model(8, 32)
    Q = model.q_matrix(model.covariance(U, r, eta))
    p, _, _ = approx.click_distribution(Q, order)
    assert p.sum() == pytest.approx(1.0, abs=1e-12)
    mean = sum(1.0 - model.vacuum_prob(Q, [l]) for l in range(8))
    assert float(np.arange(9) @ p) == pytest.approx(mean, abs=1e-10)


# ------------------------------------------------- P8 at scale (binary128 series)
def _sector_pin_cases():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sector_pins.json")
    return json.load(open(path))["cases"]


@pytest.mark.parametrize("case", _sector_pin_cases(), ids=lambda c: f"m{ {3: 70, 4: 100, 5: 144}[c['config']]}_row{c['row']}_n{c['n']}")
def test_sector_series_at_scale_matches_binary128(case):
    """Methods, Partition function and Moments calculation: the fp64 power
    series of the sector weights (sectors.cluster_sector_weights) against the
    same definition evaluated in binary128 (oracle/sectors128.c, written by
    tests/golden/make_sector_pins.py) on the rows of the 70-, 100- and 144-mode
    batches (the largest click counts, and capped-radius rows of the 144-mode
    batch), for the empty cluster and one cluster of each size up to the
    order, on every sector that carries at least 1e-8 of the estimate:
    relative 1e-12."""
    from oracle.exact import conditional_W
    from workloads import csr_rows, make_workload
    wl = make_workload(case["config"])
    C = list(csr_rows(wl.offsets, wl.modes)[case["row"]])
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    W = conditional_W(Q, C)
    W = 0.5 * (W + W.T)
    for cl in case["clusters"]:
        kap = np.array(cl["kappa"])
        ref = np.array(cl["g_hi"]) + np.array(cl["g_lo"])
        got = sectors.cluster_sector_weights(W, [tuple(cl["T"])], int(kap.max()) + 1)[0][kap]
        rel = np.abs(got / ref - 1)
        assert rel.max() < 1e-12, (cl["T"], rel.max(), int(kap[np.argmax(rel)]))


# ------------------------------------------------- P14: reference gradient
def _fd_loss(U, rows, order, w):
    def f(x):
        M = U.shape[0]
        Q = model.q_matrix(model.covariance(U, x[:M], x[M:]))
        return float(sum(wi * approx.prob_approx(Q, C, order) for wi, C in zip(w, rows)))
    return f


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_reference_gradient_matches_central_differences(order):
    """The torch autograd reference gradient (oracle/grad_ref.py) against
    central differences of the numpy oracle (h = 1e-5) on a 6-mode lossy model:
    relative 1e-7 of the largest component (FD truncation ~1e-10); its value
    equals the oracle's sum of log p_hat."""
    from oracle import grad_ref
    M = 6
    U, r, eta = small_model(M, 31, r_range=(0.6, 1.3), eta_range=(0.4, 0.9))
    rows = [[0, 2], [1, 3, 5], [0, 1, 4, 5], [1, 2, 3, 4, 5], []]
    w = np.array([0.7, 1.3, 0.9, 1.1, 0.5])
    val, gr, ge = grad_ref.loss_and_grad(U, r, eta, rows, order, w)
    f = _fd_loss(U, rows, order, w)
    x0 = np.concatenate([r, eta])
    assert val == pytest.approx(f(x0), abs=1e-12)
    fd = grad.central_fd(f, x0, range(2 * M), h=1e-5)
    g = np.concatenate([gr, ge])
    assert np.max(np.abs(g - fd)) < 1e-7 * np.max(np.abs(fd)), (g, fd)


def test_reference_gradient_product_state_closed_form():
    """U = I: p(C) = prod_C (1 - P0_i) prod_Cbar P0_i with P0_i =
    (1 + eta_i (2 - eta_i) sinh^2 r_i)^{-1/2} (Methods, Model, with loss); an
    order >= n - 1 estimate is exact, so d log p / d(r_i, eta_i) have closed
    forms."""
    from oracle import grad_ref
    M = 6
    rng = np.random.default_rng([SEED_ROOT, 96, 1])
    r = rng.uniform(0.5, 1.4, M)
    eta = rng.uniform(0.3, 0.9, M)
    C = [0, 2, 3]
    val, gr, ge = grad_ref.loss_and_grad(np.eye(M, dtype=complex), r, eta, [C], 2, [1.0])
    a = eta * (2 - eta)
    s2 = np.sinh(r) ** 2
    P0 = (1 + a * s2) ** -0.5
    dP0_dr = -0.5 * (1 + a * s2) ** -1.5 * a * 2 * np.sinh(r) * np.cosh(r)
    dP0_de = -0.5 * (1 + a * s2) ** -1.5 * (2 - 2 * eta) * s2
    click = np.isin(np.arange(M), C)
    dlog = np.where(click, -1.0 / (1 - P0), 1.0 / P0)
    assert val == pytest.approx(np.sum(np.log(np.where(click, 1 - P0, P0))), abs=1e-12)
    assert np.allclose(gr, dlog * dP0_dr, rtol=1e-9, atol=1e-12)
    assert np.allclose(ge, dlog * dP0_de, rtol=1e-9, atol=1e-12)


# ------------------------------------------------- Metropolis-Hastings chains (Discussion)
def test_mcmc_swap_proposal_is_symmetric():
    """Every swap neighbour of a pattern is drawn by exactly one cell of the
    (position, unclicked mode) grid of uniforms, and the reverse swap by exactly
    one cell from the neighbour: the proposal is symmetric, so the Metropolis
    ratio is the ratio of the targets."""
    import itertools
    from oracle import mcmc
    M, n = 6, 2
    grid = [((i + 0.5) / n, (k + 0.5) / (M - n)) for i in range(n) for k in range(M - n)]
    for row in itertools.combinations(range(M), n):
        props = [tuple(mcmc.propose(list(row), M, a, b)) for a, b in grid]
        assert len(set(props)) == n * (M - n)
        for prop in props:
            assert len(set(prop) ^ set(row)) == 2 and list(prop) == sorted(prop)
            back = [tuple(mcmc.propose(list(prop), M, a, b)) for a, b in grid]
            assert back.count(row) == 1


def test_mcmc_chain_converges_to_the_target():
    """One chain on the 15 two-click patterns of a 6-mode lossy model, target
    the exact p, 200000 steps: its visit frequencies match p restricted to two
    clicks, normalised (total variation < 0.02; the statistical spread is
    about 0.005)."""
    import itertools
    from oracle import mcmc
    M = 6
    U, r, eta = small_model(M, 41, r_range=(0.6, 1.3), eta_range=(0.4, 0.9))
    Q = model.q_matrix(model.covariance(U, r, eta))
    pats = [tuple(c) for c in itertools.combinations(range(M), 2)]
    lp = {c: float(np.log(exact.prob_exact_direct(Q, list(c))[0])) for c in pats}
    rng = np.random.default_rng([SEED_ROOT, 77])
    row, cur = [0, 1], lp[(0, 1)]
    seen = {c: 0 for c in pats}
    steps = 200000
    u = rng.random((steps, 3))
    for s in range(steps):
        rows, lps, _, _ = mcmc.mh_step([row], M, u[s], [cur], lambda c: lp[tuple(c)])
        row, cur = rows[0], lps[0]
        seen[tuple(row)] += 1
    p = np.array([np.exp(lp[c]) for c in pats])
    p /= p.sum()
    f = np.array([seen[c] for c in pats]) / steps
    assert 0.5 * np.abs(f - p).sum() < 0.02, 0.5 * np.abs(f - p).sum()


def test_mcmc_two_stage_acceptance_rules():
    """The two-stage step's decisions sit exactly at the delayed-acceptance
    thresholds (Christen & Fox 2005): for every swap between the 20
    three-click patterns of a 6-mode model, with the order-1 estimate as the
    screen and the exact p as the target, a uniform just below
    a1 = min(1, q(y)/q(x)) passes the first stage and one just above fails it,
    and likewise at a2 = min(1, p(y) q(x) / (p(x) q(y))) in the second.  The
    resulting kernel a1 a2 / (n (M - n)) satisfies detailed balance with p."""
    import itertools
    from oracle import mcmc
    M, n = 6, 3
    U, r, eta = small_model(M, 7)
    Q = model.q_matrix(model.covariance(U, r, eta))
    pats = [tuple(c) for c in itertools.combinations(range(M), n)]
    le = {c: float(np.log(exact.prob_exact_direct(Q, list(c))[0])) for c in pats}
    lh = {c: approx.prob_approx(Q, list(c), 1) for c in pats}
    grid = [((i + 0.5) / n, (k + 0.5) / (M - n)) for i in range(n) for k in range(M - n)]
    K = {}
    for x in pats:
        for a, b in grid:
            y = tuple(mcmc.propose(list(x), M, a, b))
            a1 = min(1.0, np.exp(lh[y] - lh[x]))
            a2 = min(1.0, np.exp((le[y] - le[x]) - (lh[y] - lh[x])))
            step = lambda u2, u3: mcmc.da_step([list(x)], M, [a, b, u2, u3], [lh[x]], [le[x]],
                                               lambda c: lh[tuple(c)], lambda c: le[tuple(c)])[3][0]
            assert step(a1 * (1 - 1e-9), a2 * (1 - 1e-9)) == 1
            if a1 < 1:
                assert step(a1 * (1 + 1e-9), 0.0) == 0
            if a2 < 1:
                assert step(a1 * (1 - 1e-9), a2 * (1 + 1e-9)) == 2
            K[(x, y)] = a1 * a2 / len(grid)
    for (x, y), kxy in K.items():
        lhs, rhs = np.exp(le[x]) * kxy, np.exp(le[y]) * K[(y, x)]
        assert abs(lhs - rhs) <= 1e-12 * max(lhs, rhs), (x, y, lhs, rhs)


def test_mcmc_two_stage_chain_converges_to_exact_p():
    """One two-stage chain on the 20 three-click patterns of a 6-mode model,
    screened by the order-1 estimate (whose normalised distribution is 0.03
    from p in total variation), 200000 steps: its visit frequencies match the
    exact p (total variation < 0.015), not the estimate's distribution."""
    import itertools
    from oracle import mcmc
    M, n = 6, 3
    U, r, eta = small_model(M, 7)
    Q = model.q_matrix(model.covariance(U, r, eta))
    pats = [tuple(c) for c in itertools.combinations(range(M), n)]
    le = {c: float(np.log(exact.prob_exact_direct(Q, list(c))[0])) for c in pats}
    lh = {c: approx.prob_approx(Q, list(c), 1) for c in pats}
    p = np.array([np.exp(le[c]) for c in pats]); p /= p.sum()
    q = np.array([np.exp(lh[c]) for c in pats]); q /= q.sum()
    assert 0.5 * np.abs(p - q).sum() > 0.03
    rng = np.random.default_rng([SEED_ROOT, 78])
    row = [0, 1, 2]
    h, e = lh[(0, 1, 2)], le[(0, 1, 2)]
    seen = {c: 0 for c in pats}
    steps = 200000
    u = rng.random((steps, 4))
    for s in range(steps):
        rows, hs, es, _, _ = mcmc.da_step([row], M, u[s], [h], [e], lambda c: lh[tuple(c)], lambda c: le[tuple(c)])
        row, h, e = rows[0], hs[0], es[0]
        seen[tuple(row)] += 1
    f = np.array([seen[c] for c in pats]) / steps
    assert 0.5 * np.abs(f - p).sum() < 0.015, 0.5 * np.abs(f - p).sum()
    assert 0.5 * np.abs(f - q).sum() > 0.02, 0.5 * np.abs(f - q).sum()
