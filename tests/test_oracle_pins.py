"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses a closed form,
a brute-force search, an exact rational LP solve, an independent library
(HiGHS), or an invariant of the iteration.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import lp, pqr


# ----------------------------------------------------------------------------
# prox maps (eqs. beta_update, z_update) against brute-force 1-D minimisation
# ----------------------------------------------------------------------------

def _argmin_1d(f, lo, hi):
    """Dense grid then golden-section refinement of a convex 1-D function."""
    xs = np.linspace(lo, hi, 20001)
    fx = np.array([f(x) for x in xs])
    k = int(np.argmin(fx))
    a, b = xs[max(k - 1, 0)], xs[min(k + 1, len(xs) - 1)]
    g = (math.sqrt(5) - 1) / 2
    for _ in range(200):
        c, d = b - g * (b - a), a + g * (b - a)
        if f(c) <= f(d):
            b = d
        else:
            a = c
    return 0.5 * (a + b)


@pytest.mark.parametrize("b0,v,lam,eta", [(0.3, 0.5, 0.2, 2.0), (-1.0, 0.1, 0.4, 1.5),
                                          (0.0, -3.0, 1.0, 4.0), (0.2, -0.3, 0.05, 0.7),
                                          (0.0, 0.1, 0.5, 1.0)])
def test_beta_prox_is_argmin(b0, v, lam, eta):
    # beta_argmin: argmin_b lam|b| - v b + (eta/2)(b - b0)^2
    f = lambda b: lam * abs(b) - v * b + 0.5 * eta * (b - b0) ** 2
    want = _argmin_1d(f, -10, 10)
    got = pqr.beta_prox(np.array([b0]), np.array([v]), np.array([lam]), eta)[0]
    # golden section resolves the argmin only to ~sqrt(eps); the value test is sharp
    assert abs(got - want) < 1e-6
    assert f(got) <= f(want) + 1e-15


@pytest.mark.parametrize("z0,th,tau,n,mu", [(0.5, 0.01, 0.5, 10, 0.2), (-0.3, -0.02, 0.9, 10, 1.0),
                                            (0.0, 0.0, 0.1, 5, 3.0), (1.0, -0.5, 0.3, 4, 0.5),
                                            (0.01, 0.002, 0.7, 20, 0.05)])
def test_z_prox_is_argmin(z0, th, tau, n, mu):
    # second line of fsppa_update: argmin_z (1/n) rho_tau(z) - theta z + (mu/2)(z - z0)^2
    f = lambda z: float(pqr.pinball(z, tau)) / n - th * z + 0.5 * mu * (z - z0) ** 2
    want = _argmin_1d(f, -20, 20)
    got = pqr.z_prox(np.array([z0]), np.array([th]), tau, n, mu)[0]
    assert abs(got - want) < 1e-6
    assert f(got) <= f(want) + 1e-15


def test_pinball_values():
    # rho_tau(z) = (tau - 1{z<0}) z
    assert pqr.pinball(2.0, 0.3) == pytest.approx(0.6)
    assert pqr.pinball(-2.0, 0.3) == pytest.approx(1.4)
    assert pqr.pinball(0.0, 0.7) == 0.0


# ----------------------------------------------------------------------------
# closed forms: the sample quantile and lambda_max
# ----------------------------------------------------------------------------

def _tiny(seed, n, p):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p))
    y = X[:, 0] - 0.5 * X[:, min(1, p - 1)] + rng.standard_t(3, n)
    return pqr.with_intercept(X), y


@pytest.mark.parametrize("n,tau", [(31, 0.5), (40, 0.25), (57, 0.9), (50, 0.1)])
def test_intercept_only_is_sample_quantile(n, tau):
    rng = np.random.default_rng(n)
    y = rng.standard_normal(n) * 3 + 1
    X1 = np.ones((n, 1))
    lam = np.zeros(1)
    blocks = pqr.partition(0, 1) if False else [np.array([0])]
    mu = pqr.default_mu(y, 1)
    eta = pqr.step_sizes(X1, blocks, mu)
    res = pqr.fsqrppa(X1, y, tau, lam, blocks, mu, eta, tol_gap=1e-12, max_iter=200000)
    lo, hi = pqr.quantile_minimizers(y, tau)
    assert res["rel_gap"] <= 1e-12
    assert lo - 1e-7 <= res["beta"][0] <= hi + 1e-7
    # the closed form's objective equals the solver's
    obj_cf = float(np.mean(pqr.pinball(y - lo, tau)))
    assert res["primal"] == pytest.approx(obj_cf, rel=1e-10)


def test_quantile_minimizers_brute_force():
    rng = np.random.default_rng(3)
    for n, tau in [(10, 0.5), (11, 0.5), (12, 0.25), (7, 0.9)]:
        y = rng.standard_normal(n)
        lo, hi = pqr.quantile_minimizers(y, tau)
        f = lambda c: float(np.sum(pqr.pinball(y - c, tau)))
        best = min(f(c) for c in y)
        assert f(lo) == pytest.approx(best, abs=1e-12)
        assert f(hi) == pytest.approx(best, abs=1e-12)
        # nothing outside [lo, hi] is optimal
        assert f(lo - 1e-3) > best + 1e-9 and f(hi + 1e-3) > best + 1e-9


@pytest.mark.parametrize("tau", [0.1, 0.5, 0.9])
def test_lambda_max_null_solution(tau):
    X1, y = _tiny(1, 45, 6)
    lmax = pqr.lambda_max(X1, y, tau)
    q, psi = pqr.null_dual(y, tau)
    beta = np.zeros(X1.shape[1])
    beta[0] = q
    for f in (1.0, 1.5):
        lam = np.full(X1.shape[1], f * lmax)
        lam[0] = 0.0
        cert = pqr.dual_certificate(X1, y, tau, lam, beta, psi / len(y))
        assert abs(cert["gap"]) < 1e-12
        val, _ = lp.highs(X1, y, tau, lam)
        assert cert["primal"] == pytest.approx(val, rel=1e-8)
    # just below lambda_max the null fit is no longer optimal
    lam = np.full(X1.shape[1], 0.9 * lmax)
    lam[0] = 0.0
    val, _ = lp.highs(X1, y, tau, lam)
    assert val < pqr.objective(X1, y, beta, tau, lam) - 1e-9


def test_null_dual_is_balanced_and_in_box():
    y = np.array([3.0, 1.0, 2.0, 2.0, 5.0, 2.0, 0.0])   # ties at the quantile
    for tau in (0.3, 0.5, 0.8):
        q, psi = pqr.null_dual(y, tau)
        assert abs(psi.sum()) < 1e-12
        assert np.all(psi >= tau - 1 - 1e-15) and np.all(psi <= tau + 1e-15)


# ----------------------------------------------------------------------------
# exact LP: simplex in rationals vs vertex enumeration vs the golden fixture
# ----------------------------------------------------------------------------

def _rational_instance(seed, n, p):
    rng = np.random.default_rng(seed)
    X1 = [[Fraction(1)] + [Fraction(int(v), 4) for v in rng.integers(-8, 9, p)] for _ in range(n)]
    y = [Fraction(int(v), 3) for v in rng.integers(-12, 13, n)]
    return X1, y


@pytest.mark.parametrize("seed,n,p,tau,lamv", [(0, 6, 2, Fraction(1, 2), Fraction(1, 10)),
                                               (1, 6, 2, Fraction(3, 10), Fraction(1, 5)),
                                               (2, 5, 1, Fraction(7, 10), Fraction(0)),
                                               (3, 6, 3, Fraction(9, 10), Fraction(1, 20))])
def test_simplex_matches_vertex_enumeration(seed, n, p, tau, lamv):
    X1, y = _rational_instance(seed, n, p)
    lam = [Fraction(0)] + [lamv] * p
    c, A, b = lp.lp_data(X1, y, tau, lam)
    val, x = lp.simplex_exact(c, A, b)
    best, beta = lp.vertex_enumeration(X1, y, tau, lam)
    assert val == best
    p1 = p + 1
    beta_lp = [x[j] - x[p1 + j] for j in range(p1)]
    assert lp.objective_exact(X1, y, beta_lp, tau, lam) == val


def test_golden_tiny_lp():
    """Exact optimum stored by tests/golden/make_golden.py (calls only oracle/)."""
    import json, os
    path = os.path.join(os.path.dirname(__file__), "golden", "tiny_lp.json")
    cases = json.load(open(path))
    for case in cases:
        X1 = [[Fraction(v) for v in row] for row in case["X1"]]
        y = [Fraction(v) for v in case["y"]]
        lam = [Fraction(v) for v in case["lam"]]
        tau = Fraction(case["tau"])
        best, _ = lp.vertex_enumeration(X1, y, tau, lam)
        assert best == Fraction(case["optimum"])
        # the float FS-QRPPA oracle reaches the same optimum
        Xf = np.array([[float(v) for v in r] for r in X1])
        yf = np.array([float(v) for v in y])
        lf = np.array([float(v) for v in lam])
        blocks = [np.array([0, 1]), np.arange(2, Xf.shape[1])] if Xf.shape[1] > 2 else [np.arange(Xf.shape[1])]
        mu = pqr.default_mu(yf, len(blocks))
        eta = pqr.step_sizes(Xf, blocks, mu)
        res = pqr.fsqrppa(Xf, yf, float(tau), lf, blocks, mu, eta, tol_gap=1e-11, max_iter=400000)
        assert res["primal"] == pytest.approx(float(best), rel=1e-9, abs=1e-12)


# ----------------------------------------------------------------------------
# FS-QRPPA (Algorithm 1) against HiGHS; the certificate; KKT; H-norm monotonicity
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed,n,p,G,tau,lf,tol", [(0, 80, 30, 3, 0.5, 0.2, 1e-9),
                                                   (1, 40, 60, 5, 0.3, 0.5, 1e-7),
                                                   (2, 100, 20, 2, 0.8, 0.1, 1e-9)])
def test_fsqrppa_reaches_lp_optimum(seed, n, p, G, tau, lf, tol):
    X1, y = _tiny(seed, n, p)
    lam = np.full(p + 1, lf * pqr.lambda_max(X1, y, tau))
    lam[0] = 0.0
    blocks = pqr.partition(p, G)
    mu = pqr.default_mu(y, G)
    eta = pqr.step_sizes(X1, blocks, mu)
    res = pqr.fsqrppa(X1, y, tau, lam, blocks, mu, eta, tol_gap=tol, max_iter=300000)
    val, beta_lp = lp.highs(X1, y, tau, lam)
    assert res["rel_gap"] <= tol
    assert val <= res["primal"] <= val * (1 + 2 * tol) + 1e-12
    kkt = pqr.kkt_violation(X1, y, tau, lam, res["beta"], res["theta"], zero_tol=1e-7)
    assert kkt["intercept"] < 1e-6 and kkt["stationarity"] < 1e-2 * lam.max()


def test_certificate_weak_duality():
    X1, y = _tiny(7, 50, 12)
    tau = 0.4
    lam = np.full(13, 0.15 * pqr.lambda_max(X1, y, tau))
    lam[0] = 0
    val, _ = lp.highs(X1, y, tau, lam)
    rng = np.random.default_rng(0)
    for _ in range(50):
        beta = rng.standard_normal(13) * 0.3
        theta = rng.standard_normal(50) * 0.02
        c = pqr.dual_certificate(X1, y, tau, lam, beta, theta)
        assert c["gap"] >= -1e-14
        assert c["dual"] <= val + 1e-12          # a feasible dual point bounds P* from below
        assert c["gap"] >= c["primal"] - val - 1e-12


@pytest.mark.parametrize("standardized", [True, False])
def test_certificate_weak_duality_with_unpenalized_columns(standardized):
    """lam_j = 0 on some feature columns: the certificate's dual point satisfies
    sum theta = 0 and x_j^T theta = 0 there (to rounding) and still bounds the LP
    optimum from below; on a raw design the columns are not orthogonal to the
    intercept, so the projection has to keep sum theta = 0 itself."""
    rng = np.random.default_rng(11)
    n, p = 40, 10
    X = rng.integers(0, 3, (n, p)).astype(float) + (0 if standardized else 0.5)
    Xs = pqr.standardize(X)[0] if standardized else X
    X1 = pqr.with_intercept(Xs)
    y = X1[:, 1:4] @ np.array([1.0, -0.5, 0.8]) + rng.standard_t(3, n)
    tau = 0.6
    lam = np.full(p + 1, 0.1 * pqr.lambda_max(X1, y, tau))
    lam[0] = 0
    lam[[2, 5]] = 0.0                                   # two unpenalized features
    val, beta_lp = lp.highs(X1, y, tau, lam)
    for _ in range(30):
        beta = rng.standard_normal(p + 1) * 0.3
        theta = rng.standard_normal(n) * 0.02
        c = pqr.dual_certificate(X1, y, tau, lam, beta, theta)
        t = c["theta_feasible"]
        assert abs(t.sum()) < 1e-15 and np.max(np.abs(X1[:, [2, 5]].T @ t)) < 1e-15
        assert np.all(t >= (tau - 1) / n - 1e-18) and np.all(t <= tau / n + 1e-18)
        assert c["dual"] <= val + 1e-12
        assert c["alpha"] > 0
    # a converged FS-QRPPA run certifies, to a small gap, the LP optimum
    blocks = pqr.partition(p, 2)
    mu = pqr.default_mu(y, 2)
    eta = pqr.step_sizes(X1, blocks, mu)
    res = pqr.fsqrppa(X1, y, tau, lam, blocks, mu, eta, tol_gap=1e-8, max_iter=400_000)
    assert res["rel_gap"] <= 1e-8
    assert val * (1 - 1e-12) <= res["primal"] <= val * (1 + 1e-8) + 1e-12


@pytest.mark.parametrize("tau", [0.1, 0.5, 0.93])
def test_quantized_certificate_exact_feasibility_and_agreement(tau):
    """The exactly representable dual point theta_q = unit T: its integer sum is zero,
    every entry lies in the box (checked in exact rationals against the FP64 bounds),
    its dual value bounds the LP optimum from below, and at a near-optimal iterate it
    is within the quantisation (2^-27 of the box per entry) of the FP64 certificate."""
    n, p = 60, 15
    X1, y = _tiny(13, n, p)
    lam = np.full(p + 1, 0.2 * pqr.lambda_max(X1, y, tau))
    lam[0] = 0.0
    val, _ = lp.highs(X1, y, tau, lam)
    lo, hi = Fraction((tau - 1.0) / n), Fraction(tau / n)
    rng = np.random.default_rng(3)
    for _ in range(30):
        beta = rng.standard_normal(p + 1) * 0.3
        theta = rng.standard_normal(n) * 0.02
        c = pqr.quantized_dual_certificate(X1, y, tau, lam, beta, theta)
        assert c is not None
        T, unit = c["T"], Fraction(c["unit"])
        assert int(T.sum()) == 0
        assert all(lo <= int(t) * unit <= hi for t in T)
        assert c["dual"] <= val + 1e-12
        assert 0.0 < c["alpha"] <= 1.0
    blocks = pqr.partition(p, 3)
    mu = pqr.default_mu(y, 3)
    eta = pqr.step_sizes(X1, blocks, mu)
    res = pqr.fsqrppa(X1, y, tau, lam, blocks, mu, eta, tol_gap=1e-8, max_iter=400_000)
    cf = pqr.dual_certificate(X1, y, tau, lam, res["beta"], res["theta"])
    cq = pqr.quantized_dual_certificate(X1, y, tau, lam, res["beta"], res["theta"])
    assert cf["rel_gap"] <= 1e-8
    assert abs(cq["dual"] - cf["dual"]) <= 1e-6 * abs(cf["dual"])
    assert val * (1 - 1e-6) <= cq["dual"] <= val + 1e-12


def test_dual_value_from_chunked_ratios_bounds_the_optimum():
    """dual_value (the certificate's last step, for ratios computed column chunk by
    column chunk): the maximum ratio over chunks gives a feasible alpha t, so the value
    bounds the LP optimum from below, reaches it at the exact optimal dual point, and
    scaling is applied only when some ratio exceeds 1."""
    n, p = 40, 9
    X1, y = _tiny(21, n, p)
    tau = 0.35
    lam = np.full(p + 1, 0.2 * pqr.lambda_max(X1, y, tau))
    lam[0] = 0.0
    val, _, th = lp.highs_with_duals(X1, y, tau, lam)
    rng = np.random.default_rng(4)
    for _ in range(30):
        t = pqr.project_box_sum(rng.standard_normal(n) * 0.05, (tau - 1) / n, tau / n)
        ratios = [np.max(np.abs(X1[:, 1 + c].T @ t) / lam[1 + c]) for c in np.array_split(np.arange(p), 3)]
        d = pqr.dual_value(y, t, max(ratios))
        a = min(1.0, 1.0 / max(ratios))
        assert np.max(np.abs(X1[:, 1:].T @ (a * t)) / lam[1:]) <= 1 + 1e-12
        assert d <= val + 1e-12
    assert pqr.dual_value(y, th, 0.5) == pytest.approx(float(y @ th), rel=1e-14)
    r = np.max(np.abs(X1[:, 1:].T @ th) / lam[1:])
    assert r <= 1 + 1e-8
    assert pqr.dual_value(y, th, r) == pytest.approx(val, rel=1e-7)


def test_cached_residual_step_equals_the_plain_step():
    """Carrying r^k from the previous step is the same iteration (to rounding) as
    recomputing it from (beta^k, z^k)."""
    n, p = 50, 20
    X1, y = _tiny(23, n, p)
    tau = 0.3
    lam = np.full(p + 1, 0.2 * pqr.lambda_max(X1, y, tau))
    lam[0] = 0.0
    blocks = pqr.partition(p, 3)
    mu = pqr.default_mu(y, 3)
    eta = pqr.step_sizes(X1, blocks, mu)
    b, z, t = pqr.zero_start(y, p + 1)
    b2, z2, t2 = b.copy(), z.copy(), t.copy()
    r2 = X1 @ b2 + z2 - y
    for _ in range(40):
        b, z, t = pqr.fsqrppa_step(X1, y, tau, lam, blocks, mu, eta, b, z, t)
        b2, z2, t2, r2 = pqr.fsqrppa_step_cached(X1, y, tau, lam, blocks, mu, eta, b2, z2, t2, r2)
    assert np.allclose(b, b2, rtol=1e-10, atol=1e-13)
    assert np.allclose(t, t2, rtol=1e-10, atol=1e-15)
    assert np.allclose(r2, X1 @ b2 + z2 - y, atol=1e-12)


def test_h_norm_successive_difference_non_increasing():
    X1, y = _tiny(4, 70, 40)
    tau, G = 0.5, 4
    lam = np.full(41, 0.2 * pqr.lambda_max(X1, y, tau))
    lam[0] = 0
    blocks = pqr.partition(40, G)
    mu = pqr.default_mu(y, G)
    eta = pqr.step_sizes(X1, blocks, mu)
    res = pqr.fsqrppa(X1, y, tau, lam, blocks, mu, eta, tol_gap=0.0, max_iter=3000,
                      check_every=10**9, record=True)
    h = np.array(res["history"])
    assert np.all(h >= -1e-18)
    assert np.all(np.diff(h) <= 1e-12 * h[:-1] + 1e-30)
    # Corollary 1: eventually linear decrease of the successive differences
    tail = np.log(h[-1000:] + 1e-300)
    slope = np.polyfit(np.arange(len(tail)), tail, 1)[0]
    assert slope < 0


def test_h_norm_detects_too_small_eta():
    """With eta_g far below mu * Lambda_max the metric H is indefinite and the
    successive differences stop decreasing, which is what the GPU divergence
    detector relies on."""
    X1, y = _tiny(5, 60, 30)
    tau, G = 0.5, 2
    lam = np.full(31, 0.2 * pqr.lambda_max(X1, y, tau))
    lam[0] = 0
    blocks = pqr.partition(30, G)
    mu = pqr.default_mu(y, G)
    eta = 0.05 * pqr.step_sizes(X1, blocks, mu)
    res = pqr.fsqrppa(X1, y, tau, lam, blocks, mu, eta, tol_gap=0.0, max_iter=400,
                      check_every=10**9, record=True)
    h = np.array(res["history"])
    assert np.any(np.diff(h) > 0)


# ----------------------------------------------------------------------------
# planted mistakes: the pins above must catch plausible bugs in the oracle
# ----------------------------------------------------------------------------

def _solve_small(step):
    X1, y = _tiny(11, 40, 10)
    tau, G = 0.3, 2
    lam = np.full(11, 0.2 * pqr.lambda_max(X1, y, tau))
    lam[0] = 0
    blocks = pqr.partition(10, G)
    mu = pqr.default_mu(y, G)
    eta = pqr.step_sizes(X1, blocks, mu)
    beta, z, theta = pqr.zero_start(y, 11)
    for _ in range(20000):
        beta, z, theta = step(X1, y, tau, lam, blocks, mu, eta, beta, z, theta)
    val, _ = lp.highs(X1, y, tau, lam)
    return pqr.objective(X1, y, beta, tau, lam), val


def test_planted_mistakes_are_caught(monkeypatch):
    good, val = _solve_small(pqr.fsqrppa_step)
    assert good == pytest.approx(val, rel=1e-8)
    # (a) tau and 1 - tau swapped in the z prox
    orig = pqr.z_prox
    monkeypatch.setattr(pqr, "z_prox", lambda z, th, tau, n, mu: orig(z, th, 1 - tau, n, mu))
    bad, _ = _solve_small(pqr.fsqrppa_step)
    assert abs(bad - val) > 1e-4 * val
    monkeypatch.setattr(pqr, "z_prox", orig)
    # (b) threshold lam/eta dropped to lam/(2 eta)
    origb = pqr.beta_prox
    monkeypatch.setattr(pqr, "beta_prox", lambda b, v, l, e: origb(b, v, 0.5 * l, e))
    bad, _ = _solve_small(pqr.fsqrppa_step)
    assert abs(bad - val) > 1e-4 * val


# ----------------------------------------------------------------------------
# folded-concave derivatives (eqs. scad, mcp) at hand-computed points
# ----------------------------------------------------------------------------

def test_scad_mcp_derivatives():
    lam = 0.5
    # SCAD, a = 3.7: lam on [0, lam]; (a lam - b)/(a - 1) on (lam, a lam); 0 beyond
    assert pqr.scad_deriv(0.2, lam) == pytest.approx(0.5)
    assert pqr.scad_deriv(-0.5, lam) == pytest.approx(0.5)
    assert pqr.scad_deriv(1.0, lam) == pytest.approx((1.85 - 1.0) / 2.7)
    assert pqr.scad_deriv(1.85, lam) == pytest.approx(0.0)
    assert pqr.scad_deriv(5.0, lam) == 0.0
    # MCP, a = 3: lam - b/a on [0, a lam]; 0 beyond
    assert pqr.mcp_deriv(0.3, lam) == pytest.approx(0.4)
    assert pqr.mcp_deriv(1.5, lam) == pytest.approx(0.0)
    assert pqr.mcp_deriv(2.0, lam) == 0.0


def test_lla_stage_is_weighted_l1_optimum():
    X1, y = _tiny(9, 60, 8)
    tau, G = 0.5, 2
    lmax = pqr.lambda_max(X1, y, tau)
    blocks = pqr.partition(8, G)
    mu = pqr.default_mu(y, G)
    eta = pqr.step_sizes(X1, blocks, mu)
    res = pqr.lla(X1, y, tau, 0.3 * lmax, blocks, mu, eta, L=1, penalty_kind="mcp",
                  tol_gap=1e-9, max_iter=300000)
    val, _ = lp.highs(X1, y, tau, res["lam"])
    assert res["primal"] == pytest.approx(val, rel=2e-9)


# ----------------------------------------------------------------------------
# standardisation and the back-transform
# ----------------------------------------------------------------------------

def test_standardize_and_back_transform():
    rng = np.random.default_rng(2)
    X = rng.integers(0, 3, (50, 8)).astype(float)
    X[:, 3] = 1.0   # zero variance
    Xt, m, s = pqr.standardize(X)
    ok = s > 0
    assert np.allclose(Xt[:, ok].mean(axis=0), 0, atol=1e-14)
    assert np.allclose((Xt[:, ok] ** 2).sum(axis=0), 50)
    assert s[3] == 0 and np.all(Xt[:, 3] == 0)
    bs = rng.standard_normal(9)
    bs[1 + 3] = 0
    b = pqr.back_transform(bs, m, s)
    assert np.allclose(pqr.with_intercept(Xt) @ bs, pqr.with_intercept(X) @ b)


# ---- the scoring network of the learned warm start (oracle/mlp.py) ----
def test_mlp_oracle_gradient_central_differences():
    """The FP64 oracle's backward pass against central differences of its loss, on
    every parameter block (a dropped term or transposed weight shows up here)."""
    from oracle import mlp as omlp
    rng = np.random.default_rng(3)
    prm = omlp.init_params(1)
    F = rng.standard_normal((17, 4))
    t = rng.standard_normal(17) * 0.2
    a = (rng.random(17) < 0.3).astype(float)
    g = omlp.flatten(omlp.backward(prm, F, t, a, w_reg=2.0, w_pos=3.0))
    flat = omlp.flatten(prm)
    h = 1e-6
    picks = np.concatenate([rng.choice(flat.size, 60, replace=False),
                            np.cumsum([0] + [int(np.prod(omlp.SHAPES[k])) for k in omlp.ORDER])[:-1]])
    for q in picks:
        e = np.zeros_like(flat)
        e[q] = h
        fd = (omlp.loss(omlp.unflatten(flat + e), F, t, a, 2.0, 3.0) -
              omlp.loss(omlp.unflatten(flat - e), F, t, a, 2.0, 3.0)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-7 * max(1.0, abs(g[q]))


def test_mlp_oracle_forward_closed_form():
    """With one hidden unit active per layer the network is a closed-form scalar
    chain: out = W3 silu(W2 silu(W1 f + b1) + b2) + b3, written out by hand."""
    from oracle import mlp as omlp
    prm = {k: np.zeros_like(v) for k, v in omlp.init_params(0).items()}
    names = list(prm)
    W1, b1, W2, b2, W3, b3 = (prm[k] for k in names)
    W1[0, 2] = 0.5; b1[0] = -0.1
    W2[3, 0] = 2.0; b2[3] = 0.25
    W3[0, 3] = -1.5; W3[1, 3] = 0.75; b3[:] = [0.2, -0.3]
    f = np.array([[0.0, 0.0, 1.2, 0.0]])
    sil = lambda x: x / (1 + np.exp(-x))
    h2 = sil(2.0 * sil(0.5 * 1.2 - 0.1) + 0.25)
    out, _ = omlp.forward(prm, f)
    assert np.allclose(out[0], [-1.5 * h2 + 0.2, 0.75 * h2 - 0.3], rtol=1e-14, atol=1e-15)


# ----------------------------------------------------------------------------
# KKT report (Prop. 1 with subgradients) at an exact optimum, then with planted
# violations of known size; exact LP duals; the uniqueness check
# ----------------------------------------------------------------------------

def _exact_optimum(seed, n, p, tau, lam_num):
    """Integer data, an exact rational optimum (primal beta, dual theta) from the
    simplex over Fractions, and its float copies."""
    rng = np.random.default_rng(seed)
    X = rng.integers(-3, 4, size=(n, p))
    X1 = np.hstack([np.ones((n, 1), dtype=np.int64), X])
    y = rng.integers(-6, 7, size=n)
    tau_f = Fraction(tau).limit_denominator(100)
    lam = [Fraction(0)] + [Fraction(lam_num, 10)] * p
    c, A, b = lp.lp_data(X1.tolist(), y.tolist(), tau_f, lam)
    val, x, th = lp.simplex_exact(c, A, b, duals=True)
    p1 = p + 1
    beta = [x[j] - x[p1 + j] for j in range(p1)]
    return X1, y, tau_f, lam, val, beta, th


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_exact_duals_strong_duality_and_feasibility(seed):
    """The simplex's dual is feasible for the dual of eq. main_lagrangian (box, zero sum,
    |x_j^T theta| <= lam_j), exactly in rationals, and y^T theta equals the optimum."""
    X1, y, tau, lam, val, beta, th = _exact_optimum(seed, 9, 3, 0.3, 2)
    n = len(y)
    assert sum(Fraction(int(y[i])) * th[i] for i in range(n)) == val
    assert all((tau - 1) / n <= t <= tau / n for t in th)
    for j in range(X1.shape[1]):
        d = sum(Fraction(int(X1[i, j])) * th[i] for i in range(n))
        assert (d == 0) if j == 0 else (abs(d) <= lam[j])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kkt_violation_zero_at_optimum_and_planted_sizes(seed):
    X1, y, tau, lam, val, beta, th = _exact_optimum(seed, 10, 3, 0.4, 2)
    n = len(y)
    Xf, yf = X1.astype(np.float64), y.astype(np.float64)
    lf = np.array([float(v) for v in lam])
    b = np.array([float(v) for v in beta])
    t = np.array([float(v) for v in th])
    tf = float(tau)
    k0 = pqr.kkt_violation(Xf, yf, tf, lf, b, t, zero_tol=1e-9)
    assert max(k0.values()) < 1e-12
    hi, lo = tf / n, (tf - 1) / n
    r = yf - Xf @ b
    delta = 0.37 / n
    # a dual value pushed out of the box on a row with a positive, a negative and a
    # zero residual: the box violation is exactly the push
    for sel, val_t in [(r > 1e-9, hi + delta), (r < -1e-9, lo - delta), (np.abs(r) <= 1e-9, hi + delta)]:
        rows = np.nonzero(sel)[0]
        if len(rows) == 0:
            continue
        t2 = t.copy()
        t2[rows[0]] = val_t
        k = pqr.kkt_violation(Xf, yf, tf, lf, b, t2, zero_tol=1e-9)
        assert k["dual_box"] == pytest.approx(delta, rel=1e-9)
    # the sign of a nonzero penalized coefficient flipped: x_j^T theta = lam_j sign(beta_j)
    # held, so the stationarity residual becomes 2 lam_j
    nz = [j for j in range(1, len(b)) if b[j] != 0]
    if nz:
        b2 = b.copy()
        b2[nz[0]] = -b2[nz[0]]
        k = pqr.kkt_violation(Xf, yf, tf, lf, b2, t, zero_tol=1e-9)
        assert k["stationarity"] == pytest.approx(2 * lf[nz[0]], rel=1e-12)
    # a zero coefficient made positive: the residual is lam_j - x_j^T theta
    zc = [j for j in range(1, len(b)) if b[j] == 0]
    if zc:
        j = zc[0]
        vj = float(Xf[:, j] @ t)
        b3 = b.copy()
        b3[j] = 1e-3
        k = pqr.kkt_violation(Xf, yf, tf, lf, b3, t, zero_tol=1e-9)
        assert k["stationarity"] >= abs(vj - lf[j]) * (1 - 1e-12)
        assert k["stationarity"] == pytest.approx(max(abs(vj - lf[j]), k0["stationarity"]), rel=1e-9)
    # theta shifted by delta: the intercept's residual |sum theta| is n delta
    k = pqr.kkt_violation(Xf, yf, tf, lf, b, t + delta, zero_tol=1e-9)
    assert k["intercept"] == pytest.approx(n * delta, rel=1e-9)


def test_uniqueness_check_against_exact_vertex_enumeration():
    """coef_uniqueness (with the exact dual) agrees with the number of distinct optimal
    vertices found by exact enumeration, on generic data and on planted degeneracy
    (a duplicated column: beta_1 + beta_2 is fixed but its split is not)."""
    seen = {True: 0, False: 0}
    for seed in range(6):
        X1, y, tau, lam, val, beta, th = _exact_optimum(seed, 6, 2, 0.3, 1)
        if seed >= 3:   # duplicate column 1 into column 2
            X1 = X1.copy()
            X1[:, 2] = X1[:, 1]
            c, A, b = lp.lp_data(X1.tolist(), y.tolist(), tau, lam)
            val, x, th = lp.simplex_exact(c, A, b, duals=True)
        best, pts = lp.optimal_vertices(X1.tolist(), y.tolist(), tau, lam)
        assert best == val
        u = pqr.coef_uniqueness(X1.astype(np.float64), float(tau), np.array([float(v) for v in lam]),
                                np.array([float(v) for v in th]))
        # the check is conservative: it may only claim uniqueness when it holds
        if u["unique"]:
            assert len(pts) == 1
        if seed >= 3 and any(p[1] != 0 or p[2] != 0 for p in pts):
            assert not u["unique"]
        seen[u["unique"]] += 1
    assert seen[True] >= 1 and seen[False] >= 1


def test_uniqueness_check_against_highs_face_ranges():
    """Generic Gaussian data: the check passes and HiGHS finds every coefficient's range
    over the optimal face to be a point.  Intercept only with n tau an integer: the
    check fails and the face range of beta_0 is [y_(n tau), y_(n tau + 1)] (closed form)."""
    X1, y = _tiny(5, 40, 8)
    tau = 0.5
    lam = np.full(9, 0.2 * pqr.lambda_max(X1, y, tau))
    lam[0] = 0.0
    val, beta, th = lp.highs_with_duals(X1, y, tau, lam)
    u = pqr.coef_uniqueness(X1, tau, lam, th)
    assert u["unique"]
    for (a, b) in lp.highs_face_range(X1, y, tau, lam, val, range(9), rel=1e-10):
        assert b - a < 1e-6
    # null model at lambda >= lambda_max with n tau integral: an interval of minimisers
    lam2 = np.full(9, 1.5 * pqr.lambda_max(X1, y, tau))
    lam2[0] = 0.0
    val2, beta2, th2 = lp.highs_with_duals(X1, y, tau, lam2)
    assert not pqr.coef_uniqueness(X1, tau, lam2, th2)["unique"]
    (a, b), = lp.highs_face_range(X1, y, tau, lam2, val2, [0], rel=1e-12)
    lo_q, hi_q = pqr.quantile_minimizers(y, tau)
    assert a == pytest.approx(lo_q, abs=1e-7) and b == pytest.approx(hi_q, abs=1e-7)


@pytest.mark.parametrize("seed,tau,frac", [(51, 0.5, 0.5), (52, 0.3, 0.3), (53, 0.8, 0.2)])
def test_strong_rule_screened_solve_reaches_the_optimum(seed, tau, frac):
    """The strong rule is a heuristic (it may discard an active column); the dual check
    over every discarded column (Prop. 1 at the restricted optimum) makes the screened
    solve exact: its value equals the full LP optimum and its coefficients vanish
    outside the final set.  At lambda >= lambda_max the rule keeps nothing and the null
    fit is already optimal."""
    rng = np.random.default_rng(seed)
    n, p = 80, 300
    X = rng.integers(0, 3, (n, p)).astype(float)
    X1 = pqr.with_intercept(pqr.standardize(X)[0])
    y = X1[:, 1:6] @ rng.uniform(0.5, 1.5, 5) + rng.standard_t(3, n)
    lmax = pqr.lambda_max(X1, y, tau)
    _, psi = pqr.null_dual(y, tau)
    score = X1[:, 1:].T @ psi / n
    assert np.max(np.abs(score)) == pytest.approx(lmax, rel=1e-12)
    assert len(pqr.strong_rule(score, 1.0 * lmax, lmax)) == 1     # only the maximiser
    assert len(pqr.strong_rule(score, 1.2 * lmax, lmax)) == 0
    lam = np.full(p + 1, frac * lmax)
    lam[0] = 0.0
    A = pqr.strong_rule(score, frac * lmax, lmax)
    val, beta, th, rounds, added = pqr.screened_solve(X1, y, tau, lam, A, lp.highs_with_duals)
    full, _ = lp.highs(X1, y, tau, lam)
    assert val == pytest.approx(full, rel=1e-9, abs=1e-12)
    assert pqr.objective(X1, y, beta, tau, lam) == pytest.approx(full, rel=1e-8)
    assert np.max(np.abs(X1[:, 1:].T @ th) / lam[1:]) <= 1 + 1e-8
