"""Screened warm start (pqr_solve_screened): the sequential strong rule on the null-fit
scores proposes the active set, the reduced solve and the full-design certificate make
the answer exact; the proposal itself equals the oracle's strong rule."""
import numpy as np
import pytest

from oracle import lp, pqr
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _ctx(X, **kw):
    import paper_2601_02826_amd as pq
    return pq.Context.from_tensor(H.to_device_cols(X.astype(np.uint8)), store_fmt="i8", **kw)


@pytest.mark.parametrize("tau,frac,budget,tol", [(0.5, 0.75, 0, 1e-6), (0.3, 0.6, 0, 1e-6),
                                                 (0.8, 0.5, 100, 1e-5)])
def test_screened_solve_reaches_the_lp_optimum(tau, frac, budget, tol):
    n, p = 600, 4000
    X, y = H.genotype_problem(n, p, seed=61, tau=tau, n_causal=10)
    X1, _, _ = H.oracle_design(X, True)
    lmax = pqr.lambda_max(X1, y, tau)
    lam = frac * lmax
    lam_vec = H.lam_vector(p, lam)
    val, _ = lp.highs(X1, y, tau, lam_vec)
    ctx = _ctx(X, G=4, tol_gap=tol, cert_every=100, max_iter=2_000_000)
    r = ctx.solve_screened(y, tau, lam, budget=budget, max_rounds=8)
    _, psi = pqr.null_dual(y, tau)
    score = X1[:, 1:].T @ psi / n
    A0 = pqr.strong_rule(score, lam, lmax)
    # columns within rounding of the rule's cut may fall either way
    ties = int(np.sum(np.abs(np.abs(score) - (2 * lam - lmax)) <= 1e-9 * lmax))
    want = len(A0) if budget == 0 else budget
    print(f"tau {tau}: |A| {r['active_initial']} (oracle rule {len(A0)}) -> {r['active_final']}, "
          f"{r['rounds']} rounds, {r['iters']} iterations, fallback {r['fallback']}")
    assert abs(r["active_initial"] - want) <= (ties if budget == 0 else 0)
    assert r["status"] == 0 and r["rel_gap"] <= tol and r["fallback"] == 0
    p_gpu = pqr.objective(X1, y, r["beta_std"], tau, lam_vec)
    assert val * (1 - 1e-12) <= p_gpu <= val * (1 + tol) + 1e-12
    ctx.close()


def test_graph_replay_equals_direct_launches():
    """The iteration chunks replayed as captured HIP graphs (the default) give the same
    iterates, bit for bit, as the kernels launched one by one: a lambda path with
    device warm starts, many replays per solve with certificates between them."""
    n, p, tau = 500, 300, 0.5
    X, y = H.genotype_problem(n, p, seed=13)
    runs = []
    for mode in (0, 1):
        ctx = _ctx(X, G=3, tol_gap=1e-6, cert_every=100, max_iter=2_000_000, launch_mode=mode)
        lmax = ctx.lambda_max(y, tau)
        path = [ctx.solve(y, tau, f * lmax, start="zero" if k == 0 else "device")
                for k, f in enumerate([0.8, 0.5, 0.35])]
        runs.append(path)
        ctx.close()
    for a, b in zip(*runs):
        assert a["iters"] == b["iters"] and a["iters"] >= 300
        assert np.array_equal(a["beta_std"], b["beta_std"])
        assert np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["z"], b["z"])
        assert a["primal"] == b["primal"] and a["dual"] == b["dual"]
