"""The interleaved column order on the GPU (a context over pqr_interleaved_order via
pqr_create_subset): it steps like the oracle with the corresponding non-contiguous
partition, its Lanczos step sizes bound the smaller block spectra, and it solves to
the same certified optimum as the contiguous context (the LP optimum)."""
import numpy as np
import pytest

from oracle import lp, pqr
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _problem(n=300, p=1000):
    from datagen.configs import make_ar1
    d = make_ar1(n, p)
    X = d["X"].astype(np.float64)    # the stored values (float32 draws)
    X1, _, _ = H.oracle_design(X, True)
    return X, X1, d["y"]


def _oracle_blocks(il):
    """The interleaved context's blocks as column sets of the source X1."""
    out = []
    for b, c in enumerate(il.block_columns()):
        cols = 1 + np.asarray(c, dtype=np.int64)
        if b == 0:
            cols = np.r_[0, cols]     # block 0 holds the intercept (alone by default)
        out.append(cols)
    return out


def test_step_parity_and_block_spectra():
    import paper_2601_02826_amd as pq
    n, p, G, tau = 300, 1000, 5, 0.3
    X, X1, y = _problem(n, p)
    ctx = pq.Context.from_tensor(H.to_device_cols(X), store_fmt="f64", standardize=True, G=G,
                                 iter_prec="f64")
    il = ctx.interleaved(G=G)
    blocks = _oracle_blocks(il)
    assert sorted(np.concatenate(blocks).tolist()) == list(range(p + 1))
    _, _, Lam_i = il.blocks()
    _, _, Lam_c = ctx.blocks()
    exact = np.array([pqr.block_lambda_max(X1[:, b]) for b in blocks])
    assert np.all(Lam_i >= exact * (1 - 1e-6)) and np.all(Lam_i <= exact * 1.05)
    print(f"Lambda/n contiguous {np.round(Lam_c[1:] / n, 2)}, interleaved {np.round(Lam_i[1:] / n, 2)}")
    assert Lam_i[1:].max() < 0.85 * Lam_c[1:].min()
    lam = 0.2 * pqr.lambda_max(X1, y, tau)
    lam_vec = H.lam_vector(p, lam)
    mu = pqr.default_mu(y, G, 0.1)
    eta = pqr.step_sizes(X1, blocks, mu)
    state = H.random_state(n, p, seed=7)
    for k in (1, 6):
        got = il.iterate(y, tau, lam, mu, eta, k, *state)
        b, z, t = state
        for _ in range(k):
            b, z, t = pqr.fsqrppa_step(X1, y, tau, lam_vec, blocks, mu, eta, b, z, t)
        for name, g_, w_ in zip(("beta", "z", "theta"), got, (b, z, t)):
            err = np.max(np.abs(g_ - w_)) / max(np.max(np.abs(w_)), 1e-300)
            assert err <= 3e-11, f"k={k} {name} rel err {err:.2e}"
    il.close()
    ctx.close()


@pytest.mark.parametrize("tau", [0.3, 0.5])
def test_solve_matches_contiguous_and_lp(tau):
    import paper_2601_02826_amd as pq
    n, p, G = 300, 1000, 5
    X, X1, y = _problem(n, p)
    ctx = pq.Context.from_tensor(H.to_device_cols(X), store_fmt="f32", standardize=True, G=G,
                                 tol_gap=1e-6, cert_every=100, max_iter=2_000_000)
    il = ctx.interleaved(G=G)
    lmax = ctx.lambda_max(y, tau)
    assert il.lambda_max(y, tau) == pytest.approx(lmax, rel=1e-12)
    lam = 0.3 * lmax
    lam_vec = H.lam_vector(p, lam)
    val, _ = lp.highs(X1, y, tau, lam_vec)
    r_c = ctx.solve(y, tau, lam)
    r_i = il.solve(y, tau, lam)
    print(f"tau={tau}: iterations contiguous {r_c['iters']}, interleaved {r_i['iters']}")
    for r in (r_c, r_i):
        p_gpu = pqr.objective(X1, y, r["beta_std"], tau, lam_vec)
        assert r["rel_gap"] <= 1e-6
        assert val * (1 - 1e-12) <= p_gpu <= val * (1 + 1e-6) + 1e-12
        assert r["primal"] == pytest.approx(p_gpu, rel=1e-9)
    # the back-transformed coefficients are in the source order too
    Xraw1 = pqr.with_intercept(X)
    assert np.allclose(Xraw1 @ r_i["beta"], X1 @ r_i["beta_std"], rtol=1e-8, atol=1e-8)
    il.close()
    ctx.close()
