"""Step-level parity: k iterations of Algorithm 1 on the GPU against the FP64 oracle,
from the same state with the same mu and eta, for every storage format."""
import numpy as np
import pytest

from oracle import pqr
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _oracle_steps(X1, y, tau, lam_vec, blocks, mu, eta, state, k):
    b, z, t = state
    for _ in range(k):
        b, z, t = pqr.fsqrppa_step(X1, y, tau, lam_vec, blocks, mu, eta, b, z, t)
    return b, z, t


def _check(got, want, rtol, label):
    for name, g, w in zip(("beta", "z", "theta"), got, want):
        scale = max(np.max(np.abs(w)), 1e-300)
        err = np.max(np.abs(g - w)) / scale
        assert err <= rtol, f"{label}: {name} rel err {err:.3e} > {rtol:.1e}"


@pytest.mark.parametrize("icpt", [True, False])
@pytest.mark.parametrize("iter_prec,rtol", [("f64", 1e-11), ("f32", 2e-5)])
@pytest.mark.parametrize("n,p,G", [(300, 517, 5), (1100, 130, 3)])
def test_step_parity_gaussian(iter_prec, rtol, n, p, G, icpt):
    import paper_2601_02826_amd as pq
    X, y = H.gaussian_problem(n, p, seed=21)
    X1, _, _ = H.oracle_design(X, False)
    tau = 0.3
    lam = 0.2 * pqr.lambda_max(X1, y, tau)
    ctx = pq.Context.from_tensor(H.to_device_cols(X), store_fmt="f64", standardize=False, G=G,
                                 iter_prec=iter_prec, intercept_block=int(icpt))
    Gg, bounds, Lam = ctx.blocks()
    blocks = H.oracle_blocks(p, G, icpt)
    assert Gg == len(blocks)
    assert [int(b[-1]) for b in blocks] == [int(v) for v in bounds[1:]]
    # the Lanczos estimates bound the exact block spectra from above, within the margin
    exact = np.array([pqr.block_lambda_max(X1[:, b]) for b in blocks])
    assert np.all(Lam >= exact * (1 - 1e-6)) and np.all(Lam <= exact * 1.05)
    mu = pqr.default_mu(y, G, 0.1)
    eta = pqr.step_sizes(X1, blocks, mu)
    lam_vec = H.lam_vector(p, lam)
    state = H.random_state(n, p, seed=5)
    for k in (1, 7):
        got = ctx.iterate(y, tau, lam, mu, eta, k, *state)
        want = _oracle_steps(X1, y, tau, lam_vec, blocks, mu, eta, state, k)
        _check(got, want, rtol * (3 if k > 1 else 1), f"{iter_prec} k={k}")
    ctx.close()


@pytest.mark.parametrize("store", ["i8", "2bit", "fp8", "bf16", "f32", "f64"])
def test_step_parity_genotype_formats(store):
    """Standardized genotype columns; the store formats hold the dosages exactly,
    so every format must agree with the FP64 oracle to FP32 accuracy."""
    import paper_2601_02826_amd as pq
    n, p, G = 1500, 700, 4        # n pads to 1536 (ragged tail), p to 704 (ragged group)
    X, y = H.genotype_problem(n, p, seed=3)
    X1, m, s = H.oracle_design(X, True)
    tau = 0.7
    lam = 0.15 * pqr.lambda_max(X1, y, tau)
    Xd = H.to_device_cols(X, np.uint8)
    ctx = pq.Context.from_tensor(Xd, store_fmt=store, standardize=True, G=G, iter_prec="f32")
    blocks = H.oracle_blocks(p, G)
    mu = pqr.default_mu(y, G, 0.1)
    eta = pqr.step_sizes(X1, blocks, mu)
    lam_vec = H.lam_vector(p, lam)
    state = H.random_state(n, p, seed=9)
    got = ctx.iterate(y, tau, lam, mu, eta, 3, *state)
    want = _oracle_steps(X1, y, tau, lam_vec, blocks, mu, eta, state, 3)
    _check(got, want, 5e-5, store)
    ctx.close()


def test_lambda_max_and_score():
    import paper_2601_02826_amd as pq
    n, p = 777, 250
    X, y = H.genotype_problem(n, p, seed=4)
    X1, _, _ = H.oracle_design(X, True)
    ctx = pq.Context.from_tensor(H.to_device_cols(X, np.uint8), store_fmt="i8", G=2)
    for tau in (0.1, 0.5, 0.9):
        lm, score = ctx.lambda_max(y, tau, score=True)
        want = pqr.lambda_max(X1, y, tau)
        assert lm == pytest.approx(want, rel=1e-12)
        _, psi = pqr.null_dual(y, tau)
        assert np.allclose(score, X1[:, 1:].T @ psi / n, rtol=1e-10, atol=1e-14)
    w = np.abs(np.random.default_rng(0).standard_normal(p + 1)) + 0.1
    lm = ctx.lambda_max(y, 0.5, weights=w)
    assert lm == pytest.approx(pqr.lambda_max(X1, y, 0.5, weights=w), rel=1e-12)
    ctx.close()


def test_kkt_certificate_matches_oracle():
    import paper_2601_02826_amd as pq
    n, p = 400, 333
    X, y = H.gaussian_problem(n, p, seed=8)
    X1, _, _ = H.oracle_design(X, False)
    tau = 0.6
    lam = 0.25 * pqr.lambda_max(X1, y, tau)
    ctx = pq.Context.from_tensor(H.to_device_cols(X), store_fmt="f64", standardize=False, G=3)
    beta, _, theta = H.random_state(n, p, seed=2)
    rep = ctx.kkt(y, tau, lam, beta, theta)
    want = pqr.dual_certificate(X1, y, tau, H.lam_vector(p, lam), beta, theta)
    assert rep["primal"] == pytest.approx(want["primal"], rel=1e-12)
    assert rep["dual"] == pytest.approx(want["dual"], rel=1e-9, abs=1e-14)
    ctx.close()
