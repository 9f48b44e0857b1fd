"""Batched right-hand sides on the int8 matrix cores: every (tau_k, lambda_k) reaches
its certified gap and agrees with the LP optimum of its own problem."""
import numpy as np
import pytest

from oracle import lp, pqr
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _ctx(X, **kw):
    import paper_2601_02826_amd as pq
    return pq.Context.from_tensor(H.to_device_cols(X, np.uint8), store_fmt="i8", standardize=True,
                                  rows_per_lane=16, **kw)


@pytest.mark.parametrize("K", [5, 16, 21])
def test_batch_matches_lp_optimum(K):
    n, p, G = 1500, 700, 3          # n pads to 2048 rows, p to 704 columns
    X, y = H.genotype_problem(n, p, seed=31)
    X1, _, _ = H.oracle_design(X, True)
    ctx = _ctx(X, G=G, tol_gap=1e-5, cert_every=200, max_iter=400_000)
    taus = np.array([0.2, 0.5, 0.8] * 8)[:K]
    fr = np.array([0.9, 0.6, 0.4, 0.3, 0.25, 0.2, 0.5, 0.7] * 3)[:K]
    lams = np.array([f * pqr.lambda_max(X1, y, t) for f, t in zip(fr, taus)])
    res = ctx.solve_batch(y, taus, lams)
    for k in range(K):
        lam_vec = H.lam_vector(p, lams[k])
        val, _ = lp.highs(X1, y, taus[k], lam_vec)
        p_gpu = pqr.objective(X1, y, res[k]["beta_std"], taus[k], lam_vec)
        assert res[k]["rel_gap"] <= 1e-5, (k, res[k]["rel_gap"])
        assert val * (1 - 1e-12) <= p_gpu <= val * (1 + 1e-5) + 1e-12, (k, p_gpu, val)
        assert res[k]["primal"] == pytest.approx(p_gpu, rel=1e-10)
    ctx.close()


def test_batch_rejects_unsupported_layouts():
    import paper_2601_02826_amd as pq
    n, p = 300, 64
    X, y = H.genotype_problem(n, p, seed=32)
    ctx = pq.Context.from_tensor(H.to_device_cols(X, np.uint8), store_fmt="fp8", G=2)
    with pytest.raises(pq.PQRError) as e:
        ctx.solve_batch(y, [0.5], [0.1])
    assert e.value.status == pq.PQR_ERR_UNSUPPORTED
    ctx.close()
