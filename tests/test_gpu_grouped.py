"""Grouped uneven problems (pqr_solve_grouped): many independent problems of
different shapes iterated together in shared launches.  Each problem's answer equals
its own single solve bit for bit (same kernels, same reduction order, same
certificate schedule) and the LP optimum within its certified gap."""
import numpy as np
import pytest

from oracle import lp, pqr
from tests import helpers as H

pytestmark = pytest.mark.gpu

# (n, p, tau, lambda / lambda_max): uneven rows and columns, a single-group problem,
# a problem whose padding dominates, and one with p > n
SHAPES = [(300, 200, 0.5, 0.3), (700, 1500, 0.25, 0.4), (1200, 500, 0.8, 0.35),
          (450, 3000, 0.5, 0.5), (900, 16, 0.6, 0.2), (1600, 900, 0.1, 0.45)]


def _build(kind, rows_per_lane=0):
    import paper_2601_02826_amd as pq
    ctxs, ys, taus, lams, designs = [], [], [], [], []
    for k, (n, p, tau, frac) in enumerate(SHAPES):
        if kind == "i8":
            X, y = H.genotype_problem(n, p, seed=60 + k, n_causal=min(8, p))
            Xd = H.to_device_cols(X.astype(np.uint8), np.uint8)
            kw = dict(store_fmt="i8", standardize=True, iter_prec="f32")
            X1, _, _ = H.oracle_design(X, True)
        else:
            rng = np.random.default_rng(60 + k)
            X = rng.standard_normal((n, p))
            y = X[:, :3] @ np.array([1.0, -0.5, 0.25]) + rng.standard_t(3, n)
            Xd = H.to_device_cols(X)
            kw = dict(store_fmt="f64", standardize=False, iter_prec="f64")
            X1, _, _ = H.oracle_design(X, False)
        ctx = pq.Context.from_tensor(Xd, G=3, tol_gap=1e-6, cert_every=100, max_iter=2_000_000,
                                     rows_per_lane=rows_per_lane, **kw)
        lam = frac * ctx.lambda_max(y, tau)
        ctxs.append(ctx); ys.append(y); taus.append(tau); lams.append(lam); designs.append(X1)
    return ctxs, ys, taus, lams, designs


@pytest.mark.parametrize("kind,rpl", [("i8", 0), ("i8", 16), ("f64", 0)])
def test_grouped_equals_single_solves_and_lp_optimum(kind, rpl):
    import paper_2601_02826_amd as pq
    ctxs, ys, taus, lams, designs = _build(kind, rpl)
    res, sts = pq.solve_grouped(ctxs, ys, taus, lams)
    assert sts == [pq.PQR_OK] * len(ctxs)
    for i, ctx in enumerate(ctxs):
        single = ctx.solve(ys[i], taus[i], lams[i])
        g = res[i]
        print(f"problem {i} {SHAPES[i]}: iters {g['iters']}, rel_gap {g['rel_gap']:.2e}, "
              f"nnz {g['nnz']}")
        assert g["iters"] == single["iters"] and g["certs"] == single["certs"]
        assert np.array_equal(g["beta_std"], single["beta_std"])
        assert np.array_equal(g["theta"], single["theta"]) and np.array_equal(g["z"], single["z"])
        assert g["primal"] == single["primal"] and g["dual"] == single["dual"]
        assert g["rel_gap"] <= 1e-6
        p = SHAPES[i][1]
        lam_vec = H.lam_vector(p, lams[i])
        val, _ = lp.highs(designs[i], ys[i], taus[i], lam_vec)
        obj = pqr.objective(designs[i], ys[i], g["beta_std"], taus[i], lam_vec)
        assert val * (1 - 1e-12) <= obj <= val * (1 + 1e-6) + 1e-12
        assert g["primal"] == pytest.approx(obj, rel=1e-10)
    for c in ctxs:
        c.close()


def test_grouped_error_paths():
    import paper_2601_02826_amd as pq
    ctxs, ys, taus, lams, _ = _build("i8")
    # one bad problem: its own status, the others still solved
    bad_taus = list(taus)
    bad_taus[2] = 1.5
    res, sts = pq.solve_grouped(ctxs, ys, bad_taus, lams, check=False)
    assert sts[2] == pq.PQR_ERR_INVALID_ARG
    assert all(sts[i] == pq.PQR_OK and res[i]["rel_gap"] <= 1e-6 for i in range(len(ctxs)) if i != 2)
    # the same context twice
    with pytest.raises(pq.PQRError) as e:
        pq.solve_grouped([ctxs[0], ctxs[0]], [ys[0], ys[0]], [0.5, 0.5], [lams[0], lams[0]])
    assert e.value.status == pq.PQR_ERR_INVALID_ARG
    # mixed store formats
    X, y = H.genotype_problem(300, 100, seed=99)
    other = pq.Context.from_tensor(H.to_device_cols(X.astype(np.uint8), np.uint8), store_fmt="bf16",
                                   G=2)
    with pytest.raises(pq.PQRError) as e:
        pq.solve_grouped([ctxs[0], other], [ys[0], y], [0.5, 0.5], [lams[0], 0.1])
    assert e.value.status == pq.PQR_ERR_UNSUPPORTED
    other.close()
    for c in ctxs:
        c.close()
