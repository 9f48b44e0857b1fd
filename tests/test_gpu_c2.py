"""The single-lambda genotype configuration (n = 5,000, p = 100,000 int8 dosages, 50
causal variants, heteroscedastic t3 noise, tau = 0.9, lambda = 0.1 lambda_max, 48
blocks): one FS-QRPPA solve on the GPU, its certificate recomputed by the oracle over
every column from the regenerated design."""
import numpy as np
import pytest

from datagen.configs import SPECS, make_genotype
from oracle import pqr
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_c2_solve_certified_over_all_columns():
    import torch
    import paper_2601_02826_amd as pq
    from datagen import native
    spec = SPECS["geno_5000x100k"]
    n, p, tau = spec.n, spec.p, spec.tau
    g = make_genotype(spec, with_X=False)
    thr = torch.from_numpy(g["thr"].astype(np.int64)).to(torch.int32).cuda()
    Xc = torch.empty((p, n), dtype=torch.uint8, device="cuda")
    native.genotype_device(Xc.data_ptr(), n, n, p, thr.data_ptr(), spec.seed, spec.tag,
                           torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ctx = pq.Context.from_tensor(Xc, store_fmt="i8", standardize=True, G=spec.G, tol_gap=1e-3,
                                 cert_every=100, max_iter=200_000)
    y = g["y"]
    lmax, score = ctx.lambda_max(y, tau, score=True)
    lam = spec.lam_frac * lmax
    r = ctx.solve(y, tau, lam)
    print(f"C2: {r['iters']} iterations, gap {r['rel_gap']:.2e}, nnz {r['nnz']}", flush=True)
    assert r["rel_gap"] <= 1e-3
    # the oracle's certificate of the returned point over all p columns
    tp = pqr.project_box_sum(r["theta"], (tau - 1) / n, tau / n)
    _, psi = pqr.null_dual(y, tau)
    B = r["beta_std"][1:, None]
    V, F = H.host_pass(spec, g["thr"], np.column_stack([tp, psi / n]), B)
    # lambda_max is the null-fit score's maximum (its definition), over every column
    assert lmax == pytest.approx(np.max(np.abs(V[:, 1])), rel=1e-12)
    assert np.allclose(score, V[:, 1], rtol=1e-10, atol=1e-15)
    dual = pqr.dual_value(y, tp, np.max(np.abs(V[:, 0])) / lam)
    primal = pqr._sum(pqr.pinball(y - r["beta_std"][0] - F[:, 0], tau)) / n + \
        lam * pqr._sum(np.abs(B[:, 0]))
    assert r["primal"] == pytest.approx(primal, rel=1e-10)
    assert r["dual"] == pytest.approx(dual, rel=1e-9)
    assert r["rel_gap"] == pytest.approx((primal - dual) / primal, rel=1e-5, abs=1e-12)
    ctx.close()
