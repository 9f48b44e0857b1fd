"""Batched right-hand sides on the int8 matrix cores: every (tau_k, lambda_k) reaches
its certified gap and agrees with the LP optimum of its own problem; the certified
dual (an exactly representable dual point, products exact in integers) never
exceeds that optimum."""
import numpy as np
import pytest

from oracle import lp, pqr
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _ctx(X, **kw):
    import paper_2601_02826_amd as pq
    return pq.Context.from_tensor(H.to_device_cols(X, np.uint8), store_fmt="i8", standardize=True,
                                  rows_per_lane=16, **kw)


# K = 5, 16: one 16-wide tile; 21: two; 40: three (two wavefronts per group set in the
# back-product); 128: eight (four per group set).  The LP check runs on `checked` of them.
@pytest.mark.parametrize("K,checked", [(5, 5), (16, 16), (21, 21), (40, 8), (128, 4)])
def test_batch_matches_lp_optimum(K, checked):
    n, p, G = 1500, 700, 3          # n pads to 2048 rows, p to 704 columns
    X, y = H.genotype_problem(n, p, seed=31)
    X1, _, _ = H.oracle_design(X, True)
    ctx = _ctx(X, G=G, tol_gap=1e-5, cert_every=200, max_iter=400_000)
    taus = np.resize(np.array([0.2, 0.5, 0.8]), K)
    fr = np.resize(np.array([0.9, 0.6, 0.4, 0.3, 0.25, 0.2, 0.5, 0.7]), K)
    lams = np.array([f * pqr.lambda_max(X1, y, t) for f, t in zip(fr, taus)])
    res = ctx.solve_batch(y, taus, lams)
    assert all(r["rel_gap"] <= 1e-5 for r in res)
    for k in np.linspace(0, K - 1, checked).astype(int):
        lam_vec = H.lam_vector(p, lams[k])
        val, _ = lp.highs(X1, y, taus[k], lam_vec)
        p_gpu = pqr.objective(X1, y, res[k]["beta_std"], taus[k], lam_vec)
        assert res[k]["rel_gap"] <= 1e-5, (k, res[k]["rel_gap"])
        assert val * (1 - 1e-12) <= p_gpu <= val * (1 + 1e-5) + 1e-12, (k, p_gpu, val)
        assert res[k]["primal"] == pytest.approx(p_gpu, rel=1e-10)
        # the certificate's dual point is feasible: its objective cannot pass the optimum
        assert res[k]["dual"] <= val + 1e-10 * abs(val), (k, res[k]["dual"], val)
        # and it loses no more than its quantisation (2^-27 of the box per entry) against
        # the oracle's FP64 certificate of the returned (certified) iterate
        ref = pqr.dual_certificate(X1, y, taus[k], lam_vec, res[k]["beta_std"], res[k]["theta"])
        assert res[k]["dual"] >= ref["dual"] - 1e-6 * abs(ref["dual"]), (k, res[k]["dual"], ref["dual"])
        # the oracle of the same reading (quantised point, exact zero sum) agrees to
        # rounding: the device's dual is the best of its rounds, the last one at least
        qref = pqr.quantized_dual_certificate(X1, y, taus[k], lam_vec, res[k]["beta_std"],
                                              res[k]["theta"])
        assert qref is not None
        assert res[k]["dual"] >= qref["dual"] - 1e-9 * abs(qref["dual"]), (k, res[k]["dual"], qref["dual"])
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
    # int8 codes above 127 (read as signed by the matrix cores) are refused
    X2 = X.astype(np.int64)
    X2[5, 3] = 200
    ctx = pq.Context.from_tensor(H.to_device_cols(X2.astype(np.uint8), np.uint8), store_fmt="i8",
                                 G=2, rows_per_lane=16)
    with pytest.raises(pq.PQRError) as e:
        ctx.solve_batch(y, [0.5], [0.1])
    assert e.value.status == pq.PQR_ERR_UNSUPPORTED and "127" in str(e.value)
    ctx.close()


def test_batch_rejects_sizes_beyond_exact_integer_range():
    """The int32 matrix-core sums stay exact only while n_pad * max_code * 65 < 2^31,
    and the digit buffers are addressed with 32-bit offsets (512 n_pad < 2^31): larger
    designs are refused before any batched work."""
    import torch
    import paper_2601_02826_amd as pq
    rng = np.random.default_rng(33)
    # n = 270,000 rows with one code 127: 271,360 * 127 * 65 > 2^31
    n, p = 270_000, 16
    Xc = torch.from_numpy(rng.integers(0, 3, size=(p, n), dtype=np.uint8)).to("cuda:0")
    Xc[3, 17] = 127
    y = rng.standard_normal(n)
    ctx = pq.Context.from_tensor(Xc, store_fmt="i8", G=1, rows_per_lane=16)
    with pytest.raises(pq.PQRError) as e:
        ctx.solve_batch(y, [0.5], [0.1])
    assert e.value.status == pq.PQR_ERR_UNSUPPORTED and "2^31" in str(e.value)
    ctx.close()
    del Xc
    # n_pad = 4,195,328 rows of dosages 0..2: 512 n_pad > 2^31
    n = 4_194_305
    Xc = torch.from_numpy(rng.integers(0, 3, size=(p, n), dtype=np.uint8)).to("cuda:0")
    y = rng.standard_normal(n)
    ctx = pq.Context.from_tensor(Xc, store_fmt="i8", G=1, rows_per_lane=16)
    with pytest.raises(pq.PQRError) as e:
        ctx.solve_batch(y, [0.5], [0.1])
    assert e.value.status == pq.PQR_ERR_UNSUPPORTED and "2^31" in str(e.value)
    ctx.close()


@pytest.mark.parametrize("K", [21, 128])
def test_every_launch_variant_gives_identical_iterates(K):
    """The autotuner picks among launch variants of the back-product and the union
    product; each computes the same exact integer sums, so 300 iterations under every
    forced combination equal the default bit for bit, and the tuner's own choice (and
    the candidate times it measured) are reported."""
    import paper_2601_02826_amd as pq
    n, p, G = 1500, 700, 3
    X, y = H.genotype_problem(n, p, seed=31)
    X1, _, _ = H.oracle_design(X, True)
    taus = np.resize(np.array([0.2, 0.5, 0.8]), K)
    fr = np.resize(np.array([0.9, 0.6, 0.4, 0.3, 0.25, 0.2, 0.5, 0.7]), K)
    lams = np.array([f * pqr.lambda_max(X1, y, t) for f, t in zip(fr, taus)])
    ref = None
    for o in [1 + pq.TILE_VARIANTS * bv + av for bv in range(pq.BGEMM_VARIANTS)
              for av in range(pq.BAXPY_VARIANTS)]:
        ctx = _ctx(X, G=G, tol_gap=1e-12, cert_every=100, max_iter=300, tile_override=o)
        res = ctx.solve_batch(y, taus, lams, allow_not_converged=True)
        B = np.stack([r["beta_std"] for r in res])
        Th = np.stack([r["theta"] for r in res])
        if ref is None:
            ref = (B, Th)
        else:
            assert np.array_equal(B, ref[0]) and np.array_equal(Th, ref[1]), o
        ctx.close()
    ctx = _ctx(X, G=G, tol_gap=1e-12, cert_every=100, max_iter=300)
    res = ctx.solve_batch(y, taus, lams, allow_not_converged=True)
    assert np.array_equal(np.stack([r["beta_std"] for r in res]), ref[0])
    t = ctx.batch_tiles(K)
    print(f"K={K}: tuner chose back-product {t['bgemm_variant']} {t['bgemm_ms']}, union product "
          f"{t['baxpy_variant']} {t['baxpy_ms']}")
    assert len(t["bgemm_ms"]) == pq.BGEMM_VARIANTS and len(t["baxpy_ms"]) == pq.BAXPY_VARIANTS
    assert t["bgemm_ms"][t["bgemm_variant"]] == min(t["bgemm_ms"])
    # the union product is timed once its union holds 1024 columns (never at p = 700)
    assert t["baxpy_variant"] == -1 and t["union_cols"] == 0
    ctx.close()
