"""Parity at the benchmark's full size (n = 20,000, p = 1,000,000 int8 dosages, 12
feature blocks), on outputs the oracle can compute column by column: the null-fit
scores, one Algorithm 1 step on sampled columns, and the objective and dual
feasibility of a solved point."""
import numpy as np
import pytest

from datagen.configs import SPECS, genotype_columns, make_genotype
from oracle import pqr

pytestmark = pytest.mark.gpu

N, P, G = 20_000, 1_000_000, 12


@pytest.fixture(scope="module")
def full():
    import torch
    import paper_2601_02826_amd as pq
    from datagen import native
    spec = SPECS["geno_20kx1M"]
    assert (spec.n, spec.p) == (N, P)
    g = make_genotype(spec, with_X=False)
    thr = torch.from_numpy(g["thr"].astype(np.int64)).to(torch.int32).cuda()
    Xc = torch.empty((P, N), dtype=torch.uint8, device="cuda")
    native.genotype_device(Xc.data_ptr(), N, N, P, thr.data_ptr(), spec.seed, spec.tag,
                           torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ctx = pq.Context.from_tensor(Xc, store_fmt="i8", standardize=True, G=G, tol_gap=1e-3,
                                 cert_every=50, max_iter=20000)
    ctx._keep = None
    del Xc
    torch.cuda.empty_cache()
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(P, 400, replace=False))
    yield spec, g, ctx, sample
    ctx.close()


def _std_cols(spec, cols):
    """Oracle standardization of the given columns from their own exact statistics."""
    X = genotype_columns(spec, cols).astype(np.float64)
    Xt, m, s = pqr.standardize(X)
    return Xt


def test_device_generator_matches_host_definition(full):
    import torch
    from datagen import native
    spec, g, ctx, sample = full
    cols = sample[:32]
    thr = torch.from_numpy(g["thr"][cols].astype(np.int64)).to(torch.int32).cuda()
    out = torch.empty((len(cols), N), dtype=torch.uint8, device="cuda")
    for k, j in enumerate(cols):   # one column at a time through the device twin
        native.genotype_device(out[k].data_ptr(), N, N, 1, thr[k:k + 1].data_ptr(), spec.seed,
                               spec.tag, torch.cuda.current_stream().cuda_stream, j0=int(j))
    torch.cuda.synchronize()
    want = genotype_columns(spec, cols)
    assert np.array_equal(out.cpu().numpy().T.astype(np.int8), want)


def test_scores_on_sampled_columns(full):
    spec, g, ctx, sample = full
    y = g["y"]
    lmax, score = ctx.lambda_max(y, 0.5, score=True)
    _, psi = pqr.null_dual(y, 0.5)
    Xt = _std_cols(spec, sample)
    want = Xt.T @ psi / N
    assert np.allclose(score[sample], want, rtol=1e-10, atol=1e-15)
    assert lmax >= np.max(np.abs(want)) * (1 - 1e-12)
    assert lmax == pytest.approx(np.max(np.abs(score)), rel=1e-14)


def test_one_step_on_sampled_columns(full):
    spec, g, ctx, sample = full
    y = g["y"]
    tau = 0.5
    lmax = ctx.lambda_max(y, tau)
    lam = 0.3 * lmax
    rng = np.random.default_rng(1)
    beta = np.zeros(P + 1)
    beta[0] = 0.2
    nzc = rng.choice(P, 50, replace=False)
    beta[1 + nzc] = rng.standard_normal(50) * 0.01
    z = rng.standard_normal(N) * 0.3
    theta = (rng.random(N) - 0.5) / N
    Gt, bounds, Lam = ctx.blocks()
    mu = 1e-5
    eta = 1.01 * mu * Lam
    b1, z1, t1 = ctx.iterate(y, tau, lam, mu, eta, 1, beta, z, theta)
    # z only depends on (z, theta): every row is checkable; FP32 rounds the prox
    # argument u = z + theta/mu and the thresholds, so the bound is a few FP32 ulps of
    # |z| + |theta/mu| + 1/(n mu)
    bound = 8 * np.finfo(np.float32).eps * (np.abs(z) + np.abs(theta / mu) + 1 / (N * mu))
    assert np.all(np.abs(z1 - pqr.z_prox(z, theta, tau, N, mu)) <= bound)
    # beta on sampled columns: v_j = x~_j^T theta from the oracle's columns
    Xt = _std_cols(spec, sample)
    v = Xt.T @ theta
    blk = np.searchsorted(bounds[1:], sample, side="right")    # feature block of each column
    eta_j = eta[blk]
    want = pqr.beta_prox(beta[1 + sample], v, np.full(len(sample), lam), eta_j)
    assert np.allclose(b1[1 + sample], want, rtol=1e-5, atol=1e-9)
    # intercept (its own block 0): beta0 + sum(theta) / eta_0
    assert b1[0] == pytest.approx(beta[0] + theta.sum() / eta[0], rel=1e-6)


def test_solved_point_objective_and_dual_feasibility(full):
    spec, g, ctx, sample = full
    y = g["y"]
    tau = 0.5
    lmax = ctx.lambda_max(y, tau)
    lam = 0.5 * lmax
    r = ctx.solve(y, tau, lam)
    assert r["rel_gap"] <= 1e-3
    support = np.nonzero(r["beta_std"][1:])[0]
    assert 0 < len(support) < 500
    Xs = _std_cols(spec, support)
    fit = r["beta_std"][0] + Xs @ r["beta_std"][1 + support]
    primal = np.mean(pqr.pinball(y - fit, tau)) + lam * np.abs(r["beta_std"][1 + support]).sum()
    assert r["primal"] == pytest.approx(primal, rel=1e-10)
    # dual side on the support and the sample: the projected theta's ratios never exceed
    # the device-wide maximum implied by the reported dual value
    tp = pqr.project_box_sum(r["theta"], (tau - 1) / N, tau / N)
    cols = np.union1d(support, sample)
    ratios = np.abs(_std_cols(spec, cols).T @ tp) / lam
    assert np.all(ratios <= 1.0 + 5e-2)
    assert np.max(ratios[np.isin(cols, support)]) > 0.9


def test_batched_path_objectives_and_dual_feasibility(full):
    """The benchmark's default launch configuration at full size (20 right-hand sides
    of one batched solve, padded to 32), on the sparse half of a path (lambda_max down
    to 0.2 lambda_max, where every point stays sparse): every point is certified, its
    reported objective is recomputed by the oracle from the support columns, and the
    projected dual point is feasible on sampled columns."""
    spec, g, ctx, sample = full
    y = g["y"]
    lmax = ctx.lambda_max(y, 0.5)
    lams = lmax * 0.2 ** (np.arange(20) / 19.0)
    res = ctx.solve_batch(y, np.full(20, 0.5), lams)
    print(f"batched: {res[0]['iters']} iterations, nnz {[r['nnz'] for r in res]}", flush=True)
    assert all(r["rel_gap"] <= 1e-3 for r in res)
    for k in range(20):
        r = res[k]
        support = np.nonzero(r["beta_std"][1:])[0]
        assert len(support) < 2000
        Xs = _std_cols(spec, support) if len(support) else np.zeros((N, 0))
        fit = r["beta_std"][0] + Xs @ r["beta_std"][1 + support]
        primal = (np.mean(pqr.pinball(y - fit, 0.5)) +
                  lams[k] * np.abs(r["beta_std"][1 + support]).sum())
        assert r["primal"] == pytest.approx(primal, rel=1e-9)
        tp = pqr.project_box_sum(r["theta"], -0.5 / N, 0.5 / N)
        ratios = np.abs(_std_cols(spec, sample).T @ tp) / lams[k]
        assert np.all(ratios <= 1.0 + 5e-2)


@pytest.fixture(scope="module")
def headline(full):
    """The benchmark's headline path (20 right-hand sides, lambda_max down to 0.01
    lambda_max, the dense end included) solved once at 1e-3 by the batched solver."""
    spec, g, ctx, sample = full
    y = g["y"]
    lmax = ctx.lambda_max(y, 0.5)
    lams = lmax * 0.01 ** (np.arange(20) / 19.0)
    res = ctx.solve_batch(y, np.full(20, 0.5), lams, allow_not_converged=True)
    print("gaps " + " ".join(f"{r['rel_gap']:.1e}" for r in res) + "; nnz " +
          " ".join(str(r["nnz"]) for r in res), flush=True)
    return dict(lams=lams, res=res, cache={})


def test_headline_path_is_certified(headline):
    res = headline["res"]
    assert all(r["rel_gap"] <= 1e-3 for r in res)
    assert res[-1]["nnz"] > 10_000   # the dense end of the path is part of the check


@pytest.mark.timeout(900)
def test_headline_path_certificates_over_all_columns(full, headline):
    """The headline path's certificates checked over ALL 1,000,000 columns by the
    oracle: one FP64 host pass over the regenerated design gives X~^T t_k for every
    returned dual point t_k (the batched reading's exactly representable point of the
    exported theta) and the fits X~ beta_k; the primal, dual and relative gap recomputed
    from them equal the device's."""
    from tests import helpers as H
    spec, g, ctx, sample = full
    y = g["y"]
    tau = 0.5
    lams, res = headline["lams"], headline["res"]
    pts = []
    for r in res:
        q = pqr.quantize_dual_point(r["theta"], tau, N)
        pts.append(q[0] if q is not None else pqr.project_box_sum(r["theta"], (tau - 1) / N, tau / N))
    Bm = np.column_stack([r["beta_std"][1:] for r in res])
    V, F = H.host_pass(spec, g["thr"], np.column_stack(pts), Bm)
    headline["cache"]["V"] = V
    for k, r in enumerate(res):
        lam_k = lams[k]
        dual = pqr.dual_value(y, pts[k], np.max(np.abs(V[:, k])) / lam_k)
        fit = r["beta_std"][0] + F[:, k]
        primal = pqr._sum(pqr.pinball(y - fit, tau)) / N + lam_k * pqr._sum(np.abs(Bm[:, k]))
        gap = (primal - dual) / primal
        assert r["primal"] == pytest.approx(primal, rel=1e-10), (k, r["primal"], primal)
        assert r["dual"] == pytest.approx(dual, rel=1e-9), (k, r["dual"], dual)
        assert r["rel_gap"] == pytest.approx(gap, rel=1e-5, abs=1e-12), (k, r["rel_gap"], gap)


@pytest.mark.timeout(900)
def test_headline_sparse_points_are_global_optima(full, headline):
    """For the sparse points of the headline path the global optimum itself is certified
    (Prop. 1, the restricted-solve certificate): the LP restricted to the GPU's support
    plus every column within 1 % of its dual bound is solved by HiGHS, a second full
    host pass shows |x~_j^T theta_A| <= lambda (1 + 1e-9) off that set, and the GPU's
    objective lies between that optimum and its certified gap above it."""
    from oracle import lp
    from tests import helpers as H
    spec, g, ctx, sample = full
    y = g["y"]
    tau = 0.5
    lams, res = headline["lams"], headline["res"]
    if "V" not in headline["cache"]:
        pytest.skip("needs the all-column pass of the previous test")
    V = headline["cache"]["V"]
    checked = []
    for k, r in enumerate(res):
        A = np.union1d(np.nonzero(r["beta_std"][1:])[0], np.nonzero(np.abs(V[:, k]) >= 0.99 * lams[k])[0])
        if len(A) > 300:
            continue
        XA = pqr.with_intercept(_std_cols(spec, A)) if len(A) else np.ones((N, 1))
        val, bA, thA = lp.highs_with_duals(XA, y, tau, H.lam_vector(len(A), lams[k]))
        checked.append((k, A, val, thA))
    assert len(checked) >= 3
    V2, _ = H.host_pass(spec, g["thr"], np.column_stack([c[3] for c in checked]))
    for q, (k, A, val, thA) in enumerate(checked):
        off = np.ones(P, dtype=bool)
        off[A] = False
        worst = np.max(np.abs(V2[off, q])) / lams[k]
        print(f"point {k}: |A| = {len(A)}, optimum {val:.12g}, GPU {res[k]['primal']:.12g}, "
              f"max ratio off A {worst:.9f}", flush=True)
        assert worst <= 1.0 + 1e-9, (k, worst)
        assert val * (1 - 1e-9) <= res[k]["primal"] <= val + res[k]["rel_gap"] * res[k]["primal"] * (1 + 1e-6)
        assert res[k]["dual"] <= val * (1 + 1e-9)
