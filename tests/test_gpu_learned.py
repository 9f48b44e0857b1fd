"""The learned warm start: network kernels against the FP64 oracle of oracle/mlp.py,
and the proposal + reduced solve + full KKT check against the plain solver."""
import numpy as np
import pytest

from oracle import mlp as omlp
from oracle import lp, pqr
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _bf16(a):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _random_case(B, seed):
    rng = np.random.default_rng(seed)
    P = omlp.flatten(omlp.init_params(seed, scale=1.0)).astype(np.float32)
    P[omlp.n_params() - 2:] = rng.standard_normal(2).astype(np.float32) * 0.1
    F = rng.standard_normal((B, 4)).astype(np.float32)
    t = (rng.standard_normal(B) * 0.1).astype(np.float32)
    a = (rng.random(B) < 0.2).astype(np.float32)
    return P, F, t, a


@pytest.mark.parametrize("B", [1, 200, 1037])
def test_mlp_forward_and_gradient_vs_oracle(B):
    import torch
    import paper_2601_02826_amd as pq
    P, F, t, a = _random_case(B, seed=B)
    Pd, Fd = torch.from_numpy(P).cuda(), torch.from_numpy(F).cuda()
    out = torch.empty((B, 2), dtype=torch.float32, device="cuda")
    pq.mlp_forward(Pd, Fd, out)
    # the oracle at the BF16-rounded parameters, FP64
    prm = omlp.unflatten(_bf16(P))
    want, _ = omlp.forward(prm, F.astype(np.float64))
    got = out.cpu().numpy()
    assert np.allclose(got, want, rtol=2e-5, atol=2e-5)
    grad = torch.empty_like(Pd)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ws = torch.empty(pq.mlp_workspace_bytes(B), dtype=torch.uint8, device="cuda")
    pq.mlp_grad(Pd, Fd, torch.from_numpy(t).cuda(), torch.from_numpy(a).cuda(), ws, grad, loss,
                w_reg=3.0, w_pos=2.0)
    gw = omlp.flatten(omlp.backward(prm, F.astype(np.float64), t, a, w_reg=3.0, w_pos=2.0))
    lw = omlp.loss(prm, F.astype(np.float64), t, a, w_reg=3.0, w_pos=2.0)
    g = grad.cpu().numpy()
    scale = np.max(np.abs(gw))
    assert np.max(np.abs(g - gw)) <= 1e-4 * scale
    assert float(loss.item()) == pytest.approx(lw, rel=1e-5)


def test_adam_step():
    import torch
    import paper_2601_02826_amd as pq
    rng = np.random.default_rng(5)
    n = pq.mlp_param_count()
    P = rng.standard_normal(n).astype(np.float32)
    G = rng.standard_normal(n).astype(np.float32)
    M = rng.standard_normal(n).astype(np.float32) * 0.1
    V = np.abs(rng.standard_normal(n)).astype(np.float32) * 0.1
    Pd, Gd, Md, Vd = (torch.from_numpy(x.copy()).cuda() for x in (P, G, M, V))
    pq.mlp_adam(Pd, Gd, Md, Vd, 3, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8)
    m = 0.9 * M + 0.1 * G
    v = 0.99 * V + 0.01 * G * G
    want = P - 1e-2 * (m / (1 - 0.9 ** 3)) / (np.sqrt(v / (1 - 0.99 ** 3)) + 1e-8)
    assert np.allclose(Pd.cpu().numpy(), want, rtol=1e-5, atol=1e-6)


def test_learned_warm_start_end_to_end():
    """Train on a few solved problems, then solve a held-out problem: the answer is
    certified on the full design, equals the LP optimum, and the reduced solve needs
    far fewer X-passes than the plain solve."""
    import torch
    import paper_2601_02826_amd as pq
    from paper_2601_02826_amd import learned
    n, p, G = 1500, 5000, 4
    F_all, T_all, A_all = [], [], []
    rates = []
    for seed in (41, 42, 43, 44):
        X, y = H.genotype_problem(n, p, seed=seed, n_causal=10)
        ctx = pq.Context.from_tensor(H.to_device_cols(X, np.uint8), store_fmt="i8", G=G,
                                     tol_gap=1e-4, cert_every=100, max_iter=100_000)
        for tau in (0.3, 0.6):
            lm = ctx.lambda_max(y, tau)
            Fp, Tp, Ap = learned.collect_rows(ctx, y, tau, [0.7 * lm, 0.55 * lm, 0.45 * lm],
                                              seed=seed, rates=rates)
            F_all.append(Fp); T_all.append(Tp); A_all.append(Ap)
        ctx.close()
    F, T, A = torch.cat(F_all), torch.cat(T_all), torch.cat(A_all)
    params = learned.init_params(0)
    losses = learned.train(params, F, T, A, steps=400, batch=2048, lr=3e-3, log_every=100)
    assert losses[-1] < 0.5 * losses[0]
    # held-out problem
    X, y = H.genotype_problem(n, p, seed=77, n_causal=10)
    X1, _, _ = H.oracle_design(X, True)
    tau = 0.5
    tol = 1e-4
    ctx = pq.Context.from_tensor(H.to_device_cols(X, np.uint8), store_fmt="i8", G=G,
                                 tol_gap=tol, cert_every=100, max_iter=400_000)
    lam = 0.5 * ctx.lambda_max(y, tau)
    plain = ctx.solve(y, tau, lam)
    # inactive rows were subsampled, so the raw logits overstate activity; the corrected
    # threshold is what the benchmark uses at full size.  Trained on four small problems
    # the network is too cautious after that correction (a 32-column start that needs
    # five rounds here), so this test proposes with the raw logits.
    assert learned.prior_threshold(rates) > 0
    lrn = ctx.solve_learned(y, tau, lam, params.data_ptr(), threshold=0.0, max_rounds=8)
    val, _ = lp.highs(X1, y, tau, H.lam_vector(p, lam))
    p_l = pqr.objective(X1, y, lrn["beta_std"], tau, H.lam_vector(p, lam))
    print({k: lrn[k] for k in ("rounds", "fallback", "active_initial", "active_final",
                               "reduced_iters", "rel_gap", "iters")}, "plain nnz", plain["nnz"])
    assert lrn["rel_gap"] <= tol and lrn["fallback"] == 0
    assert val * (1 - 1e-12) <= p_l <= val * (1 + tol) + 1e-12
    passes_plain = plain["iters"]
    passes_learned = lrn["reduced_iters"] * lrn["active_final"] / p + 2 * lrn["rounds"] + 1
    print(f"plain: {plain['iters']} iterations, {plain['seconds']:.3f}s; learned: |A| "
          f"{lrn['active_initial']}->{lrn['active_final']}, {lrn['rounds']} rounds, "
          f"{lrn['reduced_iters']} reduced iterations, {lrn['seconds']:.3f}s; X-passes "
          f"{passes_plain} vs {passes_learned:.1f}")
    assert passes_learned < 0.5 * passes_plain
    # the same rounds with non-learned proposals: the strong rule at the network's |A|
    # budget (reported: the two are close on these designs), and a useless network
    # (no column proposed: only the 32 forced columns, zero coefficients), which needs
    # more X-passes than the trained one
    scr = ctx.solve_screened(y, tau, lam, budget=lrn["active_initial"], max_rounds=8)
    passes_screened = scr["reduced_iters"] * scr["active_final"] / p + 2 * scr["rounds"] + 1
    assert scr["rel_gap"] <= tol
    zero = torch.zeros_like(params)
    fb = ctx.solve_learned(y, tau, lam, zero.data_ptr(), threshold=0.0, max_rounds=1)
    passes_zero = (fb["iters"] if fb["fallback"] else
                   fb["reduced_iters"] * fb["active_final"] / p + 2 * fb["rounds"] + 1)
    print(f"strong rule at the same budget: {scr['rounds']} rounds, {passes_screened:.1f} X-passes; "
          f"zero network: fallback {fb['fallback']}, {passes_zero:.1f} X-passes")
    assert fb["rel_gap"] <= tol         # certified either by the reduced solve or the fallback
    assert passes_learned < passes_zero
    ctx.close()
