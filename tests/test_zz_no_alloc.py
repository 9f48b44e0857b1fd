"""The allocation-free gradient entry point (pqr_mlp_grad_noalloc) against the
workspace entry point (pqr_mlp_grad) and the FP64 oracle: two calls in a row, the
second with a smaller batch, each equal to pqr_mlp_grad bit for bit (same kernels,
same fixed reduction order); sizes beyond the scratch are refused."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _bf16(a):
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _case(B, seed):
    rng = np.random.default_rng(seed)
    P = omlp.flatten(omlp.init_params(seed, scale=1.0)).astype(np.float32)
    F = rng.standard_normal((B, 4)).astype(np.float32)
    t = (rng.standard_normal(B) * 0.1).astype(np.float32)
    a = (rng.random(B) < 0.2).astype(np.float32)
    return P, F, t, a


def test_noalloc_gradient_equals_workspace_gradient():
    import torch
    import paper_2601_02826_amd as pq
    for B, seed in ((pq.MLP_NOALLOC_MAX_ROWS, 71), (1037, 72)):
        P, F, t, a = _case(B, seed)
        Pd, Fd = torch.from_numpy(P).cuda(), torch.from_numpy(F).cuda()
        td, ad = torch.from_numpy(t).cuda(), torch.from_numpy(a).cuda()
        g_ref = torch.empty_like(Pd)
        l_ref = torch.empty(1, dtype=torch.float32, device="cuda")
        ws = torch.empty(pq.mlp_workspace_bytes(B), dtype=torch.uint8, device="cuda")
        pq.mlp_grad(Pd, Fd, td, ad, ws, g_ref, l_ref, w_reg=3.0, w_pos=2.0)
        g = torch.full_like(Pd, float("nan"))
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        pq.mlp_grad_noalloc(Pd, Fd, td, ad, g, loss, w_reg=3.0, w_pos=2.0)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), B
        assert torch.equal(loss, l_ref), B
        # and the oracle's FP64 gradient at the BF16 parameters
        prm = omlp.unflatten(_bf16(P))
        gw = omlp.flatten(omlp.backward(prm, F.astype(np.float64), t, a, w_reg=3.0, w_pos=2.0))
        assert np.max(np.abs(g.cpu().numpy() - gw)) <= 1e-4 * np.max(np.abs(gw)), B


def test_noalloc_gradient_refuses_batches_beyond_its_scratch():
    import torch
    import paper_2601_02826_amd as pq
    B = pq.MLP_NOALLOC_MAX_ROWS + 1
    P, F, t, a = _case(B, 73)
    Pd, Fd = torch.from_numpy(P).cuda(), torch.from_numpy(F).cuda()
    g = torch.empty_like(Pd)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    with pytest.raises(pq.PQRError) as e:
        pq.mlp_grad_noalloc(Pd, Fd, torch.from_numpy(t).cuda(), torch.from_numpy(a).cuda(), g, loss)
    assert e.value.status == pq.PQR_ERR_UNSUPPORTED and "maximum" in str(e.value)
