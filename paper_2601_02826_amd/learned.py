"""Training of the per-feature scoring network behind the learned warm start.

Rows are columns of solved problems: the features of pqr_features (score
z-statistic, m_j / 2, tau, log(lambda / lambda_max)) with targets t_j =
beta~_j / sd(y) and a_j = 1{beta~_j != 0} from FS-QRPPA solutions computed by
this library on seeded synthetic problems.  Every forward, backward and
optimiser step runs in the library's kernels (pqr_mlp_grad, pqr_mlp_adam);
torch only holds device buffers and selects training rows.
"""
import numpy as np

from . import _lib as L

SHAPES = [(64, 4), (64,), (64, 64), (64,), (2, 64), (2,)]


def init_params(seed=0):
    """Parameters as a flat CUDA float32 tensor (4610): weights N(0, 1/fan_in), biases 0."""
    import torch
    rng = np.random.default_rng(seed)
    parts = []
    for shp in SHAPES:
        if len(shp) == 2:
            parts.append(rng.standard_normal(shp).ravel() / np.sqrt(shp[1]))
        else:
            parts.append(np.zeros(shp))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == L.mlp_param_count()
    return torch.from_numpy(flat).cuda()


def collect_rows(ctx, y, tau, lams, neg_ratio=4, neg_min=256, seed=0, rates=None):
    """Solve the lambda path on ctx (warm starts on the device) and return the
    feature / target rows of every solved point: all active columns plus a random
    sample of inactive ones.  With `rates` (a list), the fraction of inactive columns
    kept at every point is appended to it (for prior_threshold)."""
    import torch
    rng = np.random.default_rng(seed)
    sd = float(np.std(y))
    feats = torch.empty((ctx.p, 4), dtype=torch.float32, device="cuda")
    F, T, A = [], [], []
    for k, lam in enumerate(lams):
        r = ctx.solve(y, tau, lam, start="zero" if k == 0 else "device", allow_not_converged=True)
        ctx.features(y, tau, lam, feats.data_ptr())
        torch.cuda.synchronize()
        b = r["beta_std"][1:] / sd
        act = b != 0
        ia = np.nonzero(act)[0]
        ii = np.nonzero(~act)[0]
        take = min(len(ii), max(neg_min, neg_ratio * len(ia)))
        if rates is not None and len(ii):
            rates.append(take / len(ii))
        idx = np.concatenate([ia, rng.choice(ii, take, replace=False)]) if take else ia
        it = torch.from_numpy(idx.astype(np.int64)).cuda()
        F.append(feats.index_select(0, it))
        T.append(torch.from_numpy(b[idx].astype(np.float32)).cuda())
        A.append(torch.from_numpy(act[idx].astype(np.float32)).cuda())
    return torch.cat(F), torch.cat(T), torch.cat(A)


def prior_threshold(rates, w_pos=2.0):
    """Logit threshold that undoes the training rows' class balance: inactive columns
    were kept at rate r and active ones weighted by w_pos, so the network's odds are
    those of the population times w_pos / r; the proposal A = {logit > log(w_pos) -
    mean(log r)} is then the set of columns more likely active than not."""
    return float(np.log(w_pos) - np.mean(np.log(np.asarray(rates, dtype=np.float64))))


def train(params, F, T, A, steps=500, batch=2048, lr=3e-3, w_reg=100.0, w_pos=2.0, seed=0,
          log_every=0):
    """Adam on mini-batches of the rows; returns the loss of every step."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    B = min(batch, F.shape[0])
    ws = torch.empty(L.mlp_workspace_bytes(B), dtype=torch.uint8, device="cuda")
    losses = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, F.shape[0], (B,), generator=g, device="cuda")
        Fb = F.index_select(0, idx).contiguous()
        Tb = T.index_select(0, idx).contiguous()
        Ab = A.index_select(0, idx).contiguous()
        L.mlp_grad(params, Fb, Tb, Ab, ws, grad, loss, w_reg, w_pos)
        L.mlp_adam(params, grad, m, v, step, lr)
        losses.append(float(loss.item()) if (log_every and step % log_every == 0) or step == steps
                      or step == 1 else None)
    return [x for x in losses if x is not None]
