"""Shared helpers of the GPU tests: seeded problems and device upload."""
import numpy as np

from datagen.configs import GaussianSpec, GenotypeSpec, make_gaussian, make_genotype
from oracle import pqr


def gaussian_problem(n, p, seed, tau=0.5, nnz=5):
    d = make_gaussian(GaussianSpec(n=n, p=p, nnz=nnz, seed=seed, tag=1, tau=tau))
    return d["X"], d["y"]


def genotype_problem(n, p, seed, tau=0.5, n_causal=10):
    g = make_genotype(GenotypeSpec(n=n, p=p, n_causal=n_causal, seed=seed, tag=2, tau=tau))
    return g["X"], g["y"]


def to_device_cols(X, dtype=None):
    """Column-major device copy: a (p, n) CUDA tensor whose row j is column j."""
    import torch
    A = np.ascontiguousarray(np.asarray(X).T)
    if dtype is not None:
        A = A.astype(dtype)
    return torch.from_numpy(A).to("cuda:0")


def oracle_design(X, standardize):
    """The oracle's X1 (intercept first) for the same stored values."""
    Xf = np.asarray(X, dtype=np.float64)
    if standardize:
        Xt, m, s = pqr.standardize(Xf)
        return pqr.with_intercept(Xt), m, s
    return pqr.with_intercept(Xf), None, None


def oracle_blocks(p, G, intercept_block=True):
    return pqr.partition(p, G, align=16, intercept_block=intercept_block)


def lam_vector(p, lam, weights=None):
    v = np.full(p + 1, float(lam)) if weights is None else float(lam) * np.asarray(weights, float)
    v[0] = 0.0
    return v


def random_state(n, p, seed, scale_beta=0.05, sparsity=0.05):
    rng = np.random.default_rng(seed)
    beta = np.zeros(p + 1)
    nz = rng.random(p) < sparsity
    beta[1:][nz] = rng.standard_normal(nz.sum()) * scale_beta
    beta[0] = 0.3
    z = rng.standard_normal(n) * 0.5
    theta = (rng.random(n) - 0.5) / n
    return beta, z, theta


def host_pass(spec, thr, T, B=None, chunk=2048, workers=None):
    """One FP64 pass over every column of the generated genotype design on the host:
    the columns come from the host twin of the generator and are standardized by the
    oracle (pqr.standardize, column by column), then V = X~^T T (p x K) and, with B
    (p x K coefficients on the standardized scale), F = X~ B (n x K).  Chunks run in
    a thread pool; F sums the chunks in column order (deterministic)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    from datagen import native
    n, p = spec.n, spec.p
    T = np.ascontiguousarray(T, dtype=np.float64)
    K = T.shape[1]
    if workers is None:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    V = np.zeros((p, K))

    def work(j0):
        j1 = min(p, j0 + chunk)
        X = native.genotype_host(n, j1 - j0, thr[j0:j1], spec.seed, spec.tag, j0=j0)
        Xt, _, _ = pqr.standardize(X.astype(np.float64))
        V[j0:j1] = Xt.T @ T
        if B is None:
            return None
        Bc = B[j0:j1]
        nz = np.nonzero(np.any(Bc != 0, axis=1))[0]
        return Xt[:, nz] @ Bc[nz] if len(nz) else None

    F = np.zeros((n, B.shape[1])) if B is not None else None
    with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
        for part in ex.map(work, range(0, p, chunk)):
            if part is not None:
                F += part
    return V, F
