"""Seeded synthetic workloads: Gaussian designs and genotype-like dosage matrices.

Counter layout (every draw is one Philox4x32-10 call, key = (seed, tag)):

    stream 1  MAF of column j          counter (j, 0, 1, 0), word 0
    stream 2  genotype entry (i, j)    counter (i, j, 2, 0), words 0 and 1
    stream 3  causal-column priority   counter (j, 0, 3, 0), word 0
    stream 4  causal effect k          counter (k, 0, 4, 0), words 0 and 1
    stream 5  noise of row i           counter (i, 0, 5, 0), words 0..3
    stream 6  Gaussian entry (i, j)    counter (i, j, 6, 0), words 0 and 1
    stream 7  Gaussian-design truth    counter (j, 0, 7, 0), words 0..2
    stream 8  grouped problem i shape  counter (i, 0, 8, 0), words 0..2
    stream 9  AR(1) innovation (i, j)  counter (i, j, 9, 0), words 0 and 1
    stream 10 AR(1)-design noise of i  counter (i, 0, 10, 0), words 0 and 1

A genotype entry is the sum of two Bernoulli(MAF_j) draws, x = [w0 < T_j] +
[w1 < T_j], with the integer threshold T_j = floor(MAF_j * 2^32).  Because the
decision is an unsigned integer comparison, a device twin of this generator
reproduces every byte exactly.  Column indices here are 0-based over the p
feature columns; the intercept is not part of the stored matrix.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .philox import philox4x32, uniform01

TWO32 = 4294967296.0


def _normals_from_words(w0, w1):
    """Box-Muller on two uint32 words: returns (cos branch, sin branch)."""
    u1 = uniform01(w0)
    u2 = uniform01(w1)
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * math.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def _t3_noise(seed, tag, rows):
    """Student-t with 3 degrees of freedom, one value per row (stream 5)."""
    w = philox4x32(rows, 0, 5, 0, seed, tag)
    z1, z2 = _normals_from_words(w[0], w[1])
    z3, z4 = _normals_from_words(w[2], w[3])
    chi2 = z2 * z2 + z3 * z3 + z4 * z4
    return z1 / np.sqrt(chi2 / 3.0)


@dataclass(frozen=True)
class GaussianSpec:
    """iid N(0,1) design with a sparse truth and t3 noise."""
    n: int = 200
    p: int = 2000
    nnz: int = 10
    seed: int = 1
    tag: int = 1
    tau: float = 0.5
    lam_frac: float = 0.1
    G: int = 5


@dataclass(frozen=True)
class GenotypeSpec:
    """Dosage matrix x_ij ~ Binomial(2, MAF_j), MAF_j ~ U(0.05, 0.5)."""
    n: int = 5000
    p: int = 100_000
    n_causal: int = 50
    effect_sd: float = 0.2
    seed: int = 2
    tag: int = 2
    tau: float = 0.9
    lam_frac: float = 0.1
    G: int = 48
    maf_lo: float = 0.05
    maf_hi: float = 0.5
    hetero: float = 0.5


def make_gaussian(spec: GaussianSpec):
    """Return dict(X (n x p float64, no intercept), y, beta_star (p+1), support)."""
    n, p = spec.n, spec.p
    rows = np.arange(n, dtype=np.uint64)[:, None]
    cols = np.arange(p, dtype=np.uint64)[None, :]
    w = philox4x32(rows, cols, 6, 0, spec.seed, spec.tag)
    X, _ = _normals_from_words(w[0], w[1])
    wt = philox4x32(np.arange(p, dtype=np.uint64), 0, 7, 0, spec.seed, spec.tag)
    order = np.lexsort((np.arange(p), wt[0]))
    support = np.sort(order[: spec.nnz])
    sign = np.where((wt[1][support] & 1) == 1, -1.0, 1.0)
    mag = 0.5 + 1.5 * uniform01(wt[2][support])
    beta_star = np.zeros(p + 1)
    beta_star[support + 1] = sign * mag
    y = X @ beta_star[1:] + _t3_noise(spec.seed, spec.tag, np.arange(n, dtype=np.uint64))
    return dict(X=X, y=y, beta_star=beta_star, support=support + 1)


def make_ar1(n, p, seed=11, tag=11, rho=0.5, chunk_cols=2048):
    """The sparse simulation design of Sec. 7.1 (eq. dgp_simulation): X~ ~ N(0, Sigma)
    with Sigma_ij = rho^|i-j| (an AR(1) recursion over columns with N(0,1)
    innovations, stream 9), X_1 = Phi(X~_1), X_j = X~_j otherwise, and
    y = X_6 - X_20 + X_50 - X_100 + X_500 - X_1000 + X_p + 0.7 X_1 eps, eps ~ N(0,1)
    (stream 10); 1-based column names as in the paper, p >= 1000.  Returns
    dict(X (n x p float32), y, beta_star(tau) callable, support)."""
    from scipy.special import ndtr, ndtri
    if p < 1000:
        raise ValueError("the design names column 1000: p >= 1000")
    rows = np.arange(n, dtype=np.uint64)[:, None]
    X = np.empty((n, p), dtype=np.float32)
    prev = None
    c = math.sqrt(1.0 - rho * rho)
    for j0 in range(0, p, chunk_cols):
        j1 = min(p, j0 + chunk_cols)
        w = philox4x32(rows, np.arange(j0, j1, dtype=np.uint64)[None, :], 9, 0, seed, tag)
        e, _ = _normals_from_words(w[0], w[1])
        for j in range(j1 - j0):
            col = e[:, j] if prev is None else rho * prev + c * e[:, j]
            X[:, j0 + j] = col
            prev = col
    X1t = X[:, 0].astype(np.float64)
    X[:, 0] = ndtr(X1t)
    we = philox4x32(np.arange(n, dtype=np.uint64), 0, 10, 0, seed, tag)
    eps, _ = _normals_from_words(we[0], we[1])
    # the named terms as written; at p = 1000, X_1000 and X_p are one column and cancel
    terms = [(6, 1.0), (20, -1.0), (50, 1.0), (100, -1.0), (500, 1.0), (1000, -1.0), (p, 1.0)]
    lin = np.zeros(p + 1)
    for k, s in terms:
        lin[k] += s
    Xd = X.astype(np.float64)
    y = Xd @ lin[1:] + 0.7 * Xd[:, 0] * eps

    def beta_star(tau):
        b = lin.copy()
        b[1] = 0.7 * ndtri(tau)
        return b
    return dict(X=X, y=y, beta_star=beta_star, support=np.nonzero(lin)[0])


def genotype_maf_thresholds(spec: GenotypeSpec, cols=None):
    """MAF_j (float64) and the uint32 Bernoulli thresholds T_j for the given columns."""
    if cols is None:
        cols = np.arange(spec.p, dtype=np.uint64)
    cols = np.asarray(cols, dtype=np.uint64)
    w = philox4x32(cols, 0, 1, 0, spec.seed, spec.tag)
    maf = spec.maf_lo + (spec.maf_hi - spec.maf_lo) * uniform01(w[0])
    thr = np.floor(maf * TWO32).astype(np.uint64).astype(np.uint32)
    return maf, thr


def genotype_columns(spec: GenotypeSpec, cols, rows=None):
    """Dosages (int8, shape rows x len(cols)) for the given columns."""
    cols = np.atleast_1d(np.asarray(cols, dtype=np.uint64))
    if rows is None:
        rows = np.arange(spec.n, dtype=np.uint64)
    rows = np.asarray(rows, dtype=np.uint64)
    _, thr = genotype_maf_thresholds(spec, cols)
    w = philox4x32(rows[:, None], cols[None, :], 2, 0, spec.seed, spec.tag)
    t = thr[None, :]
    return ((w[0] < t).astype(np.int8) + (w[1] < t).astype(np.int8))


def causal_columns(spec: GenotypeSpec):
    """The n_causal columns with the smallest stream-3 priority (ties by index), sorted."""
    p = spec.p
    j = np.arange(p, dtype=np.uint64)
    pri = philox4x32(j, 0, 3, 0, spec.seed, spec.tag)[0]
    order = np.lexsort((np.arange(p), pri))
    return np.sort(order[: spec.n_causal])


def causal_effects(spec: GenotypeSpec):
    k = np.arange(spec.n_causal, dtype=np.uint64)
    w = philox4x32(k, 0, 4, 0, spec.seed, spec.tag)
    z, _ = _normals_from_words(w[0], w[1])
    return spec.effect_sd * z


def make_genotype(spec: GenotypeSpec, with_X=True, chunk_cols=4096):
    """Return dict(y, causal, effects, maf, thr[, X (n x p int8, column-major)]).

    y = sum_k x_{.,c_k} b_k + (1 + hetero*|x_{.,c_0}|) * t3, effects on the raw
    dosage scale; c_0 is the smallest causal column index.
    """
    causal = causal_columns(spec)
    b = causal_effects(spec)
    Xc = genotype_columns(spec, causal).astype(np.float64)
    noise = _t3_noise(spec.seed, spec.tag, np.arange(spec.n, dtype=np.uint64))
    y = Xc @ b + (1.0 + spec.hetero * np.abs(Xc[:, 0])) * noise
    maf, thr = genotype_maf_thresholds(spec)
    out = dict(y=y, causal=causal, effects=b, maf=maf, thr=thr)
    if with_X:
        from . import native
        if native.host_lib() is not None:
            out["X"] = native.genotype_host(spec.n, spec.p, thr, spec.seed, spec.tag)
        else:
            X = np.empty((spec.n, spec.p), dtype=np.int8, order="F")
            for j0 in range(0, spec.p, chunk_cols):
                j1 = min(spec.p, j0 + chunk_cols)
                X[:, j0:j1] = genotype_columns(spec, np.arange(j0, j1))
            out["X"] = X
    return out


# The workloads: a small Gaussian case, the genotype single-lambda case, the
# large single problem, the batched case and the learned-warm-start training
# problems.  Sizes follow the stated configurations.
SPECS = {
    "gauss_200x2000": GaussianSpec(),
    "geno_5000x100k": GenotypeSpec(),
    "geno_20kx1M": GenotypeSpec(n=20_000, p=1_000_000, n_causal=200, seed=3, tag=3,
                                tau=0.5),
    "geno_10kx500k": GenotypeSpec(n=10_000, p=500_000, n_causal=50, seed=4, tag=4,
                                  tau=0.5),
}


def grouped_specs(nprob=64, seed=5, tag=5, n_range=(500, 5000), p_range=(10_000, 200_000),
                  lam_range=(0.2, 0.6), n_causal=20):
    """Independent uneven genotype problems (stream 8 of key (seed, tag)): problem i
    has n_i ~ U{n_range}, p_i ~ U{p_range} (inclusive, from words 0 and 1),
    lambda_i / lambda_max,i ~ U(lam_range) (word 2) and tau_i = 0.1 (i mod 9) + 0.1;
    its design and response come from GenotypeSpec with key (seed, tag * 1000 + i).
    Returns a list of (GenotypeSpec, lam_frac)."""
    w = philox4x32(np.arange(nprob, dtype=np.uint64), 0, 8, 0, seed, tag)
    out = []
    for i in range(nprob):
        n = n_range[0] + int(w[0][i]) % (n_range[1] - n_range[0] + 1)
        p = p_range[0] + int(w[1][i]) % (p_range[1] - p_range[0] + 1)
        lf = lam_range[0] + (lam_range[1] - lam_range[0]) * float(uniform01(w[2][i:i + 1])[0])
        tau = round(0.1 * (i % 9) + 0.1, 10)
        out.append((GenotypeSpec(n=n, p=p, n_causal=n_causal, seed=seed, tag=tag * 1000 + i,
                                 tau=tau, lam_frac=lf), lf))
    return out
