"""The seeded input generators (test infrastructure shared by the oracle and GPU
sides): Philox4x32-10 against the published known-answer vectors, the C host twin
byte for byte against the numpy definition, and the Sec. 7.1 AR(1) design's
correlation structure, marginals and response."""
import ctypes

import numpy as np
import pytest

from datagen import KAT, native, philox4x32
from datagen.configs import GenotypeSpec, genotype_columns, genotype_maf_thresholds, make_ar1


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_numpy_known_answers(ctr, key, want):
    got = philox4x32(*ctr, *key)
    assert tuple(int(w) for w in got) == want


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_host_twin_known_answers(ctr, key, want):
    lib = native.host_lib()
    if lib is None:
        pytest.skip("host generator not built")
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.pqrgen_philox4x32(c.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                          out.ctypes.data_as(ctypes.c_void_p))
    assert tuple(int(w) for w in out) == want


def test_genotype_host_twin_matches_numpy():
    if native.host_lib() is None:
        pytest.skip("host generator not built")
    spec = GenotypeSpec(n=777, p=300, n_causal=5, seed=9, tag=4)
    cols = np.arange(40, 140, dtype=np.uint64)
    _, thr = genotype_maf_thresholds(spec, cols)
    host = native.genotype_host(spec.n, len(cols), thr, spec.seed, spec.tag, j0=40)
    ref = genotype_columns(spec, cols)
    assert np.array_equal(np.asarray(host), np.asarray(ref, dtype=np.int8))


def test_ar1_design_structure():
    """Sigma_ij = 0.5^|i-j| between the Gaussian columns (j >= 2), X_1 = Phi(X~_1) in
    (0, 1) with mean 1/2, and y = the sparse linear part + 0.7 X_1 eps."""
    n, p = 4000, 1000
    d = make_ar1(n, p)
    X = d["X"].astype(np.float64)
    Z = X[:, 1:]
    C = np.corrcoef(Z[:, :200].T)
    for lag, want in ((1, 0.5), (2, 0.25), (3, 0.125)):
        got = np.mean(np.diagonal(C, lag))
        assert abs(got - want) < 0.02, (lag, got)
    assert abs(np.mean(Z.var(axis=0)) - 1.0) < 0.02
    assert 0.0 < X[:, 0].min() and X[:, 0].max() < 1.0 and abs(X[:, 0].mean() - 0.5) < 0.02
    b = d["beta_star"](0.5)
    assert b[1] == 0.0 and np.count_nonzero(b) == 5      # p = 1000: -X_1000 + X_p = 0
    assert np.count_nonzero(make_ar1(50, 1200)["beta_star"](0.5)) == 7
    assert make_ar1(50, 1200)["beta_star"](0.3)[1] < 0 < make_ar1(50, 1200)["beta_star"](0.7)[1]
    resid = d["y"] - X @ b[1:]            # = 0.7 X_1 eps at tau = 0.5 (eps median 0)
    eps = resid / (0.7 * X[:, 0])
    assert abs(eps.mean()) < 0.05 and abs(eps.std() - 1.0) < 0.05
