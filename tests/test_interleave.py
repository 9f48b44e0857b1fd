"""The interleaved column order (the Discussion's block permutation) on the host:
the order itself, and on the paper's AR(1) simulation design (Sec. 7.1) the exact
block spectra of the library's partition taken in that order against the
contiguous one, computed by the oracle."""
import numpy as np
import pytest

from oracle import pqr
from tests import helpers as H


def _lib():
    import paper_2601_02826_amd as pq
    pq.load()   # raises if libpqr.so is not built
    return pq


@pytest.mark.parametrize("p,G", [(1, 1), (17, 1), (1000, 5), (2003, 48), (50, 50)])
def test_order_is_a_residue_major_bijection(p, G):
    pq = _lib()
    cols = pq.interleaved_order(p, G)
    assert sorted(cols.tolist()) == list(range(p))
    key = [(int(j) % G, int(j)) for j in cols]
    assert key == sorted(key)
    if G == 1:
        assert np.array_equal(cols, np.arange(p))


def test_order_rejects_bad_arguments():
    pq = _lib()
    for p, G in [(0, 1), (5, 0), (5, 6)]:
        with pytest.raises(pq.PQRError) as e:
            pq.interleaved_order(p, G)
        assert e.value.status == pq.PQR_ERR_INVALID_ARG


@pytest.mark.parametrize("p,G", [(2000, 5), (50_000, 5), (100_000, 48)])
def test_neighbours_land_in_different_blocks(p, G):
    """Under the library's partition (group-aligned contiguous runs of the context's
    columns), columns j and j + 1 share a block only where a block's slice of the
    order crosses from one residue class into the next: at most G (16 + G) pairs."""
    pq = _lib()
    cols = pq.interleaved_order(p, G)
    blocks = H.oracle_blocks(p, G)[1:]          # feature blocks, context positions (1-based)
    blk = np.empty(p, dtype=np.int64)
    for b, pos in enumerate(blocks):
        blk[cols[pos - 1]] = b
    same = int(np.sum(blk[:-1] == blk[1:]))
    assert same <= G * (16 + G)
    # the contiguous order keeps all but G - 1 neighbours together
    cont = np.empty(p, dtype=np.int64)
    for b, pos in enumerate(blocks):
        cont[pos - 1] = b
    assert int(np.sum(cont[:-1] == cont[1:])) == p - G


def test_block_spectra_on_the_ar1_design():
    """Sigma_ij = 0.5^|i-j|: a contiguous block keeps the band of neighbour
    correlations (population Lambda_max -> 3), an interleaved block holds columns at
    least G apart (0.5^5 = 0.03), so every interleaved block's Lambda_max lies below
    every contiguous block's."""
    from datagen.configs import make_ar1
    pq = _lib()
    n, p, G = 300, 1000, 5
    d = make_ar1(n, p)
    X1, _, _ = H.oracle_design(d["X"], True)
    cols = pq.interleaved_order(p, G)
    Xi = X1[:, np.r_[0, 1 + cols]]
    blocks = H.oracle_blocks(p, G)[1:]
    cont = np.array([pqr.block_lambda_max(X1[:, b]) for b in blocks]) / n
    inter = np.array([pqr.block_lambda_max(Xi[:, b]) for b in blocks]) / n
    print(f"Lambda_max / n: contiguous {np.round(cont, 2)}, interleaved {np.round(inter, 2)}")
    assert inter.max() < 0.85 * cont.min()
