"""The C ABI library loads and exports every entry point declared in include/pqr.h
(no compute calls: these run without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pqr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pqr_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ["pqr_create", "pqr_solve", "pqr_kkt", "pqr_destroy", "pqr_last_error"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_2601_02826_amd as pq
    lib = pq.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(pq.SYMBOLS) == set(_declared())


def test_binding_has_no_cpu_path():
    """The binding refuses to run without the built library."""
    import paper_2601_02826_amd._lib as L
    saved = L.LIB_PATH, L._lib
    try:
        L.LIB_PATH, L._lib = "/nonexistent/libpqr.so", None
        with pytest.raises(RuntimeError):
            L.load()
    finally:
        L.LIB_PATH, L._lib = saved


def test_binding_constants_match_the_header():
    """Sizes the binding hard-codes are the header's (and the kernels' launch variant
    counts fit the tuner's report arrays)."""
    import paper_2601_02826_amd as pq
    src = open(os.path.join(ROOT, "include", "pqr.h")).read()
    defs = dict(re.findall(r"#define (PQR_[A-Z_]+) (\d+)", src))
    assert int(defs["PQR_TILE_VARIANTS"]) == pq.TILE_VARIANTS
    assert int(defs["PQR_MLP_NOALLOC_MAX_ROWS"]) == pq.MLP_NOALLOC_MAX_ROWS
    kh = open(os.path.join(ROOT, "paper_2601_02826_amd", "csrc", "pqr_kernels.h")).read()
    m = re.search(r"kBgemmVariants = (\d+), kBaxpyVariants = (\d+)", kh)
    assert (int(m.group(1)), int(m.group(2))) == (pq.BGEMM_VARIANTS, pq.BAXPY_VARIANTS)
    assert max(pq.BGEMM_VARIANTS, pq.BAXPY_VARIANTS) <= pq.TILE_VARIANTS
