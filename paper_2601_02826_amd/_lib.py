"""ctypes binding of libpqr (include/pqr.h): argument marshalling only.

Every computation happens in the HIP library; if libpqr.so is missing this
module raises instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpqr.so")

# enums of pqr.h
PQR_OK, PQR_ERR_INVALID_ARG, PQR_ERR_OOM, PQR_ERR_DEVICE = 0, 1, 2, 3
PQR_ERR_NOT_CONVERGED, PQR_ERR_DIVERGED, PQR_ERR_UNSUPPORTED = 4, 5, 6
FMT = {"f64": 0, "f32": 1, "bf16": 2, "fp8": 3, "i8": 4, "2bit": 5}
ITER = {"f32": 0, "f64": 1}
START = {"zero": 0, "host": 1, "device": 2}
TILE_VARIANTS = 8                      # PQR_TILE_VARIANTS: size of the tuner's time arrays
BGEMM_VARIANTS, BAXPY_VARIANTS = 4, 3  # launch variants of the back- and union products

_c_dp = ctypes.POINTER(ctypes.c_double)


class pqr_design(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("src_fmt", ctypes.c_int), ("data", ctypes.c_void_p),
                ("store_fmt", ctypes.c_int), ("standardize", ctypes.c_int)]


class pqr_options(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("mu_scale", ctypes.c_double), ("G", ctypes.c_int),
                ("eta_margin", ctypes.c_double), ("lanczos_steps", ctypes.c_int),
                ("iter_prec", ctypes.c_int), ("tol_gap", ctypes.c_double),
                ("cert_every", ctypes.c_int), ("max_iter", ctypes.c_int64),
                ("stream", ctypes.c_void_p), ("profile", ctypes.c_int),
                ("intercept_block", ctypes.c_int), ("rows_per_lane", ctypes.c_int),
                ("launch_mode", ctypes.c_int), ("tile_override", ctypes.c_int)]


class pqr_result(ctypes.Structure):
    _fields_ = [("beta", _c_dp), ("beta_std", _c_dp), ("z", _c_dp), ("theta", _c_dp),
                ("iters", ctypes.c_int64), ("x_passes", ctypes.c_int64),
                ("certs", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("primal", ctypes.c_double), ("dual", ctypes.c_double),
                ("rel_gap", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("mu", ctypes.c_double), ("seconds", ctypes.c_double),
                ("sweep_ms", ctypes.c_double), ("sweep_launches", ctypes.c_int64)]


SYMBOLS = ["pqr_default_options", "pqr_create", "pqr_solve", "pqr_kkt", "pqr_lambda_max",
           "pqr_blocks", "pqr_iterate", "pqr_solve_batch", "pqr_batch_tiles", "pqr_kkt_columns", "pqr_create_subset",
           "pqr_mlp_param_count", "pqr_features", "pqr_mlp_forward", "pqr_mlp_workspace_bytes",
           "pqr_mlp_grad", "pqr_mlp_grad_noalloc", "pqr_mlp_adam", "pqr_solve_learned", "pqr_solve_screened", "pqr_solve_grouped", "pqr_solve_lla",
           "pqr_interleaved_order", "pqr_destroy", "pqr_last_error", "pqr_status_string"]


class pqr_learned_report(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int), ("fallback", ctypes.c_int),
                ("active_initial", ctypes.c_int64), ("active_final", ctypes.c_int64),
                ("reduced_iters", ctypes.c_int64), ("seconds_proposal", ctypes.c_double),
                ("seconds_reduced", ctypes.c_double), ("seconds_check", ctypes.c_double),
                ("reduced_sweep_ms", ctypes.c_double), ("reduced_sweep_bytes", ctypes.c_double),
                ("reduced_sweep_launches", ctypes.c_int64)]

_lib = None


def load():
    """Load libpqr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libpqr.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.pqr_default_options.argtypes = [ctypes.POINTER(pqr_options)]
    lib.pqr_default_options.restype = None
    lib.pqr_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(pqr_design),
                               ctypes.POINTER(pqr_options)]
    lib.pqr_create.restype = ci
    lib.pqr_solve.argtypes = [vp, _c_dp, dbl, dbl, _c_dp, ci, ctypes.POINTER(pqr_result),
                              ctypes.POINTER(pqr_result)]
    lib.pqr_solve.restype = ci
    lib.pqr_kkt.argtypes = [vp, _c_dp, dbl, dbl, _c_dp, _c_dp, _c_dp, _c_dp]
    lib.pqr_kkt.restype = ci
    lib.pqr_lambda_max.argtypes = [vp, _c_dp, dbl, _c_dp, _c_dp, _c_dp]
    lib.pqr_lambda_max.restype = ci
    lib.pqr_blocks.argtypes = [vp, ctypes.POINTER(ci), ctypes.POINTER(ci), _c_dp]
    lib.pqr_blocks.restype = ci
    lib.pqr_iterate.argtypes = [vp, _c_dp, dbl, dbl, _c_dp, dbl, _c_dp, i64, _c_dp, _c_dp, _c_dp]
    lib.pqr_iterate.restype = ci
    lib.pqr_solve_batch.argtypes = [vp, _c_dp, ci, _c_dp, _c_dp, _c_dp, ctypes.POINTER(pqr_result)]
    lib.pqr_solve_batch.restype = ci
    lib.pqr_batch_tiles.argtypes = [vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci), _c_dp, _c_dp,
                                    ctypes.POINTER(i64)]
    lib.pqr_batch_tiles.restype = ci
    _c_fp = ctypes.c_void_p
    lib.pqr_kkt_columns.argtypes = [vp, _c_dp, dbl, dbl, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp]
    lib.pqr_kkt_columns.restype = ci
    lib.pqr_create_subset.argtypes = [ctypes.POINTER(vp), vp, ctypes.POINTER(i64), i64,
                                      ctypes.POINTER(pqr_options)]
    lib.pqr_create_subset.restype = ci
    lib.pqr_interleaved_order.argtypes = [i64, ci, ctypes.POINTER(i64)]
    lib.pqr_interleaved_order.restype = ci
    lib.pqr_mlp_param_count.argtypes = []
    lib.pqr_mlp_param_count.restype = i64
    lib.pqr_features.argtypes = [vp, _c_dp, dbl, dbl, _c_dp, _c_fp, _c_dp]
    lib.pqr_features.restype = ci
    lib.pqr_mlp_forward.argtypes = [_c_fp, _c_fp, i64, _c_fp, vp]
    lib.pqr_mlp_forward.restype = ci
    lib.pqr_mlp_workspace_bytes.argtypes = [i64]
    lib.pqr_mlp_workspace_bytes.restype = i64
    lib.pqr_mlp_grad.argtypes = [_c_fp, _c_fp, _c_fp, _c_fp, i64, dbl, dbl, _c_fp, _c_fp, _c_fp, vp]
    lib.pqr_mlp_grad.restype = ci
    lib.pqr_mlp_grad_noalloc.argtypes = [_c_fp, _c_fp, _c_fp, _c_fp, i64, dbl, dbl, _c_fp, _c_fp, vp]
    lib.pqr_mlp_grad_noalloc.restype = ci
    lib.pqr_mlp_adam.argtypes = [_c_fp, _c_fp, _c_fp, _c_fp, ci, dbl, dbl, dbl, dbl, vp]
    lib.pqr_mlp_adam.restype = ci
    lib.pqr_solve_learned.argtypes = [vp, _c_dp, dbl, dbl, _c_dp, _c_fp, dbl, ci,
                                      ctypes.POINTER(pqr_result), ctypes.POINTER(pqr_learned_report)]
    lib.pqr_solve_learned.restype = ci
    lib.pqr_solve_screened.argtypes = [vp, _c_dp, dbl, dbl, _c_dp, dbl, i64, ci,
                                       ctypes.POINTER(pqr_result), ctypes.POINTER(pqr_learned_report)]
    lib.pqr_solve_screened.restype = ci
    lib.pqr_solve_grouped.argtypes = [ci, ctypes.POINTER(vp), ctypes.POINTER(_c_dp), _c_dp, _c_dp,
                                      ctypes.POINTER(_c_dp), ctypes.POINTER(pqr_result),
                                      ctypes.POINTER(ci)]
    lib.pqr_solve_grouped.restype = ci
    lib.pqr_solve_lla.argtypes = [vp, _c_dp, dbl, dbl, ci, dbl, ci, dbl, ci, _c_dp,
                                  ctypes.POINTER(i64), ctypes.POINTER(pqr_result)]
    lib.pqr_solve_lla.restype = ci
    lib.pqr_destroy.argtypes = [vp]
    lib.pqr_destroy.restype = None
    lib.pqr_last_error.argtypes = [vp]
    lib.pqr_last_error.restype = ctypes.c_char_p
    lib.pqr_status_string.argtypes = [ci]
    lib.pqr_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_c_dp)


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.shape[0] != n:
        raise ValueError(f"expected length {n}, got {a.shape[0]}")
    return a


class PQRError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:  # noqa: BLE001 - torch is optional plumbing
        pass
    return None


class Result(dict):
    """Solution and report of pqr_solve (attribute access for convenience)."""
    __getattr__ = dict.__getitem__


class Context:
    """A design matrix resident on the GPU plus its solver state (pqr_ctx)."""

    def __init__(self, data_ptr, n, p, ld=None, src_fmt="i8", store_fmt="i8", standardize=True,
                 keepalive=None, **options):
        lib = load()
        self._lib = lib
        self.n, self.p = int(n), int(p)
        self._keep = keepalive
        d = pqr_design(n=self.n, p=self.p, ld=int(ld if ld is not None else n),
                       src_fmt=FMT[src_fmt], data=ctypes.c_void_p(int(data_ptr)),
                       store_fmt=FMT[store_fmt], standardize=int(bool(standardize)))
        o = pqr_options()
        lib.pqr_default_options(ctypes.byref(o))
        for k, v in options.items():
            if k == "iter_prec":
                v = ITER[v] if isinstance(v, str) else int(v)
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        if o.stream is None:
            o.stream = _current_stream()
        self.options = o
        h = ctypes.c_void_p()
        st = lib.pqr_create(ctypes.byref(h), ctypes.byref(d), ctypes.byref(o))
        self._h = h
        if st != PQR_OK:
            msg = lib.pqr_last_error(h).decode() if h.value else "pqr_create failed"
            lib.pqr_destroy(h)
            self._h = None
            raise PQRError(st, msg)

    @classmethod
    def from_tensor(cls, Xcols, src_fmt=None, **kw):
        """Xcols: a torch CUDA tensor of shape (p, n) holding X column by column
        (i.e. X in column-major order), dtype uint8/int8, float32 or float64."""
        import torch
        if not Xcols.is_cuda or Xcols.dim() != 2 or Xcols.stride(1) != 1:
            raise ValueError("Xcols must be a CUDA tensor of shape (p, n) with unit row stride")
        if src_fmt is None:
            src_fmt = {torch.float64: "f64", torch.float32: "f32", torch.uint8: "i8",
                       torch.int8: "i8"}[Xcols.dtype]
        p, n = Xcols.shape
        return cls(Xcols.data_ptr(), n, p, ld=Xcols.stride(0), src_fmt=src_fmt, keepalive=Xcols,
                   **kw)

    def _check(self, st, ok=(PQR_OK,)):
        if st not in ok:
            raise PQRError(st, self._lib.pqr_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pqr_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    # ---- the C ABI, one method per entry point ----
    def solve(self, y, tau, lam, weights=None, start="zero", warm=None, allow_not_converged=False):
        y = _f64(y, self.n)
        w = _f64(weights, self.p + 1)
        beta = np.zeros(self.p + 1)
        beta_std = np.zeros(self.p + 1)
        z = np.zeros(self.n)
        theta = np.zeros(self.n)
        out = pqr_result(beta=_dptr(beta), beta_std=_dptr(beta_std), z=_dptr(z), theta=_dptr(theta))
        wr = None
        if warm is not None:
            wb = _f64(warm["beta_std"], self.p + 1)
            wz, wt = _f64(warm.get("z"), self.n), _f64(warm.get("theta"), self.n)
            wr = pqr_result(beta_std=_dptr(wb), z=_dptr(wz), theta=_dptr(wt))
            start = "host"
        st = self._lib.pqr_solve(self._h, _dptr(y), float(tau), float(lam), _dptr(w), START[start],
                                 ctypes.byref(wr) if wr is not None else None, ctypes.byref(out))
        ok = (PQR_OK, PQR_ERR_NOT_CONVERGED) if allow_not_converged else (PQR_OK,)
        self._check(st, ok)
        return Result(beta=beta, beta_std=beta_std, z=z, theta=theta, iters=out.iters,
                      x_passes=out.x_passes, certs=out.certs, nnz=out.nnz, primal=out.primal,
                      dual=out.dual, rel_gap=out.rel_gap, lambda_max=out.lambda_max, mu=out.mu,
                      seconds=out.seconds, sweep_ms=out.sweep_ms,
                      sweep_launches=out.sweep_launches, status=st)

    def solve_batch(self, y, taus, lams, weights=None, allow_not_converged=False):
        """pqr_solve_batch: K (tau_k, lambda_k) pairs on the same X and y."""
        taus = _f64(taus)
        lams = _f64(lams)
        K = len(taus)
        if len(lams) != K:
            raise ValueError("taus and lams differ in length")
        outs = (pqr_result * K)()
        keep = []
        for k in range(K):
            arr = dict(beta=np.zeros(self.p + 1), beta_std=np.zeros(self.p + 1),
                       z=np.zeros(self.n), theta=np.zeros(self.n))
            keep.append(arr)
            outs[k].beta, outs[k].beta_std = _dptr(arr["beta"]), _dptr(arr["beta_std"])
            outs[k].z, outs[k].theta = _dptr(arr["z"]), _dptr(arr["theta"])
        st = self._lib.pqr_solve_batch(self._h, _dptr(_f64(y, self.n)), K, _dptr(taus), _dptr(lams),
                                       _dptr(_f64(weights, self.p + 1)), outs)
        ok = (PQR_OK, PQR_ERR_NOT_CONVERGED) if allow_not_converged else (PQR_OK,)
        self._check(st, ok)
        res = []
        for k in range(K):
            o = outs[k]
            res.append(Result(**keep[k], iters=o.iters, x_passes=o.x_passes, certs=o.certs,
                              nnz=o.nnz, primal=o.primal, dual=o.dual, rel_gap=o.rel_gap,
                              mu=o.mu, seconds=o.seconds, sweep_ms=o.sweep_ms,
                              sweep_launches=o.sweep_launches, status=st))
        return res

    def batch_tiles(self, K):
        """pqr_batch_tiles: the autotuner's choices and candidate times for width K."""
        bv, av, uc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        bms, ams = np.zeros(TILE_VARIANTS), np.zeros(TILE_VARIANTS)
        self._check(self._lib.pqr_batch_tiles(self._h, int(K), ctypes.byref(bv), ctypes.byref(av),
                                              _dptr(bms), _dptr(ams), ctypes.byref(uc)))
        return dict(bgemm_variant=bv.value, baxpy_variant=av.value,
                    bgemm_ms=bms[:BGEMM_VARIANTS].tolist(), baxpy_ms=ams[:BAXPY_VARIANTS].tolist(),
                    union_cols=uc.value)

    def kkt_columns(self, y, tau, lam, beta_std, theta, weights=None):
        rep = np.zeros(4)
        v = np.zeros(self.p)
        self._check(self._lib.pqr_kkt_columns(self._h, _dptr(_f64(y, self.n)), float(tau), float(lam),
                                              _dptr(_f64(weights, self.p + 1)),
                                              _dptr(_f64(beta_std, self.p + 1)),
                                              _dptr(_f64(theta, self.n)), _dptr(rep), _dptr(v)))
        return dict(primal=rep[0], dual=rep[1], rel_gap=rep[2], max_ratio=rep[3], v=v)

    def subset(self, cols, **options):
        """pqr_create_subset: a new Context over the listed columns of this one."""
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        o = pqr_options.from_buffer_copy(self.options)
        for k, val in options.items():
            if k == "iter_prec":
                val = ITER[val] if isinstance(val, str) else int(val)
            setattr(o, k, val)
        h = ctypes.c_void_p()
        st = self._lib.pqr_create_subset(ctypes.byref(h), self._h,
                                         cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                         len(cols), ctypes.byref(o))
        if st != PQR_OK:
            msg = self._lib.pqr_last_error(h).decode() if h.value else "pqr_create_subset failed"
            self._lib.pqr_destroy(h)
            raise PQRError(st, msg)
        sub = Context.__new__(Context)
        sub._lib, sub._h, sub.n, sub.p, sub._keep, sub.options = self._lib, h, self.n, len(cols), self, o
        return sub

    def interleaved(self, G=None, **options):
        """A context over this one's columns in pqr_interleaved_order for G blocks,
        wrapped so that every per-column array is in this context's order."""
        options.pop("G", None)
        G = int(G if G is not None else (self.options.G or 48))
        cols = interleaved_order(self.p, G)
        return Interleaved(self.subset(cols, G=G, **options), cols)

    def features(self, y, tau, lam, feats_ptr, weights=None):
        """pqr_features into a device buffer of p x 4 floats; returns lambda_max."""
        lm = np.zeros(1)
        self._check(self._lib.pqr_features(self._h, _dptr(_f64(y, self.n)), float(tau), float(lam),
                                           _dptr(_f64(weights, self.p + 1)),
                                           ctypes.c_void_p(int(feats_ptr)), _dptr(lm)))
        return lm[0]

    def solve_learned(self, y, tau, lam, params_ptr, threshold=0.0, max_rounds=4, weights=None):
        beta = np.zeros(self.p + 1)
        beta_std = np.zeros(self.p + 1)
        z = np.zeros(self.n)
        theta = np.zeros(self.n)
        out = pqr_result(beta=_dptr(beta), beta_std=_dptr(beta_std), z=_dptr(z), theta=_dptr(theta))
        rep = pqr_learned_report()
        st = self._lib.pqr_solve_learned(self._h, _dptr(_f64(y, self.n)), float(tau), float(lam),
                                         _dptr(_f64(weights, self.p + 1)),
                                         ctypes.c_void_p(int(params_ptr)), float(threshold),
                                         int(max_rounds), ctypes.byref(out), ctypes.byref(rep))
        self._check(st, (PQR_OK, PQR_ERR_NOT_CONVERGED))
        return Result(beta=beta, beta_std=beta_std, z=z, theta=theta, iters=out.iters, nnz=out.nnz,
                      primal=out.primal, dual=out.dual, rel_gap=out.rel_gap,
                      lambda_max=out.lambda_max, seconds=out.seconds, status=st,
                      rounds=rep.rounds, fallback=rep.fallback, active_initial=rep.active_initial,
                      active_final=rep.active_final, reduced_iters=rep.reduced_iters,
                      seconds_proposal=rep.seconds_proposal, seconds_reduced=rep.seconds_reduced,
                      seconds_check=rep.seconds_check, reduced_sweep_ms=rep.reduced_sweep_ms,
                      reduced_sweep_bytes=rep.reduced_sweep_bytes,
                      reduced_sweep_launches=rep.reduced_sweep_launches)

    def solve_screened(self, y, tau, lam, lambda_prev=0.0, budget=0, max_rounds=4, weights=None):
        """pqr_solve_screened: strong-rule (budget 0) or top-budget score proposal, then the
        active-set rounds of the learned warm start, judged by the full certificate."""
        beta = np.zeros(self.p + 1)
        beta_std = np.zeros(self.p + 1)
        z = np.zeros(self.n)
        theta = np.zeros(self.n)
        out = pqr_result(beta=_dptr(beta), beta_std=_dptr(beta_std), z=_dptr(z), theta=_dptr(theta))
        rep = pqr_learned_report()
        st = self._lib.pqr_solve_screened(self._h, _dptr(_f64(y, self.n)), float(tau), float(lam),
                                          _dptr(_f64(weights, self.p + 1)), float(lambda_prev),
                                          int(budget), int(max_rounds), ctypes.byref(out),
                                          ctypes.byref(rep))
        self._check(st, (PQR_OK, PQR_ERR_NOT_CONVERGED))
        return Result(beta=beta, beta_std=beta_std, z=z, theta=theta, iters=out.iters, nnz=out.nnz,
                      primal=out.primal, dual=out.dual, rel_gap=out.rel_gap,
                      lambda_max=out.lambda_max, seconds=out.seconds, status=st,
                      rounds=rep.rounds, fallback=rep.fallback, active_initial=rep.active_initial,
                      active_final=rep.active_final, reduced_iters=rep.reduced_iters,
                      seconds_proposal=rep.seconds_proposal, seconds_reduced=rep.seconds_reduced,
                      seconds_check=rep.seconds_check, reduced_sweep_ms=rep.reduced_sweep_ms,
                      reduced_sweep_bytes=rep.reduced_sweep_bytes,
                      reduced_sweep_launches=rep.reduced_sweep_launches)

    def solve_lla(self, y, tau, lam, penalty="scad", a=None, L=1, wfloor=0.0, start="zero",
                  allow_not_converged=False):
        """pqr_solve_lla (Algorithm 2).  Returns the last stage's Result with extra keys
        `weights` (p+1) and `stage_iters` (L+1)."""
        kind = {"scad": 0, "mcp": 1}[penalty]
        if a is None:
            a = 3.7 if kind == 0 else 3.0
        beta = np.zeros(self.p + 1)
        beta_std = np.zeros(self.p + 1)
        z = np.zeros(self.n)
        theta = np.zeros(self.n)
        w = np.zeros(self.p + 1)
        its = (ctypes.c_int64 * (L + 1))()
        out = pqr_result(beta=_dptr(beta), beta_std=_dptr(beta_std), z=_dptr(z), theta=_dptr(theta))
        st = self._lib.pqr_solve_lla(self._h, _dptr(_f64(y, self.n)), float(tau), float(lam), kind,
                                     float(a), int(L), float(wfloor), START[start], _dptr(w), its,
                                     ctypes.byref(out))
        ok = (PQR_OK, PQR_ERR_NOT_CONVERGED) if allow_not_converged else (PQR_OK,)
        self._check(st, ok)
        return Result(beta=beta, beta_std=beta_std, z=z, theta=theta, iters=out.iters,
                      nnz=out.nnz, primal=out.primal, dual=out.dual, rel_gap=out.rel_gap,
                      seconds=out.seconds, sweep_ms=out.sweep_ms,
                      sweep_launches=out.sweep_launches, status=st, weights=w,
                      stage_iters=list(its))

    def kkt(self, y, tau, lam, beta_std, theta, weights=None):
        rep = np.zeros(4)
        self._check(self._lib.pqr_kkt(self._h, _dptr(_f64(y, self.n)), float(tau), float(lam),
                                      _dptr(_f64(weights, self.p + 1)),
                                      _dptr(_f64(beta_std, self.p + 1)),
                                      _dptr(_f64(theta, self.n)), _dptr(rep)))
        return dict(primal=rep[0], dual=rep[1], rel_gap=rep[2], max_ratio=rep[3])

    def lambda_max(self, y, tau, weights=None, score=False):
        lm = np.zeros(1)
        sc = np.zeros(self.p) if score else None
        self._check(self._lib.pqr_lambda_max(self._h, _dptr(_f64(y, self.n)), float(tau),
                                             _dptr(_f64(weights, self.p + 1)), _dptr(lm), _dptr(sc)))
        return (lm[0], sc) if score else lm[0]

    def blocks(self):
        G = ctypes.c_int()
        self._check(self._lib.pqr_blocks(self._h, ctypes.byref(G), None, None))
        bounds = (ctypes.c_int * (G.value + 1))()
        lam = np.zeros(G.value)
        self._check(self._lib.pqr_blocks(self._h, ctypes.byref(G), bounds, _dptr(lam)))
        return G.value, np.array(bounds[:], dtype=np.int64), lam

    def iterate(self, y, tau, lam, mu, eta, iters, beta_std, z, theta, weights=None):
        b = np.array(beta_std, dtype=np.float64)
        zz = np.array(z, dtype=np.float64)
        tt = np.array(theta, dtype=np.float64)
        self._check(self._lib.pqr_iterate(self._h, _dptr(_f64(y, self.n)), float(tau), float(lam),
                                          _dptr(_f64(weights, self.p + 1)), float(mu),
                                          _dptr(_f64(eta)), int(iters), _dptr(b), _dptr(zz),
                                          _dptr(tt)))
        return b, zz, tt


def interleaved_order(p, G):
    """pqr_interleaved_order: the feature columns 0..p-1 ordered by (j mod G, j)."""
    cols = np.zeros(int(p), dtype=np.int64)
    st = load().pqr_interleaved_order(int(p), int(G), cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if st != PQR_OK:
        raise PQRError(st, "pqr_interleaved_order: need 1 <= G <= p")
    return cols


class Interleaved:
    """A Context over the columns of another in interleaved order (`ctx`, element
    1 + q is source column cols[q]) with the source order at its surface: weights and
    coefficients are permuted on the way in and out; nothing else changes."""

    def __init__(self, ctx, cols):
        self.ctx, self.cols = ctx, np.asarray(cols, dtype=np.int64)
        self.n, self.p = ctx.n, ctx.p

    def _in(self, a):   # source order (p+1, intercept first) -> context order
        if a is None:
            return None
        a = np.asarray(a, dtype=np.float64)
        return np.concatenate([a[:1], a[1 + self.cols]])

    def _out(self, a):  # context order -> source order
        o = np.empty_like(a)
        o[0] = a[0]
        o[1 + self.cols] = a[1:]
        return o

    def _res(self, r):
        for k in ("beta", "beta_std", "weights"):
            if k in r and r[k] is not None and len(r[k]) == self.p + 1:
                r[k] = self._out(r[k])
        return r

    def solve(self, y, tau, lam, weights=None, start="zero", warm=None, allow_not_converged=False):
        if warm is not None:
            warm = {k: (self._in(v) if k in ("beta", "beta_std") else v) for k, v in warm.items()}
        return self._res(self.ctx.solve(y, tau, lam, weights=self._in(weights), start=start,
                                        warm=warm, allow_not_converged=allow_not_converged))

    def solve_batch(self, y, taus, lams, weights=None, allow_not_converged=False):
        return [self._res(r) for r in self.ctx.solve_batch(y, taus, lams, weights=self._in(weights),
                                                           allow_not_converged=allow_not_converged)]

    def kkt(self, y, tau, lam, beta_std, theta, weights=None):
        return self.ctx.kkt(y, tau, lam, self._in(beta_std), theta, weights=self._in(weights))

    def lambda_max(self, y, tau, weights=None, score=False):
        r = self.ctx.lambda_max(y, tau, weights=self._in(weights), score=score)
        if not score:
            return r
        lm, sc = r
        o = np.empty_like(sc)
        o[self.cols] = sc
        return lm, o

    def blocks(self):
        """(G, bounds, Lambda) of the context; bounds are positions in `cols`."""
        return self.ctx.blocks()

    def block_columns(self):
        """The source feature columns (0-based) of every block, in block order."""
        G, bounds, _ = self.ctx.blocks()
        return [self.cols[bounds[b]:bounds[b + 1]] for b in range(G)]

    def iterate(self, y, tau, lam, mu, eta, iters, beta_std, z, theta, weights=None):
        b, zz, tt = self.ctx.iterate(y, tau, lam, mu, eta, iters, self._in(beta_std), z, theta,
                                     weights=self._in(weights))
        return self._out(b), zz, tt

    def close(self):
        self.ctx.close()


# ---- the scoring network: free functions over device buffers (torch tensors) ----
def _ptr(t):
    return ctypes.c_void_p(int(t.data_ptr()))


def mlp_param_count():
    return int(load().pqr_mlp_param_count())


def mlp_forward(params, feats, out, stream=None):
    lib = load()
    B = feats.shape[0]
    st = lib.pqr_mlp_forward(_ptr(params), _ptr(feats), B, _ptr(out),
                             stream if stream is not None else _current_stream())
    if st != PQR_OK:
        raise PQRError(st, "pqr_mlp_forward failed")


def mlp_workspace_bytes(B):
    return int(load().pqr_mlp_workspace_bytes(int(B)))


def mlp_grad(params, feats, target, active, workspace, grad, loss, w_reg=1.0, w_pos=1.0,
             stream=None):
    lib = load()
    st = lib.pqr_mlp_grad(_ptr(params), _ptr(feats), _ptr(target), _ptr(active), feats.shape[0],
                          float(w_reg), float(w_pos), _ptr(workspace), _ptr(grad), _ptr(loss),
                          stream if stream is not None else _current_stream())
    if st != PQR_OK:
        raise PQRError(st, "pqr_mlp_grad failed")


MLP_NOALLOC_MAX_ROWS = 8192


def mlp_grad_noalloc(params, feats, target, active, grad, loss, w_reg=1.0, w_pos=1.0, B=None,
                     stream=None):
    """pqr_mlp_grad_noalloc: the gradient with the library's own fixed scratch (no
    workspace, no allocation); at most MLP_NOALLOC_MAX_ROWS rows."""
    lib = load()
    B = feats.shape[0] if B is None else int(B)
    st = lib.pqr_mlp_grad_noalloc(_ptr(params), _ptr(feats), _ptr(target), _ptr(active), B,
                                  float(w_reg), float(w_pos), _ptr(grad), _ptr(loss),
                                  stream if stream is not None else _current_stream())
    if st == PQR_ERR_UNSUPPORTED:
        raise PQRError(st, f"pqr_mlp_grad_noalloc: {B} rows exceed the allocation-free maximum "
                           f"of {MLP_NOALLOC_MAX_ROWS}")
    if st != PQR_OK:
        raise PQRError(st, "pqr_mlp_grad_noalloc failed")


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    lib = load()
    st = lib.pqr_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                          float(beta1), float(beta2), float(eps),
                          stream if stream is not None else _current_stream())
    if st != PQR_OK:
        raise PQRError(st, "pqr_mlp_adam failed")


def solve_grouped(ctxs, ys, taus, lams, weights=None, allow_not_converged=False, check=True):
    """pqr_solve_grouped: problem i is (ctxs[i], ys[i], taus[i], lams[i]), all iterated
    in shared launches.  Returns (results, statuses); with check, raises PQRError when
    a problem fails (NOT_CONVERGED tolerated with allow_not_converged)."""
    lib = load()
    P = len(ctxs)
    if not (len(ys) == len(taus) == len(lams) == P) or P < 1:
        raise ValueError("ctxs, ys, taus and lams must have the same nonzero length")
    yv = [_f64(ys[i], ctxs[i].n) for i in range(P)]
    wv = [None] * P if weights is None else [_f64(weights[i], ctxs[i].p + 1) for i in range(P)]
    handles = (ctypes.c_void_p * P)(*[c._h.value for c in ctxs])
    yp = (_c_dp * P)(*[_dptr(a) for a in yv])
    wp = None if weights is None else (_c_dp * P)(*[_dptr(a) for a in wv])
    outs = (pqr_result * P)()
    keep = []
    for i, c in enumerate(ctxs):
        arr = dict(beta=np.zeros(c.p + 1), beta_std=np.zeros(c.p + 1), z=np.zeros(c.n),
                   theta=np.zeros(c.n))
        keep.append(arr)
        outs[i].beta, outs[i].beta_std = _dptr(arr["beta"]), _dptr(arr["beta_std"])
        outs[i].z, outs[i].theta = _dptr(arr["z"]), _dptr(arr["theta"])
    sts = (ctypes.c_int * P)()
    st = lib.pqr_solve_grouped(P, handles, yp, _dptr(_f64(taus)), _dptr(_f64(lams)), wp, outs, sts)
    ok = (PQR_OK, PQR_ERR_NOT_CONVERGED) if allow_not_converged else (PQR_OK,)
    statuses = list(sts)
    if check and st not in ok:
        bad = next((i for i in range(P) if statuses[i] not in ok), 0)
        raise PQRError(st, f"problem {bad}: " + lib.pqr_last_error(ctxs[bad]._h).decode())
    res = []
    for i in range(P):
        o = outs[i]
        res.append(Result(**keep[i], iters=o.iters, x_passes=o.x_passes, certs=o.certs, nnz=o.nnz,
                          primal=o.primal, dual=o.dual, rel_gap=o.rel_gap,
                          lambda_max=o.lambda_max, mu=o.mu, seconds=o.seconds,
                          sweep_ms=o.sweep_ms, sweep_launches=o.sweep_launches,
                          status=statuses[i]))
    return res, statuses
