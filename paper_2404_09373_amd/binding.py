"""ctypes binding of include/isdf.h (argument marshalling only).

Every step of the fit and of the exchange build runs inside libisdf.so; this
module converts NumPy/torch arguments into the C structs and pointers the
library expects.  torch is used only for device buffers and the stream.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libisdf.so")

ISDF_OK = 0
STATUS = {
    0: "ISDF_OK", -1: "ISDF_E_ARG", -2: "ISDF_E_NOMEM", -3: "ISDF_E_HIP",
    -4: "ISDF_E_NOT_SPD", -5: "ISDF_E_RANK", -6: "ISDF_E_STATE", -7: "ISDF_E_UNSUPPORTED",
}
FIELD = {"phi": 0, "diag": 1, "points": 2, "count": 3, "theta": 4, "F": 5, "XL": 6, "XN": 7, "W": 8}
FP64, MIXED_X3, MIXED_X6 = 0, 1, 2
W_F64, W_F32 = 0, 1
MIX_THETA, MIX_W, MIX_EXCHANGE = 1, 2, 4
SEL_FULL, SEL_MLP = 0, 1

EXPORTED = [
    "isdf_plan", "isdf_plan_info", "isdf_plan_domain", "isdf_plan_domain_points",
    "isdf_plan_domain_functions", "isdf_fit", "isdf_fit_with_points", "isdf_exchange",
    "isdf_fit_get", "isdf_fit_info", "isdf_stage_times", "isdf_sync", "isdf_fit_destroy",
    "isdf_plan_destroy", "isdf_last_error", "isdf_version", "isdf_fit_with_candidates",
    "isdf_fit_selection", "isdf_fit_features", "isdf_mlp_forward", "isdf_mlp_loss_grad",
    "isdf_mlp_train", "isdf_profile", "isdf_kernel_stats", "isdf_exchange_occ", "isdf_autotune",
    "isdf_fit_batch", "isdf_exchange_occ_ri", "isdf_grids_for_threshold", "isdf_exchange_universal",
    "isdf_exchange_occ_ri_noalloc", "isdf_plan_workspace_bytes", "isdf_plan_alloc_stats",
    "isdf_fit_screen_stats",
]
NOALLOC_SCRATCH_MB = 32
MLP_NPARAM = 5313


class _MlpConfig(C.Structure):
    _fields_ = [
        ("epochs", C.c_int32),
        ("batch", C.c_int32),
        ("lr", C.c_float),
        ("beta1", C.c_float),
        ("beta2", C.c_float),
        ("eps", C.c_float),
        ("pos_weight", C.c_float),
        ("seed", C.c_uint64),
        ("stream", C.c_void_p),
    ]


class IsdfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _System(C.Structure):
    _fields_ = [
        ("lattice", C.c_double * 9),
        ("n_atoms", C.c_int32),
        ("xyz", C.POINTER(C.c_double)),
        ("n_shells", C.c_int32),
        ("shell_atom", C.POINTER(C.c_int32)),
        ("shell_l", C.POINTER(C.c_int32)),
        ("shell_alpha", C.POINTER(C.c_double)),
        ("n_levels", C.c_int32),
        ("grid", C.POINTER(C.c_int32)),
        ("alpha_bound", C.POINTER(C.c_double)),
        ("image_tol", C.c_double),
        ("eps_r", C.c_double),
        ("n_mu_ratio", C.c_double),
        ("eps_isdf", C.c_double),
        ("tie_tol", C.c_double),
        ("domain_mode", C.c_int32),
        ("pad_sys", C.c_int32),
    ]


class _Options(C.Structure):
    _fields_ = [
        ("precision", C.c_int32),
        ("selector", C.c_int32),
        ("mlp_keep", C.c_double),
        ("mlp_cutoff", C.c_double),
        ("mlp_weights", C.POINTER(C.c_float)),
        ("stream", C.c_void_p),
        ("w_batch", C.c_int32),
        ("mixed_mask", C.c_int32),
        ("eager_exchange", C.c_int32),
        ("pad0", C.c_int32),
        ("tune_file", C.c_char_p),
        ("universal_all_points", C.c_int32),
        ("universal_tile_mb", C.c_int32),
        ("w_storage", C.c_int32),
        ("pad1", C.c_int32),
        ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t),
        ("phi_budget_mb", C.c_int32),
        ("ri_rows", C.c_int32),
        ("ri_screen_tau", C.c_double),
    ]


_lib = None


def load(required: bool = True):
    """Load libisdf.so from the package directory (never builds it)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if required:
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())"
            )
        return None
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.isdf_plan.argtypes = [C.POINTER(_System), C.POINTER(_Options), C.POINTER(vp)]
    lib.isdf_plan_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.isdf_plan_domain.argtypes = [vp, C.c_int32] + [C.POINTER(C.c_int32)] * 2 + [C.POINTER(C.c_int64)] + [C.POINTER(C.c_int32)] * 3
    lib.isdf_plan_domain_points.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
    lib.isdf_plan_domain_functions.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
    lib.isdf_fit.argtypes = [vp, C.POINTER(vp)]
    lib.isdf_fit_with_points.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(vp)]
    lib.isdf_exchange.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double)]
    lib.isdf_fit_get.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_size_t]
    lib.isdf_fit_info.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.isdf_stage_times.argtypes = [vp, C.POINTER(C.c_double), C.c_int32]
    lib.isdf_sync.argtypes = [vp]
    lib.isdf_fit_destroy.argtypes = [vp]
    lib.isdf_fit_destroy.restype = None
    lib.isdf_plan_destroy.argtypes = [vp]
    lib.isdf_plan_destroy.restype = None
    lib.isdf_last_error.restype = C.c_char_p
    lib.isdf_version.restype = C.c_char_p
    fp = C.POINTER(C.c_float)
    lib.isdf_fit_with_candidates.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(vp)]
    lib.isdf_fit_selection.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.isdf_fit_features.argtypes = [vp, vp, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.isdf_mlp_forward.argtypes = [fp, vp, C.c_int64, vp, vp]
    lib.isdf_mlp_loss_grad.argtypes = [fp, vp, vp, C.c_int64, C.c_float, fp, fp, vp]
    lib.isdf_mlp_train.argtypes = [vp, vp, C.c_int64, C.POINTER(_MlpConfig), fp, fp]
    lib.isdf_profile.argtypes = [vp, C.c_int32]
    lib.isdf_exchange_occ.argtypes = [vp, vp, vp, C.c_int32, vp, C.POINTER(C.c_double)]
    lib.isdf_exchange_occ_ri.argtypes = [vp, vp, vp, C.c_int32, vp, C.POINTER(C.c_double)]
    lib.isdf_exchange_universal.argtypes = [vp, vp, vp, C.c_int32, vp, C.POINTER(C.c_double)]
    lib.isdf_exchange_occ_ri_noalloc.argtypes = [vp, vp, vp, C.c_int32, vp, C.POINTER(C.c_double)]
    lib.isdf_plan_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.isdf_plan_alloc_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.isdf_fit_screen_stats.argtypes = [vp, C.POINTER(C.c_double)]
    lib.isdf_autotune.argtypes = [vp, C.c_int32, C.c_int32, C.c_char_p]
    lib.isdf_grids_for_threshold.argtypes = [C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
                                             C.c_int32, C.POINTER(C.c_double), C.c_double,
                                             C.POINTER(C.c_int32)]
    lib.isdf_fit_batch.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, C.POINTER(vp),
                                   C.POINTER(C.c_int)]
    lib.isdf_kernel_stats.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double)]
    for name in ("isdf_plan", "isdf_plan_info", "isdf_plan_domain", "isdf_plan_domain_points",
                 "isdf_plan_domain_functions", "isdf_fit", "isdf_fit_with_points",
                 "isdf_exchange", "isdf_fit_get", "isdf_fit_info", "isdf_stage_times", "isdf_sync",
                 "isdf_fit_with_candidates", "isdf_fit_selection", "isdf_fit_features",
                 "isdf_mlp_forward", "isdf_mlp_loss_grad", "isdf_mlp_train", "isdf_profile",
                 "isdf_kernel_stats", "isdf_exchange_occ", "isdf_autotune", "isdf_fit_batch",
                 "isdf_exchange_occ_ri", "isdf_grids_for_threshold", "isdf_exchange_universal",
                 "isdf_exchange_occ_ri_noalloc", "isdf_plan_workspace_bytes", "isdf_plan_alloc_stats",
                 "isdf_fit_screen_stats"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(st: int, what: str, allow=()):
    if st != ISDF_OK and st not in allow:
        raise IsdfError(st, f"{what}: {load().isdf_last_error().decode()}")
    return st


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class Plan:
    """A multigrid-ISDF plan for one system (see include/isdf.h)."""

    def __init__(self, sysm, precision: int = FP64, selector: int = SEL_FULL, stream=None,
                 w_batch: int = 0, mlp_weights=None, mlp_keep: float = 2.0,
                 mlp_cutoff: float = 0.05, mixed_mask: int = 0, eager_exchange: bool = False,
                 tune_file=None, universal_all_points: bool = False, universal_tile_mb: int = 0,
                 w_storage: int = W_F64, workspace=None, phi_budget_mb: int = 0,
                 ri_rows: int = 0, ri_screen_tau: float = 0.0):
        lib = load()
        self._keep = []
        s = _System()
        for i, v in enumerate(np.asarray(sysm.lattice, dtype=np.float64).ravel()):
            s.lattice[i] = float(v)
        xyz = np.ascontiguousarray(sysm.xyz, dtype=np.float64)
        sa = np.ascontiguousarray(sysm.shell_atom, dtype=np.int32)
        sl = np.ascontiguousarray(sysm.shell_l, dtype=np.int32)
        sal = np.ascontiguousarray(sysm.shell_alpha, dtype=np.float64)
        grid = np.ascontiguousarray(sysm.grids, dtype=np.int32)
        ab = np.ascontiguousarray(np.asarray(sysm.alpha_bound, dtype=np.float64).reshape(-1))
        if ab.size == 0:
            ab = np.zeros(1)
        self._keep += [xyz, sa, sl, sal, grid, ab]
        s.n_atoms = xyz.shape[0]
        s.xyz = _ptr(xyz, C.c_double)
        s.n_shells = sa.size
        s.shell_atom = _ptr(sa, C.c_int32)
        s.shell_l = _ptr(sl, C.c_int32)
        s.shell_alpha = _ptr(sal, C.c_double)
        s.n_levels = grid.shape[0]
        s.grid = _ptr(grid, C.c_int32)
        s.alpha_bound = _ptr(ab, C.c_double)
        s.image_tol = float(sysm.image_tol)
        s.eps_r = float(sysm.eps_r)
        s.n_mu_ratio = float(sysm.n_mu_ratio)
        s.eps_isdf = float(sysm.eps_isdf)
        s.tie_tol = float(sysm.tie_tol)
        s.domain_mode = int(getattr(sysm, "domain_mode", 0))
        o = _Options()
        o.precision = precision
        o.selector = selector
        o.stream = C.c_void_p(stream) if stream else None
        o.w_batch = w_batch
        if mlp_weights is not None:
            wts = np.ascontiguousarray(mlp_weights, dtype=np.float32)
            assert wts.size == MLP_NPARAM
            self._keep.append(wts)
            o.mlp_weights = _ptr(wts, C.c_float)
        o.mlp_keep = float(mlp_keep)
        o.mlp_cutoff = float(mlp_cutoff)
        o.mixed_mask = int(mixed_mask)
        o.eager_exchange = 1 if eager_exchange else 0
        o.universal_all_points = 1 if universal_all_points else 0
        o.universal_tile_mb = int(universal_tile_mb)
        o.w_storage = int(w_storage)
        o.phi_budget_mb = int(phi_budget_mb)
        o.ri_rows = int(ri_rows)
        o.ri_screen_tau = float(ri_screen_tau)
        if workspace is not None:  # a CUDA tensor the plan carves its device buffers from
            self._keep.append(workspace)
            o.workspace = C.c_void_p(workspace.data_ptr())
            o.workspace_bytes = workspace.numel() * workspace.element_size()
        if tune_file is not None:
            tf = str(tune_file).encode()
            self._keep.append(tf)
            o.tune_file = tf
        h = C.c_void_p()
        _check(lib.isdf_plan(C.byref(s), C.byref(o), C.byref(h)), "isdf_plan")
        self.handle = h
        n_basis, n_mu, nd = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib.isdf_plan_info(h, C.byref(n_basis), C.byref(n_mu), C.byref(nd)), "isdf_plan_info")
        self.n_basis, self.n_mu, self.n_domains = n_basis.value, n_mu.value, nd.value

    def workspace_bytes(self) -> int:
        """High-water mark of the plan's device buffers (isdf_plan_workspace_bytes)."""
        b = C.c_size_t()
        _check(load().isdf_plan_workspace_bytes(self.handle, C.byref(b)), "isdf_plan_workspace_bytes")
        return b.value

    def alloc_stats(self) -> dict:
        """Device blocks taken so far (isdf_plan_alloc_stats)."""
        n, b, ms = C.c_int64(), C.c_double(), C.c_double()
        _check(load().isdf_plan_alloc_stats(self.handle, C.byref(n), C.byref(b), C.byref(ms)),
               "isdf_plan_alloc_stats")
        return dict(calls=n.value, bytes=b.value, ms=ms.value)

    def autotune(self, n_occ: int, reps: int = 3, json_out=None):
        """Time every GEMM tile shape on this plan's problems (one fit and
        both exchange forms) and keep the fastest; optionally write JSON."""
        path = None if json_out is None else str(json_out).encode()
        _check(load().isdf_autotune(self.handle, int(n_occ), int(reps), path), "isdf_autotune")

    def domain(self, d: int) -> dict:
        lib = load()
        lev, atom, nL, nN, nmu = (C.c_int32() for _ in range(5))
        npts = C.c_int64()
        _check(lib.isdf_plan_domain(self.handle, d, C.byref(lev), C.byref(atom), C.byref(npts),
                                    C.byref(nL), C.byref(nN), C.byref(nmu)), "isdf_plan_domain")
        pts = np.zeros(npts.value, dtype=np.int64)
        funcs = np.zeros(nL.value + nN.value, dtype=np.int32)
        _check(lib.isdf_plan_domain_points(self.handle, d, _ptr(pts, C.c_int64)), "points")
        _check(lib.isdf_plan_domain_functions(self.handle, d, _ptr(funcs, C.c_int32)), "functions")
        return dict(level=lev.value, atom=atom.value, points=pts, nL=nL.value, nN=nN.value,
                    n_mu=nmu.value, funcs=funcs)

    def fit(self, points=None, allow_rank=True, candidates=None) -> "Fit":
        lib = load()
        h = C.c_void_p()
        allow = (-5,) if allow_rank else ()
        if candidates is not None:
            flat = np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.int64) for c in candidates]))
            cnt = np.ascontiguousarray([len(c) for c in candidates], dtype=np.int64)
            st = lib.isdf_fit_with_candidates(self.handle, _ptr(flat, C.c_int64), _ptr(cnt, C.c_int64),
                                              C.byref(h))
        elif points is None:
            st = lib.isdf_fit(self.handle, C.byref(h))
        else:
            flat = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.int64) for p in points]))
            st = lib.isdf_fit_with_points(self.handle, _ptr(flat, C.c_int64), C.byref(h))
        if h.value:
            fit = Fit(self, h)
            _check(st, "isdf_fit", allow)
            fit.status = st
            return fit
        _check(st, "isdf_fit")
        raise IsdfError(-3, "isdf_fit returned no handle")

    def stage_times(self) -> np.ndarray:
        t = np.zeros(8)
        _check(load().isdf_stage_times(self.handle, _ptr(t, C.c_double), 8), "isdf_stage_times")
        return t

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().isdf_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grids_for_threshold(lattice, shell_alpha, alpha_bound, eps_K: float) -> np.ndarray:
    """Grid ladder [n_levels, 3] for the Fourier threshold eps_K
    (isdf_grids_for_threshold; host only)."""
    lib = load()
    lat = np.ascontiguousarray(lattice, dtype=np.float64).reshape(9)
    alpha = np.ascontiguousarray(shell_alpha, dtype=np.float64)
    bounds = np.ascontiguousarray(alpha_bound, dtype=np.float64).reshape(-1)
    nlev = bounds.size + 1
    out = np.zeros((nlev, 3), dtype=np.int32)
    _check(lib.isdf_grids_for_threshold(_ptr(lat, C.c_double), alpha.size, _ptr(alpha, C.c_double), nlev,
                                        _ptr(bounds, C.c_double) if bounds.size else None,
                                        float(eps_K), _ptr(out, C.c_int32)),
           "isdf_grids_for_threshold")
    return out.astype(np.int64)


def fit_batch(plans, max_concurrent: int = 4, allow_rank: bool = True):
    """Fits of several plans at once (isdf_fit_batch); returns the list of
    Fit objects in plan order.  Raises on the first failed plan after
    destroying every fit the call made."""
    lib = load()
    n = len(plans)
    hp = (C.c_void_p * n)(*[p.handle.value for p in plans])
    hf = (C.c_void_p * n)()
    sts = (C.c_int * n)()
    st = lib.isdf_fit_batch(hp, n, int(max_concurrent), hf, sts)
    fits = [Fit(p, C.c_void_p(h)) if h else None for p, h in zip(plans, hf)]
    allow = (-5,) if allow_rank else ()
    if st != ISDF_OK and (all(x == ISDF_OK for x in sts) or
                          any(x != ISDF_OK and x not in allow for x in sts)):
        for f in fits:
            if f is not None:
                f.close()
        _check(st, "isdf_fit_batch")
    for f, x in zip(fits, sts):
        if f is not None:
            f.status = x
    return fits


class Fit:
    def __init__(self, plan: Plan, handle):
        self.plan = plan
        self.handle = handle
        n = C.c_int64()
        _check(load().isdf_fit_info(handle, C.byref(n)), "isdf_fit_info")
        self.n_mu = n.value
        self.status = 0

    def selection(self) -> dict:
        nd = self.plan.n_domains
        nc = np.zeros(nd, dtype=np.int64)
        dl = np.zeros(nd)
        df = np.zeros(nd)
        fb = np.zeros(nd, dtype=np.int32)
        _check(load().isdf_fit_selection(self.handle, _ptr(nc, C.c_int64), _ptr(dl, C.c_double),
                                         _ptr(df, C.c_double), _ptr(fb, C.c_int32)), "isdf_fit_selection")
        return dict(n_candidates=nc, last_residual=dl, excluded_max=df, fallback=fb)

    def features(self, with_labels=True):
        """(features [n, 16] float32, labels [n]) as CUDA tensors."""
        import torch

        n = C.c_int64()
        load().isdf_fit_features(self.handle, None, None, 0, C.byref(n))
        X = torch.empty((n.value, 16), dtype=torch.float32, device="cuda")
        Y = torch.empty((n.value,), dtype=torch.float32, device="cuda") if with_labels else None
        _check(load().isdf_fit_features(self.handle, C.c_void_p(X.data_ptr()),
                                        C.c_void_p(Y.data_ptr()) if Y is not None else None,
                                        n.value, C.byref(n)), "isdf_fit_features")
        return X, Y

    def counts(self) -> np.ndarray:
        out = np.zeros(self.plan.n_domains, dtype=np.int64)
        self._get("count", 0, out)
        return out

    def _get(self, field: str, d: int, out: np.ndarray):
        _check(load().isdf_fit_get(self.handle, FIELD[field], d, out.ctypes.data_as(C.c_void_p),
                                   out.nbytes), f"isdf_fit_get({field})")
        return out

    def get(self, field: str, d: int = 0) -> np.ndarray:
        """Copy a stage output to the host (column-major arrays are returned as
        (rows, cols) NumPy arrays)."""
        p = self.plan
        if field in ("XL", "XN"):
            return self._get(field, 0, np.zeros((p.n_basis, self.n_mu))).T
        if field == "W":
            return self._get(field, 0, np.zeros((self.n_mu, self.n_mu))).T
        if field == "count":
            return self.counts()
        dom = p.domain(d)
        npts = dom["points"].size
        cnt = int(self.counts()[d])
        if field == "phi":
            return self._get(field, d, np.zeros((dom["nL"] + dom["nN"], npts))).T
        if field == "diag":
            return self._get(field, d, np.zeros(npts))
        if field == "points":
            return self._get(field, d, np.zeros(cnt, dtype=np.int64))
        if field in ("theta", "F"):
            return self._get(field, d, np.zeros((cnt, npts))).T
        raise KeyError(field)

    def exchange(self, D, K=None):
        """K and E_x for a density D (torch CUDA tensors; K allocated if None).
        Returns (K, e_x)."""
        import torch

        if not isinstance(D, torch.Tensor) or not D.is_cuda or D.dtype != torch.float64:
            raise TypeError("D must be a float64 CUDA tensor")
        D = D.contiguous()
        n = self.plan.n_basis
        if K is None:
            K = torch.empty((n, n), dtype=torch.float64, device=D.device)
        ex = C.c_double()
        _check(load().isdf_exchange(self.plan.handle, self.handle, C.c_void_p(D.data_ptr()),
                                    C.c_void_p(K.data_ptr()), C.byref(ex)), "isdf_exchange")
        return K, ex.value

    def exchange_occ(self, C_occ, K=None):
        """K and E_x for D = C_occ C_occ^T, C_occ an (N, n_occ) float64 CUDA
        tensor (row-major).  Returns (K, e_x)."""
        import torch

        if not isinstance(C_occ, torch.Tensor) or not C_occ.is_cuda or C_occ.dtype != torch.float64:
            raise TypeError("C_occ must be a float64 CUDA tensor")
        C_occ = C_occ.contiguous()
        n = self.plan.n_basis
        if C_occ.dim() != 2 or C_occ.shape[0] != n:
            raise ValueError("C_occ must have shape (N, n_occ)")
        if K is None:
            K = torch.empty((n, n), dtype=torch.float64, device=C_occ.device)
        ex = C.c_double()
        _check(load().isdf_exchange_occ(self.plan.handle, self.handle, C.c_void_p(C_occ.data_ptr()),
                                        int(C_occ.shape[1]), C.c_void_p(K.data_ptr()), C.byref(ex)),
               "isdf_exchange_occ")
        return K, ex.value

    def exchange_occ_ri(self, C_occ, KC=None):
        """K C for D = C C^T without forming K (isdf_exchange_occ_ri); returns
        (KC, e_x) with KC of shape (N, n_occ)."""
        import torch

        if not isinstance(C_occ, torch.Tensor) or not C_occ.is_cuda or C_occ.dtype != torch.float64:
            raise TypeError("C_occ must be a float64 CUDA tensor")
        C_occ = C_occ.contiguous()
        n = self.plan.n_basis
        if C_occ.dim() != 2 or C_occ.shape[0] != n:
            raise ValueError("C_occ must have shape (N, n_occ)")
        if KC is None:
            KC = torch.empty((n, C_occ.shape[1]), dtype=torch.float64, device=C_occ.device)
        elif KC.shape != C_occ.shape or KC.dtype != torch.float64 or not KC.is_contiguous():
            raise ValueError("KC must be a contiguous float64 tensor shaped like C_occ")
        ex = C.c_double()
        _check(load().isdf_exchange_occ_ri(self.plan.handle, self.handle, C.c_void_p(C_occ.data_ptr()),
                                           int(C_occ.shape[1]), C.c_void_p(KC.data_ptr()), C.byref(ex)),
               "isdf_exchange_occ_ri")
        return KC, ex.value

    def screen_kept(self) -> float:
        """Kept tile fraction of the last screened occ-RI exchange."""
        k = C.c_double()
        _check(load().isdf_fit_screen_stats(self.handle, C.byref(k)), "isdf_fit_screen_stats")
        return k.value

    def exchange_occ_ri_noalloc(self, C_occ, KC):
        """K C through isdf_exchange_occ_ri_noalloc (FP64, workspace in the
        library's fixed scratch array; KC caller-allocated like C_occ);
        returns (KC, e_x)."""
        import torch

        if not isinstance(C_occ, torch.Tensor) or not C_occ.is_cuda or C_occ.dtype != torch.float64:
            raise TypeError("C_occ must be a float64 CUDA tensor")
        C_occ = C_occ.contiguous()
        if C_occ.dim() != 2 or C_occ.shape[0] != self.plan.n_basis:
            raise ValueError("C_occ must have shape (N, n_occ)")
        if KC.shape != C_occ.shape or KC.dtype != torch.float64 or not KC.is_contiguous():
            raise ValueError("KC must be a contiguous float64 tensor shaped like C_occ")
        ex = C.c_double()
        _check(load().isdf_exchange_occ_ri_noalloc(self.plan.handle, self.handle,
                                                   C.c_void_p(C_occ.data_ptr()), int(C_occ.shape[1]),
                                                   C.c_void_p(KC.data_ptr()), C.byref(ex)),
               "isdf_exchange_occ_ri_noalloc")
        return KC, ex.value

    def exchange_universal(self, C_occ, KC=None):
        """K_UU C of the universal grid's pairs with every grid point as a
        fitting function (isdf_exchange_universal); returns (KC, e_x) with KC
        of shape (N, n_occ), zero outside the universal domain's functions."""
        import torch

        if not isinstance(C_occ, torch.Tensor) or not C_occ.is_cuda or C_occ.dtype != torch.float64:
            raise TypeError("C_occ must be a float64 CUDA tensor")
        C_occ = C_occ.contiguous()
        n = self.plan.n_basis
        if C_occ.dim() != 2 or C_occ.shape[0] != n:
            raise ValueError("C_occ must have shape (N, n_occ)")
        if KC is None:
            KC = torch.empty((n, C_occ.shape[1]), dtype=torch.float64, device=C_occ.device)
        elif KC.shape != C_occ.shape or KC.dtype != torch.float64 or not KC.is_contiguous():
            raise ValueError("KC must be a contiguous float64 tensor shaped like C_occ")
        ex = C.c_double()
        _check(load().isdf_exchange_universal(self.plan.handle, self.handle, C.c_void_p(C_occ.data_ptr()),
                                              int(C_occ.shape[1]), C.c_void_p(KC.data_ptr()), C.byref(ex)),
               "isdf_exchange_universal")
        return KC, ex.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().isdf_fit_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward(weights, X):
    """Logits of feature rows X (float32 CUDA tensor [n, 16])."""
    import torch

    w = np.ascontiguousarray(weights, dtype=np.float32)
    z = torch.empty((X.shape[0],), dtype=torch.float32, device=X.device)
    _check(load().isdf_mlp_forward(_ptr(w, C.c_float), C.c_void_p(X.data_ptr()), X.shape[0],
                                   C.c_void_p(z.data_ptr()), None), "isdf_mlp_forward")
    return z


def mlp_loss_grad(weights, X, Y, pos_weight):
    w = np.ascontiguousarray(weights, dtype=np.float32)
    g = np.zeros(MLP_NPARAM, dtype=np.float32)
    loss = C.c_float()
    _check(load().isdf_mlp_loss_grad(_ptr(w, C.c_float), C.c_void_p(X.data_ptr()),
                                     C.c_void_p(Y.data_ptr()), X.shape[0], float(pos_weight),
                                     _ptr(g, C.c_float), C.byref(loss), None), "isdf_mlp_loss_grad")
    return float(loss.value), g


def mlp_train(X, Y, weights, epochs=20, batch=65536, lr=1e-3, pos_weight=0.0, seed=0):
    """Train on the GPU; returns (weights float32, per-epoch mean loss)."""
    w = np.ascontiguousarray(weights, dtype=np.float32).copy()
    cfg = _MlpConfig(epochs, batch, lr, 0.9, 0.999, 1e-8, float(pos_weight), seed, None)
    hist = np.zeros(epochs, dtype=np.float32)
    _check(load().isdf_mlp_train(C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), X.shape[0],
                                 C.byref(cfg), _ptr(w, C.c_float), _ptr(hist, C.c_float)),
           "isdf_mlp_train")
    return w, hist
