"""Whole multigrid-ISDF fit and exchange build in FP64, stage by stage.

Stages (with wall-clock timers, used for the CPU baseline):
  basis      basis values on every domain
  diag       Gram diagonal
  select     pivoted-Cholesky points
  fit        Theta, M_xi, F = Theta M_xi^{-1}
  coulomb    W by FFT Poisson solves
  exchange   K and E_x
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import basis, isdf
from .coulomb import coulomb_metric
from .exchange import build_X, exchange_energy, exchange_matrix
from .plan import Plan, build_plan


@dataclasses.dataclass
class OracleResult:
    plan: Plan
    pivots: List[np.ndarray]  # per domain, local point indices in selection order
    F: List[np.ndarray]
    XL: np.ndarray
    XN: np.ndarray
    W: np.ndarray
    K: Optional[np.ndarray]
    E_x: Optional[float]
    times: Dict[str, float]
    diag: List[np.ndarray]


def run(sysm, pinned: Optional[List[np.ndarray]] = None, domains=None,
        with_exchange: bool = True, workers: int = -1, plan: Optional[Plan] = None) -> OracleResult:
    """Full oracle.  `pinned[d]` (local point indices) replaces the selection
    of domain d when given."""
    times = {k: 0.0 for k in ("plan", "basis", "diag", "select", "fit", "coulomb", "exchange")}
    t = time.perf_counter()
    if plan is None:
        plan = build_plan(sysm)
    times["plan"] = time.perf_counter() - t
    piv_list, F_list, rows_list, diag_list = [], [], [], []
    for d, dom in enumerate(plan.domains):
        t = time.perf_counter()
        Phi = basis.domain_values(plan, dom)
        times["basis"] += time.perf_counter() - t
        nL = dom.L.size
        t = time.perf_counter()
        dg = isdf.gram_diag(Phi, nL)
        times["diag"] += time.perf_counter() - t
        diag_list.append(dg)
        t = time.perf_counter()
        # a count-driven domain (ratio > 0) capped at its point count; in the
        # threshold-only mode the cap is an upper limit and eps_isdf stops it
        all_pts = pinned is None and sysm.n_mu_ratio > 0 and dom.n_mu >= dom.points.size
        if pinned is not None:
            piv = np.asarray(pinned[d], dtype=np.int64)
        elif all_pts:
            # every point of the domain requested: the points themselves are
            # the interpolation points and F = I (no selection, no solve)
            piv = np.arange(dom.points.size, dtype=np.int64)
        else:
            piv, _, _, _ = isdf.pivoted_cholesky(Phi, nL, dom.n_mu, sysm.eps_isdf, sysm.tie_tol)
        times["select"] += time.perf_counter() - t
        t = time.perf_counter()
        if all_pts:
            F = np.eye(dom.points.size)
        else:
            F, _, _ = isdf.fit_functions(Phi, nL, piv)
        times["fit"] += time.perf_counter() - t
        piv_list.append(piv)
        F_list.append(F)
        rows_list.append(Phi[piv, :])
    XL, XN = build_X(plan, piv_list, rows_list)
    t = time.perf_counter()
    W = coulomb_metric(plan, F_list, workers)
    times["coulomb"] = time.perf_counter() - t
    K = E = None
    if with_exchange and sysm.D is not None:
        t = time.perf_counter()
        K = exchange_matrix(XL, XN, W, sysm.D)
        E = exchange_energy(sysm.D, K)
        times["exchange"] = time.perf_counter() - t
    return OracleResult(plan, piv_list, F_list, XL, XN, W, K, E, times, diag_list)
