"""Density screening of the occ-RI exchange (ri_screen_tau) with localised
bond orbitals, against the oracle's screened form (exchange_occ_ri_screened):
the same tiles kept, K C equal to 1e-10 relative, the change from the
unscreened K C within the oracle's elementwise bound, and row blocks equal
to one block."""
import numpy as np
import pytest

from oracle import exchange, pipeline
from paper_2404_09373_amd import binding
from workloads import bond_orbitals, config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def bonds_cfg1():
    s = config(1)
    s.C_occ, s.D, _ = bond_orbitals(s)
    return s, pipeline.run(s)


def _tau_in_gap(B, q):
    """A threshold near quantile q of the tile bounds, placed in the widest
    relative gap between neighbouring bounds there, so that no bound lies
    within rounding of it."""
    v = np.sort(np.unique(B[B > 0]))
    i0 = int(q * len(v))
    lo, hi = max(1, i0 - 20), min(len(v) - 1, i0 + 20)
    gaps = v[lo:hi + 1] / v[lo - 1:hi]
    j = lo + int(np.argmax(gaps))
    return float(np.sqrt(v[j - 1] * v[j]))


def test_screened_occ_ri_matches_oracle(torch, bonds_cfg1):
    s, r = bonds_cfg1
    B = np.concatenate([b.ravel() for b in exchange.occ_ri_tile_bounds(r.XL, r.XN, r.W, s.C_occ, 64)])
    tau = _tau_in_gap(B, 0.4)
    ref, bound, kept = exchange.exchange_occ_ri_screened(r.XL, r.XN, r.W, s.C_occ, 64, tau)
    full = exchange.exchange_occ_ri(r.XL, r.XN, r.W, s.C_occ)
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    out = {}
    for rows in (0, 192):
        plan = binding.Plan(s, ri_screen_tau=tau, ri_rows=rows)
        fit = plan.fit()
        KC = torch.empty_like(C)
        _, e = fit.exchange_occ_ri(C, KC)
        _, e2 = fit.exchange_occ_ri(C, KC)  # replayed graph
        assert e2 == e
        out[rows] = (KC.cpu().numpy(), e, fit.screen_kept())
        fit.close()
        plan.close()
    plain = binding.Plan(s)
    pf = plain.fit()
    KC0 = torch.empty_like(C)
    pf.exchange_occ_ri(C, KC0)
    KC0 = KC0.cpu().numpy()
    pf.close()
    plain.close()
    KC, e, kept_gpu = out[0]
    scale = float(np.max(np.abs(ref)))
    d_ref = float(np.max(np.abs(KC - ref))) / scale
    d_blk = float(np.max(np.abs(out[192][0] - KC))) / scale
    change = np.abs(KC - KC0)
    print(f"[screen cfg1] tau {tau:.3e} kept {kept_gpu:.3f} (oracle {kept:.3f}); vs oracle screened {d_ref:.2e}; "
          f"row blocks {d_blk:.2e}; max change {np.max(change):.2e} (bound max {np.max(bound):.2e})")
    assert abs(kept_gpu - kept) <= 1e-12 and out[192][2] == kept_gpu
    assert d_ref <= 1e-10 and d_blk <= 1e-12
    assert np.max(change) > 0.0
    assert np.all(change <= bound + 1e-10 * scale)
    assert np.max(np.abs(full - KC0)) <= 1e-10 * scale
