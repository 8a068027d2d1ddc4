"""Host-side checks of the C ABI (no GPU): the library loads, exports every
declared symbol, builds the same multigrid plan as the oracle, and returns the
documented status codes for bad input."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import plan as oplan
from paper_2404_09373_amd import binding
from workloads import batched_cells, config, tiny_system

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    hdr = open(os.path.join(ROOT, "include", "isdf.h")).read()
    names = set(re.findall(r"\b(isdf_[a-z_]+)\s*\(", hdr))
    assert names, "no declarations found"
    for n in sorted(names):
        assert hasattr(lib, n), f"{n} declared in isdf.h but not exported"
    assert set(binding.EXPORTED) <= names


def _compare_plan(sysm):
    p = binding.Plan(sysm)
    op = oplan.build_plan(sysm)
    assert p.n_basis == op.n_basis
    assert p.n_domains == len(op.domains)
    assert p.n_mu == op.n_mu
    for d in range(p.n_domains):
        g = p.domain(d)
        od = op.domains[d]
        assert g["level"] == od.level and g["atom"] == od.atom
        assert g["nL"] == od.L.size and g["nN"] == od.N.size and g["n_mu"] == od.n_mu
        assert np.array_equal(g["points"], od.points), f"domain {d} points"
        assert np.array_equal(g["funcs"], od.G), f"domain {d} functions"
    p.close()


@pytest.mark.parametrize("which", ["cfg1", "tiny1", "tiny2", "strained", "d_two", "full_cell"])
def test_plan_matches_oracle(which):
    if which == "cfg1":
        s = config(1, with_density=False)
    elif which == "tiny1":
        s = tiny_system("one_atom")
    elif which == "tiny2":
        s = tiny_system("two_atom")
    elif which == "d_two":
        s = tiny_system("d_two")
    elif which == "full_cell":
        s = tiny_system("d_two", grids=((10, 10, 10), (20, 20, 20)))
        s.domain_mode = 1
    else:
        s = batched_cells(4)[3]  # 2x2x2 strained cell, uneven grids
        s.grids = np.array([[24, 48, 40], [48, 96, 80]])
    _compare_plan(s)


def test_plan_threshold_only_matches_oracle():
    """n_mu_ratio <= 0: every domain's point cap is the rank bound of its
    pair Gram, the same in both plans."""
    s = config(1, with_density=False)
    s.n_mu_ratio = 0.0
    s.grids = oplan.grids_for_threshold(s.lattice, s.shell_alpha, s.alpha_bound, 1e-2)
    _compare_plan(s)


_LADDER_SYSTEMS = [config(1, with_density=False), config(2, with_density=False),
                   config(4, with_density=False)] + batched_cells(4, with_density=False)


@pytest.mark.parametrize("eps_K", [0.3, 1e-2, 1e-3, 1e-5, 1e-8])
def test_grids_for_threshold_match_oracle(eps_K):
    """isdf_grids_for_threshold gives the oracle's ladder exactly (cubic,
    supercell and strained cells; the 216-atom cell at 1e-8 exceeds 256
    points on both sides)."""
    for s in _LADDER_SYSTEMS:
        ref = oplan.grids_for_threshold(s.lattice, s.shell_alpha, s.alpha_bound, eps_K)
        if ref.max() > 256:
            with pytest.raises(binding.IsdfError) as e:
                binding.grids_for_threshold(s.lattice, s.shell_alpha, s.alpha_bound, eps_K)
            assert e.value.status == -7
            continue
        got = binding.grids_for_threshold(s.lattice, s.shell_alpha, s.alpha_bound, eps_K)
        assert np.array_equal(got, ref), f"{s.name} eps_K {eps_K}: {got.tolist()} vs {ref.tolist()}"


def test_grids_for_threshold_oblique_cell_matches_oracle():
    lat = np.array([[7.0, 0.0, 0.0], [3.5, 3.0, 0.0], [1.0, 1.0, 4.0]])
    for a, e in [(0.8, 1e-2), (0.8, 1e-4), (0.3, 1e-3), (1.2, 1e-6)]:
        alphas = [0.1, a, 2.5 * a]
        ref = oplan.grids_for_threshold(lat, alphas, [a * 1.01], e)
        assert np.array_equal(binding.grids_for_threshold(lat, alphas, [a * 1.01], e), ref)


def test_grids_for_threshold_errors():
    lat = np.eye(3) * 6.74
    for alphas, bounds, eps in [([0.3], [], 0.0), ([0.3], [], 1.0), ([0.3, -1.0], [], 1e-2),
                                ([0.15, 0.3], [2.0], 1e-2)]:
        with pytest.raises(binding.IsdfError) as e:
            binding.grids_for_threshold(lat, alphas, bounds, eps)
        assert e.value.status == -1
    with pytest.raises(binding.IsdfError) as e:
        binding.grids_for_threshold(np.zeros((3, 3)), [0.3], [], 1e-2)
    assert e.value.status == -1
    with pytest.raises(binding.IsdfError) as e:
        binding.grids_for_threshold(lat, [400.0], [], 1e-12)
    assert e.value.status == -7
    lib = binding.load()
    out = np.full(3, -5, dtype=np.int32)
    alpha = np.array([0.3])
    assert lib.isdf_grids_for_threshold(None, 1, binding._ptr(alpha, C.c_double), 1, None, 1e-2,
                                        binding._ptr(out, C.c_int32)) == -1
    assert np.all(out == -5)  # untouched on error


@pytest.mark.slow
def test_plan_matches_oracle_cfg2():
    _compare_plan(config(2, with_density=False))


def _system_struct(sysm):
    """The C system struct of a workload (arrays kept alive on the struct)."""
    import ctypes as C
    s = binding._System()
    for i, v in enumerate(np.asarray(sysm.lattice, dtype=np.float64).ravel()):
        s.lattice[i] = float(v)
    keep = [np.ascontiguousarray(sysm.xyz, dtype=np.float64), np.ascontiguousarray(sysm.shell_atom, dtype=np.int32),
            np.ascontiguousarray(sysm.shell_l, dtype=np.int32), np.ascontiguousarray(sysm.shell_alpha, dtype=np.float64),
            np.ascontiguousarray(sysm.grids, dtype=np.int32),
            np.ascontiguousarray(np.asarray(sysm.alpha_bound, dtype=np.float64).reshape(-1))]
    s._keep = keep
    s.n_atoms = keep[0].shape[0]
    s.xyz = binding._ptr(keep[0], C.c_double)
    s.n_shells = keep[1].size
    s.shell_atom = binding._ptr(keep[1], C.c_int32)
    s.shell_l = binding._ptr(keep[2], C.c_int32)
    s.shell_alpha = binding._ptr(keep[3], C.c_double)
    s.n_levels = keep[4].shape[0]
    s.grid = binding._ptr(keep[4], C.c_int32)
    s.alpha_bound = binding._ptr(keep[5], C.c_double)
    s.image_tol, s.eps_r, s.n_mu_ratio = sysm.image_tol, sysm.eps_r, sysm.n_mu_ratio
    s.eps_isdf, s.tie_tol = sysm.eps_isdf, sysm.tie_tol
    return s


def _status(sysm, **over):
    for k, v in over.items():
        setattr(sysm, k, v)
    with pytest.raises(binding.IsdfError) as e:
        binding.Plan(sysm)
    return e.value.status


def test_plan_errors():
    assert _status(tiny_system("one_atom"), grids=np.array([[12, 12, 12], [26, 24, 24]])) == -7
    assert _status(tiny_system("one_atom"), grids=np.array([[24, 24, 24], [12, 12, 12]])) == -7
    s = tiny_system("one_atom")
    s.shell_alpha = s.shell_alpha.copy()
    s.shell_alpha[1] = np.nan
    assert _status(s) == -1
    s = tiny_system("one_atom")
    s.shell_l = s.shell_l.copy()
    s.shell_l[0] = 3
    assert _status(s) == -7
    s = tiny_system("one_atom")
    s.domain_mode = 2
    assert _status(s) == -1
    with pytest.raises(binding.IsdfError) as e:
        binding.Plan(tiny_system("one_atom"), w_storage=2)
    assert e.value.status == -1
    for kw in (dict(phi_budget_mb=-1), dict(ri_rows=-5), dict(ri_screen_tau=-1.0)):
        with pytest.raises(binding.IsdfError) as e:
            binding.Plan(tiny_system("one_atom"), **kw)
        assert e.value.status == -1
    # density screening runs on the FP64 exchange only
    with pytest.raises(binding.IsdfError) as e:
        binding.Plan(tiny_system("one_atom"), precision=binding.MIXED_X6, ri_screen_tau=1e-6)
    assert e.value.status == -7
    binding.Plan(tiny_system("one_atom"), precision=binding.MIXED_X6, mixed_mask=binding.MIX_W,
                 ri_screen_tau=1e-6).close()
    # a workspace needs an aligned pointer and a size (checked on the host)
    import ctypes as C
    s = binding._System()
    o = binding._Options()
    o.workspace = C.c_void_p(0x1001)
    o.workspace_bytes = 1 << 20
    h = C.c_void_p()
    sysm = tiny_system("one_atom")
    p = binding.Plan(sysm)  # a valid system struct to reuse
    p.close()
    lib = binding.load()
    o2 = binding._Options()
    o2.workspace_bytes = 1 << 20  # size without a pointer
    for opt in (o, o2):
        st = lib.isdf_plan(C.byref(_system_struct(sysm)), C.byref(opt), C.byref(h))
        assert st == -1 and not h.value
    assert _status(tiny_system("one_atom"), lattice=np.zeros((3, 3))) == -1
    assert _status(tiny_system("one_atom"), image_tol=0.0) == -1


def test_null_arguments():
    lib = binding.load()
    h = C.c_void_p()
    assert lib.isdf_plan(None, None, C.byref(h)) == -1
    assert lib.isdf_plan_info(None, None, None, None) == -1
    assert lib.isdf_fit(None, C.byref(h)) == -1
    assert lib.isdf_exchange(None, None, None, None, None) == -1
    assert lib.isdf_last_error()


def test_tune_file_errors(tmp_path):
    """The plan reads the tile-shape table at creation (no GPU work):
    missing files and out-of-range shapes are argument errors."""
    from paper_2404_09373_amd import binding
    from workloads import tiny_system

    s = tiny_system("one_atom")
    with pytest.raises(binding.IsdfError) as e:
        binding.Plan(s, tune_file=tmp_path / "missing.json")
    assert e.value.status == -1
    bad = tmp_path / "bad.json"
    bad.write_text('{"arch": "gfx950", "entries": [{"key": "e0 t1", "shape": 99}]}')
    with pytest.raises(binding.IsdfError) as e:
        binding.Plan(s, tune_file=bad)
    assert e.value.status == -1
    good = tmp_path / "good.json"
    good.write_text('{"arch": "gfx950", "entries": [{"key": "e0 t1 l0 a0 b0 c0 g0 m5 n5 k5", "shape": 2}]}')
    binding.Plan(s, tune_file=good).close()
