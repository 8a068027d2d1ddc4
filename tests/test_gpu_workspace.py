"""Caller-owned workspace (isdf_options.workspace): a plan sized by
isdf_plan_workspace_bytes after one fit and exchange repeats them inside
the caller's buffer with the same results, and a too-small buffer fails
cleanly with ISDF_E_NOMEM."""
import numpy as np
import pytest

from paper_2404_09373_amd import binding
from workloads import config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _run(torch, s, plan):
    fit = plan.fit()
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    K, e = fit.exchange(D)
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    KC = torch.empty_like(C)
    _, e_ri = fit.exchange_occ_ri(C, KC)
    out = (K.cpu().numpy(), e, KC.cpu().numpy(), e_ri, fit.get("W"))
    fit.close()
    return out


def test_workspace_repeats_fit_and_exchange(torch):
    s = config(1)
    ref_plan = binding.Plan(s)
    ref = _run(torch, s, ref_plan)
    need = ref_plan.workspace_bytes()
    print(f"workspace bytes {need / 2**20:.1f} MiB", flush=True)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    plan = binding.Plan(s, workspace=ws)
    got = _run(torch, s, plan)
    assert plan.workspace_bytes() <= need
    for a, b in ((ref[0], got[0]), (ref[2], got[2]), (ref[4], got[4])):
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
    assert abs(ref[1] - got[1]) <= 1e-13 * abs(ref[1])
    plan.close()
    # a second round in the same workspace (blocks come back from the cache)
    plan = binding.Plan(s, workspace=ws)
    again = _run(torch, s, plan)
    assert np.max(np.abs(again[0] - ref[0])) <= 1e-13 * np.max(np.abs(ref[0]))
    plan.close()


def test_workspace_too_small_is_nomem(torch):
    s = config(1)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    plan = binding.Plan(s, workspace=ws)
    with pytest.raises(binding.IsdfError) as e:
        plan.fit()
    assert e.value.status == -2
    plan.close()
