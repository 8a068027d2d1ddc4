"""Per-family kernel instrumentation on the GPU (isdf_profile,
isdf_kernel_stats), on which the benchmark's roofline figures rest.

* Bracketing launches with events changes no result: a fit and an exchange
  with every family bracketed equal, bitwise, the same work unbracketed.
* Every family the 8-atom path runs reports launches, device time and its
  algorithmic work (bytes for the HBM-bound families, flops for the GEMMs).
  That cell's universal domain takes 528 pivots, so the candidate-restricted
  selection (its own family) runs beside the batched window selection.
* A mask counts only its own families, a reset clears every counter, and
  out-of-range families and a null plan are refused.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2404_09373_amd import binding
from workloads import config

pytestmark = pytest.mark.gpu

NFAM = 9  # ISDF_K_NFAMILY
ALL = (1 << NFAM) - 1
HBM_FAMILIES = (0, 1, 6, 7, 8)  # select_column, select_pick, fft, basis, select_block
GEMM_FAMILIES = (2, 3, 4, 5)  # gemm_select, gemm_metric, gemm_fit, gemm_exchange
FFT, SELECT_BLOCK = 6, 8


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


def stats(lib, plan):
    out = []
    for f in range(NFAM):
        ms, n, by, fl = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
        assert lib.isdf_kernel_stats(plan.handle, f, C.byref(ms), C.byref(n), C.byref(by), C.byref(fl)) == 0
        out.append((ms.value, n.value, by.value, fl.value))
    return out


def run(torch, plan, s):
    fit = plan.fit()
    Cocc = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    K, e = fit.exchange_occ(Cocc)
    torch.cuda.synchronize()
    fit.close()
    return K.cpu().numpy(), e


def test_bracketing_changes_no_result_and_counts_every_family(torch):
    s = config(1)
    lib = binding.load()
    plain = binding.Plan(s, eager_exchange=True)
    prof = binding.Plan(s, eager_exchange=True)
    assert lib.isdf_profile(prof.handle, ALL) == 0
    K0, e0 = run(torch, plain, s)
    K1, e1 = run(torch, prof, s)
    print(f"[instrumentation] E_x {e0:.15f} / bracketed {e1:.15f}")
    assert np.array_equal(K0, K1) and e0 == e1
    st = stats(lib, prof)
    for f, (ms, n, by, fl) in enumerate(st):
        print(f"[instrumentation] family {f}: {n} launches, {ms:.3f} ms, {by:.3e} B, {fl:.3e} flop")
        assert n > 0 and ms > 0.0, f"family {f} reported no launches"
        if f in HBM_FAMILIES:
            assert by > 0.0
        if f in GEMM_FAMILIES:
            assert fl > 0.0
    # nothing of the unbracketed plan was counted
    assert all(n == 0 and ms == 0.0 for ms, n, _, _ in stats(lib, plain))
    plain.close()
    prof.close()


def test_mask_reset_and_bad_arguments(torch):
    s = config(1)
    lib = binding.load()
    plan = binding.Plan(s, eager_exchange=True)
    assert lib.isdf_profile(plan.handle, (1 << FFT) | (1 << SELECT_BLOCK)) == 0
    run(torch, plan, s)
    st = stats(lib, plan)
    for f, (ms, n, _, _) in enumerate(st):
        if f in (FFT, SELECT_BLOCK):
            assert n > 0 and ms > 0.0
        else:
            assert n == 0 and ms == 0.0, f"family {f} counted outside the mask"
    # a reset clears the counters and, with mask 0, nothing is counted again
    assert lib.isdf_profile(plan.handle, 0) == 0
    assert all(v == 0 for row in stats(lib, plan) for v in row)
    run(torch, plan, s)
    assert all(v == 0 for row in stats(lib, plan) for v in row)
    ms, n, by, fl = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    for bad in (-1, NFAM):
        assert lib.isdf_kernel_stats(plan.handle, bad, C.byref(ms), C.byref(n), C.byref(by), C.byref(fl)) == -1
    assert lib.isdf_profile(None, ALL) == -1
    plan.close()
