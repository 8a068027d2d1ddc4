"""Coulomb metric held in FP32 (w_storage = ISDF_W_F32) against the FP64 W
and the oracle.  W itself: the stored values are the FP64 metric rounded to
FP32 (bitwise, the fit being deterministic).  Exchange: the Hadamard factor
W is rounded to 24 bits, so K moves by at most ~2^-24 of its terms; the gate
is |dE_x| <= 1e-6 Ha/atom against the oracle and max|dK| <= 1e-6 Ha."""
import numpy as np
import pytest

from oracle import pipeline
from paper_2404_09373_amd import binding
from workloads import config, tiny_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.mark.parametrize("which", ["cfg1", "d_two"])
def test_w_fp32_storage(torch, which, cfg1_oracle):
    if which == "cfg1":
        s, ref = cfg1_oracle
    else:
        s = tiny_system("d_two", n_occ=3)
        ref = pipeline.run(s)
    p64 = binding.Plan(s)
    p32 = binding.Plan(s, w_storage=binding.W_F32)
    f64 = p64.fit()
    f32 = p32.fit()
    W64 = f64.get("W")
    W32 = f32.get("W")
    assert np.array_equal(W32, W64.astype(np.float32).astype(np.float64))
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    K64, e64 = f64.exchange(D)
    K32, e32 = f32.exchange(D)
    dK = float(np.max(np.abs(K32.cpu().numpy() - ref.K)))
    dE = abs(e32 - ref.E_x) / s.n_atoms
    print(f"[{which} W fp32] max|dK| {dK:.2e} |dE|/atom {dE:.2e} (fp64 W: "
          f"{np.max(np.abs(K64.cpu().numpy() - ref.K)):.2e})")
    assert dK <= 1e-6 and dE <= 1e-6
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    KC = torch.empty_like(C)
    _, e_ri = f32.exchange_occ_ri(C, KC)
    assert abs(e_ri - ref.E_x) / s.n_atoms <= 1e-6
    ref_kc = ref.K @ s.C_occ
    assert np.max(np.abs(KC.cpu().numpy() - ref_kc)) <= 1e-6


def test_w_fp32_with_mixed_exchange(torch, cfg1_oracle):
    """FP32 W with the BF16-split (x6) exchange: the 1e-6 Ha/atom gate."""
    s, ref = cfg1_oracle
    plan = binding.Plan(s, precision=binding.MIXED_X6, w_storage=binding.W_F32)
    fit = plan.fit()
    C = torch.tensor(s.C_occ, dtype=torch.float64, device="cuda")
    K = torch.empty((s.n_basis, s.n_basis), dtype=torch.float64, device="cuda")
    _, e = fit.exchange_occ(C, K)
    dE = abs(e - ref.E_x) / s.n_atoms
    dK = float(np.max(np.abs(K.cpu().numpy() - ref.K)))
    print(f"[cfg1 x6 + W fp32] max|dK| {dK:.2e} |dE|/atom {dE:.2e}")
    assert dE <= 1e-6 and dK <= 1e-5
