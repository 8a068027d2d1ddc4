"""GEMM tile-shape tuning on the GPU: the table is written, read back by a
new plan, and a tuned plan gives bit-identical results (the shapes change
the speed only)."""
import json

import numpy as np
import pytest

from paper_2404_09373_amd import binding
from workloads import config

pytestmark = pytest.mark.gpu


def test_autotune_roundtrip(tmp_path):
    import torch

    s = config(1)
    path = tmp_path / "tune.json"
    p0 = binding.Plan(s, eager_exchange=True)
    p0.autotune(s.n_occ, reps=1, json_out=path)
    table = json.loads(path.read_text())
    assert table["entries"], "no GEMM class met"
    for e in table["entries"]:
        assert 0 <= e["shape"] < len(table["shapes"])
        valid = [t for t in e["us"] if t >= 0]
        assert e["us"][e["shape"]] == min(valid)
    print(f"[tune] {len(table['entries'])} classes")
    p1 = binding.Plan(s, eager_exchange=True, tune_file=path)
    D = torch.tensor(s.D, dtype=torch.float64, device="cuda")
    f0, f1 = p0.fit(), p1.fit()
    K0, e0 = f0.exchange(D)
    K1, e1 = f1.exchange(D)
    assert torch.equal(K0, K1) and e0 == e1
    assert np.array_equal(f0.get("W"), f1.get("W"))
    for f in (f0, f1):
        f.close()
    for p in (p0, p1):
        p.close()
