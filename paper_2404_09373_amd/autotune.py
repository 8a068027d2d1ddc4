"""Write the FP64 GEMM tile-shape table for a workload.

    python -m paper_2404_09373_amd.autotune --config 2 --out paper_2404_09373_amd/tune/gfx950.json

Runs isdf_autotune on an FP64 plan of the workload (its fit and both
exchange forms meet every FP64 GEMM class the mixed-precision plans use
too) and writes the table that plans read through `tune_file`.
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune", "gfx950.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=DEFAULT)
    args = ap.parse_args()

    import torch

    from paper_2404_09373_amd import binding
    from workloads import config

    assert torch.cuda.is_available(), "tuning needs the GPU"
    s = config(args.config)
    plan = binding.Plan(s, stream=torch.cuda.current_stream().cuda_stream)
    plan.autotune(s.n_occ, reps=args.reps, json_out=args.out)
    plan.close()
    with open(args.out) as f:
        table = json.load(f)
    print(f"wrote {len(table['entries'])} GEMM classes to {args.out}", flush=True)


if __name__ == "__main__":
    main()
