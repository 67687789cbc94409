"""Benchmark of the CDG2 plaque operator on one MI355X.

One step = one SSP-RK3 time step (three fused operator + stage launches) of the
six-species model on the 64^3 hex grid with the Q2 basis (42,467,328 DOF,
float64), inputs resident in HBM.  Prints ONE JSON line.

  value        operator GDOF/s = 3 * DOF * steps / seconds (three operator
               applications per step)
  roofline     the fused stage kernel against the 8 TB/s HBM peak: algorithmic
               bytes per step (64 B/DOF: stage 1 reads U and writes U1, stages 2
               and 3 read two states and write one) / measured time per step
  cpu_baseline the float64 oracle (test infrastructure) timed on the host cores
               for one operator application of the same workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (dim, n, p, seed key)
    "3d-q2-64": (3, (64, 64, 64), 2, (2,)),
    "2d-q2-256": (2, (256, 256), 2, (1,)),
    "2d-q4-256": (2, (256, 256), 4, (1,)),
    "2d-q1-16": (2, (16, 16), 1, (0,)),
}
HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1403_1157_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str):
    """HBM traffic per step from the committed rocprofv3 --pmc summary of this
    workload, if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"op_kernel_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["bytes_per_step"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(dim, n, p, key, dof):
    """Oracle (float64, CPU) on the same workload: one operator application."""
    import torch

    from oracle.cdg2_oracle import Config, Oracle
    from paper_1403_1157_amd import inputs

    threads = torch.get_num_threads()
    U = torch.from_numpy(inputs.initial_modes(dim, n, p, key))
    o = Oracle(Config(dim=dim, n=n, order=p, coeffs=inputs.base_coeffs()))
    t = time.perf_counter()
    o.apply(U)
    sec = time.perf_counter() - t
    return {"value": round(dof / sec / 1e9, 6), "unit": "GDOF/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one float64 oracle operator application on the full workload "
                      f"({dof} DOF) in {sec:.2f} s; GDOF/s = DOF / seconds"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="3d-q2-64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(max(1, args.steps)):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": max(1, args.steps)}))
        return

    from paper_1403_1157_amd import inputs
    from paper_1403_1157_amd.cdg2 import Operator

    dim, n, p, key = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    U0 = torch.from_numpy(inputs.initial_modes(dim, n, p, key)).to(dev).contiguous()
    dof = U0.numel()
    op = Operator(dim, n, p, inputs.base_coeffs())
    dt = op.max_dt(U0, 0.9)
    U = U0.clone()
    out = torch.empty_like(U0)

    for _ in range(args.warmup):
        op.rk_step(U, dt, 1)
    op.sync()

    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        op.rk_step(U, dt, 1)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    op.sync()

    # operator-only launches (apply_operator, 16 B/DOF) for the plain form
    for _ in range(2):
        op.apply(U0, out)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        op.apply(U0, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_apply = ev0.elapsed_time(ev1) / args.steps
    op.sync()

    value = 3 * dof / (ms_step * 1e-3) / 1e9
    alg_bytes_step = 64.0 * dof
    achieved = alg_bytes_step / (ms_step * 1e-3) / 1e9
    traffic = read_traffic(args.workload)
    line = {
        "metric": "CDG2 operator GDOF/s (SSP-RK3 stage applications, FP64)",
        "value": round(value, 4),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: six-species CDG2 plaque model, "
                               f"{'x'.join(map(str, n))} cells, Q{p}, one SSP-RK3 step",
                   "dim": dim, "cells": list(n), "order": p, "dof": dof, "dt": dt},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": traffic},
        "apply": {"us_per_apply": round(ms_apply * 1e3, 2),
                  "gdof_s": round(dof / (ms_apply * 1e-3) / 1e9, 4),
                  "alg_gb_s": round(16.0 * dof / (ms_apply * 1e-3) / 1e9, 2)},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(dim, n, p, key, dof)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
