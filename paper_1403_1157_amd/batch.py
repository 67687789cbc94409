"""Batched instances: packed state, persistent-launch SSP-RK3 and its autotuner.

The arithmetic runs in libcdg2 (cdg2_batch_*).  This module packs and unpacks
torch tensors and picks the launch schedule: :meth:`Batch.autotune` times every
candidate (cells per work item, persistent workgroup count, item order) on the
caller's packed state and keeps the fastest, caching the choice in a JSON file
keyed by the GPU architecture and the batch's (grid, order) signature.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import cdg2 as B

CANDIDATE_EB = (16, 32, 64)
CANDIDATE_WG_PER_CU = (0, 1, 2, 4)         # 0 = one workgroup per item
CANDIDATE_ORDER = (0, 1)                   # cost-sorted, instance order


def default_cache_path() -> str:
    return os.environ.get("CDG2_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "cdg2_autotune.json"))


class Batch:
    def __init__(self, instances):
        """instances: list of dicts with keys n (2-tuple), order (1..3), coeffs."""
        self.instances = instances
        cfgs = [B.make_config(2, inst["n"], inst["order"], inst["coeffs"]) for inst in instances]
        self.b = B.cdg2_batch_create(cfgs)
        self.count = len(instances)
        self.total = B.cdg2_batch_num_dofs(self.b)
        self.offsets = [B.cdg2_batch_offset(self.b, i) for i in range(self.count)]
        self.shapes = []
        for inst in instances:
            E = inst["n"][0] * inst["n"][1]
            self.shapes.append((6, E, (inst["order"] + 1) ** 2))
        self.schedule = (32, 0, 0)

    def signature(self) -> str:
        s = ";".join(f"{i['n'][0]}x{i['n'][1]}p{i['order']}" for i in self.instances)
        return hashlib.sha256(s.encode()).hexdigest()[:16]

    def pack(self, states) -> torch.Tensor:
        out = torch.empty(self.total, dtype=torch.float64, device=states[0].device)
        for off, shp, x in zip(self.offsets, self.shapes, states):
            n = shp[0] * shp[1] * shp[2]
            out[off:off + n] = x.reshape(-1)
        return out

    def view(self, packed: torch.Tensor, i: int) -> torch.Tensor:
        shp = self.shapes[i]
        n = shp[0] * shp[1] * shp[2]
        return packed[self.offsets[i]:self.offsets[i] + n].view(shp)

    def _stream(self):
        B.cdg2_batch_set_stream(self.b, torch.cuda.current_stream().cuda_stream)

    def set_schedule(self, eb: int, nwg: int, order: int) -> None:
        B.cdg2_batch_set_schedule(self.b, eb, nwg, order)
        self.schedule = (eb, nwg, order)

    def rk(self, packed: torch.Tensor, dts, nsteps: int, graph: bool = True) -> torch.Tensor:
        if not (packed.is_cuda and packed.dtype == torch.float64 and packed.is_contiguous()
                and packed.numel() == self.total):
            raise ValueError("expected the packed float64 CUDA state")
        self._stream()
        B.cdg2_batch_rk(self.b, packed.data_ptr(), dts, nsteps, graph)
        return packed

    def sync(self) -> None:
        self._stream()
        B.cdg2_batch_sync(self.b)

    def autotune(self, packed: torch.Tensor, dts, cache_path: str | None = None, reps: int = 3):
        """Pick the fastest schedule for this batch (timed on a scratch copy of the
        packed state, one SSP-RK3 step per trial)."""
        cache_path = cache_path or default_cache_path()
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        key = f"{arch}:{self.signature()}"
        cache = {}
        if os.path.exists(cache_path):
            try:
                with open(cache_path) as f:
                    cache = json.load(f)
            except (OSError, ValueError):
                cache = {}
        if key in cache:
            self.set_schedule(*cache[key]["schedule"])
            return cache[key]
        ncu = torch.cuda.get_device_properties(0).multi_processor_count
        work = packed.clone()
        trials = []
        for eb in CANDIDATE_EB:
            for wpc in CANDIDATE_WG_PER_CU:
                nwg = ncu * wpc
                for order in CANDIDATE_ORDER:
                    self.set_schedule(eb, nwg, order)
                    self.rk(work, dts, 1, graph=False)
                    torch.cuda.synchronize()
                    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    s.record()
                    for _ in range(reps):
                        self.rk(work, dts, 1, graph=False)
                    e.record()
                    torch.cuda.synchronize()
                    trials.append((s.elapsed_time(e) / reps, (eb, nwg, order)))
        self.sync()
        trials.sort()
        best = {"schedule": list(trials[0][1]), "ms_per_step": trials[0][0],
                "trials": [[t, list(sch)] for t, sch in trials]}
        self.set_schedule(*trials[0][1])
        cache[key] = best
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
        return best

    def close(self):
        if self.b is not None:
            B.cdg2_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
