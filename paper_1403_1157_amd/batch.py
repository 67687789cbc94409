"""Batched instances: packed state, batched SSP-RK3 launches and their autotuner.

The arithmetic runs in libcdg2 (cdg2_batch_*), and so does the schedule search
(cdg2_batch_autotune times every candidate: cells per work item, persistent
workgroup count, item order).  This module packs and unpacks torch tensors and
caches the chosen schedule in a JSON file keyed by the GPU architecture, its
compute-unit count, a hash of the built library (a schedule tuned on other
kernels is not reused) and the batch's (grid, order) signature.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import cdg2 as B

_LIB_ID = None


def library_id() -> str:
    """Hash of the built libcdg2.so: changes whenever the kernels are rebuilt
    from other sources."""
    global _LIB_ID
    if _LIB_ID is None:
        h = hashlib.sha256()
        with open(B.LIB_PATH, "rb") as f:
            for chunk in iter(lambda: f.read(1 << 20), b""):
                h.update(chunk)
        _LIB_ID = h.hexdigest()[:16]
    return _LIB_ID


def default_cache_path() -> str:
    return os.environ.get("CDG2_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "cdg2_autotune.json"))


class Batch:
    def __init__(self, instances, autotune: bool = False):
        """instances: list of dicts with keys n (2-tuple), order (1..3), coeffs;
        autotune: run the library's schedule search at creation."""
        self.instances = instances
        cfgs = [B.make_config(2, inst["n"], inst["order"], inst["coeffs"]) for inst in instances]
        self.b = B.cdg2_batch_create(cfgs, autotune)
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

    def rk(self, packed: torch.Tensor, dts, nsteps: int, graph: bool = True, offsets=None) -> torch.Tensor:
        """nsteps SSP-RK3 steps in place; offsets: None (this packing) or per-instance
        element offsets of another placement inside the same packed size."""
        if not (packed.is_cuda and packed.dtype == torch.float64 and packed.is_contiguous()
                and packed.numel() == self.total):
            raise ValueError("expected the packed float64 CUDA state")
        self._stream()
        B.cdg2_batch_set_graph(self.b, graph)
        B.cdg2_batch_rk(self.b, packed.data_ptr(), offsets, dts, nsteps)
        return packed

    def sync(self) -> None:
        self._stream()
        B.cdg2_batch_sync(self.b)

    def autotune(self, cache_path: str | None = None):
        """Schedule of this batch: from the cache if present, else from the
        library's search (cdg2_batch_autotune), then cached."""
        cache_path = cache_path or default_cache_path()
        prop = torch.cuda.get_device_properties(torch.cuda.current_device())
        arch = prop.gcnArchName.split(":")[0]
        key = f"{arch}:cu{prop.multi_processor_count}:lib{library_id()}:{self.signature()}"
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
        self._stream()
        sched, ms = B.cdg2_batch_autotune(self.b)
        self.schedule = sched
        best = {"schedule": list(sched), "ms_per_step": ms}
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
