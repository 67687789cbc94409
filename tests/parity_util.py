"""Helpers for GPU-vs-oracle parity tests (comparison norms, case construction)."""
import numpy as np
import torch

from oracle.cdg2_oracle import Config, Oracle
from paper_1403_1157_amd import inputs

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def rel_errors(gpu, ora):
    """Per species: max_i |g_i - o_i| / max_i |o_i| (element by element against the
    species scale) and ||g - o||_2 / ||o||_2.  Returns the worst of each."""
    g = gpu.detach().to("cpu", torch.float64).reshape(6, -1)
    o = ora.detach().to(torch.float64).reshape(6, -1)
    d = (g - o).abs()
    scale = o.abs().amax(dim=1).clamp_min(1e-300)
    elem = float((d.amax(dim=1) / scale).max())
    norm = float((d.norm(dim=1) / o.norm(dim=1).clamp_min(1e-300)).max())
    return elem, norm


def assert_close(gpu, ora, tol, what=""):
    elem, norm = rel_errors(gpu, ora)
    assert elem <= tol and norm <= tol, f"{what}: elementwise {elem:.3e}, norm {norm:.3e} > {tol:g}"
    return elem, norm


def make_case(dim, n, p, key=(0,), coeffs=None, wall_axis=None, llf_mode="all",
              gamma1_in=(0.0, 1.0)):
    coeffs = inputs.base_coeffs() if coeffs is None else coeffs
    wall = dim - 1 if wall_axis is None else wall_axis
    U = inputs.initial_modes(dim, n, p, key, wall_axis=wall)
    cfg = Config(dim=dim, n=tuple(n), order=p, wall_axis=wall, llf_mode=llf_mode,
                 gamma1_in=tuple(gamma1_in), coeffs=coeffs)
    return torch.from_numpy(np.ascontiguousarray(U)), cfg


def oracle_for(cfg):
    return Oracle(cfg)
