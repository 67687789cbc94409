"""The allocation-free SSP-RK3 entry point (cdg2_rk_step_noalloc) against the
plain one (cdg2_rk_step), called through the C ABI: the same kernels in the same
order, so the results must be bitwise equal.  Two calls in a row, the second on
a smaller grid, so the second call reuses scratch memory that still holds the
first call's larger states; and a state beyond the scratch limit is rejected."""
import ctypes

import pytest
import torch

from paper_1403_1157_amd import cdg2 as B
from paper_1403_1157_amd import inputs

pytestmark = pytest.mark.gpu


def _run(dim, n, p, steps, key):
    cfg = B.make_config(dim, n, p, inputs.base_coeffs())
    h = B.cdg2_create(cfg)
    try:
        B.cdg2_set_stream(h, torch.cuda.current_stream().cuda_stream)
        U0 = torch.from_numpy(inputs.initial_modes(dim, n, p, key)).cuda().contiguous()
        assert U0.numel() == B.cdg2_num_dofs(h)
        dt = B.cdg2_max_dt(h, U0.data_ptr(), 0.9)
        Ua = U0.clone()
        Ub = U0.clone()
        B.cdg2_rk_step(h, Ua.data_ptr(), dt, steps)
        B.cdg2_sync(h)
        print(f"no-alloc case dim={dim} n={n} p={p} steps={steps}", flush=True)
        rc = B.lib().cdg2_rk_step_noalloc(h, ctypes.c_void_p(Ub.data_ptr()), ctypes.c_double(dt),
                                          ctypes.c_int(steps))
        assert rc == B.CDG2_OK, B.cdg2_last_error()
        B.cdg2_sync(h)
        assert torch.equal(Ua, Ub), float((Ua - Ub).abs().max())
        assert not torch.equal(Ua, U0)
    finally:
        B.cdg2_destroy(h)


def test_noalloc_matches_plain_rk_step_twice_then_smaller():
    _run(2, (40, 36), 2, 6, (11,))     # 77,760 entries
    _run(2, (12, 10), 1, 4, (12,))     # 2,880 entries: smaller, in the same scratch
    _run(3, (6, 5, 9), 2, 3, (13,))    # 3D stage kernel (nodal form), two slabs along z


def test_noalloc_rejects_states_beyond_the_scratch_limit():
    cfg = B.make_config(2, (256, 256), 4, inputs.base_coeffs())   # 9,830,400 entries, 78.6 MB
    h = B.cdg2_create(cfg)
    try:
        U = torch.zeros(B.cdg2_num_dofs(h), dtype=torch.float64, device="cuda")
        rc = B.lib().cdg2_rk_step_noalloc(h, ctypes.c_void_p(U.data_ptr()), ctypes.c_double(1e-6),
                                          ctypes.c_int(1))
        assert rc == B.CDG2_EINVAL
        assert b"scratch" in B.lib().cdg2_last_error()
    finally:
        B.cdg2_destroy(h)
