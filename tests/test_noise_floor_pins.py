"""The float64 oracle against an extended-precision evaluation of the same
discrete operator (tests/ld_operator.py, x87 80-bit long double): the FP64 noise
floor below the parity bar, and the reason for forming face jumps mode by mode.

On small grids the oracle must lie within 1e-13 (relative, per species,
element-wise against the species scale and in the 2-norm) of the
extended-precision result.  The same evaluation in float64 with the jump formed
as the plain difference of the two traces is printed beside it and must be
clearly worse: its rounding is amplified by the penalty (p+1)^2/h and the face
scaling 1/h.  The floors measured at the benchmark sizes are stated with the
readings of the paper."""
import numpy as np
import pytest
import torch

from ld_operator import LDOperator
from oracle.cdg2_oracle import Config, Oracle
from paper_1403_1157_amd import inputs


def strong():
    c = inputs.base_coeffs()
    c.update(chi0_11=0.05, chi0_13=0.03, chi0_21=0.04, chi0_22=0.02)
    return c


def rel(g, o):
    g = np.asarray(g, dtype=np.longdouble).reshape(6, -1)
    o = np.asarray(o, dtype=np.longdouble).reshape(6, -1)
    d = abs(g - o)
    elem = (d.max(1) / abs(o).max(1)).max()
    norm = (np.sqrt((d * d).sum(1)) / np.sqrt((o * o).sum(1))).max()
    return float(elem), float(norm)


@pytest.mark.parametrize("dim,n,p,cs", [(2, (16, 16), 4, "base"), (2, (16, 16), 4, "strong"),
                                        (2, (24, 20), 2, "strong"), (3, (8, 8, 8), 2, "base"),
                                        (3, (6, 5, 4), 3, "strong")])
def test_oracle_within_1e13_of_extended_precision(dim, n, p, cs):
    c = inputs.base_coeffs() if cs == "base" else strong()
    U = inputs.initial_modes(dim, n, p, (1,))          # nearly continuous fields
    truth = LDOperator(dim, n, p, c).apply(U)
    assert np.finfo(truth.dtype).eps < 1e-18           # a real extended format
    ora = Oracle(Config(dim=dim, n=n, order=p, coeffs=c)).apply(torch.from_numpy(U)).numpy()
    plain = LDOperator(dim, n, p, c, dt=np.float64).apply(U, jump="plain")
    e_or, e_pl = rel(ora, truth), rel(plain, truth)
    print(f"[floor] d{dim} {n} p{p} {cs}: oracle {e_or[0]:.1e}/{e_or[1]:.1e}, "
          f"plain-difference jump {e_pl[0]:.1e}/{e_pl[1]:.1e} (element-wise/norm)", flush=True)
    assert max(e_or) <= 1e-13, e_or
    assert max(e_pl) >= 3 * max(e_or), (e_or, e_pl)


def test_jump_forms_agree_in_extended_precision():
    """In long double both forms of the jump give the same operator to its
    rounding (they are equal in exact arithmetic)."""
    U = inputs.initial_modes(2, (8, 8), 3, (2,))
    L = LDOperator(2, (8, 8), 3, strong())
    assert max(rel(L.apply(U, jump="plain"), L.apply(U))) < 1e-16
