"""The binary32 polynomial cores of the mixed Exact path (exact.hip): the
coefficients in the kernel source, evaluated as the device does (binary32
Horner with fused multiply-adds, binary64 assembly), meet the relative
errors the source states -- atan within 4.7e-9 on the reduced range
|s| <= tan(pi/8), 2 atanh within 7.3e-10 on |t| <= 3 - 2 sqrt(2) -- and the
committed fitting script (discrete minimax by linear programming)
reproduces polynomials of that quality."""
import os
import re
import sys

import numpy as np

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_2410_15227_amd", "csrc")
sys.path.insert(0, CSRC)
import fit_cores  # noqa: E402


def coefficients(name):
    """The binary32 Horner coefficients of `float <name> = ...; <name> = fmaf(<name>, zf, ...)`."""
    src = open(os.path.join(CSRC, "exact.hip")).read()
    i = src.index(f"float {name} = ")
    block = src[i:src.index(";\n", src.index(f"{name} = fmaf({name}, zf, 0.666", i) if name == "Q" else
                            src.index(f"{name} = fmaf({name}, zf, -0.333", i))]
    vals = re.findall(r"(-?\d\.\d+)f", block)
    return np.array([float(v) for v in vals], dtype=np.float32)


def test_kernel_cores_meet_stated_errors():
    P, Q = coefficients("P"), coefficients("Q")
    assert len(P) == 6 and len(Q) == 4
    ea, eh = fit_cores.achieved(P, Q)
    assert ea <= 4.7e-9, ea
    assert eh <= 7.3e-10, eh


def test_fit_reproduces_the_cores():
    P, e1 = fit_cores.fit_atan()
    Q, e2 = fit_cores.fit_atanh()
    # the polynomial approximation itself is far below the binary32 floor
    assert e1 < 1e-10 and e2 < 1e-10
    ea, eh = fit_cores.achieved(P, Q)
    assert ea < 6e-9 and eh < 1e-9
