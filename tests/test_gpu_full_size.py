"""The plate and square-cylinder workloads at their full sizes.

Step 1 of the plate (128x96 cells x 1600 velocities) is compared element by
element with the FP64 oracle, in both precision forms.  The square (160x160 x
10 000 velocities) is beyond the oracle's reach, so its FP32-f run is
compared with the FP64 form, itself pinned to the oracle on the smaller
square cases, through properties that hold at any size: the same cycle
counts, the same steady fields, no loss of conservation.
"""
import numpy as np
import pytest

import workloads as wl
from _parity import field_errors, perturbed_state, rel_max, to_oracle
from oracle.solver import Oracle

pytestmark = pytest.mark.gpu


def test_plate_full_size_step1_against_oracle():
    """Row a1 at the plate's full size: div and R of a perturbed state."""
    from paper_1704_03151_amd import Solver
    case = wl.config3()
    print("[full] plate128x96 x 1600: step 1 against the oracle", flush=True)
    prim, pert = perturbed_state(case, 5)
    orc = Oracle(case.with_(precision="fp64"))
    for prec, tol in (("fp64", 1e-11), ("fp32f", 2e-5)):
        gpu = Solver(case, precision=prec)
        gpu.init_macro(prim)
        gpu.set_f((gpu.get_f(np.float64) * pert).astype(gpu.dtype))
        # the oracle sees the distribution as the GPU holds it
        G, H = to_oracle(gpu.get_f(np.float64))
        orc.init_macro(prim)
        orc.set_f(G, H)
        R, norms = gpu.residual()
        dG, dH = to_oracle(gpu.div(np.float64))
        gpu.close()
        orc.step1()
        eG, eH = rel_max(dG, orc.divG), rel_max(dH, orc.divH)
        Rref = orc.R.reshape(4, case.ny, case.nx)
        eR = max(rel_max(R[m], Rref[m]) for m in range(4))
        print(f"[full] {prec}: div {eG:.2e} {eH:.2e}, R {eR:.2e}", flush=True)
        assert eG < tol and eH < tol and eR < tol, (prec, eG, eH, eR)


def test_plate_full_size_steady_fp32_matches_fp64():
    """The plate converges to 1e-6 in both forms, in the same number of
    cycles, to the same fields within 1e-5."""
    from paper_1704_03151_amd import Solver
    case = wl.config3()
    out = {}
    for prec in ("fp64", "fp32f"):
        s = Solver(case, precision=prec)
        rc, n, res = s.iterate(300, tol=1e-6)
        m = s.macro()
        s.close()
        print(f"[full] plate {prec}: status {rc}, {n} cycles, residuals {res}", flush=True)
        assert rc == 0, (prec, n, res)
        out[prec] = (n, m)
    assert abs(out["fp32f"][0] - out["fp64"][0]) <= 2
    m64 = out["fp64"][1]
    err = field_errors(out["fp32f"][1], (m64["rho"], m64["U"], m64["V"], m64["T"]))
    print(f"[full] plate fp32f against fp64: {err}", flush=True)
    assert max(err.values()) < 1e-5, err


def test_square_full_size_fp32_matches_fp64():
    """The Mach-5 square: 120 cycles of both forms reach the residual level
    set by the Simpson 3/8 velocity rule (below 1e-4) with the same fields."""
    from paper_1704_03151_amd import Solver
    case = wl.config4()
    out = {}
    for prec in ("fp64", "fp32f"):
        s = Solver(case, precision=prec)
        rc, n, res = s.iterate(120, tol=1e-6)
        m = s.macro()
        s.close()
        print(f"[full] square {prec}: status {rc}, {n} cycles, residuals {res}", flush=True)
        assert np.all(np.isfinite(res)) and np.max(res) < 1e-4, (prec, res)
        out[prec] = m
    fl = case.solid == 0
    m64 = out["fp64"]
    err = field_errors(out["fp32f"], (m64["rho"], m64["U"], m64["V"], m64["T"]), fl)
    print(f"[full] square fp32f against fp64: {err}", flush=True)
    assert max(err.values()) < 1e-5, err
