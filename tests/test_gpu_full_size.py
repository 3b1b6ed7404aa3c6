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


def test_square_full_size_fp64_converges_and_fp32_reaches_its_floor():
    """The Mach-5 square (trapezoid velocity grid, capped pseudo step): the
    FP64 form converges to 1e-6 within 200 cycles.  The FP32-f form, run as
    many cycles, stalls at the resolution of FP32 storage (below 3e-5, with
    the same fields within 1e-5), and that floor is not the iteration's: the
    FP64 steady state itself, rounded to FP32, already has a residual above
    1e-6 (fluxes of order 20 through the 0.01-wide cells at the front face)."""
    from paper_1704_03151_amd import Solver
    case = wl.config4()
    print("[full] square160x160 x 10000: FP64 to 1e-6, FP32-f as many cycles", flush=True)
    s64 = Solver(case, precision="fp64")
    rc, n, res = s64.iterate(200, tol=1e-6)
    print(f"[full] square fp64: status {rc}, {n} cycles, residuals {res}", flush=True)
    assert rc == 0, (n, res)
    m64 = s64.macro()
    f64 = s64.get_f(np.float64)
    s64.close()
    s32 = Solver(case, precision="fp32f")
    rc32, n32, res32 = s32.iterate(n, tol=1e-6)
    m32 = s32.macro()
    print(f"[full] square fp32f: status {rc32}, {n32} cycles, residuals {res32}", flush=True)
    assert np.all(np.isfinite(res32)) and np.max(res32) < 3e-5, res32
    fl = case.solid == 0
    err = field_errors(m32, (m64["rho"], m64["U"], m64["V"], m64["T"]), fl)
    print(f"[full] square fp32f against fp64: {err}", flush=True)
    assert max(err.values()) < 1e-5, err
    s32.set_f(f64.astype(np.float32))
    _, res_round = s32.residual()
    s32.close()
    print(f"[full] the FP64 steady state rounded to FP32: residuals {res_round}", flush=True)
    assert np.max(res_round) > 1e-6


def test_adjoint_full_size_against_steady_state_differences():
    """The adjoint at the size it is meant for: the 64x64 cavity at Kn 0.1
    with 784 Gauss-Hermite velocities, FP64, converged to 1e-13; the lid-shear
    gradient over the 64 bottom-face temperatures against central differences
    (h = 1e-4, the step of the survey's C17) of the GPU's own steady states,
    each converged to 1e-13 at the same mass, on 8 seeded faces.  Every face
    agrees within 2.5e-4 of the largest gradient component.  The adjoint with
    its Krylov basis in float matches the double one to 1e-7 of the largest.
    The per-face
    ratios of C17's scale 1e-4 max(|g_FD|, 1e-3 max|g|) are printed: the
    differences do not shrink with h (central or 4-point stencils), so they
    are the finite differences' own uncertainty at this convergence level."""
    from paper_1704_03151_amd import Solver
    case = wl.config5(precision="fp64")
    print("[full] cavity64 Kn 0.1 x 784: adjoint against steady-state differences", flush=True)
    s = Solver(case, precision="fp64")
    rc, n, res = s.iterate(2000, tol=1e-13)
    assert rc == 0, res
    cell, side = s.wall_list()
    lid = list(np.nonzero(side == 3)[0])
    nfx = (case.nx + 1) * case.ny
    faces = [nfx + i for i in range(case.nx)]
    st, g, iters, rel = s.adjoint(1, lid, faces, tol=2e-10, max_iter=6000)
    print(f"[full] adjoint: {iters} corrections, relative residual {rel:.2e}", flush=True)
    assert st == 0
    gmax = np.max(np.abs(g))
    # the float Krylov basis reaches the same tolerance, and every face then
    # agrees with the double form to 1e-7 of the largest
    st32, g32, it32, rel32 = s.adjoint(1, lid, faces, tol=2e-10, max_iter=6000, krylov_precision="fp32")
    e32 = np.max(np.abs(g32 - g)) / gmax
    print(f"[full] adjoint with a float Krylov basis: {it32} corrections, relative residual {rel32:.2e}, "
          f"against the double form {e32:.1e} of max|g|", flush=True)
    assert st32 == 0 and e32 < 1e-7, (st32, rel32, e32)
    f0 = s.get_f()
    h = 1e-4
    pick = sorted(np.random.default_rng(1704).choice(case.nx, 8, replace=False))
    worst = 0.0
    for fi in pick:
        vals = []
        for sg in (1.0, -1.0):
            s.set_wall_T([faces[fi]], [case.wall_y[0, fi, 0] + sg * h])
            s.set_f(f0)
            rc2, _, r2 = s.iterate(3000, tol=1e-13)
            assert rc2 == 0, r2
            vals.append(s.objective(1, lid))
        s.set_wall_T([faces[fi]], [case.wall_y[0, fi, 0]])
        s.set_f(f0)
        fd = (vals[0] - vals[1]) / (2 * h)
        c17 = abs(g[fi] - fd) / (1e-4 * max(abs(fd), 1e-3 * gmax))
        print(f"[full] face {fi}: adjoint {g[fi]:.8e}, differences {fd:.8e}, error / max|g| "
              f"{abs(g[fi] - fd) / gmax:.1e}, error / C17 scale {c17:.2f}", flush=True)
        worst = max(worst, abs(g[fi] - fd) / gmax)
    assert worst < 2.5e-4, worst
    s.close()
