"""GPU adjoint (through the C ABI) against the FP64 CPU oracle:

* the transposed residual product (dr/df)^T v element by element against the
  oracle's dense complex-step Jacobian on tiny cases (1e-11 max-norm
  relative), and as <(dr/df)^T v, d> = <v, (dr/df) d> on larger ones with the
  oracle's complex-step directional derivative (1e-10);
* the wall-temperature gradient of the lid shear at a converged steady state
  against the oracle's fixed-mass tangent (plain linear solve on the dense
  Jacobian).  The GPU takes dJ/dM along the mass family from two steady
  states at masses M0 (1 +- 1e-4), good to about 1e-8 of the gradient, so
  the gradient is compared at 1e-6;
* the same in an open domain (a plate in a farfield: no mass term, and both
  sides of the plate take the one face temperature) for the pressure, shear
  and heat loads;
* both again with the Krylov basis stored in float."""
import numpy as np
import pytest

import workloads as wl
from _parity import perturbed_state, small_cases, tiny_open_plate, to_oracle
from oracle import adjoint as ad
from oracle.solver import Oracle

pytestmark = pytest.mark.gpu

N = 4


def _tiny_cavity():
    case = wl.cavity(n=N, Kn=2.0, n_levels=2, quad="gauss_hermite", nvel=8, vlo=0.0, vhi=0.0, mach=0.3,
                     precision="fp64")
    rng = np.random.default_rng(1704)
    case.wall_y[0, :, 0] = 1.0 + rng.uniform(-0.05, 0.05, N)
    return case


def _tiny_plate():
    """8 x 6 cells around a plate, farfield sides and an outflow side, 6 x 6
    velocities on [-3, 3]."""
    case = wl.flat_plate(scale=16, quad="trapezoid", nu=6, nv=6, vlo=-3.0, vhi=3.0, n_levels=1, precision="fp64",
                         Kn=0.3)
    case.face_type_x[:, -1] = wl.FACE_OUTFLOW
    return case


def _pair_at(case, seed):
    """GPU solver and oracle holding the same perturbed distribution."""
    from paper_1704_03151_amd import Solver
    gpu = Solver(case, precision="fp64")
    prim, pert = perturbed_state(case, seed)
    gpu.init_macro(prim)
    gpu.set_f(gpu.get_f() * pert)
    orc = Oracle(case)
    orc.init_macro(prim)
    orc.set_f(*to_oracle(gpu.get_f()))
    return gpu, orc


@pytest.mark.parametrize("which", ["cavity", "plate"])
def test_residual_adjoint_against_dense_jacobian(which):
    case = _tiny_cavity() if which == "cavity" else _tiny_plate()
    print(f"[adjoint] {which}: (dr/df)^T v against the dense Jacobian", flush=True)
    gpu, orc = _pair_at(case, 71)
    S = ad.Sensitivity(orc)
    J = S.jacobian()
    rng = np.random.default_rng(72)
    for _ in range(2):
        vG = rng.standard_normal(orc.G.shape) * orc.lev0.fluid
        vH = rng.standard_normal(orc.H.shape) * orc.lev0.fluid
        v = np.stack([vG.reshape(-1, case.ny, case.nx), vH.reshape(-1, case.ny, case.nx)])
        got = S.pack(*to_oracle(gpu.residual_adjoint(v)))
        ref = J.T @ S.pack(vG, vH)
        assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref)), np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    gpu.close()


@pytest.mark.parametrize("name", ["cavity16_kn10", "square20x20", "plate32x24", "box12x10_ragged", "box8_vel65"])
def test_residual_adjoint_dot_products(name):
    case = small_cases()[name].with_(precision="fp64")
    print(f"[adjoint] {name}: dot-product test", flush=True)
    gpu, orc = _pair_at(case, 73)
    S = ad.Sensitivity(orc)
    x0 = S.pack(orc.G, orc.H)
    rng = np.random.default_rng(74)
    for _ in range(3):
        d = rng.standard_normal(x0.size) * np.abs(x0)
        Jd = S.residual(x0.astype(complex) + 1e-30j * d).imag / 1e-30
        vG = rng.standard_normal(orc.G.shape) * orc.lev0.fluid
        vH = rng.standard_normal(orc.H.shape) * orc.lev0.fluid
        v = np.stack([vG.reshape(-1, case.ny, case.nx), vH.reshape(-1, case.ny, case.nx)])
        JTv = S.pack(*to_oracle(gpu.residual_adjoint(v)))
        lhs = JTv @ d
        rhs = S.pack(vG, vH) @ Jd
        scale = np.sum(np.abs(JTv * d))
        assert abs(lhs - rhs) < 1e-10 * scale, (lhs, rhs, scale)
    gpu.close()


def test_adjoint_gradient_against_oracle():
    """Lid shear of the tiny cavity, gradient with respect to three bottom
    faces and one side face, at steady states converged on both sides."""
    from paper_1704_03151_amd import Solver
    case = _tiny_cavity()
    print("[adjoint] tiny cavity: dJ/dTw", flush=True)
    gpu = Solver(case, precision="fp64")
    orc = Oracle(case)
    rc, n, res = gpu.iterate(300, tol=2e-13)
    ok, norms = orc.iterate(300, tol=2e-13)
    assert rc == 0 and ok, (rc, res, norms)
    cell, side = gpu.wall_list()
    lid = list(np.nonzero(side == 3)[0])
    nfx = (N + 1) * N
    faces = [nfx + 0, nfx + 1, nfx + 3, 0]
    st, g, iters, rel = gpu.adjoint(ad.LOAD_SHEAR, lid, faces, tol=1e-9, max_iter=2000)
    ref = ad.Sensitivity(orc).gradient(ad.LOAD_SHEAR, lid, faces)
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    print(f"[adjoint] {iters} corrections, relative residual {rel:.2e}, gradient error {err:.2e}", flush=True)
    assert st == 0
    assert err < 1e-6, (g, ref)
    gpu.close()


def test_open_domain_adjoint_gradient_against_oracle():
    """Plate loads (pressure, shear, heat, summed over both sides) with respect
    to the plate face's temperature; without the mass term the gradient is
    limited only by the linear solves, compared at 1e-7."""
    from paper_1704_03151_amd import Solver
    case, face = tiny_open_plate()
    print("[adjoint] tiny open plate: dJ/dTw", flush=True)
    gpu = Solver(case, precision="fp64")
    orc = Oracle(case)
    rc, n, res = gpu.iterate(300, tol=2e-13)
    ok, norms = orc.iterate(300, tol=2e-13)
    assert rc == 0 and ok, (rc, res, norms)
    cell, side = gpu.wall_list()
    walls = list(range(len(cell)))
    assert len(walls) == 2 and sorted(side) == [2, 3]
    S = ad.Sensitivity(orc)
    T = S.tangent(S.jacobian(), S.dr_dT([face]))
    for kind in (ad.LOAD_PRESSURE, ad.LOAD_SHEAR, ad.LOAD_HEAT):
        ref = S.dJ_df(kind, walls) @ T + S.dJ_dT(kind, walls, [face])
        st, g, iters, rel = gpu.adjoint(kind, walls, [face], tol=1e-10, max_iter=2000)
        err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
        print(f"[adjoint] kind {kind}: {iters} corrections, relative residual {rel:.2e}, error {err:.2e}",
              flush=True)
        assert st == 0
        assert err < 1e-7, (kind, g, ref)
    gpu.close()


def test_fp32_krylov_adjoint_against_oracle():
    """The adjoint with the Krylov basis and the preconditioner's vectors
    stored in float (the multiplier, dot products and the contraction in
    double, each restart refining the multiplier from the true residual): the
    tiny cavity's lid-shear gradient against the oracle's fixed-mass tangent,
    and the open plate's three loads, to the double form's tolerances.  (With
    the multiplier itself in float the residual stalled at 3e-7 on the plate,
    where the shear gradient, a near cancellation of its two sides, then
    erred by 2e-5.)"""
    from paper_1704_03151_amd import Solver
    case = _tiny_cavity()
    print("[adjoint] tiny cavity: dJ/dTw with a float Krylov basis", flush=True)
    gpu = Solver(case, precision="fp64")
    orc = Oracle(case)
    rc, n, res = gpu.iterate(300, tol=2e-13)
    ok, norms = orc.iterate(300, tol=2e-13)
    assert rc == 0 and ok, (rc, res, norms)
    cell, side = gpu.wall_list()
    lid = list(np.nonzero(side == 3)[0])
    nfx = (N + 1) * N
    faces = [nfx + 0, nfx + 1, nfx + 3, 0]
    ref = ad.Sensitivity(orc).gradient(ad.LOAD_SHEAR, lid, faces)
    st, g, iters, rel = gpu.adjoint(ad.LOAD_SHEAR, lid, faces, tol=1e-9, max_iter=2000, krylov_precision="fp32")
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    print(f"[adjoint] float basis: {iters} corrections, relative residual {rel:.2e}, error {err:.2e}",
          flush=True)
    assert st == 0 and err < 1e-8, (st, rel, g, ref)
    gpu.close()

    case, face = tiny_open_plate()
    print("[adjoint] tiny open plate: dJ/dTw with a float Krylov basis", flush=True)
    gpu = Solver(case, precision="fp64")
    orc = Oracle(case)
    rc, n, res = gpu.iterate(300, tol=2e-13)
    ok, norms = orc.iterate(300, tol=2e-13)
    assert rc == 0 and ok, (rc, res, norms)
    walls = list(range(len(gpu.wall_list()[0])))
    S = ad.Sensitivity(orc)
    T = S.tangent(S.jacobian(), S.dr_dT([face]))
    for kind in (ad.LOAD_PRESSURE, ad.LOAD_SHEAR, ad.LOAD_HEAT):
        ref = S.dJ_df(kind, walls) @ T + S.dJ_dT(kind, walls, [face])
        st, g, iters, rel = gpu.adjoint(kind, walls, [face], tol=1e-9, max_iter=2000, krylov_precision="fp32")
        err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
        print(f"[adjoint] kind {kind}, float basis: {iters} corrections, relative residual {rel:.2e}, "
              f"error {err:.2e}", flush=True)
        assert st == 0 and err < 1e-7, (kind, rel, g, ref)
    with pytest.raises(ValueError):
        gpu.adjoint(ad.LOAD_SHEAR, walls, [face], krylov_precision="fp16")
    # the C entry point itself refuses another storage type, before any work
    import ctypes
    from paper_1704_03151_amd import _C
    ids = np.ascontiguousarray(walls, np.int32)
    fc = np.ascontiguousarray([face], np.int32)
    g = np.zeros(1)
    rc = _C.lib.miugks_adjoint_ex(gpu.h, ad.LOAD_SHEAR, _C.iptr(ids), len(ids), _C.iptr(fc), 1, 1e-9, 10, 7,
                                  _C.dptr(g), None, None)
    assert rc == _C.EINVAL and b"krylov_dtype" in _C.lib.miugks_last_error(gpu.h)
    gpu.close()


def test_autograd_wall_load_matches_adjoint():
    """J(Tw) through torch.autograd: the forward value is the objective of the
    converged state and the gradient is the adjoint's."""
    import torch
    from paper_1704_03151_amd import Solver
    from paper_1704_03151_amd.autograd import steady_wall_load
    case = _tiny_cavity()
    print("[adjoint] tiny cavity: autograd", flush=True)
    gpu = Solver(case, precision="fp64")
    cell, side = gpu.wall_list()
    lid = list(np.nonzero(side == 3)[0])
    nfx = (N + 1) * N
    faces = [nfx + i for i in range(N)]
    Tw = torch.tensor(case.wall_y[0, :, 0], dtype=torch.float64, device="cuda", requires_grad=True)
    J = steady_wall_load(gpu, Tw, ad.LOAD_SHEAR, lid, faces, tol=2e-13, adj_tol=1e-9)
    (g,) = torch.autograd.grad(J, Tw)
    assert abs(J.item() - gpu.objective(ad.LOAD_SHEAR, lid)) == 0.0
    st, ref, _, _ = gpu.adjoint(ad.LOAD_SHEAR, lid, faces, tol=1e-9)
    assert st == 0 and g.device.type == "cuda"
    assert np.max(np.abs(g.cpu().numpy() - ref)) <= 1e-9 * np.max(np.abs(ref))
    gpu.close()


def test_autograd_backward_after_another_forward():
    """Two forwards at different wall temperatures, then the backward of the
    first: its gradient is the one at its own steady state (equal to a fresh
    forward and backward there), not at the state the second forward left."""
    import torch
    from paper_1704_03151_amd import Solver
    from paper_1704_03151_amd.autograd import steady_wall_load
    case = _tiny_cavity()
    print("[adjoint] tiny cavity: backward after another forward", flush=True)
    gpu = Solver(case, precision="fp64")
    cell, side = gpu.wall_list()
    lid = list(np.nonzero(side == 3)[0])
    nfx = (N + 1) * N
    faces = [nfx + i for i in range(N)]
    T1 = torch.tensor(case.wall_y[0, :, 0], dtype=torch.float64, device="cuda", requires_grad=True)
    T2 = torch.tensor(case.wall_y[0, :, 0] * 1.02, dtype=torch.float64, device="cuda", requires_grad=True)
    J1 = steady_wall_load(gpu, T1, ad.LOAD_SHEAR, lid, faces, tol=1e-12, adj_tol=1e-10)
    J2 = steady_wall_load(gpu, T2, ad.LOAD_SHEAR, lid, faces, tol=1e-12, adj_tol=1e-10)
    assert abs(J1.item() - J2.item()) > 1e-6 * abs(J1.item())
    (g1,) = torch.autograd.grad(J1, T1)
    (g2,) = torch.autograd.grad(J2, T2)
    ref = Solver(case, precision="fp64")
    T1r = T1.detach().clone().requires_grad_(True)
    Jr = steady_wall_load(ref, T1r, ad.LOAD_SHEAR, lid, faces, tol=1e-12, adj_tol=1e-10)
    (gr,) = torch.autograd.grad(Jr, T1r)
    e1 = float(torch.max(torch.abs(g1 - gr)) / torch.max(torch.abs(gr)))
    e12 = float(torch.max(torch.abs(g2 - gr)) / torch.max(torch.abs(gr)))
    print(f"[adjoint] first gradient against a fresh one {e1:.2e}; the second differs by {e12:.2e}", flush=True)
    assert abs(J1.item() - Jr.item()) <= 1e-12 * abs(Jr.item())
    assert e1 < 1e-8 and e12 > 1e-4
    gpu.close()
    ref.close()
