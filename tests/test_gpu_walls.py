"""GPU wall loads, objectives and wall-temperature changes (through the C
ABI) against the FP64 CPU oracle on seeded inputs: loads element by element
(1e-12 max-norm relative; the loads are double sums of the stored
distribution), fields after cycles with changed walls (1e-10)."""
import numpy as np
import pytest

from _parity import field_errors, perturbed_state, rel_max, small_cases, to_oracle
from oracle import adjoint as ad
from oracle.solver import Oracle

pytestmark = pytest.mark.gpu

CASES = small_cases()


def _perturbed(case, precision, seed):
    from paper_1704_03151_amd import Solver
    gpu = Solver(case, precision=precision)
    prim, pert = perturbed_state(case, seed)
    gpu.init_macro(prim)
    gpu.set_f(gpu.get_f() * pert.astype(gpu.get_f().dtype))
    return gpu, prim


@pytest.mark.parametrize("name,precision", [("cavity16_kn10", "fp64"), ("plate32x24", "fp64"),
                                            ("square20x20", "fp64"), ("box12x10_ragged", "fp32f")])
def test_wall_loads_against_oracle(name, precision):
    """Loads of every wall side (cavity walls, both sides of the plate, the
    square's four faces) of a perturbed state; the oracle reads the same
    stored distribution."""
    case = CASES[name]
    print(f"[walls] {name} {precision}: loads", flush=True)
    gpu, _ = _perturbed(case, precision, 41)
    orc = Oracle(case)
    G, H = to_oracle(gpu.get_f())
    orc.set_f(G, H)
    cell, side = gpu.wall_list()
    js = ad.wall_list(orc.lev0)
    assert np.array_equal(cell, orc.lev0.bcell[js]) and np.array_equal(side, orc.lev0.bside[js])
    got = gpu.wall_loads()
    ref = ad.wall_loads(orc.G, orc.H, orc.lev0, orc.vel, orc.gas, case.farfield)
    assert got.shape == ref.shape and got.shape[1] > 0
    for m in range(4):
        assert rel_max(got[m], ref[m]) < 1e-12, (m, rel_max(got[m], ref[m]))
    ids = np.arange(0, got.shape[1], 3)
    for kind in (ad.LOAD_PRESSURE, ad.LOAD_SHEAR, ad.LOAD_HEAT):
        J = gpu.objective(kind, ids)
        Jr = ad.objective(orc.G, orc.H, orc.lev0, orc.vel, orc.gas, case.farfield, kind, ids)
        assert abs(J - Jr) <= 1e-12 * max(abs(Jr), np.max(np.abs(ref[3] * ref[kind]))), (kind, J, Jr)
    gpu.close()


def test_set_wall_T_against_oracle():
    """New temperatures on four bottom faces and a lid face, then three
    outer cycles from the same perturbed state, against an oracle built with
    those walls; bad faces and temperatures are refused and change nothing."""
    from paper_1704_03151_amd import _C
    case = CASES["cavity16_kn10"]
    print("[walls] cavity16_kn10: set_wall_T", flush=True)
    gpu, prim = _perturbed(case, "fp64", 43)
    nfx = (case.nx + 1) * case.ny
    faces = np.array([nfx + 0, nfx + 3, nfx + 4, nfx + 15, nfx + case.ny * case.nx + 7])
    Tw = np.array([1.04, 0.97, 1.02, 0.95, 1.01])
    with pytest.raises(_C.MiugksError):
        gpu.set_wall_T([nfx + case.nx + 1], [1.0])       # an interior face
    with pytest.raises(_C.MiugksError):
        gpu.set_wall_T([nfx + 1], [0.0])
    before = gpu.wall_loads()
    gpu.set_wall_T(faces, Tw)
    c2 = case.with_(wall_y=case.wall_y.copy())
    for f, t in zip(faces, Tw):
        iy, ix = divmod(int(f) - nfx, case.nx)
        c2.wall_y[iy, ix, 0] = t
    orc = Oracle(c2)
    orc.init_macro(prim)           # the reference mass of the closed box, as on the GPU
    G, H = to_oracle(gpu.get_f())
    orc.set_f(G, H)
    got = gpu.wall_loads()
    ref = ad.wall_loads(orc.G, orc.H, orc.lev0, orc.vel, orc.gas, c2.farfield)
    assert rel_max(got[0], ref[0]) < 1e-12 and not np.allclose(got[0], before[0])
    gpu.iterate(3, tol=0.0)
    orc.iterate(3, tol=0.0)
    err = field_errors(gpu.macro(), orc.primitive(), orc.lev0.fluid)
    assert max(err.values()) < 1e-10, err
    gpu.close()
