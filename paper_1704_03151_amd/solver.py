"""Python handle of one MIUGKS problem on the GPU (thin wrapper of the C ABI).

All computation happens in libmiugks.so; this class only converts a
`workloads.Case` into the C descriptors and numpy arrays into pointers.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _C

_QUAD = {"trapezoid": _C.QUAD_TRAPEZOID, "simpson38": _C.QUAD_SIMPSON38,
         "gauss_hermite": _C.QUAD_GAUSS_HERMITE}
_PREC = {"fp64": _C.FP64, "fp32f": _C.FP32F}


def _stream_handle(stream):
    if stream is not None:
        return int(stream)
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:   # torch absent or without a device: default stream
        pass
    return 0


_ALLOCATORS = []   # every callback pair handed to the library: a context uses its pair until destroyed


def use_torch_allocator(on=True):
    """Back the device memory of the contexts created from now on by PyTorch's
    caching allocator (on=False: hipMalloc again).  The callbacks only forward
    to torch.cuda.caching_allocator_alloc / caching_allocator_delete."""
    if not on:
        return _C.lib.miugks_set_allocator(_C.ALLOC_FN(), _C.FREE_FN(), None)
    import torch

    def alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:
            return None

    def free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    pair = (_C.ALLOC_FN(alloc), _C.FREE_FN(free))
    _ALLOCATORS.append(pair)
    return _C.lib.miugks_set_allocator(pair[0], pair[1], None)


class Solver:
    """One context: create from a case, iterate, read fields."""

    def __init__(self, case, precision=None, stream=None, mass_renorm=-1):
        self.case = case
        prec = _PREC[precision or case.precision]
        self.precision = prec
        self.dtype = np.float64 if prec == _C.FP64 else np.float32
        kind = _QUAD[case.quad]
        self.u1, self.wu = _C.quadrature(kind, case.nu, case.vlo, case.vhi)
        self.v1, self.wv = _C.quadrature(kind, case.nv, case.vlo, case.vhi)
        # keep every array alive while the descriptors point at them
        self._keep = [np.ascontiguousarray(a) for a in (
            np.asarray(case.x, float), np.asarray(case.y, float),
            np.asarray(case.face_type_x, np.uint8), np.asarray(case.face_type_y, np.uint8),
            np.asarray(case.wall_x, float), np.asarray(case.wall_y, float),
            np.asarray(case.solid, np.uint8))]
        x, y, ftx, fty, wx, wy, sol = self._keep
        mesh = _C.MeshDesc(case.nx, case.ny, case.n_levels, _C.dptr(x), _C.dptr(y), _C.u8ptr(ftx),
                           _C.u8ptr(fty), _C.dptr(wx), _C.dptr(wy), _C.u8ptr(sol))
        vg = _C.VGridDesc(case.nu, case.nv, _C.dptr(self.u1), _C.dptr(self.v1), _C.dptr(self.wu),
                          _C.dptr(self.wv))
        rho, U, V, T = case.farfield
        gas = _C.GasDesc(case.K_int, case.Pr, case.omega, case.Kn, rho, U, V, T)
        sd = _C.SolverDesc(prec, case.nu1, case.nu2, case.nu_coarse, case.cfl, case.dtn_growth,
                           mass_renorm, getattr(case, "fas_levels", 0), getattr(case, "nu_coarse_cs", 0),
                           getattr(case, "cycle_gamma", 1), getattr(case, "cycle_gamma_cs", 0),
                           getattr(case, "dtn_max", 0.0))
        h = ctypes.c_void_p()
        rc = _C.lib.miugks_create(ctypes.byref(h), ctypes.byref(mesh), ctypes.byref(vg),
                                  ctypes.byref(gas), ctypes.byref(sd), ctypes.c_void_p(_stream_handle(stream)))
        if rc:
            raise _C.MiugksError(rc, _C.lib.miugks_last_error(None).decode())
        self.h = h
        # bumped by every call that changes the distribution or the wall
        # temperatures (lets a saved state be recognised as current)
        self.state_version = 0
        nc, nf, nk, nl = (ctypes.c_int() for _ in range(4))
        _C.lib.miugks_sizes(h, ctypes.byref(nc), ctypes.byref(nf), ctypes.byref(nk), ctypes.byref(nl))
        self.nc, self.n_fluid, self.nk, self.n_levels = nc.value, nf.value, nk.value, nl.value
        self.fshape = (2, self.nk, case.ny, case.nx)
        self.init_macro(case.init)

    # ------------------------------------------------------------------ plumbing
    def _check(self, rc, allow=()):
        if rc and rc not in allow:
            raise _C.MiugksError(rc, _C.lib.miugks_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            _C.lib.miugks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _cells(self, a, m=None):
        shape = (self.case.ny, self.case.nx) if m is None else (m, self.case.ny, self.case.nx)
        out = np.ascontiguousarray(np.asarray(a, float).reshape(shape))
        return out

    # ------------------------------------------------------------------ API
    def init_macro(self, prim):
        self.state_version += 1
        p = [self._cells(a) for a in prim]
        self._check(_C.lib.miugks_init_macro(self.h, *(_C.dptr(a) for a in p)))

    def iterate(self, max_cycles, tol=1e-6):
        """Returns (status, cycles_done, residual norms); status OK, ENOTCONVERGED or EDIVERGED."""
        self.state_version += 1
        n = ctypes.c_int()
        res = np.zeros(4)
        rc = _C.lib.miugks_iterate(self.h, int(max_cycles), float(tol), ctypes.byref(n), _C.dptr(res))
        self._check(rc, allow=(_C.ENOTCONVERGED, _C.EDIVERGED))
        return rc, n.value, res

    def fmg(self, cycles_per_level, tol=1e-6):
        """Full-multigrid start from the current state; returns (status, cycles run)."""
        self.state_version += 1
        n = ctypes.c_int()
        rc = _C.lib.miugks_fmg(self.h, int(cycles_per_level), float(tol), ctypes.byref(n))
        self._check(rc, allow=(_C.EDIVERGED,))
        return rc, n.value

    def explicit(self, steps):
        """Explicit time-accurate UGKS steps; returns (dt, RMS residuals of the last step)."""
        self.state_version += 1
        dt = np.zeros(1)
        res = np.zeros(4)
        self._check(_C.lib.miugks_explicit(self.h, int(steps), _C.dptr(dt), _C.dptr(res)))
        return float(dt[0]), res

    def macro(self):
        shape = (self.case.ny, self.case.nx)
        out = {k: np.zeros(shape) for k in ("rho", "U", "V", "T", "qx", "qy")}
        self._check(_C.lib.miugks_get_macro(self.h, *(_C.dptr(out[k]) for k in ("rho", "U", "V", "T", "qx", "qy"))))
        return out

    def _device_f(self, t):
        """(pointer, dtype code) of a contiguous torch tensor on the GPU shaped like f."""
        import torch
        if t.dtype not in (torch.float32, torch.float64) or tuple(t.shape) != self.fshape:
            raise ValueError(f"f must be float32/float64 shaped {self.fshape}")
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("a device f must be a contiguous tensor on the GPU")
        return ctypes.c_void_p(t.data_ptr()), (_C.FP64 if t.dtype == torch.float64 else _C.FP32F)

    def get_f(self, dtype=None, out=None):
        """The distribution [2][Nk][ny][nx] as a host array of dtype, or into
        `out`, a torch tensor on the GPU (converted there by the library)."""
        if out is not None and not isinstance(out, np.ndarray):
            ptr, code = self._device_f(out)
            self._check(_C.lib.miugks_get_f(self.h, ptr, code, 1))
            return out
        dt = np.dtype(dtype or self.dtype)
        out = np.zeros(self.fshape, dt)
        code = _C.FP64 if dt == np.float64 else _C.FP32F
        self._check(_C.lib.miugks_get_f(self.h, out.ctypes.data_as(ctypes.c_void_p), code, 0))
        return out

    def get_f_noalloc(self, dtype=None):
        """The distribution as a host array of dtype through the library's
        allocation-free entry point (miugks_get_f_noalloc)."""
        dt = np.dtype(dtype or self.dtype)
        out = np.zeros(self.fshape, dt)
        code = _C.FP64 if dt == np.float64 else _C.FP32F
        self._check(_C.lib.miugks_get_f_noalloc(self.h, out.ctypes.data_as(ctypes.c_void_p), code))
        return out

    def set_f(self, f):
        """Set the distribution from a host array or a torch tensor on the GPU."""
        self.state_version += 1
        if not isinstance(f, np.ndarray) and hasattr(f, "data_ptr"):
            ptr, code = self._device_f(f)
            self._check(_C.lib.miugks_set_f(self.h, ptr, code, 1))
            return
        a = np.ascontiguousarray(f)
        code = _C.FP64 if a.dtype == np.float64 else _C.FP32F
        if a.dtype not in (np.float64, np.float32) or a.shape != self.fshape:
            raise ValueError(f"f must be float32/float64 shaped {self.fshape}")
        self._check(_C.lib.miugks_set_f(self.h, a.ctypes.data_as(ctypes.c_void_p), code, 0))

    def wall_list(self):
        """(cell, side) of every wall side of the finest level, in library order."""
        n = ctypes.c_int()
        self._check(_C.lib.miugks_wall_list(self.h, None, None, ctypes.byref(n)))
        cell = np.zeros(n.value, np.int32)
        side = np.zeros(n.value, np.int32)
        self._check(_C.lib.miugks_wall_list(self.h, _C.iptr(cell), _C.iptr(side), ctypes.byref(n)))
        return cell, side

    def wall_loads(self):
        """Array (4, n_walls): pressure, shear, heat flux, face area per wall side."""
        n = ctypes.c_int()
        self._check(_C.lib.miugks_wall_loads(self.h, None, None, None, None, ctypes.byref(n)))
        out = np.zeros((4, n.value))
        self._check(_C.lib.miugks_wall_loads(self.h, *(_C.dptr(out[m]) for m in range(4)), ctypes.byref(n)))
        return out

    def objective(self, kind, walls):
        ids = np.ascontiguousarray(walls, np.int32)
        J = np.zeros(1)
        self._check(_C.lib.miugks_objective(self.h, int(kind), _C.iptr(ids), len(ids), _C.dptr(J)))
        return float(J[0])

    def set_wall_T(self, faces, Tw):
        self.state_version += 1
        ids = np.ascontiguousarray(faces, np.int32)
        T = np.ascontiguousarray(Tw, float)
        if T.shape != ids.shape:
            raise ValueError("one temperature per face")
        self._check(_C.lib.miugks_set_wall_T(self.h, _C.iptr(ids), _C.dptr(T), len(ids)))

    def residual_adjoint(self, v):
        """(dr/df)^T v of the steady residual at the current f (FP64 contexts)."""
        a = np.ascontiguousarray(v, np.float64)
        if a.shape != self.fshape:
            raise ValueError(f"v must be shaped {self.fshape}")
        out = np.zeros(self.fshape)
        self._check(_C.lib.miugks_residual_adjoint(self.h, a.ctypes.data_as(ctypes.c_void_p),
                                                   out.ctypes.data_as(ctypes.c_void_p), _C.FP64, 0))
        return out

    def adjoint(self, kind, walls, faces, tol=1e-10, max_iter=2000, krylov_precision="fp64"):
        """dJ/dTw of J = sum_walls S load_kind for the listed mesh faces; returns
        (status, gradient, corrections, relative residual).  krylov_precision
        "fp32" keeps the Krylov basis and the preconditioner's vectors in float
        (miugks_adjoint_ex)."""
        if krylov_precision not in ("fp64", "fp32"):
            raise ValueError("krylov_precision must be 'fp64' or 'fp32'")
        ids = np.ascontiguousarray(walls, np.int32)
        fc = np.ascontiguousarray(faces, np.int32)
        g = np.zeros(len(fc))
        it = ctypes.c_int()
        res = np.zeros(1)
        code = _C.FP32F if krylov_precision == "fp32" else _C.FP64
        rc = _C.lib.miugks_adjoint_ex(self.h, int(kind), _C.iptr(ids), len(ids), _C.iptr(fc), len(fc), float(tol),
                                      int(max_iter), code, _C.dptr(g), ctypes.byref(it), _C.dptr(res))
        self._check(rc, allow=(_C.ENOTCONVERGED,))
        return rc, g, it.value, float(res[0])

    def residual(self):
        R = np.zeros((4, self.case.ny, self.case.nx))
        res = np.zeros(4)
        self._check(_C.lib.miugks_residual(self.h, _C.dptr(R), _C.dptr(res)))
        return R, res

    def div(self, dtype=None):
        dt = np.dtype(dtype or self.dtype)
        out = np.zeros(self.fshape, dt)
        code = _C.FP64 if dt == np.float64 else _C.FP32F
        self._check(_C.lib.miugks_get_div(self.h, out.ctypes.data_as(ctypes.c_void_p), code, 0))
        return out

    def predict(self, W, R):
        W = self._cells(W, 4)
        R = self._cells(R, 4)
        out = np.zeros_like(W)
        self._check(_C.lib.miugks_predict(self.h, _C.dptr(W), _C.dptr(R), _C.dptr(out)))
        return out

    def micro_residual(self, Wt, dtype=None):
        Wt = self._cells(Wt, 4)
        dt = np.dtype(dtype or self.dtype)
        r = np.zeros(self.fshape, dt)
        ti = np.zeros((self.case.ny, self.case.nx))
        code = _C.FP64 if dt == np.float64 else _C.FP32F
        self._check(_C.lib.miugks_micro_residual(self.h, _C.dptr(Wt), r.ctypes.data_as(ctypes.c_void_p),
                                                 _C.dptr(ti), code, 0))
        return r, ti

    def set_timing(self, on=True):
        self._check(_C.lib.miugks_set_timing(self.h, 1 if on else 0))

    def timing(self):
        """{label: (launches, total ms, algorithmic bytes)} since set_timing(True)."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        launches = (ctypes.c_int * cap)()
        ms = np.zeros(cap)
        by = np.zeros(cap)
        n = _C.lib.miugks_timing(self.h, cap, names, launches, _C.dptr(ms), _C.dptr(by))
        if n < 0:
            self._check(-n)
        return {names[i].decode(): (launches[i], float(ms[i]), float(by[i])) for i in range(min(n, cap))}

    def correct(self, r, tau_inv):
        a = np.ascontiguousarray(r)
        code = _C.FP64 if a.dtype == np.float64 else _C.FP32F
        ti = self._cells(tau_inv)
        out = np.zeros_like(a)
        self._check(_C.lib.miugks_correct(self.h, a.ctypes.data_as(ctypes.c_void_p), _C.dptr(ti),
                                          out.ctypes.data_as(ctypes.c_void_p), code, 0))
        return out
