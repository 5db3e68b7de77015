"""Thin ctypes binding of libfeti (include/feti.h).

Argument marshalling only: every step of the solver runs in the HIP kernels of
libfeti.so.  If the library is missing or no HIP device is present, the calls
raise -- there is no CPU fallback.

Module-level functions carry the C names (feti_setup, feti_factor, feti_solve,
feti_newton_step, feti_footprint, feti_destroy); :class:`Problem` wraps them.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfeti.so")

FETI_OK, FETI_EINVAL, FETI_ENOMEM, FETI_EDEVICE, FETI_ENOTSPD = 0, -1, -2, -3, -4
FETI_ENOCONV, FETI_ESTATE, FETI_EBREAKDOWN = -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTSPD",
                -5: "ENOCONV", -6: "ESTATE", -7: "EBREAKDOWN"}
VARIANTS = {"classical": 0, "af": 1, "all_floating": 1}
PRECONDS = {"identity": 0, "lumped": 1, "dirichlet": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
FETI_DEVICE_PTRS = 1
FETI_PROFILE = 2
FETI_AUTOTUNE = 4
AUTOTUNE_FACTORISATIONS = 4   # factorisations that time the update forms (FETI_AUTOTUNE)
FETI_KERNEL6 = 8
FETI_LOAD_STIFFNESS = 16
FETI_WARM_START = 32
FETI_DUAL_GMRES = 64

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class feti_material(C.Structure):
    _fields_ = [("kind", C.c_int32), ("E", C.c_double), ("nu", C.c_double), ("c", C.c_double),
                ("k1", C.c_double), ("k2", C.c_double), ("kappa", C.c_double)]


class feti_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("n_elems", C.c_int64), ("hex8", C.POINTER(C.c_int64)),
                ("n_sub", C.c_int32), ("elem_sub", C.POINTER(C.c_int32)),
                ("n_mat", C.c_int32), ("mat", C.POINTER(feti_material)),
                ("elem_mat", C.POINTER(C.c_int32)), ("elem_fibers", C.POINTER(C.c_double)),
                ("n_dir", C.c_int64), ("dir_dof", C.POINTER(C.c_int64)),
                ("dir_val", C.POINTER(C.c_double)), ("body_force", C.POINTER(C.c_double)),
                ("n_pfaces", C.c_int64), ("pface", C.POINTER(C.c_int64)), ("pressure", C.c_double),
                ("order", C.c_int32)]


class feti_options(C.Structure):
    _fields_ = [("variant", C.c_int), ("precond", C.c_int), ("precision", C.c_int),
                ("rtol", C.c_double), ("max_it", C.c_int32), ("ir_tol", C.c_double),
                ("ir_max", C.c_int32), ("graph_block", C.c_int32), ("hip_stream", C.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("flags", C.c_uint64), ("kernel_tol", C.c_double)]


class feti_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("ir_sweeps", C.c_int32),
                ("n_coarse", C.c_int32), ("n_lambda", C.c_int64), ("rel_res", C.c_double),
                ("kappa_est", C.c_double), ("t_assemble", C.c_double), ("t_factor", C.c_double),
                ("t_pcg", C.c_double), ("t_total", C.c_double), ("device_bytes", C.c_size_t),
                ("kernel_gemv_launches", C.c_int32), ("kernel_update_launches", C.c_int32),
                ("kernel_gemv_ms", C.c_double), ("kernel_update_ms", C.c_double),
                ("gemv_bytes", C.c_double), ("update_flops", C.c_double), ("res_primal", C.c_double),
                ("autotune_wide", C.c_int32),
                ("autotune_db", C.c_int32), ("modified_pivots", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FetiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfeti.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1508_02599_amd.build.build()")
    # PyTorch ships its own HIP and HSA runtimes under the sonames of the ROCm
    # ones the library links.  Loaded first, the library pulls in the ROCm
    # runtimes and a later torch import adds its own: two runtimes in one
    # process, and the second can fail to see the device.  Importing torch
    # first makes the library bind to torch's runtime: one per process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.feti_setup.argtypes = [C.POINTER(feti_mesh), C.POINTER(feti_options), C.POINTER(P)]
    lib.feti_setup.restype = C.c_int
    lib.feti_footprint.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.feti_footprint.restype = C.c_int
    lib.feti_factor.argtypes = [P, C.c_void_p]
    lib.feti_factor.restype = C.c_int
    lib.feti_solve.argtypes = [P, C.c_double, C.c_void_p, C.POINTER(feti_stats)]
    lib.feti_solve.restype = C.c_int
    lib.feti_solve_noalloc.argtypes = [P, C.c_double, C.c_void_p, C.POINTER(feti_stats)]
    lib.feti_solve_noalloc.restype = C.c_int
    lib.feti_newton_step.argtypes = [P, C.c_void_p, C.c_double, C.c_void_p, C.POINTER(C.c_double),
                                     C.POINTER(feti_stats)]
    lib.feti_newton_step.restype = C.c_int
    lib.feti_set_tolerances.argtypes = [P, C.c_double, C.c_double]
    lib.feti_set_tolerances.restype = C.c_int
    lib.feti_last_error.argtypes = [P]
    lib.feti_last_error.restype = C.c_char_p
    lib.feti_destroy.argtypes = [P]
    lib.feti_destroy.restype = None
    _lib = lib
    return lib


EXPORTED = ("feti_setup", "feti_footprint", "feti_factor", "feti_solve", "feti_solve_noalloc",
            "feti_newton_step", "feti_set_tolerances", "feti_last_error", "feti_destroy")


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _mesh_struct(mesh, keep):
    """Marshal a workloads.Mesh-like object into a feti_mesh (arrays kept alive in `keep`)."""
    xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
    hex8 = np.ascontiguousarray(mesh.hex8, dtype=np.int64)
    es = np.ascontiguousarray(mesh.elem_sub, dtype=np.int32)
    em = np.ascontiguousarray(mesh.elem_mat, dtype=np.int32)
    mt = np.asarray(mesh.mat, dtype=np.float64).reshape(-1, 7)
    mats = (feti_material * mt.shape[0])()
    for k, row in enumerate(mt):
        mats[k] = feti_material(int(row[0]), *[float(v) for v in row[1:]])
    dd = np.ascontiguousarray(mesh.dir_dof, dtype=np.int64)
    dv = np.ascontiguousarray(mesh.dir_val, dtype=np.float64)
    bf = None if mesh.body_force is None else np.ascontiguousarray(mesh.body_force, dtype=np.float64)
    fb = None if getattr(mesh, "fibers", None) is None else np.ascontiguousarray(mesh.fibers, dtype=np.float64)
    pf = None if getattr(mesh, "pface", None) is None else np.ascontiguousarray(mesh.pface, dtype=np.int64)
    keep.extend([xyz, hex8, es, em, mats, dd, dv, bf, fb, pf])
    m = feti_mesh()
    m.n_nodes = xyz.shape[0]
    m.xyz = _ptr(xyz, C.c_double)
    m.n_elems = hex8.shape[0]
    m.hex8 = _ptr(hex8, C.c_int64)
    m.n_sub = int(mesh.n_sub)
    m.elem_sub = _ptr(es, C.c_int32)
    m.n_mat = mt.shape[0]
    m.mat = C.cast(mats, C.POINTER(feti_material))
    m.elem_mat = _ptr(em, C.c_int32)
    m.elem_fibers = _ptr(fb, C.c_double)
    m.n_dir = dd.shape[0]
    m.dir_dof = _ptr(dd, C.c_int64)
    m.dir_val = _ptr(dv, C.c_double)
    m.body_force = _ptr(bf, C.c_double)
    m.n_pfaces = 0 if pf is None else pf.shape[0]
    m.pface = _ptr(pf, C.c_int64)
    m.pressure = float(getattr(mesh, "pressure", 0.0))
    npe = hex8.shape[1] if hex8.ndim == 2 else 8
    if npe not in (8, 27):
        raise ValueError(f"elements with {npe} nodes: expected 8 (Q1) or 27 (Q2)")
    if pf is not None and pf.shape[1] != (4 if npe == 8 else 9):
        raise ValueError(f"pressure faces with {pf.shape[1]} nodes on {npe}-node elements")
    m.order = 1 if npe == 8 else 2
    return m


def _check(lib, handle, status):
    if status not in (FETI_OK,):
        msg = lib.feti_last_error(handle)
        raise FetiError(status, msg.decode() if msg else "")
    return status


def feti_setup(mesh, variant="af", precond="lumped", precision="fp64", rtol=1e-8, max_it=1000,
               graph_block=8, ir_tol=1e-10, ir_max=6, hip_stream=None, device_ptrs=False,
               torch_allocator=False, profile=False, autotune=True, kernel6=False, load_stiffness=False,
               warm_start=False, dual_gmres=False, kernel_tol=0.0):
    """Create a problem handle (see :class:`Problem`)."""
    return Problem(mesh, variant, precond, precision, rtol, max_it, graph_block, ir_tol, ir_max,
                   hip_stream, device_ptrs, torch_allocator, profile, autotune, kernel6, load_stiffness,
                   warm_start, dual_gmres, kernel_tol)


class Problem:
    """A FETI problem resident on the GPU."""

    def __init__(self, mesh, variant="af", precond="lumped", precision="fp64", rtol=1e-8, max_it=1000,
                 graph_block=8, ir_tol=1e-10, ir_max=6, hip_stream=None, device_ptrs=False,
                 torch_allocator=False, profile=False, autotune=True, kernel6=False, load_stiffness=False,
                 warm_start=False, dual_gmres=False, kernel_tol=0.0):
        self.lib = load_library()
        self.n_dof = 3 * int(np.asarray(mesh.xyz).shape[0])
        keep = []
        m = _mesh_struct(mesh, keep)
        o = feti_options()
        o.variant = VARIANTS[variant]
        o.precond = PRECONDS[precond]
        o.precision = PRECISIONS[precision]
        o.rtol = rtol
        o.max_it = max_it
        o.ir_tol = ir_tol
        o.ir_max = ir_max
        o.graph_block = graph_block
        o.kernel_tol = kernel_tol
        o.hip_stream = hip_stream
        o.flags = ((FETI_DEVICE_PTRS if device_ptrs else 0) | (FETI_PROFILE if profile else 0)
                   | (FETI_AUTOTUNE if autotune else 0) | (FETI_KERNEL6 if kernel6 else 0)
                   | (FETI_LOAD_STIFFNESS if load_stiffness else 0) | (FETI_WARM_START if warm_start else 0)
                   | (FETI_DUAL_GMRES if dual_gmres else 0))
        self._cb = None
        if torch_allocator:
            import torch

            def _alloc(nbytes, stream, ctx):
                return torch.cuda.caching_allocator_alloc(int(nbytes), stream=stream)

            def _free(ptr, ctx):
                torch.cuda.caching_allocator_delete(ptr)

            self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
            o.dev_alloc, o.dev_free = self._cb
        self.device_ptrs = device_ptrs
        h = C.c_void_p()
        st = self.lib.feti_setup(C.byref(m), C.byref(o), C.byref(h))
        if st != FETI_OK:
            raise FetiError(st, self.lib.feti_last_error(None).decode())
        self.h = h
        self.variant, self.precond, self.precision = variant, precond, precision

    # -------------------------------------------------------------------
    def footprint(self) -> int:
        n = C.c_size_t()
        _check(self.lib, self.h, self.lib.feti_footprint(self.h, C.byref(n)))
        return int(n.value)

    def _arg(self, a):
        if a is None:
            return None
        if self.device_ptrs:
            return C.c_void_p(int(a.data_ptr()))
        return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(C.c_void_p)

    def factor(self, U=None):
        Ua = None if U is None or self.device_ptrs else np.ascontiguousarray(U, dtype=np.float64)
        arg = self._arg(U) if self.device_ptrs else (None if Ua is None else Ua.ctypes.data_as(C.c_void_p))
        _check(self.lib, self.h, self.lib.feti_factor(self.h, arg))

    def solve(self, load_factor=1.0, out=None, allow_noconv=False):
        """Returns (u, stats).  u: numpy [3*n_nodes] (or the given device tensor)."""
        stats = feti_stats()
        if self.device_ptrs:
            assert out is not None
            ptr = C.c_void_p(int(out.data_ptr()))
            u = out
        else:
            u = np.empty(self.n_dof) if out is None else out
            ptr = u.ctypes.data_as(C.c_void_p)
        st = self.lib.feti_solve(self.h, float(load_factor), ptr, C.byref(stats))
        if not (allow_noconv and st == FETI_ENOCONV):
            _check(self.lib, self.h, st)
        return u, stats.as_dict()

    def solve_noalloc(self, out, load_factor=1.0):
        """feti_solve_noalloc into the device tensor ``out`` (needs
        device_ptrs=True); returns (out, stats)."""
        assert self.device_ptrs and out is not None
        stats = feti_stats()
        _check(self.lib, self.h, self.lib.feti_solve_noalloc(self.h, float(load_factor),
                                                             C.c_void_p(int(out.data_ptr())),
                                                             C.byref(stats)))
        return out, stats.as_dict()

    def newton_step(self, U, tau, out=None, allow_noconv=False):
        """Returns (dU, residual norm, stats) of one Newton step at U with load factor tau
        (allow_noconv: a step whose refinement stopped short of ir_tol is returned)."""
        stats = feti_stats()
        rn = C.c_double()
        if self.device_ptrs:
            dU = out
            uptr = C.c_void_p(int(U.data_ptr()))
            optr = C.c_void_p(int(out.data_ptr()))
        else:
            Ua = np.ascontiguousarray(U, dtype=np.float64)
            dU = np.empty(self.n_dof) if out is None else out
            uptr = Ua.ctypes.data_as(C.c_void_p)
            optr = dU.ctypes.data_as(C.c_void_p)
        st = self.lib.feti_newton_step(self.h, uptr, float(tau), optr, C.byref(rn), C.byref(stats))
        if not (allow_noconv and st == FETI_ENOCONV):
            _check(self.lib, self.h, st)
        return dU, rn.value, stats.as_dict()

    def set_tolerances(self, rtol, ir_tol):
        """feti_set_tolerances: dual rtol and refinement ir_tol of later calls."""
        _check(self.lib, self.h, self.lib.feti_set_tolerances(self.h, float(rtol), float(ir_tol)))

    def close(self):
        if getattr(self, "h", None):
            self.lib.feti_destroy(self.h)
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


def feti_factor(problem: Problem, U=None):
    problem.factor(U)


def feti_solve(problem: Problem, load_factor=1.0, out=None):
    return problem.solve(load_factor, out)


def feti_newton_step(problem: Problem, U, tau, out=None):
    return problem.newton_step(U, tau, out)


def feti_footprint(problem: Problem) -> int:
    return problem.footprint()


def feti_destroy(problem: Problem):
    problem.close()
