"""MI355X (gfx950) TV-regularised CT reconstruction: Python binding.

A thin ctypes layer over ``libtvreg.so`` (C ABI in ``include/tvreg.h``):
torch tensors supply device memory and the current HIP stream, every step
of the computation runs in the library's HIP kernels.  There is no CPU
fallback: if the library has not been built, importing this package raises.

Entry points mirror the C names: ``Geometry`` (tvreg_create_geometry),
``project``, ``backproject``, ``tv_grad``, ``objective_grad`` and ``solve``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch  # loads the HIP runtime the library binds to

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtvreg.so")

PARALLEL, CONE, PARALLEL_3D = 0, 1, 2
F32, F64 = 0, 1
GP, GPBB, UPN, NESTEROV = 0, 1, 2, 3
OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, ESTALL = 0, -1, -2, -3, 1, 2

_c_dp = ctypes.POINTER(ctypes.c_double)


class _Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n_views", ctypes.c_int32), ("angles_rad", _c_dp),
                ("beam", ctypes.c_int), ("det_cols", ctypes.c_int32),
                ("det_rows", ctypes.c_int32), ("pitch_u", ctypes.c_double),
                ("pitch_v", ctypes.c_double), ("src_to_centre", ctypes.c_double),
                ("src_to_det", ctypes.c_double), ("view_dirs", _c_dp)]


class _SolveParams(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("alpha", ctypes.c_double), ("tau", ctypes.c_double),
                ("eps", ctypes.c_double), ("stop_mode", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("L_bar", ctypes.c_double),
                ("mu_bar", ctypes.c_double), ("rho_L", ctypes.c_double),
                ("gpbb_K", ctypes.c_int32), ("gpbb_sigma", ctypes.c_double),
                ("gpbb_beta0", ctypes.c_double), ("max_trials", ctypes.c_int32),
                ("hist_phi", _c_dp), ("hist_gm", _c_dp), ("hist_L", _c_dp),
                ("hist_len", ctypes.c_int32), ("use_box", ctypes.c_int32),
                ("lower", ctypes.c_double), ("upper", ctypes.c_double)]


class _Tuning(ctypes.Structure):
    _fields_ = [("project_tile_cols", ctypes.c_int32), ("project_waves", ctypes.c_int32),
                ("backproject_depth", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("project_ms", (ctypes.c_double * 4) * 6),
                ("backproject_ms", ctypes.c_double * 3)]


PROJECT_TILE_COLS = (1, 2, 8, 16, 32, 64)
PROJECT_WAVES = (1, 2, 4, 8)
BACKPROJECT_DEPTHS = (4, 8, 16)


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("grad_evals", ctypes.c_int32),
                ("func_evals", ctypes.c_int32), ("phi", ctypes.c_double),
                ("gm_rel", ctypes.c_double), ("gm_abs_over_N", ctypes.c_double),
                ("L", ctypes.c_double), ("mu", ctypes.c_double),
                ("stop_reason", ctypes.c_int32)]


# Every symbol include/tvreg.h declares.
EXPORTS = ("tvreg_create_geometry", "tvreg_destroy_geometry", "tvreg_project",
           "tvreg_project_workspace_bytes", "tvreg_project_ws", "tvreg_backproject", "tvreg_matrix_scratch_bytes", "tvreg_matrix_plan",
           "tvreg_matrix_attach", "tvreg_matrix_detach", "tvreg_set_symmetry",
           "tvreg_matrix_symmetry", "tvreg_autotune_workspace_bytes",
           "tvreg_autotune", "tvreg_get_tuning", "tvreg_set_tuning", "tvreg_tv_workspace_bytes",
           "tvreg_tv_grad", "tvreg_tv_grad_noalloc", "tvreg_tv_hessvec",
           "tvreg_objective_workspace_bytes", "tvreg_objective_grad",
           "tvreg_solve_workspace_bytes", "tvreg_solve", "tvreg_solve_batched_workspace_bytes",
           "tvreg_solve_batched", "tvreg_unrolled_workspace_bytes", "tvreg_upn_unrolled_fwd",
           "tvreg_upn_unrolled_bwd", "tvreg_profile_enable", "tvreg_profile_reset",
           "tvreg_profile_get", "tvreg_last_error", "tvreg_version")

KERNELS = {"project": 0, "backproject": 1, "tv": 2, "trial": 3, "extrapolate": 4,
           "transpose": 5}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          f"`python paper_1105_4002_amd/build.py` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, st = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    L.tvreg_create_geometry.argtypes = [ctypes.POINTER(_Desc), ctypes.c_int,
                                        ctypes.POINTER(vp)]
    L.tvreg_create_geometry.restype = st
    L.tvreg_destroy_geometry.argtypes = [vp]
    L.tvreg_destroy_geometry.restype = None
    L.tvreg_project.argtypes = [vp, vp, vp, vp]
    L.tvreg_project.restype = st
    L.tvreg_project_workspace_bytes.argtypes = [vp]
    L.tvreg_project_workspace_bytes.restype = sz
    L.tvreg_project_ws.argtypes = [vp, vp, vp, vp, sz, vp]
    L.tvreg_project_ws.restype = st
    L.tvreg_backproject.argtypes = [vp, vp, vp, vp]
    L.tvreg_backproject.restype = st
    L.tvreg_matrix_scratch_bytes.argtypes = [vp]
    L.tvreg_matrix_scratch_bytes.restype = sz
    L.tvreg_matrix_plan.argtypes = [vp, vp, sz, ctypes.POINTER(sz),
                                    ctypes.POINTER(ctypes.c_int64), vp]
    L.tvreg_matrix_plan.restype = st
    L.tvreg_matrix_attach.argtypes = [vp, vp, sz, vp]
    L.tvreg_matrix_attach.restype = st
    L.tvreg_matrix_detach.argtypes = [vp]
    L.tvreg_matrix_detach.restype = st
    L.tvreg_set_symmetry.argtypes = [vp, ctypes.c_int32]
    L.tvreg_set_symmetry.restype = st
    L.tvreg_matrix_symmetry.argtypes = [vp]
    L.tvreg_matrix_symmetry.restype = ctypes.c_int32
    L.tvreg_autotune_workspace_bytes.argtypes = [vp]
    L.tvreg_autotune_workspace_bytes.restype = sz
    L.tvreg_autotune.argtypes = [vp, vp, sz, ctypes.c_int32, ctypes.POINTER(_Tuning), vp]
    L.tvreg_autotune.restype = st
    L.tvreg_get_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    L.tvreg_get_tuning.restype = st
    L.tvreg_set_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    L.tvreg_set_tuning.restype = st
    L.tvreg_tv_workspace_bytes.argtypes = [ctypes.c_int32] * 3
    L.tvreg_tv_workspace_bytes.restype = sz
    L.tvreg_tv_grad.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_int, ctypes.c_double, vp, vp,
                                                       vp, vp, sz, vp]
    L.tvreg_tv_grad.restype = st
    L.tvreg_tv_grad_noalloc.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_int, ctypes.c_double, vp,
                                                               vp, vp, vp]
    L.tvreg_tv_grad_noalloc.restype = st
    L.tvreg_tv_hessvec.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_int, ctypes.c_double, vp, vp,
                                                          vp, vp, vp, sz, vp]
    L.tvreg_tv_hessvec.restype = st
    L.tvreg_objective_workspace_bytes.argtypes = [vp]
    L.tvreg_objective_workspace_bytes.restype = sz
    L.tvreg_objective_grad.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp,
                                       sz, vp]
    L.tvreg_objective_grad.restype = st
    L.tvreg_solve_workspace_bytes.argtypes = [vp, ctypes.c_int]
    L.tvreg_solve_workspace_bytes.restype = sz
    L.tvreg_solve.argtypes = [vp, vp, ctypes.POINTER(_SolveParams), vp, vp, sz,
                              ctypes.POINTER(_SolveInfo), vp]
    L.tvreg_solve.restype = st
    L.tvreg_solve_batched_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(vp)]
    L.tvreg_solve_batched_workspace_bytes.restype = sz
    L.tvreg_solve_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(_SolveParams), ctypes.POINTER(vp), vp, sz,
                                      ctypes.c_int32, ctypes.POINTER(_SolveInfo), vp]
    L.tvreg_solve_batched.restype = st
    dp = ctypes.POINTER(ctypes.c_double)
    L.tvreg_unrolled_workspace_bytes.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.tvreg_unrolled_workspace_bytes.restype = sz
    L.tvreg_upn_unrolled_fwd.argtypes = [vp, vp, ctypes.POINTER(_SolveParams), ctypes.c_int32,
                                         ctypes.c_int32, dp, dp, vp, vp, sz, vp]
    L.tvreg_upn_unrolled_fwd.restype = st
    L.tvreg_upn_unrolled_bwd.argtypes = [vp, vp, vp, sz, vp, dp, vp, vp]
    L.tvreg_upn_unrolled_bwd.restype = st
    L.tvreg_profile_enable.argtypes = [ctypes.c_int32]
    L.tvreg_profile_enable.restype = None
    L.tvreg_profile_reset.argtypes = []
    L.tvreg_profile_reset.restype = None
    L.tvreg_profile_get.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_double)]
    L.tvreg_profile_get.restype = st
    L.tvreg_last_error.restype = ctypes.c_char_p
    L.tvreg_version.restype = ctypes.c_char_p
    return L


_lib = _load()


def lib():
    return _lib


class TvregError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.tvreg_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def _check(status: int, where: str) -> int:
    if status < 0:
        raise TvregError(status, where)
    return status


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dtype(precision: int):
    return torch.float64 if precision == F64 else torch.float32


def _ptr(t: torch.Tensor, dtype, numel: int, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Geometry:
    """Device ray tables of one scan geometry (tvreg_create_geometry)."""

    def __init__(self, desc, precision: int = F32):
        self._angles = (ctypes.c_double * len(desc.angles))(*[float(a) for a in desc.angles])
        dirs = getattr(desc, "dirs", None)
        if int(desc.beam) == PARALLEL_3D:
            flat = [float(v) for v in np.asarray(dirs, dtype=np.float64).reshape(-1)]
            if len(flat) != 3 * len(desc.angles):
                raise ValueError("a 3D parallel beam needs one direction per view")
            self._dirs = (ctypes.c_double * len(flat))(*flat)
            dp = ctypes.cast(self._dirs, _c_dp)
        else:
            self._dirs = None
            dp = _c_dp()
        d = _Desc(int(desc.nx), int(desc.ny), int(desc.nz), len(desc.angles),
                  ctypes.cast(self._angles, _c_dp), int(desc.beam), int(desc.det_cols),
                  int(desc.det_rows), float(desc.pitch_u), float(desc.pitch_v),
                  float(desc.src_to_centre), float(desc.src_to_det), dp)
        h = ctypes.c_void_p()
        _check(_lib.tvreg_create_geometry(ctypes.byref(d), int(precision), ctypes.byref(h)),
               "tvreg_create_geometry")
        self.handle = h
        self.precision = int(precision)
        self.dtype = _dtype(precision)
        self.vol_shape = (int(desc.nz), int(desc.ny), int(desc.nx))
        self.proj_shape = (len(desc.angles), int(desc.det_rows), int(desc.det_cols))
        self.N = self.vol_shape[0] * self.vol_shape[1] * self.vol_shape[2]
        self.m = self.proj_shape[0] * self.proj_shape[1] * self.proj_shape[2]

    def __del__(self):
        h = getattr(self, "handle", None)
        lib_ = globals().get("_lib")  # gone already at interpreter shutdown
        if h is not None and h.value and lib_ is not None:
            lib_.tvreg_destroy_geometry(h)
            self.handle = None

    def set_symmetry(self, use: bool) -> None:
        """Whether a stored transpose and the on-the-fly backprojector use
        the scan's symmetry (tvreg_set_symmetry; on by default).  Not while a
        matrix is attached."""
        _check(_lib.tvreg_set_symmetry(self.handle, 1 if use else 0), "tvreg_set_symmetry")

    def attach_matrix(self, device="cuda", symmetric: bool = True) -> int:
        """Builds the stored system matrix (tvreg_matrix_plan / _attach) in a
        torch allocation the geometry keeps; returns the number of non-zeros
        of A.  With symmetric (the default) a circular cone scan that maps
        onto itself under turns and the z mirror stores one cell of voxels
        (symmetric=False: every voxel).  `symmetry` then holds the voxels one
        stored entry serves."""
        self.set_symmetry(symmetric)
        scratch = torch.empty(_lib.tvreg_matrix_scratch_bytes(self.handle), dtype=torch.uint8,
                              device=device)
        nbytes = ctypes.c_size_t(0)
        nnz = ctypes.c_int64(0)
        stream = ctypes.c_void_p(torch.cuda.current_stream(scratch.device).cuda_stream)
        _check(_lib.tvreg_matrix_plan(self.handle, ctypes.c_void_p(scratch.data_ptr()),
                                      scratch.numel(), ctypes.byref(nbytes), ctypes.byref(nnz),
                                      stream), "tvreg_matrix_plan")
        del scratch
        buf = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        _check(_lib.tvreg_matrix_attach(self.handle, ctypes.c_void_p(buf.data_ptr()),
                                        buf.numel(), stream), "tvreg_matrix_attach")
        self._matrix = buf
        self.nnz = int(nnz.value)
        self.symmetry = int(_lib.tvreg_matrix_symmetry(self.handle))
        return self.nnz

    def detach_matrix(self) -> None:
        _check(_lib.tvreg_matrix_detach(self.handle), "tvreg_matrix_detach")
        self._matrix = None
        self.symmetry = 0

    @property
    def matrix_bytes(self) -> int:
        m = getattr(self, "_matrix", None)
        return 0 if m is None else m.numel()

    def autotune(self, reps: int = 5, device="cuda") -> dict:
        """Times every tile shape of the on-the-fly projector and
        backprojector on this geometry (tvreg_autotune), keeps the fastest and
        returns the choice with all timings (ms per launch)."""
        ws = torch.empty(_lib.tvreg_autotune_workspace_bytes(self.handle), dtype=torch.uint8,
                         device=device)
        t = _Tuning()
        _check(_lib.tvreg_autotune(self.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   int(reps), ctypes.byref(t), _stream(ws)), "tvreg_autotune")
        return {"project_tile_cols": t.project_tile_cols, "project_waves": t.project_waves,
                "backproject_depth": t.backproject_depth,
                "project_ms": {(c, w): t.project_ms[a][i]
                               for a, c in enumerate(PROJECT_TILE_COLS)
                               for i, w in enumerate(PROJECT_WAVES)},
                "backproject_ms": dict(zip(BACKPROJECT_DEPTHS, list(t.backproject_ms)))}

    @property
    def tuning(self) -> tuple:
        """(project_tile_cols, project_waves, backproject_depth) currently used."""
        t = _Tuning()
        _check(_lib.tvreg_get_tuning(self.handle, ctypes.byref(t)), "tvreg_get_tuning")
        return (t.project_tile_cols, t.project_waves, t.backproject_depth)

    def set_tuning(self, project_tile_cols: int, project_waves: int,
                   backproject_depth: int) -> None:
        t = _Tuning(int(project_tile_cols), int(project_waves), int(backproject_depth), 0)
        _check(_lib.tvreg_set_tuning(self.handle, ctypes.byref(t)), "tvreg_set_tuning")

    def empty_volume(self, device="cuda"):
        return torch.empty(self.vol_shape, dtype=self.dtype, device=device)

    def empty_data(self, device="cuda"):
        return torch.empty(self.proj_shape, dtype=self.dtype, device=device)


def project(geom: Geometry, x: torch.Tensor, out: Optional[torch.Tensor] = None,
            workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = A x (tvreg_project); with a workspace (project_workspace) the
    solvers' form through the companion copy (tvreg_project_ws)."""
    y = geom.empty_data(x.device) if out is None else out
    if workspace is None:
        _check(_lib.tvreg_project(geom.handle, _ptr(x, geom.dtype, geom.N, "x"),
                                  _ptr(y, geom.dtype, geom.m, "y"), _stream(x)), "tvreg_project")
    else:
        _check(_lib.tvreg_project_ws(geom.handle, _ptr(x, geom.dtype, geom.N, "x"),
                                     _ptr(y, geom.dtype, geom.m, "y"), workspace.data_ptr(),
                                     workspace.numel() * workspace.element_size(), _stream(x)),
               "tvreg_project_ws")
    return y


def project_workspace(geom: Geometry, device="cuda") -> torch.Tensor:
    return torch.empty(_lib.tvreg_project_workspace_bytes(geom.handle), dtype=torch.uint8,
                       device=device)


def backproject(geom: Geometry, r: torch.Tensor, out: Optional[torch.Tensor] = None):
    """x = A^T r (tvreg_backproject)."""
    x = geom.empty_volume(r.device) if out is None else out
    _check(_lib.tvreg_backproject(geom.handle, _ptr(r, geom.dtype, geom.m, "r"),
                                  _ptr(x, geom.dtype, geom.N, "x"), _stream(r)),
           "tvreg_backproject")
    return x


def tv_grad(x: torch.Tensor, tau: float, value: bool = True, grad: bool = True):
    """(grad T_tau(x), T_tau(x)) (tvreg_tv_grad); the value is a 0-d float64 tensor."""
    nz, ny, nx = x.shape
    prec = F64 if x.dtype == torch.float64 else F32
    n = nx * ny * nz
    g = torch.empty_like(x) if grad else None
    val = torch.empty((), dtype=torch.float64, device=x.device) if value else None
    wsb = _lib.tvreg_tv_workspace_bytes(nx, ny, nz) if value else 0
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=x.device) if value else None
    _check(_lib.tvreg_tv_grad(nx, ny, nz, prec, float(tau), _ptr(x, x.dtype, n, "x"),
                              _ptr(g, x.dtype, n, "grad") if grad else None,
                              ctypes.c_void_p(val.data_ptr()) if value else None,
                              ctypes.c_void_p(ws.data_ptr()) if value else None, wsb,
                              _stream(x)), "tvreg_tv_grad")
    return g, val


def tv_grad_noalloc(x: torch.Tensor, tau: float, value: bool = True, grad: bool = True,
                    out: torch.Tensor = None, value_out: torch.Tensor = None):
    """tv_grad through tvreg_tv_grad_noalloc: the library takes no workspace
    (its partial sums live in a static device array).  With `out` and
    `value_out` given (a tensor like x and a 0-d float64 tensor) nothing is
    allocated on this side either."""
    nz, ny, nx = x.shape
    prec = F64 if x.dtype == torch.float64 else F32
    n = nx * ny * nz
    g = (out if out is not None else torch.empty_like(x)) if grad else None
    val = None
    if value:
        val = value_out if value_out is not None else torch.empty(
            (), dtype=torch.float64, device=x.device)
        if val.dtype != torch.float64 or val.numel() != 1 or val.device != x.device:
            raise ValueError("value_out must be one float64 element on x's device")
    _check(_lib.tvreg_tv_grad_noalloc(nx, ny, nz, prec, float(tau), _ptr(x, x.dtype, n, "x"),
                                      _ptr(g, x.dtype, n, "grad") if grad else None,
                                      ctypes.c_void_p(val.data_ptr()) if value else None,
                                      _stream(x)), "tvreg_tv_grad_noalloc")
    return g, val


def tv_hessvec(y: torch.Tensor, v: torch.Tensor, tau: float, dot: bool = True):
    """(H_T(y) v, <v, grad T(y)>) (tvreg_tv_hessvec); the dot is a 0-d float64 tensor."""
    nz, ny, nx = y.shape
    prec = F64 if y.dtype == torch.float64 else F32
    n = nx * ny * nz
    out = torch.empty_like(y)
    val = torch.empty((), dtype=torch.float64, device=y.device) if dot else None
    wsb = _lib.tvreg_tv_workspace_bytes(nx, ny, nz) if dot else 0
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=y.device) if dot else None
    _check(_lib.tvreg_tv_hessvec(nx, ny, nz, prec, float(tau), _ptr(y, y.dtype, n, "y"),
                                 _ptr(v, y.dtype, n, "v"), _ptr(out, y.dtype, n, "out"),
                                 ctypes.c_void_p(val.data_ptr()) if dot else None,
                                 ctypes.c_void_p(ws.data_ptr()) if dot else None, wsb,
                                 _stream(y)), "tvreg_tv_hessvec")
    return out, val


def objective_grad(geom: Geometry, b: torch.Tensor, alpha: float, tau: float, x: torch.Tensor,
                   grad: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None):
    """(phi(x), grad phi(x)) (tvreg_objective_grad); phi is a 0-d float64 tensor."""
    g = geom.empty_volume(x.device) if grad is None else grad
    phi = torch.empty((), dtype=torch.float64, device=x.device)
    wsb = _lib.tvreg_objective_workspace_bytes(geom.handle)
    ws = workspace if workspace is not None else torch.empty(wsb, dtype=torch.uint8,
                                                             device=x.device)
    _check(_lib.tvreg_objective_grad(geom.handle, _ptr(b, geom.dtype, geom.m, "b"),
                                     float(alpha), float(tau), _ptr(x, geom.dtype, geom.N, "x"),
                                     _ptr(g, geom.dtype, geom.N, "grad"),
                                     ctypes.c_void_p(phi.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(x)),
           "tvreg_objective_grad")
    return phi, g


def objective_workspace(geom: Geometry, device="cuda") -> torch.Tensor:
    return torch.empty(_lib.tvreg_objective_workspace_bytes(geom.handle), dtype=torch.uint8,
                       device=device)


def solve_workspace(geom: Geometry, method: int = UPN, device="cuda") -> torch.Tensor:
    return torch.empty(_lib.tvreg_solve_workspace_bytes(geom.handle, int(method)),
                       dtype=torch.uint8, device=device)


def solve(geom: Geometry, b: torch.Tensor, method: int = UPN, alpha: float = 1e-2,
          tau: float = 1e-4, eps: float = 1e-6, x0: Optional[torch.Tensor] = None,
          stop_mode: int = 0, max_iter: int = 10000, L_bar: float = 1.0, mu_bar: float = 0.0,
          rho_L: float = 2.0, gpbb_K: int = 2, gpbb_sigma: float = 0.1,
          gpbb_beta0: float = 0.95, max_trials: int = 60, hist_len: int = 0,
          workspace: Optional[torch.Tensor] = None, lower: float = 0.0,
          upper: float = float("inf")):
    """Runs GP / GPBB / UPN / Nesterov (tvreg_solve) over Q = [lower, upper]^N
    (default: the nonnegative orthant).  Returns (x, info dict, history dict)."""
    x = (torch.zeros(geom.vol_shape, dtype=geom.dtype, device=b.device) if x0 is None
         else x0.detach().clone().contiguous())
    ws = workspace if workspace is not None else solve_workspace(geom, method, b.device)
    hl = max(int(hist_len), 0)
    hists = [(ctypes.c_double * max(hl, 1))() for _ in range(3)]
    p = _SolveParams(int(method), float(alpha), float(tau), float(eps), int(stop_mode),
                     int(max_iter), float(L_bar), float(mu_bar), float(rho_L), int(gpbb_K),
                     float(gpbb_sigma), float(gpbb_beta0), int(max_trials),
                     ctypes.cast(hists[0], _c_dp) if hl else None,
                     ctypes.cast(hists[1], _c_dp) if hl else None,
                     ctypes.cast(hists[2], _c_dp) if hl else None, hl,
                     *_box_fields(lower, upper))
    info = _SolveInfo()
    _check(_lib.tvreg_solve(geom.handle, _ptr(b, geom.dtype, geom.m, "b"), ctypes.byref(p),
                            _ptr(x, geom.dtype, geom.N, "x"), ctypes.c_void_p(ws.data_ptr()),
                            ws.numel(), ctypes.byref(info), _stream(b)), "tvreg_solve")
    out = {k: getattr(info, k) for k, _ in _SolveInfo._fields_}
    n = min(hl, out["iters"])
    hist = {"phi": list(hists[0])[:n], "gm": list(hists[1])[:n], "L": list(hists[2])[:n]}
    return x, out, hist


def _box_fields(lower: float, upper: float):
    """(use_box, lower, upper) of tvreg_solve_params: the orthant unless a
    box other than [0, inf) is asked for."""
    lo, hi = float(lower), float(upper)
    return (0, 0.0, 0.0) if (lo == 0.0 and hi == float("inf")) else (1, lo, hi)


def _handles(geoms):
    return (ctypes.c_void_p * len(geoms))(*[g.handle.value for g in geoms])


def solve_batched_workspace(geoms, device="cuda") -> torch.Tensor:
    nb = _lib.tvreg_solve_batched_workspace_bytes(len(geoms), _handles(geoms))
    if nb == 0:
        raise ValueError("geometries must be non-empty and share one precision")
    return torch.empty(nb, dtype=torch.uint8, device=device)


_BATCH_DEFAULTS = dict(method=UPN, alpha=1e-2, tau=1e-4, eps=1e-6, stop_mode=0, max_iter=10000,
                       L_bar=1.0, mu_bar=0.0, rho_L=2.0, max_trials=60, lower=0.0,
                       upper=float("inf"))


def solve_batched(geoms, bs, params, x0s=None, poll_rounds: int = 8,
                  workspace: Optional[torch.Tensor] = None):
    """Solves len(geoms) GP / UPN problems together (tvreg_solve_batched).

    params: one dict per problem with any of the keys method, alpha, tau,
    eps, stop_mode, max_iter, L_bar, mu_bar, rho_L, max_trials, lower, upper
    (defaults as in solve()).  GP, UPN or Nesterov.  Returns (list of x, list of info dicts, batch status)."""
    n = len(geoms)
    if not (len(bs) == n and len(params) == n):
        raise ValueError("geoms, bs and params must have one entry per problem")
    ps = []
    for q in params:
        unknown = set(q) - set(_BATCH_DEFAULTS)
        if unknown:
            raise ValueError(f"unknown batched solve parameters {sorted(unknown)}")
        ps.append({**_BATCH_DEFAULTS, **q})
    xs = []
    for i, g in enumerate(geoms):
        if x0s is None:
            xs.append(torch.zeros(g.vol_shape, dtype=g.dtype, device=bs[i].device))
        else:
            xs.append(x0s[i].detach().clone().contiguous())
    ws = workspace if workspace is not None else solve_batched_workspace(geoms, bs[0].device)
    cp = (_SolveParams * n)()
    for i, q in enumerate(ps):
        cp[i] = _SolveParams(int(q["method"]), float(q["alpha"]), float(q["tau"]),
                             float(q["eps"]), int(q["stop_mode"]), int(q["max_iter"]),
                             float(q["L_bar"]), float(q["mu_bar"]), float(q["rho_L"]), 2, 0.1,
                             0.95, int(q["max_trials"]), None, None, None, 0,
                             *_box_fields(q["lower"], q["upper"]))
    bp = (ctypes.c_void_p * n)(*[_ptr(bs[i], g.dtype, g.m, f"b[{i}]").value
                                  for i, g in enumerate(geoms)])
    xp = (ctypes.c_void_p * n)(*[_ptr(xs[i], g.dtype, g.N, f"x[{i}]").value
                                  for i, g in enumerate(geoms)])
    infos = (_SolveInfo * n)()
    status = _check(_lib.tvreg_solve_batched(n, _handles(geoms), bp, cp, xp,
                                             ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                             int(poll_rounds), infos, _stream(bs[0])),
                    "tvreg_solve_batched")
    out = [{k: getattr(infos[i], k) for k, _ in _SolveInfo._fields_} for i in range(n)]
    return xs, out, status


def profile_enable(on: bool = True) -> None:
    """Per-kernel HIP-event timing of tvreg_solve's launches (tvreg_profile_enable)."""
    _lib.tvreg_profile_enable(1 if on else 0)


def profile_reset() -> None:
    _lib.tvreg_profile_reset()


def profile_stats() -> dict:
    """{kernel name: (launches, total ms)} accumulated since the last reset."""
    out = {}
    for name, kid in KERNELS.items():
        c = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(_lib.tvreg_profile_get(kid, ctypes.byref(c), ctypes.byref(ms)), "profile_get")
        out[name] = (int(c.value), float(ms.value))
    return out


def version() -> str:
    return _lib.tvreg_version().decode()


def unrolled_workspace(geom: Geometry, K: int, ckpt_every: int = 5, device="cuda"):
    nb = _lib.tvreg_unrolled_workspace_bytes(geom.handle, int(K), int(ckpt_every))
    if nb == 0:
        raise ValueError("need K >= 1 and ckpt_every >= 1")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def upn_unrolled_fwd(geom: Geometry, b: torch.Tensor, K: int, alpha: float, tau: float = 1e-4,
                     ckpt_every: int = 5, L_replay=None, L_bar: float = 1.0,
                     mu_bar: float = 0.0, rho_L: float = 2.0, max_trials: int = 60,
                     tape: Optional[torch.Tensor] = None):
    """K unrolled UPN steps from x = 0 (tvreg_upn_unrolled_fwd).

    Returns (x^(K), tape, list of the K values of L used).  L_replay (K
    values) replaces the BT searches.  Raises TvregError also for
    TVREG_ESTALL (a BT search hit max_trials)."""
    tape = tape if tape is not None else unrolled_workspace(geom, K, ckpt_every, b.device)
    p = _SolveParams(UPN, float(alpha), float(tau), 0.0, 0, 1, float(L_bar), float(mu_bar),
                     float(rho_L), 2, 0.1, 0.95, int(max_trials), None, None, None, 0)
    Lout = (ctypes.c_double * K)()
    Lin = None
    if L_replay is not None:
        if len(L_replay) != K:
            raise ValueError("L_replay needs K values")
        Lin = (ctypes.c_double * K)(*[float(v) for v in L_replay])
    xK = geom.empty_volume(b.device)
    st = _lib.tvreg_upn_unrolled_fwd(geom.handle, _ptr(b, geom.dtype, geom.m, "b"),
                                     ctypes.byref(p), int(K), int(ckpt_every),
                                     ctypes.cast(Lin, _c_dp) if Lin is not None else None,
                                     ctypes.cast(Lout, _c_dp),
                                     _ptr(xK, geom.dtype, geom.N, "xK"),
                                     ctypes.c_void_p(tape.data_ptr()), tape.numel(), _stream(b))
    if st != OK:  # a stalled line search leaves no x^(K) either
        raise TvregError(st, "tvreg_upn_unrolled_fwd")
    return xK, tape, list(Lout)


def upn_unrolled_bwd(geom: Geometry, b: torch.Tensor, tape: torch.Tensor, xK_bar: torch.Tensor):
    """Reverse pass (tvreg_upn_unrolled_bwd): (dl/dlog alpha as float, dl/db)."""
    db = geom.empty_data(b.device)
    da = ctypes.c_double(0.0)
    _check(_lib.tvreg_upn_unrolled_bwd(geom.handle, _ptr(b, geom.dtype, geom.m, "b"),
                                       ctypes.c_void_p(tape.data_ptr()), tape.numel(),
                                       _ptr(xK_bar.contiguous(), geom.dtype, geom.N, "xK_bar"),
                                       ctypes.byref(da), _ptr(db, geom.dtype, geom.m, "dl_db"),
                                       _stream(b)), "tvreg_upn_unrolled_bwd")
    return float(da.value), db


from .unrolled import UnrolledUPN, unrolled_upn  # noqa: E402  (uses the functions above)
