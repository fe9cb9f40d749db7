"""FP64 CPU oracle for TV-regularised CT reconstruction -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C,
double precision, built with ``-O2 -fopenmp -ffp-contract=off``) through
ctypes and shares no code with the HIP library.

What each entry point follows, and what pins it (tests under ``tests/``):

================  =====================================  =========================================
entry point       paper passage                           pinned by
================  =====================================  =========================================
project           A, the system matrix (Sec. II-A)        brute-force slab lengths on 8^3 volumes;
                  (Siddon exact path length, reading)     chord-length closed form; axis-aligned
                                                          ray closed form; single-voxel projection
                  3D parallel beam over the unit sphere   in-plane directions = parallel beam;
                  (Sec. IV-A)                             axis directions = oriented column sums;
                                                          ones -> independent chord lengths
backproject       A^T (gradient of eq. 1)                 adjoint identity <Ax,y> = <x,A^T y>
                                                          against the dense brute-force matrix
tv                eq. 2, Huber-smoothed                   closed-form TV of boxes; central finite
                                                          differences; sum of gradient = 0;
                                                          quadratic regime = Neumann Laplacian / tau
gradmap_norm      eq. 10                                  closed form min(g, nu x) for x >= 0
solve (GP)        eq. 6 + Alg. 2 (BT)                     alpha = 0 vs scipy.optimize.nnls;
solve (GPBB)      Alg. 1                                  all three methods reach the same minimiser;
solve (UPN)       Alg. 3 + eq. 9                          invariants (L monotone, mu in [0, mu_bar]);
                                                          mu := L reduces UPN to GP bit for bit
solve (NESTEROV)  Nesterov's method, given mu and L       numpy textbook constant-momentum
                  (Sec. III-B, rate of eq. 8)             projected scheme on a dense problem
solve, box Q      P_Q = clip to [lower, upper] (Sec. III) scipy.optimize.lsq_linear (bounded LS);
                                                          unbounded box = numpy lstsq
tv_hessvec        derivative of the TV gradient (eq. 2)   central differences of tv's gradient;
                                                          symmetry; quadratic regime = Laplacian
unrolled          K steps of Alg. 3 and the reverse-mode   K = 1 closed form; central differences
                  gradient of l(x^(K)) in alpha and b      of the replayed forward map (same
                  (not a passage of the paper)            masks and regimes on both sides)
================  =====================================  =========================================
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "tvreg_oracle.c")

GP, GPBB, UPN, NESTEROV = 0, 1, 2, 3
CONVERGED, NOTCONV, STALL = 0, 1, 2


# TVREG_ORACLE_SANITIZE=1 selects a separate build with AddressSanitizer and
# UndefinedBehaviorSanitizer (CPU only; the process must preload libasan, see
# the README); any report aborts the process.
_SANITIZE = os.environ.get("TVREG_ORACLE_SANITIZE", "") == "1"
if _SANITIZE:
    _LIB_PATH = os.path.join(_HERE, "liboracle_san.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        flags = ["-O2"]
        if _SANITIZE:
            flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                     "-fno-sanitize-recover=all"]
        cmd = ["gcc", *flags, "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n_views", ctypes.c_int32), ("angles", ctypes.POINTER(ctypes.c_double)),
                ("cone", ctypes.c_int32), ("cols", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("pitch_u", ctypes.c_double), ("pitch_v", ctypes.c_double),
                ("src_to_centre", ctypes.c_double), ("src_to_det", ctypes.c_double),
                ("dirs", ctypes.POINTER(ctypes.c_double))]


class _Params(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("tau", ctypes.c_double), ("eps", ctypes.c_double),
                ("stop_mode", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("L_bar", ctypes.c_double), ("mu_bar", ctypes.c_double),
                ("rho_L", ctypes.c_double), ("gpbb_K", ctypes.c_int32),
                ("gpbb_sigma", ctypes.c_double), ("gpbb_beta0", ctypes.c_double),
                ("max_trials", ctypes.c_int32), ("max_squarings", ctypes.c_int32),
                ("force_mu", ctypes.c_int32), ("bt_form", ctypes.c_int32),
                ("lower", ctypes.c_double), ("upper", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("grad_evals", ctypes.c_int32),
                ("func_evals", ctypes.c_int32), ("status", ctypes.c_int32),
                ("phi", ctypes.c_double), ("gm", ctypes.c_double), ("gm0", ctypes.c_double),
                ("L", ctypes.c_double), ("mu", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(_Geom)
        L.og_project.argtypes = [gp, dp, dp]
        L.og_backproject.argtypes = [gp, dp, dp]
        L.og_project_bruteforce.argtypes = [gp, dp, dp]
        L.og_matrix_dense.argtypes = [gp, dp]
        L.og_ray_sum.argtypes = [gp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp]
        L.og_ray_sum.restype = ctypes.c_double
        L.og_nnz.argtypes = [gp]
        L.og_nnz.restype = ctypes.c_int64
        L.og_tv.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, dp, dp]
        L.og_tv.restype = ctypes.c_double
        L.og_phi.argtypes = [gp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.og_phi.restype = ctypes.c_double
        L.og_phi_grad.argtypes = [gp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.og_phi_grad.restype = ctypes.c_double
        L.og_gradmap_norm.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double]
        L.og_gradmap_norm.restype = ctypes.c_double
        L.og_gradmap_norm_box.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double]
        L.og_gradmap_norm_box.restype = ctypes.c_double
        L.og_slab_length.argtypes = [dp, dp, dp, dp]
        L.og_slab_length.restype = ctypes.c_double
        L.og_ray_endpoints.argtypes = [gp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp, dp]
        L.og_solve.argtypes = [gp, dp, ctypes.POINTER(_Params), dp, ctypes.POINTER(_Info),
                               dp, dp, dp, dp, dp, ctypes.c_int32]
        L.og_solve.restype = ctypes.c_int32
        L.og_solve_dense.argtypes = [ctypes.c_int32] * 4 + [dp, dp, ctypes.POINTER(_Params), dp,
                                                            ctypes.POINTER(_Info), dp, dp, dp,
                                                            dp, dp, ctypes.c_int32]
        L.og_solve_dense.restype = ctypes.c_int32
        L.og_num_threads.restype = ctypes.c_int32
        L.og_huber_bregman.argtypes = [dp, dp, dp, ctypes.c_double]
        L.og_huber_bregman.restype = ctypes.c_double
        L.og_tv_bregman.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, dp, dp]
        L.og_tv_bregman.restype = ctypes.c_double
        L.og_tv_hessvec.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, dp, dp, dp]
        L.og_tv_hessvec.restype = None
        L.og_unrolled.argtypes = [gp, dp, ctypes.POINTER(_Params), ctypes.c_int32,
                                  ctypes.c_int32, dp, dp, dp, dp, dp, dp, dp,
                                  ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_uint64)]
        L.og_unrolled.restype = ctypes.c_int32
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Geometry:
    """Oracle-side geometry (keeps the angle array alive)."""

    def __init__(self, g):
        self.desc = g
        self._angles = np.ascontiguousarray(np.asarray(g.angles, dtype=np.float64))
        dirs = getattr(g, "dirs", None)
        if int(g.beam) == 2:
            self._dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
            if len(self._dirs) != len(self._angles):
                raise ValueError("one direction per view is needed")
            dp = _dp(self._dirs)
        else:
            self._dirs = None
            dp = ctypes.POINTER(ctypes.c_double)()
        self.s = _Geom(g.nx, g.ny, g.nz, len(self._angles), _dp(self._angles), int(g.beam),
                       g.det_cols, g.det_rows, float(g.pitch_u), float(g.pitch_v),
                       float(g.src_to_centre), float(g.src_to_det), dp)
        self.vol_shape = (g.nz, g.ny, g.nx)
        self.proj_shape = (len(self._angles), g.det_rows, g.det_cols)

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _geom(g) -> Geometry:
    return g if isinstance(g, Geometry) else Geometry(g)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def project(g, x) -> np.ndarray:
    G = _geom(g)
    x = _f64(x).reshape(G.vol_shape)
    y = np.zeros(G.proj_shape, np.float64)
    lib().og_project(G.ref, _dp(x), _dp(y))
    return y


def backproject(g, r) -> np.ndarray:
    G = _geom(g)
    r = _f64(r).reshape(G.proj_shape)
    x = np.zeros(G.vol_shape, np.float64)
    lib().og_backproject(G.ref, _dp(r), _dp(x))
    return x


def project_bruteforce(g, x) -> np.ndarray:
    G = _geom(g)
    x = _f64(x).reshape(G.vol_shape)
    y = np.zeros(G.proj_shape, np.float64)
    lib().og_project_bruteforce(G.ref, _dp(x), _dp(y))
    return y


def matrix_dense(g) -> np.ndarray:
    G = _geom(g)
    m = int(np.prod(G.proj_shape))
    N = int(np.prod(G.vol_shape))
    A = np.zeros((m, N), np.float64)
    lib().og_matrix_dense(G.ref, _dp(A))
    return A


def ray_sum(g, v: int, row: int, col: int, x) -> float:
    G = _geom(g)
    x = _f64(x).reshape(G.vol_shape)
    return float(lib().og_ray_sum(G.ref, v, row, col, _dp(x)))


def ray_endpoints(g, v: int, row: int, col: int):
    G = _geom(g)
    p0 = np.zeros(3)
    p1 = np.zeros(3)
    lib().og_ray_endpoints(G.ref, v, row, col, _dp(p0), _dp(p1))
    return p0, p1


def slab_length(p0, p1, lo, hi) -> float:
    return float(lib().og_slab_length(_dp(_f64(p0)), _dp(_f64(p1)), _dp(_f64(lo)),
                                      _dp(_f64(hi))))


def nnz(g) -> int:
    return int(lib().og_nnz(_geom(g).ref))


def tv(x, tau: float, grad: bool = True):
    x = _f64(x)
    nz, ny, nx = x.shape
    gr = np.zeros_like(x) if grad else None
    T = lib().og_tv(nx, ny, nz, tau, _dp(x), _dp(gr) if grad else None)
    return (float(T), gr) if grad else float(T)


def huber_bregman(a, b, d, tau: float) -> float:
    return float(lib().og_huber_bregman(_dp(_f64(a)), _dp(_f64(b)), _dp(_f64(d)), tau))


def tv_bregman(x, y, tau: float) -> float:
    x = _f64(x)
    nz, ny, nx = x.shape
    return float(lib().og_tv_bregman(nx, ny, nz, tau, _dp(x), _dp(_f64(y).reshape(x.shape))))


def phi(g, b, alpha: float, tau: float, x) -> float:
    G = _geom(g)
    return float(lib().og_phi(G.ref, _dp(_f64(b).reshape(G.proj_shape)), alpha, tau,
                              _dp(_f64(x).reshape(G.vol_shape))))


def phi_grad(g, b, alpha: float, tau: float, x):
    G = _geom(g)
    gr = np.zeros(G.vol_shape, np.float64)
    f = lib().og_phi_grad(G.ref, _dp(_f64(b).reshape(G.proj_shape)), alpha, tau,
                          _dp(_f64(x).reshape(G.vol_shape)), _dp(gr))
    return float(f), gr


def gradmap_norm(x, grad, nu: float, lower: float = 0.0, upper: float = float("inf")) -> float:
    x = _f64(x)
    grad = _f64(grad)
    if lower == 0.0 and upper == float("inf"):
        return float(lib().og_gradmap_norm(x.size, _dp(x), _dp(grad), nu))
    return float(lib().og_gradmap_norm_box(x.size, _dp(x), _dp(grad), nu, lower, upper))


def default_params(method: int, alpha: float, tau: float = 1e-4, eps: float = 1e-6,
                   max_iter: int = 10000, **kw) -> dict:
    p = dict(method=method, alpha=alpha, tau=tau, eps=eps, stop_mode=0, max_iter=max_iter,
             L_bar=1.0, mu_bar=0.0, rho_L=2.0, gpbb_K=2, gpbb_sigma=0.1, gpbb_beta0=0.95,
             max_trials=60, max_squarings=30, force_mu=0, bt_form=0, lower=0.0,
             upper=float("inf"))
    p.update(kw)
    return p


def solve(g, b, x0=None, hist_len: int = 0, **params):
    """Run GP / GPBB / UPN.  Returns (x, info dict, history dict).

    History entry k (first hist_len iterations): phi of the accepted point,
    the relative gradient map, L_k (1/theta_k for GPBB), mu_k, and for UPN
    theta_{k+1}, the root Alg. 3 computes at iteration k from theta_k and
    mu_k / L_k (theta_1 = sqrt(mu_0 / L_0) at k = 0).
    """
    G = _geom(g)
    p = default_params(**params)
    P = _Params(**p)
    info = _Info()
    x = np.zeros(G.vol_shape) if x0 is None else _f64(x0).reshape(G.vol_shape).copy()
    hl = max(int(hist_len), 1)
    hp, hg, hL, hm, ht = (np.full(hl, np.nan) for _ in range(5))
    lib().og_solve(G.ref, _dp(_f64(b).reshape(G.proj_shape)), ctypes.byref(P), _dp(x),
                   ctypes.byref(info), _dp(hp), _dp(hg), _dp(hL), _dp(hm), _dp(ht), hl)
    return x, _info_dict(info), dict(phi=hp, gm=hg, L=hL, mu=hm, theta=ht)


def solve_dense(A, b, vol_shape, x0=None, hist_len: int = 0, **params):
    A = _f64(A)
    m = A.shape[0]
    nz, ny, nx = vol_shape
    p = default_params(**params)
    P = _Params(**p)
    info = _Info()
    x = np.zeros(vol_shape) if x0 is None else _f64(x0).reshape(vol_shape).copy()
    hl = max(int(hist_len), 1)
    hp, hg, hL, hm, ht = (np.full(hl, np.nan) for _ in range(5))
    lib().og_solve_dense(m, nx, ny, nz, _dp(A), _dp(_f64(b)), ctypes.byref(P), _dp(x),
                         ctypes.byref(info), _dp(hp), _dp(hg), _dp(hL), _dp(hm), _dp(ht), hl)
    return x, _info_dict(info), dict(phi=hp, gm=hg, L=hL, mu=hm, theta=ht)


def _info_dict(info: _Info) -> dict:
    return {k: getattr(info, k) for k, _ in _Info._fields_}


def noisy_data(g, x_true, unit_noise, eta: float) -> np.ndarray:
    """b = A x_true + e, e = sigma * unit_noise, sigma = eta |A x_true| / sqrt(m)
    (noise model of Sec. IV-A, eq. 11, per-ray Gaussian reading); rounded to
    float32 values so that every consumer sees identical data."""
    ax = project(g, x_true)
    sigma = eta * float(np.linalg.norm(ax)) / np.sqrt(ax.size)
    b = ax + sigma * np.asarray(unit_noise, np.float64).reshape(ax.shape)
    return b.astype(np.float32).astype(np.float64)


def tv_hessvec(y, v, tau: float) -> np.ndarray:
    """H(y) v, the Hessian of the smoothed TV at y applied to v."""
    y = _f64(y)
    nz, ny, nx = y.shape
    out = np.zeros_like(y)
    lib().og_tv_hessvec(nx, ny, nz, tau, _dp(y), _dp(_f64(v).reshape(y.shape)), _dp(out))
    return out


def unrolled(g, b, K: int, alpha: float, tau: float = 1e-4, L=None, xK_bar=None,
             L_bar: float = 1.0, rho_L: float = 2.0, mu_bar: float = 0.0,
             max_trials: int = 60, bt_form: int = 1) -> dict:
    """K unrolled UPN steps from x = 0 (og_unrolled).

    L=None runs BT for every step; an array of K values replays them.  With
    xK_bar = dl/dx^(K) the reverse pass returns dl/dalpha and dl/db.
    Returns a dict with xK, L, mu, beta, mu_state, signature, status and,
    with xK_bar, alpha_bar and b_bar."""
    G = _geom(g)
    p = _Params(**default_params(UPN, alpha, tau, L_bar=L_bar, rho_L=rho_L, mu_bar=mu_bar,
                                 max_trials=max_trials, bt_form=bt_form))
    replay = L is not None
    Ls = _f64(L).copy() if replay else np.zeros(K)
    assert Ls.shape == (K,)
    xK = np.zeros(G.vol_shape)
    mu = np.zeros(K)
    beta = np.zeros(K)
    state = np.zeros(K, np.int32)
    sig = ctypes.c_uint64(0)
    abar = np.zeros(1)
    bbar = np.zeros(G.proj_shape)
    xb = _f64(xK_bar).reshape(G.vol_shape) if xK_bar is not None else None
    st = lib().og_unrolled(G.ref, _dp(_f64(b).reshape(G.proj_shape)), ctypes.byref(p), K,
                           1 if replay else 0, _dp(Ls), _dp(xK),
                           _dp(xb) if xb is not None else None,
                           _dp(abar) if xb is not None else None,
                           _dp(bbar) if xb is not None else None, _dp(mu), _dp(beta),
                           state.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           ctypes.byref(sig))
    out = dict(status=int(st), xK=xK, L=Ls, mu=mu, beta=beta, mu_state=state,
               signature=int(sig.value))
    if xb is not None:
        out["alpha_bar"] = float(abar[0])
        out["b_bar"] = bbar
    return out


def num_threads() -> int:
    return int(lib().og_num_threads())
