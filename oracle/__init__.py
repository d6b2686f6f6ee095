"""FP64 CPU oracle for the anisotropic-equilibrium BGK lattice Boltzmann update.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package. It never imports the HIP library package and
the library never imports it; the two share no code.

This module is ctypes glue around ``lbm_oracle.c`` (the arithmetic lives there and cites the
paper's sections and equations) plus numpy conveniences. Lattices are named
``"D2Q9" | "D3Q19" | "D3Q27"``; tensor kinds ``"theta" | "A" | "Atilde"``:

* ``theta``  -- the tensor is cs^2 A^-1, the equilibrium's second central moment per unit
  density (App. E: M2 = rho (cs^2 A^-1 + s s)); the workload configurations use this form.
* ``A``      -- the tensor is A of eq:equil, used as given.
* ``Atilde`` -- the tensor is proportional to A and is normalised as A = A~ / det(A~)^(1/d)
  (Sec. 4 gives the d = 2 case, A = A~ / sqrt(det A~)).

Arrays: ``rho`` is [N], ``s`` is [d][N], populations are [q][N] with N = nz*ny*nx (x fastest)
in the oracle's own velocity order, available from :func:`lattice`.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_ORACLE_LIB lets the mutation test load a deliberately broken copy of this library.
_LIB_PATH = os.environ.get("LBM_ORACLE_LIB") or os.path.join(_HERE, "liblbm_oracle.so")

LATTICES = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2}
TENSOR_KINDS = {"theta": 0, "A": 1, "Atilde": 2}
_DIM = {"D2Q9": 2, "D3Q19": 3, "D3Q27": 3}

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build  # noqa: WPS433 (build step of this package)
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_gh1d.argtypes = [_dp, _dp]
    lib.orc_lattice.argtypes = [ctypes.c_int, _ip, _ip, _ip, _dp, _dp]
    lib.orc_tensor_to_ainv.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.orc_feq.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, _dp, _dp]
    _u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.orc_init.argtypes = [ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, _dp, _dp, _dp, _dp, ctypes.c_int]
    lib.orc_init_ext.argtypes = [ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, _dp, _dp, _dp, _u8p, _dp, ctypes.c_int]
    lib.orc_steps.argtypes = [ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, _dp, ctypes.c_double, _i64, _dp,
                              ctypes.c_int]
    lib.orc_steps_ext.argtypes = [ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, _dp, ctypes.c_double, _i64, _dp,
                                  _u8p, _dp, ctypes.c_int]
    lib.orc_steps_gray.argtypes = [ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, _dp, ctypes.c_double, _i64, _dp,
                                   _u8p, _dp, _dp, ctypes.c_int]
    lib.orc_objective.argtypes = [ctypes.c_int, _i64, _i64, _i64, _dp, _u8p, _dp, ctypes.c_int, _i64]
    lib.orc_objective.restype = ctypes.c_double
    lib.orc_moments.argtypes = [ctypes.c_int, _i64, _dp, _dp, _dp]
    lib.orc_moments_ext.argtypes = [ctypes.c_int, _i64, _dp, _u8p, _dp, _dp, _dp]
    lib.orc_num_threads.argtypes = []
    for name in ("orc_gh1d", "orc_lattice", "orc_tensor_to_ainv", "orc_feq", "orc_init", "orc_init_ext",
                 "orc_steps", "orc_steps_ext", "orc_steps_gray", "orc_moments", "orc_moments_ext",
                 "orc_num_threads"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _mask_ptr(mask, n):
    """uint8 [N] solid mask (1 = solid) or None, as a ctypes pointer plus the array kept alive."""
    if mask is None:
        return None, None
    m = np.ascontiguousarray(np.asarray(mask).reshape(n).astype(np.uint8))
    return m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), m


def _force_ptr(force, d):
    if force is None:
        return None, None
    fv = np.zeros(3)
    fv[:d] = np.asarray(force, dtype=np.float64)[:d]
    return _ptr(fv), fv


def dim(lattice: str) -> int:
    return _DIM[lattice]


def num_threads() -> int:
    """OpenMP threads the oracle uses by default on this host."""
    return int(_load().orc_num_threads())


def gauss_hermite_1d():
    """Nodes and weights of the 3-point probabilists' Gauss-Hermite rule (App. C)."""
    x = np.zeros(3)
    w = np.zeros(3)
    _load().orc_gh1d(_ptr(x), _ptr(w))
    return x, w


def lattice(name: str):
    """(c [q,3] int, w [q], cs2) in the oracle's velocity order."""
    q = ctypes.c_int()
    d = ctypes.c_int()
    c = (ctypes.c_int * 81)()
    w = np.zeros(27)
    cs2 = np.zeros(1)
    if _load().orc_lattice(LATTICES[name], ctypes.byref(q), ctypes.byref(d), c, _ptr(w), _ptr(cs2)):
        raise ValueError(name)
    cc = np.array(c[: 3 * q.value], dtype=np.int64).reshape(q.value, 3)
    return cc, w[: q.value].copy(), float(cs2[0])


def tensor_to_ainv(tensor, kind: str = "theta", d: int | None = None) -> np.ndarray:
    """A^-1 (d x d) from a tensor given in one of the three accepted forms."""
    t = np.ascontiguousarray(np.asarray(tensor, dtype=np.float64))
    if d is None:
        d = t.shape[0]
    t = np.ascontiguousarray(t[:d, :d])
    out = np.zeros((d, d))
    if _load().orc_tensor_to_ainv(d, TENSOR_KINDS[kind], _ptr(t), _ptr(out)):
        raise ValueError("tensor conversion failed")
    return out


def feq(name: str, ainv, rho: float, s, order: int = 3) -> np.ndarray:
    """Discrete equilibrium f^eq_i(rho, s) (eq:3rd_order_equilibrium, eq:feq_i)."""
    d = dim(name)
    a = np.ascontiguousarray(np.asarray(ainv, dtype=np.float64)[:d, :d])
    sv = np.ascontiguousarray(np.asarray(s, dtype=np.float64)[:d])
    out = np.zeros(27)
    if _load().orc_feq(LATTICES[name], int(order), _ptr(a), float(rho), _ptr(sv), _ptr(out)):
        raise ValueError(name)
    return out[: lattice(name)[0].shape[0]].copy()


def _shape3(shape):
    shape = tuple(int(v) for v in shape)
    if len(shape) == 2:
        shape = (shape[0], shape[1], 1)
    return shape


def init(name: str, shape, ainv, rho0, s0, order: int = 3, nthreads: int = 0, mask=None) -> np.ndarray:
    """f(0) = f^eq(rho0, s0) on a grid of shape (nx, ny[, nz]); zero on solid cells."""
    nx, ny, nz = _shape3(shape)
    d = dim(name)
    n = nx * ny * nz
    q = lattice(name)[0].shape[0]
    a = np.ascontiguousarray(np.asarray(ainv, dtype=np.float64)[:d, :d])
    r = np.ascontiguousarray(np.asarray(rho0, dtype=np.float64).reshape(n))
    s = np.ascontiguousarray(np.asarray(s0, dtype=np.float64).reshape(d, n))
    f = np.zeros((q, n))
    mp, _keep = _mask_ptr(mask, n)
    if _load().orc_init_ext(LATTICES[name], int(order), nx, ny, nz, _ptr(a), _ptr(r), _ptr(s), mp, _ptr(f),
                            int(nthreads)):
        raise ValueError(name)
    return f


def steps(name: str, shape, ainv, tau: float, f: np.ndarray, nsteps: int, order: int = 3,
          nthreads: int = 0, mask=None, force=None) -> np.ndarray:
    """Advance pre-collision populations f ([q][N]) by nsteps of eq:LBE_BGK (in place; returned),
    with optional solid mask (halfway bounce-back) and body force (exact-difference method)."""
    nx, ny, nz = _shape3(shape)
    d = dim(name)
    a = np.ascontiguousarray(np.asarray(ainv, dtype=np.float64)[:d, :d])
    if not (f.dtype == np.float64 and f.flags.c_contiguous):
        raise TypeError("f must be C-contiguous float64")
    mp, _keep_m = _mask_ptr(mask, nx * ny * nz)
    fp, _keep_f = _force_ptr(force, d)
    rc = _load().orc_steps_ext(LATTICES[name], int(order), nx, ny, nz, _ptr(a), float(tau), int(nsteps), _ptr(f),
                               mp, fp, int(nthreads))
    if rc:
        raise RuntimeError(f"orc_steps failed ({rc})")
    return f


def steps_gray(name: str, shape, ainv, tau: float, f: np.ndarray, nsteps: int, gray, order: int = 3,
               force=None, nthreads: int = 0, mask=None) -> np.ndarray:
    """Like :func:`steps` with a gray mask m ([N]): f* = (1 - m) f^BGK + m f_opp on fluid cells,
    optionally together with a solid mask (halfway bounce-back at the solid cells)."""
    nx, ny, nz = _shape3(shape)
    d = dim(name)
    a = np.ascontiguousarray(np.asarray(ainv, dtype=np.float64)[:d, :d])
    gm = np.ascontiguousarray(np.asarray(gray, dtype=np.float64).reshape(nx * ny * nz))
    fp, _keep_f = _force_ptr(force, d)
    mp, _keep_m = _mask_ptr(mask, nx * ny * nz)
    rc = _load().orc_steps_gray(LATTICES[name], int(order), nx, ny, nz, _ptr(a), float(tau), int(nsteps), _ptr(f),
                                mp, _ptr(gm), fp, int(nthreads))
    if rc:
        raise RuntimeError(f"orc_steps_gray failed ({rc})")
    return f


def objective(name: str, shape, f: np.ndarray, kind: int, plane: int = 0, mask=None, force=None) -> float:
    """Outlet mass flux (kind 0, plane x = plane) or kinetic energy (kind 1) of a state."""
    nx, ny, nz = _shape3(shape)
    d = dim(name)
    mp, _keep_m = _mask_ptr(mask, nx * ny * nz)
    fp, _keep_f = _force_ptr(force, d)
    return float(_load().orc_objective(LATTICES[name], nx, ny, nz, _ptr(np.ascontiguousarray(f)), mp, fp, int(kind),
                                       int(plane)))


def moments(name: str, f: np.ndarray, mask=None, force=None):
    """(rho [N], s [d][N]) from populations (eq:a0discrete_f, eq:a1discrete_f); with a force the
    velocity is (sum f c + F/2)/rho; solid cells give zeros."""
    d = dim(name)
    n = f.shape[1]
    rho = np.zeros(n)
    s = np.zeros((d, n))
    mp, _keep_m = _mask_ptr(mask, n)
    fp, _keep_f = _force_ptr(force, d)
    _load().orc_moments_ext(LATTICES[name], n, _ptr(np.ascontiguousarray(f)), mp, fp, _ptr(rho), _ptr(s))
    return rho, s


def run(name: str, shape, tensor, kind: str, tau: float, rho0, s0, nsteps: int, order: int = 3,
        nthreads: int = 0, mask=None, force=None):
    """Initialise at equilibrium and run nsteps; returns (f, rho, s) at t = nsteps."""
    d = dim(name)
    ainv = tensor_to_ainv(np.asarray(tensor, dtype=np.float64)[:d, :d], kind, d)
    f = init(name, shape, ainv, rho0, s0, order, nthreads, mask=mask)
    steps(name, shape, ainv, tau, f, nsteps, order, nthreads, mask=mask, force=force)
    rho, s = moments(name, f, mask=mask, force=force)
    return f, rho, s
