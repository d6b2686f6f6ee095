"""MI355X (gfx950) lattice Boltzmann update with the third-order anisotropic equilibrium of
"Lattice Boltzmann Methods with Anisotropic Equilibrium Distributions" (arXiv 2605.27004).

Thin ctypes binding of the C ABI in ``include/lbm.h`` (``lib/liblbm.so``, built by
``python paper_2605_27004_amd/build.py``). The functions keep the C names and only marshal
arguments: every step of the update runs in the HIP kernels. PyTorch is used for device
memory and streams only (:class:`Simulation`). Importing this package fails loudly when the
library has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "liblbm.so")

# ---- constants (mirror include/lbm.h) ---------------------------------------------------
LBM_OK = 0
LBM_ERR_ARG = -1
LBM_ERR_NOT_SPD = -2
LBM_ERR_TAU = -3
LBM_ERR_ALIGN = -4
LBM_ERR_HIP = -5
LBM_ERR_UNSUPPORTED = -6
LBM_ERR_NONFINITE = -7
LBM_ERR_SIZE = -8

LBM_D2Q9, LBM_D3Q19, LBM_D3Q27 = 0, 1, 2
LBM_F64, LBM_F32, LBM_F16, LBM_BF16 = 0, 1, 2, 3
LBM_TENSOR_THETA, LBM_TENSOR_A, LBM_TENSOR_ATILDE = 0, 1, 2
LBM_SHIFT_REST, LBM_SHIFT_WEIGHT = 0, 1
LBM_LAUNCH_XCD_SLABS = 1
LBM_LAUNCH_SHIFTED_PULL = 2
LBM_FLAG_MASK = 1
LBM_FLAG_GRAY = 2

LATTICES = {"D2Q9": LBM_D2Q9, "D3Q19": LBM_D3Q19, "D3Q27": LBM_D3Q27}
STORAGES = {"f64": LBM_F64, "f32": LBM_F32, "f16": LBM_F16, "bf16": LBM_BF16}
TENSOR_KINDS = {"theta": LBM_TENSOR_THETA, "A": LBM_TENSOR_A, "Atilde": LBM_TENSOR_ATILDE}
SHIFTS = {"rest": LBM_SHIFT_REST, "weight": LBM_SHIFT_WEIGHT}
STORAGE_BYTES = {LBM_F64: 8, LBM_F32: 4, LBM_F16: 2, LBM_BF16: 2}


class lbm_params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("storage", ctypes.c_int32), ("order", ctypes.c_int32),
                ("tensor_kind", ctypes.c_int32), ("shift_kind", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("tensor", ctypes.c_double * 9), ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("force", ctypes.c_double * 3)]


class lbm_derived(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("d", ctypes.c_int32), ("ainv", ctypes.c_double * 9),
                ("k", ctypes.c_double * 9), ("omega", ctypes.c_double), ("nu", ctypes.c_double),
                ("rest", ctypes.c_double * 27), ("shift", ctypes.c_double * 27), ("min_rest_ratio", ctypes.c_double)]


class lbm_grad_spec(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_int32), ("reserved", ctypes.c_int32), ("nsteps", ctypes.c_int64),
                ("checkpoint_every", ctypes.c_int64), ("outlet_plane", ctypes.c_int64)]


OBJECTIVES = {"flux": 0, "kinetic_energy": 1}


class lbm_domain(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("tensor_kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tensor", ctypes.c_double * 9), ("tau", ctypes.c_double)]


class lbm_batch_params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("storage", ctypes.c_int32), ("order", ctypes.c_int32),
                ("shift_kind", ctypes.c_int32), ("rho0", ctypes.c_double), ("ndomains", ctypes.c_int64),
                ("domains", ctypes.POINTER(lbm_domain))]


class lbm_batch_schedule(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("xcd_group", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("chunk_cells", ctypes.c_int64), ("group_bytes", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {"mode": "persistent" if self.mode == LBM_BATCH_PERSISTENT else "stepwise",
                "xcd_group": int(self.xcd_group), "wg_per_cu": int(self.wg_per_cu),
                "chunk_cells": int(self.chunk_cells), "group_bytes": int(self.group_bytes)}


LBM_BATCH_STEPWISE, LBM_BATCH_PERSISTENT = 0, 1


class lbm_batch_item(ctypes.Structure):
    _fields_ = [("domain", ctypes.c_int64), ("first_cell", ctypes.c_int64), ("cells", ctypes.c_int64),
                ("group", ctypes.c_int64), ("work_group", ctypes.c_int64)]


class LBMError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


def _bind(path: str):
    """Load the C-ABI library at `path` and declare its signatures."""
    # torch carries its own HIP runtime; importing it first makes the library bind to that
    # same runtime (matched by soname) instead of loading a second copy into the process.
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python paper_2605_27004_amd/build.py` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    ip32 = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "lbm_lattice_info": (ctypes.c_int, [i32, ip32, ip32, ip32, dp, ip32]),
        "lbm_prepare": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.POINTER(lbm_derived)]),
        "lbm_pop_bytes": (i64, [ctypes.POINTER(lbm_params)]),
        "lbm_rows_per_block": (i64, [ctypes.POINTER(lbm_params)]),
        "lbm_scratch_bytes": (i64, [ctypes.POINTER(lbm_params)]),
        "lbm_init": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(lbm_params), vp, vp, vp, vp, vp, vp, vp]),
        "lbm_step": (ctypes.c_int, [vp, i64]),
        "lbm_stream_floor": (ctypes.c_int, [vp, i64]),
        "lbm_moments": (ctypes.c_int, [vp, vp, vp, dp]),
        "lbm_moments_static": (ctypes.c_int, [vp, vp, vp, dp]),
        "lbm_get_populations": (ctypes.c_int, [vp, vp]),
        "lbm_set_populations": (ctypes.c_int, [vp, vp]),
        "lbm_get_f64": (ctypes.c_int, [vp, vp]),
        "lbm_time": (i64, [vp]),
        "lbm_set_launch": (ctypes.c_int, [vp, i32, i32, i32]),
        "lbm_grad_workspace_bytes": (i64, [vp, ctypes.POINTER(lbm_grad_spec)]),
        "lbm_grad": (ctypes.c_int, [vp, ctypes.POINTER(lbm_grad_spec), vp, dp, dp, dp, vp]),
        "lbm_objective": (ctypes.c_int, [vp, i32, i64, dp]),
        "lbm_destroy": (None, [vp]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_stream_copy": (ctypes.c_int, [vp, vp, i64, vp]),
        "lbm_batch_cells": (i64, [ctypes.POINTER(lbm_batch_params), ctypes.POINTER(ctypes.c_int64)]),
        "lbm_batch_pop_bytes": (i64, [ctypes.POINTER(lbm_batch_params)]),
        "lbm_batch_scratch_bytes": (i64, [ctypes.POINTER(lbm_batch_params)]),
        "lbm_batch_init": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(lbm_batch_params), vp, vp, vp, vp, vp,
                                          vp]),
        "lbm_batch_set_schedule": (ctypes.c_int, [vp, ctypes.POINTER(lbm_batch_schedule)]),
        "lbm_batch_get_schedule": (ctypes.c_int, [vp, ctypes.POINTER(lbm_batch_schedule)]),
        "lbm_batch_autotune": (ctypes.c_int, [vp, vp, i32, ctypes.POINTER(lbm_batch_schedule), dp]),
        "lbm_batch_step": (ctypes.c_int, [vp, i64]),
        "lbm_batch_status": (ctypes.c_int, [vp]),
        "lbm_batch_moments": (ctypes.c_int, [vp, vp, vp, dp]),
        "lbm_batch_get_f64": (ctypes.c_int, [vp, vp]),
        "lbm_batch_time": (i64, [vp]),
        "lbm_batch_set_spin_limit": (ctypes.c_int, [vp, ctypes.c_uint32]),
        "lbm_batch_destroy": (None, [vp]),
        "lbm_batch_plan": (i64, [ctypes.POINTER(lbm_batch_params), ctypes.POINTER(lbm_batch_schedule), i32,
                                 ctypes.POINTER(lbm_batch_item), i64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _bind(LIB_PATH)


def _check(rc: int) -> int:
    if rc != LBM_OK:
        raise LBMError(rc, lbm_last_error())
    return rc


def _ptr(x):
    """Device or host address of a torch tensor, an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


# ---- the C ABI, one function each ---------------------------------------------------------

def lbm_last_error() -> str:
    return (_lib.lbm_last_error() or b"").decode()


def lbm_lattice_info(lattice: int):
    """(q, d, c [q][3] list, w [q] list, opp [q] list) in the library's canonical order."""
    q, d = ctypes.c_int32(), ctypes.c_int32()
    c = (ctypes.c_int32 * 81)()
    w = (ctypes.c_double * 27)()
    opp = (ctypes.c_int32 * 27)()
    _check(_lib.lbm_lattice_info(lattice, ctypes.byref(q), ctypes.byref(d), c, w, opp))
    n = q.value
    return n, d.value, [list(c[3 * i: 3 * i + 3]) for i in range(n)], list(w[:n]), list(opp[:n])


def make_params(lattice="D3Q19", storage="f32", shape=(1, 1, 1), tensor=None, tensor_kind="theta", tau=0.8,
                order=3, rho0=1.0, shift="rest", force=None, masked=False, gray=False) -> lbm_params:
    p = lbm_params()
    p.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
    p.storage = STORAGES[storage] if isinstance(storage, str) else int(storage)
    p.order = int(order)
    p.tensor_kind = TENSOR_KINDS[tensor_kind] if isinstance(tensor_kind, str) else int(tensor_kind)
    p.shift_kind = SHIFTS[shift] if isinstance(shift, str) else int(shift)
    p.flags = (LBM_FLAG_MASK if masked else 0) | (LBM_FLAG_GRAY if gray else 0)
    nx, ny, nz = (tuple(shape) + (1, 1, 1))[:3]
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    t = [1.0 / 3.0, 0, 0, 0, 1.0 / 3.0, 0, 0, 0, 1.0 / 3.0] if tensor is None else [float(v) for v in
                                                                                      _flat9(tensor)]
    for i in range(9):
        p.tensor[i] = t[i]
    p.tau = float(tau)
    p.rho0 = float(rho0)
    fv = [0.0, 0.0, 0.0] if force is None else [float(v) for v in list(force) + [0.0] * (3 - len(force))]
    for a in range(3):
        p.force[a] = fv[a]
    return p


def _flat9(t):
    rows = [list(r) for r in t]
    out = [0.0] * 9
    for a, r in enumerate(rows):
        for b, v in enumerate(r):
            out[3 * a + b] = float(v)
    return out


def lbm_prepare(p: lbm_params) -> lbm_derived:
    out = lbm_derived()
    _check(_lib.lbm_prepare(ctypes.byref(p), ctypes.byref(out)))
    return out


def lbm_pop_bytes(p: lbm_params) -> int:
    n = _lib.lbm_pop_bytes(ctypes.byref(p))
    if n < 0:
        _check(_lib.lbm_prepare(ctypes.byref(p), None))
    return n


def lbm_rows_per_block(p: lbm_params) -> int:
    n = _lib.lbm_rows_per_block(ctypes.byref(p))
    if n < 0:
        _check(_lib.lbm_prepare(ctypes.byref(p), None))
    return int(n)


def lbm_scratch_bytes(p: lbm_params) -> int:
    n = _lib.lbm_scratch_bytes(ctypes.byref(p))
    if n < 0:
        _check(_lib.lbm_prepare(ctypes.byref(p), None))
    return n


def lbm_init(p: lbm_params, pop_a, pop_b, scratch, rho0, s0, mask=None, stream=None) -> int:
    ctx = ctypes.c_void_p()
    _check(_lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), _ptr(pop_a), _ptr(pop_b), _ptr(scratch), _ptr(rho0),
                         _ptr(s0), _ptr(mask), _ptr(stream)))
    return ctx.value


def lbm_step(ctx: int, nsteps: int) -> None:
    _check(_lib.lbm_step(ctx, int(nsteps)))


def lbm_stream_floor(ctx: int, nsteps: int) -> None:
    _check(_lib.lbm_stream_floor(ctx, nsteps))


def lbm_moments(ctx: int, rho=None, s=None, want_totals: bool = True):
    tot = (ctypes.c_double * 4)()
    _check(_lib.lbm_moments(ctx, _ptr(rho), _ptr(s), tot if want_totals else None))
    return list(tot) if want_totals else None


def lbm_moments_static(ctx: int, rho=None, s=None, want_totals: bool = True):
    """lbm_moments with the reduction in the library's static device array (allocates nothing)."""
    tot = (ctypes.c_double * 4)()
    _check(_lib.lbm_moments_static(ctx, _ptr(rho), _ptr(s), tot if want_totals else None))
    return list(tot) if want_totals else None


def lbm_get_populations(ctx: int, out) -> None:
    _check(_lib.lbm_get_populations(ctx, _ptr(out)))


def lbm_set_populations(ctx: int, inp) -> None:
    _check(_lib.lbm_set_populations(ctx, _ptr(inp)))


def lbm_get_f64(ctx: int, out) -> None:
    _check(_lib.lbm_get_f64(ctx, _ptr(out)))


def lbm_time(ctx: int) -> int:
    return int(_lib.lbm_time(ctx))


def lbm_set_launch(ctx: int, block_x: int, block_y: int, flags: int = 0) -> None:
    _check(_lib.lbm_set_launch(ctx, int(block_x), int(block_y), int(flags)))


def make_grad_spec(objective="kinetic_energy", nsteps=0, checkpoint_every=100, outlet_plane=0) -> lbm_grad_spec:
    spec = lbm_grad_spec()
    spec.objective = OBJECTIVES[objective] if isinstance(objective, str) else int(objective)
    spec.reserved = 0
    spec.nsteps = int(nsteps)
    spec.checkpoint_every = int(checkpoint_every)
    spec.outlet_plane = int(outlet_plane)
    return spec


def lbm_grad_workspace_bytes(ctx: int, spec: lbm_grad_spec) -> int:
    n = _lib.lbm_grad_workspace_bytes(ctx, ctypes.byref(spec))
    if n < 0:
        raise LBMError(int(n), lbm_last_error())
    return n


def lbm_grad(ctx: int, spec: lbm_grad_spec, workspace, dmask=None):
    """Returns (J, dtensor as a 3 x 3 nested list, dtau); dmask (device FP64 [N]) is filled in
    place when given."""
    obj = ctypes.c_double()
    dt = (ctypes.c_double * 9)()
    du = ctypes.c_double()
    _check(_lib.lbm_grad(ctx, ctypes.byref(spec), _ptr(workspace), ctypes.byref(obj), dt, ctypes.byref(du),
                         _ptr(dmask)))
    return obj.value, [list(dt[3 * a: 3 * a + 3]) for a in range(3)], du.value


def lbm_objective(ctx: int, objective="kinetic_energy", outlet_plane: int = 0) -> float:
    val = ctypes.c_double()
    kind = OBJECTIVES[objective] if isinstance(objective, str) else int(objective)
    _check(_lib.lbm_objective(ctx, kind, int(outlet_plane), ctypes.byref(val)))
    return val.value


def lbm_destroy(ctx: int) -> None:
    _lib.lbm_destroy(ctx)


def lbm_stream_copy(dst, src, nbytes: int, stream=None) -> None:
    _check(_lib.lbm_stream_copy(_ptr(dst), _ptr(src), int(nbytes), _ptr(stream)))


# ---- batches of independent domains ---------------------------------------------------------

def make_batch_params(lattice, storage, domains, order=3, shift="rest", rho0=1.0) -> lbm_batch_params:
    """Batch parameters from a list of dicts with keys shape (nx, ny, nz), tensor (3 x 3),
    tensor_kind and tau. The ctypes domain array is kept on the returned object."""
    arr = (lbm_domain * len(domains))()
    for i, dm in enumerate(domains):
        nx, ny, nz = (tuple(dm["shape"]) + (1,))[:3]
        arr[i].nx, arr[i].ny, arr[i].nz = int(nx), int(ny), int(nz)
        arr[i].tensor_kind = TENSOR_KINDS[dm.get("tensor_kind", "theta")]
        arr[i].reserved = 0
        arr[i].tensor[:] = _flat9(dm["tensor"])
        arr[i].tau = float(dm["tau"])
    p = lbm_batch_params()
    p.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
    p.storage = STORAGES[storage] if isinstance(storage, str) else int(storage)
    p.order = int(order)
    p.shift_kind = SHIFTS[shift] if isinstance(shift, str) else int(shift)
    p.rho0 = float(rho0)
    p.ndomains = len(domains)
    p.domains = ctypes.cast(arr, ctypes.POINTER(lbm_domain))
    p._keep = arr
    return p


def make_batch_schedule(mode="stepwise", xcd_group=0, wg_per_cu=0, chunk_cells=0, group_bytes=0):
    s = lbm_batch_schedule()
    s.mode = LBM_BATCH_PERSISTENT if mode == "persistent" else LBM_BATCH_STEPWISE
    s.xcd_group, s.wg_per_cu, s.reserved = int(xcd_group), int(wg_per_cu), 0
    s.chunk_cells, s.group_bytes = int(chunk_cells), int(group_bytes)
    return s


def lbm_batch_cells(p: lbm_batch_params):
    """(total cells C, per-domain cell offsets [ndomains + 1] as a list)."""
    offs = (ctypes.c_int64 * (p.ndomains + 1))()
    c = _lib.lbm_batch_cells(ctypes.byref(p), offs)
    if c < 0:
        _check(int(c))
    return int(c), list(offs)


def lbm_batch_pop_bytes(p: lbm_batch_params) -> int:
    b = _lib.lbm_batch_pop_bytes(ctypes.byref(p))
    if b < 0:
        _check(int(b))
    return int(b)


def lbm_batch_scratch_bytes(p: lbm_batch_params) -> int:
    b = _lib.lbm_batch_scratch_bytes(ctypes.byref(p))
    if b < 0:
        _check(int(b))
    return int(b)


def lbm_batch_init(p: lbm_batch_params, pop_a, pop_b, scratch, rho0, s0, stream=None) -> int:
    out = ctypes.c_void_p()
    _check(_lib.lbm_batch_init(ctypes.byref(out), ctypes.byref(p), _ptr(pop_a), _ptr(pop_b), _ptr(scratch),
                               _ptr(rho0), _ptr(s0), _ptr(stream)))
    return out.value


def lbm_batch_set_schedule(b: int, s: lbm_batch_schedule) -> None:
    _check(_lib.lbm_batch_set_schedule(b, ctypes.byref(s)))


def lbm_batch_get_schedule(b: int) -> lbm_batch_schedule:
    s = lbm_batch_schedule()
    _check(_lib.lbm_batch_get_schedule(b, ctypes.byref(s)))
    return s


def lbm_batch_autotune(b: int, backup, trial_steps: int = 20):
    """(chosen schedule, its ms per step)."""
    s = lbm_batch_schedule()
    ms = ctypes.c_double()
    _check(_lib.lbm_batch_autotune(b, _ptr(backup), int(trial_steps), ctypes.byref(s), ctypes.byref(ms)))
    return s, ms.value


def lbm_batch_step(b: int, nsteps: int) -> None:
    _check(_lib.lbm_batch_step(b, int(nsteps)))


def lbm_batch_status(b: int) -> None:
    _check(_lib.lbm_batch_status(b))


def lbm_batch_moments(b: int, rho=None, s=None, ndomains: int = 0):
    """Per-domain totals [ndomains][4] (sum rho, sum rho s) as a list of lists, or None."""
    tot = (ctypes.c_double * (4 * ndomains))() if ndomains else None
    _check(_lib.lbm_batch_moments(b, _ptr(rho), _ptr(s), tot))
    return None if tot is None else [list(tot[4 * i:4 * i + 4]) for i in range(ndomains)]


def lbm_batch_get_f64(b: int, out) -> None:
    _check(_lib.lbm_batch_get_f64(b, _ptr(out)))


def lbm_batch_time(b: int) -> int:
    return int(_lib.lbm_batch_time(b))


def lbm_batch_set_spin_limit(b: int, polls: int) -> None:
    _check(_lib.lbm_batch_set_spin_limit(b, int(polls)))


def lbm_batch_plan(p: lbm_batch_params, s: lbm_batch_schedule, cu_count: int):
    """Work lists of a persistent schedule (host only): a list of dicts with domain,
    first_cell, cells, group and work_group, in the order each work-group runs them."""
    n = _lib.lbm_batch_plan(ctypes.byref(p), ctypes.byref(s), int(cu_count), None, 0)
    if n < 0:
        _check(int(n))
    arr = (lbm_batch_item * max(int(n), 1))()
    n = _lib.lbm_batch_plan(ctypes.byref(p), ctypes.byref(s), int(cu_count), arr, int(n))
    if n < 0:
        _check(int(n))
    return [{f: getattr(arr[i], f) for f, _ in lbm_batch_item._fields_} for i in range(int(n))]


def lbm_batch_destroy(b: int) -> None:
    _lib.lbm_batch_destroy(b)


# ---- convenience wrapper: torch owns the buffers ---------------------------------------------

class Simulation:
    """A context plus the torch device buffers it runs on.

    ``rho`` is a float64 array-like [N] and ``s`` [d][N] (numpy or torch); the initial state is
    f^eq(rho, s). Work goes to ``stream`` (a torch.cuda.Stream) or torch's current stream.
    """

    def __init__(self, params: lbm_params, rho, s, device="cuda", stream=None, mask=None, buffers=None):
        import torch

        self.torch = torch
        self.params = params
        self.derived = lbm_prepare(params)
        self.q, self.d = self.derived.q, self.derived.d
        self.n = params.nx * params.ny * params.nz
        self.device = _device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # buffers: an optional dict kept by the caller; its device buffers are reused when large
        # enough (256-byte aligned by the caching allocator either way)
        bufs = buffers if buffers is not None else {}
        self.pop_a = _buffer(bufs, "pop_a", lbm_pop_bytes(params), self.device)
        self.pop_b = _buffer(bufs, "pop_b", lbm_pop_bytes(params), self.device)
        self.scratch = _buffer(bufs, "scratch", lbm_scratch_bytes(params), self.device)
        self._bufs = bufs
        rho_t = torch.as_tensor(rho, dtype=torch.float64).reshape(self.n).to(self.device)
        s_t = torch.as_tensor(s, dtype=torch.float64).reshape(self.d, self.n).to(self.device).contiguous()
        mask_t = None
        if mask is not None:
            mtype = torch.float32 if params.flags & LBM_FLAG_GRAY else torch.uint8
            mask_t = torch.as_tensor(mask).reshape(self.n).to(mtype).to(self.device).contiguous()
        torch.cuda.synchronize(self.device)
        self.ctx = lbm_init(params, self.pop_a, self.pop_b, self.scratch, rho_t, s_t, mask_t,
                            self.stream.cuda_stream)
        self.stream.synchronize()  # rho_t / s_t are read by the init kernel

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return lbm_time(self.ctx)

    def step(self, nsteps: int = 1):
        lbm_step(self.ctx, nsteps)
        return self

    def set_launch(self, block_x: int, block_y: int, flags: int = 0):
        lbm_set_launch(self.ctx, block_x, block_y, flags)

    def stream_floor(self, nsteps: int = 1):
        """Free streaming with the step's memory traffic (measurement aid; changes the state)."""
        lbm_stream_floor(self.ctx, nsteps)
        return self

    def moments(self, fields: bool = True):
        """(rho [N], s [d][N], totals[4]) as torch float64 tensors on the device (fields=False
        returns only the totals)."""
        torch = self.torch
        rho = torch.empty(self.n, dtype=torch.float64, device=self.device) if fields else None
        s = torch.empty((self.d, self.n), dtype=torch.float64, device=self.device) if fields else None
        tot = lbm_moments(self.ctx, rho, s, True)
        return rho, s, tot

    def f64(self):
        """Canonical pre-collision populations f_i(t) as a float64 [q][N] device tensor."""
        out = self.torch.empty((self.q, self.n), dtype=self.torch.float64, device=self.device)
        lbm_get_f64(self.ctx, out)
        return out

    def get_populations(self):
        out = self.torch.empty(lbm_pop_bytes(self.params), dtype=self.torch.uint8, device=self.device)
        lbm_get_populations(self.ctx, out)
        return out

    def set_populations(self, buf):
        lbm_set_populations(self.ctx, buf)

    def grad(self, objective="kinetic_energy", nsteps=0, checkpoint_every=100, outlet_plane=0, want_dmask=True):
        """Advance nsteps and return (J, dJ/dtensor [3 x 3], dJ/dtau, dJ/dm [N] device tensor or None)
        by the adjoint (see lbm_grad). The workspace comes from the buffers dict given at
        construction (reused when large enough) or is allocated for this call."""
        torch = self.torch
        spec = make_grad_spec(objective, nsteps, checkpoint_every, outlet_plane)
        ws = _buffer(self._bufs, "workspace", lbm_grad_workspace_bytes(self.ctx, spec), self.device)
        dmask = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_dmask else None
        j, dt, du = lbm_grad(self.ctx, spec, ws, dmask)
        return j, dt, du, dmask

    def objective(self, objective="kinetic_energy", outlet_plane=0) -> float:
        """J of the current state (see lbm_objective)."""
        return lbm_objective(self.ctx, objective, outlet_plane)


def _device(device):
    """torch.device with its index resolved ("cuda" -> the current CUDA device)."""
    import torch

    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def _buffer(bufs: dict, key: str, nbytes: int, device):
    """A uint8 device tensor of at least nbytes from bufs[key], replaced when too small."""
    import torch

    buf = bufs.get(key)
    if buf is None or buf.numel() < nbytes or buf.device != device:
        buf = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
        bufs[key] = buf
    return buf


class Objective:
    """J(tensor, tau, gray) of a fixed workload as a differentiable torch function.

    ``cfg`` holds lattice, storage, shape, rho [N], s [d][N] and optionally tensor_kind, order,
    force, objective ("flux" or "kinetic_energy"), nsteps, checkpoint_every and outlet_plane.
    ``obj(tensor, tau, gray=None)`` returns J (a float64 scalar tensor) after nsteps from
    f^eq(rho, s) with the given tensor (d x d or 3 x 3), tau and optional gray field [N].

    The adjoint runs only when grad mode is on and an input requires a gradient: then one
    lbm_grad call gives J and every gradient, and backward scales them. Otherwise the call is
    one forward pass (lbm_step) and lbm_objective. Device buffers (populations, scratch,
    gradient workspace) and the initial fields live on the object and are reused across calls.

    The tensor enters the update as (T + T^T) / 2, so the gradient of an off-diagonal element
    is half of lbm_grad's symmetric-direction derivative.
    """

    def __init__(self, cfg: dict, device="cuda"):
        import torch

        self.cfg = dict(cfg)
        self.device = _device(device)
        self.d = 2 if self.cfg["lattice"] == "D2Q9" else 3
        n = int(np.prod(self.cfg["shape"]))
        self._rho = torch.as_tensor(self.cfg["rho"], dtype=torch.float64).reshape(n).to(self.device)
        self._s = torch.as_tensor(self.cfg["s"], dtype=torch.float64).reshape(self.d, n).to(self.device).contiguous()
        self._bufs = {}
        self.adjoint_calls = 0
        self.forward_calls = 0

    def _simulation(self, tensor, tau, gray):
        cfg = self.cfg
        p = make_params(cfg["lattice"], cfg["storage"], cfg["shape"], tensor.detach().cpu().double().numpy(),
                        cfg.get("tensor_kind", "theta"), float(tau), cfg.get("order", 3), force=cfg.get("force"),
                        gray=gray is not None)
        return Simulation(p, self._rho, self._s, device=self.device, mask=None if gray is None else gray.detach(),
                          buffers=self._bufs)

    def value(self, tensor, tau, gray=None) -> float:
        """J alone: one forward pass, no adjoint."""
        cfg = self.cfg
        sim = self._simulation(tensor, tau, gray)
        sim.step(cfg["nsteps"])
        j = sim.objective(cfg.get("objective", "kinetic_energy"), cfg.get("outlet_plane", 0))
        sim.close()
        self.forward_calls += 1
        return j

    def gradients(self, tensor, tau, gray=None):
        """(J, dJ/dtensor per element [3 x 3] numpy, dJ/dtau, dJ/dm [N] device tensor or None)."""
        cfg = self.cfg
        sim = self._simulation(tensor, tau, gray)
        j, dt, du, dm = sim.grad(cfg.get("objective", "kinetic_energy"), cfg["nsteps"], cfg.get("checkpoint_every", 100),
                                 cfg.get("outlet_plane", 0), want_dmask=gray is not None)
        sim.close()
        self.adjoint_calls += 1
        dt = np.array(dt)
        off = ~np.eye(3, dtype=bool)
        dt[off] *= 0.5  # lbm_grad reports the derivative along E_ab + E_ba off the diagonal
        return j, dt, du, dm

    def __call__(self, tensor, tau, gray=None):
        import torch

        tau_t = torch.as_tensor(tau, dtype=torch.float64)
        track = torch.is_grad_enabled() and any(
            isinstance(t, torch.Tensor) and t.requires_grad for t in (tensor, tau, gray))
        if not track:
            return torch.tensor(self.value(tensor, float(tau_t), gray), dtype=torch.float64)
        return _objective_fn().apply(tensor, tau if isinstance(tau, torch.Tensor) else tau_t, gray, self)


_OBJECTIVE_FN = None


def _objective_fn():
    """The torch.autograd.Function behind Objective (built on first use)."""
    global _OBJECTIVE_FN
    if _OBJECTIVE_FN is not None:
        return _OBJECTIVE_FN
    import torch

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, tensor, tau, gray, obj):
            j, dt, du, dm = obj.gradients(tensor, float(tau), gray)
            d = tensor.shape[-1]
            ctx.save_for_backward(torch.as_tensor(dt[:d, :d], dtype=tensor.dtype, device=tensor.device),
                                  torch.as_tensor(du, dtype=tau.dtype, device=tau.device),
                                  dm if dm is not None else torch.zeros(0))
            ctx.gray_dtype = None if gray is None else gray.dtype
            return torch.tensor(j, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            dt, du, dm = ctx.saved_tensors
            gt = (gout.to(dt.device, torch.float64) * dt.double()).to(dt.dtype)
            gu = (gout.to(du.device, torch.float64) * du.double()).to(du.dtype)
            gg = None
            if ctx.gray_dtype is not None:
                gg = (gout.to(dm.device, torch.float64) * dm).to(ctx.gray_dtype)
            return gt, gu, gg, None

    _OBJECTIVE_FN = _Fn
    return _Fn


class Batch:
    """A batch of independent domains plus the torch device buffers it runs on.

    ``domains`` is a list of dicts (shape, tensor, tensor_kind, tau, rho [N_d], s [d][N_d]);
    the initial state of each domain is f^eq(rho, s).
    """

    def __init__(self, lattice, storage, domains, order=3, shift="rest", rho0=1.0, device="cuda", stream=None):
        import numpy as np
        import torch

        self.torch = torch
        self.params = make_batch_params(lattice, storage, domains, order, shift, rho0)
        self.ndomains = len(domains)
        self.d = 2 if self.params.lattice == LBM_D2Q9 else 3
        self.q = {LBM_D2Q9: 9, LBM_D3Q19: 19, LBM_D3Q27: 27}[self.params.lattice]
        self.cells, self.offsets = lbm_batch_cells(self.params)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.pop_bytes = lbm_batch_pop_bytes(self.params)
        self.pop_a = torch.empty(self.pop_bytes, dtype=torch.uint8, device=self.device)
        self.pop_b = torch.empty(self.pop_bytes, dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(lbm_batch_scratch_bytes(self.params), dtype=torch.uint8, device=self.device)
        rho = np.concatenate([np.asarray(dm["rho"], dtype=np.float64).reshape(-1) for dm in domains])
        s = np.concatenate([np.asarray(dm["s"], dtype=np.float64).reshape(self.d, -1) for dm in domains], axis=1)
        rho_t = torch.as_tensor(rho).to(self.device)
        s_t = torch.as_tensor(np.ascontiguousarray(s)).to(self.device)
        torch.cuda.synchronize(self.device)
        self.b = lbm_batch_init(self.params, self.pop_a, self.pop_b, self.scratch, rho_t, s_t,
                                self.stream.cuda_stream)

    def close(self):
        if getattr(self, "b", None):
            lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return lbm_batch_time(self.b)

    def step(self, nsteps: int = 1):
        lbm_batch_step(self.b, nsteps)
        return self

    def status(self):
        lbm_batch_status(self.b)

    def set_schedule(self, **kw):
        lbm_batch_set_schedule(self.b, make_batch_schedule(**kw))

    def schedule(self) -> dict:
        return lbm_batch_get_schedule(self.b).as_dict()

    def autotune(self, trial_steps: int = 20):
        """Pick the fastest schedule by measurement; returns (schedule dict, ms per step)."""
        backup = self.torch.empty(self.pop_bytes, dtype=self.torch.uint8, device=self.device)
        s, ms = lbm_batch_autotune(self.b, backup, trial_steps)
        del backup
        return s.as_dict(), ms

    def moments(self, fields: bool = True):
        """(rho [C], s [d][C] device float64 tensors or None, totals [ndomains][4] list)."""
        torch = self.torch
        rho = torch.empty(self.cells, dtype=torch.float64, device=self.device) if fields else None
        s = torch.empty((self.d, self.cells), dtype=torch.float64, device=self.device) if fields else None
        tot = lbm_batch_moments(self.b, rho, s, self.ndomains)
        return rho, s, tot

    def f64(self):
        """Canonical populations in FP64 as a device tensor [q * C]; domain i is the slice
        [q * offsets[i], q * offsets[i + 1]) viewed as [q][N_i]."""
        out = self.torch.empty(self.q * self.cells, dtype=self.torch.float64, device=self.device)
        lbm_batch_get_f64(self.b, out)
        return out

    def domain_f64(self, full, i: int):
        n = self.offsets[i + 1] - self.offsets[i]
        return full[self.q * self.offsets[i]:self.q * self.offsets[i + 1]].reshape(self.q, n)
