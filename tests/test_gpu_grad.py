"""Gradients by the hand-written adjoint (lbm_grad) against central finite differences of the
FP64 oracle (the brute-force reference) and of the library's own FP64 forward."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lbm = pytest.importorskip("paper_2605_27004_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(lattice, shape, kind="theta", force=(1e-4, -5e-5, 2e-5), seed=3, order=3):
    d = W.DIMS[lattice]
    rng = np.random.default_rng(seed)
    rho, s = W.random_fields(shape, d, seed, amp_rho=0.02, amp_s=0.03)
    n = int(np.prod(shape))
    gray = rng.uniform(0.0, 0.3, n)
    gray[rng.uniform(size=n) < 0.1] = 1.0
    t = W.config1_theta() if d == 2 else W.random_theta(seed)
    if kind in ("A", "Atilde"):
        t = W.pad3(np.linalg.inv(3.0 * t[:d, :d]))      # A with A^-1 = theta / cs^2
        if kind == "Atilde":
            t = 1.7 * t                                  # an unnormalised multiple of A
    return dict(lattice=lattice, shape=shape, d=d, rho=rho, s=s, gray=gray, tensor=t, kind=kind, tau=0.8, order=order,
                force=None if force is None else np.array(force[:d]))


def _oracle_J(c, tensor, tau, gray, steps, objective, plane, ainv0):
    """J after `steps` with the given parameters, the initial state built from the base tensor."""
    name, shape, d = c["lattice"], c["shape"], c["d"]
    f = oracle.init(name, shape, ainv0, c["rho"], c["s"], c["order"])
    ainv = oracle.tensor_to_ainv(np.asarray(tensor)[:d, :d], c["kind"], d)
    oracle.steps_gray(name, shape, ainv, tau, f, steps, gray, c["order"], force=c["force"])
    return oracle.objective(name, shape, f, 0 if objective == "flux" else 1, plane, force=c["force"])


def _gpu(c, storage, steps, objective, plane, ckpt, tensor=None, tau=None, gray=None, grad=True):
    p = lbm.make_params(c["lattice"], storage, c["shape"], c["tensor"] if tensor is None else tensor, c["kind"],
                        c["tau"] if tau is None else tau, c["order"], force=c["force"], gray=True)
    sim = lbm.Simulation(p, c["rho"], c["s"], mask=(c["gray"] if gray is None else gray).astype(np.float32))
    if grad:
        j, dt, du, dm = sim.grad(objective, steps, ckpt, plane)
        return j, np.array(dt), du, dm.cpu().numpy()
    sim.step(steps)
    return sim


CASES = [("D2Q9", (16, 12, 1), "theta", "kinetic_energy"), ("D2Q9", (16, 12, 1), "theta", "flux"),
         ("D3Q19", (8, 6, 5), "A", "kinetic_energy"), ("D3Q27", (7, 6, 5), "theta", "flux"),
         ("D2Q9", (14, 9, 1), "Atilde", "flux"), ("D3Q19", (7, 6, 5), "Atilde", "kinetic_energy"),
         ("D2Q9", (13, 10, 1), "theta", "flux", 2), ("D3Q19", (7, 7, 5), "A", "kinetic_energy", 2)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(str(v) for v in c))
def test_adjoint_matches_oracle_finite_differences(case):
    lattice, shape, kind, objective = case[:4]
    c = _case(lattice, shape, kind, order=case[4] if len(case) > 4 else 3)
    steps, ckpt, plane = 23, 5, 3
    d = c["d"]
    # the gray field is stored in single precision by the library; the oracle uses the same values
    gray = c["gray"].astype(np.float32).astype(np.float64)
    c["gray"] = gray
    ainv0 = oracle.tensor_to_ainv(c["tensor"][:d, :d], kind, d)
    j, dt, du, dm = _gpu(c, "f64", steps, objective, plane, ckpt)
    j0 = _oracle_J(c, c["tensor"], c["tau"], gray, steps, objective, plane, ainv0)
    assert abs(j - j0) <= 1e-12 * abs(j0)
    # central differences: truncation ~ h^2, rounding ~ eps |J| / h; the gate is 1e-6 of the
    # derivative plus 1e-9 of |J| (above both for these step sizes)
    def close(g, fd):
        return abs(g - fd) <= 1e-6 * abs(fd) + 1e-9 * abs(j0)

    for a in range(d):
        for b in range(a, d):
            h = 1e-5
            tp = c["tensor"].copy(); tm = c["tensor"].copy()
            tp[a, b] += h; tm[a, b] -= h
            if a != b:
                tp[b, a] += h; tm[b, a] -= h
            fd = (_oracle_J(c, tp, c["tau"], gray, steps, objective, plane, ainv0)
                  - _oracle_J(c, tm, c["tau"], gray, steps, objective, plane, ainv0)) / (2 * h)
            assert close(dt[a, b], fd), (a, b, dt[a, b], fd)
    h = 1e-5
    fd = (_oracle_J(c, c["tensor"], c["tau"] + h, gray, steps, objective, plane, ainv0)
          - _oracle_J(c, c["tensor"], c["tau"] - h, gray, steps, objective, plane, ainv0)) / (2 * h)
    assert close(du, fd), (du, fd)
    rng = np.random.default_rng(7)
    for cell in rng.choice(len(gray), 4, replace=False):
        def central(h):
            gp = gray.copy(); gm = gray.copy()
            gp[cell] += h; gm[cell] -= h
            return (_oracle_J(c, c["tensor"], c["tau"], gp, steps, objective, plane, ainv0)
                    - _oracle_J(c, c["tensor"], c["tau"], gm, steps, objective, plane, ainv0)) / (2 * h)
        # J is a polynomial of high degree in one cell's m (23 compounded blends): Richardson
        # extrapolation of two central differences removes the h^2 truncation term
        fd = (4.0 * central(5e-5) - central(1e-4)) / 3.0
        assert close(dm[cell], fd), (cell, dm[cell], fd)


def test_adjoint_matches_gpu_finite_differences_no_force():
    """Without a force, against central differences of the library's own FP64 forward. The
    initial populations are those of the base parameters; the K-independent weight shift makes
    the stored deviations mean the same populations in every context."""
    c = _case("D3Q19", (9, 7, 6), force=None, seed=5)
    steps, ckpt = 30, 30
    gray = c["gray"].astype(np.float32)

    def sim_for(tensor, tau):
        p = lbm.make_params(c["lattice"], "f64", c["shape"], tensor, "theta", tau, shift="weight", gray=True)
        return lbm.Simulation(p, c["rho"], c["s"], mask=gray)

    base = sim_for(c["tensor"], c["tau"])
    snap = base.get_populations()
    j, dt, du, _ = base.grad("kinetic_energy", steps, ckpt, 0, want_dmask=False)

    def J(tensor, tau):
        sim = sim_for(tensor, tau)
        sim.set_populations(snap)
        return sim.grad("kinetic_energy", steps, ckpt, 0, want_dmask=False)[0]

    h = 1e-4
    fd = (J(c["tensor"], c["tau"] + h) - J(c["tensor"], c["tau"] - h)) / (2 * h)
    assert abs(du - fd) <= 1e-6 * abs(fd) + 1e-9 * abs(j)
    h = 1e-5
    tp = c["tensor"].copy(); tm = c["tensor"].copy()
    tp[0, 1] += h; tp[1, 0] += h; tm[0, 1] -= h; tm[1, 0] -= h
    fd = (J(tp, c["tau"]) - J(tm, c["tau"])) / (2 * h)
    assert abs(dt[0][1] - fd) <= 1e-6 * abs(fd) + 1e-9 * abs(j)


def test_adjoint_launch_over_many_row_tiles_matches_gpu_finite_differences():
    """A grid of many adjoint work-groups (70 x 130 x 67: 65 row tiles of 128 x 2 per z-plane,
    4355 work-groups in a one-dimensional launch, every tile ragged in x: 70 of its 128 lanes),
    with force, gray cells and the flux objective: the FP64 gradient against central differences
    of the FP64 forward."""
    c = _case("D3Q19", (70, 130, 67), seed=9)
    steps, ckpt, plane = 12, 5, 69
    gray = c["gray"].astype(np.float32)

    def sim_for(tensor, tau):
        p = lbm.make_params(c["lattice"], "f64", c["shape"], tensor, "theta", tau, force=c["force"], shift="weight",
                            gray=True)
        return lbm.Simulation(p, c["rho"], c["s"], mask=gray)

    base = sim_for(c["tensor"], c["tau"])
    snap = base.get_populations()
    j, dt, du, _ = base.grad("flux", steps, ckpt, plane, want_dmask=False)
    base.close()

    def J(tensor, tau):
        sim = sim_for(tensor, tau)
        sim.set_populations(snap)
        v = sim.grad("flux", steps, ckpt, plane, want_dmask=False)[0]
        sim.close()
        return v

    h = 1e-4
    fd = (J(c["tensor"], c["tau"] + h) - J(c["tensor"], c["tau"] - h)) / (2 * h)
    print(f"[grad] many-tile dtau {du:.9e} fd {fd:.9e}", flush=True)
    assert abs(du - fd) <= 1e-5 * abs(fd) + 1e-9 * abs(j)
    h = 1e-5
    tp = c["tensor"].copy(); tm = c["tensor"].copy()
    tp[1, 2] += h; tp[2, 1] += h; tm[1, 2] -= h; tm[2, 1] -= h
    fd = (J(tp, c["tau"]) - J(tm, c["tau"])) / (2 * h)
    print(f"[grad] many-tile dT_yz {dt[1][2]:.9e} fd {fd:.9e}", flush=True)
    assert abs(dt[1][2] - fd) <= 1e-5 * abs(fd) + 1e-9 * abs(j)


def test_grad_rejects_an_adjoint_z_plane_beyond_4gib():
    """FP16 storage of an 11000^2 D2Q9 grid passes the z-plane limit (9 x 2 bytes per cell),
    but its FP32 adjoint populations would not (9 x 4 bytes): lbm_grad_workspace_bytes
    reports LBM_ERR_SIZE instead of letting the kernels' 32-bit offsets wrap."""
    shape = (11000, 11000, 1)
    rho, s = W.uniform_fields(shape, 2)
    p = lbm.make_params("D2Q9", "f16", shape, W.config1_theta(), "theta", 0.8)
    sim = lbm.Simulation(p, rho, s)
    spec = lbm.make_grad_spec("kinetic_energy", 10, 5, 0)
    rc = lbm._lib.lbm_grad_workspace_bytes(sim.ctx, ctypes.byref(spec))
    sim.close()
    del sim
    torch.cuda.empty_cache()
    assert rc == lbm.LBM_ERR_SIZE


@pytest.mark.parametrize("ckpt", [1, 4, 23, 50])
def test_checkpoint_interval_does_not_change_gradients(ckpt):
    c = _case("D2Q9", (12, 10, 1))
    ref = _gpu(c, "f64", 23, "flux", 2, 100)
    got = _gpu(c, "f64", 23, "flux", 2, ckpt)
    assert got[0] == ref[0]
    assert np.array_equal(got[1], ref[1]) and got[2] == ref[2] and np.array_equal(got[3], ref[3])


def test_fp32_adjoint_close_to_fp64():
    """FP32 storage against the library's FP64 path (which matches oracle finite differences
    to 1e-6) on every output, at the FP32 gate of the step count."""
    c = _case("D3Q19", (10, 8, 6))
    steps = 40
    a = _gpu(c, "f64", steps, "kinetic_energy", 0, 10)
    b = _gpu(c, "f32", steps, "kinetic_energy", 0, 10)
    e = [abs(b[0] - a[0]) / abs(a[0]), np.abs(b[1] - a[1]).max() / np.abs(a[1]).max(),
         abs(b[2] - a[2]) / abs(a[2]), np.abs(b[3] - a[3]).max() / np.abs(a[3]).max()]
    print(f"[grad32] f32 vs f64 T={steps}: J {e[0]:.2e} dT {e[1]:.2e} dtau {e[2]:.2e} dm {e[3]:.2e} "
          f"(gate {_tol32(steps):.2e})", flush=True)
    assert max(e) <= _tol32(steps)


def test_grad_advances_like_step():
    c = _case("D2Q9", (12, 10, 1))
    p = lbm.make_params(c["lattice"], "f64", c["shape"], c["tensor"], "theta", c["tau"], force=c["force"], gray=True)
    a = lbm.Simulation(p, c["rho"], c["s"], mask=c["gray"].astype(np.float32))
    b = lbm.Simulation(p, c["rho"], c["s"], mask=c["gray"].astype(np.float32))
    a.grad("flux", 17, 4, 1)
    b.step(17)
    assert a.t == b.t == 17
    assert torch.equal(a.f64(), b.f64())


def test_gray_forward_matches_oracle():
    c = _case("D3Q27", (9, 8, 7))
    gray = c["gray"].astype(np.float32)
    p = lbm.make_params(c["lattice"], "f64", c["shape"], c["tensor"], "theta", c["tau"], force=c["force"], gray=True)
    sim = lbm.Simulation(p, c["rho"], c["s"], mask=gray)
    sim.step(40)
    f = sim.f64().cpu().numpy()
    ainv = oracle.tensor_to_ainv(c["tensor"], "theta", 3)
    fo = oracle.init(c["lattice"], c["shape"], ainv, c["rho"], c["s"])
    oracle.steps_gray(c["lattice"], c["shape"], ainv, c["tau"], fo, 40, gray.astype(np.float64), force=c["force"])
    _, _, cc, _, _ = lbm.lbm_lattice_info(lbm.LBM_D3Q27)
    oc, _, _ = oracle.lattice("D3Q27")
    perm = [next(k for k in range(27) if list(oc[k]) == cc[i]) for i in range(27)]
    assert np.abs(f - fo[perm]).max() <= 1e-12 * np.abs(fo).max()


def test_grad_rejects_invalid_specs():
    c = _case("D2Q9", (8, 8, 1))
    p = lbm.make_params("D2Q9", "f64", (8, 8, 1), c["tensor"], "theta", 0.8)
    sim = lbm.Simulation(p, c["rho"], c["s"])
    for args in [("flux", 3, 1, 8), ("flux", 3, 0, 0), ("flux", -1, 1, 0)]:
        with pytest.raises(lbm.LBMError) as ei:
            sim.grad(*args)
        assert ei.value.code == lbm.LBM_ERR_ARG, args
    assert sim.t == 0


@pytest.mark.parametrize("lattice,shape,objective", [("D2Q9", (15, 11, 1), "flux"),
                                                     ("D3Q19", (8, 7, 6), "kinetic_energy"),
                                                     ("D3Q27", (7, 6, 5), "flux")])
def test_binary_mask_adjoint_matches_oracle_finite_differences(lattice, shape, objective):
    """Halfway bounce-back walls from a binary mask: gradients with respect to the tensor
    entries and tau, and dJ/dm at m = 0 on fluid cells (the sensitivity to adding a little
    gray there), against central differences of the FP64 oracle."""
    c = _case(lattice, shape)
    d = c["d"]
    n = int(np.prod(shape))
    rng = np.random.default_rng(21)
    mask = (rng.uniform(size=n) < 0.2).astype(np.uint8)
    steps, ckpt, plane = 21, 6, 2
    ainv0 = oracle.tensor_to_ainv(c["tensor"][:d, :d], "theta", d)

    def oracle_J(tensor, tau, gray):
        f = oracle.init(lattice, shape, ainv0, c["rho"], c["s"], mask=mask)
        ainv = oracle.tensor_to_ainv(np.asarray(tensor)[:d, :d], "theta", d)
        oracle.steps_gray(lattice, shape, ainv, tau, f, steps, gray, force=c["force"], mask=mask)
        return oracle.objective(lattice, shape, f, 0 if objective == "flux" else 1, plane, mask=mask,
                                force=c["force"])

    p = lbm.make_params(lattice, "f64", shape, c["tensor"], "theta", c["tau"], force=c["force"], masked=True)
    sim = lbm.Simulation(p, c["rho"], c["s"], mask=mask)
    j, dt, du, dm = sim.grad(objective, steps, ckpt, plane)
    dt, dm = np.array(dt), dm.cpu().numpy()
    zero = np.zeros(n)
    j0 = oracle_J(c["tensor"], c["tau"], zero)
    print(f"[grad] masked {lattice} J={j:.6e} oracle {j0:.6e}", flush=True)
    assert abs(j - j0) <= 1e-12 * abs(j0)

    def close(g, fd):
        return abs(g - fd) <= 1e-6 * abs(fd) + 1e-9 * abs(j0)

    for a in range(d):
        for b in range(a, d):
            h = 1e-5
            tp = c["tensor"].copy(); tm = c["tensor"].copy()
            tp[a, b] += h; tm[a, b] -= h
            if a != b:
                tp[b, a] += h; tm[b, a] -= h
            fd = (oracle_J(tp, c["tau"], zero) - oracle_J(tm, c["tau"], zero)) / (2 * h)
            assert close(dt[a, b], fd), (a, b, dt[a, b], fd)
    h = 1e-5
    fd = (oracle_J(c["tensor"], c["tau"] + h, zero) - oracle_J(c["tensor"], c["tau"] - h, zero)) / (2 * h)
    assert close(du, fd), (du, fd)
    assert np.all(dm[mask == 1] == 0.0)
    h = 1e-4
    for cell in rng.choice(np.flatnonzero(mask == 0), 4, replace=False):
        gp = zero.copy(); gm = zero.copy()
        gp[cell] = h; gm[cell] = -h
        fd = (oracle_J(c["tensor"], c["tau"], gp) - oracle_J(c["tensor"], c["tau"], gm)) / (2 * h)
        assert close(dm[cell], fd), (cell, dm[cell], fd)


def _objective_cfg(c, nsteps=12, objective="kinetic_energy"):
    return dict(lattice=c["lattice"], storage="f64", shape=c["shape"], rho=c["rho"], s=c["s"], force=c["force"],
                objective=objective, nsteps=nsteps, checkpoint_every=5, outlet_plane=1)


def test_autograd_function():
    """Objective as a torch function: J and the gradients of lbm_grad, scaled by backward; the
    tensor's off-diagonal elements each get half of lbm_grad's symmetric-direction derivative
    (the update uses (T + T^T) / 2). Inputs on the GPU get their gradients on the GPU."""
    c = _case("D2Q9", (10, 8, 1))
    obj = lbm.Objective(_objective_cfg(c))
    tensor = torch.tensor(c["tensor"][:2, :2], dtype=torch.float64, device="cuda", requires_grad=True)
    tau = torch.tensor(0.8, dtype=torch.float64, device="cuda", requires_grad=True)
    gray = torch.tensor(c["gray"], dtype=torch.float32, device="cuda", requires_grad=True)
    j = obj(tensor, tau, gray)
    (2.0 * j).backward()
    j2, dt, du, dm = _gpu(c, "f64", 12, "kinetic_energy", 0, 5)
    assert float(j.detach()) == j2
    half = np.where(np.eye(2, dtype=bool), 1.0, 0.5)
    assert tensor.grad.device.type == "cuda" and tau.grad.device.type == "cuda"
    assert np.allclose(tensor.grad.cpu().numpy(), 2 * dt[:2, :2] * half, rtol=1e-14, atol=0)
    assert abs(float(tau.grad) - 2 * du) <= 1e-14 * abs(du)
    assert np.allclose(gray.grad.cpu().numpy(), 2 * dm, rtol=1e-6)
    assert obj.adjoint_calls == 1 and obj.forward_calls == 0


@pytest.mark.parametrize("lattice,shape,objective", [("D2Q9", (9, 7, 1), "flux"), ("D3Q19", (6, 5, 4), "kinetic_energy")])
def test_autograd_symmetric_parameter_matches_oracle(lattice, shape, objective):
    """A scalar theta placed in both off-diagonal slots (x, y) of the tensor: dJ/dtheta through
    autograd's chain rule against central differences of the FP64 oracle."""
    c = _case(lattice, shape)
    d = c["d"]
    steps = 14
    obj = lbm.Objective(_objective_cfg(c, steps, objective))
    base = torch.tensor(c["tensor"][:d, :d], dtype=torch.float64)
    theta = torch.tensor(float(c["tensor"][0, 1]), dtype=torch.float64, requires_grad=True)
    e01 = torch.zeros(d, d, dtype=torch.float64)
    e01[0, 1] = e01[1, 0] = 1.0
    t = base * (1 - e01) + theta * e01
    j = obj(t, 0.8, None)
    j.backward()
    g = float(theta.grad)
    ainv0 = oracle.tensor_to_ainv(c["tensor"][:d, :d], "theta", d)
    zero = np.zeros(int(np.prod(shape)))
    cc = dict(c, kind="theta")

    def oj(v):
        tt = c["tensor"].copy()
        tt[0, 1] = tt[1, 0] = v
        return _oracle_J(cc, tt, 0.8, zero, steps, objective, 1, ainv0)

    h = 1e-5
    v0 = float(c["tensor"][0, 1])
    fd = (oj(v0 + h) - oj(v0 - h)) / (2 * h)
    print(f"[grad] autograd dJ/dtheta {g:.12e} oracle fd {fd:.12e}", flush=True)
    assert abs(g - fd) <= 1e-6 * abs(fd) + 1e-9 * abs(float(j))


def test_objective_without_grad_runs_no_adjoint():
    """Under torch.no_grad (or with no input requiring a gradient) the call is one forward
    pass and lbm_objective: the same J as lbm_grad's, no adjoint, and the device buffers of the
    first call are reused by the next."""
    c = _case("D3Q19", (12, 9, 7))
    obj = lbm.Objective(_objective_cfg(c, 15, "flux"))
    tensor = torch.tensor(c["tensor"], dtype=torch.float64, requires_grad=True)
    with torch.no_grad():
        j1 = obj(tensor, 0.8)
    ptr = obj._bufs["pop_a"].data_ptr()
    j2 = obj(tensor.detach(), 0.8)
    assert obj.adjoint_calls == 0 and obj.forward_calls == 2
    assert obj._bufs["pop_a"].data_ptr() == ptr
    jg = obj(tensor, 0.8)
    assert obj.adjoint_calls == 1
    assert float(j1) == float(j2) == float(jg.detach())


# FP32 storage (the gradient workload's precision: FP32 forward and adjoint populations, FP64
# parameter sums) against central differences of the FP64 oracle. Gate per group of outputs
# (J; tensor entries; tau; sampled dm), relative to the group's largest reference value:
#     tol32 = kappa T u32,  u32 = 2^-24, T the number of steps.
# Each step rounds the stored deviations, the adjoint populations and the per-cell arithmetic
# once, relative to the adjoint's own magnitude, and those errors add up at worst linearly over T
# steps. kappa is the ratio of that magnitude to the reported derivative (the derivative's
# conditioning): 1 on the gradient workload itself, 4 for the kinetic-energy objective on
# random fields, 32 for the outlet flux on random fields, whose tensor derivative is a small
# residual of the adjoint's terms (measured with an FP64-arithmetic build of the same adjoint on
# FP32 storage: every stage of the FP32 adjoint contributes, no single term dominates).
KAPPA = {"kinetic_energy": 4.0, "flux": 32.0}


def _tol32(steps, kappa=1.0):
    return kappa * steps * 2.0 ** -24


FP32_CASES = [("D2Q9", (16, 12, 1), "theta", "flux"), ("D3Q19", (8, 6, 5), "A", "kinetic_energy"),
              ("D3Q27", (7, 6, 5), "theta", "kinetic_energy")]


@pytest.mark.parametrize("case", FP32_CASES, ids=lambda c: "-".join(str(v) for v in c))
def test_fp32_adjoint_matches_oracle_finite_differences(case):
    lattice, shape, kind, objective = case
    c = _case(lattice, shape, kind)
    steps, ckpt, plane = 23, 5, 3
    d = c["d"]
    gray = c["gray"].astype(np.float32).astype(np.float64)
    c["gray"] = gray
    ainv0 = oracle.tensor_to_ainv(c["tensor"][:d, :d], kind, d)
    j, dt, du, dm = _gpu(c, "f32", steps, objective, plane, ckpt)
    j0 = _oracle_J(c, c["tensor"], c["tau"], gray, steps, objective, plane, ainv0)
    fdt = np.zeros((d, d))
    for a in range(d):
        for b in range(a, d):
            h = 1e-5
            tp = c["tensor"].copy(); tm = c["tensor"].copy()
            tp[a, b] += h; tm[a, b] -= h
            if a != b:
                tp[b, a] += h; tm[b, a] -= h
            fdt[a, b] = fdt[b, a] = (_oracle_J(c, tp, c["tau"], gray, steps, objective, plane, ainv0)
                                     - _oracle_J(c, tm, c["tau"], gray, steps, objective, plane, ainv0)) / (2 * h)
    h = 1e-5
    fdu = (_oracle_J(c, c["tensor"], c["tau"] + h, gray, steps, objective, plane, ainv0)
           - _oracle_J(c, c["tensor"], c["tau"] - h, gray, steps, objective, plane, ainv0)) / (2 * h)
    cells = np.random.default_rng(7).choice(len(gray), 4, replace=False)
    fdm = []
    for cell in cells:
        def central(hh):
            gp = gray.copy(); gm = gray.copy()
            gp[cell] += hh; gm[cell] -= hh
            return (_oracle_J(c, c["tensor"], c["tau"], gp, steps, objective, plane, ainv0)
                    - _oracle_J(c, c["tensor"], c["tau"], gm, steps, objective, plane, ainv0)) / (2 * hh)
        fdm.append((4.0 * central(5e-5) - central(1e-4)) / 3.0)
    fdm = np.array(fdm)
    e_j = abs(j - j0) / abs(j0)
    e_t = np.abs(dt[:d, :d] - fdt).max() / np.abs(fdt).max()
    e_u = abs(du - fdu) / abs(fdu)
    e_m = np.abs(dm[cells] - fdm).max() / np.abs(fdm).max()
    tol = _tol32(steps, KAPPA[objective])
    print(f"[grad32] {lattice} {kind} {objective} T={steps}: J {e_j:.2e} dT {e_t:.2e} dtau {e_u:.2e} "
          f"dm {e_m:.2e} (gate {tol:.2e})", flush=True)
    assert e_j <= tol and e_t <= tol and e_u <= tol and e_m <= tol


@pytest.mark.parametrize("lattice,shape,objective", [("D2Q9", (15, 11, 1), "flux"), ("D3Q19", (8, 7, 6), "kinetic_energy")])
def test_fp32_binary_mask_adjoint_matches_oracle_finite_differences(lattice, shape, objective):
    """Halfway bounce-back walls, FP32 storage: tensor entries, tau and dJ/dm at m = 0 on fluid
    cells against central differences of the FP64 oracle, at the FP32 gate."""
    c = _case(lattice, shape)
    d = c["d"]
    n = int(np.prod(shape))
    rng = np.random.default_rng(21)
    mask = (rng.uniform(size=n) < 0.2).astype(np.uint8)
    steps, ckpt, plane = 21, 6, 2
    ainv0 = oracle.tensor_to_ainv(c["tensor"][:d, :d], "theta", d)

    def oracle_J(tensor, tau, gray):
        f = oracle.init(lattice, shape, ainv0, c["rho"], c["s"], mask=mask)
        ainv = oracle.tensor_to_ainv(np.asarray(tensor)[:d, :d], "theta", d)
        oracle.steps_gray(lattice, shape, ainv, tau, f, steps, gray, force=c["force"], mask=mask)
        return oracle.objective(lattice, shape, f, 0 if objective == "flux" else 1, plane, mask=mask,
                                force=c["force"])

    p = lbm.make_params(lattice, "f32", shape, c["tensor"], "theta", c["tau"], force=c["force"], masked=True)
    sim = lbm.Simulation(p, c["rho"], c["s"], mask=mask)
    j, dt, du, dm = sim.grad(objective, steps, ckpt, plane)
    dt, dm = np.array(dt), dm.cpu().numpy()
    zero = np.zeros(n)
    j0 = oracle_J(c["tensor"], c["tau"], zero)
    fdt = np.zeros((d, d))
    for a in range(d):
        for b in range(a, d):
            h = 1e-5
            tp = c["tensor"].copy(); tm = c["tensor"].copy()
            tp[a, b] += h; tm[a, b] -= h
            if a != b:
                tp[b, a] += h; tm[b, a] -= h
            fdt[a, b] = fdt[b, a] = (oracle_J(tp, c["tau"], zero) - oracle_J(tm, c["tau"], zero)) / (2 * h)
    h = 1e-5
    fdu = (oracle_J(c["tensor"], c["tau"] + h, zero) - oracle_J(c["tensor"], c["tau"] - h, zero)) / (2 * h)
    cells = rng.choice(np.flatnonzero(mask == 0), 4, replace=False)
    fdm = []
    for cell in cells:
        h = 1e-4
        gp = zero.copy(); gm = zero.copy()
        gp[cell] = h; gm[cell] = -h
        fdm.append((oracle_J(c["tensor"], c["tau"], gp) - oracle_J(c["tensor"], c["tau"], gm)) / (2 * h))
    fdm = np.array(fdm)
    e_j = abs(j - j0) / abs(j0)
    e_t = np.abs(dt[:d, :d] - fdt).max() / np.abs(fdt).max()
    e_u = abs(du - fdu) / abs(fdu)
    e_m = np.abs(dm[cells] - fdm).max() / np.abs(fdm).max()
    tol = _tol32(steps, KAPPA[objective])
    print(f"[grad32] masked {lattice} {objective} T={steps}: J {e_j:.2e} dT {e_t:.2e} dtau {e_u:.2e} "
          f"dm {e_m:.2e} (gate {tol:.2e})", flush=True)
    assert np.all(dm[mask == 1] == 0.0)
    assert e_j <= tol and e_t <= tol and e_u <= tol and e_m <= tol


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_gradient_workload_full_size(lattice):
    """The gradient workload at full size (D2Q9 512^2 / D3Q19 128^3 channel with obstacles,
    2000 steps, checkpoints every 100, outlet flux): the FP64 adjoint (tau, every tensor entry,
    the two largest gray-field derivatives) against central differences of the FP64 forward
    with the initial state held fixed, and the FP32 adjoint
    (the configured precision) against the FP64 one."""
    wl = W.config4(lattice)
    gray = wl.meta["gray"].astype(np.float32)
    plane, ck, steps = wl.meta["outlet_plane"], wl.meta["checkpoint_every"], wl.steps

    def sim_for(storage, tensor=None, tau=None, g=None):
        p = lbm.make_params(lattice, storage, wl.shape, wl.tensor if tensor is None else tensor, "theta",
                            wl.tau if tau is None else tau, force=wl.meta["force"], gray=True, shift="weight")
        return lbm.Simulation(p, wl.rho, wl.s, mask=gray if g is None else g)

    base = sim_for("f64")
    snap = base.get_populations()
    j, dt, du, dm = base.grad("flux", steps, ck, plane)
    dm = dm.cpu().numpy()
    print(f"[grad] {lattice} J={j:.6e} dtau={du:.6e} dT={np.array(dt).ravel()[:3]}", flush=True)

    def J(**kw):
        sim = sim_for("f64", **kw)
        sim.set_populations(snap)
        sim.step(steps)
        rho, s, _ = sim.moments()
        n = wl.shape
        flux = (rho * s[0]).reshape(n[2], n[1], n[0])[:, :, plane]
        return float(flux.sum())

    def close(g, fd):
        return abs(g - fd) <= 1e-5 * abs(fd) + 1e-9 * abs(j)

    h = 1e-4
    fd = (J(tau=wl.tau + h) - J(tau=wl.tau - h)) / (2 * h)
    assert close(du, fd), (du, fd)
    # every independent tensor entry; an off-diagonal derivative is the one of the symmetric
    # perturbation T_ab + h, T_ba + h
    h = 1e-5
    d = 2 if lattice == "D2Q9" else 3
    for a in range(d):
        for b in range(a, d):
            tp = wl.tensor.copy(); tm = wl.tensor.copy()
            tp[a, b] += h; tm[a, b] -= h
            if a != b:
                tp[b, a] += h; tm[b, a] -= h
            fd = (J(tensor=tp) - J(tensor=tm)) / (2 * h)
            assert close(dt[a][b], fd), (a, b, dt[a][b], fd)
    h = 1e-3
    for cell in np.argsort(-np.abs(dm))[:2]:
        gp = gray.copy(); gm = gray.copy()
        gp[cell] += h; gm[cell] -= h
        fd = (J(g=gp) - J(g=gm)) / (2 * h)
        # the FP32 gray field limits the perturbation's exactness to 2^-24 relative of h
        assert abs(dm[cell] - fd) <= 1e-4 * abs(fd) + 1e-9 * abs(j), (cell, dm[cell], fd)
    f32 = sim_for("f32")
    j32, dt32, du32, dm32 = f32.grad("flux", steps, ck, plane)
    dm32 = dm32.cpu().numpy()
    print(f"[grad] {lattice} f32 vs f64: J {abs(j32 / j - 1):.2e} dtau {abs(du32 / du - 1):.2e} "
          f"dm {np.abs(dm32 - dm).max() / np.abs(dm).max():.2e}", flush=True)
    dt, dt32 = np.array(dt), np.array(dt32)
    e_t = np.abs(dt32 - dt).max() / np.abs(dt).max()
    print(f"[grad32] {lattice} full size T={steps}: J {abs(j32 / j - 1):.2e} dT {e_t:.2e} dtau {abs(du32 / du - 1):.2e} "
          f"dm {np.abs(dm32 - dm).max() / np.abs(dm).max():.2e} (gate {_tol32(steps):.2e})", flush=True)
    tol = _tol32(steps)
    assert abs(j32 / j - 1) <= tol and abs(du32 / du - 1) <= tol and e_t <= tol
    assert np.abs(dm32 - dm).max() <= tol * np.abs(dm).max()
