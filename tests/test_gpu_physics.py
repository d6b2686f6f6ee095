"""Physics of the GPU path itself (FP64 storage), beyond element-wise parity: the decay rates,
frequencies and steady profiles the oracle's pins fix, measured on runs of the HIP library.

* Plane-channel (Poiseuille) flow driven by a body force between halfway bounce-back walls, at
  second and third order: the profile's curvature gives the effective viscosity. The paper
  remarks (end of Sec. 4) that both orders look identical for such a flow. That holds on
  D2Q9 / D3Q27 exactly when A^-1_yy = 1 (wall-normal y); in general the third-order viscosity
  is cs^2 (tau - 1/2) A^-1_yy (eq:NSprefinal2), while on D3Q19 it follows the CE operator built
  with the lattice's own third moment (for a diagonal tensor cs^2 (tau - 1/2) (A^-1_yy -
  K_zz / 2)), so there the orders differ even at A^-1_yy = 1.
* Shear modes decay at the eigenvalues of the linearised Chapman-Enskog operator built with
  the lattice's own third moment; sound travels at cs sqrt(A^-1_aa).
* Sec. 4's Taylor-Green vortex: the GPU's fitted decay rates equal the oracle's.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import physics as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lbm = pytest.importorskip("paper_2605_27004_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sim(name, shape, tensor, tau, rho, s, order=3, mask=None, force=None, kind="theta"):
    p = lbm.make_params(name, "f64", shape, tensor, kind, tau, order, force=force, masked=mask is not None)
    return lbm.Simulation(p, rho, s, mask=mask)


def _channel_viscosity(name, tensor, tau, order, H=16, F=1e-6, steps=20000):
    d = W.DIMS[name]
    shape = (1, H + 2, 1)
    mask = W.channel_mask(shape, 1)
    rho0, s0 = W.uniform_fields(shape, d)
    force = np.zeros(3)
    force[0] = F
    sim = _sim(name, shape, tensor, tau, rho0, s0, order, mask=mask, force=force[:d])
    sim.step(steps)
    rho, s, _ = sim.moments()
    sim.close()
    u = s[0].cpu().numpy()[1:-1]
    v = s[1].cpu().numpy()[1:-1]
    d2 = u[2:] - 2 * u[1:-1] + u[:-2]
    assert np.abs(v).max() < 1e-12
    assert np.abs(d2 / d2.mean() - 1).max() < 1e-6          # a parabola
    return -F / d2.mean() / (P.CS2 * (tau - 0.5))            # nu_eff / (cs^2 (tau - 1/2))


def _lattice_T(name, ainv):
    c, _, _ = oracle.lattice(name)
    d = oracle.dim(name)
    return P.third_moment_derivative(lambda r, s: oracle.feq(name, ainv, r, s, 3), c, d)


def _channel_prediction(name, ainv):
    """Third-order nu_eff / (cs^2 (tau - 1/2)) of the channel from the linearised CE operator
    with the lattice's own third moment: with u_y = 0 and variation along y only, the viscous
    term couples the in-plane components through N_ab = T_ayyb (a, b != y), and the x-velocity
    under a force along x responds with 1 / (cs^2 (N^-1)_xx)."""
    d = ainv.shape[0]
    T = _lattice_T(name, ainv)
    idx = [0] if d == 2 else [0, 2]
    N = np.array([[T[a, 1, 1, b] for b in idx] for a in idx])
    return 1.0 / (P.CS2 * np.linalg.inv(N)[0, 0])


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("ainv_yy", [1.0, 0.9])
def test_poiseuille_second_vs_third_order(name, ainv_yy):
    tau = 0.8
    ainv = np.array([[1.25, 0.2, 0.05], [0.2, ainv_yy, -0.1], [0.05, -0.1, 0.7]])
    d = W.DIMS[name]
    tensor = np.zeros((3, 3))
    tensor[:d, :d] = P.CS2 * ainv[:d, :d]
    want3 = _channel_prediction(name, ainv[:d, :d])
    if name != "D3Q19":
        assert abs(want3 - ainv_yy) < 1e-9        # the paper's CE result, eq:NSprefinal2
    r2 = _channel_viscosity(name, tensor, tau, 2)
    r3 = _channel_viscosity(name, tensor, tau, 3)
    print(f"[physics] Poiseuille {name} A^-1_yy={ainv_yy}: nu2/nu0={r2:.9f} nu3/nu0={r3:.9f} "
          f"(third order predicted {want3:.9f})", flush=True)
    assert abs(r2 - 1.0) < 1e-6
    assert abs(r3 - want3) < 1e-6
    if ainv_yy == 1.0:
        # the paper's remark (both orders identical) holds on D2Q9 / D3Q27, not on D3Q19
        assert (abs(r3 - r2) < 1e-6) == (name != "D3Q19")


@pytest.mark.parametrize("name,shape,modes,tensor", [
    ("D2Q9", (32, 32, 1), (1, 1), W.config1_theta()),
    ("D3Q19", (24, 24, 1), (1, 1), W.config2_theta(0)),
    ("D3Q27", (24, 24, 1), (1, -1), W.config2_theta(0)),
])
def test_shear_modes_decay_at_lattice_ce_rates(name, shape, modes, tensor):
    d = oracle.dim(name)
    tau = 0.8 if name == "D2Q9" else 0.7
    ainv = oracle.tensor_to_ainv(np.asarray(tensor)[:d, :d], "theta", d)
    k = P.kvector(shape, modes)
    lam, vec = P.shear_modes(_lattice_T(name, ainv), ainv, tau, k, d)
    x = P.coords(shape)
    phase = np.exp(1j * (k @ x))
    for m in range(len(lam)):
        v = vec[:, m] / np.abs(vec[1:, m]).max() * 1e-3
        rho0 = 1.0 + np.real(v[0] * phase)
        s0 = np.real(v[1:, None] * phase[None, :])
        sim = _sim(name, shape, tensor, tau, rho0, s0)
        ts, amps = [], []
        for t in range(0, 301, 20):
            if t:
                sim.step(20)
            if t >= 60:
                _, s, _ = sim.moments()
                s = s.cpu().numpy()
                ts.append(t)
                amps.append(np.linalg.norm([P.project(s[a], shape, k) for a in range(d)]))
        sim.close()
        rate = -P.log_slope(ts, amps)
        print(f"[physics] {name} mode {m}: rate {rate:.6e} lattice-CE {-lam[m].real:.6e}", flush=True)
        assert abs(rate / (-lam[m].real) - 1) < 1e-2


def test_sound_speed_follows_pressure_tensor():
    name, axis, n, tau = "D3Q27", 1, 64, 0.7
    shape = (1, n, 1)
    k = np.zeros(3)
    k[axis] = 2 * np.pi / n
    freqs = []
    for tensor in (W.config2_theta(0), P.CS2 * np.eye(3)):
        rho0, s0 = W.density_wave(shape, 3, axis, 1e-4)
        sim = _sim(name, shape, tensor, tau, rho0, s0)
        ts, ys = [0], [P.project(rho0 - 1, shape, k).real]
        for t in range(1, 401):
            sim.step(1)
            rho, _, _ = sim.moments()
            ts.append(t)
            ys.append(P.project(rho.cpu().numpy() - 1, shape, k).real)
        sim.close()
        w, _ = P.fit_damped_cos(ts, ys, np.sqrt(P.CS2) * k[axis])
        freqs.append(w)
    ainv = oracle.tensor_to_ainv(W.config2_theta(0), "theta", 3)
    assert abs(freqs[0] / freqs[1] / np.sqrt(ainv[axis, axis]) - 1) < 1e-4


def _tg_rate(a_xy, order, use_gpu):
    wl = W.e1_taylor_green(a_xy, order)
    d = wl.d
    every = wl.steps // 25
    ts, ux = [], []
    if use_gpu:
        sim = _sim(wl.lattice, wl.shape, wl.tensor, wl.tau, wl.rho, wl.s, order, kind=wl.tensor_kind)
    else:
        ainv = oracle.tensor_to_ainv(wl.tensor[:d, :d], wl.tensor_kind, d)
        f = oracle.init(wl.lattice, wl.shape, ainv, wl.rho, wl.s, order)
    for t in range(0, wl.steps + 1, every):
        if t:
            if use_gpu:
                sim.step(every)
            else:
                oracle.steps(wl.lattice, wl.shape, ainv, wl.tau, f, every, order)
        if use_gpu:
            s = sim.moments()[1].cpu().numpy()
        else:
            s = oracle.moments(wl.lattice, f)[1]
        ts.append(t)
        ux.append(np.abs(s[0]).sum())
    if use_gpu:
        sim.close()
    return P.fit_exp(ts, np.array(ux) / ux[0])


@pytest.mark.parametrize("order", [2, 3])
def test_taylor_green_rates_equal_oracle(order):
    """Sec. 4's vortex at A~_xy in {0, 0.1, 0.2, 0.4}: the decay frequency fitted to the GPU
    run equals the one fitted to the oracle run; the isotropic one is the printed 3.21e-3."""
    rates = []
    for a in (0.0, 0.1, 0.2, 0.4):
        g = _tg_rate(a, order, True)
        o = _tg_rate(a, order, False)
        print(f"[physics] Taylor-Green order {order} A~_xy={a}: GPU {g:.8e} oracle {o:.8e}", flush=True)
        assert abs(g / o - 1) < 1e-9
        rates.append(g)
    assert float(f"{rates[0]:.2e}") == 3.21e-3
    assert all(rates[i] > rates[i + 1] for i in range(3))
