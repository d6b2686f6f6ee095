"""Pins of the oracle's solid-wall (halfway bounce-back) and body-force (exact-difference)
extensions. The paper only names walls and forcing as future work (Sec. 5); these pins tie the
chosen definitions to exact invariants and to textbook channel-flow results. CPU only."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import physics as P

LATS = ["D2Q9", "D3Q19", "D3Q27"]


def _ainv(name, seed=3):
    d = oracle.dim(name)
    t = W.random_theta(seed)[:d, :d] if d == 3 else W.config1_theta()[:2, :2]
    return oracle.tensor_to_ainv(t, "theta", d)


@pytest.mark.parametrize("name", LATS)
def test_force_adds_exactly_F_per_cell_per_step(name):
    """Exact-difference forcing on a uniform periodic state: every step adds F to the momentum
    of every cell and leaves the state uniform; the read-out velocity is (j + F/2)/rho."""
    d = oracle.dim(name)
    shape = (3, 4, 2 if d == 3 else 1)
    n = int(np.prod(shape))
    ainv = _ainv(name)
    F = np.array([2e-5, -1e-5, 3e-5])[:d]
    rho0, s0 = W.uniform_fields(shape, d, 1.05, np.array([0.01, -0.02, 0.005])[:d])
    f = oracle.init(name, shape, ainv, rho0, s0)
    for t in range(1, 6):
        oracle.steps(name, shape, ainv, 0.8, f, 1, force=F)
        rho, s = oracle.moments(name, f, force=F)
        j = rho[0] * s[:, 0] - F / 2
        assert np.abs(rho - 1.05).max() < 1e-14
        assert np.abs(j - (1.05 * s0[:, 0] + t * F)).max() < 1e-15
        assert np.abs(s - s[:, :1]).max() < 1e-16


@pytest.mark.parametrize("name", LATS)
def test_bounce_back_conserves_mass(name):
    d = oracle.dim(name)
    shape = (9, 8, 7 if d == 3 else 1)
    n = int(np.prod(shape))
    rng = np.random.default_rng(4)
    mask = (rng.uniform(size=n) < 0.3).astype(np.uint8)
    rho0, s0 = W.random_fields(shape, d, seed=5)
    ainv = _ainv(name)
    f = oracle.init(name, shape, ainv, rho0, s0, mask=mask)
    m0 = f.sum()
    oracle.steps(name, shape, ainv, 0.7, f, 200, mask=mask, force=np.array([1e-5, 0, 0])[:d])
    assert abs(f.sum() - m0) / m0 < 1e-13
    assert np.all(f[:, mask == 1] == 0.0)


def _poiseuille(tensor, tau, order, name="D2Q9", H=16, F=1e-6, steps=20000):
    d = oracle.dim(name)
    ny = H + 2
    shape = (1, ny, 1)
    mask = np.zeros(ny, np.uint8)
    mask[0] = mask[-1] = 1
    ainv = oracle.tensor_to_ainv(np.asarray(tensor)[:d, :d], "theta", d)
    rho0, s0 = W.uniform_fields(shape, d)
    force = np.zeros(d)
    force[0] = F
    f = oracle.init(name, shape, ainv, rho0, s0, order, mask=mask)
    oracle.steps(name, shape, ainv, tau, f, steps, order, mask=mask, force=force)
    rho, s = oracle.moments(name, f, mask=mask, force=force)
    return ainv, rho[1:-1], s[0][1:-1], s[1][1:-1]


@pytest.mark.parametrize("order", [2, 3])
def test_poiseuille_curvature_follows_viscosity(order):
    """Force-driven channel between halfway bounce-back walls: the steady profile is a parabola
    with u'' = -F / (rho nu_eff). Third order: nu_eff = cs^2 (tau - 1/2) A^-1_yy (eq:NSprefinal2
    for u_x(y)); second order: the isotropic cs^2 (tau - 1/2) -- so the two orders differ by
    A^-1_yy, which the paper's remark on Poiseuille flow (Sec. 4, end) leaves out."""
    tau, F = 0.8, 1e-6
    ainv, rho, u, v = _poiseuille(W.config1_theta(), tau, order, F=F)
    nu = P.CS2 * (tau - 0.5) * (ainv[1, 1] if order == 3 else 1.0)
    d2 = u[2:] - 2 * u[1:-1] + u[:-2]
    assert np.abs(d2 / (-F / nu) - 1).max() < 1e-6
    assert np.abs(v).max() < 1e-12 and np.abs(rho - 1).max() < 1e-10


def test_halfway_walls_at_magic_tau():
    """Isotropic BGK with halfway bounce-back puts the no-slip walls exactly half a cell
    outside the last fluid nodes when (tau - 1/2)^2 = 3/16."""
    H = 16
    ainv, rho, u, v = _poiseuille(P.CS2 * np.eye(3), 0.5 + np.sqrt(3.0) / 4.0, 3, H=H)
    y = np.arange(1, H + 1)
    roots = np.sort(np.roots(np.polyfit(y, u, 2)).real)
    assert np.abs(roots - np.array([0.5, H + 0.5])).max() < 1e-6
