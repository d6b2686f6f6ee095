"""Pins of the oracle's gray-cell model f* = (1 - m) f^BGK + m f_opp (the differentiable obstacle
used by the gradient path) and of the two objectives. CPU only."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import physics as P

LATS = ["D2Q9", "D3Q19", "D3Q27"]


def _setup(name, shape, seed=1):
    d = oracle.dim(name)
    t = W.config1_theta() if d == 2 else W.random_theta(seed)
    ainv = oracle.tensor_to_ainv(t[:d, :d], "theta", d)
    rho0, s0 = W.random_fields(shape, d, seed)
    return d, ainv, rho0, s0


@pytest.mark.parametrize("name", LATS)
def test_gray_zero_is_plain_bgk(name):
    shape = (6, 5, 4 if oracle.dim(name) == 3 else 1)
    d, ainv, rho0, s0 = _setup(name, shape)
    a = oracle.init(name, shape, ainv, rho0, s0)
    b = a.copy()
    oracle.steps(name, shape, ainv, 0.8, a, 9)
    oracle.steps_gray(name, shape, ainv, 0.8, b, 9, np.zeros(int(np.prod(shape))))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name", LATS)
def test_gray_one_reflects_on_the_node(name):
    """m = 1: every population is sent back the way it came, f_i(t+1, x + c_i) = f_opp(i)(t, x)."""
    shape = (5, 4, 3 if oracle.dim(name) == 3 else 1)
    d, ainv, rho0, s0 = _setup(name, shape)
    c, _, _ = oracle.lattice(name)
    f = oracle.init(name, shape, ainv, rho0, s0)
    f0 = f.copy()
    oracle.steps_gray(name, shape, ainv, 0.8, f, 1, np.ones(int(np.prod(shape))))
    nx, ny, nz = shape
    opp = [next(k for k in range(len(c)) if (c[k] == -c[i]).all()) for i in range(len(c))]
    for i in range(len(c)):
        g = f0[opp[i]].reshape(nz, ny, nx)
        want = np.roll(g, shift=(c[i][2], c[i][1], c[i][0]), axis=(0, 1, 2)).reshape(-1)
        assert np.array_equal(f[i], want)


@pytest.mark.parametrize("name", LATS)
def test_gray_conserves_mass(name):
    shape = (7, 6, 5 if oracle.dim(name) == 3 else 1)
    d, ainv, rho0, s0 = _setup(name, shape)
    gray = np.random.default_rng(3).uniform(0, 1, int(np.prod(shape)))
    f = oracle.init(name, shape, ainv, rho0, s0)
    m0 = f.sum()
    oracle.steps_gray(name, shape, ainv, 0.7, f, 150, gray, force=np.full(d, 1e-5))
    assert abs(f.sum() - m0) / m0 < 1e-13


def test_gray_walls_give_the_channel_profile():
    """Rows with m = 1 act as walls: the force-driven steady profile has the anisotropic
    curvature -F/(rho nu A^-1_yy) and the same wall positions as halfway bounce-back."""
    H, tau, F = 16, 0.8, 1e-6
    ny = H + 2
    shape = (1, ny, 1)
    ainv = oracle.tensor_to_ainv(W.config1_theta()[:2, :2], "theta", 2)
    rho0, s0 = W.uniform_fields(shape, 2)
    gray = np.zeros(ny)
    gray[0] = gray[-1] = 1.0
    f = oracle.init("D2Q9", shape, ainv, rho0, s0)
    oracle.steps_gray("D2Q9", shape, ainv, tau, f, 20000, gray, force=[F, 0.0])
    _, s = oracle.moments("D2Q9", f, force=[F, 0.0])
    u = s[0][1:-1]
    nu = P.CS2 * (tau - 0.5) * ainv[1, 1]
    assert np.abs((u[2:] - 2 * u[1:-1] + u[:-2]) / (-F / nu) - 1).max() < 1e-6
    mask = np.zeros(ny, np.uint8)
    mask[0] = mask[-1] = 1
    g = oracle.init("D2Q9", shape, ainv, rho0, s0, mask=mask)
    oracle.steps("D2Q9", shape, ainv, tau, g, 20000, mask=mask, force=[F, 0.0])
    _, sb = oracle.moments("D2Q9", g, mask=mask, force=[F, 0.0])
    assert np.abs(u - sb[0][1:-1]).max() < 1e-9 * np.abs(u).max()


@pytest.mark.parametrize("name", LATS)
def test_objectives_on_uniform_flow(name):
    d = oracle.dim(name)
    shape = (5, 4, 3 if d == 3 else 1)
    ainv = oracle.tensor_to_ainv((W.config1_theta() if d == 2 else W.random_theta(2))[:d, :d], "theta", d)
    s = np.array([0.02, -0.01, 0.005])[:d]
    F = np.array([1e-3, 2e-3, -1e-3])[:d]
    rho0, s0 = W.uniform_fields(shape, d, 1.1, s)
    f = oracle.init(name, shape, ainv, rho0, s0)
    n_plane = shape[1] * shape[2]
    flux = oracle.objective(name, shape, f, 0, plane=2, force=F)
    assert flux == pytest.approx(n_plane * (1.1 * s[0] + F[0] / 2), rel=1e-13)
    ke = oracle.objective(name, shape, f, 1, force=F)
    j = 1.1 * s + F / 2
    assert ke == pytest.approx(int(np.prod(shape)) * 0.5 * (j @ j) / 1.1, rel=1e-13)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_gray_with_solid_mask(name):
    """Gray cells and a solid mask together: a zero gray field is exactly the masked update,
    and any gray field on the fluid cells still conserves mass."""
    d = oracle.dim(name)
    shape = (9, 7, 5 if d == 3 else 1)
    n = int(np.prod(shape))
    rng = np.random.default_rng(12)
    mask = (rng.uniform(size=n) < 0.25).astype(np.uint8)
    rho0, s0 = W.random_fields(shape, d, seed=13)
    t = W.random_theta(2)[:d, :d] if d == 3 else W.config1_theta()[:2, :2]
    ainv = oracle.tensor_to_ainv(t, "theta", d)
    force = np.array([2e-5, -1e-5, 1e-5])[:d]
    a = oracle.init(name, shape, ainv, rho0, s0, mask=mask)
    b = a.copy()
    oracle.steps(name, shape, ainv, 0.8, a, 40, mask=mask, force=force)
    oracle.steps_gray(name, shape, ainv, 0.8, b, 40, np.zeros(n), mask=mask, force=force)
    assert np.array_equal(a, b)
    g = oracle.init(name, shape, ainv, rho0, s0, mask=mask)
    m0 = g.sum()
    gray = rng.uniform(0.0, 0.6, n) * (mask == 0)
    oracle.steps_gray(name, shape, ainv, 0.8, g, 60, gray, mask=mask, force=force)
    assert abs(g.sum() - m0) / m0 < 1e-13
    assert np.all(g[:, mask == 1] == 0.0)
