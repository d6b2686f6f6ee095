"""Pins of the linear-stability scan (oracle/stability.py) that screens the batched workload's
tensors and relaxation times, and of the batched workload generator itself."""
import numpy as np
import pytest

import oracle
import oracle.stability as S
import workloads as W


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("tau", [0.45, 0.7, 1.5, 3.0])
def test_isotropic_spectrum_at_k0_is_conserved_modes_plus_bgk_factor(name, tau):
    """At k = 0 the step is I + omega (J - I) with J the projector onto the conserved moments:
    1 + d eigenvalues equal 1 (mass, momentum), the other q - 1 - d equal 1 - 1/tau."""
    d = 2 if name == "D2Q9" else 3
    c, _, _ = oracle.lattice(name)
    q = c.shape[0]
    J = S.jacobian_at_rest(name, np.eye(d))
    ev = np.sort(np.linalg.eigvals(np.eye(q) + (J - np.eye(q)) / tau).real)
    want = np.sort(np.r_[np.ones(1 + d), np.full(q - 1 - d, 1.0 - 1.0 / tau)])
    assert np.abs(ev - want).max() < 1e-12
    assert abs(S.spectral_radius(name, np.eye(d), tau, L=4) - max(1.0, abs(1.0 - 1.0 / tau))) < 1e-12


def test_jacobian_reproduces_equilibrium_moments():
    """sum_i J_ij = 1 (mass) and sum_i J_ij c_i = c_j (momentum) for an anisotropic tensor:
    the equilibrium's zeroth and first moments are rho and rho s exactly."""
    ainv = oracle.tensor_to_ainv(W.random_theta(3), "theta", 3)
    c, _, _ = oracle.lattice("D3Q19")
    J = S.jacobian_at_rest("D3Q19", ainv)
    assert np.abs(J.sum(axis=0) - 1.0).max() < 1e-13
    assert np.abs(c.T.astype(float) @ J - c.T).max() < 1e-12


def test_shear_mode_eigenvalue_matches_oracle_decay():
    """The least-damped eigenvalue at the wave vector of a shear wave equals the per-step decay
    the oracle's own time stepping shows for that wave (linear regime)."""
    name, n, tau = "D3Q19", 16, 0.7
    ainv = np.diag([1.5, 1.0, 0.5])
    c, _, _ = oracle.lattice(name)
    J = S.jacobian_at_rest(name, ainv)
    k = np.array([0.0, 2 * np.pi / n, 0.0])
    M = np.exp(-1j * (c @ k))[:, None] * (np.eye(c.shape[0]) + (J - np.eye(c.shape[0])) / tau)
    lam = np.linalg.eigvals(M)
    shape = (4, n, 4)
    rho, s = W.shear_wave(shape, 3, 1, 0, 1e-6)
    f = oracle.init(name, shape, ainv, rho, s)
    amps = []
    for _ in range(60):
        oracle.steps(name, shape, ainv, tau, f, 1)
        amps.append(np.abs(oracle.moments(name, f)[1][0]).max())
    rate = (amps[-1] / amps[-21]) ** (1 / 20)
    # the shear mode is the eigenvalue closest to the measured rate on the real axis
    best = np.abs(np.abs(lam) - rate).min()
    assert best < 1e-6, (rate, np.sort(np.abs(lam))[-6:])


def test_unstable_draw_grows_at_the_scanned_rate():
    """A tensor with strongly negative rest populations is unstable at tau = 0.55 (stable at
    0.7). A small random perturbation of rest, run by the oracle's own time stepping on the
    scan's 16^3 box, grows in the scan's most unstable Fourier mode by exactly the scanned
    spectral radius per step."""
    name, tau, n = "D3Q19", 0.55, 16
    ainv = oracle.tensor_to_ainv(W.random_theta(2892), "theta", 3)
    radius = S.spectral_radius(name, ainv, tau, L=n)
    assert radius > 1.05
    assert S.spectral_radius(name, ainv, 0.7, L=n) <= 1 + S.STABLE_MARGIN
    c, _, _ = oracle.lattice(name)
    q = c.shape[0]
    J = S.jacobian_at_rest(name, ainv)
    k = S.wave_vectors(3, n)
    M = np.exp(-1j * (k @ c.T.astype(float)))[:, :, None] * (np.eye(q) + (J - np.eye(q)) / tau)[None]
    worst = int(np.argmax(np.abs(np.linalg.eigvals(M)).max(axis=1)))
    mx, my, mz = np.rint(k[worst] * n / (2 * np.pi)).astype(int)
    rng = np.random.default_rng(0)
    shape = (n, n, n)
    f = oracle.init(name, shape, ainv, 1.0 + 1e-12 * rng.standard_normal(n ** 3),
                    1e-12 * rng.standard_normal((3, n ** 3)))
    r = oracle.feq(name, ainv, 1.0, np.zeros(3))
    amp = []
    for _ in range(100):
        oracle.steps(name, shape, ainv, tau, f, 1)
        modes = np.fft.fftn((f - r[:, None]).reshape(q, n, n, n), axes=(1, 2, 3))  # axes z, y, x
        amp.append(np.linalg.norm(modes[:, mz, my, mx]))
    growth = (amp[-1] / amp[-21]) ** (1 / 20)
    assert abs(growth - radius) < 1e-6, (growth, radius)


def test_batched_workload_draw():
    wl = W.config5(ndomains=64)
    assert len(wl.domains) == 64
    for i, dm in enumerate(wl.domains):
        assert all(16 <= e <= 64 for e in dm["shape"])
        assert 0.55 <= dm["tau"] <= 1.5
        ev = np.linalg.eigvalsh(dm["tensor"] * 3.0)
        assert ev.min() >= 0.6 - 1e-12 and ev.max() <= 1.4 + 1e-12
        again = W.batched_domain(i)
        assert again["shape"] == dm["shape"] and again["tau"] == dm["tau"]
        assert np.array_equal(again["tensor"], dm["tensor"])
    # s_x = u0 sin(2 pi y / ny), rho = 1
    dm = wl.domains[5]
    nx, ny, nz = dm["shape"]
    y = np.arange(nx * ny * nz) // nx % ny
    assert np.allclose(dm["s"][0], 0.01 * np.sin(2 * np.pi * y / ny)) and np.all(dm["rho"] == 1.0)


def test_stored_redraw_table_keeps_low_tau_domains_stable():
    """Every domain with tau < 0.75 (where instability lives) is linearly stable after the
    stored redraws; the table was written by the screening script of this module."""
    wl = W.config5()
    assert W.batched_redraws() is not None
    for dm in wl.domains:
        if dm["tau"] < 0.75:
            assert S.is_stable("D3Q19", dm["tensor"], "theta", dm["tau"], L=8), dm["tau"]
