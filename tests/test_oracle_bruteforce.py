"""Brute-force pin of the oracle's whole update on tiny periodic grids (2 x 2, 3 x 3 x 3 and
ragged 2 x 3 x 2): a separate NumPy transcription, written from the definitions rather than
from the oracle's closed forms, must give the same populations after five steps (to 1e-14).

The transcription takes nothing from the oracle:
  - the lattice is enumerated here: all of {-1, 0, 1}^d, with the tensor-product weights of
    numpy's three-point probabilists' Gauss-Hermite rule (App. C), and for D3Q19 the subset
    |c|^2 <= 2 with the textbook weights 1/3, 1/18, 1/36;
  - the equilibrium's Hermite coefficients a^(n) are the integrals of eq:expcoeff over the
    anisotropic Maxwell-Boltzmann distribution of eq:equil, evaluated per cell by an exact
    Gauss-Hermite rule in the whitened variable; f^eq_i = w_i sum_n a^(n):H^(n)(v_i) / n!
    (eq:3rd_order_equilibrium with the weights of eq:feq_i), v_i = c_i / cs, u = s / cs;
  - one step is BGK relaxation (eq:LBE_BGK), the exact-difference body force where given, then
    a periodic shift of every direction plane by np.roll (pull and push agree on a torus).
On 2 x 2 the two opposite neighbours of a cell coincide, so a wrong wrap or a transposed axis
shows up there first. CPU only.
"""
import itertools
from math import factorial

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import _gaussian_hermite_coefficients, _hermite

CS = 1.0 / np.sqrt(3.0)


def _lattice(name):
    d = 2 if name == "D2Q9" else 3
    z, wz = np.polynomial.hermite_e.hermegauss(3)
    wz = wz / wz.sum()
    node = {int(round(v / np.sqrt(3.0))): w for v, w in zip(z, wz)}  # lattice step -> 1-D weight
    cs, ws = [], []
    for c in itertools.product((-1, 0, 1), repeat=d):
        if name == "D3Q19":
            n2 = sum(v * v for v in c)
            if n2 > 2:
                continue
            ws.append({0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}[n2])
        else:
            ws.append(float(np.prod([node[v] for v in c])))
        cs.append(c)
    return np.array(cs, dtype=np.int64), np.array(ws)


def _feq_cell(c, w, a, rho, s):
    """Equilibrium at one cell from the Gaussian's Hermite coefficients (s in lattice units)."""
    coef = _gaussian_hermite_coefficients(a, rho, np.asarray(s) / CS)
    out = np.empty(len(w))
    for i in range(len(w)):
        h = _hermite(c[i] / CS)
        out[i] = w[i] * sum(np.sum(coef[n] * h[n]) / factorial(n) for n in range(4))
    return out


def _moments(c, f):
    rho = f.sum(axis=0)
    mom = np.einsum("ia,i...->a...", c.astype(np.float64), f)
    return rho, mom


def _feq_field(c, w, a, rho, s):
    d = c.shape[1]
    out = np.empty((len(w),) + rho.shape)
    for idx in np.ndindex(rho.shape):
        out[(slice(None),) + idx] = _feq_cell(c, w, a, rho[idx], [s[k][idx] for k in range(d)])
    return out


def _step(c, w, a, tau, f, force):
    """One collide-and-stream step on fields shaped [q][nz][ny][nx] (or [q][ny][nx])."""
    rho, mom = _moments(c, f)
    s = mom / rho
    eq = _feq_field(c, w, a, rho, s)
    post = f + (eq - f) / tau
    if force is not None:
        shifted = s + np.asarray(force).reshape((-1,) + (1,) * rho.ndim) / rho
        post = post + _feq_field(c, w, a, rho, shifted) - eq
    d = c.shape[1]
    axes = tuple(range(d - 1, -1, -1))  # x is the last array axis
    return np.stack([np.roll(post[i], shift=tuple(int(v) for v in c[i]), axis=axes) for i in range(len(w))])


def _to_oracle(name, c, fb):
    """Reorder [q][...] from this file's velocity order to the oracle's, flattened to [q][N]."""
    oc = oracle.lattice(name)[0]
    d = c.shape[1]
    where = {tuple(int(v) for v in ci): i for i, ci in enumerate(c)}
    return np.stack([fb[where[tuple(int(v) for v in oc[j, :d])]].reshape(-1) for j in range(len(oc))])


CASES = [
    ("D2Q9", (2, 2), False),
    ("D2Q9", (3, 2), True),
    ("D3Q19", (3, 3, 3), False),
    ("D3Q19", (2, 3, 2), True),
    ("D3Q27", (3, 3, 3), True),
    ("D3Q27", (2, 2, 2), False),
]


@pytest.mark.parametrize("name,shape,forced", CASES)
def test_oracle_steps_match_bruteforce_transcription(name, shape, forced):
    d = len(shape)
    rng = np.random.default_rng(700 + CASES.index((name, shape, forced)))
    g = rng.normal(size=(d, d))
    q, _ = np.linalg.qr(g)
    a = q @ np.diag(rng.uniform(0.6, 1.4, d)) @ q.T
    a /= np.linalg.det(a) ** (1.0 / d)           # det A = 1 (eq:equil)
    ainv = np.linalg.inv(a)
    tau = 0.8
    fshape = tuple(reversed(shape))               # [nz][ny][nx]
    rho0 = rng.uniform(0.9, 1.1, fshape)
    s0 = rng.uniform(-0.05, 0.05, (d,) + fshape)
    force = rng.uniform(-1e-3, 1e-3, d) if forced else None

    c, w = _lattice(name)
    assert abs(w.sum() - 1.0) < 1e-15
    fb = _feq_field(c, w, a, rho0, s0)
    grid = shape if d == 3 else (shape[0], shape[1], 1)
    fo = oracle.init(name, grid, ainv, rho0.reshape(-1), s0.reshape(d, -1))
    assert np.abs(fo - _to_oracle(name, c, fb)).max() < 1e-14

    nsteps = 5
    for _ in range(nsteps):
        fb = _step(c, w, a, tau, fb, force)
    oracle.steps(name, grid, ainv, tau, fo, nsteps, force=force)
    assert np.abs(fo - _to_oracle(name, c, fb)).max() < 1e-14

    # read-out: rho and the fluid velocity (sum_i f_i c_i + F/2) / rho
    rho, mom = _moments(c, fb)
    s = (mom + (0.0 if force is None else np.asarray(force).reshape((-1,) + (1,) * d) / 2)) / rho
    ro, so = oracle.moments(name, fo, force=force)
    assert np.abs(ro - rho.reshape(-1)).max() < 1e-14
    assert np.abs(np.asarray(so)[:d] - s.reshape(d, -1)).max() < 1e-14
