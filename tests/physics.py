"""Analysis helpers for the physics pins: Fourier projections, decay-rate fits and the
linearised Chapman-Enskog operators (the paper's closed form and the lattice's own).

Nothing here evaluates the equilibrium itself; where the lattice third moment is needed it
is obtained by differentiating an equilibrium function supplied by the caller.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import curve_fit

CS2 = 1.0 / 3.0


def coords(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)]).astype(np.float64)


def kvector(shape, modes):
    """Wave vector 2 pi m_a / n_a for integer modes (m_x, m_y[, m_z])."""
    m = list(modes) + [0] * (3 - len(modes))
    return np.array([2.0 * np.pi * m[a] / shape[a] for a in range(3)])


def project(field, shape, k):
    """Complex amplitude a with field ~ Re(a exp(i k.x)) for one Fourier mode."""
    x = coords(shape)
    ph = np.exp(-1j * (k @ x))
    return 2.0 * np.mean(field * ph)


def log_slope(t, amp):
    """Least-squares slope of log(amp) against t (minus the decay rate)."""
    t = np.asarray(t, dtype=np.float64)
    y = np.log(np.abs(np.asarray(amp)))
    a = np.vstack([t, np.ones_like(t)]).T
    return float(np.linalg.lstsq(a, y, rcond=None)[0][0])


def fit_exp(t, y):
    """curve_fit of a exp(-w t) (Sec. 4's fit function); returns w."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    p, _ = curve_fit(lambda tt, a, w: a * np.exp(-w * tt), t, y, p0=(y[0], 1e-3), maxfev=20000)
    return float(p[1])


def fit_damped_cos(t, y, w0):
    """curve_fit of a exp(-g t) cos(w t + phi); returns (w, g)."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)

    def model(tt, a, g, w, ph):
        return a * np.exp(-g * tt) * np.cos(w * tt + ph)

    p, _ = curve_fit(model, t, y, p0=(y[0], 1e-3, w0, 0.0), maxfev=50000, xtol=1e-14, ftol=1e-14)
    return float(p[2]), float(p[1])


def third_moment_derivative(feq_fn, c, d):
    """T[a,b,g,e] = sum_i c_ia c_ib c_ig d f^eq_i / d s_e at rho = 1, s = 0 (central difference;
    f^eq is a cubic in s, so the error is O(h^2) of the cubic coefficients only)."""
    h = 1e-5
    q = c.shape[0]
    dfeq = np.zeros((q, d))
    for e in range(d):
        sp = np.zeros(d)
        sm = np.zeros(d)
        sp[e] = h
        sm[e] = -h
        dfeq[:, e] = (feq_fn(1.0, sp) - feq_fn(1.0, sm)) / (2 * h)
    cc = c[:, :d].astype(np.float64)
    return np.einsum("ia,ib,ig,ie->abge", cc, cc, cc, dfeq)


def paper_third_moment_derivative(ainv, d):
    """Closed form of the same tensor from App. E (eq:mom_diff1): cs^2 (A^-1_ab d_ge + ...)."""
    ai = np.asarray(ainv)[:d, :d]
    dl = np.eye(d)
    return CS2 * (np.einsum("ab,ge->abge", ai, dl) + np.einsum("bg,ae->abge", ai, dl)
                  + np.einsum("ga,be->abge", ai, dl))


def ce_operator(T, ainv, tau, k, d):
    """Linearised macroscopic operator around rest for a plane wave exp(i k.x):
    d/dt (rho^, s^) = M (rho^, s^), with
      d rho^/dt = -i k.s^,
      d s^_a/dt = -i cs^2 (A^-1 k)_a rho^ - (tau - 1/2) k_b k_g (T_abge - cs^2 A^-1_ab d_ge) s^_e
    (eq:CE3 with eq:CE4 linearised; T is the equilibrium third moment's derivative in s)."""
    ai = np.asarray(ainv)[:d, :d]
    kk = np.asarray(k)[:d]
    m = np.zeros((1 + d, 1 + d), dtype=complex)
    m[0, 1:] = -1j * kk
    m[1:, 0] = -1j * CS2 * (ai @ kk)
    visc = np.einsum("b,g,abge->ae", kk, kk, T - CS2 * np.einsum("ab,ge->abge", ai, np.eye(d)))
    m[1:, 1:] = -(tau - 0.5) * visc
    return m


def shear_modes(T, ainv, tau, k, d):
    """Eigenpairs of the non-propagating (shear) modes: |Im lambda| < cs |k| / 2."""
    m = ce_operator(T, ainv, tau, k, d)
    lam, vec = np.linalg.eig(m)
    kn = np.linalg.norm(np.asarray(k)[:d])
    sel = [i for i in range(len(lam)) if abs(lam[i].imag) < 0.5 * np.sqrt(CS2) * kn]
    return lam[sel], vec[:, sel]
