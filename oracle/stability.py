"""Linear stability of the BGK update at rest, from the FP64 oracle's own equilibrium.

TEST INFRASTRUCTURE (like the rest of ``oracle/``): used by tests and by the screening script
below that writes the stored per-domain redraw table of the batched workload.

Around the rest state (rho = 1, s = 0) one step of eq:LBE_BGK is linear in the perturbation.
For a plane wave exp(i k.x) it is the q x q matrix

    M(k) = E(k) (I + omega (J - I)),   E(k) = diag(exp(-i k.c_i)),

where J_ij = d f^eq_i / d f_j is the equilibrium's Jacobian through rho = sum f and
rho s = sum f c (at rest: J_ij = d f^eq_i/d rho + sum_a d f^eq_i/d s_a c_ja), and E is push
streaming f_i(x + c_i) <- f*_i(x). The update is linearly stable when no eigenvalue of any
M(k) exceeds 1 in modulus. J comes from ``oracle.feq``: f^eq is linear in rho at s = 0, and a
cubic polynomial in s along any line, so a two-step Richardson central difference gives its
s-derivative exactly up to rounding.

Run as a script to (re)write the batched workload's redraw table:

    python -m oracle.stability --write
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

from . import feq, lattice, tensor_to_ainv


def jacobian_at_rest(name: str, ainv, order: int = 3, h: float = 1e-3) -> np.ndarray:
    """J_ij = d f^eq_i / d f_j at rho = 1, s = 0 (oracle velocity order)."""
    c, w, _ = lattice(name)
    d = ainv.shape[0]
    q = c.shape[0]
    dr = feq(name, ainv, 1.0, np.zeros(d), order)           # f^eq(rho, 0) = rho r_i
    ds = np.zeros((q, d))
    for a in range(d):
        e = np.zeros(d)
        e[a] = 1.0

        def central(step):
            return (feq(name, ainv, 1.0, step * e, order) - feq(name, ainv, 1.0, -step * e, order)) / (2 * step)

        # exact for a cubic: D(h) = f' + h^2 f'''/6, D(2h) = f' + 4 h^2 f'''/6
        ds[:, a] = (4.0 * central(h) - central(2.0 * h)) / 3.0
    return dr[:, None] + ds @ c[:, :d].T


def wave_vectors(d: int, L: int) -> np.ndarray:
    """All k = 2 pi m / L, m in {0..L-1}^d, as [L^d, 3]."""
    m = np.stack(np.meshgrid(*([np.arange(L)] * d), indexing="ij"), -1).reshape(-1, d)
    k = np.zeros((m.shape[0], 3))
    k[:, :d] = 2.0 * np.pi * m / L
    return k


def spectral_radius(name: str, ainv, tau: float, order: int = 3, L: int = 16) -> float:
    """max over the wave vectors of an L^d periodic box of the largest |eigenvalue| of M(k)."""
    c, _, _ = lattice(name)
    q = c.shape[0]
    d = ainv.shape[0]
    J = jacobian_at_rest(name, ainv, order)
    C = np.eye(q) + (J - np.eye(q)) / tau
    k = wave_vectors(d, L)
    phase = np.exp(-1j * (k @ c.T.astype(np.float64)))      # [nk, q]
    M = phase[:, :, None] * C[None, :, :]
    return float(np.abs(np.linalg.eigvals(M)).max())


STABLE_MARGIN = 1e-9  # |lambda| <= 1 + margin counts as stable (conserved modes sit at 1)


def is_stable(name: str, tensor, kind: str, tau: float, order: int = 3, L: int = 16) -> bool:
    d = 2 if name == "D2Q9" else 3
    ainv = tensor_to_ainv(np.asarray(tensor)[:d, :d], kind, d)
    return spectral_radius(name, ainv, tau, order, L) <= 1.0 + STABLE_MARGIN


def screen_batched(ndomains: int, seed_base: int, L: int = 16, max_redraws: int = 20) -> dict:
    """Redraw counts that make every domain of the batched workload linearly stable."""
    import workloads as W

    redraws = {}
    for i in range(ndomains):
        r = 0
        while True:
            dom = W.batched_domain(i, seed_base, redraw=r)
            if is_stable("D3Q19", dom["tensor"], "theta", dom["tau"], L=L):
                break
            r += 1
            if r > max_redraws:
                raise RuntimeError(f"domain {i}: no stable draw in {max_redraws} redraws")
        if r:
            redraws[str(i)] = r
    return redraws


def main(argv):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import workloads as W

    out = {"lattice": "D3Q19", "ndomains": W.BATCH_DOMAINS, "seed_base": W.BATCH_SEED_BASE, "scan_box": 16,
           "rule": "domain i redraws (theta, tau) from its own stream redraws[i] times",
           "redraws": screen_batched(W.BATCH_DOMAINS, W.BATCH_SEED_BASE)}
    text = json.dumps(out, indent=1, sort_keys=True)
    print(text)
    if "--write" in argv:
        with open(W.BATCH_REDRAW_FILE, "w") as fh:
            fh.write(text + "\n")


if __name__ == "__main__":
    main(sys.argv[1:])
