"""Helpers shared by the GPU parity tests: run a workload through the C ABI and through the
oracle, and compare field by field (not a test module)."""
import json
import os

import numpy as np

import oracle

TOL = {"f64": 1e-12, "f32": 1e-5}


def _perm(name):
    """perm[i] = oracle index of the library's canonical direction i."""
    import paper_2605_27004_amd as lbm

    _, _, c, _, _ = lbm.lbm_lattice_info(lbm.LATTICES[name])
    oc, _, _ = oracle.lattice(name)
    idx = {tuple(v): i for i, v in enumerate(oc.tolist())}
    return np.array([idx[tuple(v)] for v in c])


def gpu_run(wl, storage, steps, order=None, shift="rest", block=None, chunks=1):
    import torch

    import paper_2605_27004_amd as lbm

    order = wl.order if order is None else order
    mask = wl.meta.get("mask")
    force = wl.meta.get("force")
    p = lbm.make_params(wl.lattice, storage, wl.shape, wl.tensor, wl.tensor_kind, wl.tau, order, shift=shift,
                        force=force, masked=mask is not None)
    sim = lbm.Simulation(p, wl.rho, wl.s, mask=mask)
    if block:
        sim.set_launch(*block)
    left = steps
    for _ in range(chunks):
        k = left // chunks if chunks > 1 else left
        sim.step(k)
        left -= k
    sim.step(left)
    rho, s, tot = sim.moments()
    f = sim.f64()
    torch.cuda.synchronize()
    out = dict(f=f.cpu().numpy(), rho=rho.cpu().numpy(), s=s.cpu().numpy(), totals=tot, t=sim.t, sim=sim)
    return out


def oracle_run(wl, steps, order=None):
    order = wl.order if order is None else order
    f, rho, s = oracle.run(wl.lattice, wl.shape, wl.tensor, wl.tensor_kind, wl.tau, wl.rho, wl.s, steps, order,
                           mask=wl.meta.get("mask"), force=wl.meta.get("force"))
    return dict(f=f[_perm(wl.lattice)], rho=rho, s=s)


def errors(g, o, u0):
    """e(f), e(rho) relative to the reference maxima; e(s) relative to u0, the initial velocity
    amplitude, or to the reference's final max |s| for flows started at rest (u0 = None)."""
    scale = u0 if u0 else np.abs(o["s"]).max()
    return dict(f=np.abs(g["f"] - o["f"]).max() / np.abs(o["f"]).max(),
                rho=np.abs(g["rho"] - o["rho"]).max() / np.abs(o["rho"]).max(),
                s=np.abs(g["s"] - o["s"]).max() / scale)


def check(wl, storage, steps, order=None, **kw):
    print(f"[parity] {wl.lattice} {wl.shape} {storage} order={order or wl.order} steps={steps}", flush=True)
    g = gpu_run(wl, storage, steps, order, **kw)
    o = oracle_run(wl, steps, order)
    e = errors(g, o, wl.u0)
    print(f"[parity] errors {e}", flush=True)
    _log(dict(lattice=wl.lattice, shape=list(wl.shape), storage=storage, order=order or wl.order, steps=steps,
              shift=kw.get("shift", "rest"), reference="oracle", **{k: float(v) for k, v in e.items()}))
    assert g["t"] == steps
    for k, v in e.items():
        assert v <= TOL[storage], (k, v)
    return g, o, e


def _log(rec):
    """Append one error record to $PARITY_LOG (JSON lines) when it is set."""
    path = os.environ.get("PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(rec) + "\n")


