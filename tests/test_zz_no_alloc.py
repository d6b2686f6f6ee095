"""lbm_moments_static (the moments read-out for callers that cannot allocate: its reduction uses the
library's static device array) against lbm_moments (the context's scratch) through the C ABI:
rho, s and the FP64 totals bit for bit, on consecutive calls whose grids shrink and grow, so a
call never sees stale partials of a larger one."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lbm = pytest.importorskip("paper_2605_27004_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sim(lattice, storage, shape, seed, masked=False):
    d = W.DIMS[lattice]
    rho, s = W.random_fields(shape, d, seed)
    t = W.config1_theta() if d == 2 else W.random_theta(seed)
    n = int(np.prod(shape))
    mask = (np.random.default_rng(seed).uniform(size=n) < 0.15).astype(np.uint8) if masked else None
    p = lbm.make_params(lattice, storage, shape, t, "theta", 0.8, masked=masked,
                        force=None if not masked else [1e-4, 0.0, 0.0][:d])
    sim = lbm.Simulation(p, rho, s, mask=mask)
    sim.step(7)
    return sim


def _both(sim):
    dev = sim.device
    ra = torch.empty(sim.n, dtype=torch.float64, device=dev)
    sa = torch.empty((sim.d, sim.n), dtype=torch.float64, device=dev)
    ta = lbm.lbm_moments(sim.ctx, ra, sa, True)
    rb = torch.full((sim.n,), -1.0, dtype=torch.float64, device=dev)
    sb = torch.full((sim.d, sim.n), -1.0, dtype=torch.float64, device=dev)
    tb = lbm.lbm_moments_static(sim.ctx, rb, sb, True)
    torch.cuda.synchronize()
    return (ra, sa, ta), (rb, sb, tb)


def test_static_moments_match_context_moments():
    big = _sim("D3Q27", "f32", (200, 33, 17), 3, masked=True)    # 561 row tiles: 561 work-groups
    small = _sim("D2Q9", "f64", (40, 30, 1), 4)                   # 8 work-groups
    larger = _sim("D3Q19", "f32", (256, 64, 40), 5)               # 2,560 tiles: the 2,048-group cap
    for sim in (big, small, big, larger, small):
        (ra, sa, ta), (rb, sb, tb) = _both(sim)
        print(f"[noalloc] {sim.params.nx}x{sim.params.ny}x{sim.params.nz} totals {tb}", flush=True)
        assert torch.equal(ra, rb) and torch.equal(sa, sb)
        assert ta == tb
    # fields only: nothing but kernels enqueued
    rb = torch.empty(small.n, dtype=torch.float64, device=small.device)
    assert lbm.lbm_moments_static(small.ctx, rb, None, False) is None
    ra = torch.empty_like(rb)
    lbm.lbm_moments(small.ctx, ra, None, False)
    torch.cuda.synchronize()
    assert torch.equal(ra, rb)
    for sim in (big, small, larger):
        sim.close()


def test_static_moments_report_nonfinite_state():
    """The error path is the same as lbm_moments': a NaN density gives LBM_ERR_NONFINITE."""
    shape = (8, 8, 1)
    rho, s = W.random_fields(shape, 2, 2)
    rho = rho.copy()
    rho[5] = np.nan
    p = lbm.make_params("D2Q9", "f64", shape, W.config1_theta(), "theta", 0.8)
    sim = lbm.Simulation(p, rho, s)
    sim.step(2)
    with pytest.raises(lbm.LBMError) as ei:
        lbm.lbm_moments_static(sim.ctx, None, None, True)
    assert ei.value.code == lbm.LBM_ERR_NONFINITE
    sim.close()
