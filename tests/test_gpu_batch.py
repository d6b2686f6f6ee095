"""GPU tests of the batched update (lbm_batch_*): many independent periodic domains of uneven
sizes, each with its own tensor and tau.

* Every domain of a batch must equal the same domain run alone through the single-grid path,
  bitwise (same per-cell arithmetic), under every schedule.
* Every domain must match the FP64 oracle within the single-grid gates (1e-12 FP64, 1e-5
  FP32) on e(f), e(rho), e(s).
* The 512-domain workload runs at full size in the autotuned schedule and is checked on sampled
  domains against the oracle and on all domains against single-domain runs and conservation.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lbm = pytest.importorskip("paper_2605_27004_amd")

from tests.gpu_common import TOL, _log, _perm  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _small_batch(n=14, seed=11, lattice="D3Q19", edges=(1, 21), u0=0.02):
    """Domains with ragged and degenerate extents (1 .. 21 per axis), random fields."""
    rng = np.random.default_rng(seed)
    d = W.DIMS[lattice]
    doms = []
    for i in range(n):
        shape = tuple(int(v) for v in rng.integers(edges[0], edges[1] + 1, 3))
        if d == 2:
            shape = (shape[0], shape[1], 1)
        if i == 0:
            shape = (1, 1, 1)
        if i == 1:
            shape = (64, 3, 2) if d == 3 else (64, 3, 1)
        rho, s = W.random_fields(shape, d, seed + i, amp_s=u0)
        t = W.random_theta(seed + i) if d == 3 else W.config1_theta()
        doms.append(dict(shape=shape, tensor=t, tensor_kind="theta", tau=float(rng.uniform(0.6, 1.4)), rho=rho, s=s))
    return doms


SCHEDULES = [dict(mode="stepwise", xcd_group=0), dict(mode="stepwise", xcd_group=1),
             dict(mode="persistent", xcd_group=1, wg_per_cu=1, chunk_cells=256, group_bytes=0),
             dict(mode="persistent", xcd_group=0, wg_per_cu=2, chunk_cells=1024, group_bytes=0),
             dict(mode="persistent", xcd_group=1, wg_per_cu=1, chunk_cells=512, group_bytes=1 << 16)]


def _single(dm, lattice, storage, steps, order=3):
    p = lbm.make_params(lattice, storage, dm["shape"], dm["tensor"], dm["tensor_kind"], dm["tau"], order)
    sim = lbm.Simulation(p, dm["rho"], dm["s"])
    sim.step(steps)
    f = sim.f64().cpu().numpy()
    sim.close()
    return f


def _batch_f(b, full, i):
    return b.domain_f64(full, i).cpu().numpy()


@pytest.mark.parametrize("lattice,storage", [("D3Q19", "f64"), ("D3Q19", "f32"), ("D3Q19", "f16"), ("D3Q19", "bf16"),
                                             ("D2Q9", "f32"), ("D3Q27", "f16")])
def test_batch_equals_single_domain_runs_bitwise(lattice, storage):
    """Every batched domain (linear population blocks) against the same domain run alone (row
    blocks): the arithmetic is shared, so the results are bitwise equal in every storage."""
    doms = _small_batch(lattice=lattice, edges=(1, 40) if lattice == "D2Q9" else (1, 21))
    steps = 23
    print(f"[batch] bitwise {lattice} {storage} {len(doms)} domains, {steps} steps", flush=True)
    b = lbm.Batch(lattice, storage, doms)
    b.step(steps)
    full = b.f64()
    torch.cuda.synchronize()
    assert b.t == steps
    for i, dm in enumerate(doms):
        ref = _single(dm, lattice, storage, steps)
        got = _batch_f(b, full, i)
        assert np.array_equal(got, ref), (i, dm["shape"], np.abs(got - ref).max())
    b.close()


@pytest.mark.parametrize("sched", SCHEDULES, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
def test_schedules_are_bitwise_identical(sched):
    doms = _small_batch(n=20, seed=4)
    print(f"[batch] schedule {sched}", flush=True)
    ref = lbm.Batch("D3Q19", "f32", doms)
    ref.step(17)
    want = ref.f64().cpu().numpy()
    ref.close()
    b = lbm.Batch("D3Q19", "f32", doms)
    b.set_schedule(**sched)
    assert b.schedule()["mode"] == sched["mode"]
    b.step(9)
    b.step(8)        # two launches: the parity carries over
    b.status()
    got = b.f64().cpu().numpy()
    b.close()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_matches_oracle(lattice, storage):
    doms = _small_batch(n=8, seed=21, lattice=lattice, edges=(2, 17))
    steps = 40
    print(f"[batch] oracle {lattice} {storage}", flush=True)
    b = lbm.Batch(lattice, storage, doms)
    b.set_schedule(mode="persistent", xcd_group=1, wg_per_cu=1, chunk_cells=512, group_bytes=0)
    b.step(steps)
    rho, s, tot = b.moments()
    full = b.f64()
    torch.cuda.synchronize()
    rho, s = rho.cpu().numpy(), s.cpu().numpy()
    perm = _perm(lattice)
    for i, dm in enumerate(doms):
        f_or, rho_or, s_or = oracle.run(lattice, dm["shape"], dm["tensor"], "theta", dm["tau"], dm["rho"], dm["s"],
                                        steps)
        a, z = b.offsets[i], b.offsets[i + 1]
        e = dict(f=np.abs(_batch_f(b, full, i) - f_or[perm]).max() / np.abs(f_or).max(),
                 rho=np.abs(rho[a:z] - rho_or).max() / np.abs(rho_or).max(),
                 s=np.abs(s[:, a:z] - s_or).max() / 0.02)
        _log(dict(test="batch_oracle", lattice=lattice, storage=storage, domain=i, shape=list(dm["shape"]),
                  steps=steps, **{k: float(v) for k, v in e.items()}))
        for k, v in e.items():
            assert v <= TOL[storage], (i, dm["shape"], k, v)
        # per-domain totals: sum rho and sum rho s of the oracle state
        j_or = [float((rho_or * s_or[a_]).sum()) for a_ in range(s_or.shape[0])]
        assert abs(tot[i][0] - rho_or.sum()) <= TOL[storage] * rho_or.sum()
        for a_ in range(len(j_or)):
            assert abs(tot[i][1 + a_] - j_or[a_]) <= TOL[storage] * rho_or.sum() * 0.02
    b.close()


def test_autotune_leaves_state_and_time_unchanged():
    doms = _small_batch(n=30, seed=8, edges=(8, 40))
    b = lbm.Batch("D3Q19", "f32", doms)
    b.step(5)
    before = b.f64().cpu().numpy()
    sched, ms = b.autotune(trial_steps=4)
    print(f"[batch] autotune chose {sched} at {ms:.4f} ms/step", flush=True)
    assert ms > 0 and b.t == 5
    assert np.array_equal(b.f64().cpu().numpy(), before)
    b.step(3)
    after = b.f64().cpu().numpy()
    b.close()
    ref = lbm.Batch("D3Q19", "f32", doms)
    ref.step(8)
    assert np.array_equal(ref.f64().cpu().numpy(), after)
    ref.close()


def test_spin_limit_failure_path_reports_and_recovers():
    """A zero spin limit makes every wait that finds its domain unfinished give up: the launch
    still ends (each wait polls at most once), lbm_batch_status reports the failure, and a
    fresh batch runs normally afterwards."""
    doms = _small_batch(n=40, seed=2, edges=(16, 40))
    b = lbm.Batch("D3Q19", "f32", doms)
    b.set_schedule(mode="persistent", xcd_group=0, wg_per_cu=1, chunk_cells=256, group_bytes=0)
    lbm.lbm_batch_set_spin_limit(b.b, 0)
    b.step(50)
    failed = False
    try:
        b.status()
    except lbm.LBMError as e:
        failed = e.code == lbm.LBM_ERR_HIP
    print(f"[batch] zero spin limit reported failure: {failed}", flush=True)
    assert failed
    b.status()  # the status word was cleared
    b.close()
    ok = lbm.Batch("D3Q19", "f32", doms)
    ok.set_schedule(mode="persistent", xcd_group=0, wg_per_cu=1, chunk_cells=256, group_bytes=0)
    ok.step(10)
    ok.status()
    ok.close()


def test_batched_workload_full_size():
    """512 D3Q19 domains (edges 16..64), 500 steps, FP32, autotuned schedule: every domain is
    bitwise its single-domain run; sampled domains match the oracle; mass is conserved."""
    wl = W.config5()
    b = lbm.Batch(wl.lattice, "f32", wl.domains)
    _, _, tot0 = b.moments(fields=False)
    sched, ms = b.autotune(trial_steps=10)
    print(f"[batch] full size: {wl.cells} cells, autotune {sched} {ms:.3f} ms/step", flush=True)
    b.step(wl.steps)
    _, s, tot = b.moments()
    full = b.f64()
    torch.cuda.synchronize()
    sizes = [int(np.prod(dm["shape"])) for dm in wl.domains]
    for i in range(len(wl.domains)):
        assert abs(tot[i][0] - tot0[i][0]) <= 1e-9 * tot0[i][0], i
    # all domains against single-domain runs (bitwise)
    for i, dm in enumerate(wl.domains):
        ref = _single(dm, wl.lattice, "f32", wl.steps)
        assert np.array_equal(_batch_f(b, full, i), ref), (i, dm["shape"])
    print("[batch] all 512 domains bitwise equal to single-domain runs", flush=True)
    # sampled domains against the oracle
    rng = np.random.default_rng(0)
    sample = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), *rng.choice(len(sizes), 3, replace=False).tolist()})
    perm = _perm(wl.lattice)
    for i in sample:
        dm = wl.domains[i]
        f_or, rho_or, s_or = oracle.run(wl.lattice, dm["shape"], dm["tensor"], "theta", dm["tau"], dm["rho"],
                                        dm["s"], wl.steps)
        a, z = b.offsets[i], b.offsets[i + 1]
        sd = s[:, a:z].cpu().numpy()
        e = dict(f=np.abs(_batch_f(b, full, i) - f_or[perm]).max() / np.abs(f_or).max(),
                 s=np.abs(sd - s_or).max() / wl.u0)
        print(f"[batch] domain {i} {dm['shape']} tau={dm['tau']:.3f}: {e}", flush=True)
        _log(dict(test="batch_full_size", domain=i, shape=list(dm["shape"]), steps=wl.steps,
                  **{k: float(v) for k, v in e.items()}))
        assert e["f"] <= TOL["f32"] and e["s"] <= TOL["f32"], (i, e)
    b.close()


@pytest.mark.parametrize("sched", SCHEDULES, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
def test_single_domain_batch_equals_grid(sched):
    """A batch of one domain (most of an XCD-placed order is padding; most persistent
    work-groups have no item) is the single-grid run, bit for bit."""
    doms = _small_batch(n=1, seed=30, edges=(20, 33))
    doms[0]["shape"] = (37, 21, 9)
    doms[0]["rho"], doms[0]["s"] = W.random_fields((37, 21, 9), 3, 31, amp_s=0.02)
    b = lbm.Batch("D3Q19", "f32", doms)
    b.set_schedule(**sched)
    b.step(11)
    b.status()
    got = _batch_f(b, b.f64(), 0)
    b.close()
    assert np.array_equal(got, _single(doms[0], "D3Q19", "f32", 11))
