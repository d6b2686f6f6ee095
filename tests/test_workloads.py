"""The seeded input generators: the workloads' stated structure (sizes, value ranges, solid
fractions, periodicity) and reproducibility. No method arithmetic is involved."""
import numpy as np

import workloads as W


def test_headline_tensor_matches_the_stated_recipe():
    t = W.random_theta(0) / W.CS2
    assert np.allclose(t, t.T)
    ev = np.linalg.eigvalsh(t)
    assert np.allclose(np.sort(ev), np.sort([1.1096, 0.8158, 0.6328]), atol=1e-4)
    assert np.allclose(t, [[0.79645, -0.02710, -0.05388], [-0.02710, 0.89102, -0.22746],
                           [-0.05388, -0.22746, 0.87071]], atol=1e-5)


def test_taylor_green_fields():
    wl = W.config2(n=16)
    assert wl.rho.shape == (16 ** 3,) and wl.s.shape == (3, 16 ** 3)
    assert abs(np.abs(wl.s).max() - wl.u0) < 1e-12
    assert abs(wl.s.sum(axis=1)).max() < 1e-12          # zero net momentum


def test_porous_mask_fraction_and_periodicity():
    shape = (48, 40, 36)
    m = W.porous_mask(shape, seed=3)
    frac = m.mean()
    assert 0.40 <= frac < 0.5
    assert np.array_equal(m, W.porous_mask(shape, seed=3))
    assert not np.array_equal(m, W.porous_mask(shape, seed=4))
    # ellipsoids wrap around the faces: solid cells touch both opposite faces somewhere
    g = m.reshape(shape[2], shape[1], shape[0])
    assert g[:, :, 0].any() and g[:, :, -1].any() and g[0].any() and g[-1].any()


def test_obstacle_channel_walls_and_obstacles():
    shape = (64, 32, 24)
    g = W.obstacle_channel(shape, seed=0).reshape(shape[2], shape[1], shape[0])
    assert np.all(g[:, 0, :] == 1) and np.all(g[:, -1, :] == 1)       # y walls
    assert np.all(g[0, :, :] == 1) and np.all(g[-1, :, :] == 1)       # z walls
    interior = g[1:-1, 1:-1, :]
    assert 0.0 < interior.mean() < 0.5                                 # some obstacles, mostly fluid
    g2 = W.obstacle_channel((64, 32, 1), seed=0).reshape(32, 64)
    assert np.all(g2[0] == 1) and np.all(g2[-1] == 1) and 0.0 < g2[1:-1].mean() < 0.5


def test_gradient_and_porous_workloads():
    wl4 = W.config4("D3Q19")
    assert wl4.shape == (128, 128, 128) and wl4.meta["outlet_plane"] == 127 and wl4.meta["checkpoint_every"] == 100
    assert wl4.steps == 2000 and np.allclose(wl4.meta["force"], [1e-5, 0, 0])
    wl3 = W.config3(n=24, steps=10)
    assert wl3.meta["mask"].dtype == np.uint8 and wl3.meta["mask"].shape == (24 ** 3,)
    assert np.allclose(wl3.tensor, W.CS2 * np.diag([1.5, 1.0, 0.5]))
    assert np.all(wl3.s == 0) and np.all(wl3.rho == 1)


def test_batched_workload_sizes():
    wl = W.config5()
    assert len(wl.domains) == W.BATCH_DOMAINS == 512
    assert wl.cells == 32650187
    edges = np.array([d["shape"] for d in wl.domains])
    assert edges.min() == 16 and edges.max() == 64
    taus = np.array([d["tau"] for d in wl.domains])
    assert taus.min() >= 0.55 and taus.max() <= 1.5
