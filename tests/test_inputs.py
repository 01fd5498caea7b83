"""The seeded input recipes: shapes, statistics, determinism, Morton order."""
import numpy as np

from paper_1208_3444_amd import inputs


def test_lattice_gaussian_shape_and_stats():
    x, psi, d = inputs.lattice_gaussian(16, 0.02, 1)
    assert x.shape == (3, 4096) and d == 1 / 16
    assert abs(psi.std() / (0.02 * d) - 1) < 0.03
    q = x - psi
    # cell-centred lattice: every coordinate is (i + 1/2) d
    frac = (q / d - 0.5) % 1.0
    assert np.allclose(np.minimum(frac, 1.0 - frac), 0.0, atol=1e-12)
    assert np.allclose(q.mean(axis=1), 0.5)


def test_morton_order_is_compact_and_deterministic():
    x1, _, _ = inputs.lattice_gaussian(8, 0.0, 7)
    x2, _, _ = inputs.lattice_gaussian(8, 0.0, 7)
    assert np.array_equal(x1, x2)
    # each aligned block of 8 consecutive particles is one 2x2x2 cell
    blocks = x1.reshape(3, -1, 8)
    ext = blocks.max(axis=2) - blocks.min(axis=2)
    assert np.allclose(ext, 1 / 8)


def test_grf_rms_and_irrotational():
    x, psi, d = inputs.lattice_grf(16, 0.1, 2)
    assert abs(np.sqrt(np.mean(psi ** 2)) - 0.1 * d) < 1e-12
    assert abs(psi.mean()) < 1e-12
    f = inputs.grf_displacement(16, 1.0, np.random.Generator(np.random.PCG64(0)))
    fk = [np.fft.fftn(f[i]) for i in range(3)]
    k = np.fft.fftfreq(16) * 16
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    curl_z = KX * fk[1] - KY * fk[0]
    assert np.abs(curl_z).max() < 1e-9 * np.abs(fk[0]).max()


def test_workloads():
    w = inputs.eds_lattice()
    assert w.N == 4096 and w.n_steps == 64 and w.eps == 0.05 / 16
    w = inputs.lcdm_grf(8, n_steps=10)
    assert w.N == 512 and w.cosmo["Om_L"] == 0.7
    e = inputs.ragged_ensemble(n_boxes=8, n_steps=3)
    sizes = np.diff(e.box_offsets)
    assert np.all((sizes >= 512) & (sizes <= 8192))
    assert e.x.shape == (3, e.box_offsets[-1])
    assert np.allclose(e.box_eps, 0.05 * sizes ** (-1 / 3))
    s = inputs.precision_sweep(16, n_targets=100)
    assert len(np.unique(s.extra["targets"])) == 100
