"""The App. C sampler on the GPU, in distribution, at sharp and eccentric
lobes (test suite S).

Every vertex's record holds the lobe under test with mixture weight 1; the
other three lobes' log(A/K) is -300, so their weights underflow to zero and
`nasg_sample` draws from the one lobe. 2^20 GPU samples are histogrammed in
(mu, phi) of the lobe's frame (mu bins at the quantiles of the vMFs of
sharpness lambda and lambda (1 + eps + a), 16 azimuth bins) and compared
by chi-square with the quadrature of the normalised lobe exp(log G - log K) over each bin (eq.
NASG with App. A's epsilon, App. B's normaliser, from the oracle), as the
oracle's own sampler is tested in `tests/test_oracle_pins.py`. The
per-sample parity of the same sampler against the extended-precision
oracle is in `tests/test_gpu_edges.py`; this checks that the stable forms
keep the distribution where lambda and a are large.
"""

import math

import numpy as np
import pytest
import scipy.stats as ss
import torch

from oracle import nasg as onasg
from tests import quad
from tests.helpers import bk9_to_rec, make_guide, to_dev

F64 = torch.float64
B = 1 << 20
K = 4   # the record kernels of the c1 guide


def _frame(rng):
    z = rng.normal(size=3)
    z /= np.linalg.norm(z)
    t = rng.normal(size=3)
    x = t - (t @ z) * z
    x /= np.linalg.norm(x)
    return z, x, np.cross(z, x)


def _mu_breaks(mu_lo, mu_hi, n=24):
    """Quadrature breaks over [mu_lo, mu_hi], geometric in 1 - mu (the lobe
    falls off like exp(-2 lam p (1 - mu)), far faster than a bin is wide)."""
    t_lo, t_hi = 1.0 - mu_hi, 1.0 - mu_lo
    if t_lo <= 0.0:
        t = np.concatenate([[0.0], np.geomspace(t_hi * 1e-10, t_hi, n)])
    else:
        t = np.geomspace(t_lo, t_hi, n)
    return np.sort(1.0 - t)


def _mu_edges(lam, a, eps):
    """Bin edges in mu at the quantiles of the vMF of sharpness lam and of
    lam (1 + eps + a), the lobe's sharpness across and along its x axis."""
    q = np.linspace(0, 1, 13)[1:-1]
    edges = [[-1.0, 1.0]]
    for s in sorted({lam, lam * (1.0 + eps + a)}):
        edges.append(1 + np.log1p(-q * -np.expm1(-2 * s)) / s)   # 1 - (vMF quantile of 1 - mu)
    return np.unique(np.concatenate(edges))


def _bin_probabilities(z, x, y, lam, a, eps, mu_e, ph_e):
    """Quadrature of exp(log G - log K) over each (mu, phi) bin."""
    T = lambda t: torch.tensor(t, dtype=F64)
    logk = float(onasg.log_normaliser(T(lam), T(a), eps))
    prob = np.zeros((len(mu_e) - 1, len(ph_e) - 1))
    for i in range(len(mu_e) - 1):
        mb = _mu_breaks(mu_e[i], mu_e[i + 1])
        for j in range(len(ph_e) - 1):
            pb = np.linspace(ph_e[j], ph_e[j + 1], 13)
            vv, ww = quad.sphere_nodes(z, x, y, mb, pb, 12)
            lg = onasg.lobe_log_g(T(vv.reshape(-1, 3)), T(z), T(x), T(lam), T(a), eps).numpy()
            prob[i, j] = (np.exp(lg - logk).reshape(ww.shape) * ww).sum()
    return prob, logk


@pytest.mark.gpu
@pytest.mark.parametrize("lam,a,eps,seed", [(2.0, 3.0, 0.0, 1), (200.0, 0.0, 0.0, 2), (1000.0, 50.0, 0.0, 3),
                                            (5000.0, 300.0, 0.0, 4), (100.0, 300.0, 0.3, 5), (1e5, 1e3, 0.0, 6)])
def test_sample_distribution(lam, a, eps, seed):
    rng = np.random.default_rng(seed)
    z, x, y = _frame(rng)
    mu_e = _mu_edges(lam, a, eps)
    ph_e = np.linspace(0, 2 * math.pi, 17)
    prob, logk = _bin_probabilities(z, x, y, lam, a, eps, mu_e, ph_e)
    assert abs(prob.sum() - 1) < 1e-6, prob.sum()

    # one 64-vertex record tile, repeated over the batch
    tile = np.empty((64, K, 9))
    tile[:, 0] = [*z, *x, lam, a, -logk]
    tile[:, 1:] = [*z, *x, 1.0, 0.0, -300.0]
    rec = to_dev(np.tile(bk9_to_rec(tile, K), B // 64))
    xi = to_dev(np.ascontiguousarray(rng.random((4, B), dtype=np.float32)))
    g, _ = make_guide("c1_f32", eps=eps, max_batch=B)
    d_gpu, _ = g.sample(rec, xi)
    v = d_gpu.cpu().numpy().T.astype(np.float64)
    g.close()
    assert np.isfinite(v).all()

    # mu from the float64-normalised direction, 1 - mu = |v - z|^2 / 2 without
    # cancellation: the sharpest bins are ~6e-8 wide in mu, below the
    # float32 direction's |v| - 1
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    mu = 1.0 - 0.5 * ((v - z) ** 2).sum(1)
    ph = np.mod(np.arctan2(v @ y, v @ x), 2 * math.pi)
    counts, _, _ = np.histogram2d(mu, ph, bins=[mu_e, ph_e])
    exp_c = prob.ravel() * B
    obs = counts.ravel()
    keep = exp_c >= 5
    chi2 = (((obs[keep] - exp_c[keep]) ** 2) / exp_c[keep]).sum()
    rest = exp_c[~keep].sum()
    if (~keep).any() and rest > 5:
        chi2 += (obs[~keep].sum() - rest) ** 2 / rest
    dof = int(keep.sum()) - 1
    assert ss.chi2.sf(chi2, dof) > 1e-4, (chi2, dof)
