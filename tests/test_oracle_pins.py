"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: a closed
form the paper derives, a textbook or library routine the method reduces to,
a printed inverse map, a limit the paper states, or finite differences.
"""

import math

import numpy as np
import pytest
import scipy.stats as ss
import torch
from scipy.spatial.transform import Rotation

from oracle import mlp, nasg, train
from tests import quad

F64 = torch.float64


def random_frame(rng):
    R = Rotation.random(random_state=rng).as_matrix()
    return R[:, 2], R[:, 0], R[:, 1]     # z, x, y (right-handed: y = z x x)


def lobe_integral(lam, a, eps, z, x, y):
    """Integral of G over S^2 by graded Gauss-Legendre quadrature."""
    v, w = quad.sphere_nodes(z, x, y)
    M, P, _ = v.shape
    vt = torch.tensor(v.reshape(-1, 3))
    lg = nasg.lobe_log_g(vt, torch.tensor(z), torch.tensor(x),
                         torch.tensor(lam, dtype=F64), torch.tensor(a, dtype=F64), eps)
    return float((torch.exp(lg).numpy().reshape(M, P) * w).sum())


# (lambda, a, eps): includes the four parameter sets of the NASG figure in Sec. 3.2
NORM_CASES = [
    (1.0, 0.0, 0.0), (10.0, 0.0, 0.0), (10.0, 10.0, 0.0), (25.0, 100.0, 0.0),
    (1e-3, 0.0, 0.0), (1e-3, 5.0, 0.0), (0.5, 0.5, 0.0), (3.0, 5.0, 0.3),
    (1e3, 2.0, 0.0), (1e4, 0.0, 0.0), (1e4, 1e3, 0.0), (50.0, 1e3, 0.0),
    (0.01, 2.0, 0.3), (200.0, 20.0, 0.3),
]


@pytest.mark.parametrize("lam,a,eps", NORM_CASES)
def test_normaliser_matches_quadrature(lam, a, eps):
    """Eq. "K for NASG" / App. B: the closed form equals the integral of G."""
    rng = np.random.default_rng(int(lam * 7 + a * 3 + eps * 11) % 2**31)
    z, x, y = random_frame(rng)
    num = lobe_integral(lam, a, eps, z, x, y)
    closed = math.exp(float(nasg.log_normaliser(torch.tensor(lam, dtype=F64),
                                                torch.tensor(a, dtype=F64), eps)))
    assert abs(num / closed - 1.0) < 1e-10, (num, closed)


def test_closed_form_by_hand():
    """The normaliser written out for lambda = 1, a = 3, eps = 0:
    K = 2 pi (1 - e^-2) / (1 * sqrt(4)) = pi (1 - e^-2)."""
    k = math.exp(float(nasg.log_normaliser(torch.tensor(1.0, dtype=F64),
                                           torch.tensor(3.0, dtype=F64))))
    assert abs(k - math.pi * (1 - math.exp(-2))) < 1e-14


@pytest.mark.parametrize("lam", [0.3, 1.0, 10.0, 200.0, 1e4])
def test_isotropic_case_is_vmf(lam):
    """a = 0, eps = 0: NASG is the spherical Gaussian and the normalised lobe
    is the von Mises-Fisher density (Sec. 3.1, eq. SG integral; Sec. 3.2)."""
    rng = np.random.default_rng(5)
    z, x, y = random_frame(rng)
    v = rng.standard_normal((200, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # directions close to the axis as well, where a sharp lobe lives
    near = z + rng.standard_normal((200, 3)) * (3.0 / max(lam, 1.0))
    near /= np.linalg.norm(near, axis=1, keepdims=True)
    v = np.concatenate([v, near])
    lobes = nasg.Lobes(z=torch.tensor(z).expand(len(v), 1, 3), x=torch.tensor(x).expand(len(v), 1, 3),
                       y=torch.tensor(y).expand(len(v), 1, 3),
                       lam=torch.full((len(v), 1), lam, dtype=F64), a=torch.zeros(len(v), 1, dtype=F64),
                       log_A=torch.zeros(len(v), 1, dtype=F64),
                       log_K=nasg.log_normaliser(torch.full((len(v), 1), lam, dtype=F64),
                                                 torch.zeros(len(v), 1, dtype=F64)),
                       eps=0.0)
    got = nasg.mixture_log_pdf(torch.tensor(v), lobes).numpy()
    ref = ss.vonmises_fisher(mu=z, kappa=lam).logpdf(v)
    assert np.max(np.abs(got - ref)) < 1e-9
    # and the unnormalised lobe is exp(lam (v.z - 1))
    lg = nasg.lobe_log_g(torch.tensor(v), torch.tensor(z), torch.tensor(x),
                         torch.tensor(lam, dtype=F64), torch.tensor(0.0, dtype=F64)).numpy()
    assert np.max(np.abs(lg - lam * (v @ z - 1.0))) < 1e-9 * max(1.0, lam)


@pytest.mark.parametrize("lam,a", [(1.0, 0.0), (10.0, 10.0), (25.0, 100.0), (0.2, 3.0)])
def test_point_values_and_limits(lam, a):
    """G(z) = 1, G(-z) = 0 (eq. NASG). Toward -z along the y meridian G tends
    to e^{-2 lam} when eps = 0, along other meridians to 0 (footnote of
    Sec. 3.2); with eps > 0 every meridian gives 0 (App. A)."""
    rng = np.random.default_rng(11)
    z, x, y = random_frame(rng)
    T = lambda t: torch.tensor(t, dtype=F64)
    lg = lambda v, e=0.0: float(nasg.lobe_log_g(T(v), T(z), T(x), T(lam), T(a), e))
    # exactly at the poles (an axis-aligned frame makes v.z exactly +-1)
    ez, ex = np.array([0, 0, 1.0]), np.array([1.0, 0, 0])
    at = lambda v: float(nasg.lobe_log_g(T(v), T(ez), T(ex), T(lam), T(a)))
    assert at(ez) == 0.0
    assert at(-ez) == -math.inf
    assert abs(lg(z)) < 1e-12
    d = 1e-4
    along_y = math.sin(math.pi - d) * y + math.cos(math.pi - d) * z
    assert abs(math.exp(lg(along_y)) - math.exp(-2 * lam)) < 1e-5 * math.exp(-2 * lam) + 1e-12
    if a > 0:
        along_x = math.sin(math.pi - d) * x + math.cos(math.pi - d) * z
        assert math.exp(lg(along_x)) < 1e-3 * math.exp(-2 * lam) + 1e-300
    # eps > 0: along the y meridian G ~ e^{-2 lam} u^eps with u = (1 - cos d)/2 -> 0
    u = (1 - math.cos(d)) / 2
    g_eps = math.exp(lg(along_y, 0.3))
    assert g_eps < 1e-2 * math.exp(-2 * lam)
    assert abs(g_eps / (math.exp(-2 * lam) * u ** 0.3) - 1) < 1e-3


def test_euler_frame_is_zyz_rotation():
    """Sec. 4.1: z and x are the images of e_z and e_x under the rotation with
    Euler angles (phi, theta, tau); y = z x x is then the image of e_y."""
    rng = np.random.default_rng(3)
    ang = rng.uniform([0, 0, 0], [2 * math.pi, math.pi, 2 * math.pi], size=(64, 3))
    phi, th, tau = ang[:, 0], ang[:, 1], ang[:, 2]
    T = torch.tensor
    z, x, y = nasg.euler_frame(T(np.cos(th)), T(np.sin(th)), T(np.cos(phi)), T(np.sin(phi)),
                               T(np.cos(tau)), T(np.sin(tau)))
    R = Rotation.from_euler("ZYZ", ang)
    assert np.allclose(z.numpy(), R.apply([0, 0, 1.0]), atol=1e-14)
    assert np.allclose(x.numpy(), R.apply([1.0, 0, 0]), atol=1e-14)
    assert np.allclose(y.numpy(), R.apply([0, 1.0, 0]), atol=1e-14)


def test_decode_follows_decoding_table():
    """Tab. decoding: sigmoid(s0) * 2 - 1, exp(s1), softmax(A); raw order
    parameter-major, lobe-minor; the frame is orthonormal."""
    rng = np.random.default_rng(8)
    K = 3
    raw = rng.standard_normal((5, 8 * K)) * 2
    lob = nasg.decode(torch.tensor(raw), K)
    r = raw.reshape(5, 8, K)
    d = 2.0 / (1.0 + np.exp(-r[:, :5])) - 1.0
    assert np.allclose(lob.z[..., 2].numpy(), d[:, 0], atol=1e-15)
    n_phi = np.hypot(d[:, 1], d[:, 2])
    assert np.allclose(lob.z[..., 0].numpy(), d[:, 2] / n_phi * np.sqrt(1 - d[:, 0] ** 2), atol=1e-14)
    assert np.allclose(lob.lam.numpy(), np.exp(r[:, 5]), rtol=1e-14)
    assert np.allclose(lob.a.numpy(), np.exp(r[:, 6]), rtol=1e-14)
    e = np.exp(r[:, 7] - r[:, 7].max(1, keepdims=True))
    assert np.allclose(np.exp(lob.log_A.numpy()), e / e.sum(1, keepdims=True), atol=1e-15)
    for u, w in [(lob.z, lob.z), (lob.x, lob.x), (lob.y, lob.y)]:
        assert np.allclose((u * w).sum(-1).numpy(), 1.0, atol=1e-14)
    assert np.allclose((lob.z * lob.x).sum(-1).numpy(), 0.0, atol=1e-14)
    # the clamp reading
    big = np.zeros((1, 8 * K)); big[0, 5 * K] = 40.0; big[0, 6 * K] = -40.0
    lb = nasg.decode(torch.tensor(big), K)
    assert float(lb.lam[0, 0]) == pytest.approx(math.exp(15.0))
    assert float(lb.a[0, 0]) == pytest.approx(math.exp(-15.0))


def test_mixture_integrates_to_one():
    """D = sum_k A_k G_k / K_k is a density (Sec. 3.1)."""
    rng = np.random.default_rng(21)
    K = 5
    raw = rng.standard_normal((1, 8 * K))
    raw[0, 5 * K:6 * K] = np.log([0.5, 2.0, 8.0, 20.0, 1.0])
    lob = nasg.decode(torch.tensor(raw), K)
    # product Gauss-Legendre grid in global coordinates, fine enough for lam <= 20
    mu, wm = quad.gl_panels(np.linspace(-1, 1, 161), 16)
    ph, wp = quad.gl_panels(np.linspace(0, 2 * math.pi, 321), 16)
    r = np.sqrt(1 - mu ** 2)
    v = np.stack(np.broadcast_arrays(r[:, None] * np.cos(ph)[None], r[:, None] * np.sin(ph)[None],
                                     mu[:, None] + 0 * ph[None]), -1).reshape(-1, 3)
    lq = nasg.mixture_log_pdf(torch.tensor(v), nasg.Lobes(
        z=lob.z.expand(len(v), K, 3), x=lob.x.expand(len(v), K, 3), y=lob.y.expand(len(v), K, 3),
        lam=lob.lam.expand(len(v), K), a=lob.a.expand(len(v), K), log_A=lob.log_A.expand(len(v), K),
        log_K=lob.log_K.expand(len(v), K), eps=0.0))
    total = (np.exp(lq.numpy()).reshape(len(mu), len(ph)) * wm[:, None] * wp[None, :]).sum()
    # the eps = 0 lobes are discontinuous at -z, which this ungraded grid
    # resolves only to about 1e-8
    assert abs(total - 1.0) < 1e-6


def _single_lobe_samples(lam, a, eps, n, seed):
    rng = np.random.default_rng(seed)
    z, x, y = random_frame(rng)
    xi = rng.random((n, 3))
    T = lambda t: torch.tensor(t, dtype=F64)
    v = nasg.sample_lobe(T(z).expand(n, 3), T(x).expand(n, 3), T(y).expand(n, 3),
                         T(np.full(n, lam)), T(np.full(n, a)),
                         T(xi[:, 0]), T(xi[:, 1]), T(xi[:, 2]), eps).numpy()
    return v, xi, (z, x, y)


@pytest.mark.parametrize("lam,a,eps", [(1.0, 0.0, 0.0), (10.0, 10.0, 0.0), (25.0, 100.0, 0.0),
                                       (3.0, 5.0, 0.3), (500.0, 2.0, 0.0), (0.05, 7.0, 0.0)])
def test_sampler_inverts_printed_inverse(lam, a, eps):
    """App. C: applying the printed inverse Phi^{-1} to the sampled (theta, phi)
    returns (s, rho) from the linear maps of (xi0, xi1)."""
    v, xi, (z, x, y) = _single_lobe_samples(lam, a, eps, 2000, 1)
    mu = np.clip(v @ z, -1, 1)
    th = np.arccos(mu)
    ph = np.arctan2(v @ y, v @ x)
    east = xi[:, 2] > 0.5
    ph_e = np.where(east, ph, np.mod(ph, 2 * math.pi) - math.pi)   # into [-pi/2, pi/2]
    s = np.exp(2 * lam * ((np.cos(th) + 1) / 2) ** (1 + eps + a * np.cos(ph_e) ** 2) - 2 * lam)
    rho = np.arctan(np.sqrt((1 + eps) / (1 + eps + a)) * np.tan(ph_e))
    s_ref = xi[:, 0] + (1 - xi[:, 0]) * math.exp(-2 * lam)
    rho_ref = math.pi * (xi[:, 1] - 0.5)
    ok = (np.abs(np.abs(ph_e) - math.pi / 2) > 1e-6) & (th > 1e-6) & (th < math.pi - 1e-6)
    assert ok.mean() > 0.95
    assert np.max(np.abs(s[ok] - s_ref[ok]) / s_ref[ok]) < 1e-8
    assert np.max(np.abs(rho[ok] - rho_ref[ok])) < 1e-8


@pytest.mark.parametrize("lam,a,eps", [(1.0, 0.0, 0.0), (10.0, 10.0, 0.0), (25.0, 100.0, 0.0),
                                       (3.0, 5.0, 0.3), (0.2, 30.0, 0.0)])
def test_sampler_azimuth_marginal(lam, a, eps):
    """The azimuth density is proportional to 1/(1+eps+a cos^2 phi) (inner
    integral of App. B), so E[cos^2 phi] = (sqrt((1+eps)(1+eps+a)) - (1+eps))/a
    (a = 0: 1/2); and the azimuth CDF matches quadrature of that density."""
    n = 200_000
    v, _, (z, x, y) = _single_lobe_samples(lam, a, eps, n, 2)
    ph = np.mod(np.arctan2(v @ y, v @ x), 2 * math.pi)
    c2 = np.cos(ph) ** 2
    expect = 0.5 if a == 0 else (math.sqrt((1 + eps) * (1 + eps + a)) - (1 + eps)) / a
    se = c2.std() / math.sqrt(n)
    assert abs(c2.mean() - expect) < 5 * se + 1e-12
    grid = np.linspace(0, 2 * math.pi, 20001)
    dens = 1.0 / (1 + eps + a * np.cos(grid) ** 2)
    cdf = np.concatenate([[0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    p = ss.kstest(ph, lambda t: np.interp(t, grid, cdf)).pvalue
    assert p > 1e-4


@pytest.mark.parametrize("lam", [0.5, 4.0, 60.0])
def test_sampler_reduces_to_vmf(lam):
    """a = 0, eps = 0: the sample's polar cosine follows the vMF marginal
    lam e^{lam mu} / (2 sinh lam) and the azimuth is uniform."""
    v, _, (z, x, y) = _single_lobe_samples(lam, 0.0, 0.0, 100_000, 3)
    mu = v @ z
    cdf = lambda m: np.expm1(lam * (m + 1)) / np.expm1(2 * lam)
    assert ss.kstest(mu, cdf).pvalue > 1e-4
    ph = np.mod(np.arctan2(v @ y, v @ x), 2 * math.pi)
    assert ss.kstest(ph / (2 * math.pi), "uniform").pvalue > 1e-4


@pytest.mark.parametrize("lam,a,eps", [(2.0, 3.0, 0.0), (10.0, 10.0, 0.0), (25.0, 100.0, 0.0),
                                       (3.0, 5.0, 0.3)])
def test_sampler_chi_square_against_pdf(lam, a, eps):
    """App. C: the pushforward of the uniform (s, rho, east/west) is the
    normalised lobe. Histogram in (mu, phi) bins against the quadrature of
    exp(log G - log K) over each bin."""
    n = 200_000
    v, _, (z, x, y) = _single_lobe_samples(lam, a, eps, n, 4)
    mu = np.clip(v @ z, -1, 1)
    ph = np.mod(np.arctan2(v @ y, v @ x), 2 * math.pi)
    q = np.linspace(0, 1, 13)[1:-1]
    d = -np.log1p(-q * -np.expm1(-2 * lam)) / lam          # vMF quantiles of 1 - mu
    mu_e = np.unique(np.concatenate([[-1.0, 1.0], 1 - d]))
    ph_e = np.linspace(0, 2 * math.pi, 17)
    counts, _, _ = np.histogram2d(mu, ph, bins=[mu_e, ph_e])
    T = lambda t: torch.tensor(t, dtype=F64)
    logk = float(nasg.log_normaliser(T(lam), T(a), eps))
    prob = np.zeros_like(counts)
    for i in range(len(mu_e) - 1):
        mb = np.linspace(mu_e[i], mu_e[i + 1], 9)
        for j in range(len(ph_e) - 1):
            pb = np.linspace(ph_e[j], ph_e[j + 1], 9)
            vv, ww = quad.sphere_nodes(z, x, y, mb, pb, 12)
            lg = nasg.lobe_log_g(T(vv.reshape(-1, 3)), T(z), T(x), T(lam), T(a), eps).numpy()
            prob[i, j] = (np.exp(lg - logk).reshape(ww.shape) * ww).sum()
    assert abs(prob.sum() - 1) < 1e-6
    exp_c = prob.ravel() * n
    obs = counts.ravel()
    keep = exp_c >= 5
    chi2 = (((obs[keep] - exp_c[keep]) ** 2) / exp_c[keep]).sum()
    chi2 += ((obs[~keep].sum() - exp_c[~keep].sum()) ** 2) / max(exp_c[~keep].sum(), 1e-300) if (~keep).any() and exp_c[~keep].sum() > 5 else 0.0
    dof = int(keep.sum()) - 1
    assert ss.chi2.sf(chi2, dof) > 1e-4


@pytest.mark.parametrize("lam,a,eps", [(1.0, 0.0, 0.0), (10.0, 10.0, 0.0), (25.0, 100.0, 0.0),
                                       (3.0, 5.0, 0.3), (0.2, 30.0, 0.0), (200.0, 4.0, 0.0)])
def test_sampler_density_by_jacobian(lam, a, eps):
    """App. C pointwise: the map (xi0, xi1) -> v of one hemisphere carries
    probability 1/2 with uniform density, so the solid-angle density at v is
    1 / (2 |dv/dxi0 x dv/dxi1|). By central differences of the sampler this
    equals G(v)/K with K in closed form (App. B), at every sample."""
    rng = np.random.default_rng(7)
    z, x, y = random_frame(rng)
    n, h = 400, 1e-6
    xi = 0.05 + 0.9 * rng.random((n, 3))
    T = lambda t: torch.tensor(t, dtype=F64)

    def smp(x0, x1):
        return nasg.sample_lobe(T(z).expand(n, 3), T(x).expand(n, 3), T(y).expand(n, 3),
                                T(np.full(n, lam)), T(np.full(n, a)),
                                T(x0), T(x1), T(xi[:, 2]), eps).numpy()

    v = smp(xi[:, 0], xi[:, 1])
    d0 = (smp(xi[:, 0] + h, xi[:, 1]) - smp(xi[:, 0] - h, xi[:, 1])) / (2 * h)
    d1 = (smp(xi[:, 0], xi[:, 1] + h) - smp(xi[:, 0], xi[:, 1] - h)) / (2 * h)
    dens = 0.5 / np.linalg.norm(np.cross(d0, d1), axis=1)
    lg = nasg.lobe_log_g(T(v), T(z), T(x), T(lam), T(a), eps).numpy()
    logk = float(nasg.log_normaliser(T(lam), T(a), eps))
    assert np.max(np.abs(dens / np.exp(lg - logk) - 1)) < 1e-5


def test_sample_value_matches_sampling_variables():
    """At a sampled direction, G equals s * u^{p-1} with u = (cos theta + 1)/2
    and p = 1 + eps + a cos^2 phi, from Phi^{-1} (App. C)."""
    lam, a, eps = 7.0, 12.0, 0.1
    v, xi, (z, x, y) = _single_lobe_samples(lam, a, eps, 500, 6)
    T = lambda t: torch.tensor(t, dtype=F64)
    lg = nasg.lobe_log_g(T(v), T(z), T(x), T(lam), T(a), eps).numpy()
    s = xi[:, 0] + (1 - xi[:, 0]) * math.exp(-2 * lam)
    u = (v @ z + 1) / 2
    c2 = (v @ x) ** 2 / (1 - (v @ z) ** 2)
    pred = np.log(s) + (eps + a * c2) * np.log(u)
    assert np.max(np.abs(lg - pred)) < 1e-9


def test_record_path_equals_decode_path():
    """The record of a decoded mixture (z, x, lambda, a, log(A_k/K_k)) carries
    the whole mixture: rebuilt from the record, the mixture pdf, its
    direction gradient and the sampler (which recovers A_k through the
    closed-form K, eq. "K for NASG") give what the decoded lobes give, in
    float64, for epsilon 0 and 0.3 and lambda, a spanning the clamp range."""
    rng = np.random.default_rng(31)
    K, B = 6, 300
    raw = rng.standard_normal((B, 8 * K)) * 2.0
    raw[:, 5 * K:7 * K] = rng.uniform(-15, 15, (B, 2 * K))
    v = rng.standard_normal((B, 3)); v /= np.linalg.norm(v, axis=1, keepdims=True)
    xi = rng.random((B, 4))
    for eps in (0.0, 0.3):
        lob = nasg.decode(torch.tensor(raw), K, eps)
        rl = nasg.lobes_from_record(lob.record(), eps)
        a = nasg.mixture_log_pdf(torch.tensor(v), lob).numpy()
        b = nasg.mixture_log_pdf(torch.tensor(v), rl).numpy()
        fin = np.isfinite(a)
        assert np.array_equal(fin, np.isfinite(b))
        assert np.max(np.abs(a[fin] - b[fin]) / np.maximum(1.0, np.abs(a[fin]))) < 1e-12
        ga = nasg.log_pdf_direction_grad(torch.tensor(v), lob).numpy()
        gb = nasg.log_pdf_direction_grad(torch.tensor(v), rl).numpy()
        ok = np.isfinite(ga).all(1)
        assert np.allclose(ga[ok], gb[ok], rtol=1e-9, atol=1e-9)
        va, ka = nasg.sample(lob, torch.tensor(xi))
        vb, kb = nasg.sample_from_record(lob.record(), torch.tensor(xi), eps)
        assert torch.equal(ka, kb)
        assert float(torch.abs(va - vb).max()) < 1e-9


@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_mixture_sampler_chi_square_against_pdf(eps):
    """The mixture sampler (inverse-CDF lobe choice composed with the App. C
    lobe sampler) draws from the mixture density D = sum_k A_k G_k / K_k
    (Sec. 3.1): chi-square of a histogram in global (cos theta, phi) bins
    against the quadrature of D over each bin. A lobe index off by one, a
    weight taken without normalisation, or a lobe sampled in another lobe's
    frame moves probability between bins far beyond the test's power."""
    rng = np.random.default_rng(32)
    K, n = 4, 400_000
    raw = rng.standard_normal((1, 8 * K))
    raw[0, 5 * K:6 * K] = np.log([3.0, 12.0, 1.0, 30.0])
    raw[0, 6 * K:7 * K] = np.log([0.5, 20.0, 2.0, 100.0])
    raw[0, 7 * K:8 * K] = [0.3, -0.4, 0.8, -1.2]
    one = nasg.decode(torch.tensor(raw), K, eps)
    rep = lambda t: t.expand(n, *t.shape[1:])
    lob = nasg.Lobes(z=rep(one.z), x=rep(one.x), y=rep(one.y), lam=rep(one.lam), a=rep(one.a),
                     log_A=rep(one.log_A), log_K=rep(one.log_K), eps=eps)
    v, k = nasg.sample(lob, torch.tensor(rng.random((n, 4))))
    v = v.numpy()
    # the lobe choice alone follows A
    freq = np.bincount(k.numpy(), minlength=K) / n
    A = torch.exp(one.log_A[0]).numpy()
    assert np.max(np.abs(freq - A) / np.sqrt(A * (1 - A) / n)) < 5
    mu_e = np.linspace(-1, 1, 13)
    ph_e = np.linspace(-math.pi, math.pi, 17)
    counts, _, _ = np.histogram2d(np.clip(v[:, 2], -1, 1), np.arctan2(v[:, 1], v[:, 0]), bins=[mu_e, ph_e])
    prob = np.zeros_like(counts)
    ez, ex, ey = np.array([0.0, 0, 1]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    for i in range(len(mu_e) - 1):
        mb = np.linspace(mu_e[i], mu_e[i + 1], 17)
        for j in range(len(ph_e) - 1):
            pb = np.linspace(ph_e[j], ph_e[j + 1], 17)
            vv, ww = quad.sphere_nodes(ez, ex, ey, mb, pb, 12)
            m = vv.reshape(-1, 3).shape[0]
            lq = nasg.mixture_log_pdf(torch.tensor(vv.reshape(-1, 3)), nasg.Lobes(
                z=one.z.expand(m, K, 3), x=one.x.expand(m, K, 3), y=one.y.expand(m, K, 3),
                lam=one.lam.expand(m, K), a=one.a.expand(m, K), log_A=one.log_A.expand(m, K),
                log_K=one.log_K.expand(m, K), eps=eps)).numpy()
            prob[i, j] = (np.exp(lq).reshape(ww.shape) * ww).sum()
    assert abs(prob.sum() - 1) < 1e-4
    exp_c, obs = prob.ravel() * n, counts.ravel()
    keep = exp_c >= 5
    chi2 = (((obs[keep] - exp_c[keep]) ** 2) / exp_c[keep]).sum()
    rest_e, rest_o = exp_c[~keep].sum(), obs[~keep].sum()
    dof = int(keep.sum()) - 1
    if rest_e >= 5:
        chi2 += (rest_o - rest_e) ** 2 / rest_e
        dof += 1
    assert ss.chi2.sf(chi2, dof) > 1e-4, (chi2, dof)


def test_choose_lobe_inverse_cdf():
    log_A = torch.log(torch.tensor([[0.1, 0.2, 0.3, 0.4]] * 5, dtype=F64))
    xi = torch.tensor([0.0, 0.15, 0.2999, 0.61, 0.99999], dtype=F64)
    assert nasg.choose_lobe(log_A, xi).tolist() == [0, 1, 1, 3, 3]
    # rounding leaves no lobe: the last lobe with positive weight
    log_B = torch.log(torch.tensor([[0.5, 0.5 - 1e-9, 0.0]], dtype=F64))
    assert nasg.choose_lobe(log_B, torch.tensor([0.9999999999])).tolist() == [1]


def _np_bf16(a):
    """Round float32 values to bfloat16 (ties to even) with integer arithmetic."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_mlp_is_plain_matmul_chain():
    """Sec. 4.1: bias-free layers with ReLU; the input gets a constant one."""
    rng = np.random.default_rng(9)
    shapes = mlp.layer_shapes(16, 3, 2)
    Ws = [rng.standard_normal(s) for s in shapes]
    feat = rng.standard_normal((7, 9))
    h = np.concatenate([feat, np.ones((7, 1))], 1)
    for W in Ws[:-1]:
        h = np.maximum(h @ W.T, 0)
    ref = h @ Ws[-1].T
    got = mlp.forward([torch.tensor(W) for W in Ws], torch.tensor(feat)).numpy()
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
    # BF16 emulation: operands rounded with integer RNE, wide accumulation
    Wb = [_np_bf16(W) for W in Ws]
    h = _np_bf16(np.concatenate([feat, np.ones((7, 1))], 1))
    for W in Wb[:-1]:
        h = _np_bf16(np.maximum((h @ W.T).astype(np.float32), 0))
    refb = h @ Wb[-1].T
    gotb = mlp.forward([torch.tensor(W) for W in Ws], torch.tensor(feat), bf16=True).numpy()
    assert np.allclose(gotb, refb, rtol=1e-12, atol=1e-12)


def test_bf16_backward_is_the_rounded_chain_rule():
    """The BF16 emulation's backward: the chain rule written out in NumPy with
    integer round-to-nearest-even, the deltas rounded to float32 then bfloat16
    at every layer (the raw-output gradient included), products and sums in
    float64. A delta left unrounded at any one layer moves that layer's
    gradient by ~2^-9 relative and fails the 1e-12 bound."""
    rng = np.random.default_rng(19)
    shapes = mlp.layer_shapes(16, 3, 2)
    Ws = [rng.standard_normal(s) * 0.4 for s in shapes]
    B = 40
    feat = rng.standard_normal((B, 9))
    g_raw = rng.standard_normal((B, shapes[-1][0])) * 1e-2
    Wb = [_np_bf16(W) for W in Ws]
    hs, ys = [_np_bf16(np.concatenate([feat, np.ones((B, 1))], 1))], []
    for W in Wb[:-1]:
        y = (hs[-1] @ W.T).astype(np.float32).astype(np.float64)
        ys.append(y)
        hs.append(_np_bf16(np.maximum(y, 0)))
    d = _np_bf16(g_raw)
    ref = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        ref[l] = d.T @ hs[l]
        if l > 0:
            d = _np_bf16((d @ Wb[l]) * (ys[l - 1] > 0))
    got = train.weight_grad_from_raw_grad([torch.tensor(W) for W in Ws], torch.tensor(feat),
                                          torch.tensor(g_raw), bf16=True)
    for a, b in zip(got, ref):
        assert np.allclose(a.numpy(), b, rtol=1e-12, atol=1e-15)
    # and without rounding the deltas the result differs at every layer
    plain = [None] * len(Ws)
    d = g_raw
    for l in range(len(Ws) - 1, -1, -1):
        plain[l] = d.T @ hs[l]
        if l > 0:
            d = (d @ Wb[l]) * (ys[l - 1] > 0)
    for a, b in zip(got, plain):
        assert np.abs(a.numpy() - b).max() > 1e-6 * np.abs(b).max()


def test_log_normaliser_derivatives():
    """d log K / d lam = 2/expm1(2 lam) - 1/lam and d log K / d a = -1/(2(1+eps+a)),
    differentiated by hand from eq. "K for NASG" with epsilon (App. B)."""
    for lam, a, eps in [(0.3, 2.0, 0.0), (5.0, 0.1, 0.2), (40.0, 30.0, 0.0)]:
        l = torch.tensor(lam, dtype=F64, requires_grad=True)
        aa = torch.tensor(a, dtype=F64, requires_grad=True)
        gl, ga = torch.autograd.grad(nasg.log_normaliser(l, aa, eps), [l, aa])
        assert abs(float(gl) - (2 / math.expm1(2 * lam) - 1 / lam)) < 1e-12
        assert abs(float(ga) + 1 / (2 * (1 + eps + a))) < 1e-12


def test_loss_gradient_matches_finite_differences():
    """Sec. 4.2: the weighted-NLL gradient of the oracle against central
    differences of its loss, for every weight of a tiny network."""
    rng = np.random.default_rng(12)
    K = 2
    shapes = mlp.layer_shapes(8, 2, K)
    Ws = [torch.tensor(rng.uniform(-0.6, 0.6, s)) for s in shapes]
    B = 6
    feat = torch.tensor(rng.standard_normal((B, 9)))
    d = rng.standard_normal((B, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    dirs = torch.tensor(d)
    w = torch.tensor(np.exp(rng.standard_normal(B)))
    for eps in (0.0, 0.25):
        L, g = train.loss_and_grad(Ws, feat, dirs, w, K, eps)
        for l, W in enumerate(Ws):
            flat = W.reshape(-1)
            fd = torch.zeros_like(flat)
            for i in range(flat.numel()):
                h = 1e-6 * max(1.0, abs(float(flat[i])))
                wp = [x.clone() for x in Ws]; wp[l].view(-1)[i] += h
                wm = [x.clone() for x in Ws]; wm[l].view(-1)[i] -= h
                fd[i] = (train.weighted_nll(wp, feat, dirs, w, K, eps)
                         - train.weighted_nll(wm, feat, dirs, w, K, eps)) / (2 * h)
            err = torch.abs(fd - g[l].reshape(-1))
            assert float(err.max()) < 1e-6 * max(1.0, float(torch.abs(g[l]).max())), (l, eps)


def test_adam_matches_library_and_hand_step():
    """Kingma and Ba's Adam: against torch.optim.Adam over several steps, and
    the first step by hand: m_hat = g, v_hat = g^2, so the update is
    -lr g / (|g| + eps)."""
    rng = np.random.default_rng(13)
    p0 = torch.tensor(rng.standard_normal(50))
    grads = [torch.tensor(rng.standard_normal(50)) for _ in range(6)]
    lr = 1e-3
    p1, m, v, t = train.adam_step(p0, grads[0], torch.zeros(50, dtype=F64), torch.zeros(50, dtype=F64), 0, lr)
    assert torch.allclose(p1, p0 - lr * grads[0] / (torch.abs(grads[0]) + 1e-8), rtol=0, atol=1e-15)
    ref = p0.clone().requires_grad_(True)
    opt = torch.optim.Adam([ref], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    p, m, v, t = p0.clone(), torch.zeros(50, dtype=F64), torch.zeros(50, dtype=F64), 0
    for g in grads:
        ref.grad = g.clone()
        opt.step()
        p, m, v, t = train.adam_step(p, g, m, v, t, lr)
    assert torch.allclose(p, ref.detach(), rtol=0, atol=1e-14)


def _constant_output_net(raw_vec, hidden=4, n_hidden=2):
    """Weights whose output is raw_vec for every input: the constant-one input
    is carried through the hidden layers in unit 0 and read by the last layer."""
    K8 = raw_vec.shape[0]
    Ws = [np.zeros((hidden, 10))]
    Ws[0][0, 9] = 1.0
    for _ in range(n_hidden - 1):
        W = np.zeros((hidden, hidden)); W[0, 0] = 1.0
        Ws.append(W)
    W = np.zeros((K8, hidden)); W[:, 0] = raw_vec
    Ws.append(W)
    return [torch.tensor(W) for W in Ws]


def test_weighted_nll_definition():
    """Sec. 4.2: the loss is the mean of w * (-log q). With a single lobe of
    eccentricity exp(-15) (the clamp floor) the mixture is the vMF density to
    about 1e-7, so the loss matches the library's vMF log-density."""
    rng = np.random.default_rng(14)
    K = 1
    lam = 6.0
    raw = np.array([0.7, -0.3, 1.1, 0.4, -0.8, math.log(lam), -15.0, 0.0])
    Ws = _constant_output_net(raw)
    B = 64
    feat = torch.tensor(rng.standard_normal((B, 9)))
    d = rng.standard_normal((B, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    w = np.exp(rng.standard_normal(B))
    lob = nasg.decode(torch.tensor(raw[None]), K)
    ref = np.mean(w * -ss.vonmises_fisher(mu=lob.z[0, 0].numpy(), kappa=lam).logpdf(d))
    L = float(train.weighted_nll(Ws, feat, torch.tensor(d), torch.tensor(w), K))
    assert abs(L - ref) < 1e-5 * abs(ref)


def test_raw_output_grad_matches_finite_differences():
    rng = np.random.default_rng(15)
    K, B = 3, 4
    raw = torch.tensor(rng.standard_normal((B, 8 * K)))
    d = rng.standard_normal((B, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    dirs, w = torch.tensor(d), torch.tensor(np.exp(rng.standard_normal(B)))
    g = train.raw_output_grad(raw, dirs, w, K, 0.1)

    def loss(r):
        return float((w * -nasg.mixture_log_pdf(dirs, nasg.decode(r, K, 0.1))).mean())
    fd = torch.zeros_like(raw)
    for i in range(B):
        for j in range(8 * K):
            rp = raw.clone(); rp[i, j] += 1e-6
            rm = raw.clone(); rm[i, j] -= 1e-6
            fd[i, j] = (loss(rp) - loss(rm)) / 2e-6
    assert float(torch.abs(fd - g).max()) < 1e-7


def test_weight_grad_from_raw_grad_is_the_chain_rule():
    """Composing raw_output_grad with the MLP backward reproduces the full
    weight gradient (same network, same data)."""
    rng = np.random.default_rng(16)
    K = 2
    Ws = [torch.tensor(rng.uniform(-0.5, 0.5, s)) for s in mlp.layer_shapes(8, 3, K)]
    feat = torch.tensor(rng.standard_normal((20, 9)))
    d = rng.standard_normal((20, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    w = torch.tensor(np.exp(rng.standard_normal(20)))
    _, full = train.loss_and_grad(Ws, feat, torch.tensor(d), w, K)
    g_raw = train.raw_output_grad(mlp.forward(Ws, feat), torch.tensor(d), w, K)
    staged = train.weight_grad_from_raw_grad(Ws, feat, g_raw)
    for a, b in zip(full, staged):
        assert torch.allclose(a, b, rtol=1e-12, atol=1e-14)


# ---- selection probability and the blended loss (Sec. 4.2, Sec. 5) ----

def _tiny_selection_net(rng, K=2, hidden=8, n_hidden=2):
    return [torch.tensor(rng.uniform(-0.6, 0.6, s)) for s in mlp.layer_shapes(hidden, n_hidden, K, selection=True)]


def _batch(rng, B):
    feat = torch.tensor(rng.standard_normal((B, 9)))
    d = rng.standard_normal((B, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    return feat, torch.tensor(d), torch.tensor(np.exp(rng.standard_normal(B)))


def test_selection_output_shape_and_decoding():
    """d = 8N + 1 outputs (Sec. 4.1); the last decodes as sigmoid (Tab.
    "decoding"): a constant logit of 0 gives c = 1/2, of log 3 gives 3/4."""
    assert mlp.layer_shapes(64, 4, 16, selection=True)[-1] == (129, 64)
    for logit, c in ((0.0, 0.5), (math.log(3.0), 0.75)):
        raw = np.concatenate([np.zeros(8), [logit]])
        Ws = _constant_output_net(raw)
        out = mlp.forward(Ws, torch.zeros(3, 9))
        assert torch.allclose(nasg.selection(out, 1), torch.full((3,), c, dtype=F64), rtol=0, atol=1e-15)


def test_blended_loss_limits():
    """e = 0 leaves KL(p || q) alone: the blended loss equals the weighted NLL
    and the selection row receives no gradient. With p_fs equal to q at each
    training direction, q_hat = q for every c: again the weighted NLL for any
    e, a zero selection gradient (to rounding), and for the lobe outputs
    d log q_hat = c d log q, so their raw-output gradient is the NLL's scaled
    per sample by e c + (1 - e)."""
    rng = np.random.default_rng(31)
    K = 2
    Ws = _tiny_selection_net(rng, K)
    feat, dirs, w = _batch(rng, 40)
    pdf = torch.tensor(np.exp(rng.uniform(-2, 1, 40)))
    nll = float(train.weighted_nll(Ws, feat, dirs, w, K))
    L0, g0 = train.blended_loss_and_grad(Ws, feat, dirs, w, pdf, K, e=0.0)
    assert abs(L0 - nll) < 1e-12 * abs(nll)
    assert float(torch.abs(g0[-1][-1]).max()) == 0.0
    q = torch.exp(nasg.mixture_log_pdf(dirs, nasg.decode(mlp.forward(Ws, feat), K)))
    Lq, gq = train.blended_loss_and_grad(Ws, feat, dirs, w, q, K, e=0.7)
    assert abs(Lq - nll) < 1e-12 * abs(nll)
    assert float(torch.abs(gq[-1][-1]).max()) < 1e-13
    raw = mlp.forward(Ws, feat)
    gb = train.blended_raw_output_grad(raw, dirs, w, q, K, e=0.7)
    gn = train.raw_output_grad(raw[:, :8 * K], dirs, w, K)
    c = nasg.selection(raw, K)
    assert torch.allclose(gb[:, :8 * K], gn * (0.7 * c + 0.3)[:, None], rtol=1e-10, atol=1e-15)
    assert float(torch.abs(gb[:, 8 * K]).max()) < 1e-15


def test_blended_loss_value_by_hand():
    """One lobe of eccentricity exp(-15) is the vMF density to ~1e-7 (scipy),
    c = sigmoid(0.4), p_fs given: the loss is mean w -(e log(c q + (1-c) p)
    + (1-e) log q) computed from scipy's vMF, not from the oracle's mixture."""
    rng = np.random.default_rng(32)
    lam, logit, e = 5.0, 0.4, 0.2
    raw = np.array([0.7, -0.3, 1.1, 0.4, -0.8, math.log(lam), -15.0, 0.0, logit])
    Ws = _constant_output_net(raw)
    feat, dirs, w = _batch(rng, 64)
    pdf = np.exp(rng.uniform(-3, 0.5, 64))
    z = nasg.decode(torch.tensor(raw[None]), 1).z[0, 0].numpy()
    q = np.exp(ss.vonmises_fisher(mu=z, kappa=lam).logpdf(dirs.numpy()))
    c = 1.0 / (1.0 + math.exp(-logit))
    ref = np.mean(w.numpy() * -(e * np.log(c * q + (1 - c) * pdf) + (1 - e) * np.log(q)))
    L = float(train.blended_nll(Ws, feat, dirs, w, torch.tensor(pdf), 1, e=e))
    assert abs(L - ref) < 1e-5 * abs(ref)


def test_blended_gradient_matches_finite_differences():
    """The blended loss's autograd gradient against central differences, every
    weight of a tiny network with the selection output."""
    rng = np.random.default_rng(33)
    K = 2
    Ws = _tiny_selection_net(rng, K)
    feat, dirs, w = _batch(rng, 6)
    pdf = torch.tensor(np.exp(rng.uniform(-2, 1, 6)))
    L, g = train.blended_loss_and_grad(Ws, feat, dirs, w, pdf, K, e=0.2)
    for l, W in enumerate(Ws):
        flat = W.reshape(-1)
        fd = torch.zeros_like(flat)
        for i in range(flat.numel()):
            h = 1e-6 * max(1.0, abs(float(flat[i])))
            wp = [x.clone() for x in Ws]; wp[l].view(-1)[i] += h
            wm = [x.clone() for x in Ws]; wm[l].view(-1)[i] -= h
            fd[i] = (train.blended_nll(wp, feat, dirs, w, pdf, K, 0.2)
                     - train.blended_nll(wm, feat, dirs, w, pdf, K, 0.2)) / (2 * h)
        err = torch.abs(fd - g[l].reshape(-1))
        assert float(err.max()) < 1e-6 * max(1.0, float(torch.abs(g[l]).max())), l
    # the raw-output form composes to the same weight gradient
    g_raw = train.blended_raw_output_grad(mlp.forward(Ws, feat), dirs, w, pdf, K, e=0.2)
    for a, b in zip(train.weight_grad_from_raw_grad(Ws, feat, g_raw), g):
        assert torch.allclose(a, b, rtol=1e-11, atol=1e-14)


def test_blend_ramp_schedule():
    """Sec. 5: b starts at 0 and rises by 1/B after every M images (M = 4,
    B = 64), reaching 1 after M B = 256 images."""
    assert train.blend_ramp(0) == 0.0 and train.blend_ramp(3) == 0.0
    assert train.blend_ramp(4) == 1 / 64 and train.blend_ramp(7) == 1 / 64
    assert train.blend_ramp(255) == 63 / 64
    assert train.blend_ramp(256) == 1.0 and train.blend_ramp(10 ** 6) == 1.0
    assert train.blend_ramp(10, M=2, B=4) == 1.0 and train.blend_ramp(5, M=2, B=4) == 0.5


# ---- direction gradient of the mixture pdf ----

def test_direction_gradient_of_isotropic_lobe():
    """a -> 0: the lobe is the vMF density exp(lam (z.v - 1)) / K, whose
    log-gradient on the sphere is lam (z - (z.v) v)."""
    rng = np.random.default_rng(41)
    raw = np.array([0.7, -0.3, 1.1, 0.4, -0.8, math.log(7.0), -15.0, 0.0])
    lob = nasg.decode(torch.tensor(np.tile(raw, (32, 1))), 1)
    d = rng.standard_normal((32, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    g = nasg.log_pdf_direction_grad(torch.tensor(d), lob).numpy()
    z = lob.z[0, 0].numpy()
    ref = 7.0 * (z[None] - (d @ z)[:, None] * d)
    assert np.abs(g - ref).max() < 1e-5 * 7.0


def test_direction_gradient_matches_finite_differences():
    """Central differences of log D along two tangent directions of the
    sphere (moving on great circles), for a random anisotropic mixture with
    and without epsilon; the gradient is tangent."""
    rng = np.random.default_rng(42)
    K, B = 4, 40
    raw = torch.tensor(rng.standard_normal((B, 8 * K)) * 1.5)
    d = rng.standard_normal((B, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    t1 = np.cross(d, rng.standard_normal((B, 3))); t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(d, t1)
    for eps in (0.0, 0.4):
        lob = nasg.decode(raw, K, eps)
        g = nasg.log_pdf_direction_grad(torch.tensor(d), lob).numpy()
        assert np.abs((g * d).sum(1)).max() < 1e-10
        h = 1e-5
        for t in (t1, t2):
            fp = nasg.mixture_log_pdf(torch.tensor(np.cos(h) * d + np.sin(h) * t), lob).numpy()
            fm = nasg.mixture_log_pdf(torch.tensor(np.cos(h) * d - np.sin(h) * t), lob).numpy()
            fd = (fp - fm) / (2 * h)
            err = np.abs(fd - (g * t).sum(1))
            assert err.max() < 1e-6 * max(1.0, np.abs(g).max()), (eps, err.max())


def test_isotropic_decode_is_vmf_mixture():
    """isotropic = True: a = 0 for every lobe and the mixture equals scipy's
    von Mises-Fisher mixture with kappa = lambda and the softmax weights."""
    rng = np.random.default_rng(51)
    K, B = 3, 16
    raw = torch.tensor(rng.standard_normal((B, 8 * K)))
    lob = nasg.decode(raw, K, isotropic=True)
    assert float(torch.abs(lob.a).max()) == 0.0
    d = rng.standard_normal((B, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    lq = nasg.mixture_log_pdf(torch.tensor(d), lob).numpy()
    A = np.exp(lob.log_A.numpy())
    ref = np.zeros(B)
    for b in range(B):
        ref[b] = np.log(sum(A[b, k] * np.exp(ss.vonmises_fisher(mu=lob.z[b, k].numpy(), kappa=float(lob.lam[b, k])).logpdf(d[b]))
                            for k in range(K)))
    assert np.abs(lq - ref).max() < 1e-9


def test_sin_theta_derivative_at_saturation():
    """sin theta = sqrt(1 - cos^2 theta) of the decode: where float64 rounds
    1 - cos^2 to zero (|raw| above ~37) its derivative is taken as zero (the
    exact one, -cos sin / 2 per unit of the raw output, is below 1e-8);
    elsewhere it is the plain chain rule, checked against central
    differences."""
    K = 1
    raw = torch.zeros(4, 8, dtype=F64)
    raw[:, 0] = torch.tensor([40.0, -45.0, 0.7, -2.0])
    raw[:, 1:5] = 0.3
    raw.requires_grad_(True)
    z = nasg.decode(raw, K).z
    (g,) = torch.autograd.grad(z[..., 0].sum() + z[..., 1].sum(), raw)
    assert torch.isfinite(g).all()
    assert float(g[0, 0]) == 0.0 and float(g[1, 0]) == 0.0
    h = 1e-6
    for i in (2, 3):
        rp, rm = raw.detach().clone(), raw.detach().clone()
        rp[i, 0] += h
        rm[i, 0] -= h
        fd = ((nasg.decode(rp, K).z[i, 0, :2].sum() - nasg.decode(rm, K).z[i, 0, :2].sum()) / (2 * h))
        assert abs(float(g[i, 0]) - float(fd)) < 1e-8
