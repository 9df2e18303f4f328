"""Seeded synthetic inputs shaped like a path tracer's guiding workload.

This module holds no NASG arithmetic: it draws vertex features, training
targets, radiance weights, uniforms and initial network weights with NumPy,
and is the only code shared between the HIP path's tests and the oracle's.
Every array it returns is float32 in the device layout (structure of arrays).

Workload recipe (the paper trains on rendered samples; there is no scene
here, so these stand in for them):
* features: position p ~ U[0,1]^3; outgoing direction and normal uniform on
  the sphere (normalised Gaussians), stored SoA as [9][n];
* training directions: a K_t-lobe von Mises-Fisher mixture whose means rotate
  with position (``VmfTarget``), or anisotropic tangent-plane Gaussians
  (``AnisoTarget``);
* training weights p / q_hat: lognormal(0, 1), independent of the direction;
* uniforms for sampling: U[0,1)^4 per vertex, SoA [4][n];
* initial weights: W_l ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), fan_in counting
  the constant-one input column.
"""

import math

import numpy as np

IN_FEATURES = 9


def rng_for(seed):
    return np.random.default_rng(seed)


def unit_vectors(n, rng):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def features(n, rng):
    """[9, n] float32: p (3), omega_o (3), normal (3)."""
    p = rng.random((n, 3))
    wo = unit_vectors(n, rng)
    nrm = unit_vectors(n, rng)
    return np.ascontiguousarray(np.concatenate([p, wo, nrm], axis=1).T.astype(np.float32))


def uniforms(n, rng):
    """[4, n] float32 in [0, 1): (xi_sel, xi0, xi1, xi2) per vertex."""
    return np.ascontiguousarray(rng.random((4, n), dtype=np.float32))


def radiance_weights(n, rng):
    """[n] float32 = exp(N(0, 1))."""
    return np.exp(rng.standard_normal(n)).astype(np.float32)


ENCODED_INPUTS = 64   # W_0's columns with the encoded input of Tab. "encoding"


def layer_shapes(hidden, n_hidden, n_lobes, selection=False, encoded=False):
    shapes = [(hidden, ENCODED_INPUTS if encoded else IN_FEATURES + 1)]
    shapes += [(hidden, hidden)] * (n_hidden - 1)
    shapes.append((8 * n_lobes + (1 if selection else 0), hidden))
    return shapes


def init_weights(shapes, rng):
    """List of float32 [out, in] matrices drawn U(-1/sqrt(in), 1/sqrt(in))."""
    mats = []
    for (o, i) in shapes:
        b = 1.0 / math.sqrt(i)
        mats.append(rng.uniform(-b, b, size=(o, i)).astype(np.float32))
    return mats


def flat_weights(mats):
    return np.concatenate([m.reshape(-1) for m in mats]).astype(np.float32)


def _basis(n):
    """Orthonormal (t, b) completing unit vectors n [m, 3] (Duff et al. 2017)."""
    sign = np.where(n[:, 2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    t = np.stack([1.0 + sign * n[:, 0] ** 2 * a, sign * b, -sign * n[:, 0]], axis=1)
    bb = np.stack([b, sign + n[:, 1] ** 2 * a, -n[:, 1]], axis=1)
    return t, bb


def _rotate(v, axis, angle):
    """Rodrigues rotation of v [m,3] about unit axis [m,3] by angle [m]."""
    c, s = np.cos(angle)[:, None], np.sin(angle)[:, None]
    return v * c + np.cross(axis, v) * s + axis * (axis * v).sum(1, keepdims=True) * (1.0 - c)


class VmfTarget:
    """Mixture of von Mises-Fisher lobes whose means rotate with position.

    Lobe j: mean mu_j(p) = Rot(r_j, 2 pi <f_j, p>) mu0_j with mu0_j, r_j
    uniform on the sphere and f_j ~ U[-1/2, 1/2]^3; concentration
    kappa_j = exp(U[0, ln 200]); weight pi_j proportional to U[0.5, 1.5].
    """

    def __init__(self, n_lobes=4, seed=0):
        rng = rng_for(seed)
        self.n = n_lobes
        self.mu0 = unit_vectors(n_lobes, rng)
        self.axis = unit_vectors(n_lobes, rng)
        self.freq = rng.uniform(-0.5, 0.5, size=(n_lobes, 3))
        self.kappa = np.exp(rng.uniform(0.0, math.log(200.0), size=n_lobes))
        w = rng.uniform(0.5, 1.5, size=n_lobes)
        self.weight = w / w.sum()

    def means(self, pos):
        """[m, J, 3] lobe means at positions pos [m, 3]."""
        m = pos.shape[0]
        out = np.empty((m, self.n, 3))
        for j in range(self.n):
            ang = 2.0 * math.pi * (pos @ self.freq[j])
            out[:, j] = _rotate(np.broadcast_to(self.mu0[j], (m, 3)),
                                np.broadcast_to(self.axis[j], (m, 3)), ang)
        return out

    def sample(self, pos, rng):
        """[3, m] float32 directions for positions pos [m, 3] (float64 in)."""
        m = pos.shape[0]
        j = rng.choice(self.n, size=m, p=self.weight)
        mu = self.means(pos)[np.arange(m), j]
        kap = self.kappa[j]
        xi = rng.random(m)
        # Wood / Jakob: cos angle = 1 + log(xi + (1 - xi) e^{-2 kappa}) / kappa
        w = 1.0 + np.log(xi + (1.0 - xi) * np.exp(-2.0 * kap)) / kap
        w = np.clip(w, -1.0, 1.0)
        ph = 2.0 * math.pi * rng.random(m)
        r = np.sqrt(np.maximum(0.0, 1.0 - w * w))
        t, b = _basis(mu)
        v = (r * np.cos(ph))[:, None] * t + (r * np.sin(ph))[:, None] * b + w[:, None] * mu
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        return np.ascontiguousarray(v.T.astype(np.float32))

    def log_pdf(self, pos, v):
        """log of the target density at unit directions v [m, 3] (float64)."""
        mu = self.means(pos)
        dots = (mu * v[:, None, :]).sum(-1)
        k = self.kappa[None, :]
        log_c = np.log(k) - np.log(2.0 * math.pi) - np.log(-np.expm1(-2.0 * k))
        terms = np.log(self.weight)[None, :] + log_c + k * (dots - 1.0)
        mx = terms.max(1, keepdims=True)
        return (mx + np.log(np.exp(terms - mx).sum(1, keepdims=True)))[:, 0]


class AnisoTarget:
    """Anisotropic lobes: tangent-plane Gaussians pushed through the exp map.

    Lobe j at position p: centre mu_j(p) and tangent frame (e1, e2) rotating
    with p like VmfTarget; a tangent offset t = (sigma_major g1, sigma_minor g2)
    with g ~ N(0, I) (redrawn while |t| >= pi) maps to
    cos|t| mu + sin|t| (t/|t|) in the (e1, e2) plane. sigma_major ~
    logU[0.1, 0.8] rad, ratio ~ logU[1, 20], sigma_minor = sigma_major / ratio.
    Only sampling is needed by the workload; densities are not.
    """

    def __init__(self, n_lobes=8, seed=0):
        rng = rng_for(seed)
        self.n = n_lobes
        self.mu0 = unit_vectors(n_lobes, rng)
        self.axis = unit_vectors(n_lobes, rng)
        self.freq = rng.uniform(-0.5, 0.5, size=(n_lobes, 3))
        self.sig_major = np.exp(rng.uniform(math.log(0.1), math.log(0.8), size=n_lobes))
        ratio = np.exp(rng.uniform(0.0, math.log(20.0), size=n_lobes))
        self.sig_minor = self.sig_major / ratio
        w = rng.uniform(0.5, 1.5, size=n_lobes)
        self.weight = w / w.sum()

    def sample(self, pos, rng):
        m = pos.shape[0]
        j = rng.choice(self.n, size=m, p=self.weight)
        ang = 2.0 * math.pi * (pos * self.freq[j]).sum(1)
        mu = _rotate(self.mu0[j], self.axis[j], ang)
        t0, b0 = _basis(self.mu0[j])
        e1 = _rotate(t0, self.axis[j], ang)
        e2 = _rotate(b0, self.axis[j], ang)
        g = rng.standard_normal((m, 2))
        t = np.stack([self.sig_major[j] * g[:, 0], self.sig_minor[j] * g[:, 1]], 1)
        rad = np.linalg.norm(t, axis=1)
        bad = rad >= math.pi
        while bad.any():
            g = rng.standard_normal((int(bad.sum()), 2))
            t[bad] = np.stack([self.sig_major[j[bad]] * g[:, 0],
                               self.sig_minor[j[bad]] * g[:, 1]], 1)
            rad = np.linalg.norm(t, axis=1)
            bad = rad >= math.pi
        safe = np.where(rad > 0, rad, 1.0)
        d = (t[:, 0:1] * e1 + t[:, 1:2] * e2) / safe[:, None]
        v = np.cos(rad)[:, None] * mu + np.sin(rad)[:, None] * d
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        return np.ascontiguousarray(v.T.astype(np.float32))


def training_batch(n, rng, target):
    """(feat [9,n], dir [3,n], w [n]) float32 for one training step."""
    feat = features(n, rng)
    dirs = target.sample(feat[0:3].T.astype(np.float64), rng)
    w = radiance_weights(n, rng)
    return feat, dirs, w


def lambert_pdf(dirs, normals):
    """Cosine-weighted (Lambertian) BSDF sampling pdf max(0, d.n)/pi at unit
    directions [3, B] (or [B, 3]) about unit normals of the same shape: the
    p_fs a renderer would supply for a diffuse surface."""
    d = np.asarray(dirs, dtype=np.float64)
    n = np.asarray(normals, dtype=np.float64)
    n = n / np.linalg.norm(n, axis=0 if d.shape[0] == 3 else -1, keepdims=True)
    c = (d * n).sum(axis=0 if d.shape[0] == 3 else -1)
    return (np.maximum(c, 0.0) / math.pi).astype(np.float32)
