"""NASG density, normaliser, mixture and direct sampler in float64 (oracle).

Test infrastructure only (see the package docstring). Every formula is the
paper's printed form, evaluated literally in float64; no stable rewrites.

Shapes: B vertices, K lobes. Directions are [B, 3]; per-lobe tensors are
[B, K] or [B, K, 3].
"""

import math
from dataclasses import dataclass

import torch

F64 = torch.float64
N_PARAM = 8          # per lobe: cos th, sin ph, cos ph, sin tau, cos tau, log lam, log a, logit
LOG_CLAMP = 15.0     # reading: log lambda and log a are clamped to [-15, 15]


@dataclass
class Lobes:
    """Decoded NASG mixture parameters for a batch (Sec. 4.1)."""
    z: torch.Tensor       # [B, K, 3] lobe axis
    x: torch.Tensor       # [B, K, 3] tangent axis
    y: torch.Tensor       # [B, K, 3] bitangent axis, z cross x
    lam: torch.Tensor     # [B, K] sharpness lambda
    a: torch.Tensor       # [B, K] eccentricity a
    log_A: torch.Tensor   # [B, K] log mixture weight (log-softmax of the logits)
    log_K: torch.Tensor   # [B, K] log normaliser
    eps: float            # App. A continuity parameter (0 = the form of Sec. 3.2)

    @property
    def n_lobes(self):
        return self.lam.shape[-1]

    def record(self):
        """[B, K, 9] = z, x, lambda, a, log(A_k / K_k)."""
        return torch.cat([self.z, self.x, self.lam[..., None], self.a[..., None],
                          (self.log_A - self.log_K)[..., None]], dim=-1)


def _unit_pair(c, s):
    """Divide a (cos, sin) pair by its norm; a zero pair becomes (1, 0).

    Reading: the decoded sine/cosine values of Tab. "decoding" are independent
    sigmoids, so they are projected onto the unit circle before use. The zero
    pair is replaced before the norm is taken, so its derivative is zero
    rather than undefined.
    """
    ok = (c * c + s * s) > 0
    c1 = torch.where(ok, c, torch.ones_like(c))
    s1 = torch.where(ok, s, torch.zeros_like(s))
    n = torch.sqrt(c1 * c1 + s1 * s1)
    return c1 / n, s1 / n


class _SinFromCos(torch.autograd.Function):
    """sin = sqrt(max(0, 1 - cos^2)) with its derivative -cos / sin, taken as
    0 where 1 - cos^2 rounds to 0 in float64 (|raw| above ~37: the exact
    derivative, -cos sin / 2 per unit of the raw output, is below 1e-8
    there, while the literal chain rule would give infinity times a
    vanishing factor)."""

    @staticmethod
    def forward(ctx, c):
        s = torch.sqrt(torch.clamp(1.0 - c * c, min=0.0))
        ctx.save_for_backward(c, s)
        return s

    @staticmethod
    def backward(ctx, g):
        c, s = ctx.saved_tensors
        safe = torch.where(s > 0, s, torch.ones_like(s))
        return torch.where(s > 0, -g * c / safe, torch.zeros_like(g))


def log_normaliser(lam, a, eps=0.0):
    """log K, with K = 2 pi (1 - e^{-2 lam}) / (lam sqrt((1+eps)(1+eps+a))).

    Eq. "K for NASG" (Sec. 3.2) and its general form with epsilon (App. B).
    """
    return torch.log(2.0 * math.pi * (1.0 - torch.exp(-2.0 * lam))
                     / (lam * torch.sqrt((1.0 + eps) * (1.0 + eps + a))))


def euler_frame(ct, st, cp, sp, ctau, stau):
    """z and x of the orthonormal lobe frame from Euler-angle sines and cosines.

    Sec. 4.1 ("Parameterization of NASG"); y is completed as z x x.
    """
    z = torch.stack([cp * st, sp * st, ct], dim=-1)
    x = torch.stack([ct * cp * ctau - sp * stau,
                     ct * sp * ctau + cp * stau,
                     -st * ctau], dim=-1)
    y = torch.linalg.cross(z, x, dim=-1)
    return z, x, y


def decode(raw, n_lobes, eps=0.0, isotropic=False):
    """Raw network outputs [B, 8K] (or [B, 8K + 1]) -> Lobes (Tab. "decoding",
    Sec. 4.1).

    Raw order (reading): o[:, p*K + k] is parameter p of lobe k; a column
    8K, when present, is the selection probability (see ``selection``).
    cos/sin values: sigmoid(s0) * 2 - 1; lambda, a: exp(s1) (after the clamp);
    mixture weights: softmax over the K logits.
    isotropic: a = 0 for every lobe (the normalised spherical Gaussian that
    the paper compares NASG against, Sec. 6); the a outputs are ignored.
    """
    raw = torch.as_tensor(raw, dtype=F64)
    r = raw[:, :N_PARAM * n_lobes].reshape(raw.shape[0], N_PARAM, n_lobes)
    d = torch.sigmoid(r[:, 0:5, :]) * 2.0 - 1.0
    ct = d[:, 0]
    st = _SinFromCos.apply(ct)
    cp, sp = _unit_pair(d[:, 2], d[:, 1])
    ctau, stau = _unit_pair(d[:, 4], d[:, 3])
    z, x, y = euler_frame(ct, st, cp, sp, ctau, stau)
    lam = torch.exp(torch.clamp(r[:, 5], -LOG_CLAMP, LOG_CLAMP))
    a = torch.exp(torch.clamp(r[:, 6], -LOG_CLAMP, LOG_CLAMP))
    if isotropic:
        a = 0.0 * a   # zero value, zero gradient
    log_A = torch.log_softmax(r[:, 7], dim=-1)
    return Lobes(z=z, x=x, y=y, lam=lam, a=a, log_A=log_A,
                 log_K=log_normaliser(lam, a, eps), eps=float(eps))


def selection(raw, n_lobes):
    """Selection probability c = sigmoid(o[8K]) (Tab. "decoding"), [B]."""
    raw = torch.as_tensor(raw, dtype=F64)
    return torch.sigmoid(raw[:, N_PARAM * n_lobes])


def lobes_from_record(rec, eps=0.0):
    """Rebuild Lobes from a [B, K, 9] record (z, x, lambda, a, log(A/K)).

    The record carries log(A_k/K_k) only, so log_A holds that value and log_K
    is zero; mixture_log_pdf uses only the difference.
    """
    rec = torch.as_tensor(rec, dtype=F64)
    z = rec[..., 0:3]
    x = rec[..., 3:6]
    y = torch.linalg.cross(z, x, dim=-1)
    return Lobes(z=z, x=x, y=y, lam=rec[..., 6], a=rec[..., 7], log_A=rec[..., 8],
                 log_K=torch.zeros_like(rec[..., 8]), eps=float(eps))


def normalize_dirs(v):
    v = torch.as_tensor(v, dtype=F64)
    return v / torch.linalg.norm(v, dim=-1, keepdim=True)


def lobe_log_g(v, z, x, lam, a, eps=0.0):
    """log G(v; [x, y, z], lam, a, eps), the NASG lobe exactly as printed.

    Eq. NASG (Sec. 3.2), with epsilon from App. A (kappa = 1):
      u = (v.z + 1)/2,  e = eps + a (v.x)^2 / (1 - (v.z)^2),
      G = exp(2 lam u^{1+e} - 2 lam) u^{e};   G(z) = 1,  G(-z) = 0.
    v broadcasts against the lobe tensors ([B, 1, 3] against [B, K, 3]).
    """
    vz = (v * z).sum(-1)
    vx = (v * x).sum(-1)
    den = 1.0 - vz * vz
    pole = den <= 0.0
    den_safe = torch.where(pole, torch.ones_like(den), den)
    u = (vz + 1.0) / 2.0
    u_safe = torch.where(pole, torch.full_like(u, 0.5), u)
    e = eps + a * vx * vx / den_safe
    log_g = 2.0 * lam * u_safe ** (1.0 + e) - 2.0 * lam + e * torch.log(u_safe)
    at_z = torch.zeros_like(log_g)
    at_minus_z = torch.full_like(log_g, -math.inf)
    return torch.where(pole, torch.where(vz > 0, at_z, at_minus_z), log_g)


def component_log_terms(v, lobes):
    """log(A_k G_k(v) / K_k) for every lobe: [B, K]."""
    v = normalize_dirs(v)[:, None, :]
    log_g = lobe_log_g(v, lobes.z, lobes.x, lobes.lam, lobes.a, lobes.eps)
    return lobes.log_A - lobes.log_K + log_g


def mixture_log_pdf(v, lobes):
    """log D(v) with D = sum_k A_k G_k / K_k (Sec. 3.1), per steradian."""
    return torch.logsumexp(component_log_terms(v, lobes), dim=-1)


def log_pdf_direction_grad(v, lobes):
    """Gradient of log D with respect to the direction, on the sphere [B, 3].

    D is evaluated at v / |v| (as ``mixture_log_pdf`` does), so at a unit v
    the float64 autograd gradient is the tangential one, (I - v v^T) times
    the Euclidean gradient of any extension of log D off the sphere.
    """
    v = torch.as_tensor(v, dtype=F64).clone().requires_grad_(True)
    (g,) = torch.autograd.grad(mixture_log_pdf(v, lobes).sum(), v)
    return g.detach()


def choose_lobe(log_A, xi_sel):
    """Inverse-CDF choice of a mixture component (reading; the paper is silent).

    Smallest k with xi_sel < A_0 + ... + A_k; the last lobe with A_k > 0 when
    rounding leaves no such k.
    """
    A = torch.exp(torch.as_tensor(log_A, dtype=F64))
    cdf = torch.cumsum(A, dim=-1)
    xi = torch.as_tensor(xi_sel, dtype=F64)[:, None]
    below = xi < cdf
    K = A.shape[-1]
    idx = torch.arange(K).expand_as(cdf)
    first = torch.where(below, idx, torch.full_like(idx, K)).min(dim=-1).values
    last_pos = torch.where(A > 0, idx, torch.full_like(idx, -1)).max(dim=-1).values
    return torch.where(first < K, first, last_pos)


def sample_lobe(z, x, y, lam, a, xi0, xi1, xi2, eps=0.0):
    """One direction from a single normalised NASG lobe, App. C as printed.

    (xi0, xi1) map linearly onto (s, rho) in [e^{-2 lam}, 1] x [-pi/2, pi/2]:
    s = xi0 + (1 - xi0) e^{-2 lam}, rho = pi (xi1 - 1/2) (reading: increasing
    maps). Phi_E(s, rho) = (theta, phi) with
      theta = arccos(2 (log s / (2 lam) + 1)^{(1+eps+a - a cos^2 rho)/((1+eps)(1+eps+a))} - 1),
      phi   = arctan(sqrt((1+eps+a)/(1+eps)) tan rho);
    Phi_W adds pi to phi and is used when xi2 <= 1/2.
    The direction is sin(theta)(cos(phi) x + sin(phi) y) + cos(theta) z.
    """
    s = xi0 + (1.0 - xi0) * torch.exp(-2.0 * lam)
    rho = math.pi * (xi1 - 0.5)
    expo = (1.0 + eps + a - a * torch.cos(rho) ** 2) / ((1.0 + eps) * (1.0 + eps + a))
    theta = torch.arccos(2.0 * (torch.log(s) / (2.0 * lam) + 1.0) ** expo - 1.0)
    phi = torch.arctan(torch.sqrt((1.0 + eps + a) / (1.0 + eps)) * torch.tan(rho))
    phi = torch.where(xi2 > 0.5, phi, phi + math.pi)
    st = torch.sin(theta)
    return (st * torch.cos(phi))[:, None] * x + (st * torch.sin(phi))[:, None] * y \
        + torch.cos(theta)[:, None] * z


def sample(lobes, xi):
    """Sample one direction per vertex from the mixture; returns (v [B,3], lobe [B]).

    xi: [B, 4] uniforms (xi_sel, xi0, xi1, xi2), used as given.
    """
    xi = torch.as_tensor(xi, dtype=F64)
    k = choose_lobe(lobes.log_A - torch.logsumexp(lobes.log_A, -1, keepdim=True), xi[:, 0])
    rows = torch.arange(xi.shape[0])
    v = sample_lobe(lobes.z[rows, k], lobes.x[rows, k], lobes.y[rows, k],
                    lobes.lam[rows, k], lobes.a[rows, k],
                    xi[:, 1], xi[:, 2], xi[:, 3], lobes.eps)
    return v, k


def sample_from_record(rec, xi, eps=0.0):
    """Sampling from [B, K, 9] records: log(A/K) -> A via the closed-form K."""
    lobes = lobes_from_record(rec, eps)
    log_K = log_normaliser(lobes.lam, lobes.a, eps)
    full = Lobes(z=lobes.z, x=lobes.x, y=lobes.y, lam=lobes.lam, a=lobes.a,
                 log_A=lobes.log_A + log_K, log_K=log_K, eps=lobes.eps)
    return sample(full, xi)
