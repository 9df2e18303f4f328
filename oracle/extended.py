"""NASG decode, lobe, normaliser, mixture and App. C sampler in extended
precision (oracle).

Test infrastructure only (see the package docstring). These are the same
literal formulas as ``oracle.nasg`` -- nothing is rewritten into a stable
form -- written in NumPy so that they can be evaluated in the host's x87
extended precision (``np.longdouble``: 64-bit significand, unit roundoff
5.4e-20) as well as in float64. The extra 11 bits over float64 keep the
literal forms accurate where float64 loses them: 1 - (v.z)^2 and
u^(1+e) - 1 within 1e-7 rad of a lobe axis, the -2 lambda + 2 lambda u^(1+e)
cancellation at lambda ~ e^15, and sigmoid(o) * 2 - 1 near +-1 for |o| ~ 40.
Every function keeps the dtype of its inputs (pass ``ld(...)`` arrays).

Shapes: B vertices, K lobes; directions [B, 3], per-lobe arrays [B, K] or
[B, K, 3].

A record or decoded frame stored in float32 is only approximately
orthonormal; the lobe of eq. NASG is defined on orthonormal frames and unit
directions, so ``project`` maps (v, z, x) to the unit v, the unit z and the
part of x orthogonal to z (Gram-Schmidt) before evaluation.

The poles v = +-z are special cases of eq. NASG (G(z) = 1, G(-z) = 0). For
stored values they are decided exactly: v is at a pole when v x z = 0, and
each component of that cross product, a difference of two products of
float32 numbers, is exact in extended precision. Where extended precision
does not carry the literal formula to 1e-7 -- the rounding of u = (v.z + 1)/2
(about 1e-19) magnified by e / u in e log u near -z and by 2 lam (1 + e) in
2 lam u^{1+e} near +z, or 1 - (v.z)^2 unresolved within ~1e-8 rad of the
axis -- the lobe is evaluated by the same literal formula in mpmath at 80
digits.
"""

import functools

import mpmath
import numpy as np

LD = np.longdouble
PI = LD("3.14159265358979323846264338327950288")
LOG_CLAMP = 15.0     # reading: log lambda and log a are clamped to [-15, 15]
N_PARAM = 8          # per lobe: cos th, sin ph, cos ph, sin tau, cos tau, log lam, log a, logit


def ld(a):
    """An array in extended precision (exact for float32/float64 inputs)."""
    return np.asarray(a, dtype=LD)


def _dot(a, b):
    return (a * b).sum(-1)


def _unit(v):
    return v / np.sqrt(_dot(v, v))[..., None]


def project(v, z, x):
    """Unit direction and orthonormal (z, x) from stored values: v / |v|,
    z / |z|, and x minus its z component, normalised (Gram-Schmidt)."""
    zu = _unit(z)
    xo = x - _dot(x, zu)[..., None] * zu
    return (None if v is None else _unit(v)), zu, _unit(xo)


def log_normaliser(lam, a, eps=0.0):
    """log K, K = 2 pi (1 - e^{-2 lam}) / (lam sqrt((1+eps)(1+eps+a))).
    Eq. "K for NASG" (Sec. 3.2) and its epsilon form (App. B)."""
    one = np.ones_like(lam)
    return np.log(2 * PI * (one - np.exp(-2 * lam)) / (lam * np.sqrt((1 + eps) * (1 + eps + a))))


def lobe_log_g(v, z, x, lam, a, eps=0.0, pole=None):
    """log G(v) for a unit v and an orthonormal frame, as printed: eq. NASG
    (Sec. 3.2) with the epsilon of App. A (kappa = 1):
      u = (v.z + 1)/2,  e = eps + a (v.x)^2 / (1 - (v.z)^2),
      log G = 2 lam u^{1+e} - 2 lam + e log u;  G(z) = 1, G(-z) = 0.
    pole: where v = +-z (default: where 1 - (v.z)^2 <= 0)."""
    vz = _dot(v, z)
    vx = _dot(v, x)
    den = 1 - vz * vz
    if pole is None:
        pole = den <= 0
    pole = pole | (den <= 0)
    den_s = np.where(pole, 1, den)
    u = (vz + 1) / 2
    u_s = np.where(pole, 0.5, u)
    e = eps + a * vx * vx / den_s
    with np.errstate(divide="ignore"):
        lg = 2 * lam * u_s ** (1 + e) - 2 * lam + e * np.log(u_s)
    return np.where(pole, np.where(vz > 0, 0, -np.inf), lg)


def exact_pole(v, z):
    """Where the stored float32 direction v is parallel to the stored axis z
    (v x z = 0, exact in extended precision for float32 inputs)."""
    c = np.cross(ld(v), ld(z))
    return (c == 0).all(-1)


def _lobe_log_g_mp(v, z, x, lam, a, eps, dps=80):
    """One lobe value by the literal formula in mpmath (stored values in,
    projection included)."""
    return _lobe_log_g_mp_cached(tuple(float(t) for t in v), tuple(float(t) for t in z),
                                 tuple(float(t) for t in x), float(lam), float(a), float(eps), dps)


@functools.lru_cache(maxsize=1 << 16)
def _lobe_log_g_mp_cached(v, z, x, lam, a, eps, dps):
    with mpmath.workdps(dps):
        V = [mpmath.mpf(t) for t in v]
        Z = [mpmath.mpf(t) for t in z]
        X = [mpmath.mpf(t) for t in x]
        nv = mpmath.sqrt(sum(t * t for t in V))
        nz = mpmath.sqrt(sum(t * t for t in Z))
        V = [t / nv for t in V]
        Z = [t / nz for t in Z]
        xz = sum(p * q for p, q in zip(X, Z))
        X = [p - xz * q for p, q in zip(X, Z)]
        nx = mpmath.sqrt(sum(t * t for t in X))
        X = [t / nx for t in X]
        vz = sum(p * q for p, q in zip(V, Z))
        vx = sum(p * q for p, q in zip(V, X))
        lam, a = mpmath.mpf(lam), mpmath.mpf(a)
        den = 1 - vz * vz
        u = (vz + 1) / 2
        e = eps + a * vx * vx / den
        return LD(mpmath.nstr(2 * lam * u ** (1 + e) - 2 * lam + e * mpmath.log(u), 30))


def stored_log_g(v, z, x, lam, a, eps=0.0):
    """log G at stored (float32) directions v [B, 1, 3] or [B, K, 3] and
    stored frames z, x [B, K, 3]: exact poles, the literal formula in
    extended precision after ``project``, and mpmath where the axis is too
    close to v for extended precision."""
    pole = exact_pole(v, z)
    vu, zu, xu = project(ld(v) + 0 * ld(z), ld(z), ld(x))
    lg = lobe_log_g(vu, zu, xu, lam, a, eps, pole)
    vz = _dot(vu, zu)
    vx = _dot(vu, xu)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = (vz + 1) / 2
        e = np.abs(eps + a * vx * vx / (1 - vz * vz))
        err = 1.1e-19 * (e / u + 2 * lam * (1 + e))
    near = ~pole & ((1 - np.abs(vz) < 1e-15) | ~(err <= 1e-7))
    if near.any():
        vb = np.broadcast_to(np.asarray(v), z.shape)
        lamb = np.broadcast_to(lam, vz.shape)
        ab = np.broadcast_to(a, vz.shape)
        for idx in zip(*np.nonzero(near)):
            lg[idx] = _lobe_log_g_mp(vb[idx], z[idx], x[idx], lamb[idx], ab[idx], eps)
    return lg


def decode(raw, K, eps=0.0):
    """Raw outputs [B, 8K (+1)] -> (z, x, lam, a, log_A, log_K), Tab.
    "decoding" and the Euler frame of Sec. 4.1, with the readings of
    ``oracle.nasg.decode`` (parameter-major order; cos/sin = sigmoid * 2 - 1;
    sin theta = sqrt(1 - cos^2); (cos, sin) pairs divided by their norm, a
    zero pair -> (1, 0); log lambda, log a clamped to [-15, 15]; softmax
    mixture weights)."""
    raw = np.asarray(raw)
    r = raw[:, :N_PARAM * K].reshape(raw.shape[0], N_PARAM, K)
    d = 2 / (1 + np.exp(-r[:, 0:5])) - 1
    ct = d[:, 0]
    st = np.sqrt(np.maximum(1 - ct * ct, 0))

    def pair(c, s):
        ok = c * c + s * s > 0
        c1, s1 = np.where(ok, c, 1), np.where(ok, s, 0)
        n = np.sqrt(c1 * c1 + s1 * s1)
        return c1 / n, s1 / n

    cp, sp = pair(d[:, 2], d[:, 1])
    ctau, stau = pair(d[:, 4], d[:, 3])
    z = np.stack([cp * st, sp * st, ct], -1)
    x = np.stack([ct * cp * ctau - sp * stau, ct * sp * ctau + cp * stau, -st * ctau], -1)
    lam = np.exp(np.clip(r[:, 5], -LOG_CLAMP, LOG_CLAMP))
    a = np.exp(np.clip(r[:, 6], -LOG_CLAMP, LOG_CLAMP))
    al = r[:, 7]
    m = al.max(-1, keepdims=True)
    log_A = al - m - np.log(np.exp(al - m).sum(-1, keepdims=True))
    return z, x, lam, a, log_A, log_normaliser(lam, a, eps)


def _lse(t):
    m = t.max(-1, keepdims=True)
    mf = np.where(np.isfinite(m), m, 0)
    with np.errstate(divide="ignore"):
        return (mf + np.log(np.exp(t - mf).sum(-1, keepdims=True)))[..., 0]


def mixture_log_pdf(v, z, x, lam, a, log_c, eps=0.0):
    """log D(v) = log sum_k c_k G_k(v), c_k = A_k / K_k (Sec. 3.1), for a unit
    v [B, 3] and lobes [B, K, ...]."""
    return _lse(log_c + lobe_log_g(v[:, None, :], z, x, lam, a, eps))


def record_log_pdf(rec, v, eps=0.0):
    """log D at stored directions v [B, 3] from stored records [B, K, 9] (z,
    x, lambda, a, log(A/K)): log sum_k c_k G_k(v) with ``stored_log_g``."""
    rec = ld(rec)
    lg = stored_log_g(ld(v)[:, None, :], rec[..., 0:3], rec[..., 3:6], rec[..., 6], rec[..., 7], eps)
    return _lse(rec[..., 8] + lg)


def lobe_dir_grad(v, z, x, lam, a, eps=0.0):
    """Gradient on the sphere of log G at a unit v (orthonormal frame), by
    the chain rule of the literal formula of ``lobe_log_g``, which depends
    on v only through v.z and v.x:
      d log G / d(v.z) = 2 lam u^{1+e} ((1+e)/(2u) + log u de/d(v.z))
                         + log u de/d(v.z) + e/(2u),
      d log G / d(v.x) = (2 lam u^{1+e} + 1) log u de/d(v.x),
    with de/d(v.z) = 2 a (v.x)^2 (v.z) / (1 - (v.z)^2)^2 and de/d(v.x) =
    2 a (v.x) / (1 - (v.z)^2); each partial multiplies the tangential part
    a - (v.a) v of its axis. Zero at the poles v = +-z."""
    vz = _dot(v, z)
    vx = _dot(v, x)
    den = 1 - vz * vz
    pole = den <= 0
    den_s = np.where(pole, 1, den)
    u = np.where(pole, 0.5, (vz + 1) / 2)
    e = eps + a * vx * vx / den_s
    de_z = 2 * a * vx * vx * vz / (den_s * den_s)
    de_x = 2 * a * vx / den_s
    lu = np.log(u)
    ue = u ** (1 + e)
    gz = 2 * lam * ue * ((1 + e) / (2 * u) + lu * de_z) + lu * de_z + e / (2 * u)
    gx = (2 * lam * ue + 1) * lu * de_x
    gz, gx = np.where(pole, 0, gz), np.where(pole, 0, gx)
    return gz[..., None] * (z - vz[..., None] * v) + gx[..., None] * (x - vx[..., None] * v)


def record_dir_grad(rec, v, eps=0.0):
    """Gradient on the sphere of log D at stored directions v [B, 3] from
    stored records [B, K, 9]: sum_k r_k grad log G_k with the lobes'
    responsibilities r_k = c_k G_k / D (``lobe_dir_grad`` after
    ``project``)."""
    rec = ld(rec)
    V = ld(v)[:, None, :]
    z, x = rec[..., 0:3], rec[..., 3:6]
    lg = stored_log_g(V, z, x, rec[..., 6], rec[..., 7], eps)
    ell = rec[..., 8] + lg
    with np.errstate(invalid="ignore"):
        r = np.exp(ell - _lse(ell)[:, None])
    r = np.where(np.isfinite(r), r, 0)
    vu, zu, xu = project(V + 0 * z, z, x)
    g = lobe_dir_grad(vu, zu, xu, rec[..., 6], rec[..., 7], eps)
    return (r[..., None] * g).sum(1)


def choose_lobe(A, xi_sel):
    """Inverse CDF over the mixture weights A [B, K] in lobe order: the
    smallest k with xi_sel * sum(A) < A_0 + ... + A_k (reading). Returns the
    index and the distance of xi_sel * sum(A) to the nearest boundary that
    decides the choice (A_0 + ... + A_k for k < K - 1), relative to sum(A)."""
    cdf = np.cumsum(A, -1)
    tot = cdf[:, -1:]
    t = ld(xi_sel)[:, None] * tot
    K = A.shape[-1]
    first = np.where(t < cdf, np.arange(K), K).min(-1)
    last = np.where(A > 0, np.arange(K), -1).max(-1)
    k = np.where(first < K, first, last)
    if K > 1:
        margin = np.abs(cdf[:, :-1] - t).min(-1) / tot[:, 0]
    else:
        margin = np.full(A.shape[0], np.inf)
    return k, margin


def sample_lobe(z, x, lam, a, xi0, xi1, xi2, eps=0.0):
    """One direction from one lobe, App. C as printed: s = xi0 + (1 - xi0)
    e^{-2 lam}, rho = pi (xi1 - 1/2) (reading: increasing maps),
      theta = arccos(2 (log s / (2 lam) + 1)^{(1+eps+a - a cos^2 rho) / ((1+eps)(1+eps+a))} - 1),
      phi = arctan(sqrt((1+eps+a)/(1+eps)) tan rho), + pi when xi2 <= 1/2,
    v = sin(theta)(cos(phi) x + sin(phi) y) + cos(theta) z, y = z x x."""
    y = np.cross(z, x)
    s = xi0 + (1 - xi0) * np.exp(-2 * lam)
    rho = PI * (xi1 - LD(0.5))
    expo = (1 + eps + a - a * np.cos(rho) ** 2) / ((1 + eps) * (1 + eps + a))
    with np.errstate(divide="ignore", invalid="ignore"):
        base = np.maximum(np.log(s) / (2 * lam) + 1, 0)
        theta = np.arccos(np.clip(2 * base ** expo - 1, -1, 1))
    # rho = -pi/2 exactly at xi1 = 0: tan rho is -inf there (a rounded pi/2
    # can land on either side of the pole of tan)
    tan_rho = np.where(xi1 == 0, -np.inf, np.tan(rho))
    phi = np.arctan(np.sqrt((1 + eps + a) / (1 + eps)) * tan_rho)
    phi = np.where(xi2 > 0.5, phi, phi + PI)
    st = np.sin(theta)
    return ((st * np.cos(phi))[:, None] * x + (st * np.sin(phi))[:, None] * y
            + np.cos(theta)[:, None] * z)


def record_sample(rec, xi, eps=0.0):
    """Sample one direction per vertex from records [B, K, 9] with uniforms
    xi [B, 4] = (xi_sel, xi0, xi1, xi2): A_k = exp(log(A_k/K_k) + log K_k)
    with K_k in closed form, the inverse-CDF choice, then the lobe's App. C
    map. Returns (v [B, 3], lobe [B], CDF margin [B])."""
    rec, xi = ld(rec), ld(xi)
    _, z, x = project(None, rec[..., 0:3], rec[..., 3:6])
    lam, a = rec[..., 6], rec[..., 7]
    A = np.exp(rec[..., 8] + log_normaliser(lam, a, eps))
    k, margin = choose_lobe(A, xi[:, 0])
    i = np.arange(rec.shape[0])
    v = sample_lobe(z[i, k], x[i, k], lam[i, k], a[i, k], xi[:, 1], xi[:, 2], xi[:, 3], eps)
    return v, k, margin


def decoded_sample(raw, K, xi, eps=0.0):
    """Sample from decoded raw outputs [B, 8K (+1)] (``decode``), as
    ``record_sample`` does from records. Returns (v, lobe, margin)."""
    z, x, lam, a, log_A, _ = decode(ld(raw), K, eps)
    xi = ld(xi)
    k, margin = choose_lobe(np.exp(log_A), xi[:, 0])
    i = np.arange(z.shape[0])
    v = sample_lobe(z[i, k], x[i, k], lam[i, k], a[i, k], xi[:, 1], xi[:, 2], xi[:, 3], eps)
    return v, k, margin


def decoded_log_pdf(raw, K, v, eps=0.0):
    """log D at directions v [B, 3] from raw outputs [B, 8K (+1)]."""
    z, x, lam, a, log_A, log_K = decode(ld(raw), K, eps)
    return mixture_log_pdf(_unit(ld(v)), z, x, lam, a, log_A - log_K, eps)
