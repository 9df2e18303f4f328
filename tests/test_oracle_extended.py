"""Pins of the extended-precision oracle (``oracle.extended``).

It evaluates the same literal formulas as the FP64 oracle, so it is pinned
(1) to the FP64 oracle where float64 is accurate (moderate parameters and
angles), (2) to closed forms the lobe reduces to, evaluated from the angle
directly, at the extremes where the literal formula cancels (a = 0: the
von Mises-Fisher lobe of eq. SG; the x and y meridians, where the anisotropy
weight is 1 and 0; the poles of eq. NASG; the polar law of the isotropic
sampler), and (3) to the same formula in mpmath at 60 digits, which checks
that x87 extended precision carries it at e^15 sharpness.
"""

import math

import mpmath
import numpy as np
import pytest
import torch

from oracle import extended as ox
from oracle import nasg as onasg
from paper_2303_08064_amd import synth
from tests import edge_inputs as E

F64 = torch.float64
LD = ox.LD


def close(got, ref):
    """|got - ref| <= 1e-6 max(1, |ref|): 100 times below the 1e-4 floor of
    the GPU gates that use this oracle as their reference."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    assert np.all(np.abs(got - ref) <= 1e-6 * np.maximum(1.0, np.abs(ref))), (got, ref)


def _moderate_records(n, K, seed, eps=0.0):
    rng = synth.rng_for(seed)
    lam = np.exp(rng.uniform(-3, 5, n))
    a = np.exp(rng.uniform(-3, 5, n))
    return E.records(lam, a, K, rng, eps, dominant=False), rng


@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_agrees_with_fp64_oracle_at_moderate_inputs(eps):
    K = 4
    rec, rng = _moderate_records(400, K, 1, eps)
    dirs = synth.unit_vectors(400, rng)
    # decode: raw outputs of moderate size
    raw = rng.normal(0.0, 2.0, (400, 8 * K))
    z, x, lam, a, log_A, log_K = ox.decode(raw, K, eps)
    lob = onasg.decode(torch.tensor(raw), K, eps)
    for got, ref in ((z, lob.z), (x, lob.x), (lam, lob.lam), (a, lob.a), (log_A, lob.log_A), (log_K, lob.log_K)):
        np.testing.assert_allclose(np.asarray(got, np.float64), ref.numpy(), rtol=1e-12, atol=1e-13)
    # mixture pdf from raw outputs and from records (frames orthonormalised
    # for the FP64 oracle exactly as ``project`` does)
    lq = ox.decoded_log_pdf(raw, K, dirs, eps)
    np.testing.assert_allclose(np.asarray(lq, np.float64),
                               onasg.mixture_log_pdf(torch.tensor(dirs), lob).numpy(), rtol=1e-11, atol=1e-11)
    R = ox.ld(rec)
    _, zu, xu = ox.project(None, R[..., 0:3], R[..., 3:6])
    R64 = rec.astype(np.float64)
    R64[..., 0:3], R64[..., 3:6] = np.asarray(zu, np.float64), np.asarray(xu, np.float64)
    lob_r = onasg.lobes_from_record(torch.tensor(R64), eps)
    d32 = dirs.astype(np.float32).astype(np.float64)
    np.testing.assert_allclose(np.asarray(ox.record_log_pdf(rec, d32, eps), np.float64),
                               onasg.mixture_log_pdf(torch.tensor(d32), lob_r).numpy(), rtol=1e-11, atol=1e-11)
    # direction gradient against the FP64 oracle's autograd, both at the unit
    # direction (autograd of log D(v / |v|) at a non-unit v carries 1/|v|)
    g = np.asarray(ox.record_dir_grad(rec, d32, eps), np.float64)
    du = d32 / np.linalg.norm(d32, axis=1, keepdims=True)
    gr = onasg.log_pdf_direction_grad(torch.tensor(du), lob_r).numpy()
    assert np.max(np.linalg.norm(g - gr, axis=1) / (np.linalg.norm(gr, axis=1) + 1)) < 1e-9
    # sampling: same lobe and direction as the FP64 oracle's record sampler
    xi = rng.uniform(0.01, 0.99, (400, 4))
    v, k, _ = ox.record_sample(R64, xi, eps)
    v2, k2 = onasg.sample_from_record(torch.tensor(R64), torch.tensor(xi), eps)
    assert np.array_equal(k, k2.numpy())
    np.testing.assert_allclose(np.asarray(v, np.float64), v2.numpy(), atol=1e-10)


def _axis_lobe(theta, psi):
    """v at polar angle theta from z = e_z, azimuth psi from x = e_x, and the
    frame, in extended precision."""
    theta, psi = ox.ld(theta), ox.ld(psi)
    v = np.stack([np.sin(theta) * np.cos(psi), np.sin(theta) * np.sin(psi), np.cos(theta)], -1)
    z = np.zeros_like(v)
    z[..., 2] = 1
    x = np.zeros_like(v)
    x[..., 0] = 1
    return v, z, x


LAMS = [1e-3, 1.0, 1e4, math.exp(15.0)]
THETAS = [1e-7, 1e-4, 0.1, 1.0, 3.0, math.pi - 1e-6]


@pytest.mark.parametrize("lam", LAMS)
def test_isotropic_lobe_closed_form_at_extremes(lam):
    """a = 0, eps = 0: log G = 2 lam (cos^2(theta/2) - 1) = -2 lam sin^2(theta/2)
    (the von Mises-Fisher lobe), from the angle, without cancellation."""
    th = np.array(THETAS)
    v, z, x = _axis_lobe(th, np.full_like(th, 0.7))
    got = ox.lobe_log_g(v, z, x, ox.ld(lam), ox.ld(0.0))
    ref = -2 * ox.ld(lam) * np.sin(ox.ld(th) / 2) ** 2
    close(got, ref)


@pytest.mark.parametrize("lam", LAMS)
@pytest.mark.parametrize("a", [1e-3, 1.0, 1e3, math.exp(15.0)])
@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_meridian_closed_forms_at_extremes(lam, a, eps):
    """On the x meridian c^2 = 1, e = eps + a; on the y meridian c^2 = 0,
    e = eps. With u = cos^2(theta/2): log G = 2 lam (u^{1+e} - 1) + e log u,
    evaluated from theta as 2 lam expm1((1+e) log u) + e log u with
    log u = 2 log cos(theta/2)."""
    th = ox.ld(np.array(THETAS))
    lu = 2 * np.log(np.cos(th / 2))
    for psi, e in ((0.0, eps + a), (math.pi / 2, eps)):
        v, z, x = _axis_lobe(th, np.full(th.shape, psi))
        if psi:          # the y meridian exactly: v has no x component
            v[:, 0] = 0
        got = ox.lobe_log_g(v, z, x, ox.ld(lam), ox.ld(a), eps)
        ref = 2 * ox.ld(lam) * np.expm1((1 + e) * lu) + e * lu
        close(got, ref)


def test_poles_are_exact():
    """G(z) = 1 and G(-z) = 0 (eq. NASG) for stored float32 values: v
    parallel to z is recognised from the exact cross product, however the
    stored frame rounds."""
    rng = synth.rng_for(3)
    z, x = E.random_frames(64, rng)
    z32, x32 = z.astype(np.float32), x.astype(np.float32)
    for sign, ref in ((1.0, 0.0), (-1.0, -np.inf)):
        v = (sign * z32)[:, None, :]
        lg = ox.stored_log_g(ox.ld(v), ox.ld(z32[:, None]), ox.ld(x32[:, None]), ox.ld(np.full((64, 1), 50.0)),
                             ox.ld(np.full((64, 1), 3.0)))
        assert np.all(np.asarray(lg, np.float64) == ref)
    assert not ox.exact_pole(np.float32([[0.0, 1e-30, 1.0]]), np.float32([[0.0, 0.0, 1.0]]))[0]


def _mp_lobe(v, z, x, lam, a, eps):
    with mpmath.workdps(60):
        V = [mpmath.mpf(float(t)) for t in v]
        Z = [mpmath.mpf(float(t)) for t in z]
        X = [mpmath.mpf(float(t)) for t in x]
        nv = mpmath.sqrt(sum(t * t for t in V))
        nz = mpmath.sqrt(sum(t * t for t in Z))
        V, Z = [t / nv for t in V], [t / nz for t in Z]
        xz = sum(p * q for p, q in zip(X, Z))
        X = [p - xz * q for p, q in zip(X, Z)]
        nx = mpmath.sqrt(sum(t * t for t in X))
        X = [t / nx for t in X]
        vz = sum(p * q for p, q in zip(V, Z))
        vx = sum(p * q for p, q in zip(V, X))
        u = (vz + 1) / 2
        e = eps + mpmath.mpf(float(a)) * vx * vx / (1 - vz * vz)
        lam = mpmath.mpf(float(lam))
        return float(2 * lam * u ** (1 + e) - 2 * lam + e * mpmath.log(u))


def test_extended_precision_carries_the_literal_formula():
    """The edge grid's sharpest cells (lambda, a up to e^15) at directions down
    to 1e-7 rad from the axis: extended precision agrees with 60-digit
    mpmath on the same formula to 1e-6 absolute (the float32 inputs are the
    same; only the working precision differs)."""
    rec, dirs, cell = E.record_grid(4, 0.0, seed=905, frames="axis")
    pick = (cell[:, 0] >= 5) & (cell[:, 1] >= 3)         # lambda >= 1e3, a >= 1e2
    idx = np.flatnonzero(pick)[::7]
    got = ox.stored_log_g(ox.ld(dirs[idx])[:, None, :], ox.ld(rec[idx, :1, 0:3]), ox.ld(rec[idx, :1, 3:6]),
                          ox.ld(rec[idx, :1, 6]), ox.ld(rec[idx, :1, 7]))[:, 0]
    for j, i in enumerate(idx):
        if ox.exact_pole(dirs[i][None], rec[i, 0, 0:3][None])[0]:
            continue
        ref = _mp_lobe(dirs[i], rec[i, 0, 0:3], rec[i, 0, 3:6], rec[i, 0, 6], rec[i, 0, 7], 0.0)
        assert abs(float(got[j]) - ref) <= 1e-6 * max(1.0, abs(ref)), (i, float(got[j]), ref)


@pytest.mark.parametrize("lam", [1e-3, 1.0, 1e4, math.exp(15.0)])
def test_isotropic_sampler_polar_law_at_extremes(lam):
    """a = 0: the App. C map reduces to cos theta = 1 + log(s) / lam with
    s = xi0 + (1 - xi0) e^{-2 lam} (the von Mises-Fisher inverse CDF), here
    as 1 - cos theta = -log(s) / lam with log s = logaddexp(log xi0,
    log(1 - xi0) - 2 lam), near both ends of xi0."""
    xi0 = ox.ld(np.array([0.0, 1e-12, 1e-3, 0.5, 0.999, 1.0 - 2.0 ** -24]))
    n = len(xi0)
    z = np.zeros((n, 3), dtype=LD)
    z[:, 2] = 1
    x = np.zeros((n, 3), dtype=LD)
    x[:, 0] = 1
    L = ox.ld(np.full(n, lam))
    v = ox.sample_lobe(z, x, L, ox.ld(np.zeros(n)), xi0, ox.ld(np.full(n, 0.3)), ox.ld(np.full(n, 0.7)))
    with np.errstate(divide="ignore"):
        one_m_ct = -np.logaddexp(np.log(xi0), np.log1p(-xi0) - 2 * L) / L
    # 1 - cos theta from the returned direction without cancellation: |v - z|^2 / 2
    got = ((v - z) ** 2).sum(-1) / 2
    np.testing.assert_allclose(np.asarray(got, np.float64), np.asarray(one_m_ct, np.float64), rtol=1e-6,
                               atol=1e-18)


def test_sampler_tangent_limit_at_xi1_zero():
    """xi1 = 0 is rho = -pi/2: tan(rho) -> -inf, phi = -pi/2 in the eastern
    map (v along -y), +pi/2 in the western one."""
    n = 2
    z = np.zeros((n, 3), dtype=LD)
    z[:, 2] = 1
    x = np.zeros((n, 3), dtype=LD)
    x[:, 0] = 1
    v = ox.sample_lobe(z, x, ox.ld([5.0, 5.0]), ox.ld([2.0, 2.0]), ox.ld([0.5, 0.5]), ox.ld([0.0, 0.0]),
                       ox.ld([0.75, 0.25]))
    v = np.asarray(v, np.float64)
    assert abs(v[0, 0]) < 1e-15 and v[0, 1] < 0 and abs(v[1, 0]) < 1e-15 and v[1, 1] > 0
