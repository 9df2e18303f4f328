"""GPU parity at the edges of the NASG method, against the extended-precision
oracle.

Records are built on the host over a grid of lobe parameters (lambda from
1e-3 to e^15, a from 0 to e^15, epsilon 0 and 0.3; eq. NASG, App. A, App. B)
and evaluated at directions within 1e-7 .. 1e-1 rad of a lobe's +z and -z, on
its y meridian and elsewhere, and sampled with extreme uniforms (App. C):
xi_sel in {0, 1/4, 1 - 2^-24}, xi0 in {0, 1e-3, 1/2, 0.999, 1 - 2^-24},
xi1 in {0, 1/4, 1/2, 1 - 2^-24}, xi2 in {1/2, 3/4}. Frames are either
uniformly oriented or along the coordinate axes (exactly orthonormal in
float32, so that directions near the axis keep full relative precision).

Every value is compared with the exact value at the kernel's own float32
inputs (``oracle.extended`` in x87 extended precision): the bound per vertex
is 1e-4 (on log q, the float32 pdf gate) plus the spread of the exact value
under perturbations of those inputs by four float32 units
(``tests.conditioning``). Sampled directions that lie within (K + 32)
float32 units of a CDF boundary of the lobe choice are left out (either
lobe is a correct choice there).
"""

import numpy as np
import pytest
import torch

from oracle import extended as ox
from tests import edge_inputs as E
from tests.conditioning import ULP, spread
from tests.helpers import bk9_to_rec, make_guide, to_dev

pytestmark = pytest.mark.gpu
K = 4
FLOOR = 1e-4
LOG_TINY = float(np.log(np.finfo(np.float32).tiny))   # below this a float32 pdf is subnormal or 0
MARGIN = (K + 32) * ULP


def _guide(eps):
    g, _ = make_guide("c1_f32", eps=eps, max_batch=1024)   # the record kernels need only K and eps
    return g


def _report(name, bad, cell, extra):
    idx = np.flatnonzero(bad)[:12]
    lines = [f"{name}: {int(bad.sum())} of {bad.size} outside the bound"]
    for i in idx:
        lam, a = E.LAMBDAS[cell[i, 0]], E.ECCS[cell[i, 1]]
        lines.append(f"  vertex {i} lambda {lam:.3g} a {a:.3g} " +
                     " ".join(f"{k} {float(v[i]):.4g}" for k, v in extra.items()))
    return "\n".join(lines)


def check_log_pdf(pdf_gpu, ref, tol, cell, name):
    """log of the kernel's float32 pdf against the exact log q: within tol
    where the pdf is a normal float32 number, below the normal range where
    the exact value is."""
    pdf_gpu = np.asarray(pdf_gpu, dtype=np.float64)
    with np.errstate(divide="ignore"):
        lg = np.log(pdf_gpu)
    normal = ref > LOG_TINY + tol
    err = np.abs(lg - ref)
    bad = normal & ~(err <= tol)
    tiny = ref < LOG_TINY - tol
    bad |= tiny & ~(pdf_gpu < 2 * np.finfo(np.float32).tiny)
    assert not bad.any(), _report(name, bad, cell, {"ref": ref, "gpu": lg, "tol": tol})
    return err[normal]


# -- GPU runs (also used by probes that store the outputs) ---------------------

def run_pdf(frames, eps):
    rec, dirs, cell = E.record_grid(K, eps, seed=901 if frames == "axis" else 902, frames=frames)
    g = _guide(eps)
    recd = to_dev(bk9_to_rec(rec, K))
    p, grad = g.pdf_grad(recd, to_dev(dirs.T))
    p2 = g.pdf(recd, to_dev(dirs.T))
    torch.cuda.synchronize()
    out = dict(rec=rec, dirs=dirs, cell=cell, pdf=p2.cpu().numpy(), pdf_g=p.cpu().numpy(),
               grad=grad.cpu().numpy().T)
    g.close()
    return out


def run_sample(frames, eps):
    rec, xi, cell = E.sample_grid(K, eps, seed=903 if frames == "axis" else 904, frames=frames)
    g = _guide(eps)
    d, p = g.sample(to_dev(bk9_to_rec(rec, K)), to_dev(np.ascontiguousarray(xi.T)))
    torch.cuda.synchronize()
    out = dict(rec=rec, xi=xi, cell=cell, dir=d.cpu().numpy().T, pdf=p.cpu().numpy())
    g.close()
    return out


# -- references ----------------------------------------------------------------

def log_pdf_fn(eps):
    return lambda r, v: ox.record_log_pdf(r, v, eps)


def dir_grad_fn(eps):
    return lambda r, v: ox.record_dir_grad(r, v, eps)


def check_pdf(out, eps, name):
    R, V = ox.ld(out["rec"]), ox.ld(out["dirs"])
    f = log_pdf_fn(eps)
    ref = f(R, V)
    tol = FLOOR + spread(f, [R, V])
    e1 = check_log_pdf(out["pdf"], ref, tol, out["cell"], name + " nasg_pdf")
    check_log_pdf(out["pdf_g"], ref, tol, out["cell"], name + " nasg_pdf_grad (pdf)")
    return e1


def on_an_axis(rec, dirs):
    """[B]: some lobe's axis is parallel to the direction or closer to it
    than ~5e-8 rad. At v = -z the epsilon = 0 lobe is discontinuous (G(-z)
    = 0), so log D has no gradient there; closer than ~5e-8 rad the
    extended-precision chain rule loses 1 - (v.z)^2."""
    R, V = ox.ld(rec), ox.ld(dirs)[:, None, :]
    z = R[..., 0:3]
    vu, zu, _ = ox.project(V + 0 * z, z, R[..., 3:6])
    vz = (vu * zu).sum(-1)
    return (ox.exact_pole(V, z) | (1 - np.abs(vz) < 1e-15)).any(-1)


def check_grad(out, eps, name):
    R, V = ox.ld(out["rec"]), ox.ld(out["dirs"])
    f = dir_grad_fn(eps)
    ref = np.asarray(f(R, V), dtype=np.float64)
    tol = FLOOR * (np.linalg.norm(ref, axis=1) + 1) + spread(f, [R, V], n_random=4)
    lq = log_pdf_fn(eps)(R, V)
    live = (lq > LOG_TINY) & ~on_an_axis(out["rec"], out["dirs"])   # a normal float32 pdf, off the axes
    err = np.linalg.norm(out["grad"] - ref, axis=1)
    bad = live & ~(err <= tol)
    assert not bad.any(), _report(name + " nasg_pdf_grad", bad, out["cell"],
                                  {"|ref|": np.linalg.norm(ref, axis=1), "err": err, "tol": tol})
    return err[live] / tol[live]


def check_sample(out, eps, name):
    R, XI = ox.ld(out["rec"]), ox.ld(out["xi"])
    fixed = XI[:, [0, 3]]            # xi_sel and xi2 decide (lobe, east/west); they are not perturbed

    def fdir(r, x12):
        xi = np.stack([fixed[:, 0], x12[:, 0], x12[:, 1], fixed[:, 1]], -1)
        return ox.record_sample(r, xi, eps)[0]

    v_ref, _, margin = ox.record_sample(R, XI, eps)
    ok = margin > MARGIN
    tol = FLOOR + spread(fdir, [R, XI[:, 1:3]])
    err = np.linalg.norm(out["dir"] - np.asarray(v_ref, dtype=np.float64), axis=1)
    bad = ok & ~(err <= tol)
    assert not bad.any(), _report(name + " nasg_sample direction", bad, out["cell"], {"err": err, "tol": tol})
    # the pdf returned with each sample, at the kernel's own direction
    D = ox.ld(out["dir"])
    f = log_pdf_fn(eps)
    ref = f(R, D)
    check_log_pdf(out["pdf"], ref, FLOOR + spread(f, [R, D]), out["cell"], name + " nasg_sample pdf")
    return int((~ok).sum())


@pytest.mark.parametrize("eps", [0.0, 0.3])
@pytest.mark.parametrize("frames", ["axis", "random"])
def test_pdf_and_direction_gradient_at_edges(frames, eps):
    out = run_pdf(frames, eps)
    check_pdf(out, eps, f"{frames} eps={eps}")
    check_grad(out, eps, f"{frames} eps={eps}")


@pytest.mark.parametrize("eps", [0.0, 0.3])
@pytest.mark.parametrize("frames", ["axis", "random"])
def test_sample_at_edges(frames, eps):
    out = run_sample(frames, eps)
    excluded = check_sample(out, eps, f"{frames} eps={eps}")
    assert excluded <= 0.02 * len(out["xi"])
