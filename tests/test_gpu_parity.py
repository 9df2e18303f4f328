"""HIP path vs the FP64 oracle on identical seeded inputs (through the C ABI).

Tolerances (FP32 path vs the FP64 oracle):
* MLP raw outputs: per-vertex ||d||/||row|| <= 1e-5 (FP32 accumulation of 64-wide dots);
* decoded records from the GPU's own raw outputs: z, x abs <= 1e-6; lambda, a
  rel <= 1e-5; log(A/K) abs <= 1e-5;
* mixture pdf: |d log q| <= 1e-4 (1e-4 relative), directions within 1e-3 rad
  of a -z_k with a_k > 0 excluded (the eps = 0 lobe is discontinuous there);
* end to end from the features (records and pdf): the same bounds plus the
  change of the exact value when the raw outputs move by the float32
  forward's rounding, per entry; the well-conditioned vertices meet the
  stage-wise bounds;
* sampled direction: |dv| <= 1e-4, vertices whose xi_sel lies within 1e-5 of
  a CDF boundary excluded (either lobe is then a correct choice);
* loss: rel <= 1e-5;
* weight gradients entry by entry: tests/test_gpu_gradients.py.
BF16 (operands rounded to bfloat16, FP32 accumulation) is compared with the
oracle's BF16 emulation; its bounds are stated at each test.
"""

import math

import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from oracle import nasg as onasg
from oracle import train as otrain
from paper_2303_08064_amd import synth
from tests import grad_check as GC
from tests.helpers import CONFIGS, bk9_to_rec, make_guide, rec_to_bk9, to_dev

pytestmark = pytest.mark.gpu

B_RAGGED = 1000      # not a multiple of 16 or 64: several tiles and a ragged tail
F64 = torch.float64


def w64(mats):
    return [torch.tensor(m, dtype=F64) for m in mats]


def inputs(B, seed):
    rng = synth.rng_for(seed)
    return synth.features(B, rng), synth.uniforms(B, rng)


def near_minus_z(v, lobes, tol=1e-3):
    """[B] mask: v within tol rad of -z_k for a lobe with a_k > 0."""
    v = torch.as_tensor(v, dtype=F64)[:, None, :]
    d = (v * lobes.z).sum(-1)
    return ((d < -math.cos(tol)) & (lobes.a > 0)).any(-1).numpy()


def cdf_margin(lobes, xi_sel):
    A = torch.exp(lobes.log_A - torch.logsumexp(lobes.log_A, -1, keepdim=True))
    C = torch.cumsum(A, -1)
    return torch.abs(C - torch.as_tensor(xi_sel, dtype=F64)[:, None]).min(-1).values.numpy()


@pytest.mark.parametrize("name", ["c1_f32", "c2_f32", "c3_f32", "c5_f32"])
def test_forward_raw_f32(name):
    g, mats = make_guide(name, out_scale=3.0)
    feat, _ = inputs(B_RAGGED, 1)
    raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
    ref = omlp.forward(w64(mats), feat.T).numpy()
    err = np.linalg.norm(raw - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() < 1e-5, err.max()


@pytest.mark.parametrize("name", ["c1_bf16", "c2_bf16", "c3_bf16", "c5_bf16"])
def test_forward_raw_bf16(name):
    """Against the oracle's BF16 emulation: 99.9% of outputs within 1e-4 of the
    row's max magnitude, all within 2e-2 (a hidden activation whose FP32 sum
    lands on the other side of a BF16 rounding boundary moves one ulp)."""
    g, mats = make_guide(name, out_scale=3.0)
    feat, _ = inputs(B_RAGGED, 2)
    raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
    ref = omlp.forward(w64(mats), feat.T, bf16=True).numpy()
    scale = np.abs(ref).max(axis=1, keepdims=True)
    rel = np.abs(raw - ref) / scale
    assert np.mean(rel < 1e-4) >= 0.999, np.mean(rel < 1e-4)
    assert rel.max() < 2e-2, rel.max()


def _gpu_lobes(g, feat, K):
    raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
    return onasg.decode(torch.tensor(raw), K)


def _entry_spread(f, raw, scale, n_random=8, seed=0):
    """Per output entry of f (the oracle on raw outputs [B, n]): the larger of
    the summed changes when each raw output moves alone by its scale and the
    largest change under joint random-sign moves."""
    base = f(raw)
    one = np.zeros_like(base)
    for j in range(raw.shape[1]):
        r = raw.clone()
        r[:, j] += scale[:, j]
        one += np.abs(f(r) - base)
    rng = np.random.default_rng(seed)
    joint = np.zeros_like(base)
    for _ in range(n_random):
        sgn = torch.as_tensor(rng.choice([-1.0, 1.0], tuple(raw.shape)), dtype=raw.dtype)
        joint = np.maximum(joint, np.abs(f(raw + sgn * scale) - base))
    return np.maximum(one, joint)


@pytest.mark.parametrize("name", ["c1_f32", "c2_f32", "c3_f32", "c5_f32"])
@pytest.mark.parametrize("scale", [1.0, 3.0])
def test_query_f32(name, scale):
    K = CONFIGS[name][2]
    g, mats = make_guide(name, out_scale=scale)
    feat, xi = inputs(B_RAGGED, 3)
    d, pdf, rec = g.query(to_dev(feat), to_dev(xi), records=True)
    d = d.cpu().numpy().T.astype(np.float64)
    pdf = pdf.cpu().numpy().astype(np.float64)
    recg = rec_to_bk9(rec, B_RAGGED, K)
    # decode stage, from the GPU's own raw outputs
    lob = _gpu_lobes(g, feat, K)
    ro = lob.record().numpy()
    assert np.abs(recg[..., 0:6] - ro[..., 0:6]).max() < 1e-6
    assert (np.abs(recg[..., 6:8] - ro[..., 6:8]) / ro[..., 6:8]).max() < 1e-5
    assert np.abs(recg[..., 8] - ro[..., 8]).max() < 1e-5
    # end to end from the features: the stage-wise bounds plus what the
    # float32 forward's rounding of the raw outputs moves the exact records
    # by (an angle from a (cos, sin) pair of norm r moves by |d pair| / r;
    # theta's sine by cot(theta) |d cos|): per entry, the larger of the summed
    # one-at-a-time changes and the largest joint change when every raw
    # output moves by twice the GPU forward's measured deviation (itself held
    # to the a-priori rounding bound tests.grad_check.raw_scale) plus 4 float32
    # units
    W = w64(mats)
    raw64 = omlp.forward(W, feat.T).detach()
    raw_gpu = torch.as_tensor(g.forward_raw(to_dev(feat)).cpu().numpy().T, dtype=F64)
    assert ((raw_gpu - raw64).abs() <= GC.raw_scale(W, feat.T, raw64)).all()
    scale = 2 * (raw_gpu - raw64).abs() + 4 * GC.U * raw64.abs()
    rec_of = lambda r: onasg.decode(r, K).record().numpy()
    re2e = rec_of(raw64)
    moved = _entry_spread(rec_of, raw64, scale)
    floor = np.array([1e-6] * 6 + [0.0, 0.0, 1e-5])
    rel = np.array([0.0] * 6 + [1e-5, 1e-5, 0.0])
    bound = floor + rel * np.abs(re2e) + moved
    err = np.abs(recg - re2e)
    assert (err <= bound).all(), (err / bound).max()
    # the well-conditioned entries (moved by less than their floor) meet the
    # stage-wise bounds end to end, within a factor of two
    base = floor + rel * np.abs(re2e)
    good = moved <= base
    assert good.mean() > 0.5, good.mean()
    assert (err[good] <= 2 * base[good]).all(), (err[good] / base[good]).max()
    lob_e2e = onasg.decode(raw64, K)
    # sampled direction
    vo, _ = onasg.sample(lob, xi.T.astype(np.float64))
    vo = vo.numpy()
    keep = cdf_margin(lob, xi[0]) > 1e-5
    assert keep.mean() > 0.99
    assert np.linalg.norm(d - vo, axis=1)[keep].max() < 1e-4
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    # pdf at the GPU's direction
    lq = onasg.mixture_log_pdf(torch.tensor(d), lob).numpy()
    ok = ~near_minus_z(d, lob)
    assert np.abs(np.log(pdf) - lq)[ok].max() < 1e-4
    # end to end: 1e-4 plus the change of the exact log q at the GPU's
    # direction under the forward's rounding of the raw outputs
    dt = torch.tensor(d)
    lq_of = lambda r: onasg.mixture_log_pdf(dt, onasg.decode(r, K)).numpy()
    lq2 = lq_of(raw64)
    moved_q = _entry_spread(lq_of, raw64, scale)
    err_q = np.abs(np.log(pdf) - lq2)
    assert (err_q <= 1e-4 + moved_q)[ok].all(), (err_q - moved_q)[ok].max()


@pytest.mark.parametrize("name", ["c3_bf16", "c2_bf16", "c5_bf16"])
def test_query_bf16(name):
    """BF16 MLP, FP32 NASG: against the BF16-emulating oracle, |d log q| median
    <= 1e-3 and p99 <= 1e-2 at the sampled directions; against the pure FP64
    oracle the same quantities are reported."""
    K = CONFIGS[name][2]
    g, mats = make_guide(name, out_scale=3.0)
    feat, xi = inputs(B_RAGGED, 4)
    d, pdf = g.query(to_dev(feat), to_dev(xi))
    d = d.cpu().numpy().T.astype(np.float64)
    lpdf = np.log(pdf.cpu().numpy().astype(np.float64))
    lob = onasg.decode(omlp.forward(w64(mats), feat.T, bf16=True), K)
    ok = ~near_minus_z(d, lob)
    err = np.abs(lpdf - onasg.mixture_log_pdf(torch.tensor(d), lob).numpy())[ok]
    assert np.median(err) <= 1e-3 and np.quantile(err, 0.99) <= 1e-2, (np.median(err), np.quantile(err, 0.99))
    # stage check: GPU raw outputs decoded by the oracle give the GPU pdf to FP32 accuracy
    lob_g = _gpu_lobes(g, feat, K)
    err2 = np.abs(lpdf - onasg.mixture_log_pdf(torch.tensor(d), lob_g).numpy())[~near_minus_z(d, lob_g)]
    assert err2.max() < 1e-4


@pytest.mark.parametrize("name", ["c2_f32", "c3_bf16", "c5_bf16"])
def test_pdf_kernel(name):
    """nasg_pdf on records at sampled, target-like and uniform directions."""
    K = CONFIGS[name][2]
    g, _ = make_guide(name, out_scale=3.0)
    B = B_RAGGED
    feat, xi = inputs(B, 5)
    d, _, rec = g.query(to_dev(feat), to_dev(xi), records=True)
    rng = synth.rng_for(6)
    tgt = synth.VmfTarget(4, seed=7).sample(feat[0:3].T.astype(np.float64), rng)
    uni = synth.unit_vectors(B, rng).T.astype(np.float32)
    lob = onasg.lobes_from_record(rec_to_bk9(rec, B, K))
    for dirs in (d.contiguous(), to_dev(tgt), to_dev(np.ascontiguousarray(uni))):
        pg = g.pdf(rec, dirs).cpu().numpy().astype(np.float64)
        dn = dirs.cpu().numpy().T.astype(np.float64)
        lq = onasg.mixture_log_pdf(torch.tensor(dn), lob).numpy()
        ok = ~near_minus_z(dn, lob)
        assert np.abs(np.log(pg) - lq)[ok].max() < 1e-4


@pytest.mark.parametrize("name", ["c1_f32", "c3_bf16", "c5_bf16"])
def test_sample_kernel(name):
    """nasg_sample on records: same lobe rule and App. C map as the oracle."""
    K = CONFIGS[name][2]
    g, _ = make_guide(name, out_scale=3.0)
    B = B_RAGGED
    feat, xi = inputs(B, 8)
    _, _, rec = g.query(to_dev(feat), to_dev(xi), records=True)
    xi2 = synth.uniforms(B, synth.rng_for(9))
    d, pdf = g.sample(rec, to_dev(xi2))
    d = d.cpu().numpy().T.astype(np.float64)
    bk9 = rec_to_bk9(rec, B, K)
    vo, _ = onasg.sample_from_record(bk9, xi2.T.astype(np.float64))
    lob = onasg.lobes_from_record(bk9)
    full = onasg.Lobes(z=lob.z, x=lob.x, y=lob.y, lam=lob.lam, a=lob.a,
                       log_A=lob.log_A + onasg.log_normaliser(lob.lam, lob.a), log_K=torch.zeros_like(lob.a), eps=0.0)
    keep = cdf_margin(full, xi2[0]) > 1e-5
    assert np.linalg.norm(d - vo.numpy(), axis=1)[keep].max() < 1e-4
    lq = onasg.mixture_log_pdf(torch.tensor(d), lob).numpy()
    assert np.abs(np.log(pdf.cpu().numpy()) - lq)[~near_minus_z(d, lob)].max() < 1e-4


def test_empty_batches():
    g, _ = make_guide("c3_bf16")
    z9 = torch.zeros(9, 0, device="cuda")
    z4 = torch.zeros(4, 0, device="cuda")
    d, p = g.query(z9, z4)
    assert d.shape == (3, 0) and p.shape == (0,)
    assert g.forward_raw(z9).shape == (128, 0)
    rec = torch.zeros(1, device="cuda")
    assert g.pdf(rec, torch.zeros(3, 0, device="cuda")).shape == (0,)
    torch.cuda.synchronize()


def _train_batch(B, seed, target_seed=1001):
    rng = synth.rng_for(seed)
    return synth.training_batch(B, rng, synth.VmfTarget(4, seed=target_seed))


def _rel_errors(gpu_list, ref_list):
    return [float(np.linalg.norm(a.numpy() - b.numpy()) / np.linalg.norm(b.numpy()))
            for a, b in zip(gpu_list, ref_list)]


@pytest.mark.parametrize("name", ["c2_f32", "c3_bf16", "c5_bf16", "c5_f32"])
def test_adam_step_and_repacked_weights(name):
    """Adam (Kingma and Ba) from the GPU gradient vs the oracle's update; then
    the kernels must see the new weights (the packed copy is refreshed)."""
    K = CONFIGS[name][2]
    g, mats = make_guide(name)
    feat, dirs, w = _train_batch(3000, 12)
    w0 = g.w.cpu().double()
    for step in range(3):
        g.loss_grad(to_dev(feat), to_dev(dirs), to_dev(w))
        grad = g.grad.cpu().double()
        m0, v0 = g.adam_m.cpu().double(), g.adam_v.cpu().double()
        g.adam_step()
        torch.cuda.synchronize()
        # the library receives its hyper-parameters as float32 (nasg_config)
        f32 = lambda x: float(np.float32(x))
        wo, mo, vo, t = otrain.adam_step(w0, grad, m0, v0, step, f32(1e-3), f32(0.9), f32(0.999), f32(1e-8))
        assert int(g.step) == step + 1 and int(g.flags) == 0
        assert torch.abs(g.w.cpu().double() - wo).max() < 1e-7
        # FP32 rounding bound of each moment update, relative to its terms
        b1, b2 = f32(0.9), f32(0.999)
        tol_m = 4e-7 * (b1 * m0.abs() + (1 - b1) * grad.abs()) + 1e-30
        tol_v = 4e-7 * (b2 * v0 + (1 - b2) * grad * grad) + 1e-30
        assert torch.all(torch.abs(g.adam_m.cpu().double() - mo) <= tol_m)
        assert torch.all(torch.abs(g.adam_v.cpu().double() - vo) <= tol_v)
        w0 = g.w.cpu().double()
    f, _ = inputs(500, 13)
    raw = g.forward_raw(to_dev(f)).cpu().numpy().T
    ref = omlp.forward(g.split(w0), f.T, bf16=(CONFIGS[name][3] == "bf16")).numpy()
    err = np.abs(raw - ref) / np.abs(ref).max(axis=1, keepdims=True)
    # a stale or misplaced packed weight gives O(1) errors; BF16 rounding
    # flips of single activations stay below 2e-2 of the row scale
    assert np.mean(err < 1e-4) > 0.995 and err.max() < 2e-2, (np.mean(err < 1e-4), err.max())


def test_adam_skips_non_finite():
    g, _ = make_guide("c2_f32")
    feat, dirs, w = _train_batch(1024, 14)
    w[5] = np.nan
    before = g.w.clone()
    g.train_step(to_dev(feat), to_dev(dirs), to_dev(w))
    torch.cuda.synchronize()
    assert int(g.flags) == 1 and int(g.step) == 0
    assert torch.equal(g.w, before)
    w[5] = 1.0
    g.train_step(to_dev(feat), to_dev(dirs), to_dev(w))
    torch.cuda.synchronize()
    assert int(g.flags) == 0 and int(g.step) == 1
    assert not torch.equal(g.w, before)


@pytest.mark.parametrize("name", ["c2_f32", "c3_bf16", "c5_bf16", "c5_f32"])
def test_training_is_deterministic(name):
    outs = []
    for _ in range(2):
        g, _ = make_guide(name)
        feat, dirs, w = _train_batch(5000, 15)
        for _ in range(3):
            g.train_step(to_dev(feat), to_dev(dirs), to_dev(w))
        torch.cuda.synchronize()
        outs.append((g.w.clone(), g.grad.clone(), g.stats.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    assert torch.equal(outs[0][2], outs[1][2])


def test_full_size_query_sampled_parity():
    """2^20 queries with the BF16 network of K = 16 lobes, in the launch
    configuration the benchmark times; 4096 sampled vertices against the
    BF16-emulating oracle, and properties of all outputs."""
    K = 16
    g, mats = make_guide("c3_bf16", out_scale=3.0)
    B = 1 << 20
    feat, xi = inputs(B, 16)
    d, pdf = g.query(to_dev(feat), to_dev(xi))
    torch.cuda.synchronize()
    dn = torch.linalg.norm(d, dim=0)
    assert torch.all(torch.abs(dn - 1) < 1e-5)
    assert torch.all(torch.isfinite(pdf)) and torch.all(pdf > 0)
    idx = np.sort(synth.rng_for(17).choice(B, 4096, replace=False))
    dd = d[:, idx].cpu().numpy().T.astype(np.float64)
    lob = onasg.decode(omlp.forward(w64(mats), feat[:, idx].T, bf16=True), K)
    err = np.abs(np.log(pdf[idx].cpu().numpy()) - onasg.mixture_log_pdf(torch.tensor(dd), lob).numpy())
    err = err[~near_minus_z(dd, lob)]
    assert np.median(err) <= 1e-3 and np.quantile(err, 0.99) <= 1e-2


def test_record_round_trip_layout():
    """The test-side record converters are inverse to each other."""
    a = np.random.default_rng(0).standard_normal((130, 8, 9)).astype(np.float32)
    back = rec_to_bk9(torch.from_numpy(bk9_to_rec(a, 8)), 130, 8)
    assert np.array_equal(back.astype(np.float32), a)


# ---- the continuous form of App. A (epsilon > 0) ----

EPS = 0.3


@pytest.mark.parametrize("name", ["c2_f32", "c3_bf16"])
def test_query_records_pdf_sample_eps(name):
    """epsilon = 0.3: decoded records (log K with epsilon), the pdf at the
    sampled direction, and the record kernels, against the oracle's
    App. A lobe on the GPU's own raw outputs."""
    K = CONFIGS[name][2]
    g, mats = make_guide(name, out_scale=3.0, eps=EPS)
    feat, xi = inputs(B_RAGGED, 21)
    d, pdf, rec = g.query(to_dev(feat), to_dev(xi), records=True)
    raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
    lob = onasg.decode(torch.tensor(raw), K, EPS)
    recg = rec_to_bk9(rec, B_RAGGED, K)
    ro = lob.record().numpy()
    assert np.abs(recg[..., 0:6] - ro[..., 0:6]).max() < 1e-6
    assert np.abs(recg[..., 8] - ro[..., 8]).max() < 1e-5
    dd = d.cpu().numpy().T.astype(np.float64)
    lq = onasg.mixture_log_pdf(torch.tensor(dd), lob).numpy()
    assert np.abs(np.log(pdf.cpu().numpy()) - lq).max() < 1e-4   # continuous: no -z exclusion needed
    vo, _ = onasg.sample(lob, xi.T.astype(np.float64))
    keep = cdf_margin(lob, xi[0]) > 1e-5
    assert np.linalg.norm(dd - vo.numpy(), axis=1)[keep].max() < 1e-4
    # record kernels with the same epsilon
    uni = synth.unit_vectors(B_RAGGED, synth.rng_for(22)).T.astype(np.float32)
    pg = g.pdf(rec, to_dev(np.ascontiguousarray(uni))).cpu().numpy().astype(np.float64)
    lobr = onasg.lobes_from_record(recg, EPS)
    lq2 = onasg.mixture_log_pdf(torch.tensor(uni.T.astype(np.float64)), lobr).numpy()
    assert np.abs(np.log(pg) - lq2).max() < 1e-4
    xi2 = synth.uniforms(B_RAGGED, synth.rng_for(23))
    d2, p2 = g.sample(rec, to_dev(xi2))
    vs, _ = onasg.sample_from_record(recg, xi2.T.astype(np.float64), EPS)
    d2 = d2.cpu().numpy().T.astype(np.float64)
    full = onasg.Lobes(z=lobr.z, x=lobr.x, y=lobr.y, lam=lobr.lam, a=lobr.a,
                       log_A=lobr.log_A + onasg.log_normaliser(lobr.lam, lobr.a, EPS),
                       log_K=torch.zeros_like(lobr.a), eps=EPS)
    keep2 = cdf_margin(full, xi2[0]) > 1e-5
    assert np.linalg.norm(d2 - vs.numpy(), axis=1)[keep2].max() < 1e-4


def test_loss_grad_f32_eps():
    """epsilon = 0.3 in the training path: loss and stage-wise gradient."""
    name, K = "c2_f32", 8
    g, mats = make_guide(name, out_scale=2.0, eps=EPS)
    feat, dirs, w = _train_batch(B_RAGGED, 24)
    g.loss_grad(to_dev(feat), to_dev(dirs), to_dev(w))
    torch.cuda.synchronize()
    W = w64(mats)
    L, grads = otrain.loss_and_grad(W, feat.T, dirs.T, w.astype(np.float64), K, EPS)
    assert abs(float(g.stats[0]) - L) <= 1e-5 * abs(L)
    raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
    g_raw = otrain.raw_output_grad(raw, dirs.T, w.astype(np.float64), K, EPS)
    staged = otrain.weight_grad_from_raw_grad(W, feat.T, g_raw)
    errs = _rel_errors(g.split(g.grad.cpu()), staged)
    assert max(errs) < 1e-4, errs


@pytest.mark.parametrize("name,eps", [("c2_f32", 0.0), ("c3_bf16", 0.0), ("c3_bf16", 0.3), ("c5_bf16", 0.0)])
def test_pdf_direction_gradient(name, eps):
    """nasg_pdf_grad: the pdf as nasg_pdf, and the gradient of log D on the
    sphere against the oracle's autograd gradient, from the same records;
    per vertex within 1e-4 of the gradient's scale (|grad| + 1) away from
    the lobe axes. Within 0.05 rad of a lobe's z or -z the FP32 evaluation
    is ill-conditioned: the anisotropy c^2 = X^2 / (X^2 + Y^2) is 0/0 there
    (X, Y carry ~1e-7 absolute rounding) and at -z the eps = 0 lobe's
    gradient diverges like u^(a c^2 - 1); those vertices (a few percent) are
    held to 1e-2."""
    K = CONFIGS[name][2]
    g, _ = make_guide(name, out_scale=3.0, eps=eps)
    feat, xi = inputs(B_RAGGED, 25)
    _, _, rec = g.query(to_dev(feat), to_dev(xi), records=True)
    uni = np.ascontiguousarray(synth.unit_vectors(B_RAGGED, synth.rng_for(26)).T.astype(np.float32))
    pdf, grad = g.pdf_grad(rec, to_dev(uni))
    lob = onasg.lobes_from_record(rec_to_bk9(rec, B_RAGGED, K), eps)
    v = torch.tensor(uni.T.astype(np.float64))
    lq = onasg.mixture_log_pdf(v, lob).numpy()
    gr = onasg.log_pdf_direction_grad(v, lob).numpy()
    gg = grad.cpu().numpy().T.astype(np.float64)
    vz = (v[:, None, :] * lob.z).sum(-1).numpy()
    ok = ~((np.abs(vz) > np.cos(5e-2)).any(-1))
    assert ok.mean() > 0.9
    near_minus_z_ = (vz < -np.cos(1e-3)).any(-1)
    assert np.abs(np.log(pdf.cpu().numpy()) - lq)[~near_minus_z_].max() < 1e-4
    err = np.linalg.norm(gg - gr, axis=1) / (np.linalg.norm(gr, axis=1) + 1.0)
    assert err[ok].max() < 1e-4, err[ok].max()
    assert err[~near_minus_z_].max() < 1e-2, err[~near_minus_z_].max()
    assert np.abs((gg * uni.T).sum(1)).max() < 1e-4 * (np.abs(gg).max() + 1)


@pytest.mark.gpu
@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_pdf_grad_rising_maximum(eps):
    """nasg_pdf_grad keeps a running maximum of the lobes' log values and
    rescales its sums when it rises. Here the lobes' log(A/K) climbs by 3
    per lobe over K = 32 lobes of moderate sharpness, so the maximum rises
    at nearly every lobe. The pdf and the gradient of log D on the sphere
    (Sec. 3.1, eq. NASG) are compared with the oracle from the same records
    at 1e-4, away from the lobe axes as in ``test_pdf_direction_gradient``."""
    K, B = 32, 4099
    rng = np.random.default_rng(31)
    z = rng.normal(size=(B, K, 3))
    z /= np.linalg.norm(z, axis=-1, keepdims=True)
    t = rng.normal(size=(B, K, 3))
    x = t - (t * z).sum(-1, keepdims=True) * z
    x /= np.linalg.norm(x, axis=-1, keepdims=True)
    lam = np.exp(rng.uniform(0.0, np.log(50.0), size=(B, K)))
    a = np.exp(rng.uniform(np.log(0.1), np.log(20.0), size=(B, K)))
    logc = 3.0 * np.arange(K)[None, :] - 90.0 + rng.uniform(-1.0, 1.0, size=(B, K))
    bk9 = np.concatenate([z, x, lam[..., None], a[..., None], logc[..., None]], -1)
    g, _ = make_guide("c5_bf16", eps=eps, max_batch=B)       # the record kernels need only K and eps
    uni = np.ascontiguousarray(synth.unit_vectors(B, synth.rng_for(32)).T.astype(np.float32))
    pdf, grad = g.pdf_grad(to_dev(bk9_to_rec(bk9, K)), to_dev(uni))
    g.close()
    rec64 = rec_to_bk9(torch.tensor(bk9_to_rec(bk9, K)), B, K)   # the float32 records the GPU read
    lob = onasg.lobes_from_record(rec64, eps)
    v = torch.tensor(uni.T.astype(np.float64))
    lq = onasg.mixture_log_pdf(v, lob).numpy()
    gr = onasg.log_pdf_direction_grad(v, lob).numpy()
    gg = grad.cpu().numpy().T.astype(np.float64)
    vz = (v[:, None, :] * lob.z).sum(-1).numpy()
    ok = ~((np.abs(vz) > np.cos(5e-2)).any(-1))
    assert ok.mean() > 0.5
    assert np.abs(np.log(pdf.cpu().numpy().astype(np.float64)) - lq)[ok].max() < 1e-4
    err = np.linalg.norm(gg - gr, axis=1) / (np.linalg.norm(gr, axis=1) + 1.0)
    assert err[ok].max() < 1e-4, err[ok].max()


# ---- isotropic lobes (a = 0: the spherical-Gaussian comparison model) ----

@pytest.mark.parametrize("name", ["c2_f32", "c3_bf16"])
def test_isotropic_query_and_gradient(name):
    """isotropic = 1: records carry a = 0 and the pdf is the vMF mixture of
    the oracle's isotropic decode; the loss and gradient follow it (FP32
    stage-wise 1e-4, BF16 2e-2) and the a outputs' weights get none."""
    K, prec = CONFIGS[name][2], CONFIGS[name][3]
    g, mats = make_guide(name, out_scale=2.0, isotropic=True)
    feat, xi = inputs(B_RAGGED, 27)
    d, pdf, rec = g.query(to_dev(feat), to_dev(xi), records=True)
    recg = rec_to_bk9(rec, B_RAGGED, K)
    assert np.all(recg[..., 7] == 0.0)
    raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
    lob = onasg.decode(torch.tensor(raw), K, isotropic=True)
    dd = d.cpu().numpy().T.astype(np.float64)
    lq = onasg.mixture_log_pdf(torch.tensor(dd), lob).numpy()
    assert np.abs(np.log(pdf.cpu().numpy()) - lq).max() < 1e-4
    tf, td, tw = _train_batch(B_RAGGED, 28)
    g.loss_grad(to_dev(tf), to_dev(td), to_dev(tw))
    torch.cuda.synchronize()
    W = w64(mats)
    traw = g.forward_raw(to_dev(tf)).cpu().numpy().T.astype(np.float64)
    g_raw = otrain.raw_output_grad(traw, td.T, tw.astype(np.float64), K, isotropic=True)
    staged = otrain.weight_grad_from_raw_grad(W, tf.T, g_raw, bf16=prec == "bf16")
    gg = g.split(g.grad.cpu())
    errs = _rel_errors(gg, staged)
    assert max(errs) < (1e-4 if prec == "f32" else 2e-2), errs
    a_rows = [6 * K + k for k in range(K)]   # canonical rows of the log a outputs
    assert float(torch.abs(gg[-1][a_rows]).max()) == 0.0


@pytest.mark.parametrize("name", ["c1_bf16", "c3_bf16", "c3s_bf16", "c2_bf16", "c3_f32", "paper_bf16"])
def test_query_batch_invariance(name):
    """Each vertex's query is computed from that vertex alone, so a ragged or
    tiny batch must give, bit for bit, what the same vertices give inside a
    larger batch: this pins the kernels' vertex indexing, tail masks and
    lane exchanges (the hidden-64 BF16 networks sample one vertex per lane
    over four 16-vertex blocks) for batches that end inside a block, inside a
    pass and inside a tile."""
    K = CONFIGS[name][2]
    g, _ = make_guide(name)
    full = 4096
    feat, xi = inputs(full, 11)
    sel_net = g.selection
    fd, xd = to_dev(feat), to_dev(xi)
    ref_sel = torch.empty(full, device="cuda") if sel_net else None
    d0, p0, r0 = g.query(fd, xd, records=True, sel_out=ref_sel)
    torch.cuda.synchronize()
    for B in (1, 15, 17, 63, 65, 129, 1000):
        f, x = to_dev(np.ascontiguousarray(feat[:, :B])), to_dev(np.ascontiguousarray(xi[:, :B]))
        sel = torch.empty(B, device="cuda") if sel_net else None
        d, p, r = g.query(f, x, records=True, sel_out=sel)
        torch.cuda.synchronize()
        assert torch.equal(d, d0[:, :B]) and torch.equal(p, p0[:B]), (name, B)
        assert np.array_equal(rec_to_bk9(r, B, K), rec_to_bk9(r0, full, K)[:B]), (name, B)
        if sel_net:
            assert torch.equal(sel, ref_sel[:B]), (name, B)
        # the same vertices as views of the full arrays: leading dimension
        # 4096 > B (rows of the inputs and outputs 4096 floats apart)
        dv, pv = g.query(fd[:, :B], xd[:, :B])
        torch.cuda.synchronize()
        assert dv.stride(0) == full and torch.equal(dv, d0[:, :B]) and torch.equal(pv, p0[:B]), (name, B)
    g.close()
