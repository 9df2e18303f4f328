"""The paper's default network on the GPU against the FP64 oracle, through
the C ABI: four hidden layers of 128 units, K = 8 lobes plus the selection
output, and the encoded input of Tab. "encoding" (Sec. 4.1, Sec. 6), BF16
and FP32. The FP32 network is held to the FP32 bounds of the other
networks: raw outputs 1e-5 per row. Its weight gradients and the BF16
network's, entry by entry at batches of 100, 777, 4131 and 20000, are in
tests/test_gpu_gradients.py.

The kernels encode the 9 raw features on the device (one-blob bins of the
position, omega_o, n, the constant one); the oracle encodes in float64 and
emulates the BF16 GEMMs. Tolerances are those of the other BF16 networks:
raw outputs 2e-2 of each row's largest value (99% of them within 1e-4,
see below). Batches are ragged against the kernels' 64-vertex (query) and
128-vertex (training) tiles.

The raw-output criterion is 99% (not 99.9%) within 1e-4 here: every BF16
rounding of a hidden activation, and of an encoded input, is decided from a
value whose float32 evaluation differs from the oracle's float64 one, and
with 64 inputs of magnitude up to one the first layer's sums are larger than
with the 9 raw features, so more activations sit near a BF16 tie. A
float32-accumulating CPU evaluation of the same BF16 network lands only
99.5-99.8% of its outputs within 1e-4 of the oracle, depending on the batch
and the weights (tests/test_oracle_encoding.py); the 2e-2 bound on every
output is unchanged.
"""

import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from oracle import nasg as onasg
from oracle import train as otrain
from paper_2303_08064_amd import synth
from tests.helpers import make_guide, to_dev

pytestmark = pytest.mark.gpu

F64 = torch.float64
E = 0.2
K = 8
NAME = "paper_bf16"


def w64(mats):
    return [torch.tensor(m, dtype=F64) for m in mats]


def _batch(B, seed):
    rng = synth.rng_for(seed)
    feat, dirs, w = synth.training_batch(B, rng, synth.VmfTarget(4, seed=1001))
    pdf = synth.lambert_pdf(dirs, feat[6:9])
    return feat, dirs, w, pdf


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _raw_err(raw, ref):
    return np.abs(raw - ref) / np.abs(ref).max(axis=1, keepdims=True)


def _check_raw(raw, ref):
    err = _raw_err(raw, ref)
    assert err.max() < 2e-2, err.max()
    assert np.mean(err < 1e-4) >= 0.99, np.mean(err < 1e-4)


@pytest.mark.parametrize("B", [1000, 64 * 300 + 17])
def test_forward_query_and_selection(B):
    g, mats = make_guide(NAME, out_scale=2.0, mis_fraction=E, max_batch=1 << 16)
    feat, _, _, _ = _batch(B, 60)
    raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
    assert raw.shape == (B, 8 * K + 1)
    ref = omlp.forward(w64(mats), feat.T, bf16=True).numpy()
    _check_raw(raw, ref)
    # the query runs the same forward; c = sigmoid(row 8K); directions and
    # pdf are those of the 8K lobe outputs
    xi = synth.uniforms(B, synth.rng_for(61))
    sel = torch.empty(B, device="cuda")
    d, pdf = g.query(to_dev(feat), to_dev(xi), sel_out=sel)
    assert np.abs(sel.cpu().numpy() - onasg.selection(torch.tensor(raw), K).numpy()).max() < 1e-6
    lob = onasg.decode(torch.tensor(raw), K)
    dd = d.cpu().numpy().T.astype(np.float64)
    assert np.abs(np.linalg.norm(dd, axis=1) - 1).max() < 1e-5
    lq = onasg.mixture_log_pdf(torch.tensor(dd), lob).numpy()
    assert np.median(np.abs(np.log(pdf.cpu().numpy()) - lq)) < 1e-5


def test_encoding_reaches_the_network():
    """Moving only the position within one one-blob bin changes the raw
    outputs as the oracle's encoded network says (a raw-feature network
    would see a linear change of three inputs)."""
    g, mats = make_guide(NAME, out_scale=2.0, mis_fraction=E)
    feat, _, _, _ = _batch(512, 62)
    f2 = feat.copy()
    f2[0] = np.clip(f2[0] + 0.02, 0, 1)
    W = w64(mats)
    for f in (feat, f2):
        raw = g.forward_raw(to_dev(f)).cpu().numpy().T.astype(np.float64)
        _check_raw(raw, omlp.forward(W, f.T, bf16=True).numpy())


def test_adam_repacks_and_training_is_deterministic():
    """Three Adam steps: the packed copy (layer 0's 16x16x32 fragments and
    the selection tile included) follows the master weights, and two runs
    agree bit for bit."""
    outs = []
    for _ in range(2):
        g, _ = make_guide(NAME, mis_fraction=E, max_batch=4096)
        feat, dirs, w, pdf = _batch(4096, 64)
        for _ in range(3):
            g.train_step(to_dev(feat), to_dev(dirs), to_dev(w), bsdf_pdf=to_dev(pdf))
        torch.cuda.synchronize()
        assert int(g.step) == 3 and int(g.flags) == 0
        outs.append((g.w.clone(), g.stats.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    f, _, _, _ = _batch(700, 65)
    raw = g.forward_raw(to_dev(f)).cpu().numpy().T
    ref = omlp.forward(g.split(g.w.cpu().double()), f.T, bf16=True).numpy()
    _check_raw(raw, ref)
    assert np.abs(raw[:, 8 * K] - ref[:, 8 * K]).max() < 1e-2 * np.abs(ref[:, 8 * K]).max()


def test_paper_schedule_training_gain():
    """The paper's configuration trained with its schedule: each iteration's
    S = 2^16 samples taken as 16 Adam steps of 4096 (Sec. 5) on the blended
    loss (e = 0.2) with a Lambertian p_fs about the normal, which knows
    nothing of the target. Held-out, by Monte Carlo with directions from the
    target p: the KL divergence to p drops below half of uniform sampling's,
    and the mean selection probability c rises from its initial ~0.5 (the
    learned density is the better proposal, so the blended loss favours it)."""
    import math
    target = synth.VmfTarget(4, seed=1001)
    g, _ = make_guide(NAME, mis_fraction=E, max_batch=4096)
    feat, dirs, _ = synth.training_batch(1 << 14, synth.rng_for(99), target)
    logp = target.log_pdf(feat[0:3].T.astype(np.float64), dirs.T.astype(np.float64))
    xi = to_dev(synth.uniforms(1 << 14, synth.rng_for(5)))
    sel = torch.empty(1 << 14, device="cuda")

    def heldout():
        _, _, rec = g.query(to_dev(feat), xi, records=True, sel_out=sel)
        lq = torch.log(g.pdf(rec, to_dev(dirs))).double().cpu().numpy()
        return float(np.mean(logp - lq)), float(sel.mean())

    kl0, c0 = heldout()
    pool = []
    for b in range(64):
        f, d, w = synth.training_batch(4096, synth.rng_for(20000 + b), target)
        pool.append(tuple(to_dev(x) for x in (f, d, w, synth.lambert_pdf(d, f[6:9]))))
    for it in range(100):
        for s in range(16):
            f, d, w, p = pool[(16 * it + s) % len(pool)]
            g.train_step(f, d, w, bsdf_pdf=p)
    torch.cuda.synchronize()
    assert int(g.step) == 1600 and int(g.flags) == 0
    kl, c1 = heldout()
    kl_uniform = float(np.mean(logp) + math.log(4 * math.pi))
    print(f"paper schedule: KL uniform {kl_uniform:.3f} init {kl0:.3f} trained {kl:.3f}; mean c {c0:.3f} -> {c1:.3f}")
    assert kl > -0.02
    assert kl < 0.5 * kl_uniform
    assert c1 > c0 + 0.1


@pytest.mark.parametrize("B", [1000, 64 * 50 + 17])
def test_f32_forward_query_and_selection(B):
    g, mats = make_guide("paper_f32", out_scale=2.0, mis_fraction=E, max_batch=1 << 16)
    feat, _, _, _ = _batch(B, 70)
    raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
    ref = omlp.forward(w64(mats), feat.T).numpy()
    err = np.linalg.norm(raw - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() < 1e-5, err.max()
    xi = synth.uniforms(B, synth.rng_for(71))
    sel = torch.empty(B, device="cuda")
    d, pdf = g.query(to_dev(feat), to_dev(xi), sel_out=sel)
    assert np.abs(sel.cpu().numpy() - onasg.selection(torch.tensor(ref), K).numpy()).max() < 1e-5
    lob = onasg.decode(torch.tensor(raw), K)
    lq = onasg.mixture_log_pdf(torch.tensor(d.cpu().numpy().T.astype(np.float64)), lob).numpy()
    assert np.median(np.abs(np.log(pdf.cpu().numpy()) - lq)) < 1e-6


@pytest.mark.parametrize("name", [NAME, "paper_f32"])
def test_edge_batches(name):
    """B = 0 launches nothing; B = 1 and B = 17 (one partial tile) match the
    oracle; B above max_batch is refused."""
    from paper_2303_08064_amd._lib import NasgError
    g, mats = make_guide(name, out_scale=2.0, mis_fraction=E, max_batch=64)
    z9, z4 = torch.zeros(9, 0, device="cuda"), torch.zeros(4, 0, device="cuda")
    d, p = g.query(z9, z4)
    assert d.shape == (3, 0) and p.shape == (0,)
    assert g.forward_raw(z9).shape == (8 * K + 1, 0)
    W = w64(mats)
    bf16 = name == NAME
    for B in (1, 17):
        feat, dirs, w, pdf = _batch(B, 80 + B)
        raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
        ref = omlp.forward(W, feat.T, bf16=bf16).numpy()
        assert (np.abs(raw - ref) / np.abs(ref).max(axis=1, keepdims=True)).max() < (2e-2 if bf16 else 1e-5)
        g.loss_grad(to_dev(feat), to_dev(dirs), to_dev(w), bsdf_pdf=to_dev(pdf))
        torch.cuda.synchronize()
        L = float(otrain.blended_nll(W, feat.T, dirs.T, w.astype(np.float64), pdf.astype(np.float64), K, e=E,
                                     bf16=bf16))
        assert abs(float(g.stats[0]) - L) <= (1e-3 if bf16 else 1e-5) * abs(L), (B, float(g.stats[0]), L)
    feat, dirs, w, pdf = _batch(65, 90)
    with pytest.raises(NasgError, match="max_batch"):
        g.loss_grad(to_dev(feat), to_dev(dirs), to_dev(w), bsdf_pdf=to_dev(pdf))
