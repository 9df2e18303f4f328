"""The selection-probability output and the blended loss (Sec. 4.2) on the
GPU against the FP64 oracle, through the C ABI.

Networks with 8K + 1 outputs: row 8K is the selection logit, c = sigmoid.
The loss is e KL(p || q_hat) + (1 - e) KL(p || q), q_hat = c q + (1 - c) p_fs,
estimated per sample with the weight w = p / q_hat (supplied) and the BSDF
pdf p_fs at the training direction (supplied; here a Lambertian lobe about
the vertex normal). Tolerances: FP32 raw outputs 1e-5 per row; c 1e-6. The
blended loss's weight gradients, entry by entry, are in
tests/test_gpu_gradients.py (c1s_f32, c2s_f32, c3s_bf16, the paper network).
"""

import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from oracle import nasg as onasg
from oracle import train as otrain
from paper_2303_08064_amd import synth
from tests.helpers import CONFIGS, make_guide, to_dev

pytestmark = pytest.mark.gpu

F64 = torch.float64
E = 0.2


def w64(mats):
    return [torch.tensor(m, dtype=F64) for m in mats]


def _batch(B, seed):
    rng = synth.rng_for(seed)
    feat, dirs, w = synth.training_batch(B, rng, synth.VmfTarget(4, seed=1001))
    pdf = synth.lambert_pdf(dirs, feat[6:9])
    return feat, dirs, w, pdf


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["c2s_f32", "c1s_f32", "c3s_bf16"])
def test_forward_and_selection_output(name):
    K, prec = CONFIGS[name][2], CONFIGS[name][3]
    g, mats = make_guide(name, out_scale=2.0, mis_fraction=E)
    feat, _, _, _ = _batch(1000, 40)
    raw = g.forward_raw(to_dev(feat)).cpu().numpy().T.astype(np.float64)
    assert raw.shape[1] == 8 * K + 1
    ref = omlp.forward(w64(mats), feat.T, bf16=prec == "bf16").numpy()
    err = np.abs(raw - ref) / np.abs(ref).max(axis=1, keepdims=True)
    if prec == "f32":
        assert err.max() < 1e-5, err.max()
    else:
        assert np.mean(err < 1e-4) >= 0.999 and err.max() < 2e-2
    # the query's selection probability is sigmoid(row 8K) of the same forward
    xi = synth.uniforms(1000, synth.rng_for(41))
    sel = torch.empty(1000, device="cuda")
    d, pdf = g.query(to_dev(feat), to_dev(xi), sel_out=sel)
    c_ref = onasg.selection(torch.tensor(raw), K).numpy()
    assert np.abs(sel.cpu().numpy() - c_ref).max() < 1e-6
    # directions and pdf are those of the 8K lobe outputs
    lob = onasg.decode(torch.tensor(raw), K)
    dd = d.cpu().numpy().T.astype(np.float64)
    lq = onasg.mixture_log_pdf(torch.tensor(dd), lob).numpy()
    assert np.median(np.abs(np.log(pdf.cpu().numpy()) - lq)) < 1e-5


@pytest.mark.parametrize("name,base", [("c2s_f32", "c2_f32"), ("c3s_bf16", "c3_bf16")])
def test_zero_fraction_matches_network_without_selection(name, base):
    """e = 0: the selection row gets no gradient, and every other weight's
    gradient and the loss equal those of the same network without the
    selection output, bit for bit (the extra tile contributes exact zeros)."""
    B = 3000
    gs, mats = make_guide(name, out_scale=2.0, mis_fraction=0.0)
    from paper_2303_08064_amd.nasg import NasgGuide
    H, NH, K, prec = CONFIGS[base]
    flat = synth.flat_weights(mats[:-1] + [mats[-1][:-1]])
    gb = NasgGuide(flat, hidden=H, n_hidden=NH, n_lobes=K, precision=prec)
    feat, dirs, w, pdf = _batch(B, 44)
    gs.loss_grad(to_dev(feat), to_dev(dirs), to_dev(w), bsdf_pdf=to_dev(pdf))
    gb.loss_grad(to_dev(feat), to_dev(dirs), to_dev(w))
    torch.cuda.synchronize()
    a, b = gs.split(gs.grad), gb.split(gb.grad)
    assert torch.all(a[-1][-1] == 0)
    for x, y in zip(a[:-1], b[:-1]):
        assert torch.equal(x, y)
    assert torch.equal(a[-1][:-1], b[-1])
    assert torch.equal(gs.stats[:2], gb.stats[:2])


@pytest.mark.parametrize("name", ["c2s_f32", "c3s_bf16"])
def test_adam_repacks_selection_row(name):
    """Adam updates the selection row and refreshes its packed copy: the
    forward after three steps matches the oracle on the updated weights."""
    K, prec = CONFIGS[name][2], CONFIGS[name][3]
    g, _ = make_guide(name, mis_fraction=E)
    feat, dirs, w, pdf = _batch(3000, 45)
    for _ in range(3):
        g.train_step(to_dev(feat), to_dev(dirs), to_dev(w), bsdf_pdf=to_dev(pdf))
    torch.cuda.synchronize()
    assert int(g.step) == 3 and int(g.flags) == 0
    f, _, _, _ = _batch(500, 46)
    raw = g.forward_raw(to_dev(f)).cpu().numpy().T
    ref = omlp.forward(g.split(g.w.cpu().double()), f.T, bf16=prec == "bf16").numpy()
    err = np.abs(raw - ref) / np.abs(ref).max(axis=1, keepdims=True)
    assert np.mean(err < 1e-4) > 0.995 and err.max() < 2e-2
    assert np.abs(raw[:, 8 * K] - ref[:, 8 * K]).max() < 1e-2 * np.abs(ref[:, 8 * K]).max()


def test_selection_training_is_deterministic():
    outs = []
    for _ in range(2):
        g, _ = make_guide("c3s_bf16", mis_fraction=E)
        feat, dirs, w, pdf = _batch(5000, 47)
        for _ in range(3):
            g.train_step(to_dev(feat), to_dev(dirs), to_dev(w), bsdf_pdf=to_dev(pdf))
        torch.cuda.synchronize()
        outs.append((g.w.clone(), g.stats.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_selection_argument_checks():
    """The binding refuses a selection network's loss without p_fs, p_fs for a
    network without the selection output, and sel_out there, before any
    launch; the C ABI refuses the same calls with NASG_E_ARG."""
    import ctypes
    from paper_2303_08064_amd._lib import NASG_E_ARG
    g, _ = make_guide("c2s_f32")
    feat, dirs, w, pdf = _batch(256, 48)
    f, d, wt, p = to_dev(feat), to_dev(dirs), to_dev(w), to_dev(pdf)
    with pytest.raises(ValueError, match="bsdf_pdf"):
        g.loss_grad(f, d, wt)
    g2, _ = make_guide("c2_f32")
    with pytest.raises(ValueError, match="bsdf_pdf"):
        g2.loss_grad(f, d, wt, bsdf_pdf=p)
    xi = to_dev(synth.uniforms(256, synth.rng_for(49)))
    with pytest.raises(ValueError, match="sel_out"):
        g2.query(f, xi, sel_out=torch.empty(256, device="cuda"))
    P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert g.lib.nasg_loss_grad(g._ctx, P(f), P(d), P(wt), None, 256, 256, st) == NASG_E_ARG
    assert b"bsdf_pdf" in g.lib.nasg_last_error()
    assert g2.lib.nasg_loss_grad(g2._ctx, P(f), P(d), P(wt), P(p), 256, 256, st) == NASG_E_ARG
    dout, pout, sel = (torch.empty(3, 256, device="cuda"), torch.empty(256, device="cuda"),
                       torch.empty(256, device="cuda"))
    assert g2.lib.nasg_query(g2._ctx, P(f), P(xi), 256, 256, P(dout), P(pout), P(sel), None, st) == NASG_E_ARG
    assert b"sel_out" in g2.lib.nasg_last_error()
