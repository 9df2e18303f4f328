"""Robustness: checkpoints, argument errors at both layers, non-finite inputs.

* A checkpoint (weights, Adam moments, step, flags) restored into a fresh
  guide continues training bit for bit as the original does.
* Every GPU entry point of the C ABI refuses NULL, misaligned, negative,
  ld < B and over-max_batch arguments with its status code, and launches
  nothing (sentinel outputs stay untouched). Only arguments that the
  library's host-side checks reject are passed: nothing here reaches a
  kernel with a bad pointer.
* The Python binding refuses tensors of the wrong dtype, device, shape,
  leading dimension or size before calling the library.
* NaN or Inf in the features or directions (not only in the weights w)
  makes the Adam step skip its update and set flag bit 0.
"""

import ctypes

import numpy as np
import pytest
import torch

from paper_2303_08064_amd import synth
from paper_2303_08064_amd._lib import NASG_E_ALIGN, NASG_E_ARG, NASG_E_SHAPE, NASG_OK, Config, State
from paper_2303_08064_amd.nasg import record_elems
from tests.helpers import make_guide, to_dev

pytestmark = pytest.mark.gpu


def _batch(B, seed):
    rng = synth.rng_for(seed)
    return synth.training_batch(B, rng, synth.VmfTarget(4, seed=1001))


@pytest.mark.parametrize("name", ["c2_f32", "c3_bf16", "c5_bf16", "paper_bf16"])
def test_checkpoint_restore_continues_bitwise(name, tmp_path):
    sel = name == "paper_bf16"
    B = 3000
    batches = []
    for i in range(6):
        f, d, w = _batch(B, 70 + i)
        extra = [to_dev(synth.lambert_pdf(d, f[6:9]))] if sel else []
        batches.append([to_dev(f), to_dev(d), to_dev(w)] + extra)

    def step(g, b):
        g.train_step(*b[:3], bsdf_pdf=b[3] if sel else None)

    ga, _ = make_guide(name, max_batch=B)
    for b in batches[:3]:
        step(ga, b)
    path = tmp_path / "ckpt.pt"
    torch.save(ga.state_dict(), path)
    for b in batches[3:]:
        step(ga, b)
    torch.cuda.synchronize()
    ref = ga.state_dict()
    gb, _ = make_guide(name, seed=7, max_batch=B)     # other initial weights, overwritten
    gb.load_state_dict(torch.load(path, weights_only=True))
    assert int(gb.step) == 3
    for b in batches[3:]:
        step(gb, b)
    torch.cuda.synchronize()
    got = gb.state_dict()
    for k in ref:
        assert torch.equal(ref[k], got[k]), k
    assert int(gb.step) == 6


def _P(t, off=0):
    return ctypes.c_void_p(t.data_ptr() + off) if t is not None else None


def test_abi_status_codes_launch_nothing():
    g, _ = make_guide("c3_bf16", max_batch=512)
    lib, ctx = g.lib, g._ctx
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    B = 256
    f, d, w = _batch(B, 77)
    feat, dirs, wts = to_dev(f), to_dev(d), to_dev(w)
    xi = to_dev(synth.uniforms(B, synth.rng_for(78)))
    rec = torch.zeros(record_elems(16, B), device="cuda")
    SENT = 12345.0
    dout = torch.full((3, B), SENT, device="cuda")
    pout = torch.full((B,), SENT, device="cuda")
    gout = torch.full((3, B), SENT, device="cuda")
    raw = torch.full((128, B), SENT, device="cuda")
    w_before = g.w.clone()
    grad_before = g.grad.clone()
    step_before = g.step.clone()

    calls = {
        "nasg_forward": lambda **k: lib.nasg_forward(k.get("ctx", ctx), k.get("feat", _P(feat)), k.get("ld", B),
                                                     k.get("B", B), k.get("out", _P(raw)), st),
        "nasg_query": lambda **k: lib.nasg_query(k.get("ctx", ctx), k.get("feat", _P(feat)), k.get("xi", _P(xi)),
                                                 k.get("ld", B), k.get("B", B), k.get("out", _P(dout)),
                                                 k.get("pdf", _P(pout)), None, k.get("rec", None), st),
        "nasg_pdf": lambda **k: lib.nasg_pdf(k.get("ctx", ctx), k.get("rec", _P(rec)), k.get("feat", _P(dirs)),
                                             k.get("ld", B), k.get("B", B), k.get("pdf", _P(pout)), st),
        "nasg_pdf_grad": lambda **k: lib.nasg_pdf_grad(k.get("ctx", ctx), k.get("rec", _P(rec)),
                                                       k.get("feat", _P(dirs)), k.get("ld", B), k.get("B", B),
                                                       k.get("pdf", _P(pout)), k.get("out", _P(gout)), st),
        "nasg_sample": lambda **k: lib.nasg_sample(k.get("ctx", ctx), k.get("rec", _P(rec)), k.get("feat", _P(xi)),
                                                   k.get("ld", B), k.get("B", B), k.get("out", _P(dout)),
                                                   k.get("pdf", _P(pout)), st),
        "nasg_loss_grad": lambda **k: lib.nasg_loss_grad(k.get("ctx", ctx), k.get("feat", _P(feat)),
                                                         k.get("dir", _P(dirs)), k.get("w", _P(wts)), None,
                                                         k.get("ld", B), k.get("B", B), st),
        "nasg_train_step": lambda **k: lib.nasg_train_step(k.get("ctx", ctx), k.get("feat", _P(feat)),
                                                           k.get("dir", _P(dirs)), k.get("w", _P(wts)), None,
                                                           k.get("ld", B), k.get("B", B), st),
    }
    # the first vector input of each call is passed as "feat"
    for name, call in calls.items():
        assert call(ctx=None) == NASG_E_ARG, name
        assert call(B=-1) == NASG_E_SHAPE, name
        assert call(ld=B - 1) == NASG_E_SHAPE, name
        assert call(feat=None) == NASG_E_ARG, name
        assert call(feat=_P(feat, 2)) == NASG_E_ALIGN, name
        assert name in lib.nasg_last_error().decode()
        if name in ("nasg_forward", "nasg_query", "nasg_pdf_grad", "nasg_sample"):
            assert call(out=None) == NASG_E_ARG, name
            assert call(out=_P(dout, 1)) == NASG_E_ALIGN, name
        if name in ("nasg_query", "nasg_pdf", "nasg_pdf_grad", "nasg_sample"):
            assert call(pdf=None) == NASG_E_ARG, name
            assert call(pdf=_P(pout, 3)) == NASG_E_ALIGN, name
        if name in ("nasg_pdf", "nasg_pdf_grad", "nasg_sample"):
            assert call(rec=None) == NASG_E_ARG, name
            assert call(rec=_P(rec, 2)) == NASG_E_ALIGN, name
        if name == "nasg_query":
            assert call(rec=_P(rec, 2)) == NASG_E_ALIGN, name
        if name == "nasg_query":
            assert call(xi=None) == NASG_E_ARG, name
        if name in ("nasg_loss_grad", "nasg_train_step"):
            assert call(B=513, ld=513) == NASG_E_SHAPE and b"max_batch" in lib.nasg_last_error(), name
            assert call(B=0, ld=0) == NASG_E_SHAPE, name
            assert call(w=None) == NASG_E_ARG, name
            assert call(dir=_P(dirs, 2)) == NASG_E_ALIGN, name
        else:
            assert call(B=0, ld=0) == NASG_OK, name      # an empty batch launches nothing
    assert lib.nasg_adam_step(None, st) == NASG_E_ARG
    assert lib.nasg_pack(None, st) == NASG_E_ARG
    torch.cuda.synchronize()
    for t in (dout, pout, gout, raw):
        assert torch.all(t == SENT)
    assert torch.equal(g.w, w_before) and torch.equal(g.grad, grad_before) and torch.equal(g.step, step_before)
    # nasg_create: bad configurations and misaligned state
    cfg = Config(64, 4, 16, 1, 0.0, 1e-3, 0.9, 0.999, 1e-8, 512, 0, 0.2, 0, 0)
    out = ctypes.c_void_p()
    state = State(*[t.data_ptr() for t in (g.w, g.grad, g.adam_m, g.adam_v, g.wpack, g.step, g.flags, g.stats,
                                           g.workspace)])
    for field, bad in (("n_lobes", 5), ("hidden", 96), ("n_hidden", 0), ("precision", 3), ("lr", -1.0),
                       ("eps", -0.5), ("mis_fraction", 1.5), ("beta1", 1.0), ("max_batch", -1)):
        c2 = Config.from_buffer_copy(cfg)
        setattr(c2, field, bad)
        assert lib.nasg_create(ctypes.byref(c2), ctypes.byref(state), ctypes.byref(out)) == NASG_E_ARG, field
        assert not out.value
    s2 = State.from_buffer_copy(state)
    s2.wpack = g.wpack.data_ptr() + 4
    assert lib.nasg_create(ctypes.byref(cfg), ctypes.byref(s2), ctypes.byref(out)) == NASG_E_ALIGN
    s2 = State.from_buffer_copy(state)
    s2.stats = None
    assert lib.nasg_create(ctypes.byref(cfg), ctypes.byref(s2), ctypes.byref(out)) == NASG_E_ARG
    g.close()


def test_binding_checks_tensors_before_launch():
    g, _ = make_guide("c2_f32", max_batch=1024)
    B = 200
    f, d, w = _batch(B, 79)
    feat, dirs, wts = to_dev(f), to_dev(d), to_dev(w)
    xi = to_dev(synth.uniforms(B, synth.rng_for(80)))
    rec = torch.zeros(record_elems(8, B), device="cuda")
    with pytest.raises(TypeError):
        g.query(feat.double(), xi)
    with pytest.raises(TypeError):
        g.query(feat.cpu(), xi)
    with pytest.raises(ValueError):
        g.query(feat[:8], xi)                          # 8 rows, not 9
    with pytest.raises(ValueError):
        g.query(feat, xi[:, :B - 1])                   # B mismatch
    wide = torch.zeros(3, 2 * B, device="cuda")
    with pytest.raises(ValueError, match="leading dimension"):
        g.query(feat, xi, dir_out=wide)                # rows at 2B apart, the kernel writes at B
    with pytest.raises(ValueError):
        g.query(feat, xi, pdf_out=torch.empty(B - 1, device="cuda"))
    with pytest.raises(ValueError):
        g.query(feat, xi, rec_out=torch.empty(record_elems(8, B) - 1, device="cuda"))
    with pytest.raises(ValueError):
        g.pdf(rec[:-1], dirs)                          # records of B vertices need whole 64-vertex tiles
    with pytest.raises(TypeError):
        g.pdf(rec.cpu(), dirs)
    with pytest.raises(ValueError):
        g.sample(rec, xi, pdf_out=torch.empty(2, B, device="cuda"))
    with pytest.raises(ValueError):
        g.pdf_grad(rec, dirs, grad_out=torch.empty(3, B - 1, device="cuda"))
    with pytest.raises(TypeError):
        g.loss_grad(feat, dirs, wts.cpu())
    with pytest.raises(ValueError):
        g.loss_grad(feat, dirs, wts[:B - 1])
    with pytest.raises(ValueError):
        g.loss_grad(feat, dirs[:, :B - 1], wts)
    with pytest.raises(ValueError):
        g.forward_raw(feat, out=torch.empty(63, B, device="cuda"))
    # a strided [rows, B] view with its own leading dimension is accepted
    big = torch.zeros(9, 3 * B, device="cuda")
    big[:, :B] = feat
    bigxi = torch.zeros(4, 3 * B, device="cuda")
    bigxi[:, :B] = xi
    d1, p1 = g.query(big[:, :B], bigxi[:, :B])
    d0, p0 = g.query(feat, xi)
    torch.cuda.synchronize()
    assert torch.equal(d1, d0) and torch.equal(p1, p0)
    g.close()


@pytest.mark.parametrize("name", ["c2_f32", "c3_bf16", "c5_bf16"])
@pytest.mark.parametrize("where", ["feat_nan", "feat_inf", "dir_nan", "dir_inf"])
def test_non_finite_inputs_skip_the_update(name, where):
    g, _ = make_guide(name, max_batch=2048)
    f, d, w = _batch(2000, 81)
    if where.startswith("feat"):
        f[3, 17] = np.nan if where.endswith("nan") else np.inf
    else:
        d[1, 1234] = np.nan if where.endswith("nan") else -np.inf
    before = [t.clone() for t in (g.w, g.adam_m, g.adam_v, g.step)]
    g.train_step(to_dev(f), to_dev(d), to_dev(w))
    torch.cuda.synchronize()
    assert int(g.flags) & 1 == 1
    assert not np.isfinite(float(g.stats[0])) or not np.isfinite(float(g.stats[2]))
    for a, b in zip((g.w, g.adam_m, g.adam_v, g.step), before):
        assert torch.equal(a, b)
    # a finite batch afterwards trains again and clears the flag
    f2, d2, w2 = _batch(2000, 82)
    g.train_step(to_dev(f2), to_dev(d2), to_dev(w2))
    torch.cuda.synchronize()
    assert int(g.flags) & 1 == 0 and int(g.step) == 1
    g.close()
