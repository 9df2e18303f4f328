"""Shared test plumbing: guide construction and layout conversions (no NASG math)."""

import numpy as np
import torch

from paper_2303_08064_amd import synth

CONFIGS = {
    # name: (hidden, n_hidden, n_lobes, precision)
    "c1_f32": (64, 3, 4, "f32"),
    "c2_f32": (64, 4, 8, "f32"),
    "c3_bf16": (64, 4, 16, "bf16"),
    "c3_f32": (64, 4, 16, "f32"),
    "c2_bf16": (64, 4, 8, "bf16"),
    "c1_bf16": (64, 3, 4, "bf16"),
    "c5_bf16": (128, 4, 32, "bf16"),
    "c5_f32": (128, 4, 32, "f32"),
    # shallower hidden-64 networks (the kernels take n_hidden in 1..4)
    "c3nh1_bf16": (64, 1, 16, "bf16"),
    "c3nh2_bf16": (64, 2, 16, "bf16"),
    "c3nh1_f32": (64, 1, 16, "f32"),
    "c3nh2_f32": (64, 2, 16, "f32"),
    # with the selection-probability output (8K + 1 outputs, the blended loss)
    "c2s_f32": (64, 4, 8, "f32"),
    "c3s_bf16": (64, 4, 16, "bf16"),
    "c1s_f32": (64, 3, 4, "f32"),
    # the paper's default network (Sec. 4.1, Sec. 6): encoded input, selection output
    "paper_bf16": (128, 4, 8, "bf16"),
    "paper_f32": (128, 4, 8, "f32"),
}
SELECTION = {"c2s_f32", "c3s_bf16", "c1s_f32", "paper_bf16", "paper_f32"}
ENCODED = {"paper_bf16", "paper_f32"}


def weights_for(name, seed=42, out_scale=1.0):
    H, NH, K, _ = CONFIGS[name]
    shapes = synth.layer_shapes(H, NH, K, selection=name in SELECTION, encoded=name in ENCODED)
    mats = synth.init_weights(shapes, synth.rng_for(seed))
    mats[-1] = (mats[-1] * out_scale).astype(np.float32)
    return mats


def make_guide(name, seed=42, out_scale=1.0, max_batch=1 << 18, **kw):
    from paper_2303_08064_amd.nasg import NasgGuide
    H, NH, K, prec = CONFIGS[name]
    mats = weights_for(name, seed, out_scale)
    if name in SELECTION:
        kw.setdefault("selection", True)
    if name in ENCODED:
        kw.setdefault("encoded", True)
    g = NasgGuide(synth.flat_weights(mats), hidden=H, n_hidden=NH, n_lobes=K, precision=prec,
                  max_batch=max_batch, **kw)
    return g, mats


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rec_to_bk9(rec, B, K):
    """Tiled record buffer [ceil(B/64)][9][K][64] -> [B, K, 9] float64 numpy."""
    n_t = (B + 63) // 64
    r = rec[: n_t * 9 * K * 64].detach().cpu().numpy().reshape(n_t, 9, K, 64)
    return r.transpose(0, 3, 2, 1).reshape(n_t * 64, K, 9)[:B].astype(np.float64)


def bk9_to_rec(bk9, K):
    """[B, K, 9] -> tiled record buffer (float32 numpy, zero-padded tail)."""
    B = bk9.shape[0]
    n_t = (B + 63) // 64
    pad = np.zeros((n_t * 64, K, 9), dtype=np.float32)
    pad[:B] = bk9
    return np.ascontiguousarray(pad.reshape(n_t, 64, K, 9).transpose(0, 3, 2, 1).reshape(-1))
