"""Element-wise gates for the weight gradient of the fused backward (test
plumbing; every gradient it uses comes from the oracle).

A weight-gradient entry dW_l[i, j] = sum_v delta_l[v, i] h_{l-1}[v, j] is a
sum over the batch whose terms can cancel, so its float32 error scales with
the magnitude of the terms, not with the sum. Each entry is held to

    1e-4 |g| + 1e-7 max|g_l| + spread + 32 u S,

* g: the oracle's gradient (float64 chain rule through the literal forms),
  started from the raw outputs the kernel saw ("stage-wise") or from the
  features ("end to end"); entries below 1e-3 of the tensor's largest are
  held to 1e-4 of that level (1e-7 max|g_l|) rather than to 1e-4 of
  themselves (float32 cannot represent what lies far below the tensor's
  scale);
* spread: the largest change of g under joint random perturbations of the
  raw outputs by the size of the forward's rounding (stage-wise
  ``forward_scale``: ``SUM`` of the magnitude of the last layer's terms,
  plus bfloat16 tie flips and ambiguous ReLUs below; end to end
  ``raw_scale``: every layer's rounding carried to the output in absolute
  value), i.e. what the float32 inputs of the NASG backward cannot
  determine;
* S = sum_v |delta_l[v, i]| |h_{l-1}[v, j]| with the deltas propagated in
  absolute value (|W|^T |delta| under the ReLU mask): the magnitude of what
  the kernel accumulates; u = 2^-24, 32 units for the float32 accumulation
  of the deltas, the products and the sums over the batch;
* flips (``flip_allowance``): discrete decisions that the kernel takes from
  float32 values and the oracle from float64 ones may go either way where
  the two differ by less than the forward's rounding (``SUM`` = 4 u of the
  magnitude of a sum's terms, plus what the layers below pass up): a ReLU
  whose pre-activation lies that close to zero (the term of that unit and
  vertex may be present or not), and, for BF16 networks, a hidden
  activation or a delta that close to a bfloat16 rounding tie (one
  bfloat16 unit either way; for the raw-output delta, within 256 u of
  itself, or for a mixture logit of the two terms its gradient is the
  difference of if that is more (``raw_grad_rounding``), plus its spread; for
  the paper network's encoded input, within
  256 u of itself, the error of its float32 exp2). The terms such a decision can move, with
  everything they feed below, are added in absolute value.
"""

import numpy as np
import torch

from oracle import mlp as omlp
from oracle import nasg as onasg
from oracle import train as otrain

F64 = torch.float64
U = 2.0 ** -24
# the encoded input is evaluated with float32 exp2 of arguments up to ~180:
# ~100 float32 units of relative error before its bfloat16 rounding
ENC_SLACK = 256 * U
# how far two float32 evaluations of a layer's sums (the kernels' MFMA
# orders and the float64 sum rounded to float32) may differ, in units of
# u times the magnitude of the terms: every bfloat16 activation of the
# hidden-128 network that the kernels rounded differently from the
# emulation (107 of 2.56 million, over four layers) lay within 0.38 u mag of
# its tie; ten times that
SUM = 4 * U


def raw_grad_rounding(raw, dirs, w, K, bsdf=None, e=0.2, eps=0.0, isotropic=False):
    """[B, n_out]: how far the kernel's float32 raw-output gradient can lie
    from the float64 one where 256 u of the gradient itself is too narrow a
    band, because the gradient is a difference. The gradient of lobe
    k's logit is dL/dlog q (r_k - A_k) (Sec. 4.2 with the softmax of Tab.
    "decoding"): the responsibility r_k = A_k G_k / (K_k q) less the mixture
    weight A_k, two float32 values; where one lobe holds nearly all the
    weight both are near 1 and the difference is exact only to units of
    their sum. So 256 u |dL/dlog q| (r_k + A_k) for a logit, 0 for the other
    outputs (products of r_k and a partial of the lobe, which the 256 u band
    covers: r_k comes from log-domain terms a few tens in size, each rounded
    to float32) and for the selection logit."""
    raw = torch.as_tensor(raw, dtype=F64)
    B = raw.shape[0]
    lobes = onasg.decode(raw, K, eps, isotropic)
    terms = onasg.component_log_terms(dirs, lobes)              # log(A_k G_k / K_k)
    r = torch.exp(terms - torch.logsumexp(terms, dim=-1, keepdim=True))
    A = torch.exp(lobes.log_A)
    gq = torch.as_tensor(w, dtype=F64) / B                        # |dL/dlog q| of the mean NLL
    if bsdf is not None:
        c = onasg.selection(raw, K)
        q = torch.exp(torch.logsumexp(terms, dim=-1))
        qh = otrain.mis_pdf(q, c, torch.as_tensor(bsdf, dtype=F64))
        gq = gq * (e * c * q / qh + (1.0 - e))
    out = torch.zeros(raw.shape, dtype=F64)
    out[:, 7 * K:8 * K] = gq.abs()[:, None] * (r + A)
    return 256 * U * out


def raw_grad(raw, dirs, w, K, bsdf=None, e=0.2, eps=0.0, isotropic=False):
    """dL/d(raw outputs) [B, n_out] from the oracle."""
    if bsdf is not None:
        return otrain.blended_raw_output_grad(raw, dirs, w, bsdf, K, e=e, eps=eps)
    return otrain.raw_output_grad(raw, dirs, w, K, eps=eps, isotropic=isotropic)


def term_magnitudes(W, feat, g_raw):
    """[S_l]: sum_v |delta_l| |h_{l-1}| per weight, deltas propagated in
    absolute value through the float64 forward's ReLU pattern."""
    W = [torch.as_tensor(m, dtype=F64) for m in W]
    _, pre = omlp.forward(W, feat, return_pre=True)
    hs = [omlp.network_input(feat, W[0].shape[1])] + [torch.relu(p.detach()) for p in pre[:-1]]
    d = torch.as_tensor(g_raw, dtype=F64).abs()
    out = [None] * len(W)
    for l in range(len(W) - 1, -1, -1):
        out[l] = d.T @ hs[l].abs()
        if l > 0:
            d = (d @ W[l].abs()) * (pre[l - 1].detach() > 0)
    return out


def _near_bf16_tie(t, slack):
    """(mask, ulp): t within `slack` of the midpoint between the two
    bfloat16 values that enclose it (where rounding to nearest may go either
    way), and the spacing of those two values. Zeros are never near a tie."""
    t = torch.as_tensor(t, dtype=F64)
    b = t.to(torch.float32).numpy().view(np.uint32)
    lo = (b & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)          # toward zero
    hi = ((b & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)  # away from zero
    lo, hi = torch.as_tensor(lo), torch.as_tensor(hi)
    ulp = (hi - lo).abs()
    mid_dist = (t - (lo + hi) / 2).abs()
    return (mid_dist <= slack) & (t != 0), ulp


def _bf16(t):
    """float64 -> float32 -> bfloat16 (to nearest even), as the BF16
    emulation rounds a delta."""
    return omlp.round_bf16(torch.as_tensor(t, dtype=F64).to(torch.float32).to(F64)).detach()


def flip_allowance(W, feat, g_raw, bf16=False, raw_grad_slack=None, raw_grad_round=None):
    """[F_l]: per weight, the sum of the magnitudes of the terms that a
    rounding-dependent decision can change (see the module docstring):
    activations that may differ (``forward_uncertainty``: bfloat16 ties,
    ambiguous ReLUs, with what the layers below pass up) times |delta|;
    deltas that may differ -- the raw-output delta near a bfloat16 tie
    (within raw_grad_slack, its spread, plus the larger of 256 u of itself
    and raw_grad_round, ``raw_grad_rounding``), a delta whose
    ReLU may go either way, a bfloat16 delta near a tie -- times |h|, each
    carried down through |W| to the layers below."""
    layers, Wb = forward_uncertainty(W, feat, bf16)
    n = len(layers)
    d = torch.as_tensor(g_raw, dtype=F64)
    dd = torch.zeros_like(d)                     # possible change of each delta
    if bf16:
        slack = 256 * U * d.abs()
        if raw_grad_round is not None:
            slack = torch.maximum(slack, raw_grad_round)
        slack = slack + (0 if raw_grad_slack is None else raw_grad_slack)
        tie, ulp = _near_bf16_tie(d, slack)
        dd = tie * ulp
        d = _bf16(d)                             # the delta the emulation multiplies with
    out = [None] * n
    for l in range(n - 1, -1, -1):
        h_in, pre, mag, dpre, _ = layers[l]
        dh_in = layers[l - 1][4] if l > 0 else torch.zeros_like(h_in)
        out[l] = dd.T @ h_in.abs() + d.abs().T @ dh_in
        if l > 0:
            pre_b = layers[l - 1][1]
            mask = pre_b > 0
            amb = pre_b.abs() <= layers[l - 1][3] + SUM * layers[l - 1][2]
            full = d @ Wb[l]
            dprev = full * mask
            ddprev = (dd @ Wb[l].abs()) * (mask | amb) + amb * full.abs()
            if bf16:
                tie, ulp = _near_bf16_tie(dprev, SUM * ((d.abs() @ Wb[l].abs()) * mask) + ddprev)
                ddprev = ddprev + tie * ulp
                dprev = _bf16(dprev)
            d, dd = dprev, ddprev
    return out


def staged_grad(W, feat, raw, dirs, w, K, bf16=False, **kw):
    """[dL/dW_l] from the given raw outputs: the NASG backward at those raw
    outputs, then the MLP chain rule (BF16-emulated when bf16)."""
    return otrain.weight_grad_from_raw_grad(W, feat, raw_grad(raw, dirs, w, K, **kw), bf16=bf16)


def forward_uncertainty(W, feat, bf16=False):
    """The float64 forward (BF16-emulated when bf16) and, per layer, how far
    a float32 evaluation may differ from it: [(h_in, pre, mag, dpre, dh_out)]
    with h_in the layer's input, pre its pre-activation, mag the magnitude
    of its terms (|W| |h_in|), dpre = |W| dh_in + SUM mag (the possible
    difference of pre: float32 summation order plus what the layers below
    pass up) and dh_out the possible difference of its activation: for BF16
    one bfloat16 unit where the activation lies within dpre + SUM (mag + a)
    of a rounding tie, and the activation itself where the ReLU may go
    either way."""
    W = [torch.as_tensor(m, dtype=F64) for m in W]
    Wb = [omlp.round_bf16(m).detach() for m in W] if bf16 else W
    h = omlp.network_input(feat, W[0].shape[1])
    dh = torch.zeros_like(h)
    if bf16:
        if W[0].shape[1] == omlp.input_width(True):
            tie, ulp = _near_bf16_tie(h, ENC_SLACK * h.abs())
            dh = tie * ulp
        h = omlp.round_bf16(h).detach()
    out = []
    for l in range(len(W)):
        pre = h @ Wb[l].T
        mag = h.abs() @ Wb[l].abs().T
        dpre = dh @ Wb[l].abs().T + SUM * mag
        if l == len(W) - 1:
            out.append((h, pre, mag, dpre, None))
            break
        a = torch.relu(pre.to(torch.float32).to(F64)) if bf16 else torch.relu(pre)
        amb = pre.abs() <= dpre + SUM * mag
        if bf16:
            tie, ulp = _near_bf16_tie(a, dpre + SUM * (mag + a))
            dh_out = tie * ulp + amb * a
            h_out = omlp.round_bf16(a).detach()
        else:
            dh_out = dpre * (pre > 0) + amb * a
            h_out = a
        out.append((h, pre, mag, dpre, dh_out))
        h, dh = h_out, dh_out
    return out, Wb


def tie_free(W, feat, bf16=True):
    """[B] mask of the vertices whose float32 forward is decided the same way
    as the float64 one at every step: no hidden activation (nor, for the
    encoded input, input value) within ``forward_uncertainty``'s reach of a
    bfloat16 rounding tie, and no ReLU that may go either way. On these the
    kernel's bfloat16 activations equal the oracle's emulation exactly."""
    layers, _ = forward_uncertainty(W, feat, bf16)
    B = layers[0][0].shape[0]
    free = torch.ones(B, dtype=torch.bool)
    for l, (_, _, _, _, dh_out) in enumerate(layers):
        if l == 0 and bf16:
            h_in = layers[0][0]
        if dh_out is not None:
            free &= ~(dh_out > 0).any(1)
    if bf16 and W[0].shape[1] == omlp.input_width(True):
        x = omlp.network_input(feat, W[0].shape[1])
        tie, _ = _near_bf16_tie(x, ENC_SLACK * x.abs())
        free &= ~tie.any(1)
    return free.numpy()


def forward_scale(W, feat, raw, bf16=False):
    """Per raw output, how far two float32 evaluations of the same network
    (the training kernel's own forward and the forward the test reads, which
    sum in their own orders) can differ: ``forward_uncertainty``'s dpre of
    the last layer, ``SUM`` of the magnitude of its terms plus the possible
    differences of its inputs (for BF16 networks, bfloat16 ties and
    ambiguous ReLUs anywhere below, carried up through |W|); at least four
    float32 units of the value."""
    layers, _ = forward_uncertainty(W, feat, bf16)
    if bf16:
        scale = layers[-1][3]
    else:
        scale = SUM * layers[-1][2]
    return torch.maximum(scale, 4 * U * torch.as_tensor(raw, dtype=F64).abs())


def raw_scale(W, feat, raw):
    """Per raw output, the size of a whole float32 forward's rounding from
    the features: each layer's rounding, 8 u of the magnitude of its terms,
    carried to the output in absolute value (|W| times the magnitude below,
    under the float64 ReLU pattern), summed over the layers; at least four
    float32 units of the value."""
    W = [torch.as_tensor(m, dtype=F64) for m in W]
    h = omlp.network_input(feat, W[0].shape[1])
    err = torch.zeros_like(h)
    for l, m in enumerate(W):
        pre = h @ m.T
        err = err @ m.abs().T + 8 * U * (h.abs() @ m.abs().T)
        if l < len(W) - 1:
            err = err * (pre > 0)
            h = torch.relu(pre)
    return torch.maximum(err, 4 * U * torch.as_tensor(raw, dtype=F64).abs())


def tolerance(W, feat, raw, dirs, w, K, scale, bf16=False, n_random=8, seed=0, **kw):
    """(g_ref, tol) lists: the oracle gradient at `raw` and the per-entry
    bound above; `scale` [B, n_out] is the perturbation size per raw output."""
    raw = torch.as_tensor(raw, dtype=F64)
    g_raw = raw_grad(raw, dirs, w, K, **kw)
    ref = otrain.weight_grad_from_raw_grad(W, feat, g_raw, bf16=bf16)
    rng = np.random.default_rng(seed)
    spread = [torch.zeros_like(g) for g in ref]
    graw_spread = torch.zeros_like(g_raw)
    for _ in range(n_random):
        sgn = torch.as_tensor(rng.choice([-1.0, 1.0], tuple(raw.shape)), dtype=F64)
        gr = raw_grad(raw + sgn * scale, dirs, w, K, **kw)
        graw_spread = torch.maximum(graw_spread, (gr - g_raw).abs())
        gp = otrain.weight_grad_from_raw_grad(W, feat, gr, bf16=bf16)
        spread = [torch.maximum(s, (a - b).abs()) for s, a, b in zip(spread, gp, ref)]
    S = term_magnitudes(W, feat, g_raw)
    Fl = flip_allowance(W, feat, g_raw, bf16, graw_spread, raw_grad_rounding(raw, dirs, w, K, **kw) if bf16 else None)
    tol = [1e-4 * g.abs() + 1e-7 * g.abs().max() + s + 32 * U * m + f for g, s, m, f in zip(ref, spread, S, Fl)]
    return ref, tol


def check_norm(gpu, ref, tol, what):
    """Each tensor: ||gpu - ref|| <= 1e-4 ||ref|| + ||tol - 1e-4 |ref|||, the
    norm form of the entry bound (1e-4 in norm where nothing but the 1e-4
    term is left, i.e. for well-conditioned tensors)."""
    for l, (a, b, t) in enumerate(zip(gpu, ref, tol)):
        a = torch.as_tensor(a, dtype=F64)
        d, n = float(torch.linalg.norm(a - b)), float(torch.linalg.norm(b))
        extra = float(torch.linalg.norm(t - 1e-4 * b.abs()))
        assert d <= 1e-4 * n + extra, (what, l, d / n, extra / n)


def check(gpu, ref, tol, what):
    """Every entry within its bound."""
    msgs = []
    for l, (a, b, t) in enumerate(zip(gpu, ref, tol)):
        a = torch.as_tensor(a, dtype=F64)
        err = (a - b).abs()
        bad = err > t
        if bad.any():
            i = int(torch.argmax(err / t))
            msgs.append(f"{what} W_{l}: {int(bad.sum())} of {bad.numel()} entries outside the bound; worst "
                        f"entry {i}: gpu {float(a.reshape(-1)[i]):.6g} ref {float(b.reshape(-1)[i]):.6g} "
                        f"bound {float(t.reshape(-1)[i]):.3g}")
    assert not msgs, "\n".join(msgs)


def rel_norms(gpu, ref):
    return [float(torch.linalg.norm(torch.as_tensor(a, dtype=F64) - b) / torch.linalg.norm(b))
            for a, b in zip(gpu, ref)]
