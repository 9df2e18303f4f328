"""The guiding MLP in float64 (oracle).

Test infrastructure only. Sec. 4.1: fully connected layers without bias and
ReLU between them; the input is padded with a constant one, which stands in
for the bias (footnote of Sec. 4.1). The input is either the 9 raw features
(position, outgoing direction, normal) followed by that one (10 values), or
the paper's encoded input of Tab. "encoding" (``encoding.encode``: 63
values) followed by that one (64 values). Which one is fixed by W_0's
column count.

Weights are a list of matrices W_l of shape [out_l, in_l]; layer l computes
h_l = relu(W_l h_{l-1}) and the last layer is linear.
"""

import torch

from . import encoding as enc

F64 = torch.float64
IN_FEATURES = 9


def input_width(encoded=False):
    """Columns of W_0: the features plus the constant one."""
    return (enc.ENCODED if encoded else IN_FEATURES) + 1


def layer_shapes(hidden, n_hidden, n_lobes, selection=False, encoded=False):
    """[(out, in)] for n_hidden hidden layers of width `hidden` and 8K outputs,
    plus one for the selection probability (Sec. 4.1: d = 8N + 1) when
    `selection` is set; W_0 reads the encoded input when `encoded` is set."""
    shapes = [(hidden, input_width(encoded))]
    shapes += [(hidden, hidden)] * (n_hidden - 1)
    shapes.append((8 * n_lobes + (1 if selection else 0), hidden))
    return shapes


def unflatten(flat, shapes):
    """Flat row-major concatenation of W_0 .. W_L -> list of matrices."""
    flat = torch.as_tensor(flat, dtype=F64)
    out, off = [], 0
    for (o, i) in shapes:
        out.append(flat[off:off + o * i].reshape(o, i))
        off += o * i
    assert off == flat.numel()
    return out


def flatten(mats):
    return torch.cat([m.reshape(-1) for m in mats])


class _RoundGradBf16(torch.autograd.Function):
    """Identity in the forward pass; in the backward pass the incoming
    gradient is rounded to float32 and then to the nearest bfloat16 (ties to
    even): a backward operand (a delta) held in BF16."""

    @staticmethod
    def forward(ctx, t):
        return t.view_as(t)

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.float32).to(torch.bfloat16).to(F64)


def round_bf16(t):
    """Round to the nearest bfloat16 (ties to even) through float32.

    In the autograd graph the rounding is the identity (straight-through), so
    gradients are those of the network with the rounded values.
    """
    r = t.detach().to(torch.float32).to(torch.bfloat16).to(F64)
    return t + (r - t.detach())


def network_input(feat, in_cols):
    """The input of W_0 for raw features [B, 9]: the features, or their
    encoding when W_0 has 64 columns, followed by the constant one."""
    feat = torch.as_tensor(feat, dtype=F64)
    if in_cols == input_width(True):
        feat = enc.encode(feat)
    elif in_cols != input_width(False):
        raise ValueError(f"W_0 has {in_cols} columns; expected {input_width(False)} or {input_width(True)}")
    return torch.cat([feat, torch.ones(feat.shape[0], 1, dtype=F64)], dim=-1)


def forward(weights, feat, bf16=False, return_pre=False):
    """Raw outputs [B, 8K (+1)] for raw features [B, 9].

    bf16=True emulates BF16 GEMMs with wide accumulation, forward and
    backward. Forward: every weight and every layer input (the features or
    their encoding, and the constant one) is rounded to bfloat16, products
    are summed in float64, and a hidden pre-activation is rounded to float32
    before the ReLU and the next rounding to bfloat16; the last layer's
    result is not rounded. Backward (under autograd): the delta of every
    layer, dL/d(pre-activation) including dL/d(raw outputs), is rounded to
    float32 and then to bfloat16 before it is used, both for that layer's
    weight gradient (delta times the layer's BF16 input, summed in float64)
    and for the delta of the layer below (the BF16 weights transposed times
    the delta, masked by the ReLU derivative).
    """
    h = network_input(feat, torch.as_tensor(weights[0]).shape[1])
    pre = []
    n = len(weights)
    for l, W in enumerate(weights):
        W = torch.as_tensor(W, dtype=F64)
        if bf16:
            W = round_bf16(W)
            h = round_bf16(h)
        y = h @ W.T
        if bf16:
            y = _RoundGradBf16.apply(y)
        pre.append(y)
        if l < n - 1:
            if bf16:
                y = y + (y.detach().to(torch.float32).to(F64) - y.detach())
            h = torch.relu(y)
    return (y, pre) if return_pre else y
