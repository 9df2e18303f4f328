"""The guiding network's encoded input in float64 (oracle).

Test infrastructure only. Sec. 4.1 and Tab. "encoding": the position is
one-blob encoded (the encoding of Mueller et al., Neural Importance
Sampling) into 57 values, the outgoing direction and the normal enter
unchanged, and the constant one that stands in for the bias (footnote of
Sec. 4.1) pads the 63 values to 64.

Readings (the paper gives the widths only):

* 57 = 3 x 19: each position coordinate gets 19 bins of its own.
* bin i of k covers [i/k, (i+1)/k); its value is a Gaussian kernel of
  standard deviation 1/k centred at the coordinate s and evaluated at the
  bin centre c_i = (i + 1/2)/k:  exp(-(c_i - s)^2 / (2 (1/k)^2)). The peak
  is 1; there is no normalisation.
* s is the position in the scene's bounding box mapped to [0, 1]; values
  outside that range follow the same formula (no clamp).
* order: the bins of x, of y, of z, then omega_o (3), n (3), then the one.
"""

import torch

F64 = torch.float64
BINS = 19             # one-blob bins per position coordinate
ENCODED = 3 * BINS + 6   # 63 encoded features; the constant one makes 64


def one_blob(s, bins=BINS):
    """[B] coordinates in [0, 1] -> [B, bins] one-blob values."""
    s = torch.as_tensor(s, dtype=F64)
    centres = (torch.arange(bins, dtype=F64) + 0.5) / bins
    sigma = 1.0 / bins
    d = centres[None, :] - s[:, None]
    return torch.exp(-d * d / (2.0 * sigma * sigma))


def encode(feat):
    """Raw features [B, 9] (p, omega_o, n) -> encoded features [B, 63]."""
    feat = torch.as_tensor(feat, dtype=F64)
    blobs = [one_blob(feat[:, i]) for i in range(3)]
    return torch.cat(blobs + [feat[:, 3:9]], dim=-1)
