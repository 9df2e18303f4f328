"""Conditioned tolerances for comparing float32 kernels with the exact oracle
(test plumbing; no NASG arithmetic of its own).

A float32 kernel sees its inputs rounded to float32 and rounds again at every
operation, so even a perfect float32 implementation can only be held to the
exact value plus the change of that value under perturbations of its inputs
of a few float32 units in the last place. ``spread`` measures that change
with the extended-precision oracle itself: each input component is
perturbed alone, relatively by ``rel`` (one-at-a-time changes are summed:
the first-order worst case), and all components are perturbed together with
random signs; the larger of the two is the allowance. Components that are
exactly zero stay zero (float32 holds them exactly). The tolerance of a
comparison is then a fixed floor (the 1e-4 of the float32 gates) plus this
allowance, so that well-conditioned vertices are held to the floor and
ill-conditioned ones (sharp or eccentric lobes seen at a grazing angle, an
azimuth pair of tiny norm) to what float32 inputs can determine.
"""

import numpy as np

ULP = 2.0 ** -24
REL = 4 * ULP          # four float32 units of relative perturbation per input


def _change(a, b):
    """|a - b| for [B] values or the Euclidean norm of the difference for
    [B, 3] vectors; equal infinities count as no change."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    same = np.asarray(a == b)
    d = np.where(same, 0.0, d)
    d = np.where(np.isnan(d), np.inf, np.abs(d))
    return d if d.ndim == 1 else np.sqrt((d * d).sum(-1))


def spread(f, inputs, rel=REL, n_random=8, seed=0, scales=None):
    """Allowance [B] for comparing a float32 kernel with f(*inputs).

    f maps a list of arrays (each [B, ...], extended precision) to [B]
    values or [B, 3] vectors. inputs are the float32 values the kernel was
    given, converted exactly. Each is perturbed relatively by `rel`, or,
    where `scales` gives an array for it, additively by that array (e.g. the
    size of a forward pass's rounding of each raw output). Returns max(sum of
    one-at-a-time changes, max change under joint random-sign
    perturbations)."""
    scales = scales or [None] * len(inputs)
    step = [x * rel if s is None else np.asarray(s, dtype=x.dtype) for x, s in zip(inputs, scales)]
    base = f(*inputs)
    B = inputs[0].shape[0]
    one_at_a_time = np.zeros(B)
    for i, x in enumerate(inputs):
        flat = x.reshape(B, -1)
        st = step[i].reshape(B, -1)
        for j in range(flat.shape[1]):
            xp = flat.copy()
            xp[:, j] = xp[:, j] + st[:, j]
            args = list(inputs)
            args[i] = xp.reshape(x.shape)
            one_at_a_time += _change(f(*args), base)
    rng = np.random.default_rng(seed)
    joint = np.zeros(B)
    for _ in range(n_random):
        args = [x + st * rng.choice([-1.0, 1.0], x.shape).astype(x.dtype) for x, st in zip(inputs, step)]
        joint = np.maximum(joint, _change(f(*args), base))
    return np.maximum(one_at_a_time, joint)
