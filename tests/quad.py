"""Composite Gauss-Legendre quadrature on the sphere for the oracle's pins.

Test helper, independent of the oracle's arithmetic: it only produces nodes
and weights in (mu = cos theta, phi) about a given frame.
"""

import numpy as np


def gl_panels(breaks, n=16):
    """Nodes and weights of n-point Gauss-Legendre on each panel [b_i, b_{i+1}]."""
    x, w = np.polynomial.legendre.leggauss(n)
    breaks = np.asarray(breaks, dtype=np.float64)
    a, b = breaks[:-1, None], breaks[1:, None]
    pts = 0.5 * (a + b) + 0.5 * (b - a) * x
    wts = 0.5 * (b - a) * w
    return pts.ravel(), wts.ravel()


def mu_breaks(n=48, dmin=1e-15):
    """Panels on [-1, 1] graded geometrically toward both poles."""
    d = np.geomspace(dmin, 1.0, n)
    return np.unique(np.concatenate([[-1.0, 0.0, 1.0], 1.0 - d, -1.0 + d]))


def phi_breaks(n=36, dmin=1e-9):
    """Panels on [0, 2 pi] graded toward pi/2 and 3 pi/2 (where a cos^2 phi -> 0)."""
    d = np.geomspace(dmin, np.pi / 2, n)
    pts = [0.0, 2 * np.pi]
    for c in (np.pi / 2, 3 * np.pi / 2):
        pts += list(c - d) + list(c + d) + [c]
    return np.unique(np.clip(pts, 0.0, 2 * np.pi))


def sphere_nodes(z, x, y, mu_b=None, phi_b=None, n=16):
    """Directions [M, P, 3] and weights [M, P] for integrating over S^2 with
    d omega = d mu d phi, mu measured along z and phi from x toward y."""
    mu, wm = gl_panels(mu_breaks() if mu_b is None else mu_b, n)
    ph, wp = gl_panels(phi_breaks() if phi_b is None else phi_b, n)
    r = np.sqrt(np.clip(1.0 - mu * mu, 0.0, None))
    c, s = np.cos(ph), np.sin(ph)
    v = (r[:, None, None] * (c[None, :, None] * x + s[None, :, None] * y)
         + mu[:, None, None] * z)
    return v, wm[:, None] * wp[None, :]
