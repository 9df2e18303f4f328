"""FP64 CPU oracle for NASG neural path guiding (arXiv 2303.08064).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark do. It shares no code, table or constant
generator with the HIP path under ``paper_2303_08064_amd/csrc``.

What it computes, in plain float64 PyTorch CPU ops:

* ``mlp``   -- the bias-free MLP of Sec. 4.1 (input padded with a constant one
               as the bias surrogate), with an optional BF16-emulation mode.
* ``encoding`` -- the encoded input of Tab. "encoding": one-blob bins of the
               position, then omega_o and n.
* ``nasg``  -- output decoding (Tab. "decoding", Euler frame of Sec. 4.1), the
               NASG lobe exactly as printed (eq. NASG; App. A with epsilon),
               its closed-form normaliser (eq. "K for NASG", App. B), the
               normalised mixture (Sec. 3.1) and the direct sampler of App. C
               written with arccos / arctan / tan as printed.
* ``train`` -- the one-sample KL gradient of Sec. 4.2 as a weighted NLL, its
               gradient by float64 autograd, and textbook Adam.

Readings of the paper where it is silent (each repeated where it is used):

* the one-blob encoding (Tab. "encoding") gives each position coordinate 19
  bins (57 = 3 x 19); bin i holds a Gaussian of standard deviation 1/19
  centred at the coordinate, evaluated at the bin centre (i + 1/2)/19;
* raw output order is parameter-major, lobe-minor: for lobe k and parameter p
  the raw value is ``o[p*K + k]`` with p = 0..7 meaning
  (cos theta, sin phi, cos phi, sin tau, cos tau, log lambda, log a, logit);
  a network with the selection probability c of Sec. 4.2 has one more
  output, ``o[8K]``, decoded as sigmoid;
* the blended loss of Sec. 4.2 uses q_hat = c q + (1 - c) p_fs with the
  BSDF pdf p_fs supplied per sample; the blend ramp b of Sec. 5 rises by
  1/B after every M images (M = 4, B = 64), capped at 1;
* sin theta = sqrt(1 - cos^2 theta); the (cos, sin) pairs of phi and tau are
  divided by their norm so the frame is exactly orthonormal (a zero pair maps
  to (1, 0)); y = z x x;
* log lambda and log a are clamped to [-15, 15] before exponentiation;
* directions are divided by their norm before evaluation;
* the mixture component is chosen by inverse CDF over A in lobe order: the
  smallest k with xi_sel < A_0 + ... + A_k (the last lobe with A_k > 0 if
  rounding leaves none);
* the sampler's linear maps are s = xi0 + (1 - xi0) exp(-2 lambda),
  rho = pi (xi1 - 1/2); xi2 > 1/2 selects the eastern map.

Parity unpinned: the conventions above (output order, pair normalisation,
clamp range, component-selection rule, the orientation of the linear maps)
are not fixed by the paper; the distributional pins in the test suite hold
independently of them.
"""

from . import encoding, mlp, nasg, train  # noqa: F401
