"""MI355X-native hot path of NASG online neural path guiding (arXiv 2303.08064).

* ``nasg``  -- torch binding of libnasg.so (query, pdf, sample, training)
* ``synth`` -- seeded synthetic vertex batches and targets
* ``build`` -- hipcc build of libnasg.so for gfx950

Submodules are imported on demand so that ``synth`` works without a GPU.
"""

__all__ = ["nasg", "synth", "build"]
