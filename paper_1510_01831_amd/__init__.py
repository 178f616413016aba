"""Nested polarized-traces Helmholtz solver for one MI355X (gfx950).

The package is split so that importing it has no side effects:

* ``media``  -- seeded synthetic velocity models, sources and receivers (input
  generation only; no arithmetic of the solver lives there).
* ``hz``     -- ctypes binding of the C-ABI library ``libhz.so`` (argument
  marshalling only; every step of the solve runs in the HIP kernels).
* ``autograd`` -- ``torch.autograd.Function`` wrapper of the misfit gradient.
* ``build``  -- compiles ``csrc/`` for gfx950 into ``libhz.so``.
"""

__all__ = ["media", "hz", "autograd", "build"]
