"""FP64 CPU oracle of the P-SWA wavefront context model.

TEST INFRASTRUCTURE ONLY. Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the
product path (the HIP library and its Python binding) never does, and shares
no code with it. The oracle is plain NumPy/SciPy in float64: slow, unblocked
and written to be checked against the paper by eye.

Submodules:
  model   -- schedule, window geometry, parallel (definition) form and the
             order-parameterised sequential form of the context model.
  entropy -- discretized-Gaussian likelihood, bits, integer CDF tables and
             the per-symbol table selection.
  train   -- the student's distillation step: the same forward restated in
             torch float64, loss, autograd gradients and AdamW (imported on
             its own: `from oracle import train`).
"""
from . import model, entropy  # noqa: F401
