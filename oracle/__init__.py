"""Oracle: plain, slow, FP64 CPU implementation of the unbinned likelihood.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the library and its Python
binding never do, and the oracle imports nothing from them.  It shares no
kernel, header, helper, table or constant generator with the HIP path.

Modules:
  dual      forward-mode dual numbers (exact gradients by the chain rule)
  models    the three PDFs written from their definitions
  nll       -sum w ln P (exactly summed) and its gradient
  philox    Philox4x64-10 counter-based generator (Salmon et al., SC'11)
  generate  accept-reject toy generation from the Philox stream
"""
from . import dual, models, nll  # noqa: F401
