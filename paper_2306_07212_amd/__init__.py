"""Python binding of libpcx.so: MI355X edge-subdivision polyhedral complex
extraction from ReLU networks (Berzins, ICML 2023).

Argument marshalling only: every step of the extraction runs in the HIP
kernels behind the C ABI of ``include/pcx.h``. There is no CPU fallback; if
the library is not built, importing ``paper_2306_07212_amd.pcx`` raises.
"""
from . import workloads  # noqa: F401  (seeded synthetic inputs; no method arithmetic)
