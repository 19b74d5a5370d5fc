"""MI355X-native double-grid on-the-fly BSE / Haydock library (gfx950 HIP).

The compute path lives in ``csrc/`` (HIP kernels behind the C ABI declared in
``include/bse_dg.h``) and is reached through the ctypes binding in ``bse``.
Import ``paper_1602_01863_amd.bse`` for the binding; it raises if the library
has not been built.
"""

__all__ = ["bse", "build"]
