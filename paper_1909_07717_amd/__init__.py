"""MI355X-native SBIP-DPPS passing-point search (arXiv 1909.07717, Sec. 4.2-4.3).

Importing the package loads nothing native.  The HIP library is loaded on first
use by :mod:`paper_1909_07717_amd.binding`; the seeded input generator lives in
:mod:`paper_1909_07717_amd.framegen` and holds none of the method's arithmetic.
"""

__all__ = ["framegen", "binding", "flops"]
