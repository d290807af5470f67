"""MI355X (gfx950) tricubic B-spline orbital evaluator.

``binding`` exposes the C ABI of ``libbspline.so`` (see ``include/bspline.h``)
with the same function names; ``accounting`` holds the byte accounting used
for roofline fractions.  Importing the package does not load the library;
``import paper_1611_02665_amd.binding`` does, and fails if it is not built.
"""

from . import accounting  # noqa: F401

__all__ = ["accounting"]
