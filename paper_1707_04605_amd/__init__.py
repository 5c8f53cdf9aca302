"""mgrt: leap-frog FE wave stepping and coarse-level linearisation (arXiv 1707.04605)
on MI355X, behind the C ABI of libmgrt.so (include/mgrt.h).

The binding loads the in-tree library and raises if it is not built: there is no CPU
fallback in this package.
"""
from .api import Context, context_for_problem, projection_weights  # noqa: F401
from .native import MgrtError  # noqa: F401
