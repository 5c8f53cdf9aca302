"""FP64 CPU oracle: test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library (``paper_1707_04605_amd``) and
never imports it; the two meet only through the seeded inputs of ``synth``.

The heavy loops live in ``mgrt_oracle.c`` (plain C, FP64, OpenMP), built by
``oracle/build.py`` into ``oracle/liboracle.so``; ``tv.py`` holds the dense TV-IRLS
reference in NumPy.
"""
from .core import Oracle, load_library  # noqa: F401
from . import tv  # noqa: F401
