"""MI355X-native levelized sparse LU (GLU3.0's method) behind a C ABI.

``glu`` is the ctypes binding of ``include/glu.h``; the work runs in the HIP
library ``libglu_mi355x.so`` built by ``_build.build()``.
"""

from .glu import (  # noqa: F401
    GLU_MODE_AUTO,
    GLU_MODE_LARGE_BLOCK,
    GLU_MODE_SMALL_BLOCK,
    GLU_MODE_STREAM,
    GLU_ORDER_AMD,
    GLU_ORDER_NATURAL,
    GLU_ORDER_USER,
    GluError,
    Handle,
    lib,
)
