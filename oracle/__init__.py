"""FP64 CPU oracle of the plane-wave multiple-scattering transmission.

TEST INFRASTRUCTURE ONLY.  It exists to check the HIP library.  Only the test
suite, the package smoke check and the benchmark's CPU-baseline leg may import
it; the library and its binding never do.  It shares no code with the HIP
path: both consume the same seeded inputs (``msgen``) and nothing else.
"""
from .transport import *  # noqa: F401,F403
from .transport import __all__ as _t_all
from .bands import *  # noqa: F401,F403
from .bands import __all__ as _b_all

__all__ = list(_t_all) + list(_b_all)
