"""CPU oracle (test infrastructure only): plain float64 / exact-integer
separable lifting for the 2-D CDF 5/3 DWT (this package's top level, from
dwt53) and float64 separable lifting for the 2-D CDF 9/7 DWT (the dwt97
submodule).  Imported only by tests, the smoke check and the benchmark's
CPU-baseline leg; the product path never uses it."""
from .dwt53 import *  # noqa: F401,F403
from .dwt53 import __all__  # noqa: F401
