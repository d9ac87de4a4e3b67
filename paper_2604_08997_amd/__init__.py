"""MI355X (gfx950) implementation of the SiPO PDHG hot path.

The compute runs in hand-written HIP kernels behind the C ABI of
``include/sipo.h`` (``libsipo.so``, built in-tree by ``build.py``); this
package is the thin Python binding over it.
"""
from .binding import (Plan, SipoError, lib, version, gaussian_taps, LIB_PATH,  # noqa: F401
                      PLAIN, RESTARTED, OPTIMAL, PRIMAL_INFEASIBLE, ITER_LIMIT, NUMERICAL, STATUS_NAMES,
                      LP, GENERAL, CASE1, CASE2, pdhg_options, solve)
from .autograd import SipoDose, dose  # noqa: F401,E402
from . import workflow  # noqa: F401,E402
