"""CPU FP64 oracle for the two-sided sketched rank estimator (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may import this
package.  The product library never does.
"""
from .pyoracle import *  # noqa: F401,F403
from . import learned  # noqa: F401,E402
from . import gap  # noqa: F401,E402
from . import rangefinder  # noqa: F401,E402
from . import qrdiag  # noqa: F401,E402
from . import hrtt  # noqa: F401,E402
