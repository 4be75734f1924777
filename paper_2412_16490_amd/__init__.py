"""MI355X-native batched contact-force QP of BODex (arXiv 2412.16490).

The compute path is a HIP (gfx950) shared library behind a C ABI
(``include/bodex_qp.h``); this package is its thin ctypes binding plus the
seeded workload generator, the autograd wrapper, the batched/persistent
launcher and the serving loop.
"""
from . import workload  # noqa: F401
