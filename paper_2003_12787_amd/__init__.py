"""MI355X-native space-time predictor (STP) of the linear ADER-DG scheme (arXiv:2003.12787).

The predictor runs in hand-written HIP kernels for gfx950 behind the C ABI of ``libstp.so``
(``include/stp.h``); ``stp`` is its Python binding and ``workloads`` the seeded synthetic inputs.
"""
from . import stp, workloads  # noqa: F401
