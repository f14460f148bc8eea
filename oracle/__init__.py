"""FP64 CPU oracle for the ST-pRRTC space-time extend path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  The C part
(``st_oracle.c``) is built with gcc by :func:`build`; ``mlp.py`` is the NumPy
FP64 reference of the proposal network.
"""
from .binding import Oracle, Planner, build, lib_path  # noqa: F401
