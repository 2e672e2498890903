"""MI355X (gfx950) hot path of the 3D XY model Monte Carlo of arXiv:1211.0780:
checkerboard Metropolis and over-relaxation sweeps, parallel-tempering
exchange and per-sweep observable reductions in hand-written HIP kernels
behind a C ABI (include/xy.h)."""
from ._capi import XYError  # noqa: F401


def Sim(*args, **kwargs):
    from .sim import Sim as _Sim
    return _Sim(*args, **kwargs)
