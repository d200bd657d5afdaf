"""MI355X (gfx950) halo-exchange buffer engine.

The rank-local work under a persistent neighborhood all-to-all-v (MPI
Advance, Sec. 2.2): GPU plan building (halo discovery, send-list transpose,
locality-aware node dedup and on-node redistribution lists), the pack
gather (Start), the redistribution pack and unpack (Wait), batched launches
captured in hipGraphs with a schedule tuner, and a fixed-order backward.

``_lib`` is the ctypes binding of ``libhx.so`` (names as in include/hx.h);
``autograd`` adds the differentiable whole-decomposition exchange.
"""
from . import _lib
from ._lib import *  # noqa: F401,F403
from ._lib import HXError, load

__all__ = [n for n in dir(_lib) if n.startswith("hx_") or n.startswith("HX_")] + [
    "HXError", "load", "HaloExchange", "HaloGather", "halo_gather"]


def __getattr__(name):
    if name in ("HaloExchange", "HaloGather", "halo_gather"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
