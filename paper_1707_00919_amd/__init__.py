"""MI355X (gfx950) parallel multicanonical simulations of the 2D Ising model.

Gross, Zierenberg, Weigel, Janke, "Massively parallel multicanonical
simulations": many walkers share one multicanonical weight table and fill one
histogram that drives the weight recursion W <- W / H; a production run at
the final weights estimates the density of states.  The work runs in
``libmuca.so`` (HIP kernels for gfx950 behind the C ABI of include/muca.h);
this package only binds it.
"""
from ._abi import LIB_PATH, MUCA_MAX_L, lib  # noqa: F401
from .solver import Batch, MucaError, Solver, state_bytes  # noqa: F401
from .server import Server  # noqa: F401
