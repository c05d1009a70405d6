"""Production analysis (muca_jackknife_log_dos, muca_canonical of
include/muca.h): jackknife error bars on ln g over the blocks of a
production run, and canonical averages by reweighting (Sec. 2.1, Sec. 3.3).
Host-side functions of libmuca; no device is needed."""
import ctypes

import numpy as np

from . import _abi
from .solver import MucaError


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _blocks(L, block_hists, omega):
    h = np.ascontiguousarray(block_hists, dtype=np.uint64)
    if h.ndim == 1:
        h = h[None, :]
    om = np.ascontiguousarray(omega, dtype=np.float64)
    if h.shape[1] != L * L + 1 or om.shape != (L * L + 1,):
        raise ValueError("block_hists must be (blocks, L*L+1) and omega L*L+1 values")
    return h, om


def production_blocks(solver, therm_sweeps, sweeps_per_block, blocks):
    """A production run as `blocks` calls; returns the (blocks, N+1) block
    histograms (the first call also runs the unrecorded sweeps)."""
    out = np.zeros((blocks, solver.N + 1), dtype=np.uint64)
    for b in range(blocks):
        solver.production(therm_sweeps if b == 0 else 0, sweeps_per_block)
        out[b] = solver.histogram()
    return out


def jackknife_log_dos(L, block_hists, omega, normalization=1):
    """(ln g, jackknife error) per bin."""
    h, om = _blocks(L, block_hists, omega)
    lng = np.zeros(L * L + 1)
    err = np.zeros(L * L + 1)
    rc = _abi.lib().muca_jackknife_log_dos(L, h.shape[0], _p(h), _p(om), normalization,
                                           _p(lng), _p(err))
    if rc != _abi.MUCA_OK:
        raise MucaError(rc, "jackknife_log_dos")
    return lng, err


def canonical(L, block_hists, omega, betas):
    """(energy per spin, its error, specific heat per spin, its error) at
    each beta."""
    h, om = _blocks(L, block_hists, omega)
    b = np.ascontiguousarray(np.atleast_1d(betas), dtype=np.float64)
    e, ee, c, ce = (np.zeros(b.size) for _ in range(4))
    rc = _abi.lib().muca_canonical(L, h.shape[0], _p(h), _p(om), b.size, _p(b), _p(e), _p(ee),
                                   _p(c), _p(ce))
    if rc != _abi.MUCA_OK:
        raise MucaError(rc, "canonical")
    return e, ee, c, ce
