"""Python face of the serving form (muca_server_* of include/muca.h).

A ``Server`` queues complete multicanonical solves, admits them by device
footprint, runs them with continuous batching and hands back ln g per
request.  ``progress()`` never blocks; a driver loop calls it between
submissions.
"""
import ctypes
import time

import numpy as np

from . import _abi
from .solver import MucaError


class Server:
    def __init__(self, mem_cap_bytes, max_active_walkers=0, batch_flags=0, policy="fifo", max_wait_s=0.0):
        """policy: "fifo" admits in arrival order; "smallest-first" admits the
        queued request of least estimated work (walkers * N * its sweeps, with
        about N/20 weight iterations) first, except that a request queued for
        longer than max_wait_s (0: 30 s) goes before any other."""
        policies = {"fifo": _abi.MUCA_SERVE_FIFO, "smallest-first": _abi.MUCA_SERVE_SMALLEST_FIRST}
        if policy not in policies:
            raise ValueError("policy must be 'fifo' or 'smallest-first'")
        self._lib = _abi.lib()
        self._s = ctypes.c_void_p()
        cfg = _abi.ServerConfig(int(mem_cap_bytes), int(max_active_walkers), int(batch_flags), policies[policy],
                                float(max_wait_s))
        rc = self._lib.muca_server_create(ctypes.byref(cfg), ctypes.byref(self._s))
        if rc != _abi.MUCA_OK:
            msg = self._lib.muca_server_last_error(None)
            raise MucaError(rc, msg.decode() if msg else "")
        self._L = {}

    def _check(self, rc):
        if rc != _abi.MUCA_OK:
            msg = self._lib.muca_server_last_error(self._s)
            raise MucaError(rc, msg.decode() if msg else "")

    def submit(self, L, walkers, seed, iter_sweeps=200, min_flatness=0.5, prod_therm=2000,
               prod_sweeps=2000, iter_therm=0, max_iterations=0, flags=0):
        """Queue one solve; returns its ticket."""
        q = _abi.Request(float(min_flatness), int(L), int(walkers), int(seed) & 0xFFFFFFFF,
                         int(flags), int(iter_therm), int(iter_sweeps), int(max_iterations),
                         int(prod_therm), int(prod_sweeps), 0)
        t = ctypes.c_uint64()
        self._check(self._lib.muca_server_submit(self._s, ctypes.byref(q), ctypes.byref(t)))
        self._L[t.value] = int(L)
        return t.value

    def progress(self):
        """Collect finished rounds, admit, launch; returns the number of events."""
        ev = ctypes.c_uint32()
        self._check(self._lib.muca_server_progress(self._s, ctypes.byref(ev)))
        return ev.value

    def take(self, ticket):
        """(result dict, ln g) of a finished request, or None while it runs."""
        L = self._L[ticket]
        res = _abi.Result()
        lng = np.zeros(L * L + 1, dtype=np.float64)
        rc = self._lib.muca_server_take(self._s, ticket, ctypes.byref(res),
                                        ctypes.c_void_p(lng.ctypes.data), lng.size)
        if rc == _abi.MUCA_PENDING:
            return None
        self._check(rc)
        del self._L[ticket]
        return res.as_dict(), lng

    def stats(self):
        c = _abi.ServerCounters()
        self._check(self._lib.muca_server_stats(self._s, ctypes.byref(c)))
        return c.as_dict()

    def drain(self, tickets, timeout_s=600.0, idle_sleep_s=2e-4):
        """Drive the server until every ticket is done; {ticket: (result, ln g)}."""
        out = {}
        left = set(tickets)
        t0 = time.monotonic()
        while left:
            if not self.progress():
                time.sleep(idle_sleep_s)
            for t in list(left):
                r = self.take(t)
                if r is not None:
                    out[t] = r
                    left.discard(t)
            if time.monotonic() - t0 > timeout_s:
                raise TimeoutError("%d requests still running" % len(left))
        return out

    def close(self):
        if self._s:
            self._lib.muca_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
