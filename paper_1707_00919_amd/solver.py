"""Python face of libmuca: one ``Solver`` per multicanonical instance.

Every method is a direct call into the C ABI of include/muca.h; PyTorch is
used only to hand the library device memory (a uint8 workspace tensor) and
the current HIP stream.  All arithmetic of the method runs in libmuca.
"""
import ctypes

import numpy as np

from . import _abi


class MucaError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("%s: %s" % (_abi.STATUS_NAMES.get(code, str(code)), message))
        self.code = code


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def state_bytes(L, walkers, seed=0, flags=0):
    """Device bytes an instance holds (0 for invalid parameters)."""
    p = _abi.MucaParams(L, walkers, seed & 0xFFFFFFFF, flags)
    return int(_abi.lib().muca_state_bytes(ctypes.byref(p)))


class Solver:
    """A population of ``walkers`` independent walkers on L x L lattices that
    share one weight table (Sec. 2.2 of the paper).

    use_torch: take the workspace from torch's caching allocator and run on
    torch's current stream (default); otherwise libmuca allocates its own
    memory and stream.
    """

    def __init__(self, L, walkers, seed, flags=0, use_torch=True, device=None):
        self._lib = _abi.lib()
        self.L, self.walkers, self.seed = int(L), int(walkers), int(seed) & 0xFFFFFFFF
        self.N = self.L * self.L
        self._h = ctypes.c_void_p()
        self._workspace = None
        p = _abi.MucaParams(self.L, self.walkers, self.seed, flags)
        nbytes = self._lib.muca_state_bytes(ctypes.byref(p))
        stream = None
        ws = None
        if use_torch and nbytes:
            import torch
            if not torch.cuda.is_available():
                raise MucaError(_abi.MUCA_ERR_DEVICE, "no GPU is visible to torch (this library runs on the GPU only)")
            dev = torch.device(device if device is not None else "cuda")
            with torch.cuda.device(dev):
                self._workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
                stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
            ws = ctypes.c_void_p(self._workspace.data_ptr())
        rc = self._lib.muca_create(ctypes.byref(p), stream, ws, nbytes, ctypes.byref(self._h))
        if rc != _abi.MUCA_OK:
            msg = self._lib.muca_last_error(None)
            self._workspace = None
            raise MucaError(rc, msg.decode() if msg else "")
        self.state_bytes = int(nbytes)

    # ------------------------------------------------------------- lifecycle
    def close(self):
        if self._h:
            self._lib.muca_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        if rc != _abi.MUCA_OK:
            msg = self._lib.muca_last_error(self._h)
            raise MucaError(rc, msg.decode() if msg else "")

    # ------------------------------------------------------------- the method
    def iterate(self, therm_sweeps, sweeps):
        """One weight iteration: sweeps, summed histogram, Eq. 4 update."""
        info = _abi.MucaInfo()
        self._check(self._lib.muca_iterate(self._h, therm_sweeps, sweeps, ctypes.byref(info)))
        return info.as_dict()

    def production(self, therm_sweeps, sweeps):
        """Sweeps at frozen weights; replaces the stored histogram."""
        info = _abi.MucaInfo()
        self._check(self._lib.muca_production(self._h, therm_sweeps, sweeps, ctypes.byref(info)))
        return info.as_dict()

    def iterate_attempts(self, therm_attempts, attempts):
        """A weight iteration counted in attempted flips per walker; it may
        start and stop inside a sweep."""
        info = _abi.MucaInfo()
        self._check(self._lib.muca_iterate_attempts(self._h, therm_attempts, attempts,
                                                    ctypes.byref(info)))
        return info.as_dict()

    def production_attempts(self, therm_attempts, attempts):
        info = _abi.MucaInfo()
        self._check(self._lib.muca_production_attempts(self._h, therm_attempts, attempts,
                                                       ctypes.byref(info)))
        return info.as_dict()

    def run_schedule(self, z=2.25, growth=1.1, dk_flat=1e-4, f_therm=30, w_min=10,
                     max_iterations=1000, stop="kl", dc_flat=0.05):
        """The paper's iteration schedule (Sec. 3) to its stop rule: d_k <
        dk_flat (Eq. 6), or with stop="chebyshev" d_c < dc_flat (App. A).
        Returns (converged, [step dicts])."""
        rules = {"kl": _abi.MUCA_STOP_KL, "chebyshev": _abi.MUCA_STOP_CHEBYSHEV}
        if stop not in rules:
            raise ValueError("stop must be 'kl' or 'chebyshev'")
        sc = _abi.Schedule(z, growth, dk_flat, dc_flat, f_therm, w_min, max_iterations, rules[stop])
        steps = (_abi.ScheduleStep * max_iterations)()
        n = ctypes.c_uint32()
        rc = self._lib.muca_run_schedule(self._h, ctypes.byref(sc), steps, max_iterations,
                                         ctypes.byref(n))
        if rc not in (_abi.MUCA_OK, _abi.MUCA_ERR_NOT_CONVERGED):
            self._check(rc)
        return rc == _abi.MUCA_OK, [steps[i].as_dict() for i in range(n.value)]

    # ---------------------------------------------------------------- outputs
    def histogram(self):
        out = np.zeros(self.N + 1, dtype=np.uint64)
        self._check(self._lib.muca_histogram(self._h, _ptr(out), out.size))
        return out

    def log_weights(self):
        out = np.zeros(self.N + 1, dtype=np.float64)
        self._check(self._lib.muca_log_weights(self._h, _ptr(out), out.size))
        return out

    def set_log_weights(self, omega):
        om = np.ascontiguousarray(omega, dtype=np.float64)
        self._check(self._lib.muca_set_log_weights(self._h, _ptr(om), om.size))

    def thresholds(self):
        out = np.zeros((self.N + 1) * 5, dtype=np.uint64)
        self._check(self._lib.muca_thresholds(self._h, _ptr(out), out.size))
        return out.reshape(self.N + 1, 5)

    def energies(self):
        out = np.zeros(self.walkers, dtype=np.int32)
        self._check(self._lib.muca_energies(self._h, _ptr(out), out.size))
        return out

    def spins(self):
        out = np.zeros(self.walkers * self.N, dtype=np.int8)
        self._check(self._lib.muca_spins(self._h, _ptr(out), out.size))
        return out.reshape(self.walkers, self.N)

    def log_dos(self, normalization=0):
        out = np.zeros(self.N + 1, dtype=np.float64)
        self._check(self._lib.muca_log_dos(self._h, normalization, _ptr(out), out.size))
        return out

    def checkpoint(self):
        """The instance's whole state as bytes (restore with ``restore``)."""
        n = int(self._lib.muca_checkpoint_bytes(self._h))
        buf = np.zeros(n, dtype=np.uint8)
        self._check(self._lib.muca_checkpoint(self._h, _ptr(buf), n))
        return buf.tobytes()

    def restore(self, state):
        """Continue from a checkpoint of an instance with the same L, walkers, seed."""
        buf = np.frombuffer(state, dtype=np.uint8).copy()
        self._check(self._lib.muca_restore(self._h, _ptr(buf), buf.size))

    def last_info(self):
        info = _abi.MucaInfo()
        self._check(self._lib.muca_last_info(self._h, ctypes.byref(info)))
        return info.as_dict()


def production_static(L, walkers, seed, sweep0, therm_sweeps, sweeps, omega, spins, energies, flags=0):
    """muca_production_static: production sweeps on caller-owned device
    lattices and energies (torch tensors in an instance's layout, see
    include/muca.h) on torch's current stream; the library allocates nothing.
    Returns the histogram (N + 1 counts)."""
    import torch
    lib = _abi.lib()
    L, walkers = int(L), int(walkers)
    p = _abi.MucaParams(L, walkers, int(seed) & 0xFFFFFFFF, flags)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    if om.size != L * L + 1:
        raise ValueError("omega must hold L*L+1 values")
    if not (spins.is_cuda and energies.is_cuda and spins.is_contiguous() and energies.is_contiguous()):
        raise ValueError("spins and energies must be contiguous device tensors")
    hist = np.zeros(L * L + 1, dtype=np.uint64)
    stream = ctypes.c_void_p(torch.cuda.current_stream(spins.device).cuda_stream)
    rc = lib.muca_production_static(ctypes.byref(p), int(sweep0), int(therm_sweeps), int(sweeps), _ptr(om),
                                    ctypes.c_void_p(spins.data_ptr()), ctypes.c_void_p(energies.data_ptr()),
                                    _ptr(hist), stream)
    if rc != _abi.MUCA_OK:
        msg = lib.muca_last_error(None)
        raise MucaError(rc, msg.decode() if msg else "")
    return hist


class Batch:
    """Many independent Solvers swept together (the batched form): one round
    runs a weight iteration, a production call or nothing for every member,
    with all members' walkers on the device at once.  Each member's results
    are bit-identical to running it alone.

    flags: ``_abi.MUCA_BATCH_GRAPH`` (replay a captured HIP graph while the
    round's shape is unchanged), ``_abi.MUCA_BATCH_AUTOTUNE`` (time the two
    kernel forms on the first rounds and keep the faster).
    """

    SKIP, ITERATE, PRODUCTION = (_abi.MUCA_BATCH_SKIP, _abi.MUCA_BATCH_ITERATE,
                                 _abi.MUCA_BATCH_PRODUCTION)

    def __init__(self, solvers, flags=0, use_torch=True):
        self._lib = _abi.lib()
        self.members = list(solvers)
        self._b = ctypes.c_void_p()
        handles = (ctypes.c_void_p * len(self.members))(*[s._h.value for s in self.members])
        stream = None
        if use_torch:
            import torch
            stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = self._lib.muca_batch_create(handles, len(self.members), stream, flags,
                                         ctypes.byref(self._b))
        if rc != _abi.MUCA_OK:
            msg = self._lib.muca_batch_last_error(None)
            raise MucaError(rc, msg.decode() if msg else "")

    def set_members(self, solvers):
        """Replace the members between rounds (buffers are reused when they fit)."""
        members = list(solvers)
        handles = (ctypes.c_void_p * len(members))(*[s._h.value for s in members])
        self._check(self._lib.muca_batch_set_members(self._b, handles, len(members)))
        self.members = members

    def _check(self, rc):
        if rc != _abi.MUCA_OK:
            msg = self._lib.muca_batch_last_error(self._b)
            raise MucaError(rc, msg.decode() if msg else "")

    def submit(self, modes, therm, sweeps):
        """Enqueue one round without waiting for it."""
        n = len(self.members)
        self._mode = np.ascontiguousarray(np.broadcast_to(modes, (n,)), dtype=np.uint32)
        th = np.ascontiguousarray(np.broadcast_to(therm, (n,)), dtype=np.uint32)
        sw = np.ascontiguousarray(np.broadcast_to(sweeps, (n,)), dtype=np.uint32)
        self._check(self._lib.muca_batch_submit(self._b, _ptr(self._mode), _ptr(th), _ptr(sw)))

    def done(self):
        """True once the submitted round has finished on the device."""
        rc = self._lib.muca_batch_query(self._b)
        if rc == _abi.MUCA_PENDING:
            return False
        self._check(rc)
        return True

    def finish(self):
        """Wait for the submitted round; per-member info dicts (None: skipped)."""
        n = len(self.members)
        infos = (_abi.MucaInfo * n)()
        self._check(self._lib.muca_batch_finish(self._b, infos))
        return [infos[i].as_dict() if self._mode[i] else None for i in range(n)]

    def run(self, modes, therm, sweeps):
        """One round: submit, then finish."""
        self.submit(modes, therm, sweeps)
        return self.finish()

    def close(self):
        if self._b:
            self._lib.muca_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
