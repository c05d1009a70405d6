"""CPU oracle for the parallel multicanonical method -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the GPU library
(``paper_1707_00919_amd``) and never imports it; the two meet only through
``muca_inputs`` (seeded synthetic inputs, none of the method's arithmetic).

Contents
  * ``OracleMuca``     -- the walker population of Sec. 2.2 stepped by the
                          plain C chain in ``muca_oracle.c``, with the host
                          weight update of Eq. 4 and the production run of
                          Sec. 3.3.
  * ``exact_dos``      -- exact density of states of the periodic L x L Ising
                          model: brute force, transfer matrix, and Kaufman's
                          closed form (the ground truth named in Sec. 3).
  * ``protocol``       -- the paper's weight-iteration schedule (Sec. 3, Eq. 7;
                          stop rules of Eq. 6 and App. A) driving OracleMuca.
  * ``analysis``       -- jackknife errors over production blocks and canonical
                          averages by reweighting (Sec. 2.1, Sec. 3.3), with
                          brute-force and transfer-matrix references.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def lib():
    """Load (building if needed) the C oracle."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        c = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_int8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.POINTER(ctypes.c_double)
        c.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        c.oracle_philox4x32_10.restype = None
        c.oracle_draw.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.c_uint32, ctypes.c_uint32]
        c.oracle_draw.restype = ctypes.c_uint32
        c.oracle_energy.argtypes = [ctypes.c_int, u8p]
        c.oracle_energy.restype = ctypes.c_int32
        c.oracle_init.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, u8p, i32p]
        c.oracle_init.restype = None
        c.oracle_thresholds.argtypes = [ctypes.c_int, dp, u64p]
        c.oracle_thresholds.restype = None
        c.oracle_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, u8p, i32p, u64p,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, u64p,
                                    ctypes.c_int]
        c.oracle_sweeps.restype = None
        c.oracle_init_ids.argtypes = [ctypes.c_int, ctypes.c_int, u32p, ctypes.c_uint32, u8p,
                                      i32p]
        c.oracle_init_ids.restype = None
        c.oracle_sweeps_ids.argtypes = [ctypes.c_int, ctypes.c_int, u32p, ctypes.c_uint32, u8p,
                                        i32p, u64p, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_int, u64p, ctypes.c_int]
        c.oracle_sweeps_ids.restype = None
        c.oracle_attempts_ids.argtypes = [ctypes.c_int, ctypes.c_int, u32p, ctypes.c_uint32, u8p,
                                          i32p, u64p, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_int, u64p, ctypes.c_int]
        c.oracle_attempts_ids.restype = None
        c.oracle_reweight.argtypes = [ctypes.c_int, dp, u64p]
        c.oracle_reweight.restype = None
        c.oracle_flatness.argtypes = [ctypes.c_int, u64p]
        c.oracle_flatness.restype = ctypes.c_double
        c.oracle_chebyshev.argtypes = [ctypes.c_int, u64p]
        c.oracle_chebyshev.restype = ctypes.c_double
        c.oracle_kl_divergence.argtypes = [ctypes.c_int, u64p, ctypes.c_int]
        c.oracle_kl_divergence.restype = ctypes.c_double
        c.oracle_width.argtypes = [ctypes.c_int, u64p]
        c.oracle_width.restype = ctypes.c_int
        c.oracle_reachable_width.argtypes = [ctypes.c_int, u64p]
        c.oracle_reachable_width.restype = ctypes.c_int
        c.oracle_log_dos.argtypes = [ctypes.c_int, u64p, dp, ctypes.c_int, dp]
        c.oracle_log_dos.restype = ctypes.c_int
        _lib = c
    return _lib


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# ---------------------------------------------------------------- primitives
def philox4x32_10(counter, key):
    """Raw Philox4x32-10 block: four uint32 outputs for a 4-word counter and
    2-word key (Salmon et al. 2011, the generator chosen in Sec. 2.3)."""
    c = np.asarray(counter, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32),
                               _p(out, ctypes.c_uint32))
    return out


def draw(seed, walker, sweep, site, domain=0):
    return int(lib().oracle_draw(seed, walker, sweep, site, domain))


def energy(L, spins):
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    assert s.size == L * L
    return int(lib().oracle_energy(L, _p(s, ctypes.c_int8)))


def thresholds(N, omega):
    """T[(N+1), 5] uint64 for the log weights omega (Sec. 2.3 acceptance)."""
    om = np.ascontiguousarray(omega, dtype=np.float64)
    assert om.size == N + 1
    t = np.zeros((N + 1) * 5, dtype=np.uint64)
    lib().oracle_thresholds(N, _p(om, ctypes.c_double), _p(t, ctypes.c_uint64))
    return t.reshape(N + 1, 5)


def reweight(omega, hist):
    """Eq. 4 in logarithmic form: omega - ln H on bins with H > 0."""
    om = np.array(omega, dtype=np.float64)
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    lib().oracle_reweight(om.size - 1, _p(om, ctypes.c_double), _p(h, ctypes.c_uint64))
    return om


def flatness(hist):
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    return float(lib().oracle_flatness(h.size - 1, _p(h, ctypes.c_uint64)))


def chebyshev(hist):
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    return float(lib().oracle_chebyshev(h.size - 1, _p(h, ctypes.c_uint64)))


def kl_divergence(hist, reach_prev):
    """Eq. 6 with Q = 1/max(reach_prev, 10); reach_prev = reachable bins in
    the previous recorded histogram's range."""
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    return float(lib().oracle_kl_divergence(h.size - 1, _p(h, ctypes.c_uint64), reach_prev))


def reachable_width(hist):
    """Reachable bins inside the covered energy range."""
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    return int(lib().oracle_reachable_width(h.size - 1, _p(h, ctypes.c_uint64)))


def width(hist):
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    return int(lib().oracle_width(h.size - 1, _p(h, ctypes.c_uint64)))


def log_dos(hist, omega, norm=0):
    """ln g from a production histogram; norm 0: ln g(E_min) = ln 2,
    norm 1: sum exp(ln g) = 2^N (Sec. 3.3).  None if the anchor is empty."""
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.zeros(h.size, dtype=np.float64)
    rc = lib().oracle_log_dos(h.size - 1, _p(h, ctypes.c_uint64), _p(om, ctypes.c_double),
                              norm, _p(out, ctypes.c_double))
    return None if rc != 0 else out


def reachable_mask(N):
    m = np.ones(N + 1, dtype=bool)
    m[1] = False
    m[N - 1] = False
    return m


# ---------------------------------------------------------------- the chain
class OracleMuca:
    """p walkers with one shared weight table (Sec. 2.2), stepped on the CPU.

    Mirrors the call semantics of the GPU library: ``iterate`` runs
    ``therm`` unrecorded sweeps, then ``sweeps`` recorded ones, sums the
    walker histograms and applies the weight update; ``production`` does the
    same with the weights frozen.  One sweep counter per instance, never
    reset, labels the random numbers of every sweep.

    walker_ids: run only these global walker indices (each walker's chain
    depends on its own index alone), e.g. a sample of a large population;
    the histogram then covers the sample only.
    """

    def __init__(self, L, walkers, seed, nthreads=0, walker_ids=None):
        if L < 4 or L % 2:
            raise ValueError("L must be even and >= 4")
        self.ids = None
        if walker_ids is not None:
            self.ids = np.ascontiguousarray(walker_ids, dtype=np.uint32)
            walkers = self.ids.size
        if walkers < 1:
            raise ValueError("walkers must be >= 1")
        self.L, self.W, self.seed = int(L), int(walkers), int(seed) & 0xFFFFFFFF
        self.N = self.L * self.L
        self.nthreads = nthreads
        self.spins = np.zeros((self.W, self.N), dtype=np.int8)
        self.energies = np.zeros(self.W, dtype=np.int32)
        lib().oracle_init_ids(self.L, self.W, self._ids_ptr(), self.seed,
                              _p(self.spins, ctypes.c_int8), _p(self.energies, ctypes.c_int32))
        self.omega = np.zeros(self.N + 1, dtype=np.float64)
        self.hist = np.zeros(self.N + 1, dtype=np.uint64)
        self.table = thresholds(self.N, self.omega)
        self.position = 0     # attempts made per walker so far
        self.iteration = 0
        self.width_prev = 0   # covered range of the previous recorded call, in bins
        self.reach_prev = 0   # reachable bins inside it

    def _ids_ptr(self):
        return None if self.ids is None else _p(self.ids, ctypes.c_uint32)

    def set_log_weights(self, omega):
        om = np.asarray(omega, dtype=np.float64)
        if om.shape != (self.N + 1,) or not np.all(np.isfinite(om)):
            raise ValueError("omega must be N+1 finite values")
        self.omega = om.copy()

    @property
    def sweep_counter(self):
        """Whole sweeps made per walker so far."""
        return self.position // self.N

    def _attempts(self, count, record):
        h = np.zeros(self.N + 1, dtype=np.uint64)
        if count:
            t = np.ascontiguousarray(self.table.reshape(-1))
            lib().oracle_attempts_ids(self.L, self.W, self._ids_ptr(), self.seed,
                                      _p(self.spins, ctypes.c_int8),
                                      _p(self.energies, ctypes.c_int32), _p(t, ctypes.c_uint64),
                                      self.position, count, 1 if record else 0,
                                      _p(h, ctypes.c_uint64), self.nthreads)
            self.position += count
        return h

    def _run(self, therm, count):
        """therm unrecorded then count recorded attempts per walker."""
        self.table = thresholds(self.N, self.omega)
        self._attempts(therm, False)
        self.hist = self._attempts(count, True)
        h = self.hist
        info = {
            "attempts": self.W * (therm + count),
            "hist_sum": int(h.sum(dtype=np.uint64)),
            "sweep_counter": self.sweep_counter,
            "position": self.position,
            "visited_bins": int(np.count_nonzero(h)),
            "flatness": flatness(h),
            "kl_divergence": kl_divergence(h, self.reach_prev),
            "chebyshev": chebyshev(h),
            "width": width(h),
        }
        self.width_prev = width(h)
        self.reach_prev = reachable_width(h)
        return info

    def iterate_attempts(self, therm, count):
        """One weight iteration (Eq. 4) over therm + count attempts per walker."""
        info = self._run(therm, count)
        self.omega = reweight(self.omega, self.hist)
        self.iteration += 1
        info["iteration"] = self.iteration
        return info

    def production_attempts(self, therm, count):
        info = self._run(therm, count)
        info["iteration"] = self.iteration
        return info

    def iterate(self, therm, sweeps):
        return self.iterate_attempts(therm * self.N, sweeps * self.N)

    def production(self, therm, sweeps):
        return self.production_attempts(therm * self.N, sweeps * self.N)

    def log_dos(self, norm=0):
        return log_dos(self.hist, self.omega, norm)
