"""The allocation-free production call (muca_production_static) against the
instance's production call (muca_production), through the C ABI.

The caller's device lattices and energies start as copies of an instance's;
both calls then run the same production sweeps (Sec. 2.1 and Sec. 3.3: sweeps
at frozen weights whose histogram is the estimate's input).  Histogram,
lattices and energies must be bit-identical.  Calls follow one another on
the same static scratch: the largest lattice first, then smaller inputs, so a
histogram left over from an earlier call would show.
"""
import sys

import numpy as np
import pytest

from muca_inputs import random_log_weights, smooth_log_weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_1707_00919_amd
    paper_1707_00919_amd.lib()
    yield


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def instance_views(s):
    """The lattices and energies inside an instance's torch workspace, in the
    layout include/muca.h documents for muca_production_static (lattices
    first, energies at the next 256-byte boundary)."""
    import torch
    wpad = (s.walkers + 63) // 64 * 64
    words = s.L * ((s.L + 31) // 32)
    nsp = words * wpad * 4
    eoff = (nsp + 255) // 256 * 256
    ws = s._workspace
    return ws[:nsp].view(torch.int32), ws[eoff:eoff + 4 * wpad].view(torch.int32), words, wpad


def unpack(spins_words, L, walkers, words, wpad):
    """+-1 spins, walker-major, from the bit-packed site-major words."""
    w = spins_words.cpu().numpy().view(np.uint32).reshape(words, wpad)[:, :walkers]
    wpr = (L + 31) // 32
    out = np.zeros((walkers, L * L), dtype=np.int8)
    for y in range(L):
        for x in range(L):
            bit = (w[y * wpr + x // 32] >> np.uint32(x % 32)) & np.uint32(1)
            out[:, y * L + x] = np.where(bit == 1, 1, -1)
    return out


# (L, walkers, seed, omega kind, kernel flags, therm, recorded): the largest
# table first, then smaller inputs; split, wide and generic kernels
CASES = [
    (128, 130, 71, "smooth", 0, 1, 1),
    (32, 1000, 72, "smooth", 0, 2, 3),
    (16, 130, 73, "random", 0x10000, 1, 2),
    (8, 65, 74, "random", 0, 0, 4),
]


def test_static_production_equals_instance_production_twice_in_a_row():
    import torch
    from paper_1707_00919_amd import Solver
    from paper_1707_00919_amd.solver import production_static
    for L, W, seed, kind, flags, therm, rec in CASES:
        note("static production: L=%d walkers=%d seed=%d flags=%#x therm=%d sweeps=%d" %
             (L, W, seed, flags, therm, rec))
        s = Solver(L, W, seed, flags=flags)
        om = smooth_log_weights(L, seed) if kind == "smooth" else random_log_weights(L, seed, 2.0)
        s.set_log_weights(om)
        s.iterate(0, 1)                      # a weight update and a sweep counter > 0
        om = s.log_weights()
        sweep0 = s.last_info()["sweep_counter"]
        spins_v, energy_v, words, wpad = instance_views(s)
        # the documented layout is the instance's: unpacked, it gives muca_spins
        torch.cuda.synchronize()
        np.testing.assert_array_equal(unpack(spins_v, L, W, words, wpad), s.spins())
        np.testing.assert_array_equal(energy_v[:W].cpu().numpy(), s.energies())
        spins_c = spins_v.clone()            # the caller's own device buffers
        energy_c = energy_v.clone()
        torch.cuda.synchronize()
        s.production(therm, rec)
        h = production_static(L, W, seed, sweep0, therm, rec, om, spins_c, energy_c, flags=flags)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(h, s.histogram())
        assert int(h.sum()) == W * L * L * rec
        assert torch.equal(spins_c, spins_v)
        assert torch.equal(energy_c, energy_v)
        # a second call continues the chain of the first, as the instance does
        s.production(0, 1)
        h2 = production_static(L, W, seed, sweep0 + therm + rec, 0, 1, om, spins_c, energy_c, flags=flags)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(h2, s.histogram())
        assert torch.equal(spins_c, spins_v)
        assert torch.equal(energy_c, energy_v)
        s.close()


def test_static_production_zero_sweeps_and_errors():
    import torch
    from paper_1707_00919_amd import MucaError, Solver, _abi
    from paper_1707_00919_amd.solver import production_static
    note("static production: zero sweeps and argument errors")
    s = Solver(8, 64, 5)
    spins_v, energy_v, _, _ = instance_views(s)
    spins_c, energy_c = spins_v.clone(), energy_v.clone()
    om = s.log_weights()
    h = production_static(8, 64, 5, 0, 0, 0, om, spins_c, energy_c)
    torch.cuda.synchronize()
    assert h.shape == (65,) and not h.any()
    assert torch.equal(spins_c, spins_v)
    bad = om.copy()
    bad[7] = np.inf
    with pytest.raises(MucaError) as e:
        production_static(8, 64, 5, 0, 0, 1, bad, spins_c, energy_c)
    assert e.value.code == _abi.MUCA_ERR_INVALID_ARG
    s.close()
