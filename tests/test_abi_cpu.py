"""CPU-side checks of the C-ABI boundary: libmuca.so loads, exports every
function include/muca.h declares, and rejects invalid parameters before it
touches a device.  No compute call is made here (there is no GPU)."""
import ctypes
import os
import re

import pytest

from paper_1707_00919_amd import _abi

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
HEADER = os.path.join(ROOT, "include", "muca.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(muca_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libmuca.so is not built (run __graft_entry__.build())")
    return _abi.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_abi.PROTOTYPES), "binding and header disagree"


def test_state_bytes_sizes(lib):
    def sb(L, W):
        p = _abi.MucaParams(L, W, 1, 0)
        return lib.muca_state_bytes(ctypes.byref(p))

    assert sb(3, 64) == 0 and sb(2, 64) == 0 and sb(130, 64) == 0 and sb(32, 0) == 0
    # L = 32, 16384 walkers: 2 MiB lattices + 64 KiB energies + histogram + table
    b = sb(32, 16384)
    assert b >= 32 * 16384 * 4 + 16384 * 4 + 1025 * 8 + 1025 * 32
    assert b < 3 * 1024 * 1024
    assert sb(4, 1) == sb(4, 64)            # walkers pad to a wave of 64


def test_create_rejects_invalid_params_without_a_device(lib):
    h = ctypes.c_void_p()
    for L, W in [(5, 64), (2, 64), (0, 64), (130, 64), (66, 64), (70, 64), (126, 64), (32, 0)]:
        p = _abi.MucaParams(L, W, 1, 0)
        rc = lib.muca_create(ctypes.byref(p), None, None, 0, ctypes.byref(h))
        assert rc == _abi.MUCA_ERR_INVALID_ARG
        assert not h.value
        assert lib.muca_last_error(None)
    assert lib.muca_create(None, None, None, 0, ctypes.byref(h)) == _abi.MUCA_ERR_INVALID_ARG


def test_static_production_rejects_invalid_arguments_without_a_device(lib):
    # argument errors return before any device call (no GPU here)
    import numpy as np
    hist = np.zeros(17, dtype=np.uint64)
    om = np.zeros(17)
    dummy = ctypes.c_void_p(0x1000)
    hp = ctypes.c_void_p(hist.ctypes.data)
    op = ctypes.c_void_p(om.ctypes.data)
    good = _abi.MucaParams(4, 64, 1, 0)
    f = lib.muca_production_static
    assert f(None, 0, 0, 1, op, dummy, dummy, hp, None) == _abi.MUCA_ERR_INVALID_ARG
    assert f(ctypes.byref(good), 0, 0, 1, None, dummy, dummy, hp, None) == _abi.MUCA_ERR_INVALID_ARG
    assert f(ctypes.byref(good), 0, 0, 1, op, None, dummy, hp, None) == _abi.MUCA_ERR_INVALID_ARG
    assert f(ctypes.byref(good), 0, 0, 1, op, dummy, dummy, None, None) == _abi.MUCA_ERR_INVALID_ARG
    for L, W in [(5, 64), (2, 64), (130, 64), (66, 64), (4, 0)]:
        p = _abi.MucaParams(L, W, 1, 0)
        assert f(ctypes.byref(p), 0, 0, 1, op, dummy, dummy, hp, None) == _abi.MUCA_ERR_INVALID_ARG
        assert lib.muca_last_error(None)
    om[3] = float("nan")
    assert f(ctypes.byref(good), 0, 0, 1, op, dummy, dummy, hp, None) == _abi.MUCA_ERR_INVALID_ARG
    assert b"finite" in lib.muca_last_error(None)
    om[3] = 0.0
    # the attempt position would pass 2^64
    assert f(ctypes.byref(good), (1 << 64) // 16, 0, 1, op, dummy, dummy, hp, None) == _abi.MUCA_ERR_OVERFLOW
    # the scratch holds the tables of the largest lattice
    assert _abi.MUCA_STATIC_SCRATCH_BYTES >= 40 * (128 * 128 + 1)


def test_null_handle_calls_are_rejected(lib):
    assert lib.muca_iterate(None, 0, 1, None) == _abi.MUCA_ERR_INVALID_ARG
    assert lib.muca_histogram(None, None, 0) == _abi.MUCA_ERR_INVALID_ARG
    assert lib.muca_destroy(None) == _abi.MUCA_OK


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the ABI structs, as a C compiler lays them
    out from include/muca.h, equal those of the ctypes mirrors."""
    import ctypes
    import subprocess
    from paper_1707_00919_amd import _abi
    structs = {"muca_params": _abi.MucaParams, "muca_info": _abi.MucaInfo,
               "muca_server_config": _abi.ServerConfig, "muca_request": _abi.Request,
               "muca_result": _abi.Result, "muca_server_counters": _abi.ServerCounters,
               "muca_schedule": _abi.Schedule, "muca_schedule_step": _abi.ScheduleStep}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "muca.h"', 'int main(void){']
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append('return 0;}')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    want = []
    for cname, py in structs.items():
        want.append("%s size %d" % (cname, ctypes.sizeof(py)))
        for f, _ in py._fields_:
            want.append("%s %s %d" % (cname, f, getattr(py, f).offset))
    assert [g for g in got if g] == want


def test_library_and_torch_share_one_hip_runtime():
    """Loading the binding before torch must not leave two HIP runtimes in the
    process (the second one to open the device would find none)."""
    import subprocess
    import sys
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libmuca.so is not built (run __graft_entry__.build())")
    code = ("from paper_1707_00919_amd import _abi\n"
            "_abi.lib()\n"
            "import torch\n"
            "maps = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(maps))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_solver_without_a_gpu_fails_loudly():
    """No CPU fallback: without a visible GPU the product path raises."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible here")
    from paper_1707_00919_amd import MucaError, Solver
    for use_torch in (True, False):
        with pytest.raises(MucaError) as e:
            Solver(4, 64, 1, use_torch=use_torch)
        assert e.value.code == _abi.MUCA_ERR_DEVICE
