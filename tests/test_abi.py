"""The C-ABI library loads and exports every function the public headers
declare; argument validation that happens before any device call works on
the CPU.  No compute calls (there is no GPU here)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(tina_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2408_16551_amd import pfb
    if not os.path.exists(pfb.LIB_PATH):
        pytest.fail("libtina_pfb.so not built (run __graft_entry__.build())")
    return pfb.load()


def test_headers_declare_the_boundary():
    names = _declared()
    for required in ("tina_pfb_plan", "tina_pfb_execute", "tina_pfb_state_create", "tina_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_lists_every_declared_symbol():
    from paper_2408_16551_amd import pfb
    assert set(_declared()) <= set(pfb.EXPORTS)


def _desc(pfb, **kw):
    d = pfb._Desc()
    d.struct_size = ctypes.sizeof(pfb._Desc)
    d.channels, d.taps, d.sample_type, d.window, d.precision, d.output, d.device = 1024, 16, 0, 1, 0, 0, 0
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,status", [
    ({"channels": 1000}, 2), ({"channels": 8}, 2), ({"channels": 16384}, 2), ({"taps": 65}, 2),
    ({"taps": 0}, 1), ({"channels": -4}, 1), ({"sample_type": 7}, 1), ({"window": 9}, 1),
    ({"precision": 9}, 1), ({"output": 5}, 1), ({"window": 4}, 1), ({"struct_size": 4}, 1),
])
def test_plan_rejects_bad_descriptors_before_device(lib, kw, status):
    from paper_2408_16551_amd import pfb
    d = _desc(pfb, **kw)
    h = ctypes.c_void_p()
    assert lib.tina_pfb_plan(ctypes.byref(d), ctypes.byref(h)) == status
    assert not h.value
    assert lib.tina_last_error().decode()


def test_null_arguments_rejected(lib):
    h = ctypes.c_void_p()
    assert lib.tina_pfb_plan(None, ctypes.byref(h)) == 1
    fw = ctypes.c_int64()
    assert lib.tina_pfb_execute(None, None, 0, None, 0, None, ctypes.byref(fw), None) == 1
    assert lib.tina_pfb_state_create(None, ctypes.byref(h)) == 1
    assert lib.tina_pfb_channels_out(None, None) == 1
    assert lib.tina_pfb_plan_destroy(None) == 0
    assert lib.tina_pfb_state_destroy(None) == 0


def test_version_string(lib):
    assert b"gfx950" in lib.tina_version()


@pytest.mark.parametrize("units,cost", [
    ([4, 8, 0, 0, 1, 4, 32, 6], [512.0] * 8),
    ([0, 0, 0], [1.0, 2.0, 3.0]),
    ([], []),
    ([1], [5.0]),
    ([100, 3, 7000, 1], [4096.0, 512.0, 1024.0, 8192.0]),
    ([5, 5, 5, 5, 5, 5, 5, 5, 5, 5], [1.0, 9.0] * 5),
])
def test_batch_split_covers_every_unit_once(lib, units, cost):
    import numpy as np
    from paper_2408_16551_amd import pfb
    b = pfb.split_units(units, cost)
    assert b[0] == 0 and b[8] == sum(units)
    assert np.all(np.diff(b) >= 0)
    # balance: no range exceeds an eighth of the cost by more than the largest unit
    if sum(units):
        per = np.repeat(np.asarray(cost, float), units)
        csum = np.concatenate([[0.0], np.cumsum(per)])
        shares = csum[b[1:]] - csum[b[:-1]]
        assert shares.max() <= csum[-1] / 8 + max(cost) + 1e-9


def test_arena_first_fit_and_coalescing(lib):
    from paper_2408_16551_amd import pfb
    # allocate 3 x 1000 (256-byte granules), free the middle, refit, overflow, free all
    ops = [1000, 1000, 1000, -1, 500, 200, 5000, -0, -2, -4, -5, 4096]
    out, used = pfb.arena_simulate(4096, ops)
    assert list(out[:3]) == [0, 1024, 2048]
    assert out[3] == 1                       # released
    assert out[4] == 1024                    # first fit reuses the hole
    assert out[5] == 1536                    # 200 -> 256 bytes, first fit in the rest of the hole
    assert out[6] == -1                      # does not fit
    assert list(out[7:11]) == [1, 1, 1, 1]
    assert out[11] == 0 and used == 4096     # everything coalesced back into one block


def test_server_config_validated_before_device(lib):
    from paper_2408_16551_amd import pfb
    c = pfb._ServerConfig()
    c.struct_size = ctypes.sizeof(pfb._ServerConfig)
    c.device, c.precision, c.max_streams, c.max_active, c.max_queued = 0, 0, 4, 2, 8
    c.hbm_budget_bytes, c.frames_per_step, c.use_graph, c.max_channels = 1 << 20, 64, 1, 1000
    h = ctypes.c_void_p()
    assert lib.tina_server_create(ctypes.byref(c), ctypes.byref(h)) == 1   # max_channels not a power of two
    c.max_channels, c.frames_per_step = 1024, 0
    assert lib.tina_server_create(ctypes.byref(c), ctypes.byref(h)) == 1
    c.frames_per_step, c.precision = 64, 17
    assert lib.tina_server_create(ctypes.byref(c), ctypes.byref(h)) == 1
    c.precision, c.dft_algorithm = 2, 1           # factored DFT on a BF16x3 server
    assert lib.tina_server_create(ctypes.byref(c), ctypes.byref(h)) == 1
    c.precision, c.dft_algorithm = 0, 3           # compensated: not a server algorithm
    assert lib.tina_server_create(ctypes.byref(c), ctypes.byref(h)) == 1
    c.dft_algorithm, c.reserved_ = 1, 5
    assert lib.tina_server_create(ctypes.byref(c), ctypes.byref(h)) == 1
    c.reserved_ = 0
    c.struct_size = 16                            # ends before the fields it needs
    assert lib.tina_server_create(ctypes.byref(c), ctypes.byref(h)) == 1
    assert not h.value
    r = pfb._Request()
    rid = ctypes.c_uint64()
    assert lib.tina_pfb_submit(None, ctypes.byref(r), ctypes.byref(rid)) == 1


def test_bench_refuses_more_than_one_gpu():
    # The build runs on one GPU; --gpus N > 1 must exit with a message, before
    # touching any device.
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0
    assert "--gpus must be 1" in (r.stdout + r.stderr)


def test_binding_validates_buffers_before_the_abi():
    # The C ABI takes raw pointers: the binding must refuse a buffer of the
    # wrong type, shape, layout or device before any call is made.
    import numpy as np
    import torch
    from paper_2408_16551_amd.pfb import check_device_tensor, check_host_array
    f32 = torch.zeros(8, 9, dtype=torch.float32)
    c64 = torch.zeros(8, 9, dtype=torch.complex64)
    with pytest.raises(ValueError, match="complex64"):
        check_device_tensor(f32, "out", torch.complex64, 2, 0, cols=9)      # float32 out: half the bytes
    with pytest.raises(ValueError, match="dimension"):
        check_device_tensor(c64.reshape(-1), "out", torch.complex64, 2, 0, cols=9)
    with pytest.raises(ValueError, match="columns"):
        check_device_tensor(c64, "out", torch.complex64, 2, 0, cols=10)
    with pytest.raises(ValueError, match="contiguous"):
        check_device_tensor(c64.t(), "out", torch.complex64, 2, 0, cols=8)
    with pytest.raises(ValueError, match="cuda:0"):
        check_device_tensor(c64, "out", torch.complex64, 2, 0, cols=9)      # a CPU tensor
    with pytest.raises(ValueError, match="torch tensor"):
        check_device_tensor(np.zeros((8, 9), np.complex64), "out", torch.complex64, 2, 0)
    check_host_array(np.zeros((8, 9), np.complex64), "out", np.complex64, 2, cols=9)
    with pytest.raises(ValueError, match="complex64"):
        check_host_array(np.zeros((8, 9), np.float32), "out", np.complex64, 2, cols=9)
    with pytest.raises(ValueError, match="float32"):
        check_host_array(np.zeros(16, np.complex64), "input", np.float32, 1)   # complex input on a real stream
    with pytest.raises(ValueError, match="C-contiguous"):
        check_host_array(np.zeros((9, 8), np.complex64).T, "out", np.complex64, 2, cols=9)
    with pytest.raises(ValueError, match="columns"):
        check_host_array(np.zeros((8, 5), np.complex64), "out", np.complex64, 2, cols=9)
