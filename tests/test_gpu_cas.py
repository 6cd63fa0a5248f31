"""Cross-XCD device-scope CAS stress: 4096 blocks of 256 threads (every
compute unit, so every XCD) increment random counters with CAS loops whose
expected values come from plain 8-byte loads or 16-byte vector loads (as the
filter's bucket loads), and with the hardware atomic add.  The total must be
exact: the filter's insert, delete and eviction kernels rely on it."""
import ctypes
import os

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "libcas_stress.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} missing: run __graft_entry__.build()")
    torch.cuda.init()
    L = ctypes.CDLL(LIB)
    L.cas_stress.restype = ctypes.c_int
    L.cas_stress.argtypes = [ctypes.c_uint32, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
    return L


@pytest.mark.parametrize("ncnt", [4096, 1 << 16, 1 << 20])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_cas_increments_are_exact(lib, ncnt, mode):
    blocks, iters = 4096, 16
    s, g = ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.cas_stress(ncnt, blocks, iters, mode, ctypes.byref(s), ctypes.byref(g)) == 0
    assert g.value == 0
    assert s.value == blocks * 256 * iters
