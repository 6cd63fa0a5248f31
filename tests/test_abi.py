"""CPU-side checks of the C ABI: libcf.so loads, exports every function the
headers declare, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def _declared():
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(cf_[a-z_0-9]+)\s*\(", text))
    return names


def test_headers_declare_the_boundary():
    names = _declared()
    for fn in ("cf_create", "cf_insert", "cf_query", "cf_delete", "cf_destroy"):
        assert fn in names


def _comment_text(h):
    text = open(os.path.join(INCLUDE, h)).read()
    return " ".join(" ".join(re.findall(r"/\*(.*?)\*/", text, flags=re.S)).replace("*", " ").split())


def test_headers_state_the_ordering_rules():
    """The scratch a filter or a set reuses across calls makes overlapping
    writers unsafe; the headers say so (the rule chosen is stream order, one
    writer at a time), and say what breaking the fetch-AND delete's rule costs."""
    cf = _comment_text("cf.h")
    assert "An insert must not overlap another insert on the same filter" in cf
    assert "one eviction queue" in cf
    assert "silently removing an unrelated fingerprint" in cf
    st = _comment_text("cf_set.h")
    assert "One batch at a time per set" in st
    assert "Order every batch call on a set on one stream" in st


def test_library_exports_every_declared_symbol():
    import paper_2603_15486_amd._binding as B
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(B.EXPORTED) == _declared()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib.util
    src = os.path.join(ROOT, "paper_2603_15486_amd", "_binding.py")
    spec = importlib.util.spec_from_file_location("cf_binding_copy", src)
    mod = importlib.util.module_from_spec(spec)
    # a copy of the module next to no library must refuse to import
    fake = tmp_path / "_binding.py"
    fake.write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("cf_binding_copy", str(fake))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="no CPU fallback"):
        spec.loader.exec_module(mod)


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the package before torch must not map a second HIP runtime
    (torch bundles its own under the same soname as /opt/rocm's)."""
    import subprocess
    import sys
    code = ("import paper_2603_15486_amd, torch\n"
            "maps = [l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l]\n"
            "print(len(set(maps)))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"


@pytest.mark.parametrize("m,b,f,expect", [
    (3, 16, 16, 1), (0, 16, 16, 1), ((1 << 32) * 2, 16, 16, 1),
    (1 << 10, 5, 16, 4), (1 << 10, 16, 12, 4), (1 << 10, 2, 16, 4),
])
def test_create_rejects_invalid_parameters_without_device(m, b, f, expect):
    import paper_2603_15486_amd as cf
    p = cf.make_params(m, b, f)
    h = ctypes.c_void_p(123)
    st = cf.LIB.cf_create(ctypes.byref(p), ctypes.byref(h))
    assert st == expect
    assert h.value is None
    assert cf.LIB.cf_last_error()
    assert cf.LIB.cf_table_bytes(ctypes.byref(p)) == 0


@pytest.mark.parametrize("m,b,f,nbytes", [
    (1, 4, 8, 8), (2, 4, 8, 8), (4, 4, 8, 16), (1 << 18, 4, 16, 1 << 21),
    (1 << 27, 16, 16, 1 << 32), (1 << 24, 4, 8, 1 << 26), (1 << 32, 32, 32, 1 << 39),
])
def test_table_bytes(m, b, f, nbytes):
    import paper_2603_15486_amd as cf
    assert cf.LIB.cf_table_bytes(ctypes.byref(cf.make_params(m, b, f))) == nbytes


@pytest.mark.parametrize("m,b,f,pl,expect", [
    (0, 4, 8, 1, 1), (1 << 32, 4, 8, 1, 1), (1 << 10, 4, 8, 2, 1), (1 << 10, 4, 8, 99, 1),
    (3, 4, 12, 1, 4),
])
def test_create_rejects_invalid_placements_without_device(m, b, f, pl, expect):
    import paper_2603_15486_amd as cf
    p = cf.make_params(m, b, f, placement=pl)
    h = ctypes.c_void_p(123)
    assert cf.LIB.cf_create(ctypes.byref(p), ctypes.byref(h)) == expect
    assert h.value is None
    assert cf.LIB.cf_table_bytes(ctypes.byref(p)) == 0


@pytest.mark.parametrize("m,b,f,nbytes", [
    (1, 4, 8, 8), (3, 4, 8, 16), (1000, 16, 16, 32000), ((1 << 32) - 1, 4, 8, 1 << 34),
    (12289, 32, 32, 12289 * 128),
])
def test_table_bytes_offset_placement(m, b, f, nbytes):
    import paper_2603_15486_amd as cf
    p = cf.make_params(m, b, f, placement=cf.CF_PLACE_OFFSET)
    assert cf.LIB.cf_table_bytes(ctypes.byref(p)) == nbytes


@pytest.mark.parametrize("buf,nbytes", [(0, 1 << 20), (8, 1 << 20), (256, 100)])
def test_create_in_rejects_bad_buffers_without_device(buf, nbytes):
    import paper_2603_15486_amd as cf
    p = cf.make_params(1 << 10, 16, 16)  # 32 KiB table
    h = ctypes.c_void_p(123)
    st = cf.LIB.cf_create_in(ctypes.byref(p), ctypes.c_void_p(buf or None), nbytes,
                             ctypes.byref(h))
    assert st == 1 and h.value is None and cf.LIB.cf_last_error()


def test_null_handles_are_rejected():
    import paper_2603_15486_amd as cf
    L = cf.LIB
    assert L.cf_destroy(None) == 0
    assert L.cf_insert(None, None, 0, None, None, None) == 1
    assert L.cf_query(None, None, 5, None, None) == 1
    assert L.cf_delete(None, None, 5, None, None) == 1
    assert L.cf_count(None, None, None) == 1
    assert L.cf_create(None, None) == 1
    assert L.cf_keygen(None, 5, 0, 0, None) == 1


@pytest.mark.parametrize("field,value", [
    ("mode", 2), ("depth", 0), ("depth", 9), ("max_requests", 0), ("max_requests", 65537),
    ("max_batch", 0),
])
def test_server_rejects_bad_configs_without_device(field, value):
    """cf_server_create checks its configuration before it touches a device:
    unknown mode, depth outside 1..8, max_requests outside 1..65536 and an
    empty max_batch are CF_EINVAL, and no handle is returned."""
    import paper_2603_15486_amd as cf
    from paper_2603_15486_amd import _binding as B
    params = (cf.cf_params * 2)(cf.make_params(1 << 10, 16, 16), cf.make_params(1 << 12, 8, 16))
    cfg = B.cf_server_config(0, 1 << 16, 64, B.CF_SERVE_BATCHED, 2, 0)
    setattr(cfg, field, value)
    h = ctypes.c_void_p(123)
    assert cf.LIB.cf_server_create(params, 2, ctypes.byref(cfg), ctypes.byref(h)) == 1
    assert h.value is None
    assert b"config" in cf.LIB.cf_last_error()


@pytest.mark.parametrize("nf,max_batch,flags,bad_fid", [
    (0, 1024, 0, None), (65537, 1024, 0, None), (3, 0, 0, None), (3, (1 << 31) + 1, 0, None),
    (3, 1024, 2, None), (3, 1024, 0, 1),
])
def test_set_rejects_bad_arguments_without_device(nf, max_batch, flags, bad_fid):
    """cf_set_create checks its arguments before it touches a device: filter
    counts outside 1..65536, max_batch outside 1..2^31, unknown flags and an
    invalid filter (named by its index) are errors, and no handle is
    returned; cf_set_bytes is 0 for the same inputs where it applies."""
    import paper_2603_15486_amd as cf
    n = max(nf, 1)
    params = (cf.cf_params * n)(*[cf.make_params(1 << 10, 16, 16) for _ in range(n)])
    if bad_fid is not None:
        params[bad_fid] = cf.make_params(1000, 16, 16)  # XOR needs a power of two
    h = ctypes.c_void_p(123)
    st = cf.LIB.cf_set_create(params, nf, max_batch, flags, ctypes.byref(h))
    assert st == 1 and h.value is None
    err = cf.LIB.cf_last_error()
    assert err
    if bad_fid is not None:
        assert f"filter {bad_fid}".encode() in err
    if flags == 0 and bad_fid is None and nf in (0, 65537):
        assert cf.LIB.cf_set_bytes(params, nf, max_batch) == 0


@pytest.mark.parametrize("ptr,n_lines,line_bytes,width,sink_off", [
    (0, 1 << 20, 128, 16, 0), (8, 1 << 20, 128, 16, 0), (4096, 3 << 20, 128, 16, 0),
    (4096, 1 << 20, 96, 16, 0), (4096, 1 << 20, 128, 4, 0), (4096, 1 << 20, 8, 16, 0),
    (4096, 1 << 20, 128, 16, 4),
])
def test_line_probe_rejects_bad_arguments_without_device(ptr, n_lines, line_bytes, width,
                                                         sink_off):
    """cf_probe_lines refuses a NULL or misaligned buffer, a line count or
    line size that is not a power of two, a read width other than 8 or 16,
    lines narrower than the read and a sink not aligned for its atomic,
    before any launch."""
    import paper_2603_15486_amd as cf
    sink = (ctypes.c_uint64 * 2)()
    assert cf.LIB.cf_probe_lines(ptr or None, n_lines, line_bytes, width, 1000, 1,
                                 ctypes.addressof(sink) + sink_off, None) == 1


@pytest.mark.parametrize("ptr,n_lines,line_bytes,read_first,sink_off", [
    (0, 1 << 20, 128, 1, 0), (4, 1 << 20, 128, 1, 0), (4096, 3 << 20, 128, 1, 0),
    (4096, 1 << 20, 96, 1, 0), (4096, 1 << 20, 4, 1, 0), (4096, 1 << 20, 128, 2, 0),
    (4096, 1 << 20, 128, 0, 4),
])
def test_atomic_probe_rejects_bad_arguments_without_device(ptr, n_lines, line_bytes, read_first,
                                                           sink_off):
    """cf_probe_atomics refuses a NULL or misaligned buffer, a line count or
    line size that is not a power of two, lines narrower than a word, a mode
    other than 0 or 1 and a misaligned sink, before any launch."""
    import paper_2603_15486_amd as cf
    sink = (ctypes.c_uint64 * 2)()
    assert cf.LIB.cf_probe_atomics(ptr or None, n_lines, line_bytes, read_first, 1000, 1,
                                   ctypes.addressof(sink) + sink_off, None) == 1


STRUCTS = ["cf_params", "cf_set_shape", "cf_set_trial", "cf_server_config", "cf_request_info",
           "cf_server_stats", "cf_tune_goal", "cf_tune_candidate"]


def test_binding_structs_match_the_c_headers(tmp_path):
    """Every struct the binding passes by pointer has the size and field
    offsets the C compiler gives it from include/*.h (a field added on one
    side only would shift every later field)."""
    import ctypes
    import shutil
    import subprocess

    import paper_2603_15486_amd._binding as B
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    structs = {name: getattr(B, name) for name in STRUCTS}
    src = ["#include <stddef.h>", "#include <stdio.h>", '#include "cf.h"', '#include "cf_set.h"',
           '#include "cf_server.h"', '#include "cf_tune.h"', "int main(void) {"]
    for name, cls in structs.items():
        src.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            src.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    src += ["return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call([gcc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o",
                           str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, f"{name}.{field}"
