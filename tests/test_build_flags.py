"""The library's build configuration (no device needed).

The insert kernels are correct under contention only as built at -O1 (built
at -O2 or -O3 they lost fingerprints in one-launch fills of a 2^20-slot
table; the GPU contention tests catch that, but only on a GPU).  These checks
keep the configuration from drifting on the CPU: every translation unit that
holds insert kernels is compiled at -O1, everything else at -O3, no unit
escapes the packed-fp32 ban, and every source in the tree is built.
"""
import os

import pytest

from paper_2603_15486_amd import build as B


def _opt(flags):
    levels = [f for f in flags if f.startswith("-O")]
    assert len(levels) == 1, levels
    return levels[0]


def test_insert_units_are_built_at_O1_and_the_rest_at_O3():
    for src in B.SOURCES:
        want = "-O1" if "insi_" in src else "-O3"
        assert _opt(B.compile_flags(src)) == want, src


def test_insert_kernels_live_only_in_O1_units():
    """An insert kernel instantiated in an -O3 unit would escape the rule
    above: the host stubs in the built objects name every kernel a unit
    holds (checked where the objects exist)."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    objs = [B.object_of(s) for s in B.SOURCES]
    if nm is None or not all(os.path.exists(o) for o in objs):
        pytest.skip("library objects not built")
    kinds = ("insert_kernel", "persist_kernel")
    for src, obj in zip(B.SOURCES, objs):
        syms = subprocess.run([nm, "-C", "--defined-only", obj], capture_output=True,
                              text=True, check=True).stdout
        has = any(k in line for line in syms.splitlines() for k in kinds)
        assert has == ("insi_" in src), src


def test_no_unit_escapes_the_packed_fp32_ban():
    for src in B.SOURCES:
        flags = B.compile_flags(src)
        i = flags.index("-target-feature")
        assert flags[i - 1] == "-Xclang" and flags[i + 1] == "-Xclang"
        assert flags[i + 2] == "-packed-fp32-ops", src


def test_every_hip_source_is_built():
    on_disk = sorted(f for f in os.listdir(B.CSRC) if f.endswith(".hip"))
    assert sorted(B.SOURCES) == on_disk
