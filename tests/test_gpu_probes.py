"""The memory-system probes behind the benchmark's ceilings (cf_probe_lines,
cf_probe_atomics): they must touch only what their declarations say, the
first word of each line, so the rates they give are those of the access
pattern they describe."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cf():
    import paper_2603_15486_amd as mod
    return mod


@pytest.mark.parametrize("read_first", [True, False])
@pytest.mark.parametrize("line_bytes", [128, 32])
def test_atomic_probe_changes_only_line_starts(cf, read_first, line_bytes):
    """2^16 CAS over 4096 lines of a zeroed buffer: every line's first word
    is hit (the chance of a miss is about e^-16 per line), and no other word
    changes."""
    words = line_bytes // 8
    n_lines = 4096
    buf = torch.zeros(n_lines * words, dtype=torch.int64, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    cf.cf_probe_atomics(buf, line_bytes, read_first, 1 << 16, 5, sink)
    torch.cuda.synchronize()
    w = buf.view(n_lines, words).cpu()
    assert int((w[:, 0] != 0).sum()) >= int(0.99 * n_lines)
    if words > 1:
        assert not bool(w[:, 1:].any())
    assert int(sink.item()) == 0


def test_line_probe_writes_nothing(cf):
    """The read probe leaves its buffer as it was and its sink at 0."""
    buf = torch.arange(1 << 16, dtype=torch.int64, device="cuda")
    ref = buf.clone()
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    for line, width in ((128, 16), (128, 8), (32, 16)):
        cf.cf_probe_lines(buf, line, width, 1 << 16, 9, sink)
    torch.cuda.synchronize()
    assert torch.equal(buf, ref)
    assert int(sink.item()) == 0
