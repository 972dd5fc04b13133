"""The packed issue-rate microbenchmark behind the bench's measured peak:
it runs, reports the lane-instructions it issued, and its rate lies between
a sane floor and the nominal ceiling of 256 CUs x 64 lanes x 2.4 GHz."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_packed_issue_rate():
    import paper_2509_01654_amd as nw
    print("[gpu case] packed issue-rate microbenchmark", flush=True)
    assert nw.packed_issue_rate(256, 16) == 256 * 256 * 16 * 64
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    n = nw.packed_issue_rate(2048, 1024)
    e1.record()
    torch.cuda.synchronize()
    rate = n / (e0.elapsed_time(e1) / 1e3)
    assert 5e12 < rate <= 256 * 64 * 2.4e9 * 1.02, rate
