"""Device micro-benchmarks (csp_microbench): each kind runs, reports a
positive rate, and rejects sizes out of range; the barrier kinds check their
combined minimum on the device."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1511_06441_amd import csp
    s = csp.Solver(0)
    yield csp, s, torch.cuda.current_stream()
    s.close()


def test_copy_and_atomics(lib):
    csp, s, st = lib
    gbps, _ = csp.csp_microbench(s.ctx, csp.MB_COPY, 8 << 20, 2, stream=st)
    assert gbps > 0
    gps, _ = csp.csp_microbench(s.ctx, csp.MB_ATOMIC, 1 << 20, 1 << 16, stream=st)
    assert gps > 0


@pytest.mark.parametrize("lg", [0, 10, 14, 18])
def test_record_loads_slab_sizes(lib, lg):
    csp, s, st = lib
    g, us = csp.csp_microbench(s.ctx, csp.MB_LOADS, 1024, 2, lg, stream=st)
    assert g > 0 and us > 0


@pytest.mark.parametrize("lg", [9, 19])
def test_record_loads_rejects_slab(lib, lg):
    csp, s, st = lib
    with pytest.raises(csp.CspError):
        csp.csp_microbench(s.ctx, csp.MB_LOADS, 1024, 2, lg, stream=st)


def test_barriers(lib):
    csp, s, st = lib
    a, b = csp.csp_microbench(s.ctx, csp.MB_BARRIER, 20, 8, 4, stream=st)
    assert a > 0 and b > 0
