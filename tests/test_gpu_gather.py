"""lap_bench_gather, the random-access microbenchmark the roofline figures are
measured against: every mode returns a positive rate on a small working set,
and arguments outside its documented ranges are refused before anything runs."""
import pytest

from tests.gpu_common import log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,in_flight,flavor", [(0, 1, 0), (0, 16, 1), (1, 1, 2), (1, 1, 3), (2, 4, 0),
                                                   (3, 8, 0), (4, 1, 0), (4, 16, 0)])
def test_gather_modes_report_a_rate(mode, in_flight, flavor):
    from paper_2311_10290_amd import bench_gather
    rate = bench_gather(4 << 20, 1 << 14, mode, in_flight, flavor)
    log(f"gather mode {mode} x{in_flight} flavor {flavor}: {rate / 1e9:.1f} G ops/s")
    assert 1e8 < rate < 1e13


def test_gather_refuses_bad_arguments():
    from paper_2311_10290_amd import LapError, bench_gather
    bad = [dict(bytes_=1 << 19, lanes=1 << 14, mode=0), dict(bytes_=4 << 20, lanes=255, mode=0),
           dict(bytes_=4 << 20, lanes=(1 << 24) + 1, mode=0), dict(bytes_=4 << 20, lanes=1 << 14, mode=5),
           dict(bytes_=4 << 20, lanes=1 << 14, mode=4, flavor=1),
           dict(bytes_=4 << 20, lanes=1 << 14, mode=0, in_flight=3),
           dict(bytes_=4 << 20, lanes=1 << 14, mode=2, flavor=1),
           dict(bytes_=4 << 20, lanes=1 << 14, mode=0, flavor=4)]
    for kw in bad:
        with pytest.raises(LapError) as ei:
            bench_gather(**kw)
        assert ei.value.code == -1, kw
