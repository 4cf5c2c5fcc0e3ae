"""Peak microbenchmarks on the device: every MFMA kind the kernels use and
the streaming copy run, and each measured rate is a sizeable fraction of the
published MI355X figure without exceeding it (5% margin for timing)."""
import pytest

pytestmark = pytest.mark.gpu

PUBLISHED = {"bf16": 2.5e15, "f64": 78.6e12, "i8": 5.0e15, "f32": 157.3e12}
HBM = 8.0e12


@pytest.fixture(scope="module")
def U():
    from paper_2508_12627_amd import ustat
    ustat.load_library()
    return ustat


@pytest.mark.parametrize("kind", list(PUBLISHED))
def test_peak_mfma(U, kind):
    rate = U.ustat_peak_mfma(kind, 4000)
    print(f"peak {kind}: {rate / 1e12:.1f} T/s", flush=True)
    assert 0.2 * PUBLISHED[kind] < rate < 1.05 * PUBLISHED[kind]


def test_peak_copy(U):
    rate = U.ustat_peak_copy(256 << 20)
    print(f"peak copy: {rate / 1e9:.0f} GB/s", flush=True)
    assert 0.2 * HBM < rate < 1.05 * HBM
