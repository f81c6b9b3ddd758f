"""Machine probes (rtcc_peak_probe) on the GPU: the sustained MFMA rates and the HBM copy bandwidth are
positive, below the published MI355X figures (FP64 78.6, FP32 157.3, BF16 2516.6 TFLOP/s dense; HBM
8 TB/s) and above a floor that a working probe clears by far (a quarter of each), and a doubled loop
length gives the same rate (the probe measures a rate, not launch overhead). A copy size that is not a
multiple of 16 KiB is refused.
"""
import pytest

pytestmark = pytest.mark.gpu

PUBLISHED = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.6, "copy": 8000.0}
ROUNDS = {"fp64": 1500, "fp32": 1500, "bf16": 3000}


@pytest.fixture(autouse=True)
def _need_gpu(require_gpu):
    yield


@pytest.mark.parametrize("kind", ["fp64", "fp32", "bf16"])
def test_mfma_rate_is_plausible(kind):
    from paper_2205_05175_amd import peak_probe
    print(f"peak probe {kind}", flush=True)
    r1 = peak_probe(kind, ROUNDS[kind])
    r2 = peak_probe(kind, 2 * ROUNDS[kind])
    print(f"  {r1:.1f} / {r2:.1f} TFLOP/s (published {PUBLISHED[kind]})", flush=True)
    for r in (r1, r2):
        assert 0.25 * PUBLISHED[kind] < r <= 1.02 * PUBLISHED[kind]
    assert abs(r2 - r1) < 0.1 * r2


def test_copy_bandwidth_is_plausible():
    from paper_2205_05175_amd import RTCCError, peak_probe
    print("peak probe copy 1 GiB", flush=True)
    g = peak_probe("copy", 1 << 30)
    print(f"  {g:.0f} GB/s", flush=True)
    assert 0.25 * PUBLISHED["copy"] < g <= 1.02 * PUBLISHED["copy"]
    with pytest.raises(RTCCError):
        peak_probe("copy", (1 << 20) + 16)
