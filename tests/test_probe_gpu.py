"""The achievable-peak microbenchmarks (selfjoin_probe_peaks) through the C
ABI: every figure is positive and within the range the chip's published
peaks allow (no figure above its published peak, none below a fifth of it)."""
import pytest

pytestmark = pytest.mark.gpu

# published dense peaks of the MI355X: TFLOP/s, GB/s
PUBLISHED = {"fp64_mfma_tflops": 78.6, "fp32_mfma_tflops": 157.3, "bf16_mfma_tflops": 2500.0,
             "fp8_mfma_tflops": 5000.0, "fp64_valu_tflops": 78.6, "hbm_read_gbs": 8000.0,
             "hbm_copy_gbs": 8000.0}


@pytest.fixture(scope="module")
def peaks():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_11287_amd as p
    print("probe: selfjoin_probe_peaks(1 GiB buffers)", flush=True)
    return p.selfjoin_probe_peaks(1 << 30)


@pytest.mark.parametrize("key", sorted(PUBLISHED))
def test_probe_within_published_peak(peaks, key):
    v = peaks[key]
    assert 0.2 * PUBLISHED[key] <= v <= 1.05 * PUBLISHED[key], (key, v)


def test_probe_without_bandwidth_buffers():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_11287_amd as p
    r = p.selfjoin_probe_peaks(0)
    assert r["hbm_read_gbs"] == 0.0 and r["hbm_copy_gbs"] == 0.0
    assert r["fp64_mfma_tflops"] > 0.0
