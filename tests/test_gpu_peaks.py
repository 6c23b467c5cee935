"""tm_measure_peaks: the library's own stream-read and MFMA-loop rates come
back positive and below the published peaks (8 TB/s HBM, 2.5 PFLOP/s dense
bf16, 157.3 TFLOP/s fp32), and a size out of range is refused."""
import pytest

from gpu_helpers import tilemag

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_plausible():
    tmg = tilemag()
    rd, bf, f32 = tmg.tm_measure_peaks(0, 256 << 20)
    print("read %.0f GB/s, bf16 %.0f TFLOP/s, fp32 %.1f TFLOP/s" % (rd, bf, f32), flush=True)
    assert 500 < rd < 8000 * 1.6  # a 256 MB buffer may be served partly from the Infinity Cache
    assert 100 < bf < 2500 * 1.05
    assert 10 < f32 < 157.3 * 1.05
    with pytest.raises(tmg.TilemagError) as ei:
        tmg.tm_measure_peaks(0, 1024)
    assert ei.value.status == tmg.TM_EINVAL
