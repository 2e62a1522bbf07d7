"""The device probe of the C ABI (ptamd_measure_device): the achievable
copy bandwidth and FMA rates that the benchmark reports next to the
datasheet peaks.  On an MI355X they must come out positive and below the
datasheet figures (HBM 8 TB/s; FP32 FMA without packed instructions half
of 157.3 TFLOP/s; FP64 78.6 TFLOP/s); argument errors are rejected."""
import pytest

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_07321_amd")


def test_device_probe_is_within_the_datasheet():
    d = P.measure_device(1 << 28, 3)
    print(f"\n{d}")
    assert 500.0 < d["copy_GBs"] <= 8000.0
    assert 5.0 < d["fma32_TFLOPs"] <= 157.3 / 2 * 1.05
    assert 2.0 < d["fma64_TFLOPs"] <= 78.6 * 1.05


@pytest.mark.parametrize("nbytes,reps", [(1000, 3), ((1 << 20) + 8, 3), (1 << 20, 0)])
def test_device_probe_rejects_bad_arguments(nbytes, reps):
    with pytest.raises(P.PtamdError) as ei:
        P.measure_device(nbytes, reps)
    assert ei.value.name == "PTAMD_EINVAL"
