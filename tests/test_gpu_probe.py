"""The instruction-peak probes used by the roofline report run through the C
ABI and return plausible rates: positive, and not above the datasheet peaks
of the instruction classes (bf16 MFMA 2.5 PFLOP/s, FP64 MFMA and vector FMA
78.6 TFLOP/s each)."""
import math

import pytest

from gpu_common import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("kind,peak", [("bf16_mfma", 2500.0), ("fp64_mfma", 78.6),
                                       ("fp64_fma", 78.6)])
def test_peak_probe(kind, peak):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1711_11418_amd.binding import peak_probe
    log(f"[probe] {kind}")
    v = peak_probe(kind)
    log(f"  {v:.1f} TFLOP/s")
    assert math.isfinite(v) and 0.05 * peak < v <= 1.05 * peak
