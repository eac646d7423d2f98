"""GPU checks of the peak microbenchmarks (adc2_peak_probe): every probe
runs through the C ABI and returns a rate that is positive and within a
plausible band of the published MI355X figure (0.3x .. 1.15x; the probes
measure what the device delivers at its current clock, so they may fall
short of the datasheet but cannot exceed it by much)."""
import pytest

import paper_2604_27451_amd as A

pytestmark = pytest.mark.gpu

DATASHEET = {A.ADC2_PEAK_MFMA_F64: 78.6, A.ADC2_PEAK_MFMA_F32: 157.3, A.ADC2_PEAK_MFMA_BF16: 2500.0,
             A.ADC2_PEAK_VALU_F64: 78.6, A.ADC2_PEAK_HBM_READ: 8000.0, A.ADC2_PEAK_HBM_COPY: 8000.0,
             A.ADC2_PEAK_MFMA_F64_RAND: 78.6, A.ADC2_PEAK_MFMA_BF16_RAND: 2500.0}


@pytest.mark.parametrize("kind", sorted(DATASHEET))
def test_peak_probe_in_band(kind):
    print(f"[case] peak probe kind {kind}", flush=True)
    r = A.adc2_peak_probe(kind, 0, 2)
    ds = DATASHEET[kind]
    print(f"  measured {r:.1f} (datasheet {ds:g})", flush=True)
    assert 0.3 * ds < r < 1.15 * ds


def test_peak_probe_rejects_bad_arguments():
    with pytest.raises(A.Adc2Error):
        A.adc2_peak_probe(42)
    with pytest.raises(A.Adc2Error):
        A.adc2_peak_probe(A.ADC2_PEAK_HBM_COPY, 1 << 20)
