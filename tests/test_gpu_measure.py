"""The measured VALU issue rate (the ALU roofline's denominator) is a plausible device figure."""
import pytest

pytestmark = pytest.mark.gpu


def test_measure_valu_rate():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    rate = sg.measure_valu_rate()
    print(f"[gpu] VALU issue rate {rate / 1e12:.2f} T lane-ops/s", flush=True)
    # between a tenth of and four times 256 CUs x 64 lanes x 2.4 GHz
    assert 3.9e12 < rate < 1.6e14
