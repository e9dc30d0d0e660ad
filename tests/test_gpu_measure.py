"""The measured VALU issue rates (the ALU roofline's denominator and two other instruction kinds)
are plausible device figures."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_measure_valu_rate(kind):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    rate = sg.measure_valu_rate(kind)
    print(f"[gpu] VALU issue rate, kind {kind}: {rate / 1e12:.2f} T lane-ops/s", flush=True)
    # between a tenth of and four times 256 CUs x 64 lanes x 2.4 GHz
    assert 3.9e12 < rate < 1.6e14


def test_measure_valu_rate_rejects_unknown_kind():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_10737_amd as sg
    with pytest.raises(sg.SograndError):
        sg.measure_valu_rate(7)
