"""The rate probes behind the roofline denominators (bdg_probe_peak) return
sustained rates a chip of 256 compute units at up to 2.4 GHz can reach: at most
64 32-bit vector lanes per unit per clock, and at most the published dense int8
matrix-core rate."""
import pytest

from paper_2102_04656_amd import bdg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bdg.lib()


def test_probe_rates_are_plausible():
    valu = bdg.probe_peak(bdg.PEAK_VALU_INT32) / 1e12
    mfma = bdg.probe_peak(bdg.PEAK_MFMA_INT8) / 1e12
    print(f"[probe] valu {valu:.2f} T ops/s, int8 mfma {mfma:.0f} T ops/s", flush=True)
    # one wave64 instruction per SIMD per 4 clocks is 64 lanes per unit per clock:
    # 256 x 64 x 2.4e9 = 39.3 T; allow clock and issue headroom, not an order of magnitude
    assert 10.0 < valu < 80.0
    assert 1000.0 < mfma < 5000.0 * 1.05
