"""The accuracy-sweep tool on a small number of realisations: errors fall
with SNR, the plain correlator flattens into the -1/M floor at high SNR
(Section IV) and the least-squares rows remove it."""
import pytest

pytestmark = pytest.mark.gpu


def test_sweep_trends():
    from paper_2206_05506_amd import sweeps
    c = sweeps._curve(511, 4, 64, 64, iters=2, seed=7)
    mae = c["mae"]
    assert mae["-10"]["fp32"] > mae["10"]["fp32"] > mae["30"]["fp32"]
    # the floor: 20 -> 30 dB barely helps the correlator, the LS rows keep falling
    assert mae["30"]["fp32"] > 0.5 * mae["20"]["fp32"]
    assert mae["30"]["fp32_ls"] < 0.5 * mae["20"]["fp32_ls"]
    assert mae["30"]["fp32_ls"] < 0.7 * mae["30"]["fp32"]
    # low precision adds little to the estimation error at moderate SNR
    assert mae["10"]["bf16"] < 1.1 * mae["10"]["fp32"]
