"""The delay model of Section IV reproduces the paper's worked numbers for
EG(255,175): 16 units take 16 clocks, FWBF's choice takes 20 clocks and
MLP-WBF's 24 lambda (eqs. (2) and (3))."""
import pytest

from paper_1206_3362_amd import delay


def test_eg255_worked_example():
    assert delay.metric_clocks(255, 16) == 16      # 255 metrics + 1 null metric, 16 units
    assert delay.fwbf_delay(255, 16) == 20         # log2 16 + 16
    for lam in (1, 5, 10):
        assert delay.mlp_wbf_delay(255, 16, lam) == 24 * lam
    # with the typical lambda of about 10, FWBF's choice is 12x shorter
    assert delay.mlp_wbf_delay(255, 16, 10) / delay.fwbf_delay(255, 16) == 12


def test_model_structure():
    # Fig. 1: 2q = 8 values leave the 3-stage network after 3 clocks
    assert delay.fwbf_delay(8, 8) == 3 + 1
    # padding with null metrics (footnote 1)
    assert delay.metric_clocks(1023, 32) == 32
    assert delay.fwbf_delay(1023, 32) == 5 + 32
    assert delay.decode_clocks(6.06, 1023, 32) == pytest.approx(6.06 * 37)
    with pytest.raises(ValueError):
        delay.fwbf_delay(255, 12)
