"""Host-side parts of bench.py that need no GPU: the single-GPU contract
(more than one GPU exits with a message) and the BER interpolation used to
place the Eb/N0 at a target BER."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_ebn0_at_target_ber():
    ebs = [3.0, 3.5, 4.0, 4.5]
    # BER decades 1e-2, 1e-3, 1e-4, 1e-5: 1e-4 is crossed exactly at 4.0 dB
    assert bench._ebn0_at(ebs, [1e-2, 1e-3, 1e-4, 1e-5], 1e-4) == pytest.approx(4.0)
    # halfway in log BER between 1e-3 (3.5 dB) and 1e-5 (4.0 dB)
    assert bench._ebn0_at([3.5, 4.0], [1e-3, 1e-5], 1e-4) == pytest.approx(3.75)
    # never crossed: None; zero counts are clamped, not log(0)
    assert bench._ebn0_at([3.0, 3.5], [1e-2, 1e-3], 1e-4) is None
    assert bench._ebn0_at([3.0, 3.5], [1e-3, 0.0], 1e-4) == pytest.approx(3.0 + 0.5 / 9, abs=1e-3)
