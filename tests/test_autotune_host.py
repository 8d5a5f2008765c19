"""Host logic of the autotuner's frame-error constraint (two-proportion test)."""
from paper_1206_3362_amd import autotune


def test_fer_constraint():
    # lower or equal error rate is always admissible
    assert autotune.fer_admissible(10, 1000, 50, 1000)
    assert autotune.fer_admissible(50, 1000, 50, 1000)
    # p1 = 0.06, p2 = 0.05, pooled 0.055: 3 sigma = 3*sqrt(.055*.945*2/1000) = 0.0306
    assert autotune.fer_admissible(60, 1000, 50, 1000)
    assert not autotune.fer_admissible(90, 1000, 50, 1000)
    # zero errors on both sides
    assert autotune.fer_admissible(0, 100, 0, 100)
    assert not autotune.fer_admissible(10, 100, 0, 100)
