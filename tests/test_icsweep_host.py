"""Host logic of the initial-condition sweep (no GPU needed)."""
import numpy as np

from paper_2509_16079_amd import icsweep as S


def test_region_of_attraction_rule():
    offs = np.array([-0.2, -0.1, 0.0, 0.1, 0.2])
    assert S.region_of_attraction(offs, [0.1, 0.01, 0.0, 0.02, 0.06]) == (-0.1, 0.1)
    assert S.region_of_attraction(offs, [0.0, 0.01, 0.0, 0.0, 0.0]) == (-0.2, 0.2)
    assert S.region_of_attraction(offs, [0.0, 0.0, 0.07, 0.0, 0.0]) is None
