"""Host-side pieces of the predictor's fine-tuning for one geometry
(calibrate.py): the split of the instances, the median and the standard
deviation the host forms from values the library returns."""
import math

import pytest

from paper_1703_01216_amd import calibrate


def test_split_holds_out_the_tail():
    fit, held = calibrate.split(96, 0.25)
    assert fit == list(range(72)) and held == list(range(72, 96))
    fit, held = calibrate.split(3, 0.01)
    assert fit == [0, 1] and held == [2]
    fit, held = calibrate.split(2, 0.99)
    assert fit == [0] and held == [1]


def test_median_and_std():
    assert calibrate.median([3.0, 1.0, 2.0]) == 2.0
    assert calibrate.median([4.0, 1.0, 3.0, 2.0]) == 2.5
    with pytest.raises(ValueError):
        calibrate.median([])
    assert calibrate.std([1.0, 1.0]) == 0.0
    assert calibrate.std([0.0, 2.0]) == pytest.approx(1.0)
    assert calibrate.std([1.0, 2.0, 3.0, 4.0]) == pytest.approx(math.sqrt(1.25))
