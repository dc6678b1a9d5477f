"""Host-side logic of the training driver: the early-stopping criterion on
the moving average of the energy variance (App. B) and the stage lists of
the Static and Adaptive schedules.  CPU only."""
import math

import pytest

from paper_2507_18700_amd.train import EarlyStop, EarlyStopState, adaptive_stages, interval_stages, static_stages


def test_delta_of_the_hidden_width():
    # delta = 10^(-log2(d_h)/2): 10^-0.5 at d_h = 2, 10^-4 at d_h = 256
    assert abs(EarlyStop.delta(2) - 10 ** -0.5) < 1e-15
    assert abs(EarlyStop.delta(256) - 1e-4) < 1e-18


def test_flat_variance_fires_after_window_plus_patience():
    st = EarlyStopState(EarlyStop(window=5, patience=3), 256)
    # first full window at index 4 sets the best; 3 steps without improvement fire at index 7
    assert st.update([1.0] * 7) is None
    assert st.update([1.0]) == 7


def test_improvements_reset_the_patience():
    rule = EarlyStop(window=2, patience=3)
    st = EarlyStopState(rule, 2)  # delta = 0.316
    seq = [10.0, 10.0, 9.0, 9.0, 9.0, 5.0, 5.0, 5.0, 5.0, 5.0]
    # averages from index 1: 10, 9.5, 9, 9, 7, 5, 5, 5, 5 -> improvements at 1, 2 (9.5 < 10 - 0.316),
    # 5 (7 < 9.5 - 0.316), 6 (5); then no improvement at 7, 8, 9 -> fires at 9
    assert st.update(seq) == 9
    assert st.best == 5.0


def test_small_changes_are_not_improvements():
    st = EarlyStopState(EarlyStop(window=1, patience=4), 256)  # delta 1e-4
    seq = [1.0 - 2e-5 * k for k in range(10)]  # 8e-5 below the best after 4 steps: no improvement yet
    assert st.update(seq) == 4


def test_stage_lists():
    assert [s.d_h for s in adaptive_stages(2, 256, 6250)] == [2, 4, 8, 16, 32, 64, 128, 256]
    assert all(s.steps == 6250 for s in adaptive_stages(2, 256, 6250))
    st = static_stages(256, 50000)
    assert len(st) == 1 and st[0].d_h == 256 and st[0].steps == 50000
    assert math.isclose(sum(s.steps for s in adaptive_stages(32, 256, 50000)), 200000)


def test_interval_stages():
    """Doubling every 200 steps over 2000 (the long-range TFIM run): eight
    widths 2..256, the last one taking the remaining 600 steps."""
    st = interval_stages(2, 256, 2000, 200)
    assert [x.d_h for x in st] == [2, 4, 8, 16, 32, 64, 128, 256]
    assert [x.steps for x in st] == [200] * 7 + [600]
    assert sum(x.steps for x in st) == 2000
    with pytest.raises(ValueError):
        interval_stages(2, 256, 1400, 200)

