"""Host logic of the hysteresis study (no GPU): stage lengths in ionic
times, window means of the history, Ne_0 from a run and its companion, and
the brackets of T_c and T_f."""

import math

import numpy as np
import pytest

from paper_1812_05711_amd import hysteresis as hy
from paper_1812_05711_amd.lbm_ec import HIST_COLS, HIST_CURRENT


def test_ionic_steps():
    # K = nu T / M^2 with nu = (0.8 - 0.5) / 3 = 0.1: K = 0.2 at T = 200
    assert hy.ionic_steps(50, 200.0) == pytest.approx(2500 / 0.2)
    assert hy.ionic_steps(50, 100.0) == pytest.approx(2 * hy.ionic_steps(50, 200.0))


def test_stages():
    st = hy.stages([200.0, 150.0, 100.0], 50, start_t0=8, dwell_t0=4)
    assert [T for T, _ in st] == [200.0, 150.0, 100.0]
    assert st[0][1] == round(8 * 12500)
    assert st[1][1] == round(4 * 2500 / 0.15)
    assert st[2][1] == round(4 * 25000)


def _hist(steps, current):
    h = np.zeros((len(steps) + 2, HIST_COLS))
    h[: len(steps), 0] = steps
    h[: len(steps), HIST_CURRENT] = current
    return h


def test_window_mean_and_ne0():
    steps = np.arange(10, 101, 10)
    run = _hist(steps, 3.0 * np.where(steps > 50, 1.2, 1.0))  # 3 columns
    comp = _hist(steps, np.full(len(steps), 1.0))               # 1 column
    assert hy.window_mean(run, HIST_CURRENT, 50, 100) == pytest.approx(3.6)
    assert hy.ne0(run, 3, comp, 1, 50, 100) == pytest.approx(1.2)
    assert hy.ne0(run, 3, comp, 1, 0, 50) == pytest.approx(1.0)
    assert math.isnan(hy.window_mean(run, HIST_CURRENT, 200, 300))
    # unused (zero) rows are outside every window with lo >= 0
    assert hy.window_mean(run, HIST_CURRENT, 0, 1000) == pytest.approx(3.0 * (5 * 1.0 + 5 * 1.2) / 10)


def test_brackets():
    Ts = [100.0, 140.0, 160.0, 170.0, 200.0]
    assert hy.bracket_rising(Ts, [1.0, 1.0, 1.0, 1.2, 1.4], 0.01) == (160.0, 170.0)
    assert hy.bracket_rising(Ts, [1.0] * 5, 0.01) == (200.0, None)
    assert hy.bracket_rising(Ts, [1.1] * 5, 0.01) == (None, 100.0)
    fall = [200.0, 150.0, 120.0, 110.0, 100.0]
    assert hy.bracket_falling(fall, [1.4, 1.3, 1.2, 1.0, 1.0], 0.01) == (110.0, 120.0)
    assert hy.bracket_falling(fall, [1.4] * 5, 0.01) == (None, 100.0)
    assert hy.bracket_falling(fall, [1.0] * 5, 0.01) == (200.0, None)
