"""The banded driver of tests/golden/make_oracle_golden.py (--threads) against
Oracle.step: the same populations bit for bit.

The driver hands the collision of each step to Oracle.collide in bands of
rows on a thread pool, and runs the oracle's moments, row transforms and
per-wavenumber Thomas solve on bands of rows (or wavenumber columns); each
of these computes every element from that element's own row or column
alone, so every band sees the same operands and performs the same
operations as the single call on the whole grid.  These cases make any slip in the band bookkeeping
(a row missed or written twice, a band given another band's moments, the
wrong reference rows in the streaming) show as a bit difference.
"""

import importlib.util
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import Oracle, Params

HERE = os.path.dirname(os.path.abspath(__file__))


def _driver():
    spec = importlib.util.spec_from_file_location(
        "make_oracle_golden", os.path.join(HERE, "golden", "make_oracle_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


CASES = [
    # ragged last band (37 = 16 + 16 + 5 with 16-row bands), noise start
    dict(nx=40, ny=37, T=300.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25,
         Lambda_g=1e-6, noise_amp=1e-3, seed=181205711),
    # Eq. 29 start, another Lambda, a grid narrower than one band is tall
    dict(nx=9, ny=24, T=200.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=1.0, Lambda=1 / 12,
         Lambda_g=1e-6, init_mode="eq29", seed=7),
    # rows longer than a band of wavenumber columns (600 = 256 + 256 + 88)
    dict(nx=600, ny=21, T=400.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25,
         Lambda_g=1e-6, noise_amp=1e-3, seed=3),
]


@pytest.mark.parametrize("band_rows", [16, 5, 4, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_banded_steps_equal_oracle_step(case, band_rows):
    drv = _driver()
    p = Params(**CASES[case])
    ref, o = Oracle(p), Oracle(p)
    with ThreadPoolExecutor(3) as pool:
        for k in (1, 4):
            ref.step(k)
            drv.step_in_bands(o, pool, k, band_rows=band_rows)
            assert o.n == ref.n
            assert np.array_equal(o.ft, ref.ft)
            assert np.array_equal(o.gt, ref.gt)
    fr, fo = ref.fields(), o.fields()
    for key in drv.FIELDS:
        assert np.array_equal(fo[key], fr[key]), key


def test_banded_driver_refuses_pending_change_of_T():
    drv = _driver()
    o = Oracle(Params(**CASES[0]))
    o.set_T(250.0)
    with ThreadPoolExecutor(2) as pool, pytest.raises(ValueError):
        drv.step_in_bands(o, pool, 1)
