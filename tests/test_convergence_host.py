"""Host logic of the convergence study (no GPU): the field from the
potential with the collision's ghost rows, the restriction to coarse nodes,
and the observed order of self-convergence."""

import math

import numpy as np
import pytest

from paper_1812_05711_amd import convergence as cv


@pytest.mark.parametrize("ny", [3, 10, 64])
def test_uniform_field_from_a_linear_potential(ny):
    y = (np.arange(ny) + 0.5) / ny
    assert np.allclose(cv.field_from_potential(1.0 - y), 1.0, rtol=0, atol=1e-13)


def test_restriction_is_the_pair_mean():
    assert np.array_equal(cv.restrict(np.array([1.0, 3.0, 5.0, 9.0])), np.array([2.0, 7.0]))


def test_second_order_profiles_give_order_two():
    # g at the nodes plus an h^2 error term: the differences to the next finer
    # grid fall as h^2
    g = lambda y: np.exp(y) + y * y
    k = lambda y: np.cos(3.0 * y)
    prof = {}
    for n in (32, 64, 128, 256, 512):
        y = (np.arange(n) + 0.5) / n
        prof[n] = g(y) + k(y) / n**2
    res = cv.self_convergence(prof)
    assert [r[0] for r in res] == [32, 64, 128, 256]
    assert res[-1][2] is None
    for ny, e, order in res[:-1]:
        assert e > 0 and abs(order - 2.0) < 0.05, (ny, order)
    with pytest.raises(ValueError):
        cv.self_convergence({10: np.zeros(10), 30: np.zeros(30)})


def test_ionic_steps():
    # tau+ = 1, T = 1200, M = 10: K = (1/6) 1200 / 100 = 2
    assert cv.ionic_steps(100) == pytest.approx(5000.0)
    assert math.isclose(cv.ionic_steps(50, T=600.0), 2 * cv.ionic_steps(50))
