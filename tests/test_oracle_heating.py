"""Pins of the heating-rate oracle (Sect. 5; efficiency of Wolfire et al.
1995) by limits and structure, not by retyping the formula."""
import numpy as np

from oracle import heating as H


def test_efficiency_limits():
    T = np.array([10.0, 100.0, 1e4, 8000.0])
    # x -> 0 (no UV, or n_e much larger than G0 T^(1/2)): both terms at full strength
    e0 = H.efficiency(np.zeros(4), T, np.full(4, 1.0))
    np.testing.assert_allclose(e0, 4.9e-2 + 3.7e-2 * (T / 1e4) ** 0.7, rtol=1e-12)
    # T = 1e4 K: 4.9e-2 + 3.7e-2 = 8.6e-2
    np.testing.assert_allclose(H.efficiency(0.0, 1e4, 1.0), 0.086, rtol=1e-12)
    # x -> infinity: eps -> 0, with log-log slopes -0.73 (first term) and -1 (second)
    big = np.array([1e12, 1e13])
    e_first = H.efficiency(big, 0.0 * big + 1.0, np.ones(2))  # T = 1: second term ~3.7e-2 1e-2.8 / x
    slope = np.log(e_first[1] / e_first[0]) / np.log(10.0)
    assert -1.0 <= slope <= -0.73 + 1e-3
    assert H.efficiency(1e30, 1e4, 1.0) < 1e-15
    # no electrons: x is infinite as soon as there is UV
    assert H.efficiency(1.0, 100.0, 0.0) == 0.0


def test_efficiency_decreases_with_the_uv_field():
    g = np.logspace(-3, 3, 61)
    e = H.efficiency(g, 100.0, 0.01)
    assert np.all(np.diff(e) < 0)


def test_rates_structure():
    n = np.array([1.0, 10.0, 1000.0])
    T = np.array([8000.0, 1000.0, 20.0])
    ne = 1e-3 * n
    g, uv, cr = H.rates(np.zeros(3), n, T, ne)
    assert np.all(g == 0) and np.all(uv == 0)            # fully screened: no photoelectric heating
    np.testing.assert_array_equal(cr, 1e-27 * n)        # cosmic rays: linear in n, unscreened
    g, uv, cr = H.rates(np.ones(3), n, T, ne)
    np.testing.assert_allclose(g, 1.7)                   # unscreened: the Draine field in Habing units
    g2, uv2, _ = H.rates(np.ones(3), 2 * n, T, ne)      # eps depends on n only through n_e:
    np.testing.assert_allclose(uv2, 2 * uv, rtol=1e-12)  # the rate is linear in n at fixed n_e
    _, uv3, _ = H.rates(np.full(3, 0.5), n, T, ne)
    assert np.all(uv3 > 0.5 * uv)                       # eps falls with G0_eff, so half the field gives more than half

