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


def test_efficiency_knee_of_the_first_term():
    """Sect. 5 (efficiency of Wolfire et al. 1995): the first term halves at
    x = G0_eff T^(1/2) / n_e = 1925.  At T = 1e-12 K the second term is below
    1e-12 of it, so eps is 4.9e-2 / 2 there; a knee read as 5000 would give
    3.27e-2."""
    T = 1e-12
    ne = np.array([1.0, 0.5, 2.0])
    g0 = 1925.0 * ne / np.sqrt(T)
    eps = H.efficiency(g0, np.full(3, T), ne)
    np.testing.assert_allclose(eps, 0.5 * 4.9e-2, rtol=1e-9)
    # a factor 10 on either side of the knee: the power law 0.73 of the first term
    for f in (0.1, 10.0):
        e = H.efficiency(f * g0[:1], np.array([T]), ne[:1])
        np.testing.assert_allclose(e, 4.9e-2 / (1.0 + f ** 0.73), rtol=1e-9)


def test_efficiency_knee_of_the_second_term():
    """Sect. 5: the second term halves at x = 5000.  At a fixed x the first
    term is the same at every temperature, so the difference between T = 1e4 K
    and T = 1e-12 K (x kept at 5000 by the field) is the second term alone,
    3.7e-2 (1 - 1e-11.2) / 2; a knee read as 1925 would give 1.03e-2."""
    ne = 1.0
    x = 5000.0
    e_hot = H.efficiency(x * ne / np.sqrt(1e4), 1e4, ne)
    e_cold = H.efficiency(x * ne / np.sqrt(1e-12), 1e-12, ne)
    np.testing.assert_allclose(e_hot - e_cold, 0.5 * 3.7e-2 * (1.0 - (1e-16) ** 0.7), rtol=1e-9)
