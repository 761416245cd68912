"""FP64 reference of the gas heating rates driven by the screening factor.

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.
Plain numpy, float64 throughout.

The paper (Sect. 5) couples the columns to the thermal balance through:

* the effective UV field, the Draine field G0 = 1.7 (Habing units)
  attenuated by the screening factor: G0_eff = chi G0;
* the photoelectric heating rate on small grains and PAHs,
  Gamma_UV = 1e-24 eps G0_eff n  (erg cm^-3 s^-1), with the efficiency of
  Wolfire et al. (1995), written with x = G0_eff T^(1/2) / n_e:
  eps = 4.9e-2 / (1 + (x / 1925)^0.73) + 3.7e-2 (T / 1e4)^0.7 / (1 + x / 5000);
* the cosmic-ray heating rate Gamma_CR = 1e-27 n  (erg cm^-3 s^-1).

n is the hydrogen density (cm^-3), T the temperature (K), n_e the electron
density (cm^-3).  The paper takes n_e from an approximation it cites but does
not state; here n_e is an input.

Pinned (tests/test_oracle_heating.py) by: the limits x -> 0 (eps -> 4.9e-2 +
3.7e-2 (T/1e4)^0.7) and x -> infinity (eps -> 0, the decay exponents 0.73
and 1 read off the log-log slope), no heating without UV (chi = 0) and a
rate linear in n, and the monotonic decrease of eps with G0_eff.
"""
from __future__ import annotations

import numpy as np

G0_DRAINE = 1.7


def efficiency(g0eff, T, ne) -> np.ndarray:
    g0eff, T, ne = (np.asarray(a, dtype=np.float64) for a in (g0eff, T, ne))
    with np.errstate(divide="ignore", invalid="ignore"):
        x = g0eff * np.sqrt(T) / ne
    x = np.where(ne > 0, x, np.where(g0eff * np.sqrt(T) > 0, np.inf, 0.0))
    return 4.9e-2 / (1.0 + (x / 1925.0) ** 0.73) + 3.7e-2 * (T / 1e4) ** 0.7 / (1.0 + x / 5000.0)


def rates(chi, n, T, ne, G0: float = G0_DRAINE):
    """(G0_eff, Gamma_UV, Gamma_CR) per cell."""
    chi, n = np.asarray(chi, dtype=np.float64), np.asarray(n, dtype=np.float64)
    g = chi * G0
    return g, 1e-24 * efficiency(g, T, ne) * g * n, 1e-27 * n
