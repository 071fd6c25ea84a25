"""The oracle's drag coefficient against the constants the paper prints for it
(tests/golden/drag_coefficient_constants.txt, each line cited).  Every check sits
at a limit where one constant shows alone, so a mistyped constant, a swapped
k branch or a wrong limit fails here.  CPU only."""
import math
from pathlib import Path

import pytest

GOLDEN = Path(__file__).parent / "golden" / "drag_coefficient_constants.txt"


def _constants():
    out = {}
    for line in GOLDEN.read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            name, value = line.split()[:2]
            out[name] = float(value)
    return out


C = _constants()


def test_fixture_is_complete():
    assert set(C) == {"drag_prefactor", "k_low", "k_high", "re_switch", "stokes_24",
                      "transition_40", "transition_10", "mach_023"}


def test_high_reynolds_subsonic_limit_is_k_high(orc):
    # Re -> inf, Ma = 0: the bracket term vanishes and 2 (0.8 k) / 1.6 = k
    assert abs(orc.drag_cd(1e15, 0.0) - C["k_high"]) < 1e-12


def test_k_changes_by_k_low_minus_k_high_at_the_switch(orc):
    re = C["re_switch"]
    below = orc.drag_cd(re * (1 - 1e-13), 0.0)
    at = orc.drag_cd(re * (1 + 1e-13), 0.0)
    assert abs((below - at) - (C["k_low"] - C["k_high"])) < 1e-9


def test_stokes_limit_coefficient(orc):
    # Re -> 0, Ma = 0: C_D - k_low -> (24/Re + 40/10)^2; the leading Re^-2 coefficient
    # is 24^2 and the next one 2 * 24 * (40/10)
    re = 1e-4
    t = orc.drag_cd(re, 0.0) - C["k_low"]
    lead = (C["stokes_24"] / re) ** 2
    nxt = 2 * C["stokes_24"] * C["transition_40"] / C["transition_10"] / re
    assert abs(t - lead - nxt) / lead < 1e-6


def test_transition_term(orc):
    # Re = 10 (below the switch), Ma = 0: (24/10 + 40/20)^2 + k_low
    re = C["transition_10"]
    expect = (C["stokes_24"] / re + C["transition_40"] / (C["transition_10"] + re)) ** 2
    assert abs(orc.drag_cd(re, 0.0) - (expect + C["k_low"])) < 1e-12


@pytest.mark.parametrize("ma", [0.5, 3.0])
def test_mach_coefficient(orc, ma):
    # Re = 10: C_D = ((24/10 + 40/20)^-1 + 0.23 Ma)^-2 + 2 (0.8 k_low + Ma) / (1.6 + Ma)
    re = C["transition_10"]
    inner = 1.0 / (C["stokes_24"] / re + C["transition_40"] / (C["transition_10"] + re))
    expect = (inner + C["mach_023"] * ma) ** -2 + 2 * (0.8 * C["k_low"] + ma) / (1.6 + ma)
    assert abs(orc.drag_cd(re, ma) - expect) < 1e-12 * expect


def test_drag_prefactor_through_the_acceleration(orc):
    # the same body at two relative speeds in the Ma -> inf limit (C_D -> 2 there for
    # every k): |a| / dv^2 = prefactor * C_D * rho_g / (r_p rho_p) is checked as a
    # ratio against the prefactor times the oracle's own C_D at those points
    import numpy as np
    from synth import ic
    p = ic.default_params(n_big=1, n_small=1, gas_on=1)
    R = 2.0
    mu0 = ic.G
    x = np.zeros((3, 2)); u = np.zeros((3, 2))
    x[:, 0] = [9.0, 0, 0]
    mu = np.array([1e-14])
    x[:, 1] = [R, 0, 0]
    vg = math.sqrt(mu0 / R) * math.sqrt(1 - 2 * p["eta"])
    rp, rho = 5.0 * ic.KM_AU, 2.0 * ic.RHO_UNIT
    acc = []
    for dv in (0.3, 0.6):   # AU/day: far supersonic, Ma >> 1
        u[:, 1] = [dv, vg, 0.0]
        a = orc.drag(p, x, u, mu, np.array([rp]), np.array([rho]), 1)
        acc.append(np.linalg.norm(a[:, 1]) / dv ** 2)
    # same rho_g, r_p, rho_p: the ratio is the ratio of the two C_D, both near 2
    assert abs(acc[1] / acc[0] - 1) < 0.02
    # the midplane gas density of Eq. 4 with Sigma = 1700 (R/1AU)^-1 g/cm^2, H/r = 0.05
    AU = ic.AU_CM
    sig = p["sigma1"] * R ** -1.0
    rho_g = sig / (math.sqrt(2 * math.pi) * p["h_over_r"] * R * AU) * AU ** 3 / ic.MSUN_G
    cd_limit = 2.0
    implied_prefactor = acc[1] * rp * rho / (rho_g * cd_limit)
    assert abs(implied_prefactor - C["drag_prefactor"]) < 0.02 * C["drag_prefactor"]
