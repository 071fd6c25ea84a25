"""Seeded synthetic initial conditions for the hybrid-step workloads.

This module only draws random orbital elements and turns them into heliocentric
Cartesian states; it holds none of the integrator's arithmetic.  Both the CPU
oracle (tests) and the HIP path (tests, bench) are fed from here.

Units: AU, day, solar mass.  G = k^2 with the Gaussian constant k.

Workload shapes (all seeded with numpy PCG64 ``default_rng(seed)``):

* ``two_giants``       -- star + Jupiter (5.2 AU) + 0.3 M_J (9.5 AU) + massless disk
                          a~U[2,12] AU; e~Rayleigh(0.01); i~Rayleigh(0.005).
* ``embryo_disk``      -- 10 embryos (log-uniform 0.1-1 M_earth, a log-uniform 1-10 AU)
                          + massless planetesimals a~U[1,10] AU, radius log-uniform
                          1-100 km, density 1.5 g/cm^3, in a gas disk
                          Sigma = 1700 (R/1AU)^-1 g/cm^2, H/r = 0.05, eta = 0.002.
* ``self_gravitating`` -- 4 growing planets (a log-uniform 0.5-4 AU; 0.1 -> 1 M_earth
                          over 1e5 yr) + 4000 massive planetesimals of 1e-4 M_earth,
                          a~U[0.5,4] AU, e,i~Rayleigh(0.005); every body interacts.
* ``batch``            -- 256 independent embryo-disk systems of uneven size.

Planet (big-body) states use gm = G(m0 + m_k); massless bodies use gm = G m0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------- constants
K_GAUSS = 0.01720209895
G = K_GAUSS * K_GAUSS                 # AU^3 Msun^-1 day^-2
M_EARTH = 3.0034896e-6                # Msun
M_JUP = 9.5458e-4                     # Msun
AU_CM = 1.495978707e13                # cm per AU
MSUN_G = 1.98847e33                   # g per Msun
RHO_UNIT = AU_CM ** 3 / MSUN_G        # Msun/AU^3 per g/cm^3  (~1.68367e6)
KM_AU = 1.0e5 / AU_CM                 # AU per km
YEAR_D = 365.25
# mean free path coefficient: lambda[AU] = MFP_COEF / rho_g[Msun/AU^3]
MU_MOL = 2.34
M_H_G = 1.6735575e-24                 # g
SIGMA_H2_CM2 = 2.0e-15                # cm^2
MFP_COEF = MU_MOL * M_H_G * RHO_UNIT / (SIGMA_H2_CM2 * AU_CM)
# isothermal sound speed squared per kelvin, k_B / (mu_mol m_H), in AU^2 day^-2 K^-1
K_BOLTZ = 1.380649e-16                # erg/K
CS2_PER_K = K_BOLTZ / (MU_MOL * M_H_G) * (86400.0 / AU_CM) ** 2


@dataclass
class Workload:
    """A system ready for either path. Arrays are SoA [3][n] float64, big bodies first."""
    name: str
    params: dict
    x: np.ndarray            # [3, n] heliocentric positions, AU
    v: np.ndarray            # [3, n] heliocentric velocities, AU/day
    m_big: np.ndarray        # [n_big] masses, Msun
    r_p: np.ndarray | None = None     # [n_small] radii, AU
    rho_p: np.ndarray | None = None   # [n_small] densities, g/cm^3
    growth: np.ndarray | None = None  # [n_big, 3] (M0, Mc, tau_c[day]); tau_c<=0: fixed mass
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.x.shape[1]


def default_params(**kw) -> dict:
    p = dict(G=G, m0=1.0, dt=1.0, rcrit_hill=3.0, bs_tol=1e-12,
             n_big=0, n_small=0, gas_on=0,
             sigma1=1700.0, gamma=1.0, r_c=0.0, r_in=0.0, h_over_r=0.05, eta=0.002,
             kdrag_exp=-2.0, rho_unit=RHO_UNIT, au_cm=AU_CM, mfp_coef=MFP_COEF,
             temp_1au=0.0, temp_beta=0.5, cs2_per_k=CS2_PER_K, eta_mode=0, dg_mode=0)
    p.update(kw)
    return p


def rayleigh(rng, sigma, size):
    u = rng.random(size)
    return sigma * np.sqrt(-2.0 * np.log1p(-u))


def _solve_kepler(M, e):
    M = np.mod(M, 2 * np.pi)
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(60):
        f = E - e * np.sin(E) - M
        E = E - f / (1 - e * np.cos(E))
    return E


def el2x(gm, a, e, inc, node, peri, M):
    """Elliptic elements -> heliocentric state, arrays of shape [k]. Returns ([3,k], [3,k])."""
    gm = np.broadcast_to(np.asarray(gm, dtype=np.float64), np.shape(a))
    E = _solve_kepler(M, e)
    cE, sE = np.cos(E), np.sin(E)
    b = a * np.sqrt(1 - e * e)
    xp = a * (cE - e)
    yp = b * sE
    n = np.sqrt(gm / a ** 3)
    edot = n / (1 - e * cE)
    vxp = -a * sE * edot
    vyp = b * cE * edot
    cO, sO = np.cos(node), np.sin(node)
    cw, sw = np.cos(peri), np.sin(peri)
    ci, si = np.cos(inc), np.sin(inc)
    r11 = cO * cw - sO * sw * ci
    r12 = -cO * sw - sO * cw * ci
    r21 = sO * cw + cO * sw * ci
    r22 = -sO * sw + cO * cw * ci
    r31 = sw * si
    r32 = cw * si
    x = np.stack([r11 * xp + r12 * yp, r21 * xp + r22 * yp, r31 * xp + r32 * yp])
    v = np.stack([r11 * vxp + r12 * vyp, r21 * vxp + r22 * vyp, r31 * vxp + r32 * vyp])
    return x, v


def _angles(rng, k):
    return (rng.random(k) * 2 * np.pi, rng.random(k) * 2 * np.pi, rng.random(k) * 2 * np.pi)


def period(gm, a):
    return 2 * np.pi * math.sqrt(a ** 3 / gm)


def two_giants(seed: int = 0, n_small: int = 1000) -> Workload:
    rng = np.random.default_rng(seed)
    m0 = 1.0
    m_big = np.array([1.0 * M_JUP, 0.3 * M_JUP])
    a_b = np.array([5.2, 9.5])
    e_b = np.array([0.05, 0.05])
    i_b = rayleigh(rng, 0.005, 2)
    O, w, M = _angles(rng, 2)
    xb, vb = el2x(G * (m0 + m_big), a_b, e_b, i_b, O, w, M)
    a_s = rng.uniform(2.0, 12.0, n_small)
    e_s = rayleigh(rng, 0.01, n_small)
    i_s = rayleigh(rng, 0.005, n_small)
    O, w, M = _angles(rng, n_small)
    xs, vs = el2x(G * m0, a_s, e_s, i_s, O, w, M)
    dt = period(G * (m0 + M_JUP), 5.2) / 20.0
    p = default_params(m0=m0, dt=dt, n_big=2, n_small=n_small, gas_on=0)
    return Workload("two_giants", p, np.hstack([xb, xs]), np.hstack([vb, vs]), m_big,
                    meta=dict(seed=seed, steps=1000))


def embryo_disk(seed: int = 0, n_small: int = 100_000, n_emb: int = 10,
                gas: bool = True) -> Workload:
    rng = np.random.default_rng(seed)
    m0 = 1.0
    m_big = M_EARTH * np.exp(rng.uniform(math.log(0.1), math.log(1.0), n_emb))
    a_b = np.exp(rng.uniform(math.log(1.0), math.log(10.0), n_emb))
    e_b = rayleigh(rng, 0.01, n_emb)
    i_b = rayleigh(rng, 0.005, n_emb)
    O, w, M = _angles(rng, n_emb)
    xb, vb = el2x(G * (m0 + m_big), a_b, e_b, i_b, O, w, M)
    a_s = rng.uniform(1.0, 10.0, n_small)
    e_s = rayleigh(rng, 0.01, n_small)
    i_s = rayleigh(rng, 0.005, n_small)
    O, w, M = _angles(rng, n_small)
    xs, vs = el2x(G * m0, a_s, e_s, i_s, O, w, M)
    r_p = KM_AU * np.exp(rng.uniform(math.log(1.0), math.log(100.0), n_small))
    rho_p = np.full(n_small, 1.5)
    dt = period(G * m0, 1.0) / 20.0
    p = default_params(m0=m0, dt=dt, n_big=n_emb, n_small=n_small, gas_on=int(gas),
                       sigma1=1700.0, gamma=1.0, r_c=0.0, r_in=0.0, h_over_r=0.05, eta=0.002)
    return Workload("embryo_disk", p, np.hstack([xb, xs]), np.hstack([vb, vs]), m_big,
                    r_p=r_p, rho_p=rho_p, meta=dict(seed=seed, steps=10_000))


def self_gravitating(seed: int = 0, n_pl: int = 4, n_pls: int = 4000) -> Workload:
    rng = np.random.default_rng(seed)
    m0 = 1.0
    a_p = np.exp(rng.uniform(math.log(0.5), math.log(4.0), n_pl))
    a_s = rng.uniform(0.5, 4.0, n_pls)
    a = np.concatenate([a_p, a_s])
    nb = n_pl + n_pls
    e = rayleigh(rng, 0.005, nb)
    i = rayleigh(rng, 0.005, nb)
    O, w, M = _angles(rng, nb)
    m_big = np.concatenate([np.full(n_pl, 0.1 * M_EARTH), np.full(n_pls, 1e-4 * M_EARTH)])
    x, v = el2x(G * (m0 + m_big), a, e, i, O, w, M)
    growth = np.zeros((nb, 3))
    growth[:n_pl, 0] = 0.1 * M_EARTH
    growth[:n_pl, 1] = 1.0 * M_EARTH
    growth[:n_pl, 2] = 1e5 * YEAR_D
    dt = period(G * m0, 0.5) / 20.0
    p = default_params(m0=m0, dt=dt, n_big=nb, n_small=0, gas_on=0)
    return Workload("self_gravitating", p, x, v, m_big, growth=growth,
                    meta=dict(seed=seed, steps=5000))


def crowded_annulus(seed: int = 0, n_big: int = 96, n_small: int = 2000,
                    close_pairs: int = 3) -> Workload:
    """Many massive bodies (0.02-0.2 M_earth, log-uniform) and massless bodies in one
    narrow annulus a~U[1.0, 1.5] AU, e~Rayleigh(0.01), i~Rayleigh(0.005), so that
    close encounters happen every step; the last close_pairs massive bodies are put
    4e-3 AU from massive bodies 0, 1, ... (a few changeover radii apart at most) with
    nearly the same velocity, so pairs of massive bodies meet as well."""
    rng = np.random.default_rng(seed)
    m0 = 1.0
    m_big = M_EARTH * np.exp(rng.uniform(math.log(0.02), math.log(0.2), n_big))
    a = rng.uniform(1.0, 1.5, n_big + n_small)
    e = rayleigh(rng, 0.01, n_big + n_small)
    i = rayleigh(rng, 0.005, n_big + n_small)
    O, w, M = _angles(rng, n_big + n_small)
    gm = np.concatenate([G * (m0 + m_big), np.full(n_small, G * m0)])
    x, v = el2x(gm, a, e, i, O, w, M)
    for q in range(close_pairs):
        k = n_big - 1 - q
        d = rng.normal(size=3)
        d *= 4e-3 / np.linalg.norm(d)
        x[:, k] = x[:, q] + d
        v[:, k] = v[:, q] * (1 + rng.normal(0, 1e-4, 3))
    dt = period(G * m0, 1.0) / 40.0
    p = default_params(m0=m0, dt=dt, n_big=n_big, n_small=n_small, gas_on=0)
    return Workload("crowded_annulus", p, x, v, m_big, meta=dict(seed=seed))


def batch(seed: int = 0, n_sys: int = 256, n_small_range=(1_000, 50_000),
          n_pl_range=(2, 8)) -> list[Workload]:
    """Uneven ensemble: per-system seed = 1000*seed + index."""
    out = []
    for s in range(n_sys):
        rng = np.random.default_rng(1000 * seed + s)
        n_pl = int(rng.integers(n_pl_range[0], n_pl_range[1] + 1))
        lo, hi = n_small_range
        ns = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        w = embryo_disk(seed=1000 * seed + s, n_small=ns, n_emb=n_pl)
        w.name = f"batch[{s}]"
        out.append(w)
    return out


def adjoint_shape(seed: int = 0, n_small: int = 20_000) -> Workload:
    w = embryo_disk(seed=seed, n_small=n_small)
    w.name = "adjoint_disk"
    w.meta["steps"] = 1000
    w.meta["checkpoint"] = 50
    return w


WORKLOADS = {
    "two_giants": two_giants,
    "embryo_disk": embryo_disk,
    "self_gravitating": self_gravitating,
    "adjoint_disk": adjoint_shape,
}
