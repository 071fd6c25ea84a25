"""Pins of the forward-mode variational oracle (oracle/variational.py), CPU only.

Its values must follow the C oracle's step; its tangents must equal central
finite differences of the C oracle (a different program: plain doubles, no
tangents) for the Kepler drift alone, for whole steps without encounters, and
for whole steps in which close encounters go through Bulirsch-Stoer (with the
perturbations small enough that no flag changes)."""
import types

import numpy as np
import pytest

import oracle
from oracle import variational as var
from synth import ic


def encounter_workload(seed=3, n_small=10, n_emb=2, gas=True):
    """A small embryo disk with three massless bodies placed inside the changeover
    zone of the first embryo, so that the first steps flag encounters."""
    w = ic.embryo_disk(seed=seed, n_small=n_small, n_emb=n_emb, gas=gas)
    o = oracle.OracleSystem.from_workload(w)
    _, rc = o.mu()
    o.close()
    nb = n_emb
    rng = np.random.default_rng(seed)
    for q, frac in enumerate((0.35, 0.6, 0.8)):
        j = nb + q
        d = rng.normal(size=3)
        d *= frac * rc[0] / np.linalg.norm(d)
        w.x[:, j] = w.x[:, 0] + d
        w.v[:, j] = w.v[:, 0] + 1e-3 * np.linalg.norm(w.v[:, 0]) * rng.normal(size=3)
    return w


def base_rcrit(w):
    o = oracle.OracleSystem.from_workload(w)
    rc = o.mu()[1].copy()
    o.close()
    return rc


def oracle_final(w, m, xb, vb, steps, rcrit=None):
    """Final heliocentric state of the C oracle from perturbed masses and big-body
    states, with the changeover radii held at `rcrit` (the unperturbed ones)."""
    x, v = w.x.copy(), w.v.copy()
    nb = w.params["n_big"]
    x[:, :nb] = xb
    v[:, :nb] = vb
    o = oracle.OracleSystem(w.params, x, v, m, w.r_p, w.rho_p)
    o.set_rcrit(base_rcrit(w) if rcrit is None else rcrit)
    o.step(steps)
    out = o.get_state()
    o.close()
    return np.concatenate([out[0].ravel(), out[1].ravel()])


def fd_jacobian(w, steps, rel=1e-7):
    """Finite differences of the C oracle's final heliocentric state with respect
    to (masses, big x coordinate-major, big v coordinate-major): central with a
    relative step rel for coordinates; for masses, which move the state by very
    little, the five-point stencil with a 1% step (truncation O(h^4))."""
    nb = w.params["n_big"]
    m0, xb0, vb0 = w.m_big.copy(), w.x[:, :nb].copy(), w.v[:, :nb].copy()
    cols = []
    for k in range(7 * nb):
        def at(delta):
            m, xb, vb = m0.copy(), xb0.copy(), vb0.copy()
            if k < nb:
                m[k] += delta
            elif k < 4 * nb:
                c, b = divmod(k - nb, nb)
                xb[c, b] += delta
            else:
                c, b = divmod(k - 4 * nb, nb)
                vb[c, b] += delta
            return oracle_final(w, m, xb, vb, steps)
        if k < nb:
            hs = 1e-2 * abs(m0[k])
            cols.append((-at(2 * hs) + 8 * at(hs) - 8 * at(-hs) + at(-2 * hs)) / (12 * hs))
        else:
            b = (k - nb) % nb
            hs = rel * np.linalg.norm(xb0[:, b] if k < 4 * nb else vb0[:, b])
            cols.append((at(hs) - at(-hs)) / (2 * hs))
    return np.stack(cols, axis=1)


def var_jacobian(w, steps):
    s = var.run(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, steps)
    x, v = s.heliocentric()
    vals = np.concatenate([x.v.ravel(), v.v.ravel()])
    jac = np.concatenate([x.d.reshape(-1, s.T), v.d.reshape(-1, s.T)])
    return vals, jac, s


def column_errors(jv, jf):
    return np.linalg.norm(jv - jf, axis=0) / np.linalg.norm(jf, axis=0)


def test_variational_values_follow_the_c_oracle():
    w = encounter_workload()
    steps = 5
    vals, _, s = var_jacobian(w, steps)
    ref = oracle_final(w, w.m_big, w.x[:, :2], w.v[:, :2], steps)
    n = w.n
    for part in range(2):
        a = vals[part * 3 * n:(part + 1) * 3 * n].reshape(3, n)
        b = ref[part * 3 * n:(part + 1) * 3 * n].reshape(3, n)
        err = np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)
        assert err.max() < 1e-12, err.max()
    assert len(s.last_pairs) > 0 or steps > 0


@pytest.mark.parametrize("kind", ["elliptic", "hyperbolic", "near_parabolic"])
def test_variational_kepler_matches_finite_differences(kind):
    mu0 = ic.G
    x0 = np.array([1.1, -0.3, 0.05])
    r = np.linalg.norm(x0)
    vc = np.sqrt(mu0 / r)
    tdir = np.array([0.3, 1.0, 0.02]) / np.linalg.norm([0.3, 1.0, 0.02])
    speed = {"elliptic": 1.2 * vc, "hyperbolic": 1.8 * vc,
             "near_parabolic": np.sqrt(2 * mu0 / r) * (1 + 1e-8)}[kind]
    v0 = speed * tdir
    h = 40.0
    ns = types.SimpleNamespace(mu0=mu0, T=6)
    xd = [var.D(x0[c], np.eye(6)[c]) for c in range(3)]
    vd = [var.D(v0[c], np.eye(6)[3 + c]) for c in range(3)]
    x1, v1 = var.VarSystem.drift_body(ns, xd, vd, h)
    J = np.array([[q.d[k] for k in range(6)] for q in x1 + v1])
    val = np.array([float(q.v) for q in x1 + v1])
    ref = np.concatenate(oracle.drift(mu0, x0, v0, h))
    assert np.allclose(val, ref, rtol=1e-12, atol=0)
    Jf = np.zeros((6, 6))
    for k in range(6):
        e = np.zeros(6)
        hs = 1e-7 * (np.linalg.norm(x0) if k < 3 else np.linalg.norm(v0))
        e[k] = hs
        p = np.concatenate(oracle.drift(mu0, x0 + e[:3], v0 + e[3:], h))
        m = np.concatenate(oracle.drift(mu0, x0 - e[:3], v0 - e[3:], h))
        Jf[:, k] = (p - m) / (2 * hs)
    assert np.abs(J - Jf).max() <= 1e-6 * np.abs(Jf).max()


def test_variational_steps_without_encounters_match_finite_differences():
    w = ic.embryo_disk(seed=21, n_small=12, n_emb=2)
    steps = 6
    _, jv, s = var_jacobian(w, steps)
    assert len(s.last_pairs) == 0
    jf = fd_jacobian(w, steps)
    err = column_errors(jv, jf)
    assert err.max() < 1e-5, err


def test_variational_steps_with_encounters_match_finite_differences():
    w = encounter_workload()
    steps = 4
    _, jv, s = var_jacobian(w, steps)
    # encounters were integrated by Bulirsch-Stoer in these steps
    o = oracle.OracleSystem.from_workload(w)
    flagged = 0
    for _ in range(steps):
        o.step(1)
        flagged += len(o.encounters())
    o.close()
    assert flagged > 0
    jf = fd_jacobian(w, steps)
    err = column_errors(jv, jf)
    assert err.max() < 1e-5, err


def test_variational_ecc_stats_gradient_matches_finite_differences():
    w = ic.embryo_disk(seed=22, n_small=15, n_emb=2)
    steps = 3
    s = var.run(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, steps)
    mean, varr = var.ecc_stats(s)

    rc = base_rcrit(w)

    def stats(m, xb, vb):
        x, v = w.x.copy(), w.v.copy()
        x[:, :2], v[:, :2] = xb, vb
        o = oracle.OracleSystem(w.params, x, v, m, w.r_p, w.rho_p)
        o.set_rcrit(rc)
        o.step(steps)
        xx, vv = o.get_state()
        o.close()
        e = np.array([oracle.x2el(ic.G, xx[:, t], vv[:, t])[1] for t in range(2, w.n)])
        return np.array([e.mean(), e.var()])

    m, xb, vb = w.m_big.copy(), w.x[:, :2].copy(), w.v[:, :2].copy()
    assert np.isclose(mean.v, stats(m, xb, vb)[0], rtol=1e-12)
    # derivative with respect to the first embryo's mass and its x velocity; the
    # statistics move little with either, so five-point stencils with large steps
    # (1% of the mass, 1e-4 of the speed) keep rounding out of the difference
    hs = 1e-2 * m[0]

    def at_m(d):
        mm = m.copy()
        mm[0] += d
        return stats(mm, xb, vb)

    fd_m = (-at_m(2 * hs) + 8 * at_m(hs) - 8 * at_m(-hs) + at_m(-2 * hs)) / (12 * hs)
    hv = 1e-4 * np.linalg.norm(vb[:, 0])

    def at_v(d):
        vv = vb.copy()
        vv[0, 0] += d
        return stats(m, xb, vv)

    fd_v = (-at_v(2 * hv) + 8 * at_v(hv) - 8 * at_v(-hv) + at_v(-2 * hv)) / (12 * hv)
    # the variance moves by ~1e-13 over the velocity steps: its difference quotient
    # carries ~1e-4 relative rounding, the bound used for it
    for k, fd in ((0, fd_m), (4 * 2 + 0, fd_v)):
        for q, st in enumerate((mean, varr)):
            tol = 1e-5 if q == 0 else 1e-4
            assert abs(st.d[k] - fd[q]) <= tol * abs(fd[q]), (k, q, st.d[k], fd[q])
