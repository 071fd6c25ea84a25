"""Parity of the HIP path with the CPU oracle (GPU tests, called through the C ABI).

Tolerances: positions and velocities of one step 1e-12 relative (per body, against
the body's own |x| and |u|); energy-drift difference 1e-10.  Kernel-level checks
use the same seeded inputs on both sides.  Encounter flags are integer decisions
that each side takes from its own floating-point minimum (the oracle's is written
independently of the kernel's): a pair may be flagged on one side only when the
deciding quantity lies within the margin the tolerances allow of its threshold
(tests/parity_helpers.py); such pairs are counted and printed, and their bodies are
left out of that step's per-body comparison.
"""
import math

import numpy as np
import pytest

from synth import ic
from parity_helpers import (compare_pairs, relerr_per_body, relerr_rows, step_close)

pytestmark = pytest.mark.gpu

G = ic.G
MU0 = G


@pytest.fixture(scope="module")
def mx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_16791_amd as m
    m.lib()
    return m


def oracle_sensitivity(o, x, u, step_index, trials=2, seed=0):
    """Per-body relative change of the oracle's own one-step result when every input
    coordinate is moved by at most one ulp (relative 2.2e-16).  A body in a deep
    encounter can amplify such differences by orders of magnitude within one step;
    the GPU is then held to the oracle's own reproducibility.  Leaves o at the
    unperturbed result (its last step is the unperturbed one)."""
    rng = np.random.default_rng(seed)
    o.set_dh(x, u, step_index)
    o.step(1)
    xr, ur = o.get_dh()
    sx = np.zeros(x.shape[1]); su = np.zeros(x.shape[1])
    for _ in range(trials):
        xp = x * (1 + rng.uniform(-2.2e-16, 2.2e-16, x.shape))
        up = u * (1 + rng.uniform(-2.2e-16, 2.2e-16, u.shape))
        o.set_dh(xp, up, step_index)
        o.step(1)
        xq, uq = o.get_dh()
        sx = np.maximum(sx, relerr_per_body(xq, xr))
        su = np.maximum(su, relerr_per_body(uq, ur))
    o.set_dh(x, u, step_index)
    o.step(1)
    return xr, ur, sx, su


def check_step(g, o, nb, sx=None, su=None, label=""):
    """One step of g (GPU) against the last step of o (oracle) from the same state.
    Without sensitivities every compared body is held to 1e-12; with them a body is
    held to max(1e-12, 10 x the oracle's own one-ulp sensitivity).  A body so loosened
    must be a member of a flagged pair (a body in an encounter), or else no more
    sensitive than the most sensitive loosened massive body (whose chaotic encounter
    reaches every body through the closing kick).  Returns (flagged pairs,
    borderline pairs, loosened bodies)."""
    xg, ug = g.get_dh()
    xo, uo = o.get_dh()
    pg, po = g.encounters(), o.encounters()
    excluded, n_border, big_border = compare_pairs(o, pg, po, xo, nb)
    if big_border:
        print(f"[parity] {label}: a massive pair is borderline; step not compared")
        return len(po), n_border, 0
    tx = ty = 1e-12
    loosened = np.zeros(xo.shape[1], dtype=bool)
    if sx is not None:
        tx = np.maximum(1e-12, 10 * sx)
        ty = np.maximum(1e-12, 10 * su)
        loosened = (tx > 1e-12) | (ty > 1e-12)
        members = set(po[:, 0].tolist()) | set(po[:, 1].tolist()) if len(po) else set()
        outside = sorted(set(np.nonzero(loosened)[0].tolist()) - members - excluded)
        if outside:
            sens = np.maximum(sx, su)
            big_loose = sens[:nb][loosened[:nb]]
            cap = float(big_loose.max()) if big_loose.size else 0.0
            worst = float(sens[outside].max())
            assert worst <= cap, (f"{label}: loosened bound on bodies outside encounters "
                                  f"{outside[:8]} (sensitivity {worst:.2e}, massive {cap:.2e})")
    ex, eu, bad_x, bad_u = step_close(xg, ug, xo, uo, excluded, tx, ty)
    print(f"[parity] {label}: pairs {len(po)}, borderline {n_border}, "
          f"loosened {int(loosened.sum())}, max rel err x {ex:.2e} u {eu:.2e}")
    assert bad_x.size == 0 and bad_u.size == 0, (label, bad_x[:8], bad_u[:8], ex, eu)
    return len(po), n_border, int(loosened.sum())


# ----------------------------------------------------------- gravity kernel
@pytest.mark.parametrize("n,nb,spread,rcf", [
    (1, 1, 1.0, 0.01), (7, 3, 1.0, 0.01), (255, 10, 5.0, 0.02), (257, 10, 5.0, 0.02),
    (1000, 40, 0.5, 0.3), (3000, 3000, 4.0, 0.002), (600, 0, 1.0, 0.1)])
def test_gravity_kernel_matches_oracle(mx, orc, n, nb, spread, rcf):
    rng = np.random.default_rng(n * 7 + nb)
    x = rng.uniform(-spread, spread, (3, n))
    mu = rng.uniform(1e-10, 1e-6, nb)
    rcrit = rng.uniform(0.5, 1.5, nb) * rcf * spread
    a_o = orc.gravity(x, mu, rcrit, nb)
    a_g = mx.gravity(x, mu, rcrit, nb).cpu().numpy()
    scale = np.abs(a_o).max() if nb else 1.0
    err = np.abs(a_g - a_o)
    assert np.all(err <= 1e-12 * np.abs(a_o) + 1e-14 * scale), err.max()


def test_gravity_changeover_zone_pairs(mx, orc):
    # every pair inside the changeover zone, including the K = 0 core
    rng = np.random.default_rng(1)
    n = 300
    x = rng.uniform(-0.05, 0.05, (3, n))
    mu = rng.uniform(1e-9, 1e-7, n)
    rcrit = np.full(n, 0.08)
    a_o = orc.gravity(x, mu, rcrit, n)
    a_g = mx.gravity(x, mu, rcrit, n).cpu().numpy()
    assert relerr_rows(a_g, a_o) < 1e-11


# -------------------------------------------------------------- drag kernel
def test_drag_kernel_matches_oracle(mx, orc):
    w = ic.embryo_disk(seed=3, n_small=5000, n_emb=6)
    o = orc.OracleSystem.from_workload(w)
    x, u = o.get_dh()
    mu, _ = o.mu()
    rho = w.rho_p * ic.RHO_UNIT
    a_o = orc.drag(w.params, x, u, mu, w.r_p, rho, w.params["n_big"])
    a_g = mx.gas_drag(w.params, x, u, mu, w.r_p, rho, w.params["n_big"]).cpu().numpy()
    nb = w.params["n_big"]
    assert np.all(a_g[:, :nb] == 0)
    assert relerr_rows(a_g[:, nb:], a_o[:, nb:]) < 1e-12


def test_drag_kernel_general_disk(mx, orc):
    """Tapered disk (gamma != 1), inner edge, other C_D exponent."""
    w = ic.embryo_disk(seed=4, n_small=3000, n_emb=3)
    p = dict(w.params, gamma=0.8, r_c=6.0, r_in=1.5, kdrag_exp=-1.0, eta=0.004)
    o = orc.OracleSystem(p, w.x, w.v, w.m_big, w.r_p, w.rho_p)
    x, u = o.get_dh()
    mu, _ = o.mu()
    rho = w.rho_p * ic.RHO_UNIT
    a_o = orc.drag(p, x, u, mu, w.r_p, rho, p["n_big"])
    a_g = mx.gas_drag(p, x, u, mu, w.r_p, rho, p["n_big"]).cpu().numpy()
    nb = p["n_big"]
    R = np.hypot(x[0, nb:], x[1, nb:])
    assert np.all(a_g[:, nb:][:, R < 1.5] == 0)
    assert relerr_rows(a_g[:, nb:], a_o[:, nb:]) < 1e-11


# -------------------------------------------------------------- Kepler drift
KEPLER_KINDS = ["disk", "eccentric", "hyperbolic", "near_parabolic", "backward", "plunging"]


@pytest.mark.parametrize("kind", KEPLER_KINDS)
def test_kepler_kernel_matches_oracle(mx, orc, kind):
    rng = np.random.default_rng(KEPLER_KINDS.index(kind))
    k = 513
    r = rng.uniform(0.5, 12, k)
    th = rng.uniform(0, 2 * np.pi, k)
    x0 = np.stack([r * np.cos(th), r * np.sin(th), rng.normal(0, 0.02, k) * r])
    vc = np.sqrt(MU0 / r)
    tang = np.stack([-np.sin(th), np.cos(th), np.zeros(k)])
    h = 18.26
    if kind == "disk":
        v0 = tang * vc * rng.uniform(0.97, 1.03, k) + rng.normal(0, 0.01, (3, k)) * vc
    elif kind == "eccentric":
        v0 = tang * vc * rng.uniform(0.2, 1.35, k)
        h = 400.0
    elif kind == "hyperbolic":
        v0 = tang * vc * rng.uniform(1.5, 3.0, k) + rng.normal(0, 0.1, (3, k)) * vc
        h = 300.0
    elif kind == "near_parabolic":
        v0 = tang * np.sqrt(2 * MU0 / np.linalg.norm(x0, axis=0)) * (1 + rng.uniform(-1e-8, 1e-8, k))
        h = 50.0
    elif kind == "backward":
        v0 = tang * vc * rng.uniform(0.9, 1.1, k)
        h = -25.0
    else:
        # near-radial infall through a close pericentre within the step (q ~ 1e-6 to
        # 1e-3 AU): the stiff case of the time equation
        rhat = x0 / np.linalg.norm(x0, axis=0)
        v0 = -rhat * vc * rng.uniform(0.5, 1.3, k) + tang * vc * 10 ** rng.uniform(-3.5, -1.5, k)
        h = 600.0
    xo = np.zeros_like(x0); vo = np.zeros_like(v0)
    for t in range(k):
        xo[:, t], vo[:, t] = orc.drift(MU0, x0[:, t], v0[:, t], h)
    xg, vg = mx.kepler_drift(MU0, x0, v0, h)
    assert relerr_rows(xg.cpu().numpy(), xo) < 1e-12
    assert relerr_rows(vg.cpu().numpy(), vo) < 1e-12


# --------------------------------------------------------------- flagging
def _flag_inputs(orc, seed, nb, ns, h, spread=0.08):
    rng = np.random.default_rng(seed)
    n = nb + ns
    a = np.concatenate([rng.uniform(3.0, 3.5, nb), rng.uniform(2.8, 3.7, ns)])
    e = rng.uniform(0, 0.05, n)
    inc = rng.uniform(0, 0.01, n)
    O = np.full(n, 0.3); w = np.full(n, 1.1)
    M = np.concatenate([rng.uniform(0, 0.5, nb), rng.normal(0.25, spread, ns)])
    x0, u0 = ic.el2x(MU0, a, e, inc, O, w, M)
    x1 = np.zeros_like(x0); u1 = np.zeros_like(u0)
    for t in range(n):
        x1[:, t], u1[:, t] = orc.drift(MU0, x0[:, t], u0[:, t], h)
    return x0, u0, x1, u1


def _flag_margin_ok(orc, x0, u0, x1, u1, i, j, rc, h):
    """Same inputs on both sides: a flag may differ only where the oracle's minimum
    lies within the rounding of the minimum itself of rc^2 (1e-12 relative, plus 64
    ulps of the squared scale of the pair's end points and slopes)."""
    r0, r1 = x0[:, j] - x0[:, i], x1[:, j] - x1[:, i]
    w0, w1 = u0[:, j] - u0[:, i], u1[:, j] - u1[:, i]
    d = orc.pair_dmin2(r0, w0, r1, w1, h)
    scale2 = max(r0 @ r0, r1 @ r1, h * h * (w0 @ w0), h * h * (w1 @ w1))
    return abs(d - rc * rc) <= 1e-12 * rc * rc + 64 * 2.2e-16 * scale2, d


@pytest.mark.parametrize("nb,ns", [(3, 700), (40, 300), (300, 0)])
def test_flag_kernel_matches_oracle(mx, orc, nb, ns):
    h = 20.0
    x0, u0, x1, u1 = _flag_inputs(orc, nb + ns, nb, ns, h)
    rcrit = np.random.default_rng(2).uniform(0.02, 0.08, nb)
    po = orc.flag(nb, rcrit, x0, u0, x1, u1, h)
    pg = mx.flag_pairs(nb, rcrit, x0, u0, x1, u1, h)
    so, sg = {tuple(p) for p in po}, {tuple(p) for p in pg}
    assert len(so) > 3
    for (i, j) in so ^ sg:  # only borderline decisions may differ
        rc = max(rcrit[i], rcrit[j] if j < nb else 0.0)
        ok, d = _flag_margin_ok(orc, x0, u0, x1, u1, i, j, rc, h)
        assert ok, (i, j, d, rc * rc)
    print(f"[parity] flag nb={nb} ns={ns}: {len(so)} pairs, {len(so ^ sg)} borderline")
    assert np.array_equal(pg, np.array(sorted(sg), dtype=np.int32).reshape(-1, 2))


# -------------------------------------------------------- whole-step parity
def _workloads():
    c1 = ic.two_giants(seed=0, n_small=400)
    c2 = ic.embryo_disk(seed=0, n_small=3000, n_emb=10)
    c3 = ic.self_gravitating(seed=0, n_pl=4, n_pls=600)
    c3.growth[:4, 2] = 40 * c3.params["dt"]   # the mass schedule moves within the test
    return {"two_giants": c1, "embryo_disk": c2, "self_gravitating": c3}


@pytest.mark.parametrize("name", ["two_giants", "embryo_disk", "self_gravitating"])
def test_step_parity_per_step(mx, orc, name):
    w = _workloads()[name]
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    nb = w.params["n_big"]
    x, u = g.get_dh()
    o.set_dh(x, u, 0)
    g.set_dh(x, u, 0)
    assert relerr_rows(g.accel(), o.accel()) < 1e-12
    n_enc = 0
    for k in range(6):
        g.step(1)
        g.sync()
        o.step(1)
        n_enc += check_step(g, o, nb, label=f"{name} step {k}")[0]
        mu_g, rc_g = g.masses()
        mu_o, rc_o = o.mu()
        assert np.allclose(mu_g, mu_o, rtol=1e-14, atol=0)
        xg, ug = g.get_dh()
        o.set_dh(xg, ug, o.step_index())      # same bits into the next step
    if name != "self_gravitating":
        assert n_enc > 0


def test_energy_matches_oracle(mx, orc):
    w = ic.self_gravitating(seed=1, n_pl=4, n_pls=900)
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    x, u = g.get_dh()
    o.set_dh(x, u, 0)
    E, L = g.energy()
    Eo, Lo = o.energy()
    assert abs(E - Eo) <= 1e-13 * abs(Eo)
    assert np.allclose(L, Lo, rtol=1e-13, atol=1e-13 * np.abs(Lo).max())


def test_energy_drift_matches_oracle(mx, orc):
    """Independent trajectories (no re-seeding) of the two-giant system."""
    w = ic.two_giants(seed=2, n_small=200)
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    x, u = g.get_dh()
    o.set_dh(x, u, 0)
    g.set_dh(x, u, 0)
    E0g, _ = g.energy()
    E0o, _ = o.energy()
    g.step(500)
    g.sync()
    o.step(500)
    Eg, _ = g.energy()
    Eo, _ = o.energy()
    dg = (Eg - E0g) / abs(E0g)
    do = (Eo - E0o) / abs(E0o)
    assert abs(dg - do) < 1e-10, (dg, do)


# ----------------------------------------------------- determinism, resume
def test_bitwise_deterministic_and_resumable(mx):
    w = ic.embryo_disk(seed=5, n_small=2000, n_emb=8)
    a = mx.System.from_workload(w)
    b = mx.System.from_workload(w)
    a.step(20)
    b.step(10)
    xb, ub = b.get_dh()
    c = mx.System.from_workload(w)
    c.set_dh(xb, ub, 10)
    c.step(10)
    b.step(10)
    xa, ua = a.get_dh()
    xb, ub = b.get_dh()
    xc, uc = c.get_dh()
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub)
    assert np.array_equal(xa, xc) and np.array_equal(ua, uc)
    assert a.step_index() == 20 and c.step_index() == 20


def test_joined_steps_equal_single_steps(mx):
    """A multi-step call joins the closing kernel of each step with the opening
    kernel of the next (one launch) and alternates the massive-body and list
    buffers between steps: the states, the last step's encounter list and the
    step count must equal those of one-step calls, bit for bit."""
    w = ic.embryo_disk(seed=7, n_small=3000, n_emb=6)
    a = mx.System.from_workload(w)
    b = mx.System.from_workload(w)
    a.step(9)
    for _ in range(9):
        b.step(1)
    xa, ua = a.get_dh()
    xb, ub = b.get_dh()
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub)
    assert np.array_equal(a.encounters(), b.encounters())
    assert a.step_index() == b.step_index() == 9
    assert a.energy()[0] == b.energy()[0]
    assert a.counters() == b.counters()


@pytest.mark.parametrize("name,kw,group", [
    ("embryo_disk", dict(seed=2, n_small=3000, n_emb=8), "bs"),
    ("self_gravitating", dict(seed=1, n_pl=4, n_pls=600), "force_kick"),
])
def test_launch_modes_give_identical_states(mx, name, kw, group):
    """Eager, graph, timed and profiled launches run the same kernels on the same
    data: identical states, and a positive time for every timed launch."""
    w = getattr(ic, name)(**kw)
    a = mx.System.from_workload(w)
    b = mx.System.from_workload(w)
    c = mx.System.from_workload(w)
    a.set_launch_mode("graph")
    a.step(12)
    c.step(12)
    ms, nl = b.step_timed(5, group)
    ms3, nl3 = b.step_timed(3, group, stride=2)
    prof = b.step_profiled(4)
    assert nl == 5 and len(ms) == 5 and min(ms) > 0.0
    assert nl3 == 2 and ms3[0] > 0.0 and ms3[1] == 0.0 and ms3[2] > 0.0
    assert set(prof) == set(mx.System.KERNELS)
    xa, ua = a.get_dh()
    xb, ub = b.get_dh()
    xc, uc = c.get_dh()
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub)
    assert np.array_equal(xa, xc) and np.array_equal(ua, uc)
    assert a.step_index() == b.step_index() == c.step_index() == 12
    f, npairs = b.counters()
    assert f >= 0 and npairs >= 0


@pytest.mark.parametrize("name,kw,joined", [
    ("embryo_disk", dict(seed=2, n_small=3000, n_emb=8), True),
    ("self_gravitating", dict(seed=1, n_pl=4, n_pls=600), False),
])
def test_joined_launch_timing(mx, name, kw, joined):
    """The joined-launch timing group: every timed step but the last of the call
    carries one joined launch on the fused path, none where steps are not joined
    (more than 64 massive bodies); the states equal plain eager steps."""
    w = getattr(ic, name)(**kw)
    a = mx.System.from_workload(w)
    b = mx.System.from_workload(w)
    a.step(7)
    ms, nl = b.step_timed(7, "step_joined", stride=2)  # steps 0, 2, 4, 6 timed
    assert len(ms) == 7
    if joined:
        assert nl == 3 and min(ms[0], ms[2], ms[4]) > 0.0
        assert ms[1] == ms[3] == ms[5] == ms[6] == 0.0
    else:
        assert nl == 0 and max(ms) == 0.0
    xa, ua = a.get_dh()
    xb, ub = b.get_dh()
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub)
    assert a.step_index() == b.step_index() == 7


def _joint_cases():
    return {
        "embryo_disk": lambda: ic.embryo_disk(seed=11, n_small=4000, n_emb=10),
        "close_planets": _close_planets_workload,
        "long_list": lambda: _planets_with_cloud(n_far=50, k=320, close_pair=False),
        "disk_model": _joint_disk_model,
    }


def _joint_disk_model():
    w = ic.embryo_disk(seed=4, n_small=2000, n_emb=6)
    w.params = dict(w.params, **DISK_MODES["all"])
    return w


@pytest.mark.parametrize("case", ["embryo_disk", "close_planets", "long_list", "disk_model"])
def test_joint_launches_equal_single_steps(mx, case):
    """A call of several steps on a single system with at most 64 massive bodies
    runs each step's encounter integrator in one launch with the closing of that
    step and the opening of the next.  Without a pair of massive bodies in an
    encounter the boundary is prepared and the integrator closes and opens its
    massless members itself (with more than 256 pairs, long_list, after the
    general plan); with such a pair (close_planets) the tile blocks wait for the
    integrator.  States, the last list, the step count and the counters must
    equal those of one-step calls bit for bit, over enough steps to cycle the
    three phases."""
    w = _joint_cases()[case]()
    a = mx.System.from_workload(w)
    b = mx.System.from_workload(w)
    n = 8
    a.step(n)
    for _ in range(n):
        b.step(1)
    xa, ua = a.get_dh()
    xb, ub = b.get_dh()
    print(f"[joint] {case}: {len(a.encounters())} pairs in the last step, "
          f"{a.counters()[1]} flagged in {n} steps", flush=True)
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub)
    assert np.array_equal(a.encounters(), b.encounters())
    assert a.step_index() == b.step_index() == n
    assert a.counters() == b.counters()
    assert a.energy()[0] == b.energy()[0]
    if case == "close_planets":
        saw = False
        c = mx.System.from_workload(w)
        for _ in range(n):
            c.step(1)
            e = c.encounters()
            saw |= bool(len(e)) and bool(np.any(e[:, 1] < w.params["n_big"]))
        assert saw
    if case == "long_list":
        assert a.counters()[1] > 256 * n // 2


def _bound_pair_disk(n_small=3000):
    """An embryo disk whose first two embryos form a bound pair well inside each
    other's changeover radius: an encounter between massive bodies in every step."""
    w = ic.embryo_disk(seed=3, n_small=n_small, n_emb=6)
    m = w.m_big
    x = w.x.copy()
    v = w.v.copy()
    rH = np.linalg.norm(x[:, 0]) * (m[0] / 3) ** (1 / 3)
    d = 0.3 * rH
    x[:, 1] = x[:, 0] + np.array([d, 0.0, 0.0])
    v[:, 1] = v[:, 0] + np.array([0.0, math.sqrt(G * (m[0] + m[1]) / d), 0.0])
    w.x, w.v = x, v
    return w


def test_joint_launches_pause_with_frequent_massive_pairs(mx):
    """Where massive bodies meet in most steps the joint launch waits for its
    integrator and is slower than two launches: after a synchronisation that sees
    more than a fifth of 32 or more joint launches wait, calls step with separate
    launches (same bits).  A fresh system starts with joint launches."""
    w = _bound_pair_disk()
    a = mx.System.from_workload(w)
    b = mx.System.from_workload(w)
    c = mx.System.from_workload(w)
    ms, nl = c.step_timed(6, "step_joint")
    assert nl == 5
    a.step(40)
    a.sync()
    ms, nl = a.step_timed(6, "step_joint")
    assert nl == 0
    a.step(10)
    for _ in range(56):
        b.step(1)
    e = b.encounters()
    assert len(e) and np.any(e[:, 1] < w.params["n_big"])
    xa, ua = a.get_dh()
    xb, ub = b.get_dh()
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub)
    assert a.step_index() == b.step_index() == 56


def test_joint_launch_timing(mx):
    """The joint-launch timing group times the launches of the sequence mx_step
    runs (one per step but the last); the states equal plain eager steps."""
    w = ic.embryo_disk(seed=2, n_small=3000, n_emb=8)
    a = mx.System.from_workload(w)
    b = mx.System.from_workload(w)
    a.step(7)
    ms, nl = b.step_timed(7, "step_joint", stride=2)  # steps 0, 2, 4, 6 timed
    assert nl == 3 and min(ms[0], ms[2], ms[4]) > 0.0
    assert ms[1] == ms[3] == ms[5] == ms[6] == 0.0
    xa, ua = a.get_dh()
    xb, ub = b.get_dh()
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub)
    assert a.step_index() == b.step_index() == 7


def test_heliocentric_roundtrip(mx, orc):
    w = ic.two_giants(seed=3, n_small=100)
    g = mx.System.from_workload(w)
    x, v = g.get_state()
    assert np.allclose(x, w.x, rtol=0, atol=0)
    assert relerr_rows(v, w.v) < 1e-14


# ----------------------------------------------------------------- errors
def test_error_paths(mx):
    w = ic.two_giants(seed=0, n_small=10)
    bad = dict(w.params, m0=-1.0)
    with pytest.raises(mx.MxError) as e:
        mx.System(bad, w.x, w.v, w.m_big)
    assert e.value.code == -1
    m = w.m_big.copy(); m[0] = 0.0
    with pytest.raises(mx.MxError) as e:
        mx.System(w.params, w.x, w.v, m)
    assert e.value.code == -1
    x = w.x.copy(); x[0, 5] = np.nan
    g = mx.System(w.params, x, w.v, w.m_big)
    g.step(1)
    with pytest.raises(mx.MxError) as e:
        g.sync()
    assert e.value.code in (-6, -4)


def _close_planets_workload(n_far=200):
    """Three planets, two of them inside each other's changeover radius, with a cloud
    of massless bodies around the pair: big-big components and shared copies."""
    return _planets_with_cloud(n_far, k=40, close_pair=True)


def _planets_with_cloud(n_far, k, close_pair):
    """Three planets (the second inside the first one's changeover radius when
    close_pair, else far out) with k massless bodies in a cloud of 0.6 Hill radii
    around the first and n_far massless bodies on near-circular orbits."""
    rng = np.random.default_rng(9)
    mJ = ic.M_JUP
    a_p = 5.2
    vp = math.sqrt(G * (1 + mJ) / a_p)
    rH = a_p * (mJ / 3) ** (1 / 3)
    m = np.array([mJ, 0.3 * mJ, 0.1 * mJ])
    xb = np.array([[a_p, a_p + 0.7 * rH, -8.0], [0.0, 0.15 * rH, 1.0], [0.0, 0.0, 0.01]])
    vb = np.array([[0.0, 0.0, -0.1 * vp * 0.5], [vp, vp * 1.002, -0.8 * vp * 0.6], [0.0, 1e-5, 0.0]])
    if not close_pair:
        xb[:, 1] = [-9.0, 2.0, 0.02]
        vb[:, 1] = [-0.2 * vp * 0.74, -0.97 * vp * 0.74, 0.0]
    d = rng.normal(0, 0.6 * rH, (3, k)); d[2] *= 0.1
    xs = xb[:, :1] + d
    vs = vb[:, :1] + rng.normal(0, 0.02 * vp, (3, k))
    a = rng.uniform(2.0, 12.0, n_far)
    xf, vf = ic.el2x(G, a, rng.uniform(0, 0.05, n_far), rng.uniform(0, 0.01, n_far),
                     rng.uniform(0, 6.28, n_far), rng.uniform(0, 6.28, n_far), rng.uniform(0, 6.28, n_far))
    x = np.hstack([xb, xs, xf]); v = np.hstack([vb, vs, vf])
    P = 2 * math.pi * math.sqrt(a_p ** 3 / (G * (1 + mJ)))
    p = ic.default_params(m0=1.0, dt=P / 400.0, n_big=3, n_small=k + n_far, gas_on=0)
    return ic.Workload("close_planets", p, x, v, m)


def test_step_parity_big_components(mx, orc):
    w = _close_planets_workload()
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    nb = w.params["n_big"]
    x, u = g.get_dh()
    o.set_dh(x, u, 0)
    g.set_dh(x, u, 0)
    saw_bigbig = False
    for k in range(4):
        x, u = g.get_dh()
        g.step(1)
        g.sync()
        xo, uo, sx, su = oracle_sensitivity(o, x, u, k)
        po = o.encounters()
        saw_bigbig |= bool(np.any(po[:, 1] < 3))
        check_step(g, o, nb, sx, su, label=f"big components step {k}")
    assert saw_bigbig


def test_step_parity_long_encounter_list(mx, orc):
    """More than 256 flagged pairs in a step of the fused path (no big-big pair):
    the encounter integrator's first block takes the general plan while the other
    blocks wait for it."""
    w = _planets_with_cloud(n_far=50, k=320, close_pair=False)
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    nb = w.params["n_big"]
    x, u = g.get_dh()
    o.set_dh(x, u, 0)
    g.set_dh(x, u, 0)
    longest = 0
    for k in range(2):
        x, u = g.get_dh()
        g.step(1)
        g.sync()
        xo, uo, sx, su = oracle_sensitivity(o, x, u, k)
        po = o.encounters()
        assert not np.any(po[:, 1] < 3)
        longest = max(longest, len(po))
        check_step(g, o, nb, sx, su, label=f"long list step {k}")
    assert longest > 256


def test_flag_kernel_large_list(mx, orc):
    """More flagged pairs than the planner keeps in LDS (global-scratch sort path)."""
    h = 20.0
    x0, u0, x1, u1 = _flag_inputs(orc, 77, 6, 6000, h, spread=0.02)
    rcrit = np.full(6, 0.25)
    po = orc.flag(6, rcrit, x0, u0, x1, u1, h)
    pg = mx.flag_pairs(6, rcrit, x0, u0, x1, u1, h)
    assert len(po) > 2048
    so, sg = {tuple(p) for p in po}, {tuple(p) for p in pg}
    for (i, j) in so ^ sg:
        ok, d = _flag_margin_ok(orc, x0, u0, x1, u1, i, j, rcrit[i], h)
        assert ok, (i, j, d)
    print(f"[parity] large flag list: {len(so)} pairs, {len(so ^ sg)} borderline")
    assert np.array_equal(pg, np.array(sorted(sg), dtype=np.int32).reshape(-1, 2))


def test_force_split_layout_full_size(mx, orc):
    """The 4,004-body self-gravitating case in the launch configuration the
    benchmark times (symmetric 64 x 64 tile pairs, one wave per workgroup): the
    stored end-of-step force against the oracle's direct sum, every body."""
    w = ic.self_gravitating(seed=0)
    g = mx.System.from_workload(w)
    x, u = g.get_dh()
    mu, rcrit = g.masses()
    a_g = g.accel()
    a_o = orc.gravity(x, mu, rcrit, w.params["n_big"])
    assert relerr_rows(a_g, a_o) < 1e-12
    g.step(1)
    g.sync()
    x1, _ = g.get_dh()
    mu1, rc1 = g.masses()
    assert relerr_rows(g.accel(), orc.gravity(x1, mu1, rc1, w.params["n_big"])) < 1e-12


def test_full_size_embryo_disk_step(mx, orc):
    """One step of the 100,000-body embryo disk (the benchmark workload) against
    the oracle on the same input state, every body."""
    w = ic.embryo_disk(seed=0)
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    x, u = g.get_dh()
    g.step(1)
    g.sync()
    xo, uo, sx, su = oracle_sensitivity(o, x, u, 0, trials=2)
    n_pairs, _, _ = check_step(g, o, w.params["n_big"], sx, su, label="embryo disk full size")
    assert n_pairs > 0


def test_culled_flagging_wide_disk_with_planted_pairs(mx, orc):
    """The all-massive encounter test that rejects whole chunk pairs by distance
    (bodies over 0.5-4 AU, so most chunk pairs are rejected), with close pairs of
    massive bodies planted at several distances: every pair the oracle flags is
    found, and each step matches the oracle from the same state."""
    w = ic.self_gravitating(seed=5, n_pl=4, n_pls=1500)
    nb = w.params["n_big"]
    g0 = mx.System.from_workload(w)
    _, rc = g0.masses()
    g0.close()
    rng = np.random.default_rng(5)
    order = np.argsort(np.linalg.norm(w.x[:, :nb], axis=0))
    for k in order[[40, 400, 800, 1200, 1480]]:   # partners at different distances
        j = int(rng.integers(4, nb))
        d = rng.normal(size=3)
        w.x[:, j] = w.x[:, k] + 0.4 * rc[k] * d / np.linalg.norm(d)
        w.v[:, j] = w.v[:, k] * (1.0 + 1e-4)
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    x, u = g.get_dh()
    o.set_dh(x, u, 0)
    g.set_dh(x, u, 0)
    pairs = 0
    for k in range(3):
        x, u = g.get_dh()
        g.step(1)
        g.sync()
        xo, uo, sx, su = oracle_sensitivity(o, x, u, k)
        pairs += check_step(g, o, nb, sx, su, label=f"culled flagging step {k}")[0]
    assert pairs >= 10


def test_deep_encounters_with_step_halvings(mx, orc):
    """Massless bodies aimed at an embryo with impact parameters of 0.3-3% of its
    changeover radius and slow approach: the encounter integrator has to halve its
    step repeatedly (the rounds that try eight step sizes at once must pick the
    step the sequential control would accept).  Several steps, each started from
    the same state on both sides, every body against the oracle within its own
    one-ulp sensitivity."""
    w = ic.embryo_disk(seed=8, n_small=200, n_emb=3)
    o = orc.OracleSystem.from_workload(w)
    rc = o.mu()[1].copy()
    o.close()
    nb = w.params["n_big"]
    rng = np.random.default_rng(8)
    h = w.params["dt"]
    for q, b in enumerate((0.003, 0.01, 0.03)):
        j = nb + q
        # start one step before closest approach, at impact parameter b rc
        vrel = 0.3 * rc[0] / h
        dirn = rng.normal(size=3)
        dirn /= np.linalg.norm(dirn)
        perp = np.cross(dirn, rng.normal(size=3))
        perp /= np.linalg.norm(perp)
        w.x[:, j] = w.x[:, 0] + b * rc[0] * perp - vrel * h * dirn
        w.v[:, j] = w.v[:, 0] + vrel * dirn
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    x, u = g.get_dh()
    flagged = 0
    for k in range(4):
        g.set_dh(x, u, k)
        g.step(1)
        g.sync()
        xo, uo, sx, su = oracle_sensitivity(o, x, u, k, trials=2)
        po = {tuple(p) for p in o.encounters()}
        flagged += sum(1 for (i, jj) in po if i == 0 and nb <= jj < nb + 3)
        check_step(g, o, nb, sx, su, label=f"deep encounters step {k}")
        x, u = g.get_dh()
    assert flagged >= 3


@pytest.mark.parametrize("nb,ns,close", [(96, 2000, 3), (200, 3000, 3), (600, 0, 4)])
def test_step_parity_crowded_annulus(mx, orc, nb, ns, close):
    """Many massive bodies with encounters every step, in the layouts the step
    takes above 64 massive bodies: 64 < n_big < 128 with massless bodies (wide
    kick layout), n_big >= 128 with massless bodies (split partial sums of the
    massless targets and their finish), and an all-massive system shaped like the
    self-gravitating disk with pairs of massive bodies in encounters (separate
    flagging, planning and integration kernels).  Four steps, each from the same
    state on both sides, every body against the oracle."""
    w = ic.crowded_annulus(seed=nb, n_big=nb, n_small=ns, close_pairs=close)
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    x, u = g.get_dh()
    o.set_dh(x, u, 0)
    g.set_dh(x, u, 0)
    assert relerr_rows(g.accel(), o.accel()) < 1e-12
    pairs = bigbig = 0
    for k in range(4):
        x, u = g.get_dh()
        g.step(1)
        g.sync()
        xo, uo, sx, su = oracle_sensitivity(o, x, u, k)
        po = o.encounters()
        bigbig += int(np.sum(po[:, 1] < nb)) if len(po) else 0
        pairs += check_step(g, o, nb, sx, su, label=f"crowded nb={nb} ns={ns} step {k}")[0]
    assert pairs > 20 and bigbig > 0


# ----------------------------------------------- disk model of Sect. 3.1 (Eqs. 2, 6, 10-12)
DISK_MODES = {
    "temperature": dict(temp_1au=280.0, temp_beta=0.5),
    "eta_eq6": dict(temp_1au=200.0, temp_beta=0.75, eta_mode=1),
    "gravity_edge": dict(dg_mode=1, r_in=1.3),
    "gravity_series": dict(dg_mode=1, gamma=0.8, r_c=15.0, r_in=0.6),
    "all": dict(temp_1au=250.0, temp_beta=0.6, eta_mode=1, dg_mode=1, gamma=1.2, r_c=20.0,
                r_in=0.9),
}


@pytest.mark.parametrize("mode", sorted(DISK_MODES))
def test_gas_kernel_disk_model_matches_oracle(mx, orc, mode):
    """Drag plus disk gravity of the general disk on the massless bodies, every body
    against the oracle."""
    w = ic.embryo_disk(seed=21, n_small=4000, n_emb=5)
    p = dict(w.params, **DISK_MODES[mode])
    o = orc.OracleSystem(p, w.x, w.v, w.m_big, w.r_p, w.rho_p)
    x, u = o.get_dh()
    mu, _ = o.mu()
    rho = w.rho_p * ic.RHO_UNIT
    a_o = orc.drag(p, x, u, mu, w.r_p, rho, p["n_big"])
    a_g = mx.gas_drag(p, x, u, mu, w.r_p, rho, p["n_big"]).cpu().numpy()
    nb = p["n_big"]
    assert np.all(a_g[:, :nb] == 0)
    assert np.any(a_o[:, nb:] != 0)
    assert relerr_rows(a_g[:, nb:], a_o[:, nb:]) < 1e-12


def test_step_parity_disk_model(mx, orc):
    """Whole steps with the temperature profile, eta(R), a tapered gamma != 1 disk with
    an inner edge and disk gravity; each step from the same state on both sides."""
    w = ic.embryo_disk(seed=22, n_small=3000, n_emb=6)
    w.params = dict(w.params, **DISK_MODES["all"])
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    nb = w.params["n_big"]
    x, u = g.get_dh()
    o.set_dh(x, u, 0)
    g.set_dh(x, u, 0)
    pairs = 0
    for k in range(5):
        x, u = g.get_dh()
        g.step(1)
        g.sync()
        xo, uo, sx, su = oracle_sensitivity(o, x, u, k)
        pairs += check_step(g, o, nb, sx, su, label=f"disk model step {k}")[0]
    assert pairs > 0
    with pytest.raises(mx.MxError) as e:
        mx.Adjoint(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, 2, 1)
    assert e.value.code == -1


# --------------------------------- time-dependent physics (Sects. 3.1-3.3, 3.6)
def _physics_workload():
    """Embryo disk in a gas disk where embryo 0 grows through both phases, opens a
    gap and migrates inward through both phases, fast enough that every law acts
    within a dozen steps, with the step switch armed just inside its orbit."""
    w = ic.embryo_disk(seed=31, n_small=3000, n_emb=4)
    dt = w.params["dt"]
    import oracle as _o
    o = _o.OracleSystem.from_workload(w)
    xh, vh = o.get_state()
    a0 = _o.x2el(ic.G * (1 + w.m_big[0]), xh[:, 0], vh[:, 0])[0]
    o.close()
    m0 = w.m_big[0]
    planets = [dict(M0=m0, Mc=4 * m0, tau_c=3 * dt, Mf=60 * m0, tau_g=5 * dt, R_I=2e-5,
                    da1=-0.04 * a0, tau1=4 * dt, da2=-0.03 * a0, tau2=6 * dt, gap_C=4.0),
               {}, dict(M0=w.m_big[2], Mc=2 * w.m_big[2], tau_c=6 * dt), {}]
    return w, planets, dict(a_switch=a0 * 0.975, a_min=0.6 * a0)


def test_step_parity_time_dependent_physics(mx, orc):
    """Growth (both phases), radii, gap, migration (both phases) and the step switch:
    each step from the same state on both sides (positions and velocities handed
    over, the time and the physics state kept by each side), every body, the
    masses, radii, time and step size against the oracle."""
    w, planets, sw = _physics_workload()
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    g.set_planet_physics(planets, **sw)
    o.set_physics(planets, **sw)
    nb = w.params["n_big"]
    x, u = g.get_dh()
    o.set_xu(x, u)
    switched_at = None
    rng = np.random.default_rng(0)
    for k in range(14):
        g.step(1)
        g.sync()
        # the oracle's own one-ulp sensitivity from copies of its whole state
        xs, us = o.get_dh()
        sx = np.zeros(w.n); su = np.zeros(w.n)
        ref = o.clone()
        ref.step(1)
        xr, ur = ref.get_dh()
        for _ in range(2):
            c = o.clone()
            c.set_xu(xs * (1 + rng.uniform(-2.2e-16, 2.2e-16, xs.shape)),
                     us * (1 + rng.uniform(-2.2e-16, 2.2e-16, us.shape)))
            c.step(1)
            xq, uq = c.get_dh()
            sx = np.maximum(sx, relerr_per_body(xq, xr))
            su = np.maximum(su, relerr_per_body(uq, ur))
            c.close()
        ref.close()
        o.step(1)
        check_step(g, o, nb, sx, su, label=f"physics step {k}")
        mu_g, rc_g = g.masses()
        mu_o, rc_o = o.mu()
        assert np.allclose(mu_g, mu_o, rtol=1e-14, atol=0), k
        assert np.allclose(rc_g, rc_o, rtol=1e-13, atol=0), k
        assert np.allclose(g.radii(), o.radii(), rtol=1e-12, atol=0), k
        tg, hg = g.time()
        assert abs(tg - o.time()) <= 1e-12 * abs(o.time()) and hg == o.step_size(), k
        if switched_at is None and hg != w.params["dt"]:
            switched_at = k
        xg, ug = g.get_dh()
        o.set_xu(xg, ug)
    assert mu_g[0] > 10 * w.m_big[0] * ic.G          # into the runaway phase
    assert switched_at is not None                    # the step switch happened
    # a restart puts the clock at step_index dt with the initial step
    x, u = g.get_dh()
    g.set_dh(x, u, 14)
    assert g.time() == (14 * w.params["dt"], w.params["dt"])


def test_physics_rejected_where_unsupported(mx):
    w = ic.crowded_annulus(seed=1, n_big=96, n_small=100, close_pairs=0)
    g = mx.System.from_workload(w)
    with pytest.raises(mx.MxError) as e:
        g.set_planet_physics([{}] * 96)
    assert e.value.code == -1
    b = mx.Batch.from_workloads([ic.embryo_disk(seed=2, n_small=100, n_emb=3)])
    with pytest.raises(mx.MxError):
        b.system(0).set_planet_physics([{}] * 3)


# ---------------------------------------------- body removal (Sect. 3.5, mce_cent)
def _removal_workload(seed=41, n_small=4000):
    """Embryo disk where a fifth of the massless bodies are unbound (heliocentric
    speed 1.2-2 times the escape speed), a tenth plunge towards the star (angular
    momentum cut so that q < r_cen for half of them) and one embryo is unbound."""
    w = ic.embryo_disk(seed=seed, n_small=n_small, n_emb=5)
    rng = np.random.default_rng(seed)
    nb = w.params["n_big"]
    idx = rng.permutation(np.arange(nb, w.n))
    unb, plunge = idx[: n_small // 5], idx[n_small // 5: n_small // 5 + n_small // 10]
    for t in unb:
        r = np.linalg.norm(w.x[:, t])
        vesc = math.sqrt(2 * G / r)
        w.v[:, t] *= rng.uniform(1.2, 2.0) * vesc / np.linalg.norm(w.v[:, t])
    for t in plunge:
        r = np.linalg.norm(w.x[:, t])
        rhat = w.x[:, t] / r
        vt = w.v[:, t] - (w.v[:, t] @ rhat) * rhat
        # mostly radial inward motion with a small tangential part
        w.v[:, t] = -0.6 * math.sqrt(G / r) * rhat + rng.uniform(0.002, 0.03) * vt
    w.v[:, 2] *= 1.6
    return w


def test_removal_and_compaction_match_oracle(mx, orc):
    """Every step: a removal check (statuses compared exactly), then each few steps a
    compaction (index maps compared exactly); the states, from the same input each
    step, against the oracle's; the smaller system steps on."""
    w = _removal_workload()
    g = mx.System.from_workload(w)
    o = orc.OracleSystem.from_workload(w)
    nb = w.params["n_big"]
    x, u = g.get_dh()
    o.set_xu(x, u)
    r_cen = 0.05
    removed = 0
    for k in range(8):
        eg = g.check_removal(r_cen)
        eo = o.check_removal(r_cen)
        assert eg == eo and np.array_equal(g.status(), o.status()), k
        if k % 3 == 1:
            kg, mg = g.compact()
            ko, mo = o.compact()
            assert kg == ko and np.array_equal(mg, mo), k
            removed += kg
            xs, us = g.get_dh()
            xo, uo = o.get_dh()
            assert np.array_equal(xs, xo) and np.array_equal(us, uo)   # the same survivors
            assert np.array_equal(g.accel(), o.accel()) or relerr_rows(g.accel(), o.accel()) < 1e-12
        g.step(1)
        g.sync()
        o.step(1)
        check_step(g, o, nb, label=f"removal step {k}")
        xg, ug = g.get_dh()
        o.set_xu(xg, ug)
    st = g.status()
    assert removed > 500 and st[2] == -3 and g.masses()[0][2] == 0.0
    assert np.any(st == -2) or removed > 0
    E, L = g.energy()
    assert np.isfinite(E)
