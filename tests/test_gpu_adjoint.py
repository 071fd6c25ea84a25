"""Adjoint of the hybrid step on the GPU (reverse mode through the C ABI), checked
against the oracle's forward-mode variational equations and against central
finite differences of the GPU forward run with the changeover radii held fixed.
"""
import numpy as np
import pytest

from synth import ic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_16791_amd as m
    m.lib()
    return m


def encounter_workload(seed=3, n_small=10, n_emb=2):
    """Tiny embryo disk with three massless bodies inside the first embryo's
    changeover zone (encounters through Bulirsch-Stoer in the first steps)."""
    import oracle
    w = ic.embryo_disk(seed=seed, n_small=n_small, n_emb=n_emb)
    o = oracle.OracleSystem.from_workload(w)
    rc = o.mu()[1].copy()
    o.close()
    rng = np.random.default_rng(seed)
    for q, frac in enumerate((0.35, 0.6, 0.8)):
        j = n_emb + q
        d = rng.normal(size=3)
        d *= frac * rc[0] / np.linalg.norm(d)
        w.x[:, j] = w.x[:, 0] + d
        w.v[:, j] = w.v[:, 0] + 1e-3 * np.linalg.norm(w.v[:, 0]) * rng.normal(size=3)
    return w


def theta_grad(gm, g_x, g_v, nb):
    return np.concatenate([gm, g_x[:, :nb].reshape(-1), g_v[:, :nb].reshape(-1)])


@pytest.mark.parametrize("case", ["encounters", "smooth"])
def test_adjoint_matches_oracle_variational(mx, orc, case):
    from oracle import variational as var
    if case == "encounters":
        w, steps, every = encounter_workload(), 6, 4
    else:
        w, steps, every = ic.embryo_disk(seed=31, n_small=20, n_emb=3), 7, 3
    nb, n = w.params["n_big"], w.n
    a = mx.Adjoint(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, steps, every)
    xf, vf = a.forward()
    xf, vf = xf.cpu().numpy(), vf.cpu().numpy()
    rng = np.random.default_rng(7)
    gx, gv = rng.normal(size=(3, n)), rng.normal(size=(3, n)) * 100.0
    gm, g_x, g_v = (t.cpu().numpy() for t in a.backward(gx, gv))
    a.close()
    s = var.run(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, steps)
    x, v = s.heliocentric()
    assert np.abs(xf - x.v).max() <= 1e-10 * np.abs(x.v).max()
    ref = np.einsum("cn,cnt->t", gx, x.d) + np.einsum("cn,cnt->t", gv, v.d)
    got = theta_grad(gm, g_x, g_v, nb)
    # masses, positions, velocities: each block against its own scale
    for lo, hi in ((0, nb), (nb, 4 * nb), (4 * nb, 7 * nb)):
        err = np.abs(got[lo:hi] - ref[lo:hi]).max()
        assert err <= 1e-8 * np.abs(ref[lo:hi]).max(), (case, lo, err, ref[lo:hi], got[lo:hi])


def gpu_loss(mx, w, m, xb, vb, steps, every, rcrit):
    """mean(e) + var(e) of the massless bodies after `steps`, GPU forward run."""
    x, v = w.x.copy(), w.v.copy()
    nb = w.params["n_big"]
    x[:, :nb], v[:, :nb] = xb, vb
    a = mx.Adjoint(w.params, x, v, m, w.r_p, w.rho_p, steps, every, rcrit=rcrit)
    xf, vf = a.forward()
    a.close()
    e = ecc(xf.cpu().numpy(), vf.cpu().numpy())[nb:]
    return e.mean() + e.var()


def ecc(x, v):
    h = np.cross(x.T, v.T)
    r = np.linalg.norm(x, axis=0)
    ev = np.cross(v.T, h) / ic.G - (x / r).T
    return np.linalg.norm(ev, axis=1)


def test_hybrid_run_gradient_matches_finite_differences(mx):
    torch = pytest.importorskip("torch")
    w = ic.embryo_disk(seed=41, n_small=600, n_emb=3)
    steps, every = 30, 8
    nb = w.params["n_big"]
    probe = mx.Adjoint(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, 1, 1)
    rcrit = probe.rcrit()
    probe.close()
    spec = dict(params=w.params, x=w.x, v=w.v, r_p=w.r_p, rho_p=w.rho_p, n_steps=steps,
                checkpoint_every=every, rcrit=rcrit)
    dev = "cuda"
    m = torch.tensor(w.m_big, dtype=torch.float64, device=dev, requires_grad=True)
    xb = torch.tensor(w.x[:, :nb], dtype=torch.float64, device=dev, requires_grad=True)
    vb = torch.tensor(w.v[:, :nb], dtype=torch.float64, device=dev, requires_grad=True)
    xf, vf = mx.hybrid_run(m, xb, vb, spec)
    h = torch.linalg.cross(xf.T, vf.T)
    r = torch.linalg.norm(xf, dim=0)
    ev = torch.linalg.cross(vf.T, h) / ic.G - (xf / r).T
    e = torch.linalg.norm(ev, dim=1)[nb:]
    loss = e.mean() + e.var(unbiased=False)
    loss.backward()
    assert np.isclose(loss.item(), gpu_loss(mx, w, w.m_big, w.x[:, :nb], w.v[:, :nb], steps,
                                            every, rcrit), rtol=1e-13)
    gm, gx, gvv = m.grad.cpu().numpy(), xb.grad.cpu().numpy(), vb.grad.cpu().numpy()
    base = (w.m_big, w.x[:, :nb], w.v[:, :nb])
    checks = [("m", 0, None), ("m", 2, None), ("x", 1, 0), ("x", 0, 2), ("v", 2, 1), ("v", 0, 0)]
    for kind, k, c in checks:
        if kind == "m":
            hs = 1e-3 * w.m_big[k]
        elif kind == "x":
            hs = 1e-6 * np.linalg.norm(w.x[:, k])
        else:
            hs = 1e-6 * np.linalg.norm(w.v[:, k])

        def at(d):
            mm, xx, vv = (b.copy() for b in base)
            if kind == "m":
                mm[k] += d
            elif kind == "x":
                xx[c, k] += d
            else:
                vv[c, k] += d
            return gpu_loss(mx, w, mm, xx, vv, steps, every, rcrit)

        fd = (-at(2 * hs) + 8 * at(hs) - 8 * at(-hs) + at(-2 * hs)) / (12 * hs)
        g = gm[k] if kind == "m" else (gx[c, k] if kind == "x" else gvv[c, k])
        # rounding of the loss (a few ulp of ~1e-2 in each run) divided by the step
        noise = 20 * 2.2e-16 * abs(loss.item()) / hs
        assert abs(g - fd) <= 2e-5 * abs(fd) + noise, (kind, k, c, g, fd, noise)


def test_adjoint_checkpointing_does_not_change_the_gradient(mx):
    w = encounter_workload(seed=5, n_small=40, n_emb=3)
    steps = 9
    rng = np.random.default_rng(1)
    gx, gv = rng.normal(size=(3, w.n)), rng.normal(size=(3, w.n))
    outs = []
    for every in (1, 4, 9):
        a = mx.Adjoint(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, steps, every)
        xf, vf = a.forward()
        g = [t.cpu().numpy() for t in a.backward(gx, gv)]
        a.close()
        outs.append((xf.cpu().numpy(), g))
    for xf, g in outs[1:]:
        assert np.array_equal(xf, outs[0][0])
        for p, q in zip(g, outs[0][1]):
            assert np.array_equal(p, q)


def test_adjoint_backward_repeats_bitwise(mx):
    """Two reverse passes of one adjoint, and one of a second adjoint built the same
    way, give the same bits: the reductions leave their block counter at zero and
    the encounter subsystems' member marks are cleared after every step."""
    w = encounter_workload(seed=8, n_small=80, n_emb=3)
    steps, every = 8, 3
    rng = np.random.default_rng(4)
    gx, gv = rng.normal(size=(3, w.n)), rng.normal(size=(3, w.n)) * 10.0
    runs = []
    a = mx.Adjoint(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, steps, every)
    a.forward()
    for _ in range(2):
        runs.append([t.cpu().numpy() for t in a.backward(gx, gv)])
    a.close()
    b = mx.Adjoint(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, steps, every)
    b.forward()
    runs.append([t.cpu().numpy() for t in b.backward(gx, gv)])
    b.close()
    for g in runs[1:]:
        for p, q in zip(g, runs[0]):
            assert np.array_equal(p, q)
    assert all(np.isfinite(p).all() for p in runs[0])


def test_adjoint_many_massive_bodies(mx):
    """40 massive bodies and 2,000 massless ones: 166 columns in the kick's
    reductions, 40 waves summing the encounter contributions, the massive momentum
    summed over 40 lanes.  The adjoint of a linear functional of the final state
    matches central differences of the GPU forward run (changeover radii held
    fixed) for masses, positions and velocities of the first, a middle and the last
    massive body, and checkpointing does not change it."""
    w = ic.embryo_disk(seed=17, n_small=2000, n_emb=40)
    nb, n = w.params["n_big"], w.n
    steps = 12
    probe = mx.Adjoint(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, 1, 1)
    rcrit = probe.rcrit()
    probe.close()
    rng = np.random.default_rng(23)
    gx, gv = rng.normal(size=(3, n)), rng.normal(size=(3, n)) * 50.0

    def grads(every):
        a = mx.Adjoint(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, steps, every, rcrit=rcrit)
        a.forward()
        g = [t.cpu().numpy() for t in a.backward(gx, gv)]
        a.close()
        return g

    def value(m, x, v):
        a = mx.Adjoint(w.params, x, v, m, w.r_p, w.rho_p, steps, steps, rcrit=rcrit)
        xf, vf = (t.cpu().numpy() for t in a.forward())
        a.close()
        return float(np.sum(gx * xf) + np.sum(gv * vf))

    g5 = grads(5)
    for p, q in zip(grads(1), g5):
        assert np.array_equal(p, q)
    gm, g_x, g_v = g5
    assert np.isfinite(gm).all() and np.isfinite(g_x).all() and np.isfinite(g_v).all()
    checks = [("m", 0, None), ("m", nb - 1, None), ("x", 20, 1), ("x", nb - 1, 0),
              ("v", 0, 2), ("v", nb - 1, 1)]
    for kind, k, c in checks:
        if kind == "m":
            hs = 1e-3 * w.m_big[k]
        elif kind == "x":
            hs = 1e-6 * np.linalg.norm(w.x[:, k])
        else:
            hs = 1e-6 * np.linalg.norm(w.v[:, k])

        def at(d):
            m, x, v = w.m_big.copy(), w.x.copy(), w.v.copy()
            if kind == "m":
                m[k] += d
            elif kind == "x":
                x[c, k] += d
            else:
                v[c, k] += d
            return value(m, x, v)

        fd = (-at(2 * hs) + 8 * at(hs) - 8 * at(-hs) + at(-2 * hs)) / (12 * hs)
        g = gm[k] if kind == "m" else (g_x[c, k] if kind == "x" else g_v[c, k])
        # measured: relative differences of 2e-8 .. 1.5e-7 (the stencil's truncation
        # and the rounding of the functional over 12 steps)
        assert abs(g - fd) <= 1e-5 * abs(fd), (kind, k, c, g, fd)


def test_hybrid_run_default_rcrit_is_a_constant_of_the_map(mx):
    """Without spec['rcrit'] the changeover radii come from the base state (spec's x,
    v and m_big), not from the differentiated inputs: the run and its gradient are
    those of the explicit-radius path bit for bit, on a system with bodies inside a
    changeover zone, and the mass gradient matches central differences of the GPU
    forward run with those radii frozen."""
    torch = pytest.importorskip("torch")
    w = encounter_workload(seed=6, n_small=60, n_emb=3)
    steps, every = 5, 2
    nb = w.params["n_big"]
    probe = mx.Adjoint(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, 1, 1)
    rcrit = probe.rcrit()
    probe.close()
    base = dict(params=w.params, x=w.x, v=w.v, r_p=w.r_p, rho_p=w.rho_p, n_steps=steps,
                checkpoint_every=every)
    grads, losses = [], []
    for spec in (dict(base, m_big=w.m_big), dict(base, rcrit=rcrit)):
        m = torch.tensor(w.m_big * 1.01, dtype=torch.float64, device="cuda", requires_grad=True)
        xb = torch.tensor(w.x[:, :nb], dtype=torch.float64, device="cuda", requires_grad=True)
        vb = torch.tensor(w.v[:, :nb], dtype=torch.float64, device="cuda", requires_grad=True)
        xf, vf = mx.hybrid_run(m, xb, vb, spec)
        h = torch.linalg.cross(xf.T, vf.T)
        r = torch.linalg.norm(xf, dim=0)
        e = torch.linalg.norm(torch.linalg.cross(vf.T, h) / ic.G - (xf / r).T, dim=1)[nb:]
        loss = e.mean() + e.var(unbiased=False)
        loss.backward()
        losses.append(loss.item())
        grads.append([t.grad.cpu().numpy() for t in (m, xb, vb)])
    assert losses[0] == losses[1]
    for p, q in zip(grads[0], grads[1]):
        assert np.array_equal(p, q)
    with pytest.raises(ValueError):
        mx.hybrid_run(m, xb, vb, base)
    mm0 = w.m_big * 1.01
    for k in range(nb):
        hs = 1e-4 * mm0[k]

        def at(d):
            mm = mm0.copy()
            mm[k] += d
            return gpu_loss(mx, w, mm, w.x[:, :nb], w.v[:, :nb], steps, every, rcrit)

        fd = (-at(2 * hs) + 8 * at(hs) - 8 * at(-hs) + at(-2 * hs)) / (12 * hs)
        noise = 20 * 2.2e-16 * abs(losses[0]) / hs
        assert abs(grads[0][0][k] - fd) <= 1e-4 * abs(fd) + noise, (k, grads[0][0][k], fd)
