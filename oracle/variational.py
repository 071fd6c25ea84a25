"""Forward-mode variational equations of the hybrid step (TEST INFRASTRUCTURE ONLY).

A second, slow CPU implementation of the hybrid step in which every quantity
carries, next to its value, its derivatives with respect to a set of parameters
(dual numbers with a tangent axis).  The parameters are the masses of the
massive bodies and their initial heliocentric positions and velocities.  The
tangents are propagated through exactly the arithmetic of the step: the
democratic-heliocentric conversion (Sect. 2, mco_h2dh / mco_dh2h), the
changeover-weighted gravity (Sect. 2.1.3), the gas drag of Sect. 3.1 (Eqs. 1, 3,
4, 5, 7; the k switch of Eq. 7 taken on the value), the jumps by the
massive-body momentum, the Kepler drift and the Bulirsch-Stoer integration of
the encounter subsystems.  Every discrete decision (encounter flags, changeover
branch, drag regime, Bulirsch-Stoer acceptance) is taken on the values, so the
tangents are the derivatives of the map that the value run follows.

The Kepler drift follows the same textbook difference forms of Kepler's equation
as oracle.c (eccentric anomaly, hyperbolic anomaly, universal variable near
parabolic); the converged anomaly is given its tangent by differentiating the
solved equation (one Newton step in dual arithmetic from the converged value).
Encounter flags come from the C oracle (or_flag) evaluated on the values.

The changeover radii are functions of the initial masses and orbits; as in the
finite-difference protocol they are held fixed (no tangent).  Only tests may use
this module; it shares nothing with the HIP library.
"""
from __future__ import annotations

import math

import numpy as np

from . import flag as _c_flag

PI = math.pi


# ------------------------------------------------------------------ dual arrays
class D:
    """Array of values `v` (shape S) with tangents `d` (shape S + (T,))."""

    __slots__ = ("v", "d")
    __array_ufunc__ = None  # numpy arrays defer to the reflected operators below

    def __init__(self, v, d):
        self.v = np.asarray(v, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)

    @staticmethod
    def const(v, T):
        v = np.asarray(v, dtype=np.float64)
        return D(v, np.zeros(v.shape + (T,)))

    @property
    def T(self):
        return self.d.shape[-1]

    def __getitem__(self, k):
        return D(self.v[k], self.d[k])

    def __setitem__(self, k, val):
        val = lift(val, self.T)
        self.v[k] = val.v
        self.d[k] = val.d

    def copy(self):
        return D(self.v.copy(), self.d.copy())

    def __add__(self, o):
        o = lift(o, self.T)
        return D(self.v + o.v, self.d + o.d)

    __radd__ = __add__

    def __sub__(self, o):
        o = lift(o, self.T)
        return D(self.v - o.v, self.d - o.d)

    def __rsub__(self, o):
        return lift(o, self.T) - self

    def __neg__(self):
        return D(-self.v, -self.d)

    def __mul__(self, o):
        o = lift(o, self.T)
        return D(self.v * o.v, self.d * o.v[..., None] + o.d * self.v[..., None])

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = lift(o, self.T)
        q = self.v / o.v
        return D(q, (self.d - o.d * q[..., None]) / o.v[..., None])

    def __rtruediv__(self, o):
        return lift(o, self.T) / self


def lift(x, T):
    if isinstance(x, D):
        return x
    return D.const(x, T)


def chain(x, fv, dfv):
    return D(fv, x.d * np.asarray(dfv, dtype=np.float64)[..., None])


def sqrt(x):
    s = np.sqrt(x.v)
    return chain(x, s, 0.5 / s)


def sin(x):
    return chain(x, np.sin(x.v), np.cos(x.v))


def cos(x):
    return chain(x, np.cos(x.v), -np.sin(x.v))


def sinh(x):
    return chain(x, np.sinh(x.v), np.cosh(x.v))


def cosh(x):
    return chain(x, np.cosh(x.v), np.sinh(x.v))


def exp(x):
    e = np.exp(x.v)
    return chain(x, e, e)


def powc(x, p):
    """x ** p for a constant exponent p."""
    return chain(x, x.v ** p, p * x.v ** (p - 1.0))


def stack(parts):
    return D(np.stack([p.v for p in parts]), np.stack([p.d for p in parts]))


# ------------------------------------------------------------------ the step
class VarSystem:
    """Hybrid-step state with tangents.  x, u: D of shape [3, n] (DH)."""

    def __init__(self, params, x_h, v_h, m_big, r_p=None, rho_p=None):
        p = dict(params)
        self.p = p
        self.nb = nb = int(p["n_big"])
        self.n = n = nb + int(p["n_small"])
        self.T = T = 7 * nb
        self.G = p["G"]
        self.mu0 = p["G"] * p["m0"]
        x_h = np.asarray(x_h, dtype=np.float64)
        v_h = np.asarray(v_h, dtype=np.float64)
        m_big = np.asarray(m_big, dtype=np.float64)
        # parameter seeds: masses, then big x (coordinate-major), then big v
        m = D(m_big.copy(), np.zeros((nb, T)))
        xh = D(x_h.copy(), np.zeros((3, n, T)))
        vh = D(v_h.copy(), np.zeros((3, n, T)))
        for k in range(nb):
            m.d[k, k] = 1.0
            for c in range(3):
                xh.d[c, k, nb + c * nb + k] = 1.0
                vh.d[c, k, 4 * nb + c * nb + k] = 1.0
        self.mu = m * self.G
        # heliocentric -> DH: u = v - (sum m v) / (m0 + sum m), masses of big bodies
        mtot = self.mu0
        for k in range(nb):
            mtot = self.mu[k] + mtot
        self.x = xh.copy()
        u = vh.copy()
        for c in range(3):
            P = D.const(0.0, T)
            for k in range(nb):
                P = P + self.mu[k] * vh[c, k]
            V = P / mtot
            u[c] = vh[c] - D(np.broadcast_to(V.v, (n,)), np.broadcast_to(V.d, (n, T)))
        self.u = u
        # changeover radii from the values (held fixed)
        from . import x2el
        self.rcrit = np.zeros(nb)
        for k in range(nb):
            el = x2el(self.mu0 + self.mu.v[k], x_h[:, k], v_h[:, k])
            a = el[0]
            if not (a > 0.0) or not math.isfinite(a):
                a = float(np.linalg.norm(x_h[:, k]))
            self.rcrit[k] = p["rcrit_hill"] * a * np.cbrt(self.mu.v[k] / (3.0 * self.mu0))
        ns = n - nb
        self.r_p = np.zeros(ns) if r_p is None else np.asarray(r_p, dtype=np.float64)
        self.rho_p = (np.ones(ns) if rho_p is None else np.asarray(rho_p, dtype=np.float64)) \
            * p["rho_unit"]
        self.ag = self.gravity(self.x)

    # ---------------------------------------------------------------- forces
    def kfun(self, s2, rc):
        """changeover K of the direct-force listing (values only decide the branch)"""
        q = (sqrt(s2) - 0.1 * rc) / (0.9 * rc)
        return q * q * q * (10.0 + q * (-15.0 + 6.0 * q))

    def gravity(self, x):
        """a_t = sum over massive s != t of mu_s K/s^3 (x_s - x_t), ascending s."""
        n, nb, T = self.n, self.nb, self.T
        a = D.const(np.zeros((3, n)), T)
        for s in range(nb):
            d = [x[c, s:s + 1] - x[c] for c in range(3)]   # [n] each, x_s - x_t
            s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
            rct = np.zeros(n)
            rct[:nb] = self.rcrit
            rc = np.maximum(self.rcrit[s], rct)
            rc2 = rc * rc
            mask_self = np.arange(n) == s
            s2v = np.where(mask_self, 1.0, s2.v)
            s2 = D(s2v, np.where(mask_self[:, None], 0.0, s2.d))
            r = sqrt(s2)
            w = 1.0 / (s2 * r)
            # changeover branch on values
            inner = s2.v < rc2
            if inner.any():
                rcs = np.where(rc > 0, rc, 1.0)
                K = self.kfun(s2, rcs)
                K = D(np.where(s2.v <= 0.01 * rc2, 0.0, K.v),
                      np.where((s2.v <= 0.01 * rc2)[:, None], 0.0, K.d))
                wK = w * K
                w = D(np.where(inner, wK.v, w.v), np.where(inner[:, None], wK.d, w.d))
            w = D(np.where(mask_self, 0.0, w.v), np.where(mask_self[:, None], 0.0, w.d))
            f = w * self.mu[s:s + 1]
            for c in range(3):
                a[c] = a[c] + f * d[c]
        return a

    def momentum(self, u):
        T = self.T
        P = []
        for c in range(3):
            acc = D.const(0.0, T)
            for k in range(self.nb):
                acc = acc + self.mu[k] * u[c, k]
            P.append(acc)
        return P

    def drag(self, x, u):
        """Gas drag on the massless bodies (Sect. 3.1); zero for massive bodies."""
        p, n, nb, T = self.p, self.n, self.nb, self.T
        a = D.const(np.zeros((3, n)), T)
        if not p["gas_on"] or n == nb:
            return a
        mu0 = self.mu0
        P = self.momentum(u)
        sl = slice(nb, n)
        X, Y = x[0, sl], x[1, sl]
        R = sqrt(X * X + Y * Y)
        vk = sqrt(mu0 / R)
        om = vk / R
        hg = p["h_over_r"] * R
        cs = hg * om
        taper = 1.0
        if p["r_c"] > 0.0:
            taper = exp((1.0 / p["r_c"]) ** (2.0 - p["gamma"]) - powc(R / p["r_c"], 2.0 - p["gamma"]))
        sig = powc(R, -p["gamma"]) * (p["sigma1"] * p["rho_unit"] / p["au_cm"]) * taper
        rhog = sig / (math.sqrt(2.0 * PI) * hg)
        vg = vk * math.sqrt(1.0 - 2.0 * p["eta"])
        gx = -(vg * Y / R)
        gy = vg * X / R
        dvx = u[0, sl] + P[0] / mu0 - gx
        dvy = u[1, sl] + P[1] / mu0 - gy
        dvz = u[2, sl] + P[2] / mu0
        dv = sqrt(dvx * dvx + dvy * dvy + dvz * dvz)
        ma = dv / cs
        lam = p["mfp_coef"] / rhog
        nu = (1.0 / 3.0) * math.sqrt(8.0 / PI) * cs * lam
        re = 2.0 * D.const(self.r_p, T) * dv / nu
        k = np.where(re.v < 1.0e5, 0.4, 0.2)
        inner = 1.0 / (24.0 / re + 40.0 / (10.0 + re)) + 0.23 * ma
        cd = powc(inner, p["kdrag_exp"]) + 2.0 * (0.8 * k + ma) / (1.6 + ma)
        f = -(3.0 / 8.0) * (cd / D.const(self.r_p, T)) * (rhog / D.const(self.rho_p, T)) * dv
        ok = (R.v > 0.0) & (R.v >= p["r_in"]) & (sig.v > 0.0) & (dv.v > 0.0)
        for c, dvc in enumerate((dvx, dvy, dvz)):
            ac = f * dvc
            a[c, sl] = D(np.where(ok, ac.v, 0.0), np.where(ok[:, None], ac.d, 0.0))
        return a

    # ---------------------------------------------------------------- drift
    def drift_body(self, x0, v0, h):
        """Kepler drift of one body (D of shape [3] each) about mu0 over h."""
        mu = self.mu0
        T = self.T
        r0 = sqrt(x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2])
        vv = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2]
        sg = x0[0] * v0[0] + x0[1] * v0[1] + x0[2] * v0[2]
        alpha = 2.0 / r0 - vv / mu
        ar = float(alpha.v * r0.v)
        if ar > 1e-6:
            a = 1.0 / alpha
            nn = sqrt(mu * alpha * alpha * alpha)
            c = 1.0 - r0 * alpha
            s = sg * sqrt(alpha / mu)
            dm = nn * h
            E = _solve(lambda E: E - c.v * math.sin(E) + s.v * (1.0 - math.cos(E)) - dm.v,
                       lambda E: 1.0 - c.v * math.cos(E) + s.v * math.sin(E), dm.v - 2.0,
                       dm.v + 2.0, dm.v)
            Ed = D.const(E, T)
            F = Ed - c * sin(Ed) + s * (1.0 - cos(Ed)) - dm
            Fp = 1.0 - c.v * math.cos(E) + s.v * math.sin(E)
            Ed = D(E, -F.d / Fp)
            omc = 2.0 * sin(0.5 * Ed) * sin(0.5 * Ed)
            r = a * (1.0 - c * cos(Ed) + s * sin(Ed))
            f = 1.0 - (a / r0) * omc
            g = h - (Ed - sin(Ed)) / nn
            fd = -(sqrt(mu * a) * sin(Ed) / (r * r0))
            gd = 1.0 - (a / r) * omc
        elif ar < -1e-6:
            a = 1.0 / alpha
            nn = sqrt(-mu * alpha * alpha * alpha)
            c = 1.0 - r0 * alpha
            s = sg * sqrt(-alpha / mu)
            dn = nn * h

            def HF(H):
                return c.v * math.sinh(H) + s.v * (math.cosh(H) - 1.0) - H - dn.v

            if dn.v >= 0:
                lo, hi = 0.0, 1.0
                while HF(hi) < 0:
                    lo, hi = hi, 2.0 * hi
            else:
                lo, hi = -1.0, 0.0
                while HF(lo) > 0:
                    lo, hi = 2.0 * lo, lo
            H = _solve(HF, lambda H: c.v * math.cosh(H) + s.v * math.sinh(H) - 1.0, lo, hi,
                       0.5 * (lo + hi))
            Hd = D.const(H, T)
            F = c * sinh(Hd) + s * (cosh(Hd) - 1.0) - Hd - dn
            Fp = c.v * math.cosh(H) + s.v * math.sinh(H) - 1.0
            Hd = D(H, -F.d / Fp)
            chm1 = 2.0 * sinh(0.5 * Hd) * sinh(0.5 * Hd)
            r = a * (1.0 - c * cosh(Hd) - s * sinh(Hd))
            f = 1.0 + (a / r0) * chm1
            g = h - (sinh(Hd) - Hd) / nn
            fd = -(sqrt(-mu * a) * sinh(Hd) / (r * r0))
            gd = 1.0 + (a / r) * chm1
        else:
            beta = mu * alpha

            def UF(S):
                cc = _stumpff_val(beta.v * S * S)
                return (r0.v * S * cc[1] + sg.v * S * S * cc[2] + mu * S ** 3 * cc[3] - h,
                        r0.v * cc[0] + sg.v * S * cc[1] + mu * S * S * cc[2])

            if h >= 0:
                lo, hi = 0.0, h / r0.v
                while UF(hi)[0] < 0:
                    lo, hi = hi, 2.0 * hi
            else:
                lo, hi = h / r0.v, 0.0
                while UF(lo)[0] > 0:
                    lo, hi = 2.0 * lo, lo
            S = _solve(lambda S: UF(S)[0], lambda S: UF(S)[1], lo, hi, 0.5 * (lo + hi))
            Sd = D.const(S, T)
            cc = _stumpff_dual(beta * Sd * Sd)
            F = r0 * Sd * cc[1] + sg * Sd * Sd * cc[2] + mu * Sd * Sd * Sd * cc[3] - h
            Sd = D(S, -F.d / UF(S)[1])
            cc = _stumpff_dual(beta * Sd * Sd)
            G1, G2, G3 = Sd * cc[1], Sd * Sd * cc[2], Sd * Sd * Sd * cc[3]
            r = r0 * cc[0] + sg * G1 + mu * G2
            f = 1.0 - mu * G2 / r0
            g = h - mu * G3
            fd = -(mu * G1 / (r * r0))
            gd = 1.0 - mu * G2 / r
        x1 = [f * x0[c] + g * v0[c] for c in range(3)]
        v1 = [fd * x0[c] + gd * v0[c] for c in range(3)]
        return x1, v1

    # ---------------------------------------------------------------- BS
    def bs_force(self, xs, mu_m, rc_m, pl):
        m = len(xs)
        acc = []
        for k in range(m):
            p = xs[k]
            r2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2]
            r = sqrt(r2)
            f = -(self.mu0 / (r2 * r))
            acc.append([f * p[c] for c in range(3)])
        for a, b in pl:
            d = [xs[b][c] - xs[a][c] for c in range(3)]
            s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
            rc = max(rc_m[a], rc_m[b])
            # complementary part (1 - K) of the pair force: all of it inside
            # 0.1 rc, none of it outside rc
            if s2.v > 0.0 and s2.v < rc * rc:
                w = 1.0 / (s2 * sqrt(s2))
                if s2.v > 0.01 * rc * rc:
                    w = w * (1.0 - self.kfun(s2, rc))
            else:
                w = D.const(0.0, self.T)
            for c in range(3):
                acc[a][c] = acc[a][c] + mu_m[b] * w * d[c]
                acc[b][c] = acc[b][c] - mu_m[a] * w * d[c]
        return acc

    def stoermer(self, xs, vs, mu_m, rc_m, pl, H, nsub):
        dt = H / nsub
        m = len(xs)
        xo = [[xs[k][c] for c in range(3)] for k in range(m)]
        acc = self.bs_force(xo, mu_m, rc_m, pl)
        d = [[None] * 3 for _ in range(m)]
        for k in range(m):
            for c in range(3):
                d[k][c] = dt * (vs[k][c] + 0.5 * dt * acc[k][c])
                xo[k][c] = xo[k][c] + d[k][c]
        for _ in range(1, nsub):
            acc = self.bs_force(xo, mu_m, rc_m, pl)
            for k in range(m):
                for c in range(3):
                    d[k][c] = d[k][c] + dt * dt * acc[k][c]
                    xo[k][c] = xo[k][c] + d[k][c]
        acc = self.bs_force(xo, mu_m, rc_m, pl)
        vo = [[d[k][c] / dt + 0.5 * dt * acc[k][c] for c in range(3)] for k in range(m)]
        return xo, vo

    def bs(self, xs, vs, mu_m, rc_m, pl, h, tol):
        """Bulirsch-Stoer of one subsystem (Stoermer n = 2..16, Aitken-Neville in
        (H/n)^2, acceptance on values); xs, vs: lists of [3] D per member."""
        KMAX = 8
        m = len(xs)
        done, H, fails = 0.0, h, 0
        while abs(h - done) > 1e-14 * abs(h):
            rem = h - done
            if abs(H) > abs(rem):
                H = rem
            xsc = [1.0 / float(sum(xs[k][c].v ** 2 for c in range(3))) for k in range(m)]
            vsc = [1.0 / float(sum(vs[k][c].v ** 2 for c in range(3))) for k in range(m)]
            tab = []
            accepted = -1
            for k in range(KMAX):
                nk = 2 * (k + 1)
                xo, vo = self.stoermer(xs, vs, mu_m, rc_m, pl, H, nk)
                row = [[xo[b][c] for b in range(m) for c in range(3)] +
                       [vo[b][c] for b in range(m) for c in range(3)]]
                for j in range(1, k + 1):
                    ratio = nk / (2 * (k - j + 1))
                    den = ratio * ratio - 1.0
                    left, up = row[j - 1], tab[k - 1][j - 1]
                    row.append([left[i] + (left[i] - up[i]) / den for i in range(6 * m)])
                tab.append(row)
                if k >= 1:
                    best, prev = row[k], row[k - 1]
                    err = 0.0
                    for b in range(m):
                        for c in range(3):
                            ex = best[3 * b + c].v - prev[3 * b + c].v
                            ev = best[3 * m + 3 * b + c].v - prev[3 * m + 3 * b + c].v
                            err = max(err, ex * ex * xsc[b], ev * ev * vsc[b])
                    if err <= tol * tol:
                        accepted = k
                        break
            if accepted >= 0:
                best = tab[accepted][accepted]
                xs = [[best[3 * b + c] for c in range(3)] for b in range(m)]
                vs = [[best[3 * m + 3 * b + c] for c in range(3)] for b in range(m)]
                done += H
                fails = 0
                if accepted <= 4:
                    H = 2.0 * H
            else:
                H = 0.5 * H
                fails += 1
                if fails > 30:
                    raise RuntimeError("variational BS: halving limit")
        return xs, vs

    def subsystems(self, pairs):
        """Decomposition of the flagged pairs (the C oracle's rules): big-big
        components, then one subsystem per flagged small body with copies of the
        big components it touches.  Returns (members, local pairs, keep_from)."""
        nb = self.nb
        par = list(range(nb))

        def root(a):
            while par[a] != a:
                a = par[a]
            return a

        inbig = [False] * nb
        for i, j in pairs:
            if j < nb:
                ri, rj = root(i), root(j)
                if ri != rj:
                    if ri < rj:
                        par[rj] = ri
                    else:
                        par[ri] = rj
                inbig[i] = inbig[j] = True
        out = []
        for r in range(nb):
            if not inbig[r] or root(r) != r:
                continue
            mem = [b for b in range(nb) if inbig[b] and root(b) == r]
            pl = [(mem.index(i), mem.index(j)) for i, j in pairs if j < nb and root(i) == r]
            out.append((mem, pl, 0))
        smalls = sorted(set(j for i, j in pairs if j >= nb))
        for j in smalls:
            mem = []
            for i, jj in pairs:
                if jj != j:
                    continue
                r = root(i)
                for b in range(nb):
                    same = b == i or (inbig[i] and inbig[b] and root(b) == r)
                    if same and b not in mem:
                        mem.append(b)
            mem.sort()
            nbm = len(mem)
            pl = []
            for a, b in pairs:
                if b < nb:
                    if a in mem and b in mem:
                        pl.append((mem.index(a), mem.index(b)))
                elif b == j:
                    pl.append((mem.index(a), nbm))
            out.append((mem + [j], pl, nbm))
        return out

    # ---------------------------------------------------------------- step
    def half_kick(self, hh):
        ad = self.drag(self.x, self.u)
        for c in range(3):
            self.u[c] = self.u[c] + hh * (self.ag[c] + ad[c])

    def jump(self, hh):
        P = self.momentum(self.u)
        for c in range(3):
            dx = hh * P[c] / self.mu0
            self.x[c] = self.x[c] + D(np.broadcast_to(dx.v, (self.n,)),
                                      np.broadcast_to(dx.d, (self.n, self.T)))

    def step(self):
        n, nb, T = self.n, self.nb, self.T
        h = self.p["dt"]
        hh = 0.5 * h
        self.half_kick(hh)
        self.jump(hh)
        x0, u0 = self.x.copy(), self.u.copy()
        x1 = D.const(np.zeros((3, n)), T)
        u1 = D.const(np.zeros((3, n)), T)
        for t in range(n):
            xa, va = self.drift_body([x0[c, t] for c in range(3)], [u0[c, t] for c in range(3)], h)
            for c in range(3):
                x1[c, t] = xa[c]
                u1[c, t] = va[c]
        pairs = _c_flag(nb, self.rcrit, x0.v, u0.v, x1.v, u1.v, h)
        pairs = [(int(i), int(j)) for i, j in pairs]
        self.last_pairs = pairs
        mu_all = [self.mu[k] for k in range(nb)]
        for mem, pl, keep in self.subsystems(pairs):
            xs = [[x0[c, b] for c in range(3)] for b in mem]
            vs = [[u0[c, b] for c in range(3)] for b in mem]
            mu_m = [mu_all[b] if b < nb else D.const(0.0, T) for b in mem]
            rc_m = [self.rcrit[b] if b < nb else 0.0 for b in mem]
            xs, vs = self.bs(xs, vs, mu_m, rc_m, pl, h, self.p["bs_tol"])
            for k in range(keep, len(mem)):
                for c in range(3):
                    x1[c, mem[k]] = xs[k][c]
                    u1[c, mem[k]] = vs[k][c]
        self.x, self.u = x1, u1
        self.jump(hh)
        self.ag = self.gravity(self.x)
        self.half_kick(hh)

    def heliocentric(self):
        P = self.momentum(self.u)
        v = self.u.copy()
        for c in range(3):
            s = P[c] / self.mu0
            v[c] = self.u[c] + D(np.broadcast_to(s.v, (self.n,)),
                                 np.broadcast_to(s.d, (self.n, self.T)))
        return self.x.copy(), v


def eccentricity(x, v, gm):
    """|e| of every body from heliocentric x, v (D of shape [3, n])."""
    hx = x[1] * v[2] - x[2] * v[1]
    hy = x[2] * v[0] - x[0] * v[2]
    hz = x[0] * v[1] - x[1] * v[0]
    r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2])
    ex = (v[1] * hz - v[2] * hy) / gm - x[0] / r
    ey = (v[2] * hx - v[0] * hz) / gm - x[1] / r
    ez = (v[0] * hy - v[1] * hx) / gm - x[2] / r
    return sqrt(ex * ex + ey * ey + ez * ez)


def run(params, x_h, v_h, m_big, r_p, rho_p, n_steps):
    """Run n_steps; returns the system (with tangents w.r.t. masses, big x, big v)."""
    s = VarSystem(params, x_h, v_h, m_big, r_p, rho_p)
    for _ in range(n_steps):
        s.step()
    return s


def ecc_stats(s):
    """mean and variance of e over the massless bodies, heliocentric, gm = G m0."""
    x, v = s.heliocentric()
    e = eccentricity(x, v, s.mu0)[s.nb:]
    ns = e.v.shape[0]
    mean = D(e.v.mean(), e.d.mean(axis=0))
    dev = e - D(np.broadcast_to(mean.v, (ns,)), np.broadcast_to(mean.d, (ns, s.T)))
    sq = dev * dev
    var = D(sq.v.mean(), sq.d.mean(axis=0))
    return mean, var


# ------------------------------------------------------------------ helpers
def _solve(F, Fp, lo, hi, x):
    """Newton in a bisection bracket on a scalar equation (values only)."""
    for _ in range(200):
        f = F(x)
        if f == 0.0:
            return x
        if f < 0:
            lo = x
        else:
            hi = x
        xn = x - f / Fp(x)
        if abs(xn - x) <= 4 * 2.220446049250313e-16 * abs(xn):
            return xn
        if not (lo < xn < hi):
            xn = 0.5 * (lo + hi)
        if abs(xn - x) <= 4 * 2.220446049250313e-16 * abs(xn):
            return xn
        x = xn
    raise RuntimeError("variational Kepler: no convergence")


def _stumpff_val(z):
    if abs(z) < 0.5:
        out = []
        for k in range(4):
            term, ssum = 1.0 / math.factorial(k), 0.0
            for j in range(60):
                ssum += term
                term *= -z / ((2 * j + k + 1.0) * (2 * j + k + 2.0))
                if abs(term) < 1e-40:
                    break
            out.append(ssum)
        return out
    if z > 0:
        sz = math.sqrt(z)
        return [math.cos(sz), math.sin(sz) / sz, (1 - math.cos(sz)) / z, (sz - math.sin(sz)) / (z * sz)]
    sz = math.sqrt(-z)
    return [math.cosh(sz), math.sinh(sz) / sz, (math.cosh(sz) - 1) / (-z),
            (math.sinh(sz) - sz) / (-z * sz)]


def _stumpff_dual(z):
    """c0..c3 of a scalar dual z by their series (used near parabolic, |z| small)."""
    T = z.T
    out = []
    for k in range(4):
        term = D.const(1.0 / math.factorial(k), T)
        ssum = D.const(0.0, T)
        for j in range(40):
            ssum = ssum + term
            term = term * (-z) / ((2 * j + k + 1.0) * (2 * j + k + 2.0))
        out.append(ssum)
    return out
