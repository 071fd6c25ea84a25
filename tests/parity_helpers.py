"""Comparison helpers of the GPU parity tests (CPU-side numpy, no GPU calls).

Per step both paths start from the same state.  Positions and velocities must agree
to 1e-12 relative per body.  Encounter flags are integer decisions taken from
floating-point minima computed independently on each side (the oracle evaluates the
Hermite interpolant in its basis-function form, the GPU in monomial form): a pair may
be flagged on one side only when the oracle's deciding separation lies within what
the per-step position tolerance allows of the changeover radius.  The two positions
of a pair may each differ by 1e-12 of their distance from the star, so the separation
by at most 2e-12 max(|x_i|, |x_j|); the margin doubles that and adds 1e-12 rc for the
rounding of the minimum itself.  Bodies in such pairs are excluded from the per-body
comparison of that step (their integrator differs) and counted; if a pair of two
massive bodies is borderline, the whole step is skipped (every body feels them).
"""
import numpy as np

POS_TOL = 1e-12


def relerr_per_body(a, b):
    num = np.linalg.norm(a - b, axis=0)
    den = np.linalg.norm(b, axis=0)
    den = np.where(den > 0, den, 1.0)
    return num / den


def relerr_rows(a, b):
    """max over bodies of |a_t - b_t| / |b_t| (3-vectors per body)."""
    return float(relerr_per_body(a, b).max()) if a.size else 0.0


def borderline_margin(rc, xi, xj):
    """Largest |d_min - rc| at which the two sides may decide a pair differently."""
    return 4.0 * POS_TOL * max(np.linalg.norm(xi), np.linalg.norm(xj)) + 1e-12 * rc


def compare_pairs(o, pg, po, x_ref, nb):
    """Encounter lists of one step on the GPU (pg) and in the oracle o (po, its last
    step), x_ref the oracle's state after the step ([3][n]).  Asserts that every
    pair in one list only is borderline; returns (excluded bodies, number of
    borderline pairs, whether a massive pair was borderline)."""
    sg = {tuple(int(v) for v in p) for p in pg}
    so = {tuple(int(v) for v in p) for p in po}
    excluded, big_pair = set(), False
    for (i, j) in sorted(sg ^ so):
        d2, rc2 = o.last_pair_dmin2(i, j)
        rc = float(np.sqrt(rc2))
        gap = abs(float(np.sqrt(d2)) - rc)
        m = borderline_margin(rc, x_ref[:, i], x_ref[:, j])
        assert gap <= m, (f"pair {(i, j)} flagged on one side only "
                          f"({'gpu' if (i, j) in sg else 'oracle'}) with |d_min - rc| = {gap:.3e} "
                          f"> margin {m:.3e}")
        excluded.add(j)
        if j < nb:
            excluded.add(i)
            big_pair = True
    return excluded, len(sg ^ so), big_pair


def step_close(xg, ug, xo, uo, excluded, tol_x=POS_TOL, tol_u=POS_TOL):
    """Per-body relative errors of one step, the excluded bodies left out; tol_x and
    tol_u may be per-body arrays."""
    keep = np.ones(xo.shape[1], dtype=bool)
    if excluded:
        keep[sorted(excluded)] = False
    ex = relerr_per_body(xg, xo)
    eu = relerr_per_body(ug, uo)
    tx = np.broadcast_to(np.asarray(tol_x, dtype=float), ex.shape)
    tu = np.broadcast_to(np.asarray(tol_u, dtype=float), eu.shape)
    bad_x = np.nonzero(keep & (ex > tx))[0]
    bad_u = np.nonzero(keep & (eu > tu))[0]
    return (float(ex[keep].max()) if keep.any() else 0.0,
            float(eu[keep].max()) if keep.any() else 0.0, bad_x, bad_u)
