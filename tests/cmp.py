"""Comparison helpers of the parity tests (GPU result against the oracle).

normwise(g, o): max over fields of max|g - o| / max|o| (the normwise
reading of "1e-12 relative").

Per-cell figures, for the positive fields (D, E, rho, P, eps), where
low-density and atmosphere cells would hide behind the stellar scale in a
normwise figure:

percell(g, o, comps): |g - o| / |o| per cell (cells whose oracle value lies
more than `floor`, 20 decades by default, below the field's largest value
are measured against that floor).  For quantities computed from identical
inputs by well-conditioned arithmetic (the recovered rho).

percell_local(g, o, comps, radius): |g - o| / max|o| over the cells within
`radius` cells (a square).  A stage output is a sum of the cell's old value
and flux differences of its stencil; next to the stellar surface an
atmosphere-level D or E is the difference of stellar-level fluxes, so its
rounding is that of the largest value the stencil reaches.  radius = 3 per
Runge-Kutta stage between the common input and the compared output (the
reach of the 6-point stencil); far from such neighbours this is a plain
per-cell relative figure.  The fluxes of D and E are bounded by the
neighbouring D and E (|v| < 1, P < E), so the neighbourhood maximum bounds
every term.

percell_cond(gp, op, oq, comps): recovered P and eps per cell, measured
against max(1, kappa 1e-2) |o| with kappa = (E/D)^2 / eps.  eps is the
difference of terms of order (E/D) w <= (E/D)^2 evaluated at the root z,
which the solvers find to a relative tolerance of 1e-15: both the rounding
and the root tolerance move eps by up to ~(E/D)^2 1e-15 absolute, so the
bar 1e-12 max(1, kappa 1e-2) leaves a factor 10 above that; for
well-conditioned cells (kappa <= 100) it is the plain per-cell figure.

All return a float that also carries where the worst cell is.
"""
import numpy as np
from scipy.ndimage import maximum_filter


class Err(float):
    """An error figure that also remembers where it is largest."""
    where = ""

    def __repr__(self):
        return "%.3e at %s" % (float(self), self.where)


def _mark(worst, where):
    e = Err(worst)
    e.where = where
    return e


def normwise(g, o, comps=None):
    comps = range(g.shape[0]) if comps is None else comps
    worst, where = 0.0, ""
    for c in comps:
        scale = np.abs(o[c]).max()
        d = np.abs(g[c] - o[c])
        err = d.max() if scale == 0.0 else d.max() / scale
        if err > worst or not where:
            idx = np.unravel_index(np.argmax(d), d.shape)
            worst, where = err, "field %d index %s (gpu %r, oracle %r)" % (
                c, tuple(int(i) for i in idx), float(g[c][idx]), float(o[c][idx]))
    return _mark(worst, where)


def percell(g, o, comps, floor=1e-20):
    worst, where = 0.0, ""
    for c in comps:
        den = np.maximum(np.abs(o[c]), floor * np.abs(o[c]).max())
        den = np.where(den > 0.0, den, 1.0)
        r = np.abs(g[c] - o[c]) / den
        m = float(r.max())
        if m > worst or not where:
            idx = np.unravel_index(np.argmax(r), r.shape)
            worst, where = m, "field %d index %s (gpu %r, oracle %r)" % (
                c, tuple(int(i) for i in idx), float(g[c][idx]), float(o[c][idx]))
    return _mark(worst, where)


def percell_local(g, o, comps, radius=3):
    worst, where = 0.0, ""
    for c in comps:
        a = np.abs(o[c])
        den = maximum_filter(a, size=2 * radius + 1, mode="nearest") if radius > 0 else a
        den = np.where(den > 0.0, den, 1.0)
        r = np.abs(g[c] - o[c]) / den
        m = float(r.max())
        if m > worst or not where:
            idx = np.unravel_index(np.argmax(r), r.shape)
            worst, where = m, "field %d index %s (gpu %r, oracle %r, local scale %r)" % (
                c, tuple(int(i) for i in idx), float(g[c][idx]), float(o[c][idx]), float(den[idx]))
    return _mark(worst, where)


def percell_cond(gp, op, oq, comps=(4, 5)):
    """gp, op: primitives (6 fields); oq: the conserved state they were
    recovered from (D = oq[0], E = oq[4])."""
    with np.errstate(divide="ignore", invalid="ignore"):
        kappa = (oq[4] / oq[0]) ** 2 / np.abs(op[5])
    kappa = np.where(np.isfinite(kappa), kappa, np.inf)
    worst, where = 0.0, ""
    for c in comps:
        with np.errstate(invalid="ignore"):
            den = np.abs(op[c]) * np.maximum(1.0, kappa * 1e-2)
        den = np.where(np.isnan(den), np.inf, den)       # 0 * inf: eps = 0, no figure
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(gp[c] == op[c], 0.0, np.abs(gp[c] - op[c]) / np.where(den > 0.0, den, 1.0))
        m = float(r.max())
        if m > worst or not where:
            idx = np.unravel_index(np.argmax(r), r.shape)
            worst, where = m, "field %d index %s (gpu %r, oracle %r, kappa %.3g)" % (
                c, tuple(int(i) for i in idx), float(gp[c][idx]), float(op[c][idx]), float(kappa[idx]))
    return _mark(worst, where)
