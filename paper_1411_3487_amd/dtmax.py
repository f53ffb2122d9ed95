"""Decision rules of the largest-time-step test of Sec. V.B (Table 1).

The paper finds the largest usable time step of the mode scheme for a chain
length in two groups of tests, both on the same observables Q: the
autocorrelation of the end-to-end vector, that of the middle bond, and the
mean square displacement of the middle bead about the centre of mass.

* Equilibrium group: the equilibrium values Q(0) at a time step, divided by
  their Monte Carlo values, must all lie within 5 % of one.
* Dynamical group: at a few fixed times tau, the effective decay constant
  Q~(tau) = (1/Q) dQ/dtau (a numerical derivative) at a time step, divided by
  its value at the smallest time step, must lie within 10 % of one.  Data
  that noise dominates are left out.

The final value for the length is the smaller of the two groups' results.

Readings where the paper leaves the rule open:

* The largest time step of a group is the largest one of the contiguous run
  of passing steps that starts at the smallest tested step; a pass above a
  failure does not count, and if the smallest step already fails the group
  gives no value (None).
* The derivative is a central difference of ln Q on the sampled lag grid
  (power-of-two multiples of the sampling interval), at the lag nearest the
  requested time; an autocorrelation that at that lag has fallen below 5 %
  of its value at lag 0 in the reference run is taken as noise and skipped.

Pure numpy: no simulation arithmetic, used by the benchmark harness.
"""
from __future__ import annotations

import numpy as np

Q0_TOL = 0.05
QT_TOL = 0.10
DECAYED = 0.05


def contiguous_dtau_max(dtaus, passes):
    """Largest time step of the passing run that starts at the smallest
    tested step, or None if the smallest one fails."""
    order = np.argsort(np.asarray(dtaus, dtype=float), kind="stable")
    best = None
    for i in order:
        if not passes[i]:
            break
        best = float(dtaus[i])
    return best


def q0_passes(ratios, tol=Q0_TOL):
    """Equilibrium group: every ratio to the Monte Carlo value within tol."""
    return bool(all(abs(float(r) - 1.0) <= tol for r in ratios))


def decay_constant(q, lags, t):
    """Q~ = d ln Q / d tau at the lag nearest t, by a central difference over
    the neighbouring lags of the grid.  Returns (value, lag used); value is
    None where Q is not positive at both neighbours."""
    q = np.asarray(q, dtype=float)
    lags = np.asarray(lags, dtype=float)
    j = int(np.argmin(np.abs(lags - t)))
    j = min(max(j, 1), len(lags) - 2)
    lo, hi = q[j - 1], q[j + 1]
    if not (lo > 0 and hi > 0):
        return None, float(lags[j])
    return float((np.log(hi) - np.log(lo)) / (lags[j + 1] - lags[j - 1])), float(lags[j])


def qt_ratios(curve, ref, lags, times, names, autocorr=None, tol=QT_TOL, decayed=DECAYED):
    """Dynamical group at one time step.

    curve, ref: (n_lags, n_obs) arrays of Q at the lags, for this time step
    and for the smallest one; names: the n_obs observable names; autocorr:
    per observable, True for an autocorrelation (subject to the noise cut),
    default all but the last.  Returns (ratios {"name@lag": ratio}, ok),
    ok = every kept ratio within tol of one (True if nothing is kept)."""
    curve = np.asarray(curve, dtype=float)
    ref = np.asarray(ref, dtype=float)
    lags = np.asarray(lags, dtype=float)
    if autocorr is None:
        autocorr = [i < len(names) - 1 for i in range(len(names))]
    ratios, ok = {}, True
    for i, name in enumerate(names):
        for t in times:
            j = int(np.argmin(np.abs(lags - t)))
            if autocorr[i] and ref[j, i] < decayed * ref[0, i]:
                continue
            qa, tt = decay_constant(curve[:, i], lags, t)
            qb, _ = decay_constant(ref[:, i], lags, t)
            if qa is None or qb is None or qb == 0:
                continue
            r = qa / qb
            ratios[f"{name}@{tt:g}"] = r
            ok = ok and abs(r - 1.0) <= tol
    return ratios, bool(ok)
