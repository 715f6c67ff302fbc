"""Independent global-grid restatement of the update, for pinning the oracle.

One periodic Cartesian grid, neighbours by np.roll, vectorised numpy: no
patches, no halos, no offsets.  It evaluates the same expressions as the
paper's scheme (Section 2 eqs. (2)-(5)) in the same operation order as the
oracle, so on a periodic grid the oracle's patch decomposition must agree with
it bit for bit.  Test-only code.
"""
import numpy as np


def _pressure(q, d, gamma):
    jj = q[1] * q[1]
    for k in range(1, d):
        jj = jj + q[1 + k] * q[1 + k]
    return (gamma - 1.0) * (q[d + 1] - 0.5 * jj / q[0])


def _flux(q, d, j, gamma):
    p = _pressure(q, d, gamma)
    jd = q[1 + j]
    f = [jd]
    for k in range(d):
        v = jd * q[1 + k] / q[0]
        if k == j:
            v = v + p
        f.append(v)
    f.append((q[d + 1] + p) * jd / q[0])
    return np.stack(f)


def _lam(q, d, j, gamma):
    p = _pressure(q, d, gamma)
    return np.abs(q[1 + j] / q[0]) + np.sqrt(gamma * p / q[0])


def _rusanov(L, R, d, j, gamma):
    fL, fR = _flux(L, d, j, gamma), _flux(R, d, j, gamma)
    lL, lR = _lam(L, d, j, gamma), _lam(R, d, j, gamma)
    a = np.where(np.isnan(lL), lL, np.where(np.isnan(lR), lR, np.where(lL > lR, lL, lR)))
    return 0.5 * ((fL + fR) - a * (R - L))


def step(q, d, dt, dx, gamma=1.4):
    """One periodic step of a global grid q[s][(Z,) Y, X] with cell widths dx[axis]."""
    out = q.copy()
    for j in range(d):
        ax = q.ndim - 1 - j  # x is the last array axis
        qm = np.roll(q, 1, axis=ax)
        qp = np.roll(q, -1, axis=ax)
        Fm = _rusanov(qm, q, d, j, gamma)
        Fp = _rusanov(q, qp, d, j, gamma)
        r = dt / dx[j]
        out = out - r * (Fp - Fm)
    return out
