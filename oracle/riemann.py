"""Exact solution of the Riemann problem for the 1-D Euler equations (ideal gas).

TEST INFRASTRUCTURE: used to pin the oracle (and through it the GPU path) on
the shock-tube workload.  The paper only states the PDE (Section 2, eq. (2));
the exact Riemann solution is the textbook one (Toro, "Riemann Solvers and
Numerical Methods for Fluid Dynamics", ch. 4): the star-region pressure is the
root of the pressure function f_L(p) + f_R(p) + (u_R - u_L) = 0, each f_K being
the shock (Rankine-Hugoniot) branch for p > p_K and the isentropic rarefaction
branch otherwise; the solution is then sampled along x/t.
"""
import numpy as np


def _sound(gamma, rho, p):
    return np.sqrt(gamma * p / rho)


def _f_side(p, rho_k, p_k, a_k, gamma):
    """Pressure function of one side and its derivative."""
    if p > p_k:  # shock branch
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        sq = np.sqrt(A / (p + B))
        f = (p - p_k) * sq
        df = sq * (1.0 - 0.5 * (p - p_k) / (B + p))
    else:  # rarefaction branch
        e = (gamma - 1.0) / (2.0 * gamma)
        f = 2.0 * a_k / (gamma - 1.0) * ((p / p_k) ** e - 1.0)
        df = 1.0 / (rho_k * a_k) * (p / p_k) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma=1.4, tol=1e-15, max_iter=200):
    """(p*, u*) of the Riemann problem with primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = _sound(gamma, rl, pl), _sound(gamma, rr, pr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated; not handled")
    # start from the two-rarefaction approximation (always positive)
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((al + ar - 0.5 * (gamma - 1.0) * (ur - ul)) /
         (al / pl ** e + ar / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-14)
    for _ in range(max_iter):
        fl, dfl = _f_side(p, rl, pl, al, gamma)
        fr, dfr = _f_side(p, rr, pr, ar, gamma)
        step = (fl + fr + ur - ul) / (dfl + dfr)
        p_new = max(p - step, 1e-14)
        if abs(p_new - p) <= tol * 0.5 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _f_side(p, rl, pl, al, gamma)
    fr, _ = _f_side(p, rr, pr, ar, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def star_densities(left, right, p_star, gamma=1.4):
    """Densities left and right of the contact in the star region."""
    out = []
    g1 = (gamma - 1.0) / (gamma + 1.0)
    for rho_k, _u, p_k in (left, right):
        r = p_star / p_k
        if r > 1.0:
            out.append(rho_k * (r + g1) / (g1 * r + 1.0))
        else:
            out.append(rho_k * r ** (1.0 / gamma))
    return tuple(out)


def wave_speeds(left, right, gamma=1.4):
    """Characteristic speeds of the solution.

    Returns a dict with 'contact' and, per side, either 'shock' or
    ('head', 'tail') of the rarefaction fan.
    """
    p_s, u_s = star_state(left, right, gamma)
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = _sound(gamma, rl, pl), _sound(gamma, rr, pr)
    res = {"contact": u_s, "p_star": p_s}
    if p_s > pl:
        res["left_shock"] = ul - al * np.sqrt((gamma + 1.0) / (2.0 * gamma) * p_s / pl +
                                              (gamma - 1.0) / (2.0 * gamma))
    else:
        a_s = al * (p_s / pl) ** ((gamma - 1.0) / (2.0 * gamma))
        res["left_head"] = ul - al
        res["left_tail"] = u_s - a_s
    if p_s > pr:
        res["right_shock"] = ur + ar * np.sqrt((gamma + 1.0) / (2.0 * gamma) * p_s / pr +
                                               (gamma - 1.0) / (2.0 * gamma))
    else:
        a_s = ar * (p_s / pr) ** ((gamma - 1.0) / (2.0 * gamma))
        res["right_head"] = ur + ar
        res["right_tail"] = u_s + a_s
    return res


def sample(left, right, xi, gamma=1.4):
    """Primitive solution (rho, u, p) at similarity coordinates xi = (x - x0)/t."""
    xi = np.asarray(xi, dtype=np.float64)
    p_s, u_s = star_state(left, right, gamma)
    rsl, rsr = star_densities(left, right, p_s, gamma)
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = _sound(gamma, rl, pl), _sound(gamma, rr, pr)
    g = gamma
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for i, s in np.ndenumerate(xi):
        if s <= u_s:  # left of the contact
            if p_s > pl:
                S = ul - al * np.sqrt((g + 1) / (2 * g) * p_s / pl + (g - 1) / (2 * g))
                w = (rl, ul, pl) if s <= S else (rsl, u_s, p_s)
            else:
                head = ul - al
                tail = u_s - al * (p_s / pl) ** ((g - 1) / (2 * g))
                if s <= head:
                    w = (rl, ul, pl)
                elif s >= tail:
                    w = (rsl, u_s, p_s)
                else:
                    c = 2 / (g + 1) + (g - 1) / ((g + 1) * al) * (ul - s)
                    w = (rl * c ** (2 / (g - 1)),
                         2 / (g + 1) * (al + (g - 1) / 2 * ul + s),
                         pl * c ** (2 * g / (g - 1)))
        else:  # right of the contact
            if p_s > pr:
                S = ur + ar * np.sqrt((g + 1) / (2 * g) * p_s / pr + (g - 1) / (2 * g))
                w = (rr, ur, pr) if s >= S else (rsr, u_s, p_s)
            else:
                head = ur + ar
                tail = u_s + ar * (p_s / pr) ** ((g - 1) / (2 * g))
                if s >= head:
                    w = (rr, ur, pr)
                elif s <= tail:
                    w = (rsr, u_s, p_s)
                else:
                    c = 2 / (g + 1) - (g - 1) / ((g + 1) * ar) * (ur - s)
                    w = (rr * c ** (2 / (g - 1)),
                         2 / (g + 1) * (-ar + (g - 1) / 2 * ur + s),
                         pr * c ** (2 * g / (g - 1)))
        rho[i], u[i], p[i] = w
    return rho, u, p


def cell_averages(left, right, x_faces, t, x0=0.5, gamma=1.4, sub=64):
    """Cell averages of the exact density/velocity/pressure over cells with
    the given face coordinates (midpoint rule with `sub` samples per cell)."""
    x_faces = np.asarray(x_faces, dtype=np.float64)
    n = x_faces.size - 1
    frac = (np.arange(sub) + 0.5) / sub
    xs = x_faces[:-1, None] + (x_faces[1:] - x_faces[:-1])[:, None] * frac[None, :]
    rho, u, p = sample(left, right, (xs - x0) / t, gamma)
    return rho.reshape(n, sub).mean(1), u.reshape(n, sub).mean(1), p.reshape(n, sub).mean(1)
