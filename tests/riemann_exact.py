"""Exact solution of the Riemann problem of the 1-D Euler equations for an
ideal gas (the inviscid reference of the shock-tube case, Sec. III A).

Textbook construction: the star-region pressure p* is the root of
    f_L(p*) + f_R(p*) + (u_R - u_L) = 0,
with f_K the shock (Rankine-Hugoniot) branch for p* > p_K and the
rarefaction (isentropic) branch otherwise; Newton's method from the
two-rarefaction estimate.  The solution is then sampled on x/t.
Test reference only.
"""
import math

import numpy as np


def _fk(p, rho_k, p_k, gamma):
    a_k = math.sqrt(gamma * p_k / rho_k)
    if p > p_k:                                  # shock
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        s = math.sqrt(A / (p + B))
        f = (p - p_k) * s
        df = s * (1.0 - 0.5 * (p - p_k) / (p + B))
    else:                                        # rarefaction
        e = (gamma - 1.0) / (2.0 * gamma)
        f = 2.0 * a_k / (gamma - 1.0) * ((p / p_k) ** e - 1.0)
        df = 1.0 / (rho_k * a_k) * (p / p_k) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma):
    """(p*, u*) for left/right states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    e = (gamma - 1.0) / (2.0 * gamma)
    # two-rarefaction estimate
    p = ((al + ar - 0.5 * (gamma - 1.0) * (ur - ul)) / (al / pl ** e + ar / pr ** e)) ** (1.0 / e)
    for _ in range(100):
        fl, dl = _fk(p, rl, pl, gamma)
        fr, dr = _fk(p, rr, pr, gamma)
        step = (fl + fr + ur - ul) / (dl + dr)
        pn = max(p - step, 1e-12)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, gamma)
    fr, _ = _fk(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, gamma, s):
    """(rho, u, p) at the similarity coordinates s = (x - x0)/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    s = np.asarray(s, dtype=float)
    rho, u, p = np.empty_like(s), np.empty_like(s), np.empty_like(s)
    for k, sk in enumerate(s.ravel()):
        if sk <= us:                                         # left of the contact
            if ps > pl:
                rs = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                S = ul - al * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl + (gamma - 1.0) / (2.0 * gamma))
                st = (rl, ul, pl) if sk < S else (rs, us, ps)
            else:
                rs = rl * (ps / pl) ** (1.0 / gamma)
                ast = al * (ps / pl) ** ((gamma - 1.0) / (2.0 * gamma))
                head, tail = ul - al, us - ast
                if sk < head:
                    st = (rl, ul, pl)
                elif sk > tail:
                    st = (rs, us, ps)
                else:
                    uf = 2.0 / (gamma + 1.0) * (al + 0.5 * (gamma - 1.0) * ul + sk)
                    c = 2.0 / (gamma + 1.0) + g1 / al * (ul - sk)
                    st = (rl * c ** (2.0 / (gamma - 1.0)), uf, pl * c ** (2.0 * gamma / (gamma - 1.0)))
        else:                                                # right of the contact
            if ps > pr:
                rs = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                S = ur + ar * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr + (gamma - 1.0) / (2.0 * gamma))
                st = (rr, ur, pr) if sk > S else (rs, us, ps)
            else:
                rs = rr * (ps / pr) ** (1.0 / gamma)
                ast = ar * (ps / pr) ** ((gamma - 1.0) / (2.0 * gamma))
                head, tail = ur + ar, us + ast
                if sk > head:
                    st = (rr, ur, pr)
                elif sk < tail:
                    st = (rs, us, ps)
                else:
                    uf = 2.0 / (gamma + 1.0) * (-ar + 0.5 * (gamma - 1.0) * ur + sk)
                    c = 2.0 / (gamma + 1.0) - g1 / ar * (ur - sk)
                    st = (rr * c ** (2.0 / (gamma - 1.0)), uf, pr * c ** (2.0 * gamma / (gamma - 1.0)))
        rho.flat[k], u.flat[k], p.flat[k] = st
    return rho, u, p
