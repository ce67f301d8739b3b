"""Exact Riemann solver for the 1-D Euler equations of an ideal gas (test helper).

Textbook construction (Toro, Riemann Solvers and Numerical Methods for Fluid
Dynamics, Ch. 4): Newton iteration on the pressure function
f_L(p) + f_R(p) + u_R - u_L = 0, then sampling of the self-similar solution.
"""
import math

import numpy as np


def _fk(p, rk, pk, gm):
    ak = math.sqrt(gm * pk / rk)
    if p > pk:  # shock
        A, B = 2.0 / ((gm + 1.0) * rk), (gm - 1.0) / (gm + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    e = (gm - 1.0) / (2.0 * gm)
    return (2.0 * ak / (gm - 1.0)) * ((p / pk) ** e - 1.0), (1.0 / (rk * ak)) * (p / pk) ** (-(gm + 1.0) / (2.0 * gm))


def star_state(L, R, gm):
    rL, uL, pL = L
    rR, uR, pR = R
    p = 0.5 * (pL + pR)
    for _ in range(200):
        fL, dL = _fk(p, rL, pL, gm)
        fR, dR = _fk(p, rR, pR, gm)
        dp = (fL + fR + uR - uL) / (dL + dR)
        pn = max(p - dp, 1e-14)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _fk(p, rL, pL, gm)
    fR, _ = _fk(p, rR, pR, gm)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)

    def rho_star(rk, pk):
        if p > pk:
            g = (gm - 1.0) / (gm + 1.0)
            return rk * ((p / pk + g) / (g * p / pk + 1.0))
        return rk * (p / pk) ** (1.0 / gm)

    return p, u, rho_star(rL, pL), rho_star(rR, pR)


def sample(L, R, gm, s):
    """Density, velocity, pressure at similarity coordinates s = (x - x0)/t (array)."""
    rL, uL, pL = L
    rR, uR, pR = R
    ps, us, rsL, rsR = star_state(L, R, gm)
    aL, aR = math.sqrt(gm * pL / rL), math.sqrt(gm * pR / rR)
    out = np.zeros((len(s), 3))
    for n, S in enumerate(np.asarray(s)):
        if S <= us:  # left of contact
            if ps > pL:
                SL = uL - aL * math.sqrt((gm + 1) / (2 * gm) * ps / pL + (gm - 1) / (2 * gm))
                out[n] = (rL, uL, pL) if S <= SL else (rsL, us, ps)
            else:
                SH, ast = uL - aL, aL * (ps / pL) ** ((gm - 1) / (2 * gm))
                ST = us - ast
                if S <= SH:
                    out[n] = (rL, uL, pL)
                elif S >= ST:
                    out[n] = (rsL, us, ps)
                else:
                    c = 2 / (gm + 1) + (gm - 1) / ((gm + 1) * aL) * (uL - S)
                    out[n] = (rL * c ** (2 / (gm - 1)), 2 / (gm + 1) * (aL + (gm - 1) / 2 * uL + S),
                              pL * c ** (2 * gm / (gm - 1)))
        else:
            if ps > pR:
                SR = uR + aR * math.sqrt((gm + 1) / (2 * gm) * ps / pR + (gm - 1) / (2 * gm))
                out[n] = (rR, uR, pR) if S >= SR else (rsR, us, ps)
            else:
                SH, ast = uR + aR, aR * (ps / pR) ** ((gm - 1) / (2 * gm))
                ST = us + ast
                if S >= SH:
                    out[n] = (rR, uR, pR)
                elif S <= ST:
                    out[n] = (rsR, us, ps)
                else:
                    c = 2 / (gm + 1) - (gm - 1) / ((gm + 1) * aR) * (uR - S)
                    out[n] = (rR * c ** (2 / (gm - 1)), 2 / (gm + 1) * (-aR + (gm - 1) / 2 * uR + S),
                              pR * c ** (2 * gm / (gm - 1)))
    return out
