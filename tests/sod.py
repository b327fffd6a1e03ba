"""Sod's shock tube (the paper's Sec. 5.2 setup: [-1/2, 1/2], t = 0.18,
(rho, v, p) = (1, 0, 1) | (1/8, 0, 1/10)) on a periodic mesh, and its exact
solution.  The tube is mirrored onto [-1/2, 3/2] so that the periodic wrap
joins equal states; the mirrored jump at x = 1 sends waves that meet the
original ones only at x = 1/2 after t = 0.18."""
import numpy as np

from paper_2004_08503_amd import workloads as W

GAMMA = 1.4
LEFT = (1.0, 0.0, 1.0)
RIGHT = (0.125, 0.0, 0.1)
T_END = 0.18


def problem(nx, p, limiter=W.SUBCELL):
    """nx elements per unit length (2 nx on the mirrored domain)."""
    return W.Problem(dim=1, nx=2 * nx, ny=1, p=p, eq=W.EULER, lx=2.0, gamma=GAMMA, limiter=limiter)


def initial(prob):
    x, _, _ = W.node_coords(prob)
    n1 = prob.p + 1
    # a node on an element face takes the state of its own element:
    # classify by the element centre
    xc = (np.floor(np.arange(prob.num_nodes) / n1) + 0.5) * (prob.lx / prob.nx) - 0.5
    left = (xc < 0.0) | (xc >= 1.0)
    rho = np.where(left, LEFT[0], RIGHT[0])
    pr = np.where(left, LEFT[2], RIGHT[2])
    u = np.zeros((3, prob.num_nodes))
    u[0] = rho
    u[2] = pr / (GAMMA - 1.0)
    return x - 0.5, u


def _f(p, rho, pk, c, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * np.sqrt(A / (p + B))
    return 2.0 * c / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def exact(xi, g=GAMMA, L=LEFT, R=RIGHT):
    """(rho, v, p) of the Riemann problem at self-similar coordinates
    xi = x / t (Toro's pressure function, solved by bisection)."""
    rl, vl, pl = L
    rr, vr, pr = R
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    lo, hi = 1e-12, 10.0 * max(pl, pr)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _f(mid, rl, pl, cl, g) + _f(mid, rr, pr, cr, g) + vr - vl > 0.0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    vs = 0.5 * (vl + vr) + 0.5 * (_f(ps, rr, pr, cr, g) - _f(ps, rl, pl, cl, g))
    out = np.zeros((3, len(xi)))
    for i, s in enumerate(xi):
        if s < vs:   # left of the contact
            if ps > pl:   # left shock
                sl = vl - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s < sl:
                    out[:, i] = (rl, vl, pl)
                else:
                    r = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
                    out[:, i] = (r, vs, ps)
            else:         # left rarefaction
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                if s < vl - cl:
                    out[:, i] = (rl, vl, pl)
                elif s > vs - cs:
                    out[:, i] = (rl * (ps / pl) ** (1 / g), vs, ps)
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (vl - s))
                    v = 2 / (g + 1) * (cl + (g - 1) / 2 * vl + s)
                    r = rl * (c / cl) ** (2 / (g - 1))
                    out[:, i] = (r, v, pl * (c / cl) ** (2 * g / (g - 1)))
        else:        # right of the contact
            if ps > pr:   # right shock
                sr = vr + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s > sr:
                    out[:, i] = (rr, vr, pr)
                else:
                    r = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
                    out[:, i] = (r, vs, ps)
            else:         # right rarefaction
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                if s > vr + cr:
                    out[:, i] = (rr, vr, pr)
                elif s < vs + cs:
                    out[:, i] = (rr * (ps / pr) ** (1 / g), vs, ps)
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (vr - s))
                    v = 2 / (g + 1) * (-cr + (g - 1) / 2 * vr + s)
                    r = rr * (c / cr) ** (2 / (g - 1))
                    out[:, i] = (r, v, pr * (c / cr) ** (2 * g / (g - 1)))
    return out


def density_l1(prob, x, u, w, t=T_END):
    """L1 error of the density on [-1/2, 1/2] (Gauss-Lobatto quadrature per
    element, nodes on the interval's end faces included once per element)."""
    inside = (x >= -0.5) & (x <= 0.5)
    n1 = prob.p + 1
    elem = np.arange(prob.num_nodes) // n1
    xc = (elem + 0.5) * (prob.lx / prob.nx) - 0.5
    keep = (xc > -0.5) & (xc < 0.5)
    ex = exact(x[keep] / t)
    wn = np.tile(w, prob.nx)[keep] * (prob.lx / prob.nx)
    return float(np.sum(wn * np.abs(u[0][keep] - ex[0]))), inside
