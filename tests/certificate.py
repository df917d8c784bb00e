"""Optimality certificate for a Beckmann solution, from duality alone.

Test infrastructure, independent of ``oracle/`` and of the library: it takes a flux
u and a potential phi from either side and brackets the exact optimal transport
cost W1 of the source s (Manhattan ground cost on the receiver x time grid):

* lower bound (weak duality of the Beckmann problem, the dual Kantorovich form of
  Section 2.1): for any phi whose differences across neighbouring cells are at most
  the grid step (|phi_i - phi_(i-1)| <= dx along receivers, <= dt along time),
  dx dt <phi, s> <= W1.  ``lip_below`` turns the returned potential into such a
  function (the largest one below it), so the bound holds whatever its accuracy.
* upper bound: dx dt sum|u| is the cost of a flux that moves s up to the residual
  r = div u + s; ``residual_flux`` builds a flux v with div v = -r (each trace's
  residual gathered along time to its first sample, then those sums along the
  first sample's column), so u + v is feasible and dx dt (sum|u| + sum|v|) >= W1.

div is the negative transpose of the backward-difference gradient (the reading of
the divergence boundary rows that makes the adjoint identity of Section 2.2 hold).
"""
from __future__ import annotations

import numpy as np


def cell_measure(nr: int, nt: int, dx: float, dt: float) -> float:
    """dx dt, with the spacing of a length-1 axis taken as 1 (a single trace)."""
    return (dx if nr > 1 else 1.0) * (dt if nt > 1 else 1.0)


def divergence(ux, ut, dx, dt):
    """(div u)_(i,j) = ([i<nr-1] ux_(i+1,j) - [i>0] ux_(i,j))/dx + the same along time."""
    ux = np.asarray(ux, np.float64)
    ut = np.asarray(ut, np.float64)
    nr, nt = ux.shape
    d = np.zeros((nr, nt))
    if nr > 1:
        d[:-1] += ux[1:] / dx
        d[1:] -= ux[1:] / dx
    if nt > 1:
        d[:, :-1] += ut[:, 1:] / dt
        d[:, 1:] -= ut[:, 1:] / dt
    return d


def lip_below(phi, dx, dt):
    """The largest function below phi whose neighbour differences are at most dx
    (receiver axis) and dt (time axis): min over y of phi(y) + dx|i - i'| + dt|j - j'|.
    The l1 cone is separable, so a forward and a backward min-plus pass per axis
    compute it exactly."""
    p = np.array(phi, np.float64, copy=True)
    nr, nt = p.shape
    for j in range(1, nt):
        np.minimum(p[:, j], p[:, j - 1] + dt, out=p[:, j])
    for j in range(nt - 2, -1, -1):
        np.minimum(p[:, j], p[:, j + 1] + dt, out=p[:, j])
    for i in range(1, nr):
        np.minimum(p[i], p[i - 1] + dx, out=p[i])
    for i in range(nr - 2, -1, -1):
        np.minimum(p[i], p[i + 1] + dx, out=p[i])
    return p


def residual_flux(r, dx, dt):
    """A flux v with div v = -r for a zero-sum r: along each trace the flux through
    the edge before sample j carries the residual of samples >= j, which collects
    the trace's net residual m_i at sample 0; along column 0 the flux before
    receiver i carries m of receivers >= i."""
    r = np.asarray(r, np.float64)
    nr, nt = r.shape
    vx = np.zeros((nr, nt))
    vt = np.zeros((nr, nt))
    if nt > 1:
        vt[:, 1:] = dt * np.cumsum(r[:, ::-1], axis=1)[:, ::-1][:, 1:]
    if nr > 1:
        m = r.sum(axis=1)
        vx[1:, 0] = dx * np.cumsum(m[::-1])[::-1][1:]
    return vx, vt


def transport_bounds(s, ux, ut, phi, dx, dt):
    """(lower, transport of u, upper): lower <= W1(s) <= upper."""
    s = np.asarray(s, np.float64)
    nr, nt = s.shape
    cm = cell_measure(nr, nt, dx, dt)
    lower = cm * float((lip_below(phi, dx, dt) * s).sum())
    r = divergence(ux, ut, dx, dt) + s
    w = cm * float(np.abs(np.asarray(ux, np.float64)).sum() + np.abs(np.asarray(ut, np.float64)).sum())
    vx, vt = residual_flux(r, dx, dt)
    # the residual sums to zero up to rounding; what is left is carried across the
    # grid's diameter
    diam = (nr - 1) * dx + (nt - 1) * dt
    upper = w + cm * (float(np.abs(vx).sum() + np.abs(vt).sum()) + abs(float(r.sum())) * diam)
    return lower, w, upper
