"""Kink-aware central differences of <w, C(U)> for the convective operator.

C is piecewise quadratic in U: away from the kinks of the Lax-Friedrichs
lambda = max(|u-.n|, |u+.n|) the central difference of f(t) = <w, C(U + t d)>
equals f'(0) up to rounding.  Along a random direction, some face quadrature
points cross a kink inside [-eps, eps].  The face part of f is a sum over
face points q of g_q(t) = dA_q [w](x_q) . R(u-(t), u+(t); n), so the error of
the central difference is exactly the sum, over those points only, of
(g_q(eps) - g_q(-eps)) / (2 eps) - g_q'(0).  This helper finds the points
whose active side or active sign can change for |t| <= eps (the candidate
crossings of |a(t)| = |b(t)|, a(t) = 0 and b(t) = 0 with a, b linear in t)
and evaluates that sum with the oracle's flux R and its directional
derivative (the oracle's tie rule at t = 0).

Periodic axis-aligned box meshes of uniform cells only (the configurations
this is used on); face traces at Gauss points are interpolated from the nodal
face planes (Gauss-Lobatto end nodes) with the oracle's 1D tables.
"""
import numpy as np
import torch

from oracle import basis
from oracle.convective import Convective


def _traces(V, n, cells, S):
    """For d = 0, 1, 2: (minus, plus) traces, each (3, ncells * nq^2), of the
    field V ([3][N] nodal values) at the Gauss points of the faces normal to d;
    minus is the cell, plus its periodic +d neighbour."""
    nx, ny, nz = cells
    Vc = V.reshape(3, nz, ny, nx, n, n, n)          # (comp, cz, cy, cx, l, j, i)
    out = []
    for d in range(3):
        ax = 6 - d                                   # node axis along d: i (x), j (y), l (z)
        cax = 3 - d                                  # cell axis along d: cx, cy, cz
        hi = Vc.select(ax, n - 1)
        lo = torch.roll(Vc.select(ax, 0), shifts=-1, dims=cax)
        um = torch.einsum("pa,qb,...ab->...pq", S, S, hi)
        up = torch.einsum("pa,qb,...ab->...pq", S, S, lo)
        out.append((um.reshape(3, -1), up.reshape(3, -1)))
    return out


def kink_correction(U, D, W, degree, cells, nq, h, eps):
    """(correction, number of points) such that central difference - correction = f'(0).

    U, D, W: torch tensors [3][N] (any device); h: the uniform cell size
    (faces have area h^2)."""
    n = degree + 1
    xq, wq = basis.gauss_rule(nq)
    S = torch.as_tensor(basis.lagrange_values(basis.gll_nodes(degree), xq), dtype=U.dtype, device=U.device)
    tu, td, tw = (_traces(V, n, cells, S) for V in (U, D, W))
    wface = np.outer(wq, wq).ravel() * h * h
    corr, count = 0.0, 0
    for d in range(3):
        um, up = tu[d]
        dum, dup = td[d]
        wm, wp = tw[d]
        a, b, da, db = um[d], up[d], dum[d], dup[d]
        cand = torch.stack([(b - a) / (da - db), (-b - a) / (da + db), -a / da, -b / db])   # inf/nan: no crossing
        near = (cand.abs() <= eps).any(dim=0)
        idx = torch.nonzero(near).flatten()
        if idx.numel() == 0:
            continue
        count += int(idx.numel())
        pick = lambda t: t[:, idx].cpu().numpy()
        um_, up_, dum_, dup_, jw = pick(um), pick(up), pick(dum), pick(dup), pick(wm - wp)
        dA = wface[(idx.cpu().numpy()) % (nq * nq)]
        nrm = np.zeros((3, idx.numel()))
        nrm[d] = 1.0

        def g(t):
            R = Convective.flux(um_ + t * dum_, up_ + t * dup_, nrm)
            return dA * np.sum(jw * R, axis=0)

        gp0 = dA * np.sum(jw * Convective.flux_jvp(um_, up_, nrm, dum_, dup_), axis=0)
        corr += float(np.sum((g(eps) - g(-eps)) / (2.0 * eps) - gp0))
    return corr, count
