"""Geometric multigrid V-cycle preconditioner (oracle; test infrastructure).

Sec. 5.1 (Poisson solver) of the paper: one V-cycle of geometric multigrid
over the mesh hierarchy, a Chebyshev polynomial smoother (the Chebyshev
acceleration of point Jacobi, degree 5 for both pre- and post-smoothing,
smoothing range 20 on every level, eigenvalue estimates from a Krylov run on
every level), a Chebyshev iteration as coarse solver whose length is chosen
so that the Chebyshev error estimate reaches 1e-3, and level transfers by the
tensorial embedding of a mother cell's polynomials into its children.

Readings fixed here (and used identically by the GPU path):
* hierarchy: halve every direction whose cell count is even, until no count
  is even (down to one cell on 2^m meshes); the operator is discretised anew
  on every level with the same coefficients and penalty rule; on a curved
  mesh the finest level keeps the curved operator and the coarse levels are
  the undeformed box (sides and grading kept);
* transfer: prolongation P evaluates the mother's nodal polynomial at the
  child's nodes, the child covering half of the mother's reference cell in
  every halved direction (reference-cell embedding); restriction is P^T;
* smoother: S(b, x) = x + q(D^{-1}A) D^{-1} (b - A x), the degree-5 error
  polynomial on [lambda/20, lambda], lambda = 1.2 x the largest Ritz value of
  15 Lanczos steps on D^{-1/2} A D^{-1/2} from a SplitMix64(seed + level)
  start vector (mean removed for singular problems); from x = 0 the residual
  product is skipped;
* coarse solver: the same Chebyshev iteration from zero on
  [theta_min / 1.2, 1.2 theta_max], theta from Lanczos with full
  re-orthogonalisation (fp64, min(64, dim) steps, the null vector D^{1/2} 1
  deflated for singular problems), degree m = ceil(acosh(1/tol) /
  acosh((b+a)/(b-a))), i.e. the smallest m with 1/T_m((b+a)/(b-a)) <= tol;
* V-cycle: x = S(b, 0); xc = V(P^T (b - A x)) one level down; x += P xc;
  x = S(b, x); on the coarsest level x = coarse solve of b.
"""
import math

import numpy as np
import scipy.sparse as sp

from . import basis, curved, mesh as omesh, rng, sipg, solvers


def level_counts(nc):
    """Cell counts of the hierarchy, finest first."""
    out = [tuple(int(c) for c in nc)]
    while True:
        nxt = tuple(c // 2 if c % 2 == 0 else c for c in out[-1])
        if nxt == out[-1]:
            return out
        out.append(nxt)


def coarser_mesh(m, counts):
    """The same box with the given cell counts (shear is not supported)."""
    if m.shear is not None:
        raise ValueError("multigrid hierarchy: sheared meshes are not supported")
    vx, vy, vz = m.verts
    return omesh.BoxMesh(m.k, *counts, lx=vx[-1] - vx[0], ly=vy[-1] - vy[0], lz=vz[-1] - vz[0], y0=vy[0],
                         periodic=m.periodic, y_tanh_gamma=m.gamma, neumann=m.neumann)


def prolongation(fine, coarse):
    """Sparse P (fine.ndofs x coarse.ndofs): the mother's polynomial at the child's nodes."""
    n = fine.n
    nodes = basis.gll_nodes(fine.k)
    ratio = [fine.nc[d] // coarse.nc[d] for d in range(3)]
    assert all(r in (1, 2) and fine.nc[d] == r * coarse.nc[d] for d, r in enumerate(ratio))
    # E[d][s][i, a] = l_a((s + xi_i) / ratio_d): child s of the mother along d
    E = [[basis.lagrange_values(nodes, (s + nodes) / r) for s in range(r)] for r in ratio]
    rows, cols, vals = [], [], []
    nb = n ** 3
    loc = np.arange(nb)
    for cf in range(fine.ncells):
        ix = fine.cell_coords(cf)
        mother = coarse.cell_index(*[ix[d] // ratio[d] for d in range(3)])
        s = [ix[d] % ratio[d] for d in range(3)]
        B = np.kron(E[2][s[2]], np.kron(E[1][s[1]], E[0][s[0]]))
        rows.append(np.repeat(cf * nb + loc, nb))
        cols.append(np.tile(mother * nb + loc, nb))
        vals.append(B.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fine.ndofs, coarse.ndofs))


def chebyshev_interval(apply, dinv, r, a, b, degree, x0=None):
    """x0 + q(D^{-1}A) D^{-1} (r - A x0): Chebyshev acceleration of Jacobi on [a, b]
    (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1), error
    polynomial of the given degree (degree-1 operator products, one more with x0)."""
    theta, delta = 0.5 * (b + a), 0.5 * (b - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    res = np.array(r, dtype=np.float64) if x0 is None else r - apply(x0)
    d = (dinv * res) / theta
    x = d.copy() if x0 is None else x0 + d
    for _ in range(1, degree):
        res = res - apply(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * res)
        x = x + d
        rho = rho_new
    return x


def coarse_degree(a, b, tol):
    """Smallest m with 1 / T_m((b+a)/(b-a)) <= tol."""
    return max(1, int(math.ceil(math.acosh(1.0 / tol) / math.acosh((b + a) / (b - a)))))


def lanczos_full(apply_sym, v0, steps, null=None):
    """Extreme Ritz values of Lanczos with full re-orthogonalisation (and deflation of ``null``)."""
    def deflate(w):
        return w if null is None else w - (null @ w) * null
    V = []
    v = deflate(np.array(v0, dtype=np.float64))
    v = v / np.linalg.norm(v)
    alphas, betas = [], []
    for j in range(steps):
        V.append(v)
        w = apply_sym(v)
        alpha = w @ v
        w = deflate(w)
        for u in V:
            w = w - (u @ w) * u
        for u in V:                      # twice is enough (Kahan)
            w = w - (u @ w) * u
        alphas.append(alpha)
        beta = np.linalg.norm(w)
        scale = max(abs(a) for a in alphas)
        if j == steps - 1 or beta <= 1e-8 * scale:      # invariant subspace reached
            break
        betas.append(beta)
        v = deflate(w / beta)
        v = v / np.linalg.norm(v)
    m = len(alphas)
    T = np.diag(alphas) + np.diag(betas[:m - 1], 1) + np.diag(betas[:m - 1], -1)
    ev = np.linalg.eigvalsh(T)
    return ev[0], ev[-1]


class Multigrid:
    """V-cycle preconditioner for mu M + nu A (SIPG) on a box mesh."""

    def __init__(self, mesh, mass_coeff=0.0, diff_coeff=1.0, penalty_scale=1.0, degree=5, smoothing_range=20.0,
                 lanczos_steps=15, safety=1.2, seed=42, singular=False, coarse_tol=1e-3):
        self.degree, self.range = int(degree), float(smoothing_range)
        counts = level_counts(mesh.nc)
        self.meshes = [mesh] + [coarser_mesh(mesh, c) for c in counts[1:]]
        # a curved finest level keeps its curved operator; the coarse levels
        # rediscretise on the undeformed box (coarser_mesh builds affine boxes)
        self.ops = [(curved.CurvedSIPG if isinstance(m, curved.CurvedBoxMesh) else sipg.SIPG)(
            m, mass_coeff, diff_coeff, penalty_scale) for m in self.meshes]
        self.A = [op.assemble() for op in self.ops]
        self.dinv = [1.0 / A.diagonal() for A in self.A]
        self.P = [prolongation(self.meshes[l], self.meshes[l + 1]) for l in range(len(self.meshes) - 1)]
        self.lam = []
        for l in range(len(self.meshes) - 1):
            A, d = self.A[l], self.A[l].diagonal()
            v0 = rng.uniform_pm1(seed + l, A.shape[0])
            if singular:
                v0 = v0 - v0.mean()
            ritz, _ = solvers.lanczos_ritz(lambda v: (A @ (v / np.sqrt(d))) / np.sqrt(d), v0, lanczos_steps)
            self.lam.append(safety * ritz[-1])
        Ac, dc = self.A[-1], self.A[-1].diagonal()
        null = None
        if singular:
            null = np.sqrt(dc) / np.linalg.norm(np.sqrt(dc))
        steps = min(64, Ac.shape[0] - (1 if singular else 0))
        v0 = rng.uniform_pm1(seed + len(self.meshes) - 1, Ac.shape[0])
        tmin, tmax = lanczos_full(lambda v: (Ac @ (v / np.sqrt(dc))) / np.sqrt(dc), v0, steps, null)
        self.coarse_interval = (tmin / safety, safety * tmax)
        self.coarse_m = coarse_degree(*self.coarse_interval, coarse_tol)

    @property
    def levels(self):
        return len(self.meshes)

    def smooth(self, l, b, x=None):
        A = self.A[l]
        return chebyshev_interval(lambda u: A @ u, self.dinv[l], b, self.lam[l] / self.range, self.lam[l],
                                  self.degree, x0=x)

    def coarse_solve(self, b):
        A = self.A[-1]
        a, bb = self.coarse_interval
        return chebyshev_interval(lambda u: A @ u, self.dinv[-1], b, a, bb, self.coarse_m)

    def vcycle(self, b, l=0):
        if l == self.levels - 1:
            return self.coarse_solve(b)
        A = self.A[l]
        x = self.smooth(l, b)
        xc = self.vcycle(self.P[l].T @ (b - A @ x), l + 1)
        x = x + self.P[l] @ xc
        return self.smooth(l, b, x)
