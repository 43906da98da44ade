"""SIPG operator on iso-parametric curved cells (oracle; test infrastructure).

Sec. 5 (implementation): the cells may be curved, with an iso-parametric
geometry, i.e. each cell's map from the reference cube is the degree-k
tensor-product Lagrange interpolant, at the cell's GLL nodes, of the physical
positions of those nodes; every integral uses Gauss quadrature with k+1
points per direction and the Jacobian of that map at each point (on curved
cells this rule defines the operator, it is no longer exact).

The physical positions come from a smooth deformation of the box mesh (after
the tanh grading): with t = (p - origin) / length per direction and
s(t) = sin(2 pi t),

    x = p + a * (lx s(t_y) s(t_z),  ly s(t_z) s(t_x),  lz s(t_x) s(t_y)),

periodic in every direction, so periodic faces stay translates of each other;
on a bounding side of a non-periodic direction the wall itself is curved.
Interior faces are conforming because neighbours share their face nodes.

The bilinear form is the one of ``sipg`` (interior and periodic faces with
central fluxes and tau_F = max(tau_e), Dirichlet faces with 2 tau, nothing on
homogeneous Neumann faces), tau_e = s (k+1)^2 (A_int/2 + A_bnd) / V with the
areas and volumes integrated on the curved cells.  Everything here is plain
dense linear algebra per cell and face, evaluated point by point; nothing
exploits the separable form of the deformation.

Pins (tests/test_oracle_curved.py): a = 0 gives the affine operator of
``sipg``; normals and surface measures of an interior face agree from both
sides; constants in the null space on a periodic curved mesh; symmetry and
semi-definiteness; order k+1 convergence of a manufactured solution on a
curved periodic mesh.
"""
import numpy as np
import scipy.sparse as sp

from . import basis
from .mesh import BoxMesh
from .sipg import Tables, _kron3


def deform(mesh, amp, P):
    """Physical points of box points P (m, 3) under the deformation of amplitude amp."""
    lo = np.array([mesh.verts[d][0] for d in range(3)])
    L = np.array([mesh.verts[d][-1] - mesh.verts[d][0] for d in range(3)])
    S = np.sin(2 * np.pi * (P - lo) / L)
    D = np.stack([L[0] * S[:, 1] * S[:, 2], L[1] * S[:, 2] * S[:, 0], L[2] * S[:, 0] * S[:, 1]], axis=1)
    return P + amp * D


class CurvedBoxMesh(BoxMesh):
    """A box mesh whose cells carry the iso-parametric image of the deformation."""

    def __init__(self, *args, amp=0.0, **kw):
        super().__init__(*args, **kw)
        if self.shear is not None:
            raise ValueError("curved cells: shear is not supported")
        self.amp = float(amp)
        self.gll = basis.gll_nodes(self.k)

    def box_nodes(self, c):
        """Box points of the cell's GLL nodes, (n^3, 3), x index fastest."""
        o, h = self.cell_origin_h(c)
        xi = self.gll
        L, J, I = np.meshgrid(xi, xi, xi, indexing="ij")
        return o + np.stack([I.ravel(), J.ravel(), L.ravel()], axis=1) * h

    def node_xyz(self, c):
        """Physical positions of the cell's nodes (n^3, 3)."""
        return deform(self, self.amp, self.box_nodes(c))

    def _lagr(self, t, deriv):
        return (basis.lagrange_derivatives if deriv else basis.lagrange_values)(self.gll, t)

    def map_at(self, c, xi):
        """x_h(xi) for reference points xi (m, 3)."""
        n = self.n
        X = self.node_xyz(c).reshape(n, n, n, 3)             # [l, j, i, r]
        Lx, Ly, Lz = (self._lagr(xi[:, d], False) for d in range(3))
        return np.einsum("pl,pj,pi,ljir->pr", Lz, Ly, Lx, X)

    def jac_at(self, c, xi):
        """J[p, r, d] = d x_h,r / d xi_d at reference points xi (m, 3)."""
        n = self.n
        X = self.node_xyz(c).reshape(n, n, n, 3)
        V = [self._lagr(xi[:, d], False) for d in range(3)]
        Dv = [self._lagr(xi[:, d], True) for d in range(3)]
        J = np.empty((xi.shape[0], 3, 3))
        for d in range(3):
            f = [Dv[e] if e == d else V[e] for e in range(3)]
            J[:, :, d] = np.einsum("pl,pj,pi,ljir->pr", f[2], f[1], f[0], X)
        return J

    def jacobian(self, c):
        raise TypeError("curved cells have no constant Jacobian")


def _cell_points(T):
    L, J, I = np.meshgrid(T.xq, T.xq, T.xq, indexing="ij")
    return np.stack([I.ravel(), J.ravel(), L.ravel()], axis=1), _kron3(T.wq, T.wq, T.wq)


def _face_points(T, f):
    d, s = divmod(f, 2)
    t = [T.xq, T.xq, T.xq]
    t[d] = np.array([float(s)])
    L, J, I = np.meshgrid(t[2], t[1], t[0], indexing="ij")
    wt = [T.wq, T.wq, T.wq]
    wt[d] = np.ones(1)
    return np.stack([I.ravel(), J.ravel(), L.ravel()], axis=1), _kron3(wt[2], wt[1], wt[0])


def _phys_grads(Gref, Jinv):
    """grad_a[p, i] = sum_b Jinv[p, b, a] Gref_b[p, i]."""
    return [sum(Jinv[:, b, a][:, None] * Gref[b] for b in range(3)) for a in range(3)]


class CurvedSIPG:
    """mu M + nu A on a CurvedBoxMesh, point-by-point quadrature."""

    def __init__(self, mesh, mass_coeff=0.0, diff_coeff=1.0, penalty_scale=1.0, cells=None):
        """cells: compute tau_e only for these cells and their face neighbours (for
        row-restricted applications on large meshes); None: every cell."""
        self.mesh = mesh
        self.mu, self.nu = float(mass_coeff), float(diff_coeff)
        self.T = T = Tables(mesh.k)
        self.xq_cell, self.wq_cell = _cell_points(T)
        self.Phi = _kron3(T.S, T.S, T.S)
        S, D = T.S, T.D
        self.Gref = [_kron3(S, S, D), _kron3(S, D, S), _kron3(D, S, S)]
        self.face_tabs = []
        for f in range(6):
            d, s = divmod(f, 2)
            val = [T.S, T.S, T.S]
            val[d] = T.e[s]
            Tr = _kron3(val[2], val[1], val[0])
            G = []
            for b in range(3):
                mats = [T.S, T.S, T.S]
                mats[d] = T.e[s]
                mats[b] = T.de[s] if b == d else T.D
                G.append(_kron3(mats[2], mats[1], mats[0]))
            self.face_tabs.append((Tr, G) + _face_points(T, f))
        self._faces = {}
        k = mesh.k
        self.tau_e = np.full(mesh.ncells, np.nan)
        need = range(mesh.ncells)
        if cells is not None:
            need = set(cells)
            for c in cells:
                need.update(cn for cn in (mesh.neighbor(c, f) for f in range(6)) if cn >= 0)
        for c in need:
            a = 0.0
            for f in range(6):
                A = self.face(c, f)[2].sum()
                a += A if mesh.neighbor(c, f) < 0 else 0.5 * A
            self.tau_e[c] = penalty_scale * (k + 1) ** 2 * a / self.volume(c)

    def volume(self, c):
        J = self.mesh.jac_at(c, self.xq_cell)
        return np.sum(self.wq_cell * np.abs(np.linalg.det(J)))

    def face(self, c, f):
        """(Tr, grads[3], dA, m): traces, physical gradients at the face points, the
        surface measure with weights, and J^{-T} e_d normalised (pointing towards +d)."""
        key = (c, f)
        if key not in self._faces:
            Tr, Gref, xi, wt = self.face_tabs[f]
            J = self.mesh.jac_at(c, xi)
            Jinv = np.linalg.inv(J)
            d = f // 2
            m = Jinv[:, d, :]                         # row d of J^{-1} = J^{-T} e_d
            mn = np.linalg.norm(m, axis=1)
            dA = wt * np.abs(np.linalg.det(J)) * mn
            self._faces[key] = (Tr, _phys_grads(Gref, Jinv), dA, m / mn[:, None])
        return self._faces[key]

    def cell_block(self, c):
        J = self.mesh.jac_at(c, self.xq_cell)
        w = self.wq_cell * np.abs(np.linalg.det(J))
        grads = _phys_grads(self.Gref, np.linalg.inv(J))
        K = sum(g.T @ (w[:, None] * g) for g in grads)
        M = self.Phi.T @ (w[:, None] * self.Phi)
        return self.mu * M + self.nu * K

    def face_block(self, cL, cR, d):
        """2n^3 x 2n^3 block between L (its face +d) and R (its face -d), n = L's normal."""
        TrL, gL, dA, nL = self.face(cL, 2 * d + 1)
        TrR, gR, _, _ = self.face(cR, 2 * d)
        GnL = sum(nL[:, a][:, None] * gL[a] for a in range(3))
        GnR = sum(nL[:, a][:, None] * gR[a] for a in range(3))
        Jmp = np.hstack([TrL, -TrR])
        Avg = 0.5 * np.hstack([GnL, GnR])
        W = dA[:, None]
        tauF = max(self.tau_e[cL], self.tau_e[cR])
        return self.nu * (-(Avg.T @ (W * Jmp)) - (Jmp.T @ (W * Avg)) + tauF * (Jmp.T @ (W * Jmp)))

    def bface_block(self, c, f):
        Tr, g, dA, nrm = self.face(c, f)
        sgn = 1.0 if f % 2 == 1 else -1.0          # outward normal
        Gn = sgn * sum(nrm[:, a][:, None] * g[a] for a in range(3))
        W = dA[:, None]
        return self.nu * (-(Gn.T @ (W * Tr)) - (Tr.T @ (W * Gn)) + 2.0 * self.tau_e[c] * (Tr.T @ (W * Tr)))

    def assemble(self):
        m = self.mesh
        nb = m.n ** 3
        loc = np.arange(nb)
        rows, cols, vals = [], [], []

        def add(r, cc, B):
            R, C = np.meshgrid(r, cc, indexing="ij")
            rows.append(R.ravel())
            cols.append(C.ravel())
            vals.append(B.ravel())

        for c in range(m.ncells):
            add(c * nb + loc, c * nb + loc, self.cell_block(c))
        for cL, cR, d in m.interior_faces():
            idx = np.concatenate([cL * nb + loc, cR * nb + loc])
            add(idx, idx, self.face_block(cL, cR, d))
        for c, f in m.boundary_faces():          # Dirichlet only; Neumann faces add nothing
            add(c * nb + loc, c * nb + loc, self.bface_block(c, f))
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(m.ndofs, m.ndofs))
        return A.tocsr()

    def apply_cells(self, u, cells):
        """(H u) on the DoFs of the listed cells, shape (len(cells), n^3)."""
        m = self.mesh
        nb = m.n ** 3
        U = u.reshape(m.ncells, nb)
        out = np.zeros((len(cells), nb))
        for r, c in enumerate(cells):
            y = self.cell_block(c) @ U[c]
            for f in range(6):
                d, s = divmod(f, 2)
                cn = m.neighbor(c, f)
                if cn < 0:
                    if not m.neumann[f]:
                        y += self.bface_block(c, f) @ U[c]
                elif s == 1:
                    B = self.face_block(c, cn, d)
                    y += B[:nb, :nb] @ U[c] + B[:nb, nb:] @ U[cn]
                else:
                    B = self.face_block(cn, c, d)
                    y += B[nb:, :nb] @ U[cn] + B[nb:, nb:] @ U[c]
            out[r] = y
        return out

    def rhs(self, f):
        """b_i = (f, phi_i) on the curved cells (k+1 Gauss points; no boundary data)."""
        m = self.mesh
        nb = m.n ** 3
        b = np.zeros(m.ndofs)
        for c in range(m.ncells):
            J = m.jac_at(c, self.xq_cell)
            X = m.map_at(c, self.xq_cell)
            w = self.wq_cell * np.abs(np.linalg.det(J))
            b[c * nb:(c + 1) * nb] = self.Phi.T @ (w * f(X[:, 0], X[:, 1], X[:, 2]))
        return b

    def l2_error(self, u, exact, nq=None):
        m = self.mesh
        T = Tables(m.k, m.k + 3 if nq is None else nq)
        xi, wq = _cell_points(T)
        Phi = _kron3(T.S, T.S, T.S)
        nb = m.n ** 3
        err = 0.0
        for c in range(m.ncells):
            J = m.jac_at(c, xi)
            X = m.map_at(c, xi)
            diff = Phi @ u[c * nb:(c + 1) * nb] - exact(X[:, 0], X[:, 1], X[:, 2])
            err += np.sum(wq * np.abs(np.linalg.det(J)) * diff ** 2)
        return np.sqrt(err)
