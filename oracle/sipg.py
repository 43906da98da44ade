"""SIPG Laplace / Helmholtz operator by direct quadrature (oracle; test infrastructure).

What is computed (paper Sec. 3.2, pressure Poisson step, eqs. poissonspat,
ipflux, taue, tau; the viscous step with its fluxes U* and F^nu*; matrix form
of Sec. 4.4, eqs. poissonmat and viscous).  Summing the element-wise weak
forms over both elements of every face gives, with [u] = u^- - u^+,
{{w}} = (w^- + w^+)/2 and n the normal of the minus side,

  a(v,u) = sum_K (grad v, grad u)_K
         - sum_{F interior or periodic} [ ({{grad v}}.n, [u]) + ([v], {{grad u}}.n) - tau_F ([v],[u]) ]_F
         - sum_{F Dirichlet}            [ (grad v.n, u) + (v, grad u.n) - 2 tau_F (v,u) ]_F

  tau_e = s (k+1)^2 (A(interior faces)/2 + A(boundary faces)) / V      (eq. taue; s = penalty scale)
  tau_F = max(tau_e^-, tau_e^+) on interior faces, tau_e^- on boundary faces  (eq. tau)

Homogeneous Neumann faces add nothing to a(v,u): there the flux takes the
cell's own trace (P* = p_h for the pressure on the velocity-Dirichlet part,
U* = u_h for the velocity on the Neumann part) and the flux of the gradient
is boundary data, which belongs to the right-hand side; their area still
counts in tau_e (eq. taue sums A over both boundary parts).  Inhomogeneous
Neumann data is not modelled here.

Helmholtz (viscous step, scalar form applied per component): H = mu M + nu A,
mu = gamma_0 / dt.  Right-hand side of the Dirichlet problem:
  b_i = (f, phi_i) + nu sum_{F Dirichlet} [ -(grad phi_i.n, g)_F + 2 tau_F (phi_i, g)_F ].

All integrals use Gauss quadrature with n_q = k+1 points per direction on
cells and (tangentially) on faces (Sec. 5).  Element matrices are dense
n^3 x n^3 blocks built from the Kronecker-product evaluation matrices of the
tensor basis -- no sum factorisation.  Everything is fp64.

Pins (tests/test_oracle_sipg.py): symmetry, positive semi-definiteness and
one-dimensional null space on periodic meshes, definiteness with Dirichlet
walls, equality with the independent Kronecker-sum construction (``kron``),
consistency (polynomials of degree <= k reproduced exactly), the coercivity
threshold of the 1D penalty, the first Laplace eigenvalue (2 pi)^2, and
optimal L2 convergence of order k+1 on a manufactured solution; with
Neumann sides (tests/test_oracle_neumann.py): constants in the null space,
the first Neumann eigenvalue pi^2, and order k+1 convergence on a
manufactured solution with zero normal derivative on the Neumann sides.
"""
import numpy as np
import scipy.sparse as sp

from . import basis


def _kron3(mz, my, mx):
    return np.kron(mz, np.kron(my, mx))


class Tables:
    """1D evaluation tables for degree k with nq Gauss points."""

    def __init__(self, k, nq=None):
        self.k = k
        self.n = k + 1
        self.nq = self.n if nq is None else nq
        self.nodes = basis.gll_nodes(k)
        self.xq, self.wq = basis.gauss_rule(self.nq)
        self.S = basis.lagrange_values(self.nodes, self.xq)        # (nq, n)
        self.D = basis.lagrange_derivatives(self.nodes, self.xq)   # (nq, n)
        self.e = [basis.lagrange_values(self.nodes, [s]) for s in (0.0, 1.0)]       # (1, n)
        self.de = [basis.lagrange_derivatives(self.nodes, [s]) for s in (0.0, 1.0)]  # (1, n)


def _ref_gradients_cell(T):
    """Reference-gradient evaluation matrices G_b (nq^3 x n^3), b = x, y, z."""
    S, D = T.S, T.D
    return [_kron3(S, S, D), _kron3(S, D, S), _kron3(D, S, S)]


def cell_matrices(T, J):
    """(K_e, M_e) of one affine cell with constant Jacobian J (3x3)."""
    detJ = abs(np.linalg.det(J))
    Jinv = np.linalg.inv(J)
    w = _kron3(T.wq, T.wq, T.wq) * detJ
    Phi = _kron3(T.S, T.S, T.S)
    G = _ref_gradients_cell(T)
    K = np.zeros((T.n ** 3, T.n ** 3))
    for a in range(3):
        Ga = sum(Jinv[b, a] * G[b] for b in range(3))   # d phi / d x_a
        K += Ga.T @ (w[:, None] * Ga)
    M = Phi.T @ (w[:, None] * Phi)
    return K, M


def face_eval(T, J, f):
    """Trace, physical normal derivative and quadrature measure on face f.

    Returns (Tr, Gn, dA, nrm): Tr[q,i] = phi_i(x_q), Gn[q,i] = grad phi_i(x_q) . n
    with n the unit normal pointing towards +d (the direction of the face,
    independent of the side), dA[q] = tangential weight * surface Jacobian.
    """
    d, s = divmod(f, 2)
    Jinv = np.linalg.inv(J)
    detJ = abs(np.linalg.det(J))
    m = Jinv.T[:, d]                     # J^{-T} e_d
    nrm = m / np.linalg.norm(m)
    # tangential evaluation matrices per direction (x, y, z)
    val = [T.S, T.S, T.S]
    val[d] = T.e[s]
    Tr = _kron3(val[2], val[1], val[0])
    G = []
    for b in range(3):
        mats = [T.S, T.S, T.S]
        mats[d] = T.e[s]
        mats[b] = T.de[s] if b == d else T.D
        G.append(_kron3(mats[2], mats[1], mats[0]))
    grad = [sum(Jinv[b, a] * G[b] for b in range(3)) for a in range(3)]
    Gn = sum(nrm[a] * grad[a] for a in range(3))
    wt = [T.wq, T.wq, T.wq]
    wt[d] = np.ones(1)
    dA = _kron3(wt[2], wt[1], wt[0]) * detJ * np.linalg.norm(m)
    return Tr, Gn, dA, nrm


def interior_face_block(T, JL, JR, d, tauF):
    """2n^3 x 2n^3 block of the face terms between L (face +d) and R (face -d)."""
    TrL, GnL, dA, _ = face_eval(T, JL, 2 * d + 1)
    TrR, GnR, _, _ = face_eval(T, JR, 2 * d)
    Jmp = np.hstack([TrL, -TrR])
    Avg = 0.5 * np.hstack([GnL, GnR])
    W = dA[:, None]
    return -(Avg.T @ (W * Jmp)) - (Jmp.T @ (W * Avg)) + tauF * (Jmp.T @ (W * Jmp))


def dirichlet_face_block(T, J, f, tauF):
    """n^3 x n^3 block of the Dirichlet face terms on face f (outward normal)."""
    Tr, Gn, dA, _ = face_eval(T, J, f)
    if f % 2 == 0:
        Gn = -Gn          # outward normal points towards -d on a low face
    W = dA[:, None]
    return -(Gn.T @ (W * Tr)) - (Tr.T @ (W * Gn)) + 2.0 * tauF * (Tr.T @ (W * Tr))


def penalty_per_cell(mesh, penalty_scale=1.0):
    """tau_e = s (k+1)^2 (A_int/2 + A_bnd)/V per cell (eq. taue; A_bnd: Dirichlet and
    Neumann faces alike)."""
    k = mesh.k
    if mesh.shear is None:
        # axis-aligned box cells: face areas are products of two edge lengths,
        # all cells at once (the same formula as the loop below)
        cx, cy, cz = mesh.cell_coords(np.arange(mesh.ncells))
        idx = (cx, cy, cz)
        h = [np.diff(mesh.verts[d])[idx[d]] for d in range(3)]
        a = np.zeros(mesh.ncells)
        for d in range(3):
            area = h[(d + 1) % 3] * h[(d + 2) % 3]
            for s, end in ((0, 0), (1, mesh.nc[d] - 1)):
                bnd = (~np.bool_(mesh.periodic[d])) & (idx[d] == end)
                a += np.where(bnd, area, 0.5 * area)
        return penalty_scale * (k + 1) ** 2 * a / (h[0] * h[1] * h[2])
    tau = np.empty(mesh.ncells)
    for c in range(mesh.ncells):
        a = 0.0
        for f in range(6):
            A = mesh.face_area(c, f)
            a += A if mesh.neighbor(c, f) < 0 else 0.5 * A
        tau[c] = penalty_scale * (k + 1) ** 2 * a / mesh.volume(c)
    return tau


class SIPG:
    """The operator mu M + nu A on a mesh, with dense blocks cached by geometry."""

    def __init__(self, mesh, mass_coeff=0.0, diff_coeff=1.0, penalty_scale=1.0):
        self.mesh = mesh
        self.mu = float(mass_coeff)
        self.nu = float(diff_coeff)
        self.T = Tables(mesh.k)
        self.tau_e = penalty_per_cell(mesh, penalty_scale)
        self._cache = {}

    @staticmethod
    def _key(*arrs):
        return tuple(np.round(np.concatenate([np.ravel(a) for a in arrs]), 15).tolist())

    def cell_block(self, c):
        J = self.mesh.jacobian(c)
        key = ("cell", self._key(J))
        if key not in self._cache:
            K, M = cell_matrices(self.T, J)
            self._cache[key] = self.mu * M + self.nu * K
        return self._cache[key]

    def face_block(self, cL, cR, d):
        JL, JR = self.mesh.jacobian(cL), self.mesh.jacobian(cR)
        tauF = max(self.tau_e[cL], self.tau_e[cR])
        key = ("int", d, self._key(JL, JR, [tauF]))
        if key not in self._cache:
            self._cache[key] = self.nu * interior_face_block(self.T, JL, JR, d, tauF)
        return self._cache[key]

    def bface_block(self, c, f):
        J = self.mesh.jacobian(c)
        key = ("dir", f, self._key(J, [self.tau_e[c]]))
        if key not in self._cache:
            self._cache[key] = self.nu * dirichlet_face_block(self.T, J, f, self.tau_e[c])
        return self._cache[key]

    # -- assembled matrix ----------------------------------------------------
    def assemble(self):
        """Global sparse matrix (scipy CSR), duplicates summed."""
        m = self.mesh
        nb = m.n ** 3
        rows, cols, vals = [], [], []
        loc = np.arange(nb)

        def add(r, cidx, B):
            rr, cc = np.meshgrid(r, cidx, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(B.ravel())

        for c in range(m.ncells):
            add(c * nb + loc, c * nb + loc, self.cell_block(c))
        for cL, cR, d in m.interior_faces():
            idx = np.concatenate([cL * nb + loc, cR * nb + loc])
            add(idx, idx, self.face_block(cL, cR, d))
        for c, f in m.boundary_faces():
            add(c * nb + loc, c * nb + loc, self.bface_block(c, f))
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(m.ndofs, m.ndofs))
        return A.tocsr()

    def mass_matrix(self):
        m = self.mesh
        blocks = [cell_matrices(self.T, m.jacobian(c))[1] for c in range(m.ncells)]
        return sp.block_diag(blocks, format="csr")

    # -- row-restricted application (full-size sampling) ---------------------
    def apply_cells(self, u, cells):
        """(H u) restricted to the DoFs of the listed cells, shape (len(cells), n^3)."""
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
                elif s == 1:      # c is the minus side (L) of this face
                    B = self.face_block(c, cn, d)
                    y += B[:nb, :nb] @ U[c] + B[:nb, nb:] @ U[cn]
                else:             # c is the plus side (R)
                    B = self.face_block(cn, c, d)
                    y += B[nb:, :nb] @ U[cn] + B[nb:, nb:] @ U[c]
            out[r] = y
        return out

    def apply_block_stencil(self, u):
        """H u on a uniform periodic box mesh (every cell a translate of one cell,
        one penalty): the assembled matrix is one diagonal block plus, per
        direction, the two off-diagonal blocks of the face matrix, so the product
        is a few dense block products over all cells at once.  Same operator as
        ``assemble``; u and the result are flat [N]."""
        m = self.mesh
        if not all(m.periodic) or m.shear is not None or m.gamma > 0:
            raise ValueError("block stencil needs a uniform periodic box mesh")
        nb = m.n ** 3
        U = u.reshape(m.ncells, nb)
        cells = np.arange(m.ncells)
        cx, cy, cz = m.cell_coords(cells)
        nx, ny, nz = m.nc
        diag = self.cell_block(0).copy()
        Y = np.zeros_like(U)
        for d in range(3):
            idx = [cx, cy, cz]
            up, dn = list(idx), list(idx)
            up[d] = (idx[d] + 1) % m.nc[d]
            dn[d] = (idx[d] - 1) % m.nc[d]
            plus = m.cell_index(*up)
            minus = m.cell_index(*dn)
            B = self.face_block(0, m.neighbor(0, 2 * d + 1), d)
            diag += B[:nb, :nb] + B[nb:, nb:]        # the cell as minus side of its +d face and plus side of its -d face
            Y += U[plus] @ B[:nb, nb:].T + U[minus] @ B[nb:, :nb].T
        Y += U @ diag.T
        return Y.ravel()

    def diagonal_cells(self, cells):
        """diag(H) restricted to the listed cells."""
        m = self.mesh
        nb = m.n ** 3
        out = np.zeros((len(cells), nb))
        for r, c in enumerate(cells):
            dg = np.diag(self.cell_block(c)).copy()
            for f in range(6):
                d, s = divmod(f, 2)
                cn = m.neighbor(c, f)
                if cn < 0:
                    if not m.neumann[f]:
                        dg += np.diag(self.bface_block(c, f))
                elif s == 1:
                    B = self.face_block(c, cn, d)
                    dg += np.diag(B[:nb, :nb])
                    if cn == c:
                        dg += np.diag(B[:nb, nb:]) + np.diag(B[nb:, :nb]) + np.diag(B[nb:, nb:])
                else:
                    if cn == c:
                        continue          # counted with the s == 1 face above
                    B = self.face_block(cn, c, d)
                    dg += np.diag(B[nb:, nb:])
            out[r] = dg
        return out

    # -- right-hand side -----------------------------------------------------
    def rhs(self, f, g=None, nq=None):
        """b_i = (f, phi_i) + Dirichlet data terms; f, g callables of (x, y, z).

        Integrals by a Gauss rule of nq points (default n_q = k+1, which is the
        paper's rule and therefore the definition of b for non-polynomial f).
        """
        m = self.mesh
        T = self.T if nq is None else Tables(m.k, nq)
        nb = m.n ** 3
        xq = T.xq
        Phi = _kron3(T.S, T.S, T.S)
        Lq, Jq, Iq = np.meshgrid(xq, xq, xq, indexing="ij")
        ref = np.stack([Iq.ravel(), Jq.ravel(), Lq.ravel()], axis=1)
        wq = _kron3(T.wq, T.wq, T.wq)
        b = np.zeros(m.ndofs)
        if m.shear is None:
            # axis-aligned cells: the same quadrature for all cells at once
            cx, cy, cz = m.cell_coords(np.arange(m.ncells))
            o = np.stack([m.verts[0][cx], m.verts[1][cy], m.verts[2][cz]], axis=1)
            h = np.stack([m.verts[0][cx + 1], m.verts[1][cy + 1], m.verts[2][cz + 1]], axis=1) - o
            X = o[:, None, :] + ref[None, :, :] * h[:, None, :]
            fv = f(X[..., 0], X[..., 1], X[..., 2]) * (wq[None, :] * np.prod(h, axis=1)[:, None])
            b += (fv @ Phi).ravel()
        else:
            for c in range(m.ncells):
                J = m.jacobian(c)
                o, _ = m.cell_origin_h(c)
                X = m.shear @ o + ref @ J.T
                fv = f(X[:, 0], X[:, 1], X[:, 2])
                b[c * nb:(c + 1) * nb] += Phi.T @ (wq * abs(np.linalg.det(J)) * fv)
        if g is not None:
            for c, fc in m.boundary_faces():
                J = m.jacobian(c)
                Tr, Gn, dA, _ = face_eval(T, J, fc)
                if fc % 2 == 0:
                    Gn = -Gn
                X = self._face_points(T, c, fc)
                gv = g(X[:, 0], X[:, 1], X[:, 2])
                b[c * nb:(c + 1) * nb] += self.nu * (-(Gn.T @ (dA * gv)) + 2.0 * self.tau_e[c] * (Tr.T @ (dA * gv)))
        return b

    def _face_points(self, T, c, f):
        m = self.mesh
        d, s = divmod(f, 2)
        axes = [T.xq, T.xq, T.xq]
        axes[d] = np.array([float(s)])
        Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        ref = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        o, _ = m.cell_origin_h(c)
        x0 = o if m.shear is None else m.shear @ o
        return x0 + ref @ m.jacobian(c).T


def l2_error(mesh, u, exact, nq=None):
    """|| u_h - exact ||_{L2} by a Gauss rule with nq = k+3 points per direction."""
    k = mesh.k
    T = Tables(k, k + 3 if nq is None else nq)
    Phi = _kron3(T.S, T.S, T.S)
    wq = _kron3(T.wq, T.wq, T.wq)
    Lq, Jq, Iq = np.meshgrid(T.xq, T.xq, T.xq, indexing="ij")
    ref = np.stack([Iq.ravel(), Jq.ravel(), Lq.ravel()], axis=1)
    nb = mesh.n ** 3
    err = 0.0
    for c in range(mesh.ncells):
        J = mesh.jacobian(c)
        o, _ = mesh.cell_origin_h(c)
        x0 = o if mesh.shear is None else mesh.shear @ o
        X = x0 + ref @ J.T
        diff = Phi @ u[c * nb:(c + 1) * nb] - exact(X[:, 0], X[:, 1], X[:, 2])
        err += np.sum(wq * abs(np.linalg.det(J)) * diff ** 2)
    return np.sqrt(err)


def integral_weights(mesh):
    """w_i = integral of phi_i over its cell (so 1^T M x = sum_i w_i x_i)."""
    T = Tables(mesh.k)
    nb = mesh.n ** 3
    Phi = _kron3(T.S, T.S, T.S)
    wq = _kron3(T.wq, T.wq, T.wq)
    out = np.empty(mesh.ndofs)
    for c in range(mesh.ncells):
        out[c * nb:(c + 1) * nb] = Phi.T @ wq * abs(np.linalg.det(mesh.jacobian(c)))
    return out
