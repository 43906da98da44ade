"""Divergence, gradient, mass and the div-div projection of variant V3c (oracle; test infrastructure).

Sec. 4.2, variants V3a and V3c, and Sec. 4 (matrix formulation):
* divergence operator A (eq. av3, without the factor gamma_0/dt):
    (A u)_i = (grad phi_i, u)_K - (phi_i, {{u}}^ND . n)_dK, summed over cells;
* gradient operator B (eq. bv3, without the factor dt/gamma_0):
    (B p)_{i,a} = (d_a phi_i, p)_K - (phi_i, {{p}}^ND n_a)_dK;
  with the central average on interior faces and {{w}}^ND = w^- (the cell's
  own trace) on boundary faces, Dirichlet and Neumann alike (Sec. 3.1);
* block-diagonal mass matrix M and div-div penalty D_e = (div v, div u)_K
  (eq. div-div), penalty tau_D = zeta_D |u_bar| h dt per cell with u_bar the
  cell average of the velocity and h = V^(1/3) (eq. tauD);
* local projection (eq. project, V3: tau_C = 0): per cell
  (M_e + tau_D,e D_e) u = rhs_e, solved here by a dense solve.
All integrals by Gauss quadrature with k+1 points per direction (exact on
affine cells), built from dense Kronecker-product evaluation matrices.  On
curved (iso-parametric) cells, Sec. 5, A and B take the Jacobian of the cell
map at every cell and face quadrature point (normals and surface measures by
Nanson's formula); there the k+1-point rule defines the operators, and a
larger ``nq`` is available for the pins that need exact integration.  The
cell mass, the div-div matrix D_e, the penalty's volume average and the
projection use the same per-point Jacobians on curved cells.
"""
import numpy as np
import scipy.sparse as sp

from . import sipg


def _cell_grad(T, J):
    """Physical gradient matrices G[a][q, i] = d_a phi_i(x_q), Phi, and weights w_q |det J|."""
    Phi = sipg._kron3(T.S, T.S, T.S)
    G = sipg._ref_gradients_cell(T)
    Jinv = np.linalg.inv(J)
    grad = [sum(Jinv[b, a] * G[b] for b in range(3)) for a in range(3)]
    w = sipg._kron3(T.wq, T.wq, T.wq) * abs(np.linalg.det(J))
    return grad, Phi, w


def _curved(m):
    return hasattr(m, "jac_at")


def _tables(m, nq):
    return sipg.Tables(m.k) if nq is None else sipg.Tables(m.k, nq)


def _cell_geo(T, m, c):
    """(grad, Phi, w) of cell c: per-point Jacobians on curved cells."""
    if not _curved(m):
        return _cell_grad(T, m.jacobian(c))
    Z, Y, X = np.meshgrid(T.xq, T.xq, T.xq, indexing="ij")
    J = m.jac_at(c, np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    Jinv = np.linalg.inv(J)
    G = sipg._ref_gradients_cell(T)
    grad = [sum(Jinv[:, b, a][:, None] * G[b] for b in range(3)) for a in range(3)]
    w = sipg._kron3(T.wq, T.wq, T.wq) * np.abs(np.linalg.det(J))
    return grad, sipg._kron3(T.S, T.S, T.S), w


def _face_geo(T, m, c, f):
    """(Tr, dA, nrm) of face f of cell c: traces at the face points, surface
    weights, and unit normals towards +d, one row per point (mq, 3)."""
    if not _curved(m):
        Tr, _, dA, nrm = sipg.face_eval(T, m.jacobian(c), f)
        return Tr, dA, np.repeat(np.asarray(nrm)[None, :], dA.size, axis=0)
    d, s = divmod(f, 2)
    val = [T.S, T.S, T.S]
    val[d] = T.e[s]
    Tr = sipg._kron3(val[2], val[1], val[0])
    t = [T.xq, T.xq, T.xq]
    t[d] = np.array([float(s)])
    Z, Y, X = np.meshgrid(t[2], t[1], t[0], indexing="ij")
    wt = [T.wq, T.wq, T.wq]
    wt[d] = np.ones(1)
    J = m.jac_at(c, np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    mv = np.linalg.inv(J)[:, d, :]                   # J^{-T} e_d per point
    mn = np.linalg.norm(mv, axis=1)
    dA = sipg._kron3(wt[2], wt[1], wt[0]) * np.abs(np.linalg.det(J)) * mn
    return Tr, dA, mv / mn[:, None]


def _faces(m):
    """Interior faces (cL, cR, d) and boundary faces (c, f), Dirichlet and Neumann alike:
    the ND average is the own trace on both boundary parts (Sec. 3.1)."""
    return m.interior_faces(), sorted(m.boundary_faces() + m.neumann_faces())


class _Blocks:
    """Dense blocks added at (row offset, column offset), summed into a sparse matrix."""

    def __init__(self, shape):
        self.shape, self.r, self.c, self.v = shape, [], [], []

    def add(self, r0, c0, blk):
        rr, cc = np.meshgrid(r0 + np.arange(blk.shape[0]), c0 + np.arange(blk.shape[1]), indexing="ij")
        self.r.append(rr.ravel())
        self.c.append(cc.ravel())
        self.v.append(blk.ravel())

    def tocsr(self):
        return sp.coo_matrix((np.concatenate(self.v), (np.concatenate(self.r), np.concatenate(self.c))),
                             shape=self.shape).tocsr()


def divergence_matrix(m, nq=None):
    """A as a sparse (N x 3N) matrix acting on [u_x; u_y; u_z]; nq points per
    direction (default k+1)."""
    T = _tables(m, nq)
    nb, N = m.n ** 3, m.ndofs
    A = _Blocks((N, 3 * N))
    for c in range(m.ncells):
        grad, Phi, w = _cell_geo(T, m, c)
        for a in range(3):
            A.add(c * nb, a * N + c * nb, grad[a].T @ (w[:, None] * Phi))
    inner, bnd = _faces(m)
    for cL, cR, d in inner:
        TrL, dA, nrm = _face_geo(T, m, cL, 2 * d + 1)
        TrR = _face_geo(T, m, cR, 2 * d)[0]
        for a in range(3):
            for (ct, Trt, sgn) in ((cL, TrL, 1.0), (cR, TrR, -1.0)):   # outward normal sgn * nrm
                for (cu, Tru) in ((cL, TrL), (cR, TrR)):
                    blk = -sgn * 0.5 * (Trt.T @ ((dA * nrm[:, a])[:, None] * Tru))
                    A.add(ct * nb, a * N + cu * nb, blk)
    for c, f in bnd:
        Tr, dA, nrm = _face_geo(T, m, c, f)
        sgn = 1.0 if f % 2 == 1 else -1.0
        for a in range(3):
            A.add(c * nb, a * N + c * nb, -sgn * (Tr.T @ ((dA * nrm[:, a])[:, None] * Tr)))
    return A.tocsr()


def gradient_matrix(m, nq=None):
    """B as a sparse (3N x N) matrix, output [B_x; B_y; B_z]; nq points per
    direction (default k+1)."""
    T = _tables(m, nq)
    nb, N = m.n ** 3, m.ndofs
    B = _Blocks((3 * N, N))
    for c in range(m.ncells):
        grad, Phi, w = _cell_geo(T, m, c)
        for a in range(3):
            B.add(a * N + c * nb, c * nb, grad[a].T @ (w[:, None] * Phi))
    inner, bnd = _faces(m)
    for cL, cR, d in inner:
        TrL, dA, nrm = _face_geo(T, m, cL, 2 * d + 1)
        TrR = _face_geo(T, m, cR, 2 * d)[0]
        for a in range(3):
            for (ct, Trt, sgn) in ((cL, TrL, 1.0), (cR, TrR, -1.0)):
                for (cp, Trp) in ((cL, TrL), (cR, TrR)):
                    blk = -sgn * 0.5 * (Trt.T @ ((dA * nrm[:, a])[:, None] * Trp))
                    B.add(a * N + ct * nb, cp * nb, blk)
    for c, f in bnd:
        Tr, dA, nrm = _face_geo(T, m, c, f)
        sgn = 1.0 if f % 2 == 1 else -1.0
        for a in range(3):
            B.add(a * N + c * nb, c * nb, -sgn * (Tr.T @ ((dA * nrm[:, a])[:, None] * Tr)))
    return B.tocsr()


def _rows(m, cells, nq, fields, lift):
    """Rows of the listed cells of A (fields = 3 -> 1) or B (1 -> 3): cell term
    and the six faces of each cell, face by face as the assembled matrices
    (interior faces with the low cell's geometry)."""
    T = _tables(m, nq)
    nb = m.n ** 3
    out = np.zeros((3 if fields == 1 else 1, len(cells), nb))
    for r, c in enumerate(cells):
        grad, Phi, w = _cell_geo(T, m, c)
        lift(out[:, r], c, [grad[a].T @ (w[:, None] * Phi) for a in range(3)], None, None)
        for f in range(6):
            d, s = divmod(f, 2)
            cn = m.neighbor(c, f)
            Tr = _face_geo(T, m, c, f)[0]
            if cn >= 0:
                _, dA, nrm = _face_geo(T, m, c if s == 1 else cn, 2 * d + 1)
                Trn = _face_geo(T, m, cn, 2 * d + 1 - s)[0]
            else:
                _, dA, nrm = _face_geo(T, m, c, f)
                Trn = None
            sgn = 1.0 if s == 1 else -1.0
            lift(out[:, r], c, None, (Tr, Trn, cn, dA, sgn * nrm), None)
    return out


def divergence_cells(m, u, cells, nq=None):
    """(A u) on the rows of the listed cells, shape (len(cells), n^3)."""
    U = np.asarray(u, dtype=np.float64).reshape(3, m.ncells, -1)

    def lift(o, c, cellblk, face, _):
        if cellblk is not None:
            o[0] += sum(cellblk[a] @ U[a, c] for a in range(3))
            return
        Tr, Trn, cn, dA, nout = face
        avg = [Tr @ U[a, c] if Trn is None else 0.5 * (Tr @ U[a, c] + Trn @ U[a, cn]) for a in range(3)]
        o[0] -= Tr.T @ (dA * sum(nout[:, a] * avg[a] for a in range(3)))

    return _rows(m, cells, nq, 3, lift)[0]


def gradient_cells(m, p, cells, nq=None):
    """(B p) on the rows of the listed cells, shape (3, len(cells), n^3)."""
    P = np.asarray(p, dtype=np.float64).reshape(m.ncells, -1)

    def lift(o, c, cellblk, face, _):
        if cellblk is not None:
            for a in range(3):
                o[a] += cellblk[a] @ P[c]
            return
        Tr, Trn, cn, dA, nout = face
        avg = Tr @ P[c] if Trn is None else 0.5 * (Tr @ P[c] + Trn @ P[cn])
        for a in range(3):
            o[a] -= Tr.T @ (dA * nout[:, a] * avg)

    return _rows(m, cells, nq, 1, lift)


def mass_apply(m, v):
    """M v for scalar fields stacked [n_fields][N] (flattened)."""
    T = sipg.Tables(m.k)
    nb = m.n ** 3
    V = np.asarray(v, dtype=np.float64).reshape(-1, m.ncells, nb)
    out = np.empty_like(V)
    for c in range(m.ncells):
        M = sipg.cell_matrices(T, m.jacobian(c))[1]
        out[:, c] = V[:, c] @ M.T
    return out.ravel()


def divdiv_cell(T, J):
    """D_e (3 n^3 x 3 n^3): (div v, div u)_K, blocks [a][b] = (d_a phi_i, d_b phi_j)."""
    grad, _, w = _cell_grad(T, J)
    return np.block([[grad[a].T @ (w[:, None] * grad[b]) for b in range(3)] for a in range(3)])


def cell_mass_divdiv(m, c, nq=None):
    """(M_e, D_e) of cell c with per-point Jacobians (curved cells, Sec. 5):
    M_e = (phi_i, phi_j)_K, D_e = (div v, div u)_K in [a][b] blocks."""
    T = _tables(m, nq)
    grad, Phi, w = _cell_geo(T, m, c)
    M = Phi.T @ (w[:, None] * Phi)
    D = np.block([[grad[a].T @ (w[:, None] * grad[b]) for b in range(3)] for a in range(3)])
    return M, D


def _weights_volume(m, c):
    """Integral weights of the cell's basis functions and the cell volume."""
    if not _curved(m):
        return None, m.volume(c)
    T = sipg.Tables(m.k)
    _, Phi, w = _cell_geo(T, m, c)
    return Phi.T @ w, w.sum()


def penalty_tau(m, u, zeta, dt):
    """tau_D per cell = zeta |u_bar| V^(1/3) dt, u_bar the cell average of the velocity [3][N]."""
    wts = None if _curved(m) else sipg.integral_weights(m).reshape(m.ncells, -1)
    U = np.asarray(u, dtype=np.float64).reshape(3, m.ncells, -1)
    tau = np.empty(m.ncells)
    for c in range(m.ncells):
        wc, V = _weights_volume(m, c)
        if wc is None:
            wc = wts[c]
        ubar = np.array([wc @ U[a, c] for a in range(3)]) / V
        tau[c] = zeta * np.linalg.norm(ubar) * V ** (1.0 / 3.0) * dt
    return tau


def projection_solve(m, tau, rhs, cells=None):
    """Per cell (M_e (x) I_3 + tau_e D_e) x_e = rhs_e; rhs and result [3][N] (or the listed cells, (3, len, n^3))."""
    T = sipg.Tables(m.k)
    nb = m.n ** 3
    cl = range(m.ncells) if cells is None else list(cells)
    R = np.asarray(rhs, dtype=np.float64).reshape(3, -1, nb)
    out = np.zeros((3, len(cl), nb))
    for r, c in enumerate(cl):
        if _curved(m):
            M, D = cell_mass_divdiv(m, c)
        else:
            J = m.jacobian(c)
            M, D = sipg.cell_matrices(T, J)[1], divdiv_cell(T, J)
        Ae = np.kron(np.eye(3), M) + tau[c] * D
        src = R[:, c] if cells is None else R[:, r]
        out[:, r] = np.linalg.solve(Ae, src.ravel()).reshape(3, nb)
    return out.ravel() if cells is None else out
