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
affine cells), built from dense Kronecker-product evaluation matrices.
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


def _faces(m):
    """Interior faces (cL, cR, d) and boundary faces (c, f), Dirichlet and Neumann alike:
    the ND average is the own trace on both boundary parts (Sec. 3.1)."""
    return m.interior_faces(), sorted(m.boundary_faces() + m.neumann_faces())


def divergence_matrix(m):
    """A as a sparse (N x 3N) matrix acting on [u_x; u_y; u_z]."""
    T = sipg.Tables(m.k)
    nb, N = m.n ** 3, m.ndofs
    A = sp.lil_matrix((N, 3 * N))
    loc = np.arange(nb)
    for c in range(m.ncells):
        grad, Phi, w = _cell_grad(T, m.jacobian(c))
        for a in range(3):
            A[np.ix_(c * nb + loc, a * N + c * nb + loc)] += grad[a].T @ (w[:, None] * Phi)
    inner, bnd = _faces(m)
    for cL, cR, d in inner:
        TrL, _, dA, nrm = sipg.face_eval(T, m.jacobian(cL), 2 * d + 1)
        TrR, _, _, _ = sipg.face_eval(T, m.jacobian(cR), 2 * d)
        for a in range(3):
            for (ct, Trt, sgn) in ((cL, TrL, 1.0), (cR, TrR, -1.0)):   # outward normal sgn * nrm
                for (cu, Tru) in ((cL, TrL), (cR, TrR)):
                    blk = -sgn * 0.5 * nrm[a] * (Trt.T @ (dA[:, None] * Tru))
                    A[np.ix_(ct * nb + loc, a * N + cu * nb + loc)] += blk
    for c, f in bnd:
        Tr, _, dA, nrm = sipg.face_eval(T, m.jacobian(c), f)
        sgn = 1.0 if f % 2 == 1 else -1.0
        for a in range(3):
            A[np.ix_(c * nb + loc, a * N + c * nb + loc)] += -sgn * nrm[a] * (Tr.T @ (dA[:, None] * Tr))
    return A.tocsr()


def gradient_matrix(m):
    """B as a sparse (3N x N) matrix, output [B_x; B_y; B_z]."""
    T = sipg.Tables(m.k)
    nb, N = m.n ** 3, m.ndofs
    B = sp.lil_matrix((3 * N, N))
    loc = np.arange(nb)
    for c in range(m.ncells):
        grad, Phi, w = _cell_grad(T, m.jacobian(c))
        for a in range(3):
            B[np.ix_(a * N + c * nb + loc, c * nb + loc)] += grad[a].T @ (w[:, None] * Phi)
    inner, bnd = _faces(m)
    for cL, cR, d in inner:
        TrL, _, dA, nrm = sipg.face_eval(T, m.jacobian(cL), 2 * d + 1)
        TrR, _, _, _ = sipg.face_eval(T, m.jacobian(cR), 2 * d)
        for a in range(3):
            for (ct, Trt, sgn) in ((cL, TrL, 1.0), (cR, TrR, -1.0)):
                for (cp, Trp) in ((cL, TrL), (cR, TrR)):
                    blk = -sgn * 0.5 * nrm[a] * (Trt.T @ (dA[:, None] * Trp))
                    B[np.ix_(a * N + ct * nb + loc, cp * nb + loc)] += blk
    for c, f in bnd:
        Tr, _, dA, nrm = sipg.face_eval(T, m.jacobian(c), f)
        sgn = 1.0 if f % 2 == 1 else -1.0
        for a in range(3):
            B[np.ix_(a * N + c * nb + loc, c * nb + loc)] += -sgn * nrm[a] * (Tr.T @ (dA[:, None] * Tr))
    return B.tocsr()


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


def penalty_tau(m, u, zeta, dt):
    """tau_D per cell = zeta |u_bar| V^(1/3) dt, u_bar the cell average of the velocity [3][N]."""
    wts = sipg.integral_weights(m).reshape(m.ncells, -1)
    U = np.asarray(u, dtype=np.float64).reshape(3, m.ncells, -1)
    tau = np.empty(m.ncells)
    for c in range(m.ncells):
        V = m.volume(c)
        ubar = np.array([wts[c] @ U[a, c] for a in range(3)]) / V
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
        J = m.jacobian(c)
        M = sipg.cell_matrices(T, J)[1]
        Ae = np.kron(np.eye(3), M) + tau[c] * divdiv_cell(T, J)
        src = R[:, c] if cells is None else R[:, r]
        out[:, r] = np.linalg.solve(Ae, src.ravel()).reshape(3, nb)
    return out.ravel() if cells is None else out
