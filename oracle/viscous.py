"""Viscous operator in the symmetric-gradient form (oracle; test infrastructure).

Sec. 3.2, implicit viscous step, with s = 1 (SIPG) and F^nu(u) = 2 nu eps(u),
eps(u) = (grad u + grad u^T)/2, homogeneous Dirichlet data on Dirichlet faces
(g_u = 0) and homogeneous Neumann data (h = 0, g_p = 0) on Neumann faces:

  a(v, u) = mu (v, u) + sum_K (eps(v), 2 nu eps(u))_K
          - sum_F ({{2 nu eps(v)}}, [u] (x) n)_F - sum_F ([v], {{2 nu eps(u)}} n)_F
          + sum_F tau nu ([v], [u])_F,

on interior faces with n the unit normal of the minus side and [w] = w- - w+;
on a Dirichlet face the averages are the own values, [w] = w, and the penalty
is 2 tau nu; a Neumann face adds nothing (U* = u_h there, so the first face
term vanishes, and the flux F^nu* is data, which belongs to the right-hand
side).  tau is the SIPG penalty of eqs. taue/tau.  Cell and face integrals by
Gauss quadrature with k+1 points, dense blocks from Kronecker evaluation
matrices, assembled into a sparse 3N x 3N matrix acting on [u_x; u_y; u_z].
"""
import numpy as np
import scipy.sparse as sp

from . import sipg


def _face_grads(T, J, f):
    """Trace Tr, physical gradient matrices grad[a] at the face points, dA, unit normal towards +d."""
    d, s = divmod(f, 2)
    Jinv = np.linalg.inv(J)
    detJ = abs(np.linalg.det(J))
    m = Jinv.T[:, d]
    nrm = m / np.linalg.norm(m)
    val = [T.S, T.S, T.S]
    val[d] = T.e[s]
    Tr = sipg._kron3(val[2], val[1], val[0])
    G = []
    for b in range(3):
        mats = [T.S, T.S, T.S]
        mats[d] = T.e[s]
        mats[b] = T.de[s] if b == d else T.D
        G.append(sipg._kron3(mats[2], mats[1], mats[0]))
    grad = [sum(Jinv[b, a] * G[b] for b in range(3)) for a in range(3)]
    wt = [T.wq, T.wq, T.wq]
    wt[d] = np.ones(1)
    dA = sipg._kron3(wt[2], wt[1], wt[0]) * detJ * np.linalg.norm(m)
    return Tr, grad, dA, nrm


def _cell_block(T, J, mu, nu):
    """[c][c'] = mu delta M + nu (delta sum_a G_a^T W G_a + G_c'^T W G_c)."""
    Phi = sipg._kron3(T.S, T.S, T.S)
    G = sipg._ref_gradients_cell(T)
    Jinv = np.linalg.inv(J)
    grad = [sum(Jinv[b, a] * G[b] for b in range(3)) for a in range(3)]
    w = sipg._kron3(T.wq, T.wq, T.wq) * abs(np.linalg.det(J))
    M = Phi.T @ (w[:, None] * Phi)
    K = sum(grad[a].T @ (w[:, None] * grad[a]) for a in range(3))
    blk = [[None] * 3 for _ in range(3)]
    for c in range(3):
        for cp in range(3):
            B = nu * (grad[cp].T @ (w[:, None] * grad[c]))
            if c == cp:
                B = B + mu * M + nu * K
            blk[c][cp] = B
    return blk


def _face_terms(Tv, gradv, Tu, gradu, W, n, nu, pen):
    """Boundary-face blocks [c][c'] of -(2nu eps(v), u (x) n) - (v, 2nu eps(u) n) + pen (v, u)
    (own traces and gradients, n the outward normal)."""
    Gnv = sum(n[a] * gradv[a] for a in range(3))
    Gnu = sum(n[a] * gradu[a] for a in range(3))
    blk = [[None] * 3 for _ in range(3)]
    for c in range(3):
        for cp in range(3):
            B = -nu * (n[c] * (gradv[cp].T @ (W[:, None] * Tu)) + n[cp] * (Tv.T @ (W[:, None] * gradu[c])))
            if c == cp:
                B = B - nu * (Gnv.T @ (W[:, None] * Tu) + Tv.T @ (W[:, None] * Gnu)) + pen * (Tv.T @ (W[:, None] * Tu))
            blk[c][cp] = B
    return blk


def viscous_matrix(m, mu, nu, penalty_scale=1.0):
    """Sparse 3N x 3N matrix of a(v, u)."""
    T = sipg.Tables(m.k)
    nb, N = m.n ** 3, m.ndofs
    tau = sipg.penalty_per_cell(m, penalty_scale)
    rows, cols, vals = [], [], []

    def add(c, cell_r, cp, cell_c, B):
        r = c * N + cell_r * nb + np.arange(nb)
        cc = cp * N + cell_c * nb + np.arange(nb)
        R, Cc = np.meshgrid(r, cc, indexing="ij")
        rows.append(R.ravel())
        cols.append(Cc.ravel())
        vals.append(B.ravel())

    for cell in range(m.ncells):
        blk = _cell_block(T, m.jacobian(cell), mu, nu)
        for c in range(3):
            for cp in range(3):
                add(c, cell, cp, cell, blk[c][cp])
    for cL, cR, d in m.interior_faces():
        TrL, gL, dA, nrm = _face_grads(T, m.jacobian(cL), 2 * d + 1)
        TrR, gR, _, _ = _face_grads(T, m.jacobian(cR), 2 * d)
        pen = nu * max(tau[cL], tau[cR])
        sides = ((cL, TrL, gL, 1.0), (cR, TrR, gR, -1.0))   # jump sign of each side
        for (cv, Tv, gv, sv) in sides:
            for (cu, Tu, gu, su) in sides:
                blk = _interior_pair(Tv, gv, sv, Tu, gu, su, dA, nrm, nu, pen)
                for c in range(3):
                    for cp in range(3):
                        add(c, cv, cp, cu, blk[c][cp])
    for cell, f in m.boundary_faces():
        Tr, g, dA, nrm = _face_grads(T, m.jacobian(cell), f)
        n_out = nrm if f % 2 == 1 else -nrm
        blk = _face_terms(Tr, g, Tr, g, dA, n_out, nu, 2.0 * nu * tau[cell])
        for c in range(3):
            for cp in range(3):
                add(c, cell, cp, cell, blk[c][cp])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * N, 3 * N))
    return A.tocsr()


def _interior_pair(Tv, gv, sv, Tu, gu, su, W, n, nu, pen):
    """Interior-face blocks between a test side (sign sv in [v]) and a trial side (su in [u]):
    -({{2nu eps(v)}}, [u] (x) n) takes 1/2 of the test side's eps and the trial side's jump;
    -([v], {{2nu eps(u)}} n) the test side's jump and 1/2 of the trial side's eps."""
    Gnv = sum(n[a] * gv[a] for a in range(3))
    Gnu = sum(n[a] * gu[a] for a in range(3))
    blk = [[None] * 3 for _ in range(3)]
    for c in range(3):
        for cp in range(3):
            B = -nu * (0.5 * su * n[c] * (gv[cp].T @ (W[:, None] * Tu))
                       + 0.5 * sv * n[cp] * (Tv.T @ (W[:, None] * gu[c])))
            if c == cp:
                B = B - nu * (0.5 * su * (Gnv.T @ (W[:, None] * Tu)) + 0.5 * sv * (Tv.T @ (W[:, None] * Gnu)))
                B = B + pen * sv * su * (Tv.T @ (W[:, None] * Tu))
            blk[c][cp] = B
    return blk


def viscous_apply_cells(m, U, cells, mu, nu, penalty_scale=1.0):
    """(H U) restricted to the rows of the listed cells, shape (3, len(cells), n^3).

    The same blocks as ``viscous_matrix``, built for each listed cell from its
    own cell integral and its six faces (blocks cached by geometry), so that
    sampled rows of full-size meshes can be checked without assembling."""
    T = sipg.Tables(m.k)
    nb = m.n ** 3
    tau = sipg.penalty_per_cell(m, penalty_scale)
    Uc = U.reshape(3, m.ncells, nb)
    cache = {}

    def key(*arrs):
        return tuple(np.round(np.concatenate([np.ravel(a) for a in arrs]), 15).tolist())

    def mult(blk, V):
        return np.stack([sum(blk[c][cp] @ V[cp] for cp in range(3)) for c in range(3)])

    out = np.zeros((3, len(cells), nb))
    for r, cell in enumerate(cells):
        J = m.jacobian(cell)
        kc = ("cell", key(J))
        if kc not in cache:
            cache[kc] = _cell_block(T, J, mu, nu)
        y = mult(cache[kc], Uc[:, cell])
        for f in range(6):
            d, s = divmod(f, 2)
            cn = m.neighbor(cell, f)
            if cn < 0:
                if m.neumann[f]:
                    continue
                kb = ("bnd", f, key(J, [tau[cell]]))
                if kb not in cache:
                    Tr, g, dA, nrm = _face_grads(T, J, f)
                    n_out = nrm if s == 1 else -nrm
                    cache[kb] = _face_terms(Tr, g, Tr, g, dA, n_out, nu, 2.0 * nu * tau[cell])
                y += mult(cache[kb], Uc[:, cell])
                continue
            cL, cR = (cell, cn) if s == 1 else (cn, cell)
            JL, JR = m.jacobian(cL), m.jacobian(cR)
            pen = nu * max(tau[cL], tau[cR])
            kf = ("int", d, s, key(JL, JR, [pen]))
            if kf not in cache:
                TrL, gL, dA, nrm = _face_grads(T, JL, 2 * d + 1)
                TrR, gR, _, _ = _face_grads(T, JR, 2 * d)
                sideL, sideR = (TrL, gL, 1.0), (TrR, gR, -1.0)
                own, other = (sideL, sideR) if s == 1 else (sideR, sideL)
                cache[kf] = (_interior_pair(*own, *own, dA, nrm, nu, pen),
                             _interior_pair(*own, *other, dA, nrm, nu, pen))
            b_own, b_other = cache[kf]
            y += mult(b_own, Uc[:, cell]) + mult(b_other, Uc[:, cn])
        out[:, r] = y
    return out


# ---------------------------------------------------------------- curved cells
# The same bilinear form on iso-parametric curved cells (Sec. 5): the Jacobian,
# and with it the physical gradients, the unit normal and the surface measure,
# are taken at every quadrature point (k+1 Gauss points per direction on
# cells and faces), and tau_e comes from the curved areas and volumes (the
# penalty of the curved SIPG oracle).  The blocks are those above with the
# normal moved inside the point sums.

def _pair_pts(Tv, gv, sv, Tu, gu, su, W, n, nu, pen):
    """_interior_pair with a normal n (m, 3) that varies over the face points."""
    Gnv = sum(n[:, a][:, None] * gv[a] for a in range(3))
    Gnu = sum(n[:, a][:, None] * gu[a] for a in range(3))
    blk = [[None] * 3 for _ in range(3)]
    for c in range(3):
        for cp in range(3):
            B = -nu * (0.5 * su * (gv[cp].T @ ((W * n[:, c])[:, None] * Tu))
                       + 0.5 * sv * (Tv.T @ ((W * n[:, cp])[:, None] * gu[c])))
            if c == cp:
                B = B - nu * (0.5 * su * (Gnv.T @ (W[:, None] * Tu)) + 0.5 * sv * (Tv.T @ (W[:, None] * Gnu)))
                B = B + pen * sv * su * (Tv.T @ (W[:, None] * Tu))
            blk[c][cp] = B
    return blk


def _bnd_pts(Tr, g, W, n, nu, pen):
    """_face_terms (own traces on both sides of the form) with a per-point outward normal n (m, 3)."""
    Gn = sum(n[:, a][:, None] * g[a] for a in range(3))
    blk = [[None] * 3 for _ in range(3)]
    for c in range(3):
        for cp in range(3):
            B = -nu * ((g[cp].T @ ((W * n[:, c])[:, None] * Tr)) + (Tr.T @ ((W * n[:, cp])[:, None] * g[c])))
            if c == cp:
                B = B - nu * (Gn.T @ (W[:, None] * Tr) + Tr.T @ (W[:, None] * Gn)) + pen * (Tr.T @ (W[:, None] * Tr))
            blk[c][cp] = B
    return blk


class CurvedViscous:
    """The symmetric-gradient viscous operator on a CurvedBoxMesh, point by point."""

    def __init__(self, mesh, mass_coeff, diff_coeff, penalty_scale=1.0, cells=None):
        from .curved import CurvedSIPG
        self.mesh = mesh
        self.mu, self.nu = float(mass_coeff), float(diff_coeff)
        # tables, face geometry and tau_e (curved areas and volumes) of the scalar operator
        self.s = CurvedSIPG(mesh, mass_coeff, diff_coeff, penalty_scale, cells=cells)

    def cell_block(self, c):
        from .curved import _phys_grads
        s, m = self.s, self.mesh
        J = m.jac_at(c, s.xq_cell)
        w = s.wq_cell * np.abs(np.linalg.det(J))
        grad = _phys_grads(s.Gref, np.linalg.inv(J))
        M = s.Phi.T @ (w[:, None] * s.Phi)
        K = sum(g.T @ (w[:, None] * g) for g in grad)
        blk = [[None] * 3 for _ in range(3)]
        for c1 in range(3):
            for c2 in range(3):
                B = self.nu * (grad[c2].T @ (w[:, None] * grad[c1]))
                if c1 == c2:
                    B = B + self.mu * M + self.nu * K
                blk[c1][c2] = B
        return blk

    def face_pairs(self, cL, cR, d):
        """{(test side, trial side): blocks} for sides 'L' and 'R' of an interior face (normal of L)."""
        s = self.s
        TrL, gL, dA, nL = s.face(cL, 2 * d + 1)
        TrR, gR, _, _ = s.face(cR, 2 * d)
        pen = self.nu * max(s.tau_e[cL], s.tau_e[cR])
        sides = {"L": (TrL, gL, 1.0), "R": (TrR, gR, -1.0)}
        return {(a, b): _pair_pts(*sides[a], *sides[b], dA, nL, self.nu, pen) for a in "LR" for b in "LR"}

    def bface_block(self, c, f):
        Tr, g, dA, nrm = self.s.face(c, f)
        n_out = nrm if f % 2 == 1 else -nrm
        return _bnd_pts(Tr, g, dA, n_out, self.nu, 2.0 * self.nu * self.s.tau_e[c])

    def assemble(self):
        m = self.mesh
        nb, N = m.n ** 3, m.ndofs
        rows, cols, vals = [], [], []

        def add(cell_r, cell_c, blk):
            for c1 in range(3):
                for c2 in range(3):
                    r = c1 * N + cell_r * nb + np.arange(nb)
                    cc = c2 * N + cell_c * nb + np.arange(nb)
                    R, C = np.meshgrid(r, cc, indexing="ij")
                    rows.append(R.ravel())
                    cols.append(C.ravel())
                    vals.append(blk[c1][c2].ravel())

        for cell in range(m.ncells):
            add(cell, cell, self.cell_block(cell))
        for cL, cR, d in m.interior_faces():
            P = self.face_pairs(cL, cR, d)
            idx = {"L": cL, "R": cR}
            for (a, b), blk in P.items():
                add(idx[a], idx[b], blk)
        for cell, f in m.boundary_faces():
            add(cell, cell, self.bface_block(cell, f))
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * N, 3 * N))
        return A.tocsr()

    def apply_cells(self, U, cells):
        """(H U) on the rows of the listed cells, shape (3, len(cells), n^3)."""
        m = self.mesh
        nb = m.n ** 3
        Uc = U.reshape(3, m.ncells, nb)

        def mult(blk, V):
            return np.stack([sum(blk[c][cp] @ V[cp] for cp in range(3)) for c in range(3)])

        out = np.zeros((3, len(cells), nb))
        for r, cell in enumerate(cells):
            y = mult(self.cell_block(cell), Uc[:, cell])
            for f in range(6):
                d, s = divmod(f, 2)
                cn = m.neighbor(cell, f)
                if cn < 0:
                    if not m.neumann[f]:
                        y += mult(self.bface_block(cell, f), Uc[:, cell])
                    continue
                if s == 1:
                    P = self.face_pairs(cell, cn, d)
                    y += mult(P[("L", "L")], Uc[:, cell]) + mult(P[("L", "R")], Uc[:, cn])
                else:
                    P = self.face_pairs(cn, cell, d)
                    y += mult(P[("R", "R")], Uc[:, cell]) + mult(P[("R", "L")], Uc[:, cn])
            out[:, r] = y
        return out
