"""Convective operator with local Lax-Friedrichs flux (oracle; test infrastructure).

Paper Sec. 3.2, explicit convective step (eq. convstepspat and the flux
definition after it) and its matrix form eq. advect (Sec. 4.4).  For the
velocity U (three components, each in the scalar DG space) the operator is

  C(U)_{i,a} = - sum_K (d_b phi_i, u_a u_b)_K + sum_K (phi_i, R_a)_{dK},

R = F*(u-, u+) n with n the outward normal of K:
  R = 1/2 (u- (u-.n) + u+ (u+.n)) + lam (u- - u+),  lam = max(|u-.n|, |u+.n|)
(Lambda/2 of the paper, evaluated at every face quadrature point).  On
Dirichlet faces the exterior state is the mirror u+ = 2 g - u-, which gives
the paper's Dirichlet flux; on outflow (Neumann) faces it is u+ = u-, which
gives the paper's flux F^c(u-).n there (no Lax-Friedrichs term).  C equals F^c(U) of eq. advect, so the explicit
update is gamma_0 U^ = sum alpha U - dt M^{-1} C + F.

Integrals use Gauss quadrature with n_q points per direction on cells and
tangentially on faces (Sec. 5 over-integration; default floor(3(k+1)/2)).
Dense per-cell evaluation matrices, no sum factorisation; fp64.  On curved
(iso-parametric) cells, Sec. 5, the Jacobian of the cell map is taken at
every cell and face quadrature point, with face normals and surface measures
from Nanson's formula; the flux is written for a normal per face point.

The vector-Jacobian product is not in the paper; it is the exact transpose of
the derivative of C (piecewise quadratic in U), with the tie rule: the minus
side is active in the max when |u-.n| >= |u+.n|, and sgn(0) = 0.
  cell:  g_{j,c} = - (phi_j, (u.grad) w_c + sum_a u_a d_c w_a)_K
  faces: the face contributes int [w].R, hence g- += phi- J-^T [w], g+ += phi+ J+^T [w],
         J- = 1/2((u-.n) I + u- (x) n) + lam I + (u- - u+) (x) dlam/du-,
         J+ = 1/2((u+.n) I + u+ (x) n) - lam I + (u- - u+) (x) dlam/du+;
  Dirichlet faces: g- += phi- (J- - J+)^T w-;  outflow faces: g- += phi- (J- + J+)^T w-.

Pins (tests/test_oracle_convective.py): free stream, conservation,
homogeneity of degree 2, Lax-Friedrichs dissipation identity, quadrature
invariance with lam = 0, channel profile; JVP against central differences,
VJP against the transpose of the brute-force Jacobian, Euler identity; with
outflow sides (tests/test_oracle_conv_outflow.py): a constant field gives
C = 0 exactly, JVP against central differences, VJP against the Jacobian; on
curved cells (tests/test_oracle_conv_curved.py): zero amplitude gives the
affine operator, free-stream preservation (exact quadrature of the cofactor
integrands), conservation, order-k consistency with div(u (x) u), JVP, VJP
and the Euler identity.
"""
import numpy as np

from . import basis
from .sipg import _kron3


class Convective:
    def __init__(self, mesh, nq=None, g=None):
        self.mesh = mesh
        k = mesh.k
        self.n = k + 1
        self.nq = basis.default_conv_points(k) if nq is None else int(nq)
        nodes = basis.gll_nodes(k)
        self.xq, self.wq = basis.gauss_rule(self.nq)
        S = basis.lagrange_values(nodes, self.xq)
        D = basis.lagrange_derivatives(nodes, self.xq)
        self.S, self.D = S, D
        self.Phi = _kron3(S, S, S)
        self.Gref = [_kron3(S, S, D), _kron3(S, D, S), _kron3(D, S, S)]
        self.wcell = _kron3(self.wq, self.wq, self.wq)
        e = [basis.lagrange_values(nodes, [s]) for s in (0.0, 1.0)]
        self.Tr = []
        for f in range(6):
            d, s = divmod(f, 2)
            mats = [S, S, S]
            mats[d] = e[s]
            self.Tr.append(_kron3(mats[2], mats[1], mats[0]))
        wt = []
        for d in range(3):
            w3 = [self.wq, self.wq, self.wq]
            w3[d] = np.ones(1)
            wt.append(_kron3(w3[2], w3[1], w3[0]))
        self.wface = wt
        self.g = g      # Dirichlet velocity callable (x,y,z) -> (3, m); None means g = 0

    # -- geometry helpers ------------------------------------------------------
    # Affine cells have one Jacobian; curved (iso-parametric) cells, meshes
    # with a ``jac_at`` method, take the Jacobian of their map at every
    # quadrature point (Sec. 5: the cell geometry enters through the Jacobian
    # at each point).  Face normals follow Nanson's formula n dA = det J J^{-T}
    # N_ref dA_ref, per point.
    def _curved(self):
        return hasattr(self.mesh, "jac_at")

    def _face_ref(self, d, s):
        axes = [self.xq, self.xq, self.xq]
        axes[d] = np.array([float(s)])
        Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def _cell_geo(self, c):
        if self._curved():
            Z, Y, X = np.meshgrid(self.xq, self.xq, self.xq, indexing="ij")
            J = self.mesh.jac_at(c, np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
            Jinv = np.linalg.inv(J)
            detJ = np.abs(np.linalg.det(J))
            Gphys = [sum(Jinv[:, b, a][:, None] * self.Gref[b] for b in range(3)) for a in range(3)]
            return Gphys, self.wcell * detJ
        J = self.mesh.jacobian(c)
        Jinv = np.linalg.inv(J)
        detJ = abs(np.linalg.det(J))
        Gphys = [sum(Jinv[b, a] * self.Gref[b] for b in range(3)) for a in range(3)]
        return Gphys, self.wcell * detJ

    def _face_geo(self, c, d, s):
        """Unit normal along +xi_d (3, m) and surface weights (m,) of face (d, s) of cell c."""
        mq = self.nq ** 2
        if self._curved():
            J = self.mesh.jac_at(c, self._face_ref(d, s))
            Jinv = np.linalg.inv(J)
            m = Jinv[:, d, :].T                                   # (3, mq): J^{-T} e_d
            nm = np.linalg.norm(m, axis=0)
            return m / nm, self.wface[d] * np.abs(np.linalg.det(J)) * nm
        J = self.mesh.jacobian(c)
        Jinv = np.linalg.inv(J)
        m = Jinv.T[:, d]
        nrm = m / np.linalg.norm(m)
        dA = self.wface[d] * abs(np.linalg.det(J)) * np.linalg.norm(m)
        return np.repeat(nrm[:, None], mq, axis=1), dA

    def _face_points(self, c, f):
        d, s = divmod(f, 2)
        ref = self._face_ref(d, s)
        if self._curved():
            return self.mesh.map_at(c, ref)
        o, _ = self.mesh.cell_origin_h(c)
        x0 = o if self.mesh.shear is None else self.mesh.shear @ o
        return x0 + ref @ self.mesh.jacobian(c).T

    def _gvals(self, c, f):
        m = self.nq ** 2
        if self.g is None:
            return np.zeros((3, m))
        X = self._face_points(c, f)
        return np.asarray(self.g(X[:, 0], X[:, 1], X[:, 2]), dtype=np.float64).reshape(3, m)

    # -- flux and its derivative -------------------------------------------------
    @staticmethod
    def flux(um, up, n, lam_on=True):
        """R(u-, u+; n) at face points; um, up and the unit normals n have shape (3, m)."""
        a = np.sum(n * um, axis=0)
        b = np.sum(n * up, axis=0)
        R = 0.5 * (um * a + up * b)
        if lam_on:
            lam = np.maximum(np.abs(a), np.abs(b))
            R = R + lam * (um - up)
        return R

    @staticmethod
    def flux_jac_T(um, up, n, w):
        """(J-^T w, J+^T w) at each face point, with the tie rule of the module doc."""
        a = np.sum(n * um, axis=0)
        b = np.sum(n * up, axis=0)
        lam = np.maximum(np.abs(a), np.abs(b))
        minus_active = np.abs(a) >= np.abs(b)
        dlm = np.where(minus_active, np.sign(a), 0.0)[None, :] * n
        dlp = np.where(minus_active, 0.0, np.sign(b))[None, :] * n
        jump_u_w = np.sum((um - up) * w, axis=0)
        Jm = 0.5 * (a * w + n * np.sum(um * w, axis=0)) + lam * w + dlm * jump_u_w
        Jp = 0.5 * (b * w + n * np.sum(up * w, axis=0)) - lam * w + dlp * jump_u_w
        return Jm, Jp

    @staticmethod
    def flux_jvp(um, up, n, dum, dup):
        a = np.sum(n * um, axis=0)
        b = np.sum(n * up, axis=0)
        da = np.sum(n * dum, axis=0)
        db = np.sum(n * dup, axis=0)
        lam = np.maximum(np.abs(a), np.abs(b))
        minus_active = np.abs(a) >= np.abs(b)
        dlam = np.where(minus_active, np.sign(a) * da, np.sign(b) * db)
        return 0.5 * (dum * a + um * da + dup * b + up * db) + dlam * (um - up) + lam * (dum - dup)

    # -- operator, row-restricted ------------------------------------------------
    def _cells(self, U, cells):
        nb = self.n ** 3
        return U.reshape(3, self.mesh.ncells, nb)

    def forward_cells(self, U, cells, lam_on=True):
        """C(U) restricted to the listed cells: shape (3, len(cells), n^3)."""
        m = self.mesh
        V = self._cells(U, cells)
        out = np.zeros((3, len(cells), self.n ** 3))
        for r, c in enumerate(cells):
            Gphys, w = self._cell_geo(c)
            uq = self.Phi @ V[:, c, :].T                      # (nq^3, 3)
            for a in range(3):
                out[a, r] -= sum(Gphys[b].T @ (w * uq[:, a] * uq[:, b]) for b in range(3))
            for f in range(6):
                d, s = divmod(f, 2)
                cn = m.neighbor(c, f)
                if cn < 0:
                    nrm, dA = self._face_geo(c, d, s)
                    nout = nrm if s == 1 else -nrm
                    um = (self.Tr[f] @ V[:, c, :].T).T
                    # outflow (Neumann) face: the flux of the own trace, F^c(u-).n
                    up = um if m.neumann[f] else 2.0 * self._gvals(c, f) - um
                    R = self.flux(um, up, nout, lam_on)
                    out[:, r] += (self.Tr[f].T @ (dA * R).T).T
                elif s == 1:
                    nrm, dA = self._face_geo(c, d, 1)
                    um = (self.Tr[2 * d + 1] @ V[:, c, :].T).T
                    up = (self.Tr[2 * d] @ V[:, cn, :].T).T
                    R = self.flux(um, up, nrm, lam_on)
                    out[:, r] += (self.Tr[f].T @ (dA * R).T).T
                else:
                    nrm, dA = self._face_geo(cn, d, 1)
                    um = (self.Tr[2 * d + 1] @ V[:, cn, :].T).T
                    up = (self.Tr[2 * d] @ V[:, c, :].T).T
                    R = self.flux(um, up, nrm, lam_on)
                    out[:, r] -= (self.Tr[f].T @ (dA * R).T).T
        return out

    def forward(self, U, lam_on=True):
        return self.forward_cells(U, range(self.mesh.ncells), lam_on).reshape(3, -1).ravel()

    def jvp(self, U, dU):
        """Directional derivative dC(U)[dU] (full vector)."""
        m = self.mesh
        V = self._cells(U, None)
        dV = self._cells(dU, None)
        nb = self.n ** 3
        out = np.zeros((3, m.ncells, nb))
        for c in range(m.ncells):
            Gphys, w = self._cell_geo(c)
            uq = self.Phi @ V[:, c, :].T
            duq = self.Phi @ dV[:, c, :].T
            for a in range(3):
                out[a, c] -= sum(Gphys[b].T @ (w * (duq[:, a] * uq[:, b] + uq[:, a] * duq[:, b]))
                                 for b in range(3))
            for f in range(6):
                d, s = divmod(f, 2)
                cn = m.neighbor(c, f)
                if cn < 0:
                    nrm, dA = self._face_geo(c, d, s)
                    nout = nrm if s == 1 else -nrm
                    um = (self.Tr[f] @ V[:, c, :].T).T
                    dum = (self.Tr[f] @ dV[:, c, :].T).T
                    up = um if m.neumann[f] else 2.0 * self._gvals(c, f) - um
                    dR = self.flux_jvp(um, up, nout, dum, dum if m.neumann[f] else -dum)
                    out[:, c] += (self.Tr[f].T @ (dA * dR).T).T
                    continue
                L, R_ = (c, cn) if s == 1 else (cn, c)
                nrm, dA = self._face_geo(L, d, 1)
                um = (self.Tr[2 * d + 1] @ V[:, L, :].T).T
                up = (self.Tr[2 * d] @ V[:, R_, :].T).T
                dum = (self.Tr[2 * d + 1] @ dV[:, L, :].T).T
                dup = (self.Tr[2 * d] @ dV[:, R_, :].T).T
                dR = self.flux_jvp(um, up, nrm, dum, dup)
                sign = 1.0 if s == 1 else -1.0
                out[:, c] += sign * (self.Tr[f].T @ (dA * dR).T).T
        return out.ravel()

    def vjp_cells(self, U, W, cells):
        """(dC/dU)^T W restricted to the listed cells: shape (3, len(cells), n^3)."""
        m = self.mesh
        V = self._cells(U, None)
        Wc = self._cells(W, None)
        out = np.zeros((3, len(cells), self.n ** 3))
        for r, c in enumerate(cells):
            Gphys, w = self._cell_geo(c)
            uq = self.Phi @ V[:, c, :].T                                   # (q, a)
            gw = np.stack([np.stack([Gphys[b] @ Wc[a, c] for b in range(3)], axis=1)
                           for a in range(3)], axis=1)                      # (q, a, b): d_b w_a
            for cc in range(3):
                t = np.einsum("qb,qb->q", uq, gw[:, cc, :]) + np.einsum("qa,qa->q", uq, gw[:, :, cc])
                out[cc, r] -= self.Phi.T @ (w * t)
            for f in range(6):
                d, s = divmod(f, 2)
                cn = m.neighbor(c, f)
                if cn < 0:
                    nrm, dA = self._face_geo(c, d, s)
                    nout = nrm if s == 1 else -nrm
                    um = (self.Tr[f] @ V[:, c, :].T).T
                    up = um if m.neumann[f] else 2.0 * self._gvals(c, f) - um
                    wm = (self.Tr[f] @ Wc[:, c, :].T).T
                    Jm, Jp = self.flux_jac_T(um, up, nout, wm)
                    # u+ = u- (outflow) or u+ = 2g - u- (Dirichlet)
                    out[:, r] += (self.Tr[f].T @ (dA * (Jm + Jp if m.neumann[f] else Jm - Jp)).T).T
                    continue
                L, R_ = (c, cn) if s == 1 else (cn, c)
                nrm, dA = self._face_geo(L, d, 1)
                um = (self.Tr[2 * d + 1] @ V[:, L, :].T).T
                up = (self.Tr[2 * d] @ V[:, R_, :].T).T
                jw = (self.Tr[2 * d + 1] @ Wc[:, L, :].T).T - (self.Tr[2 * d] @ Wc[:, R_, :].T).T
                Jm, Jp = self.flux_jac_T(um, up, nrm, jw)
                out[:, r] += (self.Tr[f].T @ (dA * (Jm if s == 1 else Jp)).T).T
        return out

    def vjp(self, U, W):
        return self.vjp_cells(U, W, range(self.mesh.ncells)).ravel()

    def jacobian(self, U):
        """Dense Jacobian by JVPs of unit vectors (brute force; tiny meshes only)."""
        N = U.size
        Jm = np.zeros((N, N))
        e = np.zeros(N)
        for j in range(N):
            e[j] = 1.0
            Jm[:, j] = self.jvp(U, e)
            e[j] = 0.0
        return Jm
