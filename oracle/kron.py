"""Kronecker-sum construction and exact direct solve (oracle; test infrastructure).

A second construction of the SIPG operator, independent of the 3D element
assembly in ``sipg``: on a uniform, fully periodic Cartesian mesh every
integral of Sec. 3.2 factorises over the three coordinate directions, so

  A = K_z (x) M_y (x) M_x + M_z (x) K_y (x) M_x + M_z (x) M_y (x) K_x,
  H = mu M_z (x) M_y (x) M_x + nu A,

with M_d the 1D DG mass matrix and K_d the 1D SIPG matrix in direction d
(cell stiffness plus the point terms of the 1D face fluxes, using the 3D
penalty tau of eq. taue).  Here the lexicographic DoF order (Z, Y, X) with
X = cx*n + i is used; ``to_lex``/``from_lex`` permute to and from the
cell-wise order of the rest of the oracle.

The direct solve is fast diagonalisation (Lynch, Rice & Thomas 1964): with
K_d V_d = M_d V_d Lambda_d and V_d^T M_d V_d = I, A^{-1} = V Lambda^{-1} V^T,
V = V_z (x) V_y (x) V_x.  On the singular periodic Laplacian the zero mode is
dropped, which yields the solution with zero integral mean.
"""
import numpy as np
import scipy.linalg as sla

from . import basis


def sipg_1d(k, ncell, h, tau, periodic=True):
    """(K1, M1): 1D SIPG stiffness (with face terms) and mass, ncell*(k+1) square."""
    n = k + 1
    nodes = basis.gll_nodes(k)
    xq, wq = basis.gauss_rule(n)
    S = basis.lagrange_values(nodes, xq)
    D = basis.lagrange_derivatives(nodes, xq)
    e0, e1 = basis.lagrange_values(nodes, [0.0])[0], basis.lagrange_values(nodes, [1.0])[0]
    d0, d1 = basis.lagrange_derivatives(nodes, [0.0])[0] / h, basis.lagrange_derivatives(nodes, [1.0])[0] / h
    N = ncell * n
    K = np.zeros((N, N))
    M = np.zeros((N, N))
    kloc = D.T @ (wq[:, None] * D) / h
    mloc = S.T @ (wq[:, None] * S) * h
    for e in range(ncell):
        sl = slice(e * n, (e + 1) * n)
        K[sl, sl] += kloc
        M[sl, sl] += mloc
    nfaces = ncell if periodic else ncell - 1
    for e in range(nfaces):
        L, R = e, (e + 1) % ncell
        # jump [v] = v_L(1) - v_R(0); average {{v'}} = (v_L'(1) + v_R'(0))/2, normal +1
        jmp = np.zeros(N)
        avg = np.zeros(N)
        jmp[L * n:(L + 1) * n] += e1
        jmp[R * n:(R + 1) * n] -= e0
        avg[L * n:(L + 1) * n] += 0.5 * d1
        avg[R * n:(R + 1) * n] += 0.5 * d0
        K += -np.outer(avg, jmp) - np.outer(jmp, avg) + tau * np.outer(jmp, jmp)
    if not periodic:
        for e, ev, dv, sgn in ((0, e0, d0, -1.0), (ncell - 1, e1, d1, 1.0)):
            sl = slice(e * n, (e + 1) * n)
            dn = sgn * dv
            K[sl, sl] += -np.outer(dn, ev) - np.outer(ev, dn) + 2 * tau * np.outer(ev, ev)
    return K, M


class KronPeriodic:
    """Uniform periodic box [0,lx]x[0,ly]x[0,lz], nx*ny*nz cells, degree k."""

    def __init__(self, k, nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, mass_coeff=0.0, diff_coeff=1.0,
                 penalty_scale=1.0):
        self.k, self.n = k, k + 1
        self.nc = (nx, ny, nz)
        h = (lx / nx, ly / ny, lz / nz)
        vol = h[0] * h[1] * h[2]
        area = 2 * (h[1] * h[2] + h[0] * h[2] + h[0] * h[1])
        self.tau = penalty_scale * (k + 1) ** 2 * (area / 2) / vol
        self.mu, self.nu = float(mass_coeff), float(diff_coeff)
        self.K, self.M = [], []
        for d in range(3):
            K1, M1 = sipg_1d(k, self.nc[d], h[d], self.tau, periodic=True)
            self.K.append(K1)
            self.M.append(M1)
        self.V, self.lam = [], []
        for d in range(3):
            lam, V = sla.eigh(self.K[d], self.M[d])
            self.lam.append(lam)
            self.V.append(V)

    @property
    def shape(self):
        n = self.n
        return (self.nc[2] * n, self.nc[1] * n, self.nc[0] * n)

    def to_lex(self, u):
        nx, ny, nz = self.nc
        n = self.n
        a = u.reshape(nz, ny, nx, n, n, n)            # cz, cy, cx, l, j, i
        return a.transpose(0, 3, 1, 4, 2, 5).reshape(self.shape)

    def from_lex(self, U):
        nx, ny, nz = self.nc
        n = self.n
        a = U.reshape(nz, n, ny, n, nx, n)            # cz, l, cy, j, cx, i
        return a.transpose(0, 2, 4, 1, 3, 5).ravel()

    @staticmethod
    def _apply_axis(U, mat, axis):
        return np.moveaxis(np.tensordot(mat, np.moveaxis(U, axis, 0), axes=(1, 0)), 0, axis)

    def _tensor_apply(self, U, mz, my, mx):
        U = self._apply_axis(U, mx, 2)
        U = self._apply_axis(U, my, 1)
        return self._apply_axis(U, mz, 0)

    def apply(self, u):
        """H u in cell-wise order via the Kronecker sum."""
        U = self.to_lex(u)
        Kx, Ky, Kz = self.K
        Mx, My, Mz = self.M
        out = self.nu * (self._tensor_apply(U, Kz, My, Mx) + self._tensor_apply(U, Mz, Ky, Mx)
                         + self._tensor_apply(U, Mz, My, Kx))
        if self.mu != 0.0:
            out = out + self.mu * self._tensor_apply(U, Mz, My, Mx)
        return self.from_lex(out)

    def eigenvalues(self):
        """All eigenvalues of the pencil (H, M), as a 3D array over (Z, Y, X) modes."""
        lx, ly, lz = self.lam
        return self.mu + self.nu * (lz[:, None, None] + ly[None, :, None] + lx[None, None, :])

    def solve(self, b, zero_tol=1e-9):
        """Exact H^{-1} b by fast diagonalisation; zero modes dropped."""
        B = self.to_lex(b)
        Vx, Vy, Vz = self.V
        C = self._tensor_apply(B, Vz.T, Vy.T, Vx.T)
        lam = self.eigenvalues()
        scale = np.abs(lam).max()
        inv = np.where(np.abs(lam) > zero_tol * scale, 1.0 / np.where(lam == 0, 1, lam), 0.0)
        return self.from_lex(self._tensor_apply(C * inv, Vz, Vy, Vx))
