"""Inverse mass matrix and the explicit convective substep (oracle; test infrastructure).

The mass matrix M is block diagonal over the cells (the paper's matrix form
of the convective step, eq. advect), each block (phi_i, phi_j)_K assembled by
Gauss quadrature with n_q = k+1 points (exact for the degree-2k integrand on
affine cells).  With BDF1 / extrapolation order 1 and no body force, eq.
advect reads  U_hat = U^n - dt M^{-1} F^c(U^n),  F^c the convective operator.
Here the blocks are inverted by a dense solve per cell.
"""
import numpy as np

from . import sipg


def inverse_mass_cells(mesh, v):
    """M^{-1} v for a scalar field v (length mesh.ndofs): one dense solve per cell."""
    T = sipg.Tables(mesh.k)
    nb = mesh.n ** 3
    V = np.asarray(v, dtype=np.float64).reshape(mesh.ncells, nb)
    out = np.empty_like(V)
    cache = {}
    for c in range(mesh.ncells):
        J = mesh.jacobian(c)
        key = tuple(np.round(J.ravel(), 15))
        if key not in cache:
            cache[key] = sipg.cell_matrices(T, J)[1]
        out[c] = np.linalg.solve(cache[key], V[c])
    return out.ravel()


def convective_step(conv, U, dt):
    """U - dt M^{-1} C(U) for a velocity [3][N] with the oracle convective operator."""
    m = conv.mesh
    C = conv.forward(U).reshape(3, m.ndofs)
    Uv = np.asarray(U, dtype=np.float64).reshape(3, m.ndofs)
    return np.concatenate([Uv[a] - dt * inverse_mass_cells(m, C[a]) for a in range(3)])
