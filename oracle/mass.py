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


def inverse_mass_cells(mesh, v, cells=None):
    """M^{-1} v, one dense solve per cell.

    cells None: v is a scalar field of mesh.ndofs values.  Otherwise v holds
    the blocks of the listed cells only, shape (len(cells), n^3), and so does
    the result (M is block diagonal, so a cell needs nothing but its block).
    """
    T = sipg.Tables(mesh.k)
    nb = mesh.n ** 3
    cl = range(mesh.ncells) if cells is None else list(cells)
    V = np.asarray(v, dtype=np.float64).reshape(len(cl), nb)
    out = np.empty_like(V)
    cache = {}
    for r, c in enumerate(cl):
        J = mesh.jacobian(c)
        key = tuple(np.round(J.ravel(), 15))
        if key not in cache:
            cache[key] = sipg.cell_matrices(T, J)[1]
        out[r] = np.linalg.solve(cache[key], V[r])
    return out.ravel() if cells is None else out


def convective_step(conv, U, dt):
    """U - dt M^{-1} C(U) for a velocity [3][N] with the oracle convective operator."""
    m = conv.mesh
    C = conv.forward(U).reshape(3, m.ndofs)
    Uv = np.asarray(U, dtype=np.float64).reshape(3, m.ndofs)
    return np.concatenate([Uv[a] - dt * inverse_mass_cells(m, C[a]) for a in range(3)])


def convective_step_cells(conv, U, dt, cells):
    """The substep on the listed cells only, shape (3, len(cells), n^3)."""
    m = conv.mesh
    C = np.asarray(conv.forward_cells(U, cells)).reshape(3, len(cells), -1)
    Uc = np.asarray(U, dtype=np.float64).reshape(3, m.ncells, -1)[:, cells]
    return np.stack([Uc[a] - dt * inverse_mass_cells(m, C[a], cells) for a in range(3)])
