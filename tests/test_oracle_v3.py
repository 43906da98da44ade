"""Pins of the oracle's V3c operators: divergence, gradient, div-div penalty and projection.

Consistency pins: for a global polynomial of degree <= k per direction the
central average equals the trace everywhere, so A u = -M div(u) and
B p = -M grad(p) hold exactly (the divergence and gradient are taken
analytically here).  Structure pins: A = -B^T on periodic meshes, and on
meshes with boundary faces the difference is the boundary face mass, computed
here by an independent tensor formula.  The penalty and projection are pinned
by closed forms and limits.
"""
import math

import numpy as np
import pytest

from oracle import basis, mass as omass, mesh, sipg, v3
import dgmf_inputs as inp


def _poly(coef):
    """p(x, y, z) = sum c[i, j, l] x^i y^j z^l and its gradient."""
    n = coef.shape[0]

    def val(x, y, z):
        return sum(coef[i, j, l] * x ** i * y ** j * z ** l for i in range(n) for j in range(n) for l in range(n))

    def grad(x, y, z):
        gx = sum(i * coef[i, j, l] * x ** (i - 1) * y ** j * z ** l for i in range(1, n) for j in range(n)
                 for l in range(n))
        gy = sum(j * coef[i, j, l] * x ** i * y ** (j - 1) * z ** l for i in range(n) for j in range(1, n)
                 for l in range(n))
        gz = sum(l * coef[i, j, l] * x ** i * y ** j * z ** (l - 1) for i in range(n) for j in range(n)
                 for l in range(1, n))
        return gx, gy, gz
    return val, grad


@pytest.mark.parametrize("k", [2, 3])
def test_divergence_of_global_polynomials(k):
    # no periodic direction: a global polynomial is not periodic
    m = mesh.BoxMesh(k, 3, 2, 2, lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(False, False, False),
                     y_tanh_gamma=1.3)
    X = m.node_coords()
    comps, div = [], np.zeros(m.ndofs)
    for a in range(3):
        val, grad = _poly(inp.uniform(40 + a, (k + 1) ** 3).reshape(k + 1, k + 1, k + 1))
        comps.append(val(X[:, 0], X[:, 1], X[:, 2]))
        div += grad(X[:, 0], X[:, 1], X[:, 2])[a]
    A = v3.divergence_matrix(m)
    got = A @ np.concatenate(comps)
    want = -v3.mass_apply(m, div)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


@pytest.mark.parametrize("k", [2, 3])
def test_gradient_of_global_polynomials(k):
    m = mesh.BoxMesh(k, 2, 3, 2, lx=1.0, ly=2.0, lz=1.5, y0=-1.0, periodic=(False, False, False),
                     y_tanh_gamma=1.1)
    X = m.node_coords()
    val, grad = _poly(inp.uniform(50, (k + 1) ** 3).reshape(k + 1, k + 1, k + 1))
    B = v3.gradient_matrix(m)
    got = B @ val(X[:, 0], X[:, 1], X[:, 2])
    g = grad(X[:, 0], X[:, 1], X[:, 2])
    want = -np.concatenate([v3.mass_apply(m, g[a]) for a in range(3)])
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


def test_divergence_is_minus_gradient_transpose_on_periodic_meshes():
    m = mesh.BoxMesh(2, 3, 2, 2, lx=1.0, ly=0.7, lz=1.2)
    A = v3.divergence_matrix(m).toarray()
    B = v3.gradient_matrix(m).toarray()
    assert np.abs(A + B.T).max() <= 1e-13 * np.abs(A).max()


def _lagrange(nodes, x):
    L = np.ones((len(x), len(nodes)))
    for j, xj in enumerate(nodes):
        for mm, xm in enumerate(nodes):
            if mm != j:
                L[:, j] *= (x - xm) / (xj - xm)
    return L


def test_boundary_terms_are_the_face_mass():
    """A + B^T = -(sum over boundary faces of n_a (phi_i, phi_j)_F), face mass by its own Gauss rule."""
    k = 2
    m = mesh.BoxMesh(k, 2, 2, 1, lx=1.0, ly=1.5, lz=0.5, periodic=(True, False, False))
    n, nb, N = m.n, m.n ** 3, m.ndofs
    x, w = np.polynomial.legendre.leggauss(k + 2)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    L = _lagrange(basis.gll_nodes(k), x)
    Mh = L.T @ (w[:, None] * L)
    want = np.zeros((N, 3 * N))
    for c, f in m.boundary_faces():
        d, s = divmod(f, 2)
        _, h = m.cell_origin_h(c)
        t = [a for a in range(3) if a != d]
        area = h[t[0]] * h[t[1]]
        e = n - 1 if s else 0
        idx = []
        for p2 in range(n):
            for p1 in range(n):
                ijk = [0, 0, 0]
                ijk[d], ijk[t[0]], ijk[t[1]] = e, p1, p2
                idx.append(c * nb + (ijk[2] * n + ijk[1]) * n + ijk[0])
        Fm = area * np.kron(Mh, Mh)
        sgn = 1.0 if s else -1.0
        want[np.ix_(idx, [d * N + i for i in idx])] -= sgn * Fm
    A = v3.divergence_matrix(m).toarray()
    B = v3.gradient_matrix(m).toarray()
    assert np.abs(A + B.T - want).max() <= 1e-13 * np.abs(A).max()


def test_divdiv_kernel_and_energy():
    k = 3
    T = sipg.Tables(k)
    m = mesh.BoxMesh(k, 1, 1, 1, lx=0.5, ly=1.5, lz=2.0, periodic=(False, False, False))
    J = m.jacobian(0)
    D = v3.divdiv_cell(T, J)
    X = m.node_coords()
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    u = np.concatenate([y ** 2 + z, z * x, x * y])          # divergence-free
    assert np.abs(D @ u).max() <= 1e-12 * np.abs(D).max() * np.abs(u).max()
    u = np.concatenate([x, np.zeros_like(x), np.zeros_like(x)])   # div = 1
    assert abs(u @ D @ u - m.volume(0)) <= 1e-13


def test_penalty_of_a_constant_field():
    m = mesh.BoxMesh(2, 2, 3, 1, lx=1.0, ly=2.0, lz=0.5, y0=-1.0, periodic=(True, False, True), y_tanh_gamma=1.0)
    U = np.concatenate([np.full(m.ndofs, 0.3), np.full(m.ndofs, -0.4), np.full(m.ndofs, 1.2)])
    tau = v3.penalty_tau(m, U, 2.0, 0.01)
    for c in range(m.ncells):
        assert abs(tau[c] - 2.0 * 1.3 * m.volume(c) ** (1 / 3) * 0.01) <= 1e-14


def test_projection_limits():
    m = mesh.BoxMesh(2, 2, 2, 2)
    rhs = inp.uniform(60, 3 * m.ndofs)
    x0 = v3.projection_solve(m, np.zeros(m.ncells), rhs)
    want = np.concatenate([omass.inverse_mass_cells(m, rhs.reshape(3, -1)[a]) for a in range(3)])
    assert np.abs(x0 - want).max() <= 1e-12 * np.abs(want).max()
    T = sipg.Tables(m.k)
    nb = m.n ** 3
    energies = []
    for t in (0.0, 1.0, 10.0, 100.0):
        x = v3.projection_solve(m, np.full(m.ncells, t), rhs).reshape(3, m.ncells, nb)
        e = 0.0
        for c in range(m.ncells):
            xe = x[:, c].ravel()
            e += xe @ v3.divdiv_cell(T, m.jacobian(c)) @ xe
        energies.append(e)
    assert all(energies[i + 1] < 0.5 * energies[i] for i in range(3))
