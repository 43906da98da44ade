"""Pins of the oracle's inverse mass matrix and explicit convective substep.

The mass blocks are pinned by textbook values (the linear element) and by the
L2 projection property: M^{-1} b reproduces a function of the discrete space
exactly when b holds its integrals against the basis, computed here by a
separate higher-order Gauss rule and a Lagrange basis written out in this file.
The substep is pinned by steady states of the convective term and by
consistency with the exact (u . grad) u of a divergence-free field.
"""
import math

import numpy as np
import pytest

from oracle import basis, convective, mass, mesh
import dgmf_inputs as inp

TWO_PI = 2.0 * math.pi


def _lagrange(nodes, x):
    """L[q, j] = l_j(x_q) from the product formula."""
    L = np.ones((len(x), len(nodes)))
    for j, xj in enumerate(nodes):
        for m, xm in enumerate(nodes):
            if m != j:
                L[:, j] *= (x - xm) / (xj - xm)
    return L


def _load_vector(m, f, nq):
    """b_i = int_K f phi_i over every cell with an nq-point Gauss rule per direction."""
    x, w = np.polynomial.legendre.leggauss(nq)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    L = _lagrange(basis.gll_nodes(m.k), x)
    b = np.empty((m.ncells, m.n ** 3))
    for c in range(m.ncells):
        o, h = m.cell_origin_h(c)
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        p = np.stack([o[0] + h[0] * X, o[1] + h[1] * Y, o[2] + h[2] * Z])
        J = m.jacobian(c)
        if m.shear is not None:
            p = np.einsum("ab,bzyx->azyx", m.shear, p)
        fq = f(*p) * np.einsum("z,y,x->zyx", w, w, w) * abs(np.linalg.det(J))
        b[c] = np.einsum("zyx,zl,yj,xi->lji", fq, L, L, L).ravel()
    return b.ravel()


def test_linear_element_closed_form():
    """k = 1: the 1D mass on [0,1] is [[1/3, 1/6], [1/6, 1/3]], its inverse [[4, -2], [-2, 4]]."""
    m = mesh.BoxMesh(1, 1, 1, 1, lx=0.5, ly=1.0, lz=2.0, periodic=(False, False, False))
    e0 = np.zeros(m.ndofs)
    e0[0] = 1.0
    col = np.array([4.0, -2.0])
    want = np.einsum("l,j,i->lji", col, col, col).ravel() / (0.5 * 1.0 * 2.0)
    np.testing.assert_allclose(mass.inverse_mass_cells(m, e0), want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_projection_reproduces_tensor_polynomials(k):
    """Graded channel cells: f in Q_k on every cell is its own L2 projection."""
    m = mesh.BoxMesh(k, 2, 3, 2, lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, True),
                     y_tanh_gamma=1.5)
    cx = inp.uniform(10 + k, 3 * (k + 1)).reshape(3, k + 1)

    def f(x, y, z):
        px = sum(cx[0, p] * x ** p for p in range(k + 1))
        py = sum(cx[1, p] * y ** p for p in range(k + 1))
        pz = sum(cx[2, p] * z ** p for p in range(k + 1))
        return px * py * pz

    b = _load_vector(m, f, k + 3)
    X = m.node_coords()
    want = f(X[:, 0], X[:, 1], X[:, 2])
    got = mass.inverse_mass_cells(m, b)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


def test_projection_on_sheared_cells():
    """Parallelepiped cells: a polynomial of total degree k in x, y, z is in the space."""
    k = 3
    sh = np.array([[1.0, 0.3, 0.1], [0.0, 1.1, -0.2], [0.05, 0.0, 0.9]])
    m = mesh.BoxMesh(k, 2, 2, 2, shear=sh)

    def f(x, y, z):
        return 0.5 + x - 2.0 * y * z + x * y * z + 0.3 * z ** 3 - y ** 2 * x

    b = _load_vector(m, f, k + 3)
    X = m.node_coords()
    want = f(X[:, 0], X[:, 1], X[:, 2])
    got = mass.inverse_mass_cells(m, b)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


def test_step_keeps_free_stream():
    m = mesh.BoxMesh(2, 2, 2, 3)
    op = convective.Convective(m)
    U = np.concatenate([np.full(m.ndofs, 0.7), np.full(m.ndofs, -0.2), np.full(m.ndofs, 1.3)])
    np.testing.assert_allclose(mass.convective_step(op, U, 0.05), U, rtol=0, atol=1e-14)


def test_step_keeps_parallel_shear_flow():
    """u = (g(y), 0, 0): div(u (x) u) = 0 and the continuous nodal field has no face jumps."""
    m = mesh.BoxMesh(3, 2, 3, 2, lx=1.0, ly=1.0, lz=1.0)
    op = convective.Convective(m)
    X = m.node_coords()
    U = np.concatenate([np.sin(TWO_PI * X[:, 1]) + 0.4, np.zeros(m.ndofs), np.zeros(m.ndofs)])
    np.testing.assert_allclose(mass.convective_step(op, U, 0.1), U, rtol=0, atol=1e-13)


def _tg_advection(x, y, z):
    """(u . grad) u of the Taylor-Green field, which equals div(u (x) u) since div u = 0."""
    s, c = np.sin, np.cos
    a, b, g = TWO_PI * x, TWO_PI * y, TWO_PI * z
    u, v = s(a) * c(b) * c(g), -c(a) * s(b) * c(g)
    du = (TWO_PI * c(a) * c(b) * c(g), -TWO_PI * s(a) * s(b) * c(g), -TWO_PI * s(a) * c(b) * s(g))
    dv = (TWO_PI * s(a) * s(b) * c(g), -TWO_PI * c(a) * c(b) * c(g), TWO_PI * c(a) * s(b) * s(g))
    return np.stack([u * du[0] + v * du[1], u * dv[0] + v * dv[1], np.zeros_like(x)])


@pytest.mark.parametrize("k", [2, 3])
def test_step_is_consistent_with_the_advection_term(k):
    """(U - step(U, dt)) / dt -> (u . grad) u at the nodes, at order about k in h."""
    errs = []
    for nc in (4, 8):
        m = mesh.BoxMesh(k, nc, nc, nc)
        op = convective.Convective(m)
        X = m.node_coords()
        U = inp.taylor_green(X[:, 0], X[:, 1], X[:, 2]).ravel()
        dt = 1e-3
        est = (U - mass.convective_step(op, U, dt)) / dt
        ex = _tg_advection(X[:, 0], X[:, 1], X[:, 2]).ravel()
        errs.append(np.sqrt(np.mean((est - ex) ** 2)))
    assert errs[1] < 0.1 * np.abs(ex).max()
    assert errs[0] / errs[1] > 2.0 ** (k - 0.5)


def test_sampled_cells_match_the_whole_mesh():
    m = mesh.BoxMesh(2, 3, 2, 2, lx=1.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, True),
                     y_tanh_gamma=1.2)
    op = convective.Convective(m)
    X = m.node_coords()
    U = (inp.parabolic(X[:, 0], X[:, 1], X[:, 2]) + 0.2 * inp.uniform(3, 3 * m.ndofs).reshape(3, -1)).ravel()
    cells = [0, 4, 11]
    full = mass.convective_step(op, U, 0.07).reshape(3, m.ncells, -1)[:, cells]
    np.testing.assert_allclose(mass.convective_step_cells(op, U, 0.07, cells), full, rtol=0, atol=1e-14)
