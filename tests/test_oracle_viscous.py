"""Pins of the oracle's symmetric-gradient viscous operator.

Consistency: for a velocity field that is a polynomial of degree <= k per
direction and vanishes on the Dirichlet boundary, SIPG reproduces the strong
form exactly: a(phi_i e_c, u) = (phi_i, mu u - div(2 nu eps(u)))_c, whose
right-hand side is computed here analytically from the polynomial's
coefficients.  Structure: symmetry, translations in the null space of the
periodic operator, and definiteness with Dirichlet faces.
"""
import numpy as np
import pytest

from oracle import mesh, viscous, v3
import dgmf_inputs as inp


class Poly:
    """p = sum c[i, j, l] x^i y^j z^l."""

    def __init__(self, c):
        self.c = np.asarray(c, dtype=np.float64)

    def __call__(self, x, y, z):
        n = self.c.shape
        return sum(self.c[i, j, l] * x ** i * y ** j * z ** l for i in range(n[0]) for j in range(n[1])
                   for l in range(n[2]))

    def d(self, a):
        c = self.c
        idx = np.arange(c.shape[a], dtype=np.float64)
        shape = [1, 1, 1]
        shape[a] = -1
        dc = (c * idx.reshape(shape))
        dc = np.take(dc, range(1, c.shape[a]), axis=a) if c.shape[a] > 1 else np.zeros_like(c)
        return Poly(dc)

    def __mul__(self, o):
        a, b = self.c, o.c
        out = np.zeros(tuple(a.shape[i] + b.shape[i] - 1 for i in range(3)))
        for i, j, l in np.ndindex(*a.shape):
            out[i:i + b.shape[0], j:j + b.shape[1], l:l + b.shape[2]] += a[i, j, l] * b
        return Poly(out)

    def __add__(self, o):
        s = tuple(max(self.c.shape[i], o.c.shape[i]) for i in range(3))
        out = np.zeros(s)
        out[:self.c.shape[0], :self.c.shape[1], :self.c.shape[2]] += self.c
        out[:o.c.shape[0], :o.c.shape[1], :o.c.shape[2]] += o.c
        return Poly(out)

    def scale(self, f):
        return Poly(f * self.c)


def _lin(c0, cx, cy, cz):
    c = np.zeros((2, 2, 2))
    c[0, 0, 0], c[1, 0, 0], c[0, 1, 0], c[0, 0, 1] = c0, cx, cy, cz
    return Poly(c)


def test_consistency_with_the_strong_form():
    k, mu, nu = 3, 2.0, 0.7
    m = mesh.BoxMesh(k, 2, 2, 3, lx=1.0, ly=1.0, lz=1.0, periodic=(False, False, False))
    bx = Poly(np.array([[[0.0]], [[1.0]], [[-1.0]]]))            # x (1 - x)
    by = Poly(np.array([[[0.0], [1.0], [-1.0]]]))                # y (1 - y)
    bz = Poly(np.array([[[0.0, 1.0, -1.0]]]))                    # z (1 - z)
    b = bx * by * bz
    u = [b * _lin(1.0, 1.0, 0.0, 0.0), b * _lin(2.0, 0.0, -1.0, 1.0), b * _lin(0.5, 0.0, 1.0, 0.0)]
    div = u[0].d(0) + u[1].d(1) + u[2].d(2)
    f = []
    for a in range(3):
        lap = u[a].d(0).d(0) + u[a].d(1).d(1) + u[a].d(2).d(2)
        f.append(u[a].scale(mu) + (lap + div.d(a)).scale(-nu))   # mu u - nu (lap u + grad div u)
    X = m.node_coords()
    U = np.concatenate([p(X[:, 0], X[:, 1], X[:, 2]) for p in u])
    F = np.concatenate([p(X[:, 0], X[:, 1], X[:, 2]) for p in f])
    A = viscous.viscous_matrix(m, mu, nu)
    got = A @ U
    want = v3.mass_apply(m, F)
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


def test_symmetric_with_translations_in_the_periodic_null_space():
    m = mesh.BoxMesh(2, 2, 3, 2, lx=1.0, ly=1.3, lz=0.8)
    A = viscous.viscous_matrix(m, 0.0, 1.0).toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    for a in range(3):
        e = np.zeros(3 * m.ndofs)
        e[a * m.ndofs:(a + 1) * m.ndofs] = 1.0
        assert np.abs(A @ e).max() <= 1e-12 * np.abs(A).max()


def test_definite_with_dirichlet_faces():
    m = mesh.BoxMesh(2, 2, 2, 2, lx=1.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, True), y_tanh_gamma=1.0)
    A = viscous.viscous_matrix(m, 0.0, 1.0).toarray()
    assert np.linalg.eigvalsh(0.5 * (A + A.T))[0] > 0


@pytest.mark.parametrize("case", ["periodic_k2", "channel_k3", "one_cell_k2", "neumann_k2"])
def test_row_restricted_apply_equals_matrix(case):
    """viscous_apply_cells (per-cell blocks, for sampling full-size meshes) equals the
    assembled matrix on every row."""
    if case == "periodic_k2":
        m = mesh.BoxMesh(2, 3, 2, 2, lx=1.0, ly=0.8, lz=1.2)
    elif case == "channel_k3":
        m = mesh.BoxMesh(3, 2, 3, 2, lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, True),
                         y_tanh_gamma=1.5)
    elif case == "one_cell_k2":
        m = mesh.BoxMesh(2, 1, 2, 1, periodic=(True, False, True))
    else:
        m = mesh.BoxMesh(2, 2, 2, 2, periodic=(False, False, True), neumann=(True, False, False, True, False, False))
    U = inp.uniform(77, 3 * m.ndofs)
    want = viscous.viscous_matrix(m, 3.0, 0.4, 1.0) @ U
    got = viscous.viscous_apply_cells(m, U, list(range(m.ncells)), 3.0, 0.4, 1.0)
    want = want.reshape(3, m.ncells, -1)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
