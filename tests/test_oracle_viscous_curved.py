"""Pins of the oracle's symmetric-gradient viscous operator on curved cells.

Fixed by facts outside the curved viscous oracle: with zero amplitude it is
the affine operator of ``viscous.viscous_matrix`` (pinned on its own); the six
rigid motions a + w x x are in the null space of the mass-free form on a box
with homogeneous Neumann sides all round (their nodal interpolant on the
iso-parametric cells is exactly a + w x x_h, whose symmetric gradient
vanishes at every point and whose traces agree across faces, whatever the
quadrature); the form is symmetric, and definite with Dirichlet walls; the
row-restricted apply equals the assembled matrix; and a manufactured
divergence-free solution on a curved periodic mesh converges at order k+1.
A transposed inverse Jacobian, a normal taken outside the point sums or
from the wrong side, or a lost coupling term fails one of them.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import curved, mesh as omesh, viscous
import dgmf_inputs as inp

TWO_PI = 2.0 * math.pi


def test_zero_amplitude_is_the_affine_operator():
    kw = dict(lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, False), y_tanh_gamma=1.3,
              neumann=(False, False, False, False, True, False))
    cm = curved.CurvedBoxMesh(2, 2, 2, 2, amp=0.0, **kw)
    am = omesh.BoxMesh(2, 2, 2, 2, **kw)
    A = viscous.CurvedViscous(cm, 2.0, 0.5, 1.0).assemble()
    B = viscous.viscous_matrix(am, 2.0, 0.5, 1.0)
    assert abs(A - B).max() <= 1e-12 * abs(B).max()


def _rigid(m, a, w):
    X = np.concatenate([m.node_xyz(c) for c in range(m.ncells)])
    return np.concatenate([a[i] + np.cross(w, X)[:, i] for i in range(3)])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_rigid_motions_in_the_null_space(k):
    m = curved.CurvedBoxMesh(k, 2, 2, 2, amp=0.05, periodic=(False, False, False), neumann=(True,) * 6)
    A = viscous.CurvedViscous(m, 0.0, 0.7, 1.0).assemble()
    scale = abs(A).max()
    for j in range(6):
        a, w = np.zeros(3), np.zeros(3)
        (a if j < 3 else w)[j % 3] = 1.0
        u = _rigid(m, a, w)
        assert np.abs(A @ u).max() <= 1e-11 * scale * np.abs(u).max()
    # a pure strain is not a rigid motion
    X = np.concatenate([m.node_xyz(c) for c in range(m.ncells)])
    u = np.concatenate([X[:, 0], np.zeros(m.ndofs), np.zeros(m.ndofs)])
    assert np.abs(A @ u).max() > 1e-3 * scale


def test_symmetric_and_definite_with_walls():
    m = curved.CurvedBoxMesh(2, 2, 2, 2, amp=0.06, lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, True))
    A = viscous.CurvedViscous(m, 0.0, 1.0, 1.0).assemble()
    assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > 1e-8 * ev.max()


@pytest.mark.parametrize("case", ["periodic_k2", "walls_neumann_k2", "one_cell_k1"])
def test_row_restricted_apply_equals_matrix(case):
    if case == "periodic_k2":
        m = curved.CurvedBoxMesh(2, 3, 2, 2, amp=0.05)
    elif case == "walls_neumann_k2":
        m = curved.CurvedBoxMesh(2, 2, 3, 2, amp=0.04, lx=2.0, ly=2.0, lz=1.0, y0=-1.0, y_tanh_gamma=1.2,
                                 periodic=(True, False, False), neumann=(False, False, False, False, True, False))
    else:
        m = curved.CurvedBoxMesh(1, 1, 2, 1, amp=0.05, periodic=(True, False, True))
    op = viscous.CurvedViscous(m, 3.0, 0.4, 1.0)
    U = inp.uniform(78, 3 * m.ndofs)
    want = (op.assemble() @ U).reshape(3, m.ncells, -1)
    got = op.apply_cells(U, list(range(m.ncells)))
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.slow
def test_manufactured_solution_converges():
    """u = (sin 2pi y, sin 2pi z, sin 2pi x) (divergence-free, periodic): mu u - div(2 nu eps(u))
    = (mu + 4 pi^2 nu) u; L2 error of the discrete solution at order >= k + 1 - 0.5."""
    k, mu, nu = 2, 1.0, 0.1
    errs = []
    for nc in (3, 6):
        m = curved.CurvedBoxMesh(k, nc, nc, nc, amp=0.03)
        op = viscous.CurvedViscous(m, mu, nu, 1.0)
        ex = [lambda x, y, z: np.sin(TWO_PI * y), lambda x, y, z: np.sin(TWO_PI * z),
              lambda x, y, z: np.sin(TWO_PI * x)]
        s = op.s
        b = np.concatenate([s.rhs(lambda x, y, z, e=e: (mu + 4 * math.pi ** 2 * nu) * e(x, y, z)) for e in ex])
        U = spla.spsolve(op.assemble().tocsc(), b)
        N = m.ndofs
        errs.append(math.sqrt(sum(s.l2_error(U[c * N:(c + 1) * N], ex[c]) ** 2 for c in range(3))))
    order = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert order >= k + 1 - 0.5, (errs, order)
