"""Pins of the oracle's SIPG operator on iso-parametric curved cells.

Fixed by facts outside the curved oracle: with zero amplitude it is the
affine operator of the (separately pinned) ``sipg`` module; an interior face
seen from either cell has the same normal and surface measure (the two
iso-parametric maps share the face nodes); constants lie in the null space of
the periodic Laplacian whatever the quadrature; and a manufactured solution
on a curved periodic mesh converges at order k+1.  A wrong Jacobian, a
transposed inverse or a normal taken from the wrong side fails one of them.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import curved, mesh as omesh, sipg


def test_zero_amplitude_is_the_affine_operator():
    kw = dict(lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, False), y_tanh_gamma=1.3,
              neumann=(False, False, False, False, True, False))
    cm = curved.CurvedBoxMesh(2, 3, 2, 2, amp=0.0, **kw)
    am = omesh.BoxMesh(2, 3, 2, 2, **kw)
    A = curved.CurvedSIPG(cm, 2.0, 0.5, 1.0).assemble()
    B = sipg.SIPG(am, 2.0, 0.5, 1.0).assemble()
    assert abs(A - B).max() <= 1e-12 * abs(B).max()


def test_interior_faces_agree_from_both_sides():
    m = curved.CurvedBoxMesh(3, 3, 3, 2, amp=0.05, periodic=(True, True, True))
    op = curved.CurvedSIPG(m)
    for cL, cR, d in m.interior_faces():
        _, _, dAL, nL = op.face(cL, 2 * d + 1)
        _, _, dAR, nR = op.face(cR, 2 * d)
        assert np.abs(dAL - dAR).max() <= 1e-12 * dAL.max()
        assert np.abs(nL - nR).max() <= 1e-12
    # the physical face points coincide too (up to a period on wrap-around faces)
    T = op.T
    xiL, _ = curved._face_points(T, 1)
    xiR, _ = curved._face_points(T, 0)
    xl = m.map_at(0, xiL)
    xr = m.map_at(1, xiR)
    assert np.abs(xl - xr).max() <= 1e-13


def test_deformation_really_curves_the_cells():
    m = curved.CurvedBoxMesh(3, 2, 2, 2, amp=0.05)
    xi = np.random.default_rng(1).uniform(0, 1, (20, 3))
    J = m.jac_at(3, xi)
    assert np.abs(J - J[0]).max() > 1e-3        # not constant over the cell


def test_periodic_constants_symmetry_and_semidefinite():
    m = curved.CurvedBoxMesh(2, 3, 2, 2, amp=0.06, periodic=(True, True, True))
    A = curved.CurvedSIPG(m, 0.0, 1.0, 1.0).assemble()
    assert np.abs(A @ np.ones(m.ndofs)).max() <= 1e-11 * abs(A).max()
    assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() >= -1e-11 * ev.max() and np.sum(ev < 1e-10 * ev.max()) == 1


def test_dirichlet_and_neumann_walls_on_curved_cells():
    m = curved.CurvedBoxMesh(2, 2, 3, 2, amp=0.04, ly=2.0, y0=-1.0, periodic=(True, False, True),
                             neumann=(False, False, True, True, False, False))
    A = curved.CurvedSIPG(m, 0.0, 1.0, 1.0).assemble()
    assert np.abs(A @ np.ones(m.ndofs)).max() <= 1e-11 * abs(A).max()     # Neumann walls: singular
    md = curved.CurvedBoxMesh(2, 2, 3, 2, amp=0.04, ly=2.0, y0=-1.0, periodic=(True, False, True))
    Ad = curved.CurvedSIPG(md, 0.0, 1.0, 1.0).assemble()
    assert np.linalg.eigvalsh(Ad.toarray()).min() > 0                      # Dirichlet walls: definite


def _u(x, y, z):
    return np.sin(2 * math.pi * x) * np.sin(2 * math.pi * y) * np.sin(2 * math.pi * z)


def test_manufactured_solution_converges_at_order_k_plus_1():
    """-lap u + u = f on the curved periodic unit cube, u = sin sin sin (periodic in x)."""
    k = 2
    errs = []
    for nc in (4, 8):
        m = curved.CurvedBoxMesh(k, nc, nc, nc, amp=0.04, periodic=(True, True, True))
        op = curved.CurvedSIPG(m, 1.0, 1.0, 1.0)
        b = op.rhs(lambda x, y, z: (12 * math.pi ** 2 + 1) * _u(x, y, z))
        x = spla.spsolve(op.assemble().tocsc(), b)
        errs.append(op.l2_error(x, _u))
    rate = math.log2(errs[0] / errs[1])
    assert rate > k + 1 - 0.4, (errs, rate)
    assert errs[1] < 2e-2


def test_multigrid_on_a_curved_finest_level():
    """The V-cycle with a curved finest level (coarse levels on the undeformed box)
    is a symmetric positive definite preconditioner that cuts CG iterations."""
    from oracle import multigrid as omg, solvers
    m = curved.CurvedBoxMesh(2, 4, 4, 2, amp=0.05, periodic=(True, True, True))
    mg = omg.Multigrid(m, 1.0, 1.0, 1.0)
    assert isinstance(mg.ops[0], curved.CurvedSIPG) and not isinstance(mg.meshes[1], curved.CurvedBoxMesh)
    A = mg.A[0]
    g = np.random.default_rng(3)
    r1, r2 = g.uniform(-1, 1, m.ndofs), g.uniform(-1, 1, m.ndofs)
    z1, z2 = mg.vcycle(r1), mg.vcycle(r2)
    assert abs(r2 @ z1 - r1 @ z2) <= 1e-10 * abs(r1 @ z2) and r1 @ z1 > 0
    b = g.uniform(-1, 1, m.ndofs)
    dinv = 1.0 / A.diagonal()
    _, it_mg, st, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(m.ndofs), mg.vcycle, 1e-10, 200)
    _, it_j, st2, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(m.ndofs), lambda r: dinv * r, 1e-10, 2000)
    assert st == solvers.OK and st2 == solvers.OK and it_mg < it_j / 2
