"""Pins of the oracle's SIPG operator with homogeneous Neumann sides.

Homogeneous Neumann faces add no term to the bilinear form (Sec. 3.2: the
flux takes the own trace, the gradient flux is data) while their area counts
in tau_e (eq. taue).  Checked against facts that do not come from the oracle:
constants lie in the null space once no Dirichlet face is left; the first
eigenvalue of A x = lambda M x on the unit cube is pi^2 times the number of
Dirichlet directions (a Neumann direction admits cos(pi x) and the constant,
a Dirichlet one needs sin(pi x)); and a manufactured solution with zero
normal derivative on the Neumann sides converges at order k+1.  A Neumann
face treated as Dirichlet (or dropped from tau_e) fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import mesh as omesh, multigrid as omg, sipg

ALL_N = (True,) * 6


def test_neumann_flags_are_ignored_in_periodic_directions():
    m = omesh.BoxMesh(2, 2, 2, 2, periodic=(True, False, True), neumann=ALL_N)
    assert m.neumann == (False, False, True, True, False, False)
    assert m.has_neumann()
    assert len(m.boundary_faces()) == 0 and len(m.neumann_faces()) == 2 * 4


@pytest.mark.parametrize("k, cells, periodic, gamma", [
    (2, (3, 2, 2), (False, False, False), 0.0),
    (3, (2, 3, 2), (True, False, True), 1.5),     # channel pressure: Neumann walls in y
    (1, (2, 2, 3), (False, True, False), 0.0),
])
def test_constants_span_the_null_space(k, cells, periodic, gamma):
    m = omesh.BoxMesh(k, *cells, ly=2.0, y0=-1.0, periodic=periodic, y_tanh_gamma=gamma, neumann=ALL_N)
    A = sipg.SIPG(m, 0.0, 1.0, 1.0).assemble()
    one = np.ones(m.ndofs)
    assert np.abs(A @ one).max() <= 1e-11 * abs(A).max()
    assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
    ev = np.linalg.eigvalsh(A.toarray())
    scale = ev.max()
    assert ev.min() >= -1e-11 * scale
    assert np.sum(ev < 1e-10 * scale) == 1           # only the constant
    # the same mesh with Dirichlet sides is definite: the flags change the operator
    md = omesh.BoxMesh(k, *cells, ly=2.0, y0=-1.0, periodic=periodic, y_tanh_gamma=gamma)
    if not all(periodic):
        Ad = sipg.SIPG(md, 0.0, 1.0, 1.0).assemble()
        assert np.abs(Ad @ one).max() > 1e-3 * abs(Ad).max()


def test_penalty_counts_neumann_faces_like_dirichlet_faces():
    md = omesh.BoxMesh(2, 3, 2, 2, periodic=(False, True, True))
    mn = omesh.BoxMesh(2, 3, 2, 2, periodic=(False, True, True), neumann=(True, False) + (False,) * 4)
    # eq. taue: the whole boundary area, both parts
    assert np.array_equal(sipg.penalty_per_cell(md), sipg.penalty_per_cell(mn))
    h = 1.0 / 3.0
    # a cell on the x boundary: A_int/2 + A_bnd = (1 + 4) / 2 * a_x... computed from the definition
    c = md.cell_index(0, 0, 0)
    ax, ay, az = 0.5 * 0.5, h * 0.5, h * 0.5
    expect = 9 * (ax + ax / 2 + ay + az) / (h * 0.25)
    assert abs(sipg.penalty_per_cell(mn)[c] - expect) <= 1e-12 * expect


@pytest.mark.parametrize("neumann, n_dirichlet", [
    (ALL_N, 0),
    ((True, True, False, False, False, False), 2),
    ((False, False, True, True, True, True), 1),
    ((True, False, False, False, False, False), None),   # mixed in x: sin(pi x / 2) mode
])
def test_first_eigenvalue(neumann, n_dirichlet):
    m = omesh.BoxMesh(4, 2, 2, 2, periodic=(False, False, False), neumann=neumann)
    op = sipg.SIPG(m, 0.0, 1.0, 1.0)
    A, M = op.assemble().toarray(), op.mass_matrix().toarray()
    ev = sla.eigh(A, M, eigvals_only=True, subset_by_index=[0, 2])
    if n_dirichlet == 0:
        assert abs(ev[0]) <= 1e-9 and abs(ev[1] - math.pi ** 2) <= 1e-5 * math.pi ** 2
    elif n_dirichlet is None:
        # x: Neumann at 0, Dirichlet at 1 -> cos(pi x / 2); y, z Dirichlet -> sin(pi y) sin(pi z)
        lam = (math.pi / 2) ** 2 + 2 * math.pi ** 2
        assert abs(ev[0] - lam) <= 1e-5 * lam
    else:
        lam = n_dirichlet * math.pi ** 2
        assert abs(ev[0] - lam) <= 1e-5 * lam


def _u(x, y, z):
    return np.cos(math.pi * x) * np.sin(math.pi * y) * np.sin(math.pi * z)


def test_manufactured_solution_converges_at_order_k_plus_1():
    """-lap u = f, u = cos(pi x) sin(pi y) sin(pi z): du/dn = 0 on x = 0, 1 (Neumann),
    u = 0 on the y and z sides (homogeneous Dirichlet)."""
    k = 2
    errs = []
    for nc in (2, 4):
        m = omesh.BoxMesh(k, nc, nc, nc, periodic=(False, False, False), neumann=(True, True) + (False,) * 4)
        op = sipg.SIPG(m, 0.0, 1.0, 1.0)
        b = op.rhs(lambda x, y, z: 3 * math.pi ** 2 * _u(x, y, z))
        x = spla.spsolve(op.assemble().tocsc(), b)
        errs.append(sipg.l2_error(m, x, _u))
    rate = math.log2(errs[0] / errs[1])
    assert rate > k + 1 - 0.4, (errs, rate)
    # the same right-hand side with Dirichlet x sides converges to another function
    m = omesh.BoxMesh(k, 4, 4, 4, periodic=(False, False, False))
    op = sipg.SIPG(m, 0.0, 1.0, 1.0)
    x = spla.spsolve(op.assemble().tocsc(), op.rhs(lambda x, y, z: 3 * math.pi ** 2 * _u(x, y, z)))
    assert sipg.l2_error(m, x, _u) > 10 * errs[1]


def test_apply_cells_and_diagonal_match_assembly():
    m = omesh.BoxMesh(2, 3, 2, 2, ly=2.0, y0=-1.0, periodic=(True, False, False), y_tanh_gamma=1.2,
                      neumann=(False, False, True, True, False, True))
    op = sipg.SIPG(m, 3.0, 0.5, 1.0)
    A = op.assemble()
    u = np.random.default_rng(3).uniform(-1, 1, m.ndofs)
    cells = list(range(m.ncells))
    assert np.abs(op.apply_cells(u, cells).ravel() - A @ u).max() <= 1e-12 * np.abs(A @ u).max()
    assert np.abs(op.diagonal_cells(cells).ravel() - A.diagonal()).max() <= 1e-12 * np.abs(A.diagonal()).max()


def test_multigrid_hierarchy_keeps_the_neumann_sides():
    m = omesh.BoxMesh(2, 4, 4, 2, periodic=(True, False, True), neumann=ALL_N)
    c = omg.coarser_mesh(m, (2, 2, 1))
    assert c.neumann == m.neumann
    mg = omg.Multigrid(m, 0.0, 1.0, 1.0, singular=True)
    r = np.random.default_rng(4).uniform(-1, 1, m.ndofs)
    r -= r.mean()
    z = mg.vcycle(r)
    assert np.isfinite(z).all() and np.dot(r, z) > 0       # a positive definite preconditioner on 1^perp
