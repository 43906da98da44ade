"""Pins of the oracle's SIPG operator against what the mathematics fixes.

Independent checks: symmetry and semi-definiteness, null space of the
periodic Laplacian, the Kronecker-sum construction (built from 1D point
fluxes, not from the 3D face assembly), consistency (exact reproduction of
polynomials of degree <= k including Dirichlet data terms), the first
periodic eigenvalue (2 pi)^2, optimal L2 order k+1, the 1D coercivity
threshold, and the row-restricted/diagonal paths against the CSR matrix.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import kron, mesh, sipg, solvers
import dgmf_inputs as inp


def _sym_rel(A):
    return abs(A - A.T).max() / abs(A).max()


MESHES = {
    "periodic_2c_k2": lambda: mesh.BoxMesh(2, 2, 2, 2),
    "periodic_aniso_k3": lambda: mesh.BoxMesh(3, 3, 2, 1, lx=1.3, ly=0.7, lz=0.4),
    "dirichlet_y_tanh_k2": lambda: mesh.BoxMesh(2, 2, 3, 2, lx=2 * math.pi, ly=2.0, lz=math.pi, y0=-1.0,
                                              periodic=(True, False, True), y_tanh_gamma=1.8),
    "all_dirichlet_k2": lambda: mesh.BoxMesh(2, 2, 2, 2, periodic=(False, False, False)),
    "sheared_periodic_k2": lambda: mesh.BoxMesh(2, 2, 2, 2, shear=[[1, 0.3, 0], [0, 1, 0.2], [0.1, 0, 1]]),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_symmetry_and_semidefinite(name):
    m = MESHES[name]()
    op = sipg.SIPG(m, penalty_scale=1.0)
    A = op.assemble().toarray()
    assert _sym_rel(A) < 1e-14
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    periodic = all(m.periodic)
    if periodic:
        assert ev[0] > -1e-12 * ev[-1]
        assert abs(ev[0]) < 1e-11 * ev[-1]
        assert ev[1] > 1e-6 * ev[-1]          # one-dimensional null space
        ones = np.ones(m.ndofs)
        assert np.abs(A @ ones).max() < 1e-12 * np.abs(A).max()
    else:
        assert ev[0] > 1e-8 * ev[-1]          # Dirichlet walls: definite


@pytest.mark.slow
def test_c0_semidefinite_dense():
    w = inp.POISSON_C0
    m = mesh.BoxMesh(w.degree, *w.cells)
    A = sipg.SIPG(m, penalty_scale=w.penalty_scale).assemble().toarray()
    assert _sym_rel(A) < 1e-14
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-12 * ev[-1] and ev[1] > 1e-8 * ev[-1]
    assert np.abs(A.sum(axis=1)).max() < 1e-12 * np.abs(A).max()


def test_c0_penalty_is_k1_squared_over_h():
    w = inp.POISSON_C0
    m = mesh.BoxMesh(w.degree, *w.cells)
    tau = sipg.penalty_per_cell(m, w.penalty_scale)
    np.testing.assert_allclose(tau, (w.degree + 1) ** 2 / 0.25, rtol=1e-14)


@pytest.mark.parametrize("k,cells,lengths,mu", [(2, (2, 3, 2), (1.0, 1.0, 1.0), 0.0),
                                                (3, (3, 2, 2), (1.3, 0.7, 0.4), 5.0),
                                                (1, (1, 2, 3), (1.0, 2.0, 1.0), 0.0),
                                                (4, (2, 2, 2), (1.0, 1.0, 1.0), 1000.0)])
def test_kronecker_sum_equals_assembly(k, cells, lengths, mu):
    m = mesh.BoxMesh(k, *cells, lx=lengths[0], ly=lengths[1], lz=lengths[2])
    nu = 0.01 if mu > 100 else 1.0
    op = sipg.SIPG(m, mass_coeff=mu, diff_coeff=nu)
    A = op.assemble()
    kr = kron.KronPeriodic(k, *cells, *lengths, mass_coeff=mu, diff_coeff=nu)
    u = np.random.default_rng(0).uniform(-1, 1, m.ndofs)
    y1, y2 = A @ u, kr.apply(u)
    assert np.abs(y1 - y2).max() < 1e-13 * np.abs(y1).max()


def test_first_periodic_eigenvalue_is_2pi_squared():
    kr = kron.KronPeriodic(3, 8, 8, 8)
    lam = np.sort(kr.eigenvalues().ravel())
    assert abs(lam[0]) < 1e-8
    np.testing.assert_allclose(lam[1:7], (2 * math.pi) ** 2, rtol=2e-4)   # 6-fold (+-x, +-y, +-z)
    # the same value from the 3D assembly on a small mesh (generalised eigenproblem)
    m = mesh.BoxMesh(3, 4, 4, 4)
    op = sipg.SIPG(m)
    ev = sla.eigh(op.assemble().toarray(), op.mass_matrix().toarray(), eigvals_only=True, subset_by_index=[0, 1])
    assert abs(ev[1] - (2 * math.pi) ** 2) < 0.01 * (2 * math.pi) ** 2


@pytest.mark.parametrize("k", range(1, 8))
def test_1d_coercivity_threshold(k):
    """1D periodic GLL-SIPG is PSD with a 1D null space iff tau*h > k(k+1)/2."""
    h = 0.5
    thr = k * (k + 1) / 2 / h
    for fac, psd in ((0.98, False), (1.02, True)):
        K1, _ = kron.sipg_1d(k, 4, h, fac * thr)
        ev = np.linalg.eigvalsh(K1)
        if psd:
            assert ev[0] > -1e-10 * ev[-1] and ev[1] > 1e-10 * ev[-1]
        else:
            assert ev[0] < -1e-8 * ev[-1]


def _poly_y(k):
    c = [0.3, -0.5, 0.8, 0.2, -0.4, 0.1, 0.05, -0.02][:k + 1]
    p = lambda y: sum(ci * y ** i for i, ci in enumerate(c))
    d2 = lambda y: sum(ci * i * (i - 1) * y ** (i - 2) for i, ci in enumerate(c) if i >= 2)
    return p, d2


@pytest.mark.parametrize("k", [1, 2, 4])
def test_consistency_polynomial_in_y_channel(k):
    """u = p(y), deg p <= k, g = p on the walls: H u_I = b exactly (Galerkin consistency)."""
    m = mesh.BoxMesh(k, 2, 4, 2, lx=2 * math.pi, ly=2.0, lz=math.pi, y0=-1.0,
                     periodic=(True, False, True), y_tanh_gamma=1.8)
    mu, nu = 1000.0, 0.01
    op = sipg.SIPG(m, mass_coeff=mu, diff_coeff=nu)
    p, d2 = _poly_y(k)
    X = m.node_coords()
    uI = p(X[:, 1])
    b = op.rhs(lambda x, y, z: mu * p(y) - nu * d2(y), g=lambda x, y, z: p(y))
    Hu = op.assemble() @ uI
    assert np.abs(Hu - b).max() < 1e-12 * np.abs(b).max()
    Hu2 = op.apply_cells(uI, list(range(m.ncells))).ravel()
    assert np.abs(Hu2 - b).max() < 1e-12 * np.abs(b).max()


def test_consistency_qk_all_dirichlet():
    k = 2
    m = mesh.BoxMesh(k, 2, 2, 3, lx=1.0, ly=0.8, lz=1.5, periodic=(False, False, False))
    op = sipg.SIPG(m, mass_coeff=0.0, diff_coeff=1.0)
    u = lambda x, y, z: (x ** 2 - 0.5 * x) * (y + 0.2) * (1 - z ** 2) + 0.7 * x * y * z
    lap = lambda x, y, z: 2 * (y + 0.2) * (1 - z ** 2) + (x ** 2 - 0.5 * x) * (y + 0.2) * (-2)
    X = m.node_coords()
    uI = u(X[:, 0], X[:, 1], X[:, 2])
    b = op.rhs(lambda x, y, z: -lap(x, y, z), g=u)
    Hu = op.assemble() @ uI
    assert np.abs(Hu - b).max() < 1e-12 * np.abs(b).max()


def test_helmholtz_is_mu_mass_plus_nu_laplace():
    m = MESHES["dirichlet_y_tanh_k2"]()
    H = sipg.SIPG(m, mass_coeff=7.0, diff_coeff=0.3).assemble()
    A = sipg.SIPG(m, mass_coeff=0.0, diff_coeff=1.0).assemble()
    M = sipg.SIPG(m, mass_coeff=1.0, diff_coeff=0.0).assemble()
    assert abs(H - 7.0 * M - 0.3 * A).max() < 1e-13 * abs(H).max()
    assert abs(M - sipg.SIPG(m).mass_matrix()).max() < 1e-15 * abs(M).max()
    ev = np.linalg.eigvalsh(H.toarray())
    assert ev[0] > 0


@pytest.mark.parametrize("name", list(MESHES) + ["periodic_1cell_x"])
def test_apply_cells_and_diagonal_match_csr(name):
    m = mesh.BoxMesh(2, 1, 2, 2) if name == "periodic_1cell_x" else MESHES[name]()
    op = sipg.SIPG(m, mass_coeff=3.0, diff_coeff=0.5)
    A = op.assemble()
    u = np.random.default_rng(1).uniform(-1, 1, m.ndofs)
    cells = list(range(m.ncells))
    y = op.apply_cells(u, cells).ravel()
    assert np.abs(y - A @ u).max() < 1e-13 * np.abs(y).max()
    dg = op.diagonal_cells(cells).ravel()
    assert np.abs(dg - A.diagonal()).max() < 1e-14 * np.abs(dg).max()


def test_optimal_l2_convergence_order():
    """Periodic Poisson with f = 3(2pi)^2 sin sin sin: L2 error of order k+1."""
    k = 3
    errs = []
    for nc in (2, 4, 8):
        m = mesh.BoxMesh(k, nc, nc, nc)
        op = sipg.SIPG(m, penalty_scale=1.0 / 3.0)
        b = op.rhs(inp.poisson_rhs_sin3)
        b -= b.mean()
        kr = kron.KronPeriodic(k, nc, nc, nc, penalty_scale=1.0 / 3.0)
        x = kr.solve(b)
        errs.append(sipg.l2_error(m, x, inp.sin3))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 1 - 0.3, (errs, rates)


def test_fdm_solution_solves_assembled_system():
    w = inp.POISSON_C0
    m = mesh.BoxMesh(w.degree, *w.cells)
    op = sipg.SIPG(m, penalty_scale=w.penalty_scale)
    A = op.assemble()
    b = op.rhs(inp.poisson_rhs_sin3)
    b -= b.mean()
    kr = kron.KronPeriodic(w.degree, *w.cells, penalty_scale=w.penalty_scale)
    x = kr.solve(b)
    assert np.linalg.norm(A @ x - b) < 1e-11 * np.linalg.norm(b)
    wts = sipg.integral_weights(m)
    assert abs(wts @ x) < 1e-12 * np.abs(x).max()          # zero integral mean
    assert abs(wts.sum() - 1.0) < 1e-14                     # partition of unity on the unit cube


@pytest.mark.parametrize("k,cells,lengths", [(1, (3, 2, 4), (1.0, 1.0, 1.0)), (2, (2, 3, 1), (0.7, 1.1, 0.4)),
                                             (3, (4, 4, 4), (1.0, 1.0, 1.0)), (4, (2, 2, 3), (1.0, 2.0, 1.5))])
def test_block_stencil_apply(k, cells, lengths):
    """The block-stencil product (all cells at once) equals the assembled matrix, including
    directions with a single periodic cell."""
    m = mesh.BoxMesh(k, *cells, *lengths)
    op = sipg.SIPG(m, mass_coeff=3.0, diff_coeff=0.5, penalty_scale=1.0 / 3.0)
    u = inp.uniform(21 + k, m.ndofs)
    want = op.assemble() @ u
    got = op.apply_block_stencil(u)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
