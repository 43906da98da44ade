"""Pins of the oracle's PCG, Lanczos and Chebyshev against exact linear algebra."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import kron, mesh, rng, sipg, solvers
import dgmf_inputs as inp


@pytest.fixture(scope="module")
def c0():
    w = inp.POISSON_C0
    m = mesh.BoxMesh(w.degree, *w.cells)
    op = sipg.SIPG(m, penalty_scale=w.penalty_scale)
    A = op.assemble()
    b = op.rhs(inp.poisson_rhs_sin3)
    kr = kron.KronPeriodic(w.degree, *w.cells, penalty_scale=w.penalty_scale)
    return m, op, A, b, kr


def _gauge(m, x):
    wts = sipg.integral_weights(m)
    return x - (wts @ x) / wts.sum()


def test_jacobi_pcg_reaches_tolerance_and_fdm(c0):
    m, op, A, b, kr = c0
    dinv = 1.0 / A.diagonal()
    x, it, st, rel = solvers.pcg(lambda v: A @ v, b, np.zeros_like(b), lambda r: dinv * r, 1e-10, 1000,
                                 project_mean=True)
    assert st == solvers.OK
    bp = b - b.mean()
    assert np.linalg.norm(bp - A @ x) <= 1.01e-10 * np.linalg.norm(bp)
    xf = kr.solve(bp)
    err = np.linalg.norm(_gauge(m, x) - xf) / np.linalg.norm(xf)
    assert err < 1e-8
    assert 5 <= it < 400


def test_pcg_status_codes():
    A = np.diag([1.0, 2.0, 3.0, 4.0])
    b = np.ones(4)
    _, it, st, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(4), lambda r: r, 1e-14, 1)
    assert st == solvers.NOT_CONVERGED and it == 1
    _, _, st, _ = solvers.pcg(lambda v: A @ v, np.array([1.0, np.nan, 0, 0]), np.zeros(4), lambda r: r, 1e-10, 10)
    assert st == solvers.NONFINITE
    _, _, st, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(4), lambda r: -r, 1e-10, 10)
    assert st == solvers.BREAKDOWN
    _, _, st, _ = solvers.pcg(lambda v: -(A @ v), b, np.zeros(4), lambda r: r, 1e-10, 10)
    assert st == solvers.BREAKDOWN
    x, it, st, _ = solvers.pcg(lambda v: A @ v, b, np.ones(4) / np.diag(A), lambda r: r, 1e-10, 10)
    assert st == solvers.OK and it == 0


def test_cg_exact_in_n_steps_on_small_spd():
    rng_ = np.random.default_rng(3)
    Q = rng_.standard_normal((6, 6))
    A = Q @ Q.T + 6 * np.eye(6)
    b = rng_.standard_normal(6)
    x, it, st, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(6), lambda r: r, 1e-13, 6)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10)


def test_lanczos_brackets_largest_eigenvalue():
    m = mesh.BoxMesh(3, 3, 3, 3)
    op = sipg.SIPG(m, penalty_scale=1.0 / 3.0)
    A = op.assemble()
    d = A.diagonal()
    S = lambda v: (A @ (v / np.sqrt(d))) / np.sqrt(d)
    v0 = rng.uniform_pm1(11, m.ndofs)
    v0 -= v0.mean()
    ritz, T = solvers.lanczos_ritz(S, v0, 15)
    lam_max = np.linalg.eigvalsh((A.toarray() / np.sqrt(d)[:, None]) / np.sqrt(d)[None, :])[-1]
    assert ritz[-1] <= lam_max * (1 + 1e-12)
    assert lam_max <= 1.2 * ritz[-1]
    # with as many steps as unknowns Lanczos is exact on a tiny matrix
    B = np.diag([1.0, 2.0, 5.0, 9.0])
    r2, _ = solvers.lanczos_ritz(lambda v: B @ v, np.ones(4), 4)
    np.testing.assert_allclose(r2, [1, 2, 5, 9], rtol=1e-12)


def test_chebyshev_closed_form_on_eigenvectors():
    m = mesh.BoxMesh(2, 2, 2, 2)
    A = sipg.SIPG(m).assemble().toarray()
    d = np.diag(A)
    dinv = 1.0 / d
    # eigenpairs of D^{-1} A via the symmetric form
    lam, W = np.linalg.eigh(A / np.sqrt(d)[:, None] / np.sqrt(d)[None, :])
    lam_max = 1.2 * lam[-1]
    for idx in (1, 5, len(lam) // 2, len(lam) - 1):
        v = W[:, idx] / np.sqrt(d)           # eigenvector of D^{-1}A
        r = d * v                             # so that D^{-1} r = v
        z = solvers.chebyshev_jacobi(lambda u: A @ u, dinv, r, lam_max, 20.0, 5)
        q = solvers.chebyshev_polynomial_value(lam[idx], lam_max, 20.0, 5)
        np.testing.assert_allclose(z, q * v, rtol=1e-10, atol=1e-12 * np.abs(v).max())


def test_chebyshev_operator_is_symmetric():
    m = mesh.BoxMesh(2, 2, 2, 2, periodic=(True, False, True))
    A = sipg.SIPG(m).assemble()
    dinv = 1.0 / A.diagonal()
    g = np.random.default_rng(4)
    x, y = g.standard_normal(m.ndofs), g.standard_normal(m.ndofs)
    P = lambda r: solvers.chebyshev_jacobi(lambda u: A @ u, dinv, r, 2.0, 20.0, 5)
    assert abs(x @ P(y) - P(x) @ y) < 1e-12 * abs(x @ P(y))


def test_flexible_beta_equals_standard_with_linear_preconditioner(c0):
    m, op, A, b, kr = c0
    dinv = 1.0 / A.diagonal()
    xa, ia, _, _ = solvers.pcg(lambda v: A @ v, b, np.zeros_like(b), lambda r: dinv * r, 1e-10, 500, project_mean=True)
    xb, ib, _, _ = solvers.pcg(lambda v: A @ v, b, np.zeros_like(b), lambda r: dinv * r, 1e-10, 500, project_mean=True,
                               flexible=True)
    assert ia == ib
    assert np.linalg.norm(xa - xb) < 1e-9 * np.linalg.norm(xa)
