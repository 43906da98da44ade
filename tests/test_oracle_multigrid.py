"""Pins of the oracle's geometric multigrid V-cycle preconditioner.

Transfers are pinned by exact reproduction of polynomials, the Chebyshev
pieces by closed forms (error polynomial on eigenvectors, known spectra of
the periodic 1D Laplacian), and the V-cycle by what multigrid must deliver:
a symmetric positive definite preconditioner whose PCG iteration count does
not grow under refinement and is far below point Jacobi's.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import basis, mesh, multigrid as mgm, solvers
import dgmf_inputs as inp


def test_level_counts():
    assert mgm.level_counts((64, 64, 64)) == [(64,) * 3, (32,) * 3, (16,) * 3, (8,) * 3, (4,) * 3, (2,) * 3, (1,) * 3]
    assert mgm.level_counts((48, 32, 48)) == [(48, 32, 48), (24, 16, 24), (12, 8, 12), (6, 4, 6), (3, 2, 3),
                                              (3, 1, 3)]
    assert mgm.level_counts((3, 5, 1)) == [(3, 5, 1)]


@pytest.mark.parametrize("k,nc", [(1, (4, 2, 2)), (2, (2, 4, 3)), (3, (2, 2, 2)), (4, (4, 1, 2))])
def test_prolongation_embeds_polynomials(k, nc):
    """A polynomial of degree <= k per direction on the mother cells is the same function on the children."""
    fine = mesh.BoxMesh(k, *nc, lx=1.0, ly=1.5, lz=0.8, periodic=(False, False, False))
    coarse = mgm.coarser_mesh(fine, mgm.level_counts(nc)[1])
    cx = inp.uniform(30 + k, 3 * (k + 1)).reshape(3, k + 1)

    def f(x, y, z):
        return (sum(cx[0, p] * x ** p for p in range(k + 1)) * sum(cx[1, p] * y ** p for p in range(k + 1))
                * sum(cx[2, p] * z ** p for p in range(k + 1)))

    Xf, Xc = fine.node_coords(), coarse.node_coords()
    P = mgm.prolongation(fine, coarse)
    uf = P @ f(Xc[:, 0], Xc[:, 1], Xc[:, 2])
    want = f(Xf[:, 0], Xf[:, 1], Xf[:, 2])
    assert np.abs(uf - want).max() <= 1e-12 * np.abs(want).max()


def test_prolongation_rows_sum_to_one():
    """Constants are embedded exactly: every row of P sums to one, including non-halved directions."""
    fine = mesh.BoxMesh(3, 4, 3, 2)
    coarse = mgm.coarser_mesh(fine, (2, 3, 1))
    P = mgm.prolongation(fine, coarse)
    np.testing.assert_allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0, rtol=0, atol=1e-13)


def test_chebyshev_error_polynomial_on_eigenvectors():
    """Error after the iteration is T_m((theta - lam)/delta) / T_m(theta/delta) times the initial error."""
    n = 12
    Q, _ = np.linalg.qr(inp.uniform(3, n * n).reshape(n, n))
    lam = np.linspace(0.3, 2.0, n)
    A = (Q * lam) @ Q.T
    a, b, m = 0.25, 2.1, 6
    theta, delta = 0.5 * (a + b), 0.5 * (b - a)
    for j in (0, 5, 11):
        e = Q[:, j]
        x = mgm.chebyshev_interval(lambda u: A @ u, np.ones(n), A @ e, a, b, m)
        g = C.Chebyshev.basis(m)
        np.testing.assert_allclose(e - x, g((theta - lam[j]) / delta) / g(theta / delta) * e, atol=1e-13)
        x1 = mgm.chebyshev_interval(lambda u: A @ u, np.ones(n), A @ e, a, b, m, x0=0.3 * e)
        np.testing.assert_allclose(e - x1, 0.7 * g((theta - lam[j]) / delta) / g(theta / delta) * e, atol=1e-13)


def test_coarse_degree_closed_form():
    # 1/T_m(sigma) <= tol  <=>  m >= acosh(1/tol)/acosh(sigma)
    for a, b, tol in ((0.1, 3.0, 1e-3), (1.0, 2.0, 1e-6), (0.01, 1.0, 1e-3)):
        m = mgm.coarse_degree(a, b, tol)
        sigma = (b + a) / (b - a)
        assert 1.0 / math.cosh(m * math.acosh(sigma)) <= tol < 1.0 / math.cosh((m - 1) * math.acosh(sigma))


def test_full_lanczos_extremes_of_periodic_laplacian():
    """Periodic 1D Laplacian: eigenvalues 2 - 2 cos(2 pi j / N), null vector constant (deflated)."""
    N = 40
    A = 2 * np.eye(N) - np.roll(np.eye(N), 1, 1) - np.roll(np.eye(N), -1, 1)
    v0 = inp.uniform(4, N)
    lo, hi = mgm.lanczos_full(lambda v: A @ v, v0, N - 1, null=np.ones(N) / math.sqrt(N))
    assert abs(lo - (2 - 2 * math.cos(2 * math.pi / N))) < 1e-12
    assert abs(hi - 4.0) < 1e-12


@pytest.fixture(scope="module")
def periodic_hierarchies():
    out = {}
    for nc in (4, 8):
        m = mesh.BoxMesh(2, nc, nc, nc)
        out[nc] = (m, mgm.Multigrid(m, 0.0, 1.0, 1.0 / 3.0, singular=True))
    return out


def test_vcycle_is_symmetric_positive_definite(periodic_hierarchies):
    m, mg = periodic_hierarchies[4]
    x, y = inp.uniform(6, m.ndofs), inp.uniform(7, m.ndofs)
    Bx, By = mg.vcycle(x), mg.vcycle(y)
    assert abs(x @ By - y @ Bx) <= 1e-13 * abs(x @ Bx)
    for s in range(8, 12):
        v = inp.uniform(s, m.ndofs)
        v -= v.mean()
        assert v @ mg.vcycle(v) > 0


def test_coarse_solver_reaches_its_tolerance(periodic_hierarchies):
    m, mg = periodic_hierarchies[4]
    A = mg.A[-1].toarray()
    b = inp.uniform(13, A.shape[0])
    b -= b.mean()
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    xs -= xs.mean()
    x = mg.coarse_solve(b)
    e = x - xs
    e -= e.mean()
    assert math.sqrt(e @ A @ e) <= 1e-3 * math.sqrt(xs @ A @ xs)


def test_mg_pcg_iterations_do_not_grow_under_refinement(periodic_hierarchies):
    its = {}
    for nc, (m, mg) in periodic_hierarchies.items():
        A = mg.A[0]
        b = inp.uniform(5, m.ndofs)
        _, it, st, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(m.ndofs), mg.vcycle, 1e-10, 100, project_mean=True)
        assert st == solvers.OK
        its[nc] = it
        if nc == 8:
            d = A.diagonal()
            _, itj, _, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(m.ndofs), lambda r: r / d, 1e-10, 2000,
                                       project_mean=True)
            assert itj > 8 * it
    assert its[4] <= 15 and abs(its[8] - its[4]) <= 1


def test_mg_on_graded_dirichlet_helmholtz():
    m = mesh.BoxMesh(2, 8, 8, 8, lx=2 * math.pi, ly=2.0, lz=math.pi, y0=-1.0, periodic=(True, False, True),
                     y_tanh_gamma=1.5)
    mg = mgm.Multigrid(m, 100.0, 0.01, 1.0)
    A = mg.A[0]
    b = inp.uniform(5, m.ndofs)
    _, it, st, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(m.ndofs), mg.vcycle, 1e-10, 100)
    assert st == solvers.OK and it <= 12
