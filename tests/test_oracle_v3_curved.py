"""Pins of the oracle's divergence A and gradient B (variant V3c) on curved cells.

Sec. 4.2 (eqs. av3, bv3) with the curved iso-parametric cells of Sec. 5.
Fixed by facts outside the oracle:
  - zero amplitude gives the affine operators (pinned separately);
  - with enough points to integrate exactly (the cofactors of J have degree
    <= 2k per reference direction): A and B annihilate constants on a
    periodic curved mesh (3k per direction, n_q >= (3k+1)/2), and A = -B^T
    there (integration by parts of div(p u), 4k per direction,
    n_q >= (4k+1)/2) -- a wrong cofactor, a transposed inverse or a normal
    of the wrong size breaks these;
  - with the defining k+1 points, A applied to the interpolant of a smooth
    periodic field tends to -(phi_i, div u) at a rate that rises with the
    degree;
  - the coordinate functions lie in the iso-parametric space, so their
    physical gradients are the unit vectors at every point; D_e annihilates
    constant fields, is semi-definite and gives u.D u = V for u = (x, 0, 0);
    the penalty of a constant field uses the curved volume; zero amplitude
    gives the affine penalty and projection.
"""
import numpy as np
import pytest

from oracle import curved, mesh as omesh, sipg, v3
import dgmf_inputs as inp


def test_zero_amplitude_is_the_affine_operator():
    kw = dict(lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, False), y_tanh_gamma=1.3,
              neumann=(False, False, False, False, True, False))
    cm = curved.CurvedBoxMesh(2, 2, 3, 2, amp=0.0, **kw)
    am = omesh.BoxMesh(2, 2, 3, 2, **kw)
    for f in (v3.divergence_matrix, v3.gradient_matrix):
        A, B = f(cm), f(am)
        assert abs(A - B).max() <= 1e-13 * abs(B).max()


@pytest.mark.parametrize("k", [2, 3])
def test_exact_quadrature_identities_on_a_periodic_curved_mesh(k):
    m = curved.CurvedBoxMesh(k, 2, 3, 2, amp=0.07, periodic=(True, True, True))
    N = m.ndofs
    nq = 2 * k + 1
    A = v3.divergence_matrix(m, nq=nq)
    B = v3.gradient_matrix(m, nq=nq)
    one = np.ones(N)
    for a in range(3):
        u = np.zeros(3 * N)
        u[a * N:(a + 1) * N] = 1.0
        assert np.abs(A @ u).max() < 1e-13 * abs(A).max()
    assert np.abs(B @ one).max() < 1e-13 * abs(B).max()
    assert abs(A + B.T).max() < 1e-13 * abs(A).max()
    # with the defining k+1 points neither identity is exact on curved cells
    A1 = v3.divergence_matrix(m)
    assert abs(A1 + v3.gradient_matrix(m).T).max() > 1e-8 * abs(A1).max()


def _u(x, y, z):
    tp = 2 * np.pi
    return np.stack([np.sin(tp * y) * np.cos(tp * z) + np.sin(tp * x),
                     np.sin(tp * z) + 0.2 * np.cos(tp * y),
                     np.cos(tp * x) * np.sin(tp * z)])


def _div_u(x, y, z):
    tp = 2 * np.pi
    return tp * np.cos(tp * x) - 0.2 * tp * np.sin(tp * y) + tp * np.cos(tp * x) * np.cos(tp * z)


def _consistency_error(k, nc):
    m = curved.CurvedBoxMesh(k, nc, nc, nc, amp=0.06, periodic=(True, True, True))
    X = np.concatenate([m.node_xyz(c) for c in range(m.ncells)])
    U = np.asarray(_u(X[:, 0], X[:, 1], X[:, 2])).ravel()
    Au = (v3.divergence_matrix(m) @ U).reshape(m.ncells, -1)
    T = sipg.Tables(k)
    Z, Y, Xg = np.meshgrid(T.xq, T.xq, T.xq, indexing="ij")
    xi = np.stack([Xg.ravel(), Y.ravel(), Z.ravel()], axis=1)
    Phi = sipg._kron3(T.S, T.S, T.S)
    wq = sipg._kron3(T.wq, T.wq, T.wq)
    ref = np.empty_like(Au)
    for c in range(m.ncells):
        xq = m.map_at(c, xi)
        w = wq * np.abs(np.linalg.det(m.jac_at(c, xi)))
        ref[c] = -Phi.T @ (w * _div_u(xq[:, 0], xq[:, 1], xq[:, 2]))
    return np.linalg.norm(Au - ref) / np.linalg.norm(ref)


def test_divergence_consistency_with_the_continuous_operator():
    e2 = _consistency_error(3, 2)
    e4 = _consistency_error(3, 4)
    assert e4 < 0.2 * e2 and e4 < 0.02


def test_physical_gradient_of_the_coordinates_is_the_identity():
    """The iso-parametric space holds the coordinate functions exactly, so their
    physical gradients at every quadrature point are the unit vectors."""
    m = curved.CurvedBoxMesh(3, 2, 2, 2, amp=0.08, ly=1.3, y_tanh_gamma=1.1, periodic=(True, False, True))
    T = sipg.Tables(3)
    for c in (0, 5):
        grad, _, _ = v3._cell_geo(T, m, c)
        X = m.node_xyz(c)
        for a in range(3):
            for r in range(3):
                assert np.abs(grad[a] @ X[:, r] - (1.0 if a == r else 0.0)).max() < 1e-12


def test_divdiv_and_penalty_on_curved_cells():
    kw = dict(ly=2.0, y0=-1.0, periodic=(True, False, True), y_tanh_gamma=1.3)
    m = curved.CurvedBoxMesh(3, 2, 3, 2, amp=0.06, **kw)
    nb = m.n ** 3
    M, D = v3.cell_mass_divdiv(m, 3)
    # constant vector fields are divergence-free at every point
    const = np.concatenate([np.full(nb, 0.3), np.full(nb, -1.2), np.full(nb, 0.7)])
    assert np.abs(D @ const).max() < 1e-12 * np.abs(D).max()
    assert np.all(np.linalg.eigvalsh(D) > -1e-12 * np.abs(D).max())
    # u = (x, 0, 0): div u = 1 at every point, so v . D u = (div v, 1)_K and u . D u = V
    X = m.node_xyz(3)
    u = np.concatenate([X[:, 0], np.zeros(nb), np.zeros(nb)])
    w, V = v3._weights_volume(m, 3)
    assert abs(u @ D @ u - V) < 1e-12 * V
    assert abs(w.sum() - V) < 1e-14 * V and abs(np.ones(nb) @ M @ np.ones(nb) - V) < 1e-13 * V
    # penalty of a constant field: zeta |c| V^(1/3) dt with the curved volume
    N = m.ndofs
    U = np.concatenate([np.full(N, 0.3), np.full(N, -1.2), np.full(N, 0.7)])
    tau = v3.penalty_tau(m, U, 2.0, 1e-2)
    vols = np.array([v3._weights_volume(m, c)[1] for c in range(m.ncells)])
    assert np.abs(tau - 2.0 * np.linalg.norm([0.3, -1.2, 0.7]) * vols ** (1 / 3) * 1e-2).max() < 1e-14
    assert np.ptp(vols) > 1e-3 * vols.mean()          # graded cells: the volumes differ


def test_curved_penalty_and_projection_reduce_to_affine():
    kw = dict(lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, False), y_tanh_gamma=1.3)
    cm = curved.CurvedBoxMesh(2, 2, 3, 2, amp=0.0, **kw)
    am = omesh.BoxMesh(2, 2, 3, 2, **kw)
    U = inp.uniform(51, 3 * am.ndofs)
    ta, tc = v3.penalty_tau(am, U, 1.0, 0.1), v3.penalty_tau(cm, U, 1.0, 0.1)
    assert np.abs(ta - tc).max() < 1e-14 * np.abs(ta).max()
    rhs = inp.uniform(52, 3 * am.ndofs)
    xa, xc = v3.projection_solve(am, ta, rhs), v3.projection_solve(cm, ta, rhs)
    assert np.abs(xa - xc).max() < 1e-11 * np.abs(xa).max()


def test_row_restricted_operators_equal_the_assembled_rows():
    kw = dict(lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, True), y_tanh_gamma=1.3,
              neumann=(False, False, False, True, False, False))
    for m in (curved.CurvedBoxMesh(2, 3, 3, 2, amp=0.05, **kw), omesh.BoxMesh(2, 3, 3, 2, **kw)):
        nb = m.n ** 3
        u = inp.uniform(61, 3 * m.ndofs)
        p = inp.uniform(62, m.ndofs)
        cells = [0, 4, 8, 17]
        Au = (v3.divergence_matrix(m) @ u).reshape(m.ncells, nb)[cells]
        Bp = (v3.gradient_matrix(m) @ p).reshape(3, m.ncells, nb)[:, cells]
        assert np.abs(v3.divergence_cells(m, u, cells) - Au).max() < 1e-13 * np.abs(Au).max()
        assert np.abs(v3.gradient_cells(m, p, cells) - Bp).max() < 1e-13 * np.abs(Bp).max()
