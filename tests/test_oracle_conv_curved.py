"""Pins of the oracle's convective operator on iso-parametric curved cells.

Sec. 5: curved cells take the Jacobian of the iso-parametric map at every
quadrature point; the operator is the one of Sec. 3.2 (eq. convstepspat).
Fixed by facts outside the oracle:
  - zero amplitude gives the affine operator (pinned separately);
  - free-stream preservation: with n_q = floor(3(k+1)/2) points the cell and
    face integrands of a constant flux are polynomials of degree <= 3k per
    reference direction (the cofactors of J have degree <= 2k), so both are
    integrated exactly and the divergence theorem on each curved cell gives
    C(const) = 0 to rounding; a wrong cofactor, a transposed inverse or a
    normal of the wrong size breaks this;
  - conservation on a periodic curved mesh (single-valued fluxes);
  - consistency with the continuous operator: for a smooth field, C tends to
    (phi_i, div(u (x) u)) with the physical derivatives, at a rate that rises
    with the degree;
  - JVP against central differences, VJP against the brute-force Jacobian,
    the Euler identity of a degree-2 homogeneous operator.
"""
import numpy as np

from oracle import convective, curved, mesh as omesh
import dgmf_inputs as inp


def _nodal(m, fun):
    X = np.concatenate([m.node_xyz(c) for c in range(m.ncells)])
    return np.asarray(fun(X[:, 0], X[:, 1], X[:, 2])).ravel()


def test_zero_amplitude_is_the_affine_operator():
    kw = dict(lx=2.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, False), y_tanh_gamma=1.3,
              neumann=(False, False, False, False, True, False))
    cm = curved.CurvedBoxMesh(2, 2, 3, 2, amp=0.0, **kw)
    am = omesh.BoxMesh(2, 2, 3, 2, **kw)
    U = inp.uniform(3, 3 * am.ndofs)
    W = inp.uniform(4, 3 * am.ndofs)
    A = convective.Convective(am)
    C = convective.Convective(cm)
    assert np.abs(C.forward(U) - A.forward(U)).max() <= 1e-13 * np.abs(A.forward(U)).max()
    assert np.abs(C.vjp(U, W) - A.vjp(U, W)).max() <= 1e-13 * np.abs(A.vjp(U, W)).max()


def test_free_stream_is_preserved_on_curved_cells():
    const = (0.7, -0.4, 0.25)
    m = curved.CurvedBoxMesh(3, 2, 3, 2, amp=0.08, periodic=(True, True, True))
    U = np.concatenate([np.full(m.ndofs, v) for v in const])
    out = convective.Convective(m).forward(U)
    assert np.abs(out).max() < 1e-13
    # walls with the same constant as Dirichlet data, an outflow side, tanh grading
    mw = curved.CurvedBoxMesh(2, 2, 3, 2, amp=0.06, ly=2.0, y0=-1.0, y_tanh_gamma=1.2,
                              periodic=(True, False, False), neumann=(False, False, False, False, True, False))
    g = lambda x, y, z: np.stack([np.full_like(x, v) for v in const])
    U = np.concatenate([np.full(mw.ndofs, v) for v in const])
    assert np.abs(convective.Convective(mw, g=g).forward(U)).max() < 1e-13
    # no-slip walls (g = 0) on the same mesh do not keep the constant
    assert np.abs(convective.Convective(mw).forward(U)).max() > 1e-2


def test_conservation_on_a_periodic_curved_mesh():
    m = curved.CurvedBoxMesh(2, 3, 2, 2, amp=0.07, periodic=(True, True, True))
    U = inp.uniform(11, 3 * m.ndofs)
    S = convective.Convective(m).forward(U).reshape(3, -1).sum(axis=1)
    assert np.abs(S).max() < 1e-13


def _u(x, y, z):
    tp = 2 * np.pi
    return np.stack([np.sin(tp * y) * np.cos(tp * z) + 0.5,
                     np.sin(tp * z) + 0.2 * np.cos(tp * x),
                     np.cos(tp * x) * np.sin(tp * y)])


def _div_uu(x, y, z):
    """sum_b d_b (u_a u_b) by central differences of the closed form (error ~1e-9)."""
    e = 1e-5
    out = 0.0
    for b in range(3):
        p = [x, y, z]
        q = [x, y, z]
        p[b] = p[b] + e
        q[b] = q[b] - e
        up, uq = _u(*p), _u(*q)
        out = out + (up * up[b] - uq * uq[b]) / (2 * e)
    return out


def _consistency_error(k, nc, amp):
    m = curved.CurvedBoxMesh(k, nc, nc, nc, amp=amp, periodic=(True, True, True))
    op = convective.Convective(m)
    U = _nodal(m, _u)
    C = op.forward(U).reshape(3, m.ncells, -1)
    # (phi_i, f) by the same cell quadrature, f at the physical points
    Z, Y, X = np.meshgrid(op.xq, op.xq, op.xq, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    B = np.zeros_like(C)
    for c in range(m.ncells):
        xq = m.map_at(c, xi)
        wq = op.wcell * np.abs(np.linalg.det(m.jac_at(c, xi)))
        f = _div_uu(xq[:, 0], xq[:, 1], xq[:, 2])
        B[:, c] = (op.Phi.T @ (wq[:, None] * f.T)).T
    return np.linalg.norm(C - B) / np.linalg.norm(B)


def test_consistency_with_the_continuous_operator():
    # order k in this weak residual: a factor 2^3 per halving of h at k = 3 (affine cells: 0.121)
    e2 = _consistency_error(3, 2, 0.06)
    e4 = _consistency_error(3, 4, 0.06)
    assert e4 < 0.16 * e2 and e4 < 0.02
    # the curvature is really felt: the affine operator on the deformed nodes is far off
    m = curved.CurvedBoxMesh(3, 4, 4, 4, amp=0.06, periodic=(True, True, True))
    am = omesh.BoxMesh(3, 4, 4, 4, periodic=(True, True, True))
    U = _nodal(m, _u)
    d = convective.Convective(am).forward(U) - convective.Convective(m).forward(U)
    assert np.linalg.norm(d) > 5 * e4 * np.linalg.norm(convective.Convective(m).forward(U))


def test_jvp_vjp_and_euler_identity_on_curved_cells():
    # x-: Dirichlet with data g, x+: outflow; y periodic; z-: outflow, z+: Dirichlet
    m = curved.CurvedBoxMesh(1, 2, 2, 2, amp=0.07, periodic=(False, True, False),
                             neumann=(False, True, False, False, True, False))
    g = lambda x, y, z: np.stack([0.3 + 0 * x, 0.2 * np.sin(x), -0.1 + 0 * z])
    op = convective.Convective(m, nq=3, g=g)
    U = _nodal(m, _u) + 0.3 * inp.uniform(5, 3 * m.ndofs)
    Jm = op.jacobian(U)
    rng = np.random.default_rng(6)
    eps = 1e-6
    for _ in range(4):
        d = rng.uniform(-1, 1, U.size)
        fd = (op.forward(U + eps * d) - op.forward(U - eps * d)) / (2 * eps)
        jv = op.jvp(U, d)
        assert np.abs(fd - jv).max() < 1e-6 * np.abs(jv).max()
    W = rng.uniform(-1, 1, U.size)
    vj = op.vjp(U, W)
    assert np.abs(vj - Jm.T @ W).max() < 1e-12 * np.abs(vj).max()
    # Euler identity with g = 0 (degree-2 homogeneous)
    op0 = convective.Convective(m, nq=3)
    vj0 = op0.vjp(U, W)
    assert abs(vj0 @ U - 2 * (W @ op0.forward(U))) < 1e-12 * abs(vj0 @ U)
