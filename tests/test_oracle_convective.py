"""Pins of the oracle's convective operator, JVP and VJP."""
import math

import numpy as np
import pytest

from oracle import convective, mesh
import dgmf_inputs as inp


def _field(m, fn, seed=None, noise=0.0):
    X = m.node_coords()
    U = np.asarray(fn(X[:, 0], X[:, 1], X[:, 2]), dtype=np.float64)
    if seed is not None:
        U = U + noise * inp.uniform(seed, U.size).reshape(U.shape)
    return U.ravel()


@pytest.fixture(scope="module")
def per():
    m = mesh.BoxMesh(2, 2, 2, 3, lx=1.0, ly=1.0, lz=1.0)
    return m, convective.Convective(m)


def test_free_stream_is_zero(per):
    m, op = per
    U = np.concatenate([np.full(m.ndofs, 0.7), np.full(m.ndofs, -0.2), np.full(m.ndofs, 1.3)])
    assert np.abs(op.forward(U)).max() < 1e-13


def test_conservation_and_homogeneity(per):
    m, op = per
    U = _field(m, inp.taylor_green, seed=1, noise=0.3)
    C = op.forward(U).reshape(3, -1)
    scale = np.abs(C).max()
    assert np.abs(C.sum(axis=1)).max() < 1e-13 * scale * m.ndofs
    C2 = op.forward(2.5 * U).reshape(3, -1)
    assert np.abs(C2 - 2.5 ** 2 * C).max() < 1e-13 * np.abs(C2).max()


def test_lax_friedrichs_dissipation_identity(per):
    m, op = per
    U = _field(m, inp.taylor_green, seed=2, noise=0.5)
    lhs = U @ (op.forward(U) - op.forward(U, lam_on=False))
    # sum over faces of int lam |[u]|^2, evaluated face by face
    V = U.reshape(3, m.ncells, -1)
    rhs = 0.0
    for cL, cR, d in m.interior_faces():
        nrm, dA = op._face_geo(cL, d, 1)          # unit normals (3, m), one per face point
        um = (op.Tr[2 * d + 1] @ V[:, cL, :].T).T
        up = (op.Tr[2 * d] @ V[:, cR, :].T).T
        lam = np.maximum(np.abs(np.sum(nrm * um, axis=0)), np.abs(np.sum(nrm * up, axis=0)))
        rhs += np.sum(dA * lam * np.sum((um - up) ** 2, axis=0))
    assert rhs > 0
    assert abs(lhs - rhs) < 1e-12 * rhs


def test_quadrature_invariance_without_lf():
    k = 3
    m = mesh.BoxMesh(k, 2, 2, 2)
    U = _field(m, inp.taylor_green, seed=3, noise=0.2)
    nq_min = (3 * k) // 2 + 1
    a = convective.Convective(m, nq=nq_min).forward(U, lam_on=False)
    b = convective.Convective(m, nq=nq_min + 2).forward(U, lam_on=False)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()
    # with the LF term the rules differ (|u.n| is not a polynomial)
    a = convective.Convective(m, nq=nq_min).forward(U)
    b = convective.Convective(m, nq=nq_min + 2).forward(U)
    assert np.abs(a - b).max() > 1e-8 * np.abs(a).max()


@pytest.mark.parametrize("k", [2, 4])
def test_channel_profile_is_steady(k):
    m = mesh.BoxMesh(k, 2, 4, 2, lx=2 * math.pi, ly=2.0, lz=math.pi, y0=-1.0,
                     periodic=(True, False, True), y_tanh_gamma=1.8)
    op = convective.Convective(m)
    q = lambda y: 0.3 * (1 - y ** 2) * (y + 0.5) if k >= 3 else 0.3 * (1 - y ** 2)
    U = _field(m, lambda x, y, z: np.stack([1 - y ** 2, 0 * y, q(y)]))
    assert np.abs(op.forward(U)).max() < 1e-12


MIXED = lambda: mesh.BoxMesh(1, 2, 2, 2, lx=1.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(True, False, True),
                             y_tanh_gamma=1.5)


def _gwall(x, y, z):
    return np.stack([0.3 + 0 * x, 0.2 * np.sin(x), -0.1 + 0 * z])


@pytest.mark.parametrize("case", ["periodic", "dirichlet_g"])
def test_jvp_central_differences_and_vjp_transpose(case):
    if case == "periodic":
        m = mesh.BoxMesh(1, 2, 2, 2)
        op = convective.Convective(m, nq=3)
    else:
        m = MIXED()
        op = convective.Convective(m, nq=3, g=_gwall)
    U = _field(m, inp.taylor_green, seed=5, noise=0.3)
    Jm = op.jacobian(U)
    g = np.random.default_rng(6)
    eps = 1e-6
    for _ in range(5):
        d = g.uniform(-1, 1, U.size)
        fd = (op.forward(U + eps * d) - op.forward(U - eps * d)) / (2 * eps)
        jv = op.jvp(U, d)
        assert np.abs(fd - jv).max() < 1e-6 * np.abs(jv).max()
        np.testing.assert_allclose(Jm @ d, jv, atol=1e-13 * np.abs(jv).max())
    W = g.uniform(-1, 1, U.size)
    vj = op.vjp(U, W)
    assert np.abs(vj - Jm.T @ W).max() < 1e-12 * np.abs(vj).max()


def test_euler_identity_and_adjoint(per):
    m, op = per
    U = _field(m, inp.taylor_green, seed=7, noise=0.1)
    g = np.random.default_rng(8)
    W = g.uniform(-1, 1, U.size)
    d = g.uniform(-1, 1, U.size)
    vj = op.vjp(U, W)
    assert abs(vj @ U - 2 * (W @ op.forward(U))) < 1e-12 * abs(vj @ U)
    assert abs(W @ op.jvp(U, d) - vj @ d) < 1e-12 * abs(vj @ d)


def test_vjp_cells_matches_full(per):
    m, op = per
    U = _field(m, inp.taylor_green, seed=9, noise=0.1)
    W = np.random.default_rng(10).uniform(-1, 1, U.size)
    full = op.vjp(U, W).reshape(3, m.ncells, -1)
    cells = [0, 5, 11]
    np.testing.assert_allclose(op.vjp_cells(U, W, cells), full[:, cells], rtol=0, atol=1e-14 * np.abs(full).max())
    Cf = op.forward(U).reshape(3, m.ncells, -1)
    np.testing.assert_allclose(op.forward_cells(U, cells), Cf[:, cells], rtol=0, atol=1e-14 * np.abs(Cf).max())


def test_kink_aware_central_differences():
    """Central differences of <w, C(U)> with a step large enough to cross many LF kinks,
    minus the exact per-point correction at the points that may cross one
    (tests/fd_kinks.py), equal <VJP(U, w), d>; without the correction they do not."""
    import torch
    from tests.fd_kinks import kink_correction
    k, nc, nq = 2, (3, 3, 3), 4
    m = mesh.BoxMesh(k, *nc)
    op = convective.Convective(m, nq=nq)
    X = m.node_coords()
    U = (inp.taylor_green(X[:, 0], X[:, 1], X[:, 2]) + 0.01 * inp.uniform(31, 3 * m.ndofs).reshape(3, -1)).ravel()
    W = inp.uniform(32, U.size)
    g = op.vjp(U, W)
    eps = 2e-3
    worst_raw, worst = 0.0, 0.0
    for j in range(4):
        D = inp.uniform(40 + j, U.size)
        fd = W @ (op.forward(U + eps * D) - op.forward(U - eps * D)) / (2 * eps)
        corr, count = kink_correction(torch.as_tensor(U), torch.as_tensor(D), torch.as_tensor(W), k, nc, nq,
                                      1.0 / 3, eps)
        an = g @ D
        assert count > 0
        worst_raw = max(worst_raw, abs(fd - an) / abs(an))
        worst = max(worst, abs(fd - corr - an) / abs(an))
    assert worst_raw > 1e-6          # the kinks are crossed ...
    assert worst < 1e-11             # ... and the correction accounts for all of them
