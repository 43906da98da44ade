"""Pins of the oracle's convective operator with outflow (Neumann) sides.

Sec. 3.2, explicit convective step: on the Neumann part the flux is F^c(u_h).n
of the cell's own trace.  Fixed by facts outside the oracle: a constant field
on a domain whose only boundaries are outflow sides gives C = 0 (integration
by parts per cell, single-valued fluxes); the sum of C over all test functions
is the net momentum flux through the outflow sides, computed in closed form
for a linear field; the JVP matches central differences of the forward
operator, the VJP the transposed Jacobian, and the VJP satisfies the Euler
identity of a degree-2 homogeneous operator.
"""
import numpy as np

from oracle import convective, mesh
import dgmf_inputs as inp

OUT_X = (True, True, False, False, False, False)


def test_constant_field_is_steady_with_outflow_sides():
    m = mesh.BoxMesh(2, 3, 2, 2, periodic=(False, True, True), neumann=OUT_X)
    op = convective.Convective(m)
    U = np.concatenate([np.full(m.ndofs, 0.7), np.full(m.ndofs, -0.2), np.full(m.ndofs, 0.4)])
    assert np.abs(op.forward(U)).max() < 1e-13
    # the same field against no-slip walls is not steady
    md = mesh.BoxMesh(2, 3, 2, 2, periodic=(False, True, True))
    assert np.abs(convective.Convective(md).forward(U)).max() > 1e-2


def test_net_momentum_flux_through_outflow_sides():
    """U = (1 + x/2, 0.3, 0.2 y): sum_i C_{i,a} = int_{x=1} u_a u_x - int_{x=0} u_a u_x."""
    m = mesh.BoxMesh(1, 2, 2, 2, periodic=(False, True, True), neumann=OUT_X)
    op = convective.Convective(m)
    X = m.node_coords()
    U = np.concatenate([1 + 0.5 * X[:, 0], np.full(m.ndofs, 0.3), 0.2 * X[:, 1]])
    S = op.forward(U).reshape(3, -1).sum(axis=1)
    expect = np.array([1.5 * 1.5 - 1.0, 0.3 * 1.5 - 0.3, 0.2 * 0.5 * (1.5 - 1.0)])
    assert np.abs(S - expect).max() < 1e-13


def _gwall(x, y, z):
    return np.stack([0.3 + 0 * x, 0.2 * np.sin(x), -0.1 + 0 * z])


def test_jvp_vjp_with_outflow_and_dirichlet_sides():
    # x-: Dirichlet inflow with data g, x+: outflow; z-: outflow, z+: Dirichlet; y periodic
    m = mesh.BoxMesh(1, 2, 2, 2, periodic=(False, True, False),
                     neumann=(False, True, False, False, True, False))
    op = convective.Convective(m, nq=3, g=_gwall)
    X = m.node_coords()
    U = np.asarray(inp.taylor_green(X[:, 0], X[:, 1], X[:, 2])).ravel() + 0.3 * inp.uniform(5, 3 * m.ndofs)
    Jm = op.jacobian(U)
    g = np.random.default_rng(6)
    eps = 1e-6
    for _ in range(5):
        d = g.uniform(-1, 1, U.size)
        fd = (op.forward(U + eps * d) - op.forward(U - eps * d)) / (2 * eps)
        jv = op.jvp(U, d)
        assert np.abs(fd - jv).max() < 1e-6 * np.abs(jv).max()
    W = g.uniform(-1, 1, U.size)
    vj = op.vjp(U, W)
    assert np.abs(vj - Jm.T @ W).max() < 1e-12 * np.abs(vj).max()


def test_euler_identity_with_outflow_sides():
    m = mesh.BoxMesh(2, 2, 3, 2, periodic=(False, True, True), neumann=OUT_X)
    op = convective.Convective(m)
    X = m.node_coords()
    U = np.asarray(inp.taylor_green(X[:, 0], X[:, 1], X[:, 2])).ravel() + 0.1 * inp.uniform(7, 3 * m.ndofs)
    W = np.random.default_rng(8).uniform(-1, 1, U.size)
    vj = op.vjp(U, W)
    assert abs(vj @ U - 2 * (W @ op.forward(U))) < 1e-12 * abs(vj @ U)
