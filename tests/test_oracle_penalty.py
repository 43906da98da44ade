"""Pin of the oracle's interior-penalty terms (eqs. taue, tau, ipflux).

The SIPG matrix is affine in the penalty scale s: A(s) = C + s P, where P
holds only the penalty face terms.  So A(1) - A(0) = P, and every block of P
is a penalty value times a face mass, which this test computes on its own:

* tau_e = (k+1)^2 (A_int/2 + A_bnd)/V from the cell's box sizes (eq. taue);
* an interior face carries max(tau_e^-, tau_e^+) (eq. tau), so the block of
  P coupling the two cells is -max(...) (phi_i^-, phi_j^+)_F;
* a Dirichlet face carries 2 tau_e (the boundary flux of eq. ipflux), so the
  diagonal block of a wall cell is 2 tau_e (phi_i, phi_j)_wall plus the
  interior-face masses of its other faces with their own penalties.

The face masses use a Gauss rule of k+2 points and a Lagrange basis written
out in this file.  The mesh has three graded y-layers between Dirichlet walls,
so the wall layer and the middle layer have different tau_e (different h_y,
and only the wall layer counts a boundary face): replacing the max by a mean,
or the boundary factor 2 by 1, changes P and fails the test.
"""
import numpy as np
import pytest

from oracle import basis, mesh, sipg


def _lagrange(nodes, x):
    L = np.ones((len(x), len(nodes)))
    for j, xj in enumerate(nodes):
        for m, xm in enumerate(nodes):
            if m != j:
                L[:, j] *= (x - xm) / (xj - xm)
    return L


def _face_mass(k, h_t1, h_t2, side_a, side_b, d):
    """(phi_i^a, phi_j^b) over a face normal to d of tangential sizes h_t1, h_t2.

    side_a, side_b: which end (0 or 1) of the reference interval along d the
    face is for the cell of the row (a) and of the column (b).
    """
    n = k + 1
    x, w = np.polynomial.legendre.leggauss(k + 2)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    nodes = basis.gll_nodes(k)
    L = _lagrange(nodes, x)                       # tangential values at the points
    end = _lagrange(nodes, np.array([0.0, 1.0]))  # values at the two ends along d
    # trace of phi_(l,j,i) on the face: the factor along d is the end value,
    # the other two factors are tangential values at the points
    def trace(side):
        mats = [L, L, L]
        mats[d] = end[side:side + 1]
        return np.kron(mats[2], np.kron(mats[1], mats[0]))   # (points, n^3)
    wt = [w, w, w]
    wt[d] = np.ones(1)
    W = np.kron(wt[2], np.kron(wt[1], wt[0])) * h_t1 * h_t2
    Ta, Tb = trace(side_a), trace(side_b)
    return Ta.T @ (W[:, None] * Tb)


def _tau_e(k, h, wall_faces):
    """eq. taue for a box cell with sizes h and the given number of wall faces (per direction)."""
    areas = [h[1] * h[2], h[0] * h[2], h[0] * h[1]]
    a = 0.0
    for d in range(3):
        a += wall_faces[d] * areas[d] + 0.5 * (2 - wall_faces[d]) * areas[d]
    return (k + 1) ** 2 * a / (h[0] * h[1] * h[2])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_penalty_blocks(k):
    def build(s):
        m = mesh.BoxMesh(k, 2, 3, 2, lx=1.2, ly=2.0, lz=0.9, y0=-1.0,
                         periodic=(True, False, True), y_tanh_gamma=1.6)
        return m, sipg.SIPG(m, penalty_scale=s).assemble().toarray()

    m, A1 = build(1.0)
    _, A0 = build(0.0)
    P = A1 - A0
    nb = m.n ** 3
    hy = np.diff(m.verts[1])
    assert abs(hy[0] - hy[1]) > 0.1 * hy[0]          # graded: the layers differ
    hx, hz = 1.2 / 2, 0.9 / 2
    h_wall = (hx, hy[0], hz)
    h_mid = (hx, hy[1], hz)
    tau_wall = _tau_e(k, h_wall, (0, 1, 0))
    tau_mid = _tau_e(k, h_mid, (0, 0, 0))
    assert abs(tau_wall - tau_mid) > 0.05 * tau_mid

    # interior y-face between the wall cell (cx, cy, cz) = (0, 0, 0) and (0, 1, 0)
    cL, cR = m.cell_index(0, 0, 0), m.cell_index(0, 1, 0)
    tauF = max(tau_wall, tau_mid)
    want = -tauF * _face_mass(k, hx, hz, 1, 0, 1)
    got = P[cL * nb:(cL + 1) * nb, cR * nb:(cR + 1) * nb]
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-12 * scale

    # diagonal block of the wall cell: wall face (2 tau_e), its interior
    # y-face (tauF), and four periodic faces in x and z within its layer
    want = 2.0 * tau_wall * _face_mass(k, hx, hz, 0, 0, 1)
    want += tauF * _face_mass(k, hx, hz, 1, 1, 1)
    for s in (0, 1):
        want += tau_wall * _face_mass(k, hy[0], hz, s, s, 0)
        want += tau_wall * _face_mass(k, hx, hy[0], s, s, 2)
    got = P[cL * nb:(cL + 1) * nb, cL * nb:(cL + 1) * nb]
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()

    # middle cell: both y-faces are interior faces with the wall layers
    cM = cR
    want = tauF * (_face_mass(k, hx, hz, 0, 0, 1) + _face_mass(k, hx, hz, 1, 1, 1))
    for s in (0, 1):
        want += tau_mid * _face_mass(k, hy[1], hz, s, s, 0)
        want += tau_mid * _face_mass(k, hx, hy[1], s, s, 2)
    got = P[cM * nb:(cM + 1) * nb, cM * nb:(cM + 1) * nb]
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_penalty_rhs_factor():
    """The Dirichlet data term of the right-hand side carries the same 2 tau_e (eq. ipflux):
    with g = 1 and f = 0, b(s=1) - b(s=0) = 2 tau_e nu (phi_i, 1)_wall on the wall cell."""
    k = 2
    def build(s):
        m = mesh.BoxMesh(k, 2, 3, 2, lx=1.2, ly=2.0, lz=0.9, y0=-1.0,
                         periodic=(True, False, True), y_tanh_gamma=1.6)
        op = sipg.SIPG(m, mass_coeff=0.0, diff_coeff=0.7, penalty_scale=s)
        zero = lambda x, y, z: 0.0 * x
        one = lambda x, y, z: 1.0 + 0.0 * x
        return m, op.rhs(zero, one)
    m, b1 = build(1.0)
    _, b0 = build(0.0)
    nb = m.n ** 3
    hy = np.diff(m.verts[1])
    hx, hz = 0.6, 0.45
    tau_wall = _tau_e(k, (hx, hy[0], hz), (0, 1, 0))
    c = m.cell_index(1, 0, 1)
    want = 2.0 * tau_wall * 0.7 * _face_mass(k, hx, hz, 0, 0, 1).sum(axis=1)
    got = (b1 - b0)[c * nb:(c + 1) * nb]
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
