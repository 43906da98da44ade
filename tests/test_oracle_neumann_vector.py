"""Pins of the oracle's V3c and viscous operators with Neumann sides.

The ND average is the own trace on both boundary parts (Sec. 3.1), so the
divergence and gradient operators do not distinguish Neumann from Dirichlet
sides.  The symmetric-gradient viscous operator has no term on a homogeneous
Neumann face (Sec. 3.2), so on a box whose sides are all Neumann every rigid
motion u = a + w x (x) (six modes, continuous, eps(u) = 0) lies in the null
space of its mu = 0 part, exactly; one Dirichlet side removes all of them.
"""
import numpy as np
import pytest

from oracle import mesh as omesh, v3 as ov3, viscous as ovisc

ALL_N = (True,) * 6


def test_divergence_and_gradient_treat_both_boundary_parts_alike():
    kw = dict(lx=1.0, ly=2.0, lz=1.5, y0=-1.0, periodic=(False, False, True), y_tanh_gamma=1.2)
    mn = omesh.BoxMesh(2, 2, 3, 2, neumann=(True, False, True, True, False, False), **kw)
    md = omesh.BoxMesh(2, 2, 3, 2, **kw)
    assert abs(ov3.divergence_matrix(mn) - ov3.divergence_matrix(md)).max() == 0.0
    assert abs(ov3.gradient_matrix(mn) - ov3.gradient_matrix(md)).max() == 0.0


def _rigid_modes(m):
    X = m.node_coords()
    modes = []
    for a in range(3):                        # translations
        U = np.zeros((3, m.ndofs))
        U[a] = 1.0
        modes.append(U.ravel())
    for w in np.eye(3):                       # rotations w x x
        U = np.cross(np.broadcast_to(w, X.shape), X).T
        modes.append(U.ravel())
    return modes


@pytest.mark.parametrize("k", [1, 2])
def test_rigid_motions_span_the_null_space_with_neumann_sides(k):
    m = omesh.BoxMesh(k, 2, 2, 2, lx=1.0, ly=0.8, lz=1.3, periodic=(False, False, False), neumann=ALL_N)
    A = ovisc.viscous_matrix(m, 0.0, 1.0, 1.0)
    scale = abs(A).max()
    for U in _rigid_modes(m):
        assert np.abs(A @ U).max() <= 1e-11 * scale * np.abs(U).max()
    assert abs(A - A.T).max() <= 1e-12 * scale
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() >= -1e-10 * ev.max() and np.sum(ev < 1e-9 * ev.max()) == 6
    # one Dirichlet side pins every rigid motion
    md = omesh.BoxMesh(k, 2, 2, 2, lx=1.0, ly=0.8, lz=1.3, periodic=(False, False, False),
                       neumann=(False,) + (True,) * 5)
    Ad = ovisc.viscous_matrix(md, 0.0, 1.0, 1.0)
    assert np.linalg.eigvalsh(Ad.toarray()).min() > 1e-9 * ev.max()
