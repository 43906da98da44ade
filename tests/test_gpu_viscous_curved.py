"""GPU parity of the symmetric-gradient viscous operator on iso-parametric curved cells.

The library applies the stored-metric scalar SIPG operator to every component
and adds the component coupling, with the Jacobian taken in closed form at
every point; the oracle (``oracle.viscous.CurvedViscous``) builds dense blocks
point by point from the full tensor interpolation of the node positions.
Small meshes compare the apply entry by entry with the oracle's assembled
3N x 3N matrix (periodic, Dirichlet and Neumann walls, tanh grading, degrees
1-6); the curved channel at full
size compares the rows of sampled cells with the oracle's row-restricted
apply.  The implicit viscous solve (Jacobi and inverse-mass PCG) is compared
with the oracle's iteration on its assembled matrix.  Node coordinates,
quadrature points and the load vector on curved cells are compared with the
oracle's map and its right-hand side, and a manufactured viscous problem
built through the library converges to the oracle's discrete solution.
"""
import math

import numpy as np
import pytest
import torch

import dgmf_inputs as inp
from oracle import curved, solvers, viscous as ovisc
from tests.gpu_util import dev, host, rel_err, require_gpu, sample_cells

pytestmark = pytest.mark.gpu

YW = (0, 0, 1, 1, 0, 0)
CASES = {
    # name: (k, cells, lengths, y0, periodic, gamma, neumann, amp, mu, nu)
    "k1_dirichlet_box": (1, (3, 2, 2), (1, 0.8, 1.2), 0.0, (0, 0, 0), 0.0, (0,) * 6, 0.08, 1.0, 1.0),
    "k2_periodic": (2, (3, 2, 2), (1, 1, 1), 0.0, (1, 1, 1), 0.0, (0,) * 6, 0.05, 0.0, 1.0),
    "k3_channel_dirichlet": (3, (2, 3, 2), (2 * math.pi, 2, math.pi), -1.0, (1, 0, 1), 1.5, (0,) * 6, 0.03,
                             100.0, 0.01),
    "k4_channel_neumann": (4, (2, 2, 2), (2 * math.pi, 2, math.pi), -1.0, (1, 0, 1), 1.2, YW, 0.04, 0.0, 1.0),
    "k5_periodic_xz": (5, (2, 1, 2), (1, 1, 1), 0.0, (1, 0, 1), 0.0, (0,) * 6, 0.06, 1.0, 0.5),
    "k6_mixed": (6, (2, 2, 1), (1, 1, 1), 0.0, (1, 1, 0), 0.0, (0, 0, 0, 0, 1, 0), 0.05, 0.0, 1.0),
}


def _pair(name, mu=None):
    import paper_1607_01323_amd as dg
    k, cells, L, y0, per, gam, neu, amp, mu0, nu = CASES[name]
    mu = mu0 if mu is None else mu
    om = curved.CurvedBoxMesh(k, *cells, lx=L[0], ly=L[1], lz=L[2], y0=y0, periodic=tuple(bool(p) for p in per),
                              y_tanh_gamma=gam, neumann=tuple(bool(f) for f in neu), amp=amp)
    gm = dg.Mesh(k, *cells, *L, y0=y0, periodic=per, y_tanh_gamma=gam, store_qp_metric=True, neumann=neu,
                 curve_amp=amp)
    return om, gm, dg.SipgOperator(gm, mu, nu, 1.0), mu, nu


@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_oracle_small(name):
    require_gpu()
    print(f"[case] curved viscous {name}", flush=True)
    om, gm, gop, mu, nu = _pair(name)
    A = ovisc.CurvedViscous(om, mu, nu, 1.0).assemble()
    U = inp.uniform(140, 3 * om.ndofs)
    err = rel_err(host(gop.viscous_apply(dev(U))), A @ U)
    print(f"  rel. err {err:.2e}", flush=True)
    assert err < 1e-12
    gm.close()


def test_rigid_motions_in_the_null_space():
    """All-Neumann curved box without mass: the interpolated rigid motions give zero."""
    require_gpu()
    import paper_1607_01323_amd as dg
    print("[case] curved viscous rigid motions", flush=True)
    om = curved.CurvedBoxMesh(3, 2, 2, 2, amp=0.05, periodic=(False,) * 3, neumann=(True,) * 6)
    gm = dg.Mesh(3, 2, 2, 2, periodic=(0, 0, 0), store_qp_metric=True, neumann=(1,) * 6, curve_amp=0.05)
    gop = dg.SipgOperator(gm, 0.0, 0.7, 1.0)
    X = host(gm.node_coords()).reshape(3, -1).T
    scale = np.abs(host(gop.viscous_apply(dev(inp.uniform(141, 3 * om.ndofs))))).max()
    for j in range(6):
        a, w = np.zeros(3), np.zeros(3)
        (a if j < 3 else w)[j % 3] = 1.0
        R = np.concatenate([a[i] + np.cross(w, X)[:, i] for i in range(3)])
        assert np.abs(host(gop.viscous_apply(dev(R)))).max() <= 1e-11 * scale * np.abs(R).max()
    gm.close()


def test_full_size_sampled_rows():
    """The curved channel (48 x 32 x 48 cells, k = 4): rows of sampled cells."""
    require_gpu()
    import paper_1607_01323_amd as dg
    w = inp.CHANNEL_CURVED_C4
    print(f"[case] curved viscous full-size {w.name}", flush=True)
    gm = dg.Mesh.from_workload(w)
    gop = dg.SipgOperator(gm, w.mass_coeff, w.diff_coeff, w.penalty_scale)
    U = inp.uniform(142, 3 * gm.ndofs)
    Y = host(gop.viscous_apply(dev(U))).reshape(3, gm.ncells, -1)
    om = curved.CurvedBoxMesh(w.degree, *w.cells, lx=w.lengths[0], ly=w.lengths[1], lz=w.lengths[2], y0=w.y0,
                              periodic=w.periodic, y_tanh_gamma=w.y_tanh_gamma, amp=w.curve_amp)
    cells = sample_cells(w.cells, 10, 7)
    ref = ovisc.CurvedViscous(om, w.mass_coeff, w.diff_coeff, w.penalty_scale, cells=cells).apply_cells(U, cells)
    err = rel_err(Y[:, cells], ref)
    print(f"  {len(cells)} cells, rel. err {err:.2e}", flush=True)
    assert err < 1e-12
    gm.close()


@pytest.mark.parametrize("name,precond", [("k2_periodic", "jacobi"), ("k3_channel_dirichlet", "jacobi"),
                                          ("k4_channel_neumann", "mass")])
def test_viscous_cg_matches_oracle(name, precond):
    """PCG to 1e-10 with the scalar operator's inverse diagonal (or the inverse mass
    matrix) on every component, against the same iteration on the oracle's matrix."""
    require_gpu()
    from oracle import curved as ocurved
    print(f"[case] curved viscous cg {name} {precond}", flush=True)
    om, gm, gop, mu, nu = _pair(name, mu=1.0 if CASES[name][8] == 0.0 else None)
    A = ovisc.CurvedViscous(om, mu, nu, 1.0).assemble()
    if precond == "jacobi":
        dinv = np.tile(1.0 / ocurved.CurvedSIPG(om, mu, nu, 1.0).assemble().diagonal(), 3)
        prec = lambda r: dinv * r
    else:
        M = ocurved.CurvedSIPG(om, 1.0, 0.0, 1.0).assemble()   # the curved mass matrix (mu = 1, nu = 0)
        import scipy.sparse.linalg as spla
        lu = spla.splu(M.tocsc())
        prec = lambda r: np.concatenate([lu.solve(r[c * om.ndofs:(c + 1) * om.ndofs]) for c in range(3)])
    b = inp.uniform(143, 3 * om.ndofs)
    x0 = inp.uniform(144, 3 * om.ndofs)
    _, itr, st, _ = solvers.pcg(lambda v: A @ v, b, x0.copy(), prec, 1e-10, 3000)
    assert st == solvers.OK
    xg = dev(x0)
    out = gop.viscous_cg(dev(b), xg, rtol=1e-10, max_iter=3000, check_every=4, precond=precond)
    print(f"  iterations: library {out.iterations}, oracle {itr}", flush=True)
    assert out.status == 0 and abs(out.iterations - itr) <= 1
    assert np.linalg.norm(b - A @ host(xg)) <= 2e-10 * np.linalg.norm(b)
    gm.close()


def test_coordinates_and_load_vector():
    """Node coordinates, quadrature points and (f, phi_i) on curved cells."""
    require_gpu()
    from oracle import basis
    print("[case] curved coordinates and load vector", flush=True)
    om, gm, gop, mu, nu = _pair("k3_channel_dirichlet")
    k, n = om.k, om.n
    X = host(gm.node_coords()).reshape(3, gm.ncells, n ** 3)
    ref = np.stack([om.node_xyz(c) for c in range(om.ncells)])            # (cells, n^3, 3)
    assert np.abs(X.transpose(1, 2, 0) - ref).max() <= 1e-13 * np.abs(ref).max()
    xg, _ = basis.gauss_rule(n)
    xi = np.array([(xg[qx], xg[qy], xg[qz]) for qz in range(n) for qy in range(n) for qx in range(n)])
    Q = host(gop.quadrature_points()).reshape(3, gm.ncells, n ** 3)
    refq = np.stack([om.map_at(c, xi) for c in range(om.ncells)])
    assert np.abs(Q.transpose(1, 2, 0) - refq).max() <= 1e-13 * np.abs(refq).max()
    f = lambda x, y, z: np.sin(x) * np.cos(0.7 * y) + z * z
    fq = f(*[Q[d].ravel() for d in range(3)])
    b = host(gop.integrate(dev(fq)))
    bref = curved.CurvedSIPG(om, mu, nu, 1.0).rhs(f)
    assert rel_err(b, bref) < 1e-12
    gm.close()


def test_manufactured_viscous_problem():
    """mu u - div(2 nu eps(u)) = f on a curved periodic box, right-hand side formed
    through the library's quadrature points and load vector; the library's solve
    equals the oracle's discrete solution and is close to the exact field."""
    require_gpu()
    import scipy.sparse.linalg as spla
    print("[case] curved viscous manufactured solution", flush=True)
    om, gm, gop, mu, nu = _pair("k2_periodic", mu=10.0)
    t = 2 * math.pi
    # u = (sin ty, sin tz, sin tx): divergence-free, eps(u) = grad u sym, div(2 eps u) = lap u
    ex = [lambda x, y, z: np.sin(t * y), lambda x, y, z: np.sin(t * z), lambda x, y, z: np.sin(t * x)]
    fs = [lambda x, y, z, g=g: (mu + nu * t * t) * g(x, y, z) for g in ex]
    Q = host(gop.quadrature_points())
    Qn = Q.reshape(3, -1)
    b = np.concatenate([host(gop.integrate(dev(fc(*Qn)))) for fc in fs])
    A = ovisc.CurvedViscous(om, mu, nu, 1.0).assemble()
    xs = spla.spsolve(A.tocsc(), b)
    xg = dev(np.zeros_like(b))
    out = gop.viscous_cg(dev(b), xg, rtol=1e-12, max_iter=5000, check_every=8)
    assert out.status == 0
    assert rel_err(host(xg), xs) < 1e-9
    X = host(gm.node_coords()).reshape(3, -1)
    exact = np.concatenate([g(*X) for g in ex])
    err = np.abs(host(xg) - exact).max()
    print(f"  max nodal error {err:.2e}", flush=True)
    assert err < 0.1
    gm.close()
