"""GPU parity of the SIPG operator with homogeneous Neumann sides.

Both apply kernels (the z-marching one on axis-aligned cells and the
stored-metric one) and their diagonals are compared entry by entry with the
oracle's assembled matrix on small meshes: every degree, all-Neumann
(singular) boxes, the channel pressure operator (Neumann walls in y, periodic
x and z, tanh grading), mixed Neumann/Dirichlet sides, a single cell, and a
long z direction split into several z segments.  CG (Jacobi, fp32 multigrid)
on singular Neumann problems is compared with the oracle's iteration counts
and true residual; at the full channel size the apply is checked on sampled
cells and the multigrid solve on the oracle's residual over all cells.
The convective (outflow sides), V3c and viscous operators on Neumann meshes
are checked in their own test files.
"""
import math

import numpy as np
import pytest
import torch

import dgmf_inputs as inp
from oracle import mesh as omesh, multigrid as omg, sipg as osipg, solvers
from tests.gpu_util import dev, host, rel_err, require_gpu, sample_cells

pytestmark = pytest.mark.gpu

ALL = (1, 1, 1, 1, 1, 1)
YWALLS = (0, 0, 1, 1, 0, 0)
CASES = {
    # name: (k, cells, lengths, y0, periodic, gamma, neumann, mu, nu)
    "k2_all_neumann": (2, (3, 2, 2), (1, 1, 1), 0.0, (0, 0, 0), 0.0, ALL, 0.0, 1.0),
    "k3_channel_pressure": (3, (3, 4, 2), (2 * math.pi, 2, math.pi), -1.0, (1, 0, 1), 1.5, YWALLS, 0.0, 1.0),
    "k4_mixed_sides": (4, (2, 3, 3), (1, 0.7, 1.3), 0.0, (0, 0, 0), 0.0, (1, 0, 0, 1, 1, 0), 1.0, 0.5),
    "k1_one_cell": (1, (1, 1, 1), (1, 1, 1), 0.0, (0, 0, 0), 0.0, ALL, 0.0, 1.0),
    "k5_outflow_x": (5, (3, 2, 2), (2, 1, 1), 0.0, (0, 1, 1), 0.0, (0, 1, 0, 0, 0, 0), 100.0, 0.01),
    "k6_neumann_z": (6, (2, 2, 2), (1, 1, 1), 0.0, (1, 1, 0), 0.0, (0, 0, 0, 0, 1, 1), 0.0, 1.0),
    "k7_channel": (7, (2, 2, 2), (1, 2, 1), -1.0, (1, 0, 1), 1.2, YWALLS, 0.0, 1.0),
    # several z segments and ragged x-y tiles of the z-marching kernel
    "k3_long_z": (3, (6, 5, 30), (1, 1, 1), 0.0, (0, 0, 0), 0.0, (0, 1, 0, 0, 1, 1), 1.0, 1.0),
}


def _singular(name):
    """No Dirichlet face and no mass term: constants span the null space."""
    k, cells, L, y0, per, gam, neu, mu, nu = CASES[name]
    return mu == 0.0 and all(per[d] or (neu[2 * d] and neu[2 * d + 1]) for d in range(3))


def _pair(name, metric, penalty=1.0):
    import paper_1607_01323_amd as dg
    k, cells, L, y0, per, gam, neu, mu, nu = CASES[name]
    om = omesh.BoxMesh(k, *cells, lx=L[0], ly=L[1], lz=L[2], y0=y0, periodic=tuple(bool(p) for p in per),
                       y_tanh_gamma=gam, neumann=tuple(bool(f) for f in neu))
    oop = osipg.SIPG(om, mu, nu, penalty)
    gm = dg.Mesh(k, *cells, *L, y0=y0, periodic=per, y_tanh_gamma=gam, store_qp_metric=metric, neumann=neu)
    gop = dg.SipgOperator(gm, mu, nu, penalty)
    return om, oop, gm, gop


@pytest.mark.parametrize("metric", [False, True])
@pytest.mark.parametrize("name", list(CASES))
def test_apply_and_diagonal_match_assembled_matrix(name, metric):
    require_gpu()
    print(f"[case] neumann apply {name} metric={metric}", flush=True)
    om, oop, gm, gop = _pair(name, metric)
    A = oop.assemble()
    u = inp.uniform(110, om.ndofs)
    ref = A @ u
    assert rel_err(host(gop.apply(dev(u))), ref) < 1e-12
    assert rel_err(host(gop.apply(dev(u, torch.float32))), ref) < 1e-5
    assert rel_err(host(gop.diagonal()), A.diagonal()) < 1e-13
    assert rel_err(host(gop.diagonal(torch.float32)), A.diagonal()) < 1e-6
    if _singular(name):
        one = host(gop.apply(dev(np.ones(om.ndofs))))
        assert np.abs(one).max() <= 1e-11 * np.abs(ref).max()
    gm.close()


def test_jacobi_cg_on_singular_neumann_problem():
    require_gpu()
    print("[case] neumann jacobi cg k2_all_neumann", flush=True)
    om, oop, gm, gop = _pair("k2_all_neumann", False)
    A = oop.assemble()
    b = inp.uniform(7, om.ndofs)
    dinv = 1.0 / A.diagonal()
    xr, itr, st, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(om.ndofs), lambda r: dinv * r, 1e-10, 500,
                                 project_mean=True)
    assert st == solvers.OK
    xg = dev(np.zeros(om.ndofs))
    out = gop.cg(dev(b), xg, rtol=1e-10, max_iter=500, project_mean=True)
    assert out.status == 0 and abs(out.iterations - itr) <= 1
    bp = b - b.mean()
    r = bp - A @ host(xg)
    r -= r.mean()
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(bp)
    gm.close()


@pytest.mark.parametrize("name, metric", [("k3_channel_pressure", False), ("k3_channel_pressure", True),
                                          ("k4_mixed_sides", False)])
def test_multigrid_pcg_matches_oracle(name, metric):
    require_gpu()
    print(f"[case] neumann multigrid {name} metric={metric}", flush=True)
    om, oop, gm, gop = _pair(name, metric)
    singular = _singular(name)
    mg = omg.Multigrid(om, CASES[name][7], CASES[name][8], 1.0, seed=42, singular=singular)
    A = mg.A[0]
    b = inp.uniform(8, om.ndofs)
    _, itr, st, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(om.ndofs), mg.vcycle, 1e-10, 200,
                                project_mean=singular, flexible=True)
    assert st == solvers.OK
    xg = dev(np.zeros(om.ndofs))
    out = gop.cg(dev(b), xg, rtol=1e-10, max_iter=200, precond="multigrid", precond_dtype=torch.float32, seed=42,
                 project_mean=singular)
    assert out.status == 0
    print(f"  iterations: library {out.iterations}, oracle {itr}", flush=True)
    assert abs(out.iterations - itr) <= 2
    bp = b - b.mean() if singular else b
    r = bp - A @ host(xg)
    if singular:
        r -= r.mean()
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(bp)
    gm.close()


def test_full_size_channel_pressure():
    """Channel pressure Poisson (48x32x48, k = 4, stored metric, Neumann walls):
    sampled cells of the apply, then fp32-multigrid PCG to 1e-10 on the oracle's
    residual over every cell."""
    require_gpu()
    import paper_1607_01323_amd as dg
    w = inp.CHANNEL_PRESSURE_C4
    print(f"[case] neumann full-size {w.name}", flush=True)
    om = omesh.BoxMesh(w.degree, *w.cells, lx=w.lengths[0], ly=w.lengths[1], lz=w.lengths[2], y0=w.y0,
                       periodic=w.periodic, y_tanh_gamma=w.y_tanh_gamma, neumann=w.neumann)
    oop = osipg.SIPG(om, w.mass_coeff, w.diff_coeff, w.penalty_scale)
    gm = dg.Mesh.from_workload(w)
    gop = dg.SipgOperator(gm, w.mass_coeff, w.diff_coeff, w.penalty_scale)
    u = inp.uniform(9, om.ndofs)
    y = host(gop.apply(dev(u))).reshape(om.ncells, -1)
    cells = sample_cells(w.cells, 24, 11)
    assert rel_err(y[cells], oop.apply_cells(u, cells)) < 1e-12
    b = inp.uniform(10, om.ndofs)
    b -= b.mean()
    xg = torch.zeros(om.ndofs, dtype=torch.float64, device="cuda")
    out = gop.cg(dev(b), xg, rtol=1e-10, max_iter=200, precond="multigrid", precond_dtype=torch.float32, seed=42,
                 project_mean=True)
    assert out.status == 0
    print(f"[result] channel pressure MG iterations {out.iterations}, solve {out.solve_s:.3f} s", flush=True)
    r = b - oop.apply_cells(host(xg), list(range(om.ncells))).ravel()
    r -= r.mean()
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(b)
    # 41 on the box: the near-wall cells of the tanh grading (aspect ratio ~ 18)
    # weaken the point-Jacobi Chebyshev smoother; a loose ceiling guards against
    # a preconditioner that stopped working
    assert out.iterations <= 80
    gm.close()
