"""GPU parity of the geometric multigrid V-cycle preconditioner and MG-PCG.

The oracle builds its own hierarchy, eigenvalue estimates and coarse solver
(oracle.multigrid, same readings and the same SplitMix64 start vectors); the
GPU's estimates are compared with the oracle's, never fed into it.  Bars: one
V-cycle in fp64 within 1e-9 of the oracle's (fp32: 1e-4), lambdas within 1e-9
(fp32: 1e-4) and the same coarse Chebyshev degree; MG-PCG iteration counts
within 1 of the oracle's (fp32 preconditioner: 2) and a true residual below
2e-10; at full size, the true residual and the distance to the exact discrete
solution (fast diagonalisation) on the periodic Poisson cube, and the
oracle's residual over all cells on the channel mesh.
"""
import math

import numpy as np
import pytest
import torch

import dgmf_inputs as inp
from oracle import kron, mesh as omesh, multigrid as omg, sipg as osipg, solvers
from tests.gpu_util import dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu

CASES = {
    # name: (k, cells, lengths, y0, periodic, gamma, mu, nu, penalty)
    "k2_periodic_poisson": (2, (4, 4, 4), (1, 1, 1), 0.0, (1, 1, 1), 0.0, 0.0, 1.0, 1.0 / 3.0),
    "k3_aniso_coarsening": (3, (4, 2, 6), (1, 0.5, 1.5), 0.0, (1, 1, 1), 0.0, 0.0, 1.0, 1.0 / 3.0),
    "k1_dirichlet_helmholtz": (1, (8, 4, 4), (1, 1, 1), 0.0, (0, 0, 0), 0.0, 10.0, 1.0, 1.0),
    "k2_channel_helmholtz": (2, (4, 6, 4), (2 * math.pi, 2.0, math.pi), -1.0, (1, 0, 1), 1.5, 100.0, 0.01, 1.0),
    "k4_periodic_helmholtz": (4, (2, 2, 2), (1, 1, 1), 0.0, (1, 1, 1), 0.0, 1000.0, 0.01, 1.0),
}


def _setup(k, cells, L, y0, per, gam, mu, nu, pen):
    import paper_1607_01323_amd as dg
    om = omesh.BoxMesh(k, *cells, lx=L[0], ly=L[1], lz=L[2], y0=y0, periodic=tuple(bool(p) for p in per),
                       y_tanh_gamma=gam)
    gm = dg.Mesh(k, *cells, *L, y0=y0, periodic=per, y_tanh_gamma=gam)
    gop = dg.SipgOperator(gm, mu, nu, pen)
    singular = all(per) and mu == 0.0
    return om, gm, gop, singular


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("pdtype", [torch.float64, torch.float32])
def test_vcycle_matches_oracle(name, pdtype):
    require_gpu()
    print(f"[case] multigrid vcycle {name} {pdtype}", flush=True)
    c = CASES[name]
    om, gm, gop, singular = _setup(*c)
    mg = omg.Multigrid(om, c[6], c[7], c[8], seed=42, singular=singular)
    r = inp.uniform(17, om.ndofs)
    z = host(gop.precond_apply(dev(r), precond_dtype=pdtype, seed=42, project_mean=singular))
    levels, lams, m, iv = gop.precond_info()
    assert levels == mg.levels and m == mg.coarse_m
    tol_lam = 1e-9 if pdtype == torch.float64 else 1e-4
    for l in range(levels - 1):
        assert abs(lams[l] - mg.lam[l]) <= tol_lam * mg.lam[l]
    assert abs(iv[0] - mg.coarse_interval[0]) <= tol_lam * mg.coarse_interval[0] * 10
    assert abs(iv[1] - mg.coarse_interval[1]) <= tol_lam * mg.coarse_interval[1]
    zr = mg.vcycle(r)
    assert rel_err(z, zr) < (1e-9 if pdtype == torch.float64 else 1e-4)
    # a second application reuses the cached hierarchy and is deterministic
    z2 = host(gop.precond_apply(dev(r), precond_dtype=pdtype, seed=42, project_mean=singular))
    assert np.array_equal(z, z2)
    gm.close()


@pytest.mark.parametrize("name", ["k2_periodic_poisson", "k2_channel_helmholtz", "k3_aniso_coarsening"])
@pytest.mark.parametrize("pdtype", [torch.float64, torch.float32])
def test_mg_pcg_matches_oracle(name, pdtype):
    require_gpu()
    print(f"[case] multigrid pcg {name} {pdtype}", flush=True)
    c = CASES[name]
    om, gm, gop, singular = _setup(*c)
    mg = omg.Multigrid(om, c[6], c[7], c[8], seed=42, singular=singular)
    A = mg.A[0]
    b = inp.uniform(5, om.ndofs)
    flex = pdtype == torch.float32
    _, itr, st, _ = solvers.pcg(lambda v: A @ v, b, np.zeros(om.ndofs), mg.vcycle, 1e-10, 200,
                                project_mean=singular, flexible=flex)
    assert st == solvers.OK
    xg = dev(np.zeros(om.ndofs))
    out = gop.cg(dev(b), xg, rtol=1e-10, max_iter=200, check_every=4, precond="multigrid", precond_dtype=pdtype,
                 seed=42, project_mean=singular)
    assert out.status == 0
    assert abs(out.iterations - itr) <= (1 if pdtype == torch.float64 else 2)
    xs = host(xg)
    bp = b - b.mean() if singular else b
    r = bp - A @ xs
    if singular:
        r -= r.mean()
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(bp)
    gm.close()


def test_mg_rejects_sheared_meshes_and_bad_parameters():
    require_gpu()
    import paper_1607_01323_amd as dg
    sh = ((1.0, 0.2, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))
    gm = dg.Mesh(2, 2, 2, 2, store_qp_metric=True, shear=sh)
    gop = dg.SipgOperator(gm, 0.0, 1.0, 1.0)
    r = torch.zeros(gm.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.DgmfError, match="UNSUPPORTED"):
        gop.precond_apply(r)
    gm.close()
    gm = dg.Mesh(2, 2, 2, 2)
    gop = dg.SipgOperator(gm, 0.0, 1.0, 1.0)
    with pytest.raises(dg.DgmfError, match="INVALID"):
        gop.precond_apply(r, mg_coarse_tol=2.0)
    with pytest.raises(dg.DgmfError, match="INVALID"):
        gop.precond_info()                      # nothing built yet
    gm.close()


def test_full_size_poisson_mg():
    """Periodic Poisson on the 64^3-cell degree-3 cube, fp32 V-cycle inside fp64 CG."""
    require_gpu()
    import paper_1607_01323_amd as dg
    w = inp.POISSON_C2
    print(f"[case] multigrid full-size {w.name}", flush=True)
    gm = dg.Mesh(w.degree, *w.cells, *w.lengths, periodic=w.periodic)
    gop = dg.SipgOperator(gm, w.mass_coeff, w.diff_coeff, w.penalty_scale)
    om = omesh.BoxMesh(w.degree, *w.cells)
    oop = osipg.SIPG(om, w.mass_coeff, w.diff_coeff, w.penalty_scale)
    kr = kron.KronPeriodic(w.degree, *w.cells, mass_coeff=w.mass_coeff, diff_coeff=w.diff_coeff,
                           penalty_scale=w.penalty_scale)
    for rhs in ("configured", "random"):
        b = oop.rhs(inp.poisson_rhs_sin3) if rhs == "configured" else inp.uniform(5, om.ndofs)
        xg = dev(np.zeros(om.ndofs))
        out = gop.cg(dev(b), xg, rtol=1e-10, max_iter=200, check_every=4, precond="multigrid",
                     precond_dtype=torch.float32, seed=42, project_mean=True)
        assert out.status == 0
        bp = b - b.mean()
        xs = host(xg)
        assert np.linalg.norm(bp - kr.apply(xs)) <= 2e-10 * np.linalg.norm(bp)
        xf = kr.solve(bp)
        xs, xf = xs - xs.mean(), xf - xf.mean()
        err = np.linalg.norm(xs - xf) / np.linalg.norm(xf)
        print(f"[result] {rhs} rhs: MG iterations {out.iterations}, setup {out.setup_s:.3f} s, "
              f"solve {out.solve_s:.3f} s, rel. error vs exact discrete solution {err:.2e}", flush=True)
        assert out.iterations <= 20 and err < 1e-7
    gm.close()


def test_full_size_channel_mg():
    """Channel Helmholtz (stored-metric finest level, 48x32x48 cells, k = 4) with the fp32 V-cycle."""
    require_gpu()
    import paper_1607_01323_amd as dg
    w = inp.CHANNEL_C4
    print(f"[case] multigrid full-size {w.name}", flush=True)
    om = omesh.BoxMesh(w.degree, *w.cells, lx=w.lengths[0], ly=w.lengths[1], lz=w.lengths[2], y0=w.y0,
                       periodic=w.periodic, y_tanh_gamma=w.y_tanh_gamma)
    oop = osipg.SIPG(om, w.mass_coeff, w.diff_coeff, w.penalty_scale)
    b = oop.rhs(inp.channel_rhs(w.mass_coeff, w.diff_coeff))
    gm = dg.Mesh.from_workload(w)
    gop = dg.SipgOperator(gm, w.mass_coeff, w.diff_coeff, w.penalty_scale)
    xm = torch.zeros(om.ndofs, dtype=torch.float64, device="cuda")
    out = gop.cg(dev(b), xm, rtol=1e-10, max_iter=200, precond="multigrid", precond_dtype=torch.float32, seed=42)
    assert out.status == 0
    xs = host(xm)
    r = b - oop.apply_cells(xs, list(range(om.ncells))).ravel()
    print(f"[result] channel MG iterations {out.iterations}", flush=True)
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(b)
    gm.close()


def test_graph_replays_match_eager_launches():
    """The V-cycle replayed from its captured HIP graph equals the kernel-by-kernel
    launches bit for bit, on every replay, with eager work in between."""
    require_gpu()
    c = CASES["k3_aniso_coarsening"]
    om, gm, gop, singular = _setup(*c)
    rs = [dev(inp.uniform(100 + i, om.ndofs)) for i in range(3)]
    kw = dict(precond_dtype=torch.float32, seed=42, project_mean=singular)
    eager = [host(gop.precond_apply(r, mg_graph=False, **kw)) for r in rs]
    for rep in range(4):
        for i, r in enumerate(rs):
            z = host(gop.precond_apply(r, mg_graph=True, **kw))
            assert np.array_equal(z, eager[i]), (rep, i)
            torch.cuda.synchronize()
            _ = host(gop.precond_apply(rs[(i + 1) % 3], mg_graph=False, **kw))   # eager work between replays
    b = inp.uniform(5, om.ndofs)
    outs = []
    for graph in (False, True, True):
        x = dev(np.zeros(om.ndofs))
        o = gop.cg(dev(b), x, rtol=1e-10, max_iter=200, check_every=2, precond="multigrid",
                   precond_dtype=torch.float32, seed=42, project_mean=singular, mg_graph=graph)
        outs.append((o.iterations, host(x)))
    assert outs[0][0] == outs[1][0] == outs[2][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[1][1], outs[2][1])
    gm.close()
