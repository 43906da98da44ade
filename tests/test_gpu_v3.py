"""GPU parity of the mass apply and the V3c operators: divergence, gradient,
div-div penalty and the element-local projection solve.

Small meshes (several wavefront tiles, every degree, periodic and boundary
faces, tanh grading, single-cell periodic directions) are compared entry by
entry with the oracle's assembled matrices and dense per-cell solves; at the
full convective and channel sizes the duality <q, A u> = -<B q, u> (periodic)
holds to rounding and the projection is checked on sampled cells.
"""
import math

import numpy as np
import pytest
import torch

import dgmf_inputs as inp
from oracle import mesh as omesh, v3 as ov3
from tests.gpu_util import dev, host, rel_err, require_gpu, sample_cells

pytestmark = pytest.mark.gpu

MESHES = {
    # name: (k, cells, lengths, y0, periodic, gamma)
    "k1_periodic": (1, (3, 2, 4), (1, 1, 1), 0.0, (1, 1, 1), 0.0),
    "k2_dirichlet": (2, (2, 3, 2), (1, 0.7, 1.3), 0.0, (0, 0, 0), 0.0),
    "k3_channel": (3, (3, 4, 2), (2 * math.pi, 2, math.pi), -1.0, (1, 0, 1), 1.5),
    "k4_mixed": (4, (2, 2, 3), (0.5, 1, 2), 0.0, (0, 1, 1), 0.0),
    "k5_one_cell_periodic": (5, (1, 2, 1), (1, 1, 1), 0.0, (1, 1, 0), 0.0),
    "k6": (6, (2, 1, 2), (1, 1, 1), 0.0, (1, 0, 1), 0.0),
    "k7": (7, (1, 2, 1), (1, 1.5, 1), 0.0, (0, 1, 0), 0.0),
}


def _pair(k, cells, L, y0, per, gam):
    import paper_1607_01323_amd as dg
    om = omesh.BoxMesh(k, *cells, lx=L[0], ly=L[1], lz=L[2], y0=y0, periodic=tuple(bool(p) for p in per),
                       y_tanh_gamma=gam)
    gm = dg.Mesh(k, *cells, *L, y0=y0, periodic=per, y_tanh_gamma=gam)
    return om, gm


@pytest.mark.parametrize("name", list(MESHES))
def test_mass_divergence_gradient_small(name):
    require_gpu()
    print(f"[case] v3 operators {name}", flush=True)
    om, gm = _pair(*MESHES[name])
    N = om.ndofs
    U = inp.uniform(70, 3 * N)
    P = inp.uniform(71, N)
    ref_m = ov3.mass_apply(om, U)
    assert rel_err(host(gm.mass(dev(U))), ref_m) < 1e-13
    assert rel_err(host(gm.mass(dev(U, torch.float32))), ref_m) < 2e-6      # three fp32 sweeps of <= 8 terms
    x = dev(U)
    gm.mass(x, out=x)
    assert rel_err(host(x), ref_m) < 1e-13
    A = ov3.divergence_matrix(om)
    assert rel_err(host(gm.divergence(dev(U))), A @ U) < 1e-12
    B = ov3.gradient_matrix(om)
    assert rel_err(host(gm.gradient(dev(P))), B @ P) < 1e-12
    gm.close()


def _cell_residual(om, tau, rhs, x, rtol):
    """max over cells of the true residual ||rhs_e - A_e x_e|| (A_e = M_e + tau_e D_e from
    the oracle) over its bound rtol ||rhs_e|| + 100 eps ||A_e|| ||x_e||: CG stops on
    its recursive residual, and the true one can only be resolved to the
    rounding floor of forming A_e x_e."""
    from oracle import sipg as osipg
    T = osipg.Tables(om.k)
    R = rhs.reshape(3, om.ncells, -1)
    X = x.reshape(3, om.ncells, -1)
    worst = 0.0
    for c in range(om.ncells):
        J = om.jacobian(c)
        Ae = np.kron(np.eye(3), osipg.cell_matrices(T, J)[1]) + tau[c] * ov3.divdiv_cell(T, J)
        xe, be = X[:, c].ravel(), R[:, c].ravel()
        r = be - Ae @ xe
        bound = rtol * np.linalg.norm(be) + 100 * np.finfo(float).eps * np.linalg.norm(Ae, 2) * np.linalg.norm(xe)
        worst = max(worst, np.linalg.norm(r) / bound)
    return worst


@pytest.mark.parametrize("name", ["k1_periodic", "k3_channel", "k4_mixed", "k6"])
def test_penalty_and_projection_small(name):
    require_gpu()
    print(f"[case] v3 projection {name}", flush=True)
    om, gm = _pair(*MESHES[name])
    N, n3 = om.ndofs, om.n ** 3
    U = inp.uniform(72, 3 * N) + 0.5
    tau = host(gm.divdiv_penalty(dev(U), 3.0, 0.02))
    tau_ref = ov3.penalty_tau(om, U, 3.0, 0.02)
    assert rel_err(tau, tau_ref) < 1e-13
    # a spread of penalties, including zero (pure inverse mass) and large ones
    tau = np.abs(inp.uniform(73, om.ncells)) * 50.0
    tau[0] = 0.0
    rhs = inp.uniform(74, 3 * N)
    its = torch.zeros(om.ncells, dtype=torch.int32, device="cuda")
    x = host(gm.projection_solve(dev(tau), dev(rhs), rtol=1e-13, max_iter=3 * n3, iterations=its))
    ref = ov3.projection_solve(om, tau, rhs)
    # the true residual of every cell within its bound; the error within
    # cond(M_e + tau D_e) (up to ~1e3 at k = 6) times the residual
    assert _cell_residual(om, tau, rhs, x, 1e-13) <= 1.0
    assert rel_err(x, ref) < 1e-9
    it = its.cpu().numpy()
    print(f"  iterations per cell: min {it.min()} max {it.max()} (local size {3 * n3})", flush=True)
    assert it.max() <= 3 * n3 and it[0] <= 2           # tau = 0: the preconditioner is the exact inverse
    # restart from the solution: nothing to do; max_iter = 0 leaves x untouched
    x2 = gm.projection_solve(dev(tau), dev(rhs), x=dev(x), rtol=1e-8, iterations=its)
    assert int(its.max()) == 0 and rel_err(host(x2), x) == 0.0
    x3 = gm.projection_solve(dev(tau), dev(rhs), x=dev(rhs), max_iter=0)
    assert np.array_equal(host(x3), rhs)
    gm.close()


def test_v3_rejects_bad_arguments():
    require_gpu()
    import paper_1607_01323_amd as dg
    sh = ((1.0, 0.2, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))
    gm = dg.Mesh(2, 2, 2, 2, store_qp_metric=True, shear=sh)
    u = torch.zeros(3 * gm.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.DgmfError, match="UNSUPPORTED"):
        gm.divergence(u)
    gm.close()
    gm = dg.Mesh(2, 2, 2, 2)
    u = torch.zeros(3 * gm.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.DgmfError, match="INVALID"):
        gm.divdiv_penalty(u, -1.0, 0.1)
    with pytest.raises(dg.DgmfError, match="INVALID"):
        gm.projection_solve(torch.zeros(gm.ncells, dtype=torch.float64, device="cuda"), u, x=u)   # x aliases rhs
    gm.close()


FULL = {"convective_periodic_32c_k5": inp.CONVECTIVE_C3, "channel_48x32x48_k4": inp.CHANNEL_C4}


@pytest.mark.parametrize("name", list(FULL))
def test_full_size(name):
    require_gpu()
    import paper_1607_01323_amd as dg
    w = FULL[name]
    print(f"[case] v3 full-size {name}", flush=True)
    om = omesh.BoxMesh(w.degree, *w.cells, lx=w.lengths[0], ly=w.lengths[1], lz=w.lengths[2], y0=w.y0,
                       periodic=w.periodic, y_tanh_gamma=w.y_tanh_gamma)
    gm = dg.Mesh(w.degree, *w.cells, *w.lengths, y0=w.y0, periodic=w.periodic, y_tanh_gamma=w.y_tanh_gamma)
    N, n3 = om.ndofs, om.n ** 3
    U = dev(inp.uniform(80, 3 * N))
    Q = dev(inp.uniform(81, N))
    AU = gm.divergence(U)
    BQ = gm.gradient(Q)
    lhs, rhs = float(torch.dot(Q, AU)), -float(torch.dot(BQ, U))
    scale = float(torch.linalg.vector_norm(Q) * torch.linalg.vector_norm(AU))
    if all(w.periodic):
        assert abs(lhs - rhs) <= 1e-12 * scale
    cells = sample_cells(w.cells, 16, 9)
    tau = gm.divdiv_penalty(U + 0.3, 1.0, 1e-2)
    tau_h = host(tau)
    Uh = host(U) + 0.3
    rhs_v = inp.uniform(82, 3 * N)
    its = torch.zeros(om.ncells, dtype=torch.int32, device="cuda")
    x = host(gm.projection_solve(tau, dev(rhs_v), rtol=1e-13, max_iter=3 * n3, iterations=its)).reshape(3, om.ncells,
                                                                                                         -1)
    R = rhs_v.reshape(3, om.ncells, -1)[:, cells]
    ref = ov3.projection_solve(om, tau_h, R, cells=cells)
    assert rel_err(x[:, cells], ref) < 1e-9
    # tau on the sampled cells, from the oracle's definition
    from oracle import sipg as osipg
    gwc = osipg.integral_weights(omesh.BoxMesh(w.degree, 1, 1, 1)).reshape(-1)   # unit-cube basis integrals
    Uc = Uh.reshape(3, om.ncells, -1)
    for c in cells:
        V = om.volume(c)
        ubar = np.array([gwc @ Uc[a, c] for a in range(3)])
        assert abs(tau_h[c] - np.linalg.norm(ubar) * V ** (1 / 3) * 1e-2) <= 1e-13 * max(tau_h[c], 1e-300)
    print(f"  projection iterations: max {int(its.max())}, mean {float(its.float().mean()):.1f}", flush=True)
    gm.close()


def test_divergence_gradient_projection_with_neumann_sides():
    """The ND average is the own trace on Neumann sides as on Dirichlet ones (Sec. 3.1)."""
    require_gpu()
    import paper_1607_01323_amd as dg
    print("[case] v3 operators with Neumann sides", flush=True)
    neu = (1, 0, 1, 1, 0, 0)
    om = omesh.BoxMesh(3, 3, 2, 2, lx=1.0, ly=2.0, lz=1.0, y0=-1.0, periodic=(False, False, True),
                       y_tanh_gamma=1.2, neumann=tuple(bool(f) for f in neu))
    gm = dg.Mesh(3, 3, 2, 2, 1.0, 2.0, 1.0, y0=-1.0, periodic=(0, 0, 1), y_tanh_gamma=1.2, neumann=neu)
    U = inp.uniform(75, 3 * om.ndofs)
    P = inp.uniform(76, om.ndofs)
    assert rel_err(host(gm.divergence(dev(U))), ov3.divergence_matrix(om) @ U) < 1e-12
    assert rel_err(host(gm.gradient(dev(P))), ov3.gradient_matrix(om) @ P) < 1e-12
    tau = np.abs(inp.uniform(77, om.ncells)) * 10.0
    x = host(gm.projection_solve(dev(tau), dev(U), rtol=1e-13, max_iter=3 * om.n ** 3))
    assert rel_err(x, ov3.projection_solve(om, tau, U)) < 1e-9
    gm.close()
