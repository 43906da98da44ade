"""GPU parity of the SIPG apply, diagonal, coordinates and load vector with the CPU oracle.

Bar: fp64 within 1e-12 relative (max norm, relative to the largest reference
entry); fp32 within 1e-5 relative.  Small meshes compare every entry with the
assembled CSR matrix; the full-size workloads compare sampled cells (corners
included, so periodic wrap and walls are covered) with the oracle's
row-restricted dense-block apply.
"""
import math

import numpy as np
import pytest
import torch

import dgmf_inputs as inp
from oracle import mesh as omesh, sipg as osipg
from tests.gpu_util import dev, host, rel_err, require_gpu, sample_cells

pytestmark = pytest.mark.gpu

CASES = {
    # name: (degree, cells, lengths, y0, periodic, gamma, mu, nu, s)
    "c0_poisson_k3": (3, (4, 4, 4), (1, 1, 1), 0, (1, 1, 1), 0, 0.0, 1.0, 1 / 3),
    "k1_ragged": (1, (5, 3, 7), (1, 1, 1), 0, (1, 1, 1), 0, 0.0, 1.0, 1.0),
    "k2_aniso": (2, (3, 4, 2), (1.3, 0.7, 0.4), 0, (1, 1, 1), 0, 2.0, 0.5, 1.0),
    "k4_helmholtz": (4, (3, 3, 3), (1, 1, 1), 0, (1, 1, 1), 0, 1000.0, 0.01, 1.0),
    "k5_dirichlet_all": (5, (2, 3, 2), (1, 0.8, 1.5), 0, (0, 0, 0), 0, 0.0, 1.0, 1.0),
    "k6_channel": (6, (2, 3, 2), (2 * math.pi, 2, math.pi), -1, (1, 0, 1), 1.8, 1000.0, 0.01, 1.0),
    "k7_small": (7, (2, 2, 2), (1, 1, 1), 0, (1, 1, 1), 0, 0.0, 1.0, 1.0),
    "one_cell_periodic": (3, (1, 2, 1), (1, 1, 1), 0, (1, 1, 1), 0, 1.0, 1.0, 1.0),
    "one_cell_dirichlet": (2, (1, 1, 1), (1, 1, 1), 0, (0, 0, 0), 0, 0.0, 1.0, 1.0),
    "k4_channel_tanh": (4, (3, 5, 2), (2 * math.pi, 2, math.pi), -1, (1, 0, 1), 1.8, 1000.0, 0.01, 1.0),
    # ragged x-y tiles and several z segments of the z-marching kernel
    "k3_uniform_long_z": (3, (7, 5, 37), (1, 1, 1), 0, (1, 1, 1), 0, 0.0, 1.0, 1 / 3),
    "k4_uniform_aniso_ragged": (4, (9, 3, 21), (1.3, 0.4, 2.0), 0, (1, 1, 1), 0, 1000.0, 0.01, 1.0),
    "k3_dirichlet_long_z": (3, (6, 5, 30), (1, 1, 1), 0, (0, 0, 0), 0, 1.0, 1.0, 1.0),
}


def _pair(name):
    import paper_1607_01323_amd as dg
    k, cells, L, y0, per, gam, mu, nu, s = CASES[name]
    om = omesh.BoxMesh(k, *cells, lx=L[0], ly=L[1], lz=L[2], y0=y0, periodic=tuple(bool(p) for p in per),
                       y_tanh_gamma=gam)
    oop = osipg.SIPG(om, mass_coeff=mu, diff_coeff=nu, penalty_scale=s)
    gm = dg.Mesh(k, *cells, *L, y0=y0, periodic=per, y_tanh_gamma=gam)
    gop = dg.SipgOperator(gm, mass_coeff=mu, diff_coeff=nu, penalty_scale=s)
    return om, oop, gm, gop


@pytest.mark.parametrize("name", list(CASES))
def test_apply_and_diagonal_match_assembled_matrix(name):
    require_gpu()
    print(f"[case] sipg apply {name}", flush=True)
    om, oop, gm, gop = _pair(name)
    A = oop.assemble()
    u = inp.uniform(100, om.ndofs)
    ref = A @ u
    y = host(gop.apply(dev(u)))
    assert rel_err(y, ref) < 1e-12
    y32 = host(gop.apply(dev(u, torch.float32)))
    assert rel_err(y32, ref) < 1e-5
    d = host(gop.diagonal())
    assert rel_err(d, A.diagonal()) < 1e-13
    d32 = host(gop.diagonal(torch.float32))
    assert rel_err(d32, A.diagonal()) < 1e-6
    gm.close()


def test_apply_is_deterministic_and_linear():
    require_gpu()
    om, oop, gm, gop = _pair("k4_channel_tanh")
    u = dev(inp.uniform(1, om.ndofs))
    v = dev(inp.uniform(2, om.ndofs))
    a1 = host(gop.apply(u))
    a2 = host(gop.apply(u))
    assert np.array_equal(a1, a2)
    b = host(gop.apply(v))
    c = host(gop.apply(2.0 * u - 3.0 * v))
    assert rel_err(c, 2 * a1 - 3 * b) < 1e-13
    gm.close()


def test_coordinates_and_load_vector():
    require_gpu()
    om, oop, gm, gop = _pair("k4_channel_tanh")
    X = host(gm.node_coords())
    np.testing.assert_allclose(X.T, om.node_coords(), rtol=0, atol=1e-14)
    Q = host(gop.quadrature_points())
    f = inp.channel_rhs(1000.0, 0.01)
    fq = f(Q[0], Q[1], Q[2])
    b = host(gop.integrate(dev(fq)))
    assert rel_err(b, oop.rhs(f)) < 1e-13
    gm.close()


FULL = {
    "helmholtz_periodic_32c_k4": inp.HELMHOLTZ_C1,
    "poisson_periodic_64c_k3": inp.POISSON_C2,
    "channel_48x32x48_k4_cartesian": inp.CHANNEL_C4,
}


@pytest.mark.parametrize("name", list(FULL))
def test_full_size_sampled_cells(name):
    require_gpu()
    import paper_1607_01323_amd as dg
    w = FULL[name]
    print(f"[case] sipg full-size {name}", flush=True)
    om = omesh.BoxMesh(w.degree, *w.cells, lx=w.lengths[0], ly=w.lengths[1], lz=w.lengths[2], y0=w.y0,
                       periodic=w.periodic, y_tanh_gamma=w.y_tanh_gamma)
    oop = osipg.SIPG(om, mass_coeff=w.mass_coeff, diff_coeff=w.diff_coeff, penalty_scale=w.penalty_scale)
    gm = dg.Mesh(w.degree, *w.cells, *w.lengths, y0=w.y0, periodic=w.periodic, y_tanh_gamma=w.y_tanh_gamma)
    gop = dg.SipgOperator(gm, w.mass_coeff, w.diff_coeff, w.penalty_scale)
    u = inp.uniform(7, om.ndofs)
    y = host(gop.apply(dev(u))).reshape(om.ncells, -1)
    cells = sample_cells(w.cells, 48, 3)
    ref = oop.apply_cells(u, cells)
    assert rel_err(y[cells], ref) < 1e-12
    dg_ = host(gop.diagonal()).reshape(om.ncells, -1)
    assert rel_err(dg_[cells], oop.diagonal_cells(cells)) < 1e-13
    y32 = host(gop.apply(dev(u, torch.float32))).reshape(om.ncells, -1)
    assert rel_err(y32[cells], ref) < 1e-5
    gm.close()
