"""The allocation-free CG entry point (dgmf_cg_solve_noalloc) against dgmf_cg_solve.

Both run the same kernels on the same inputs; the allocation-free one takes its
workspace from the library's static device buffer, which keeps the previous
call's contents.  Two calls in a row (the second on a smaller mesh, so stale
values of the first lie in the buffer) must give the iterates, iteration counts
and residuals of dgmf_cg_solve with a fresh workspace, to 1e-12 relative (fp64).
Requests the static buffer cannot hold, and the multigrid preconditioner (which
allocates its hierarchy), are refused before any work.
"""
import numpy as np
import pytest
import torch

import dgmf_inputs as inp
from tests.gpu_util import dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu

CASES = [
    # (workload, cells, solver keywords): the first is the larger one
    (inp.HELMHOLTZ_C1, (6, 5, 4), dict(precond="jacobi", rtol=1e-10, max_iter=2000)),
    (inp.HELMHOLTZ_C1, (6, 5, 4), dict(precond="chebyshev", precond_dtype=torch.float32, rtol=1e-10,
                                       max_iter=2000, seed=3)),
    (inp.POISSON_C0, None, dict(precond="jacobi", rtol=1e-10, max_iter=2000, project_mean=True)),
    (inp.POISSON_C0, (3, 3, 2), dict(precond="mass", rtol=1e-10, max_iter=4000, project_mean=True)),
]


def _mesh_op(w, cells):
    import paper_1607_01323_amd as dg
    cells = cells or w.cells
    m = dg.Mesh(w.degree, *cells, *w.lengths, y0=w.y0, periodic=w.periodic, y_tanh_gamma=w.y_tanh_gamma)
    return m, dg.SipgOperator(m, w.mass_coeff, w.diff_coeff, w.penalty_scale)


def test_noalloc_matches_workspace_solve_on_consecutive_calls():
    require_gpu()
    for k, (w, cells, kw) in enumerate(CASES):
        print(f"[case] cg_solve_noalloc {k}: {w.name} cells={cells or w.cells} {kw}", flush=True)
        m, op = _mesh_op(w, cells)
        N = m.ndofs
        b = inp.uniform(100 + k, N)
        if kw.get("project_mean"):
            b = b - b.mean()
        x0 = 0.1 * inp.uniform(200 + k, N)
        xa = dev(x0)
        ra = op.cg(dev(b), xa, check_every=4, **kw)
        xb = dev(x0)
        rb = op.cg_noalloc(dev(b), xb, check_every=4, **kw)
        assert rb.status == 0 and ra.status == 0
        assert rb.iterations == ra.iterations
        assert abs(rb.rel_residual - ra.rel_residual) <= 1e-12 * max(ra.rel_residual, 1e-300) + 1e-22
        assert rb.lambda_max == pytest.approx(ra.lambda_max, rel=1e-12, abs=0.0)
        assert rel_err(host(xb), host(xa)) <= 1e-12
        m.close()


def test_noalloc_refuses_what_it_cannot_hold():
    require_gpu()
    import paper_1607_01323_amd as dg
    print("[case] cg_solve_noalloc refusals", flush=True)
    w = inp.POISSON_C0
    m = dg.Mesh(w.degree, 32, 32, 32, *w.lengths, periodic=w.periodic)   # 2.1M DoF: > 64 MiB of workspace
    op = dg.SipgOperator(m, w.mass_coeff, w.diff_coeff, w.penalty_scale)
    b = torch.zeros(m.ndofs, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(dg.DgmfError) as ei:
        op.cg_noalloc(b, x, precond="jacobi")
    assert ei.value.status == dg.INVALID and "static buffer" in str(ei.value)
    m.close()
    m, op = _mesh_op(w, None)
    b = torch.zeros(m.ndofs, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(dg.DgmfError) as ei:
        op.cg_noalloc(b, x, precond="multigrid")
    assert ei.value.status == dg.UNSUPPORTED
    m.close()
