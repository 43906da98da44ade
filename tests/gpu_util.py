"""Helpers shared by the GPU parity tests (no arithmetic of the method)."""
import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def rel_err(a, ref):
    scale = np.abs(ref).max()
    return np.abs(a - ref).max() / (scale if scale > 0 else 1.0)


def sample_cells(mesh_shape, count, seed):
    """Boundary-heavy sample of cell indices: the 8 corners plus random cells."""
    nx, ny, nz = mesh_shape
    corners = [(x, y, z) for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)]
    idx = {(cz * ny + cy) * nx + cx for cx, cy, cz in corners}
    rng = np.random.default_rng(seed)
    idx.update(rng.integers(0, nx * ny * nz, size=count).tolist())
    return sorted(idx)
