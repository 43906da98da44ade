"""Box meshes of affine hexahedra (oracle; test infrastructure).

Sec. 3.1 of the paper: a tessellation into hexahedra, interior faces shared
by a minus and a plus element with opposite normals, exterior faces split into
Dirichlet and Neumann parts.  Here: an axis-aligned box
[0,lx] x [y0,y0+ly] x [0,lz] cut into nx*ny*nz cells, each direction either
periodic (wrap-around faces count as interior faces) or bounded at both ends,
each bounding side Dirichlet or homogeneous Neumann (``neumann``, six flags
in face-id order; ignored in periodic directions).
The y vertices may be graded with the hyperbolic channel mapping of Sec. 7.1,
y = y0 + ly/2 * (1 + tanh(gamma (2t-1)) / tanh(gamma)), t in [0,1].

Numbering (shared convention, not shared code):
  cell c = (cz*ny + cy)*nx + cx,
  DoF  g = c*n^3 + (l*n + j)*n + i, x node index i fastest, n = k+1,
  face id f = 2*d + s, direction d in {x,y,z}, side s=0 the low face, s=1 the high face.

Cells may carry a general constant Jacobian (``jac``, 3x3, x = x0 + J xi),
used by the oracle's tests of sheared lattices; box meshes use diag(h).
"""
import numpy as np

from . import basis


class BoxMesh:
    def __init__(self, degree, nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, y0=0.0,
                 periodic=(True, True, True), y_tanh_gamma=0.0, shear=None, neumann=(False,) * 6):
        self.k = int(degree)
        self.n = self.k + 1
        self.nc = (int(nx), int(ny), int(nz))
        self.periodic = tuple(bool(p) for p in periodic)
        self.neumann = tuple(bool(neumann[f]) and not self.periodic[f // 2] for f in range(6))
        self.gamma = float(y_tanh_gamma)
        t = np.arange(ny + 1) / ny
        if self.gamma > 0:
            yv = y0 + 0.5 * ly * (1.0 + np.tanh(self.gamma * (2 * t - 1)) / np.tanh(self.gamma))
        else:
            yv = y0 + ly * t
        self.verts = (np.linspace(0.0, lx, nx + 1), yv, np.linspace(0.0, lz, nz + 1))
        # optional constant shear: physical x = J_shear @ (box point); keeps a lattice
        self.shear = None if shear is None else np.asarray(shear, dtype=np.float64)
        self.ncells = nx * ny * nz
        self.ndofs = self.ncells * self.n ** 3

    # -- cell indexing -------------------------------------------------------
    def cell_index(self, cx, cy, cz):
        nx, ny, _ = self.nc
        return (cz * ny + cy) * nx + cx

    def cell_coords(self, c):
        nx, ny, _ = self.nc
        return c % nx, (c // nx) % ny, c // (nx * ny)

    def cell_origin_h(self, c):
        idx = self.cell_coords(c)
        o = np.array([self.verts[d][idx[d]] for d in range(3)])
        h = np.array([self.verts[d][idx[d] + 1] - self.verts[d][idx[d]] for d in range(3)])
        return o, h

    def jacobian(self, c):
        """Constant Jacobian dx/dxi of the affine map of cell c."""
        _, h = self.cell_origin_h(c)
        J = np.diag(h)
        if self.shear is not None:
            J = self.shear @ J
        return J

    def neighbor(self, c, f):
        """Cell across face f of cell c, or -1 on the boundary (Dirichlet or Neumann)."""
        d, s = divmod(f, 2)
        idx = list(self.cell_coords(c))
        idx[d] += 1 if s == 1 else -1
        if idx[d] < 0 or idx[d] >= self.nc[d]:
            if not self.periodic[d]:
                return -1
            idx[d] %= self.nc[d]
        return self.cell_index(*idx)

    def interior_faces(self):
        """(cL, cR, d): cR is the +d neighbour of cL (periodic wrap included)."""
        out = []
        for c in range(self.ncells):
            for d in range(3):
                cr = self.neighbor(c, 2 * d + 1)
                if cr >= 0:
                    out.append((c, cr, d))
        return out

    def boundary_faces(self):
        """(c, f) for every face of a cell on the Dirichlet boundary."""
        return [(c, f) for c in range(self.ncells) for f in range(6)
                if self.neighbor(c, f) < 0 and not self.neumann[f]]

    def neumann_faces(self):
        """(c, f) for every face of a cell on the Neumann boundary."""
        return [(c, f) for c in range(self.ncells) for f in range(6) if self.neighbor(c, f) < 0 and self.neumann[f]]

    def has_neumann(self):
        return any(self.neumann)

    # -- geometry ------------------------------------------------------------
    def face_area(self, c, f):
        """Area of face f of cell c: det J * |J^{-T} e_d| for the affine map."""
        J = self.jacobian(c)
        d = f // 2
        return abs(np.linalg.det(J)) * np.linalg.norm(np.linalg.inv(J).T[:, d])

    def volume(self, c):
        return abs(np.linalg.det(self.jacobian(c)))

    def node_coords(self):
        """Physical coordinates of every DoF, shape (ndofs, 3)."""
        xi = basis.gll_nodes(self.k)
        n = self.n
        L, Jj, I = np.meshgrid(xi, xi, xi, indexing="ij")       # (l, j, i) -> z, y, x
        ref = np.stack([I.ravel(), Jj.ravel(), L.ravel()], axis=1)  # (n^3, 3)
        out = np.empty((self.ndofs, 3))
        for c in range(self.ncells):
            o, _ = self.cell_origin_h(c)
            x0 = o if self.shear is None else self.shear @ o
            out[c * n ** 3:(c + 1) * n ** 3] = x0 + ref @ self.jacobian(c).T
        return out
