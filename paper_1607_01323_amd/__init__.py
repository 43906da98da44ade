"""Python binding of libdgmf: matrix-free DG operators on MI355X (gfx950).

Thin ctypes marshalling over the C-ABI declared in ``include/dgmf.h``; every
step of the computation runs in the library's HIP kernels.  Tensors are
PyTorch device tensors (contiguous, dtype as documented per call) and work
is enqueued on ``torch.cuda.current_stream()``.  There is no CPU fallback:
if the built library is missing, importing this package raises.

Build the library with ``python paper_1607_01323_amd/build.py``.
"""
import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgmf.so")

OK, INVALID, HIP_ERROR, OOM, NOT_CONVERGED, BREAKDOWN, NONFINITE, UNSUPPORTED = range(8)
STATUS_NAMES = ["OK", "INVALID", "HIP_ERROR", "OOM", "NOT_CONVERGED", "BREAKDOWN", "NONFINITE", "UNSUPPORTED"]
F64, F32 = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_1607_01323_amd/build.py` (hipcc, gfx950)")
_lib = ctypes.CDLL(LIB_PATH)

_vp, _i64 = ctypes.c_void_p, ctypes.c_int64


class BoxDesc(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double), ("y0", ctypes.c_double),
                ("periodic", ctypes.c_int * 3), ("y_tanh_gamma", ctypes.c_double), ("store_qp_metric", ctypes.c_int),
                ("shear", ctypes.c_double * 9), ("neumann", ctypes.c_int * 6), ("curve_amp", ctypes.c_double)]


class SipgDesc(ctypes.Structure):
    _fields_ = [("mass_coeff", ctypes.c_double), ("diff_coeff", ctypes.c_double),
                ("penalty_scale", ctypes.c_double), ("n_q", ctypes.c_int)]


class CgParams(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int), ("check_every", ctypes.c_int),
                ("precond", ctypes.c_int), ("precond_dtype", ctypes.c_int), ("cheb_degree", ctypes.c_int),
                ("smoothing_range", ctypes.c_double), ("lanczos_steps", ctypes.c_int),
                ("lambda_safety", ctypes.c_double), ("seed", ctypes.c_uint64), ("project_mean", ctypes.c_int),
                ("flexible", ctypes.c_int), ("mg_coarse_tol", ctypes.c_double), ("mg_graph", ctypes.c_int)]


class CgResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("status", ctypes.c_int), ("setup_s", ctypes.c_double), ("solve_s", ctypes.c_double)]


class ConvDesc(ctypes.Structure):
    _fields_ = [("n_q", ctypes.c_int)]


def _sig(name, *args):
    f = getattr(_lib, name)
    f.restype = ctypes.c_int
    f.argtypes = list(args)
    return f


_lib.dgmf_last_error.restype = ctypes.c_char_p
_lib.dgmf_last_error.argtypes = []
_lib.dgmf_version.restype = ctypes.c_int
_mesh_create = _sig("dgmf_mesh_create", ctypes.POINTER(BoxDesc), ctypes.POINTER(_vp))
_mesh_info = _sig("dgmf_mesh_info", _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64))
_mesh_coords = _sig("dgmf_mesh_node_coords", _vp, _vp, _vp)
_mesh_destroy = _sig("dgmf_mesh_destroy", _vp)
_inv_mass = _sig("dgmf_inverse_mass_apply", _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp)
_mass = _sig("dgmf_mass_apply", _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp)
_div = _sig("dgmf_divergence_apply", _vp, _vp, _vp, _vp)
_visc = _sig("dgmf_viscous_apply", _vp, _vp, _vp, _vp)
_visc_ws = _sig("dgmf_viscous_cg_workspace_bytes", _vp, ctypes.POINTER(ctypes.c_size_t))
_visc_cg = _sig("dgmf_viscous_cg_solve", _vp, _vp, _vp, ctypes.POINTER(CgParams), _vp, ctypes.c_size_t, _vp,
                ctypes.POINTER(CgResult))
_grad = _sig("dgmf_gradient_apply", _vp, _vp, _vp, _vp)
_divdiv_tau = _sig("dgmf_divdiv_penalty", _vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp)
_proj = _sig("dgmf_projection_solve", _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _vp, _vp)
_sipg_create = _sig("dgmf_sipg_create", _vp, ctypes.POINTER(SipgDesc), ctypes.POINTER(_vp))
_apply = _sig("dgmf_operator_apply", _vp, ctypes.c_int, _vp, _vp, _vp)
_diag = _sig("dgmf_operator_diagonal", _vp, ctypes.c_int, _vp, _vp)
_qpts = _sig("dgmf_quadrature_points", _vp, _vp, _vp)
_integ = _sig("dgmf_integrate", _vp, _vp, _vp, _vp)
_ws_bytes = _sig("dgmf_cg_workspace_bytes", _vp, ctypes.POINTER(CgParams), ctypes.POINTER(ctypes.c_size_t))
_cg = _sig("dgmf_cg_solve", _vp, _vp, _vp, ctypes.POINTER(CgParams), _vp, ctypes.c_size_t, _vp,
           ctypes.POINTER(CgResult))
_cg_noalloc = _sig("dgmf_cg_solve_noalloc", _vp, _vp, _vp, ctypes.POINTER(CgParams), _vp, ctypes.POINTER(CgResult))
_pc_apply = _sig("dgmf_precond_apply", _vp, ctypes.POINTER(CgParams), _vp, _vp, _vp)
_pc_info = _sig("dgmf_precond_info", _vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double))
_conv_create = _sig("dgmf_convective_create", _vp, ctypes.POINTER(ConvDesc), ctypes.POINTER(_vp))
_conv_apply = _sig("dgmf_convective_apply", _vp, _vp, _vp, _vp)
_conv_vjp = _sig("dgmf_convective_vjp", _vp, _vp, _vp, _vp, _vp)
_conv_step = _sig("dgmf_convective_step", _vp, ctypes.c_double, _vp, _vp, _vp)
_op_destroy = _sig("dgmf_op_destroy", _vp)


class DgmfError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.dgmf_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES[status] if 0 <= status < 8 else status}: {msg}")


def _check(st, where):
    if st != OK:
        raise DgmfError(st, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, numel, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def version():
    return _lib.dgmf_version()


class Mesh:
    """Box mesh of affine hexahedra (see ``dgmf_box_desc``); ``neumann``: six per-side
    flags (x-, x+, y-, y+, z-, z+), homogeneous Neumann instead of Dirichlet;
    ``curve_amp``: amplitude of the iso-parametric curved-cell deformation."""

    def __init__(self, degree, nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, y0=0.0, periodic=(1, 1, 1),
                 y_tanh_gamma=0.0, store_qp_metric=False, shear=None, neumann=(0, 0, 0, 0, 0, 0), curve_amp=0.0):
        sh = [0.0] * 9 if shear is None else [float(v) for row in shear for v in row]
        if len(neumann) != 6:
            raise ValueError("neumann: six per-side flags")
        d = BoxDesc(degree, nx, ny, nz, lx, ly, lz, y0, (ctypes.c_int * 3)(*[int(bool(p)) for p in periodic]),
                    y_tanh_gamma, int(bool(store_qp_metric)), (ctypes.c_double * 9)(*sh),
                    (ctypes.c_int * 6)(*[int(bool(f)) for f in neumann]), float(curve_amp))
        self._h = _vp()
        _check(_mesh_create(ctypes.byref(d), ctypes.byref(self._h)), "mesh_create")
        nc, nd = _i64(), _i64()
        _check(_mesh_info(self._h, ctypes.byref(nc), ctypes.byref(nd)), "mesh_info")
        self.degree = degree
        self.ncells, self.ndofs = nc.value, nd.value
        self._ops = []

    @classmethod
    def from_workload(cls, w):
        return cls(w.degree, *w.cells, *w.lengths, y0=w.y0, periodic=w.periodic, y_tanh_gamma=w.y_tanh_gamma,
                   store_qp_metric=w.store_qp_metric, neumann=getattr(w, "neumann", (0,) * 6),
                   curve_amp=getattr(w, "curve_amp", 0.0))

    def node_coords(self):
        out = torch.empty(3 * self.ndofs, dtype=torch.float64, device="cuda")
        _check(_mesh_coords(self._h, _ptr(out, torch.float64, 3 * self.ndofs, "xyz"), _stream()), "node_coords")
        return out.view(3, self.ndofs)

    def mass(self, src, out=None):
        """M src for one or more scalar fields laid out [n_fields][N] (fp64 or fp32); out may be src."""
        return self._block_mass(_mass, "mass_apply", src, out)

    def divergence(self, u, out=None):
        """A u: weak divergence with central fluxes (eq. av3 without gamma_0/dt); u [3][N] -> [N]."""
        if out is None:
            out = torch.empty(self.ndofs, dtype=torch.float64, device=u.device)
        _check(_div(self._h, _ptr(u, torch.float64, 3 * self.ndofs, "u"), _ptr(out, torch.float64, self.ndofs, "out"),
                    _stream()), "divergence_apply")
        return out

    def gradient(self, p, out=None):
        """B p: weak gradient with central fluxes (eq. bv3 without dt/gamma_0); p [N] -> [3][N]."""
        if out is None:
            out = torch.empty(3 * self.ndofs, dtype=torch.float64, device=p.device)
        _check(_grad(self._h, _ptr(p, torch.float64, self.ndofs, "p"),
                     _ptr(out, torch.float64, 3 * self.ndofs, "out"), _stream()), "gradient_apply")
        return out

    def divdiv_penalty(self, u, zeta, dt, out=None):
        """tau_D per cell = zeta |u_bar| V^(1/3) dt (eq. tauD)."""
        if out is None:
            out = torch.empty(self.ncells, dtype=torch.float64, device=u.device)
        _check(_divdiv_tau(self._h, _ptr(u, torch.float64, 3 * self.ndofs, "u"), float(zeta), float(dt),
                           _ptr(out, torch.float64, self.ncells, "tau"), _stream()), "divdiv_penalty")
        return out

    def projection_solve(self, tau, rhs, x=None, rtol=1e-12, max_iter=1000, iterations=None):
        """Per cell (M_e + tau_e D_e) x_e = rhs_e by element-local CG; x (in/out) starts at zero when None."""
        if x is None:
            x = torch.zeros_like(rhs)
        it = _vp(None) if iterations is None else _ptr(iterations, torch.int32, self.ncells, "iterations")
        _check(_proj(self._h, _ptr(tau, torch.float64, self.ncells, "tau"), _ptr(rhs, torch.float64, 3 * self.ndofs,
                     "rhs"), _ptr(x, torch.float64, 3 * self.ndofs, "x"), float(rtol), int(max_iter), it, _stream()),
               "projection_solve")
        return x

    def _block_mass(self, fn, name, src, out):
        if src.numel() % self.ndofs:
            raise ValueError(f"src must hold a whole number of fields of {self.ndofs} values")
        nf = src.numel() // self.ndofs
        dt = {torch.float64: F64, torch.float32: F32}.get(src.dtype)
        if dt is None:
            raise TypeError(f"src must be float64 or float32, got {src.dtype}")
        if out is None:
            out = torch.empty_like(src)
        _check(fn(self._h, dt, nf, _ptr(src, src.dtype, src.numel(), "src"), _ptr(out, src.dtype, src.numel(), "out"),
                  _stream()), name)
        return out

    def inverse_mass(self, src, out=None):
        """M^{-1} src for one or more scalar fields laid out [n_fields][N] (fp64 or fp32); out may be src."""
        if src.numel() % self.ndofs:
            raise ValueError(f"src must hold a whole number of fields of {self.ndofs} values")
        nf = src.numel() // self.ndofs
        dt = {torch.float64: F64, torch.float32: F32}.get(src.dtype)
        if dt is None:
            raise TypeError(f"src must be float64 or float32, got {src.dtype}")
        if out is None:
            out = torch.empty_like(src)
        _check(_inv_mass(self._h, dt, nf, _ptr(src, src.dtype, src.numel(), "src"),
                         _ptr(out, src.dtype, src.numel(), "out"), _stream()), "inverse_mass_apply")
        return out

    def close(self):
        for op in self._ops:
            op.close()
        self._ops = []
        if self._h:
            _check(_mesh_destroy(self._h), "mesh_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Op:
    def __init__(self, mesh):
        self.mesh = mesh
        self._h = _vp()
        mesh._ops.append(self)

    def close(self):
        if self._h:
            _check(_op_destroy(self._h), "op_destroy")
            self._h = None


class SipgOperator(_Op):
    """H = mass_coeff M + diff_coeff A (SIPG), see ``dgmf_sipg_desc``."""

    def __init__(self, mesh, mass_coeff=0.0, diff_coeff=1.0, penalty_scale=1.0, n_q=0):
        super().__init__(mesh)
        d = SipgDesc(mass_coeff, diff_coeff, penalty_scale, n_q)
        _check(_sipg_create(mesh._h, ctypes.byref(d), ctypes.byref(self._h)), "sipg_create")
        self.nq = mesh.degree + 1

    def apply(self, src, out=None):
        dt = F64 if src.dtype == torch.float64 else F32
        if out is None:
            out = torch.empty_like(src)
        _check(_apply(self._h, dt, _ptr(src, src.dtype, self.mesh.ndofs, "src"),
                      _ptr(out, src.dtype, self.mesh.ndofs, "dst"), _stream()), "operator_apply")
        return out

    def viscous_apply(self, u, out=None):
        """H_eps u for a velocity [3][N]: mu M + the SIPG form of (eps(v), 2 nu eps(u))."""
        n = 3 * self.mesh.ndofs
        if out is None:
            out = torch.empty_like(u)
        _check(_visc(self._h, _ptr(u, torch.float64, n, "u"), _ptr(out, torch.float64, n, "out"), _stream()),
               "viscous_apply")
        return out

    def diagonal(self, dtype=torch.float64):
        out = torch.empty(self.mesh.ndofs, dtype=dtype, device="cuda")
        _check(_diag(self._h, F64 if dtype == torch.float64 else F32, _ptr(out, dtype, self.mesh.ndofs, "diag"),
                     _stream()), "operator_diagonal")
        return out

    def quadrature_points(self):
        m = self.mesh.ncells * self.nq ** 3
        out = torch.empty(3 * m, dtype=torch.float64, device="cuda")
        _check(_qpts(self._h, _ptr(out, torch.float64, 3 * m, "xyz"), _stream()), "quadrature_points")
        return out.view(3, m)

    def integrate(self, f_qp):
        m = self.mesh.ncells * self.nq ** 3
        b = torch.empty(self.mesh.ndofs, dtype=torch.float64, device="cuda")
        _check(_integ(self._h, _ptr(f_qp, torch.float64, m, "f_qp"), _ptr(b, torch.float64, self.mesh.ndofs, "b"),
                      _stream()), "integrate")
        return b

    _PRECONDS = {"jacobi": 0, "chebyshev": 1, "multigrid": 2, "mass": 3}

    def _params(self, rtol, max_iter, check_every, precond, precond_dtype, cheb_degree, smoothing_range,
                lanczos_steps, lambda_safety, seed, project_mean, flexible, mg_coarse_tol, mg_graph=True):
        if precond not in self._PRECONDS:
            raise ValueError(f"precond must be one of {sorted(self._PRECONDS)}")
        if flexible is None:
            flexible = precond in ("chebyshev", "multigrid") and precond_dtype == torch.float32
        return CgParams(rtol, max_iter, check_every, self._PRECONDS[precond],
                        F64 if precond_dtype == torch.float64 else F32, cheb_degree, smoothing_range, lanczos_steps,
                        lambda_safety, seed, int(bool(project_mean)), int(bool(flexible)), mg_coarse_tol,
                        int(bool(mg_graph)))

    def precond_apply(self, r, precond_dtype=torch.float32, cheb_degree=5, smoothing_range=20.0, lanczos_steps=15,
                      lambda_safety=1.2, seed=0, project_mean=False, mg_coarse_tol=0.0, out=None, mg_graph=True):
        """z = B r, one multigrid V-cycle (fp64 in and out, computed in precond_dtype)."""
        p = self._params(0.0, 0, 1, "multigrid", precond_dtype, cheb_degree, smoothing_range, lanczos_steps,
                         lambda_safety, seed, project_mean, False, mg_coarse_tol, mg_graph)
        n = self.mesh.ndofs
        if out is None:
            out = torch.empty_like(r)
        _check(_pc_apply(self._h, ctypes.byref(p), _ptr(r, torch.float64, n, "r"), _ptr(out, torch.float64, n, "z"),
                         _stream()), "precond_apply")
        return out

    def precond_info(self):
        """(levels, per-level lambdas, coarse degree, coarse interval) of the built multigrid hierarchy."""
        lv, deg = ctypes.c_int(), ctypes.c_int()
        lam = (ctypes.c_double * 32)()
        iv = (ctypes.c_double * 2)()
        _check(_pc_info(self._h, ctypes.byref(lv), lam, ctypes.byref(deg), iv), "precond_info")
        return lv.value, list(lam[:lv.value]), deg.value, (iv[0], iv[1])

    def cg(self, b, x, rtol=1e-10, max_iter=1000, check_every=8, precond="jacobi", precond_dtype=torch.float64,
           cheb_degree=5, smoothing_range=20.0, lanczos_steps=15, lambda_safety=1.2, seed=0, project_mean=False,
           flexible=None, raise_on_failure=True, mg_coarse_tol=0.0, mg_graph=True):
        """PCG on H x = b; x (fp64, device) holds the initial guess and receives the solution.

        precond: "jacobi", "chebyshev", "multigrid" or "mass" (inverse mass matrix, the
        viscous-step preconditioner).  flexible=None picks the
        Polak-Ribiere (flexible) beta exactly when the preconditioner runs in fp32.
        """
        p = self._params(rtol, max_iter, check_every, precond, precond_dtype, cheb_degree, smoothing_range,
                         lanczos_steps, lambda_safety, seed, project_mean, flexible, mg_coarse_tol, mg_graph)
        nbytes = ctypes.c_size_t()
        _check(_ws_bytes(self._h, ctypes.byref(p), ctypes.byref(nbytes)), "cg_workspace_bytes")
        ws = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device="cuda")
        res = CgResult()
        st = _cg(self._h, _ptr(b, torch.float64, self.mesh.ndofs, "b"), _ptr(x, torch.float64, self.mesh.ndofs, "x"),
                 ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()), nbytes.value, _stream(), ctypes.byref(res))
        out = CgOutcome(res.iterations, res.rel_residual, res.lambda_max, res.status, res.setup_s, res.solve_s)
        if st not in (OK, NOT_CONVERGED, BREAKDOWN, NONFINITE) or (raise_on_failure and st != OK):
            raise DgmfError(st, "cg_solve")
        return out

    def cg_noalloc(self, b, x, rtol=1e-10, max_iter=1000, check_every=8, precond="jacobi",
                   precond_dtype=torch.float64, cheb_degree=5, smoothing_range=20.0, lanczos_steps=15,
                   lambda_safety=1.2, seed=0, project_mean=False, flexible=None, raise_on_failure=True):
        """cg() on the library's static workspace (dgmf_cg_solve_noalloc): no device
        allocation by the library or here; precond "jacobi", "chebyshev" or "mass"."""
        p = self._params(rtol, max_iter, check_every, precond, precond_dtype, cheb_degree, smoothing_range,
                         lanczos_steps, lambda_safety, seed, project_mean, flexible, 0.0, False)
        res = CgResult()
        st = _cg_noalloc(self._h, _ptr(b, torch.float64, self.mesh.ndofs, "b"),
                         _ptr(x, torch.float64, self.mesh.ndofs, "x"), ctypes.byref(p), _stream(),
                         ctypes.byref(res))
        out = CgOutcome(res.iterations, res.rel_residual, res.lambda_max, res.status, res.setup_s, res.solve_s)
        if st not in (OK, NOT_CONVERGED, BREAKDOWN, NONFINITE) or (raise_on_failure and st != OK):
            raise DgmfError(st, "cg_solve_noalloc")
        return out

    def viscous_cg(self, b, x, rtol=1e-10, max_iter=1000, check_every=8, precond="jacobi", raise_on_failure=True):
        """PCG on H_eps x = b (the symmetric-gradient viscous operator); b, x: fp64 [3][N],
        x holds the initial guess and receives the solution.  precond: "jacobi" (the scalar
        operator's diagonal) or "mass" (the inverse mass matrix)."""
        if precond not in ("jacobi", "mass"):
            raise ValueError("precond must be 'jacobi' or 'mass'")
        n = 3 * self.mesh.ndofs
        p = CgParams()
        p.rtol, p.max_iter, p.check_every, p.precond = rtol, max_iter, check_every, 0 if precond == "jacobi" else 3
        nbytes = ctypes.c_size_t()
        _check(_visc_ws(self._h, ctypes.byref(nbytes)), "viscous_cg_workspace_bytes")
        ws = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device="cuda")
        res = CgResult()
        st = _visc_cg(self._h, _ptr(b, torch.float64, n, "b"), _ptr(x, torch.float64, n, "x"), ctypes.byref(p),
                      ctypes.c_void_p(ws.data_ptr()), nbytes.value, _stream(), ctypes.byref(res))
        out = CgOutcome(res.iterations, res.rel_residual, 0.0, res.status, res.setup_s, res.solve_s)
        if st not in (OK, NOT_CONVERGED, BREAKDOWN, NONFINITE) or (raise_on_failure and st != OK):
            raise DgmfError(st, "viscous_cg_solve")
        return out


@dataclass
class CgOutcome:
    iterations: int
    rel_residual: float
    lambda_max: float
    status: int
    setup_s: float
    solve_s: float


class ConvectiveOperator(_Op):
    """C(U) of the divergence-form convective term with local Lax-Friedrichs flux."""

    def __init__(self, mesh, n_q=0):
        super().__init__(mesh)
        d = ConvDesc(n_q)
        _check(_conv_create(mesh._h, ctypes.byref(d), ctypes.byref(self._h)), "convective_create")

    def apply(self, u, out=None):
        n = 3 * self.mesh.ndofs
        if out is None:
            out = torch.empty_like(u)
        _check(_conv_apply(self._h, _ptr(u, torch.float64, n, "u"), _ptr(out, torch.float64, n, "out"), _stream()),
               "convective_apply")
        return out

    def step(self, u, dt, out=None):
        """u - dt M^{-1} C(u), one explicit convective substep."""
        n = 3 * self.mesh.ndofs
        if out is None:
            out = torch.empty_like(u)
        _check(_conv_step(self._h, float(dt), _ptr(u, torch.float64, n, "u"), _ptr(out, torch.float64, n, "out"),
                          _stream()), "convective_step")
        return out

    def vjp(self, u, w, out=None):
        n = 3 * self.mesh.ndofs
        if out is None:
            out = torch.empty_like(u)
        _check(_conv_vjp(self._h, _ptr(u, torch.float64, n, "u"), _ptr(w, torch.float64, n, "w"),
                         _ptr(out, torch.float64, n, "grad"), _stream()), "convective_vjp")
        return out


class Convective(torch.autograd.Function):
    """Differentiable C(U): forward by the convective kernel, backward by the VJP kernel."""

    @staticmethod
    def forward(ctx, u, op):
        u = u.contiguous()
        ctx.save_for_backward(u)
        ctx.op = op
        return op.apply(u)

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        return ctx.op.vjp(u, g.contiguous()), None


def apply(op, x, out=None):
    """H x through the operator's apply (SIPG: fp64 or fp32 input; convective: C(x))."""
    return op.apply(x, out)


def cg(op, b, x0, **params):
    """Preconditioned CG on H x = b from x0 (updated in place); params as SipgOperator.cg."""
    return op.cg(b, x0, **params)
