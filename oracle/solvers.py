"""Textbook iterative solvers (oracle; test infrastructure).

Sec. 5.1 of the paper: the linear systems are solved by preconditioned
conjugate gradients with matrix-free products; the Poisson preconditioner is
built on a Chebyshev polynomial smoother that needs only the operator and its
diagonal, with eigenvalue estimates from an initial Krylov run; singular
(all-Neumann / periodic) Poisson problems are solved on the zero-mean
subspace by projecting the right-hand side and the operator product.

Readings fixed here (and used identically by the GPU path):
* convergence when ||r_k||_2 <= rtol * ||b||_2 on the recursive residual,
  with b already projected in the singular case;
* Chebyshev preconditioner = the Chebyshev acceleration of point-Jacobi
  (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 12.1)
  started from zero on the interval [lambda/range, lambda], with a degree-m
  error polynomial (m-1 operator products);
* eigenvalue estimate = Lanczos without re-orthogonalisation on
  D^{-1/2} A D^{-1/2}; lambda = safety * largest Ritz value.
"""
import numpy as np

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE = 0, 4, 5, 6


def pcg(apply, b, x0, precond, rtol, max_iter, project_mean=False, record=None, flexible=False):
    """Preconditioned CG (Hestenes-Stiefel form with Fletcher-Reeves beta).

    flexible=True uses beta = <z_new, r_new - r_old>/<z_old, r_old> (Polak-Ribiere,
    the flexible CG of Notay, SIAM J. Sci. Comput. 22, 2000).

    Returns (x, iterations, status, rel_residual).  ``record`` (a list) gets
    the iterate after every iteration when given.
    """
    b = np.array(b, dtype=np.float64)
    if project_mean:
        b = b - b.mean()
    x = np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if not np.isfinite(bnorm) or not np.all(np.isfinite(x)):
        return x, 0, NONFINITE, np.nan
    Ax = apply(x)
    if project_mean:
        Ax = Ax - Ax.mean()
    r = b - Ax
    tol = rtol * bnorm
    rnorm = np.linalg.norm(r)
    if rnorm <= tol:
        return x, 0, OK, rnorm / bnorm if bnorm > 0 else 0.0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, max_iter + 1):
        if not rz > 0:
            return x, it - 1, (NONFINITE if not np.isfinite(rz) else BREAKDOWN), rnorm / bnorm
        q = apply(p)
        if project_mean:
            q = q - q.mean()
        pq = p @ q
        if not pq > 0:
            return x, it - 1, (NONFINITE if not np.isfinite(pq) else BREAKDOWN), rnorm / bnorm
        alpha = rz / pq
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        rnorm = np.sqrt(r @ r)
        if record is not None:
            record.append(x.copy())
        if not np.isfinite(rnorm):
            return x, it, NONFINITE, np.nan
        if rnorm <= tol:
            return x, it, OK, rnorm / bnorm
        z = precond(r)
        rz_new = r @ z
        beta = (z @ (r - r_old)) / rz if flexible else rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, max_iter, NOT_CONVERGED, rnorm / bnorm


def lanczos_ritz(apply_sym, v0, steps):
    """Ritz values of ``steps`` Lanczos steps (no re-orthogonalisation)."""
    v = v0 / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    for j in range(steps):
        w = apply_sym(v) - beta * v_prev
        alpha = w @ v
        w = w - alpha * v
        alphas.append(alpha)
        beta = np.linalg.norm(w)
        if j < steps - 1:
            betas.append(beta)
            if beta == 0.0:
                break
            v_prev, v = v, w / beta
    m = len(alphas)
    T = np.diag(alphas) + np.diag(betas[:m - 1], 1) + np.diag(betas[:m - 1], -1)
    return np.linalg.eigvalsh(T), T


def chebyshev_jacobi(apply, dinv, r, lam_max, smoothing_range, degree):
    """z = q(D^{-1}A) D^{-1} r: Chebyshev acceleration of Jacobi from z = 0.

    The error after the iteration is T_m((theta - lam)/delta)/T_m(theta/delta)
    times the initial error on [a, b] = [lam_max/range, lam_max],
    theta = (a+b)/2, delta = (b-a)/2, m = degree; m-1 operator products.
    """
    a = lam_max / smoothing_range
    bnd = lam_max
    theta, delta = 0.5 * (bnd + a), 0.5 * (bnd - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    res = np.array(r, dtype=np.float64)
    d = (dinv * res) / theta
    z = d.copy()
    for _ in range(1, degree):
        res = res - apply(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * res)
        z = z + d
        rho = rho_new
    return z


def chebyshev_polynomial_value(lam, lam_max, smoothing_range, degree):
    """Closed form q(lam) = (1 - T_m((theta-lam)/delta)/T_m(theta/delta)) / lam."""
    from numpy.polynomial import chebyshev as C
    a = lam_max / smoothing_range
    theta, delta = 0.5 * (lam_max + a), 0.5 * (lam_max - a)
    Tm = C.Chebyshev.basis(degree)
    return (1.0 - Tm((theta - lam) / delta) / Tm(theta / delta)) / lam
