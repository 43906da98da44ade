"""1D tables of the nodal tensor-product basis (oracle; test infrastructure).

Follows the paper's Sec. 3.1 ("Preliminaries": tensor-product Lagrange
polynomials on Legendre-Gauss-Lobatto nodes) and Sec. 5 ("Implementation":
Gauss quadrature with n_q = k+1 points per direction for the linear forms,
floor(3k/2)+1 for the convective term).  The reference interval is [0, 1].

Pins (tests/test_oracle_basis.py): GLL endpoints and symmetry, Gauss exactness
on monomials up to degree 2 n_q - 1, sum of weights = 1, Lagrange cardinality,
derivative exactness on polynomials, GLL quadrature weights equal the
integrals of the Lagrange polynomials.
"""
import numpy as np
from numpy.polynomial import legendre as _leg


def gll_nodes(k):
    """Legendre-Gauss-Lobatto nodes of degree k on [0, 1] (k+1 points).

    The nodes are the roots of (1 - x^2) P_k'(x) on [-1, 1] (Sec. 3.1),
    mapped affinely to [0, 1].  Interior roots come from numpy's Legendre
    root finder and are polished with Newton steps on P_k'.
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    dP = _leg.Legendre.basis(k).deriv()
    ddP = dP.deriv()
    x = np.sort(np.real(dP.roots())) if k > 1 else np.zeros(0)
    for _ in range(3):
        x = x - dP(x) / ddP(x)
    x = np.concatenate(([-1.0], x, [1.0]))
    return 0.5 * (x + 1.0)


def gauss_rule(nq):
    """Gauss-Legendre rule with nq points on [0, 1]; weights sum to 1."""
    x, w = _leg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """V[q, j] = l_j(x_q) for the Lagrange polynomials through ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                V[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return V


def lagrange_derivatives(nodes, x):
    """D[q, j] = l_j'(x_q), by differentiating the product formula term by term."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for j in range(n):
        for m in range(n):
            if m == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[m]))
            for l in range(n):
                if l != j and l != m:
                    term *= (x - nodes[l]) / (nodes[j] - nodes[l])
            D[:, j] += term
    return D


def gll_weights(k):
    """Integrals of the GLL Lagrange polynomials over [0, 1].

    Computed by an exact Gauss rule (k+1 points integrate degree k exactly),
    i.e. int l_j = sum_q w_q l_j(x_q).  Equal to the GLL quadrature weights.
    """
    x, w = gauss_rule(k + 1)
    return w @ lagrange_values(gll_nodes(k), x)


def default_conv_points(k):
    """Convective over-integration points per direction, floor(3(k+1)/2).

    The paper's Sec. 5 states floor(3k/2)+1; the benchmark configuration
    uses floor(3(k+1)/2).  On affine cells both integrate the u (x) u terms
    exactly; they differ only through the Lax-Friedrichs |u.n| factor.
    """
    return (3 * (k + 1)) // 2
