"""1D quadrature rules and tensor-product Lagrange polynomials (oracle).

Sec. 3 (algorithmic developments) of the paper: Gaussian quadrature with k+1
points per direction; Lagrange bases with nodes in the Gauss (G) or the
Gauss-Lobatto (GL) points; Sec. 3.1 (face integrals) motivates GL nodes.
Everything here is evaluated directly from the defining formulas.
"""
from __future__ import annotations

import itertools

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss(n: int):
    """n-point Gauss-Legendre rule on [0,1] (points ascending, weights sum to 1)."""
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto(n: int):
    """n-point Gauss-Lobatto rule on [0,1]: endpoints plus the roots of P'_{n-1}.

    Weights 2 / (n (n-1) P_{n-1}(x)^2) on [-1,1], halved for [0,1].  The
    interior roots from the companion matrix are polished by Newton steps on
    P'_{n-1}.
    """
    if n < 2:
        raise ValueError("Gauss-Lobatto needs n >= 2")
    m = n - 1
    cm = np.zeros(m + 1)
    cm[m] = 1.0  # P_m in Legendre coefficients
    dcm = npleg.legder(cm)
    ddcm = npleg.legder(dcm)
    interior = np.sort(np.real(npleg.legroots(dcm))) if m >= 2 else np.array([])
    for _ in range(3):
        interior = interior - npleg.legval(interior, dcm) / npleg.legval(interior, ddcm)
    x = np.concatenate(([-1.0], interior, [1.0]))
    w = 2.0 / (n * (n - 1) * npleg.legval(x, cm) ** 2)
    return 0.5 * (x + 1.0), 0.5 * w


def equispaced(q: int):
    """The q+1 equispaced points j/q of [0,1] (nodes of the geometry map)."""
    return np.arange(q + 1, dtype=np.float64) / q


def lagrange(nodes, x):
    """Matrix L[i, j] = l_j(x_i) of the Lagrange polynomials on `nodes` (product formula)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                out[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return out


def lagrange_deriv(nodes, x):
    """Matrix L'[i, j] = l_j'(x_i): sum over m of the products with factor m differentiated."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(x), n))
    for j in range(n):
        for m in range(n):
            if m == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[m]))
            for l in range(n):
                if l != j and l != m:
                    term = term * (x - nodes[l]) / (nodes[j] - nodes[l])
            out[:, j] += term
    return out


def multi_indices(n: int, dim: int):
    """Lexicographic multi-indices (x fastest) of an n^dim tensor grid, int[n^dim][dim]."""
    idx = np.array(list(itertools.product(range(n), repeat=dim)), dtype=np.int64)
    return idx[:, ::-1].copy()  # itertools varies the last entry fastest


def tensor_points(pts1d, dim: int):
    """Tensor grid of 1D points, float64[n^dim][dim], lexicographic x fastest."""
    pts1d = np.asarray(pts1d, dtype=np.float64)
    mi = multi_indices(len(pts1d), dim)
    return pts1d[mi]


def tensor_weights(w1d, dim: int):
    w1d = np.asarray(w1d, dtype=np.float64)
    mi = multi_indices(len(w1d), dim)
    return np.prod(w1d[mi], axis=1)


def tensor_basis(nodes1d, points):
    """Phi[q, i] = prod_a l_{i_a}(points[q, a]): d-dimensional Lagrange polynomials
    on the tensor grid of `nodes1d`, evaluated directly at arbitrary points."""
    points = np.atleast_2d(points)
    dim = points.shape[1]
    n = len(nodes1d)
    mi = multi_indices(n, dim)
    per_dir = [lagrange(nodes1d, points[:, a]) for a in range(dim)]  # [a] -> [Q][n]
    out = np.ones((points.shape[0], len(mi)))
    for a in range(dim):
        out *= per_dir[a][:, mi[:, a]]
    return out


def tensor_basis_grad(nodes1d, points):
    """dPhi[b][q, i] = d/dxi_b of the d-dimensional Lagrange polynomial i at points[q]."""
    points = np.atleast_2d(points)
    dim = points.shape[1]
    n = len(nodes1d)
    mi = multi_indices(n, dim)
    val = [lagrange(nodes1d, points[:, a]) for a in range(dim)]
    der = [lagrange_deriv(nodes1d, points[:, a]) for a in range(dim)]
    grads = []
    for b in range(dim):
        g = np.ones((points.shape[0], len(mi)))
        for a in range(dim):
            g *= (der[a] if a == b else val[a])[:, mi[:, a]]
        grads.append(g)
    return grads
