"""Triangle geometry and the 3-point quadrature rule (oracle).

The discretisation of Sec. II-A uses a flat-triangle surface mesh.  The
scalar operator here uses one piecewise-constant basis function per triangle
and Galerkin testing.  Integrals over a triangle use the symmetric 3-point
rule with interior points at barycentric (2/3, 1/6, 1/6) and its
permutations, each of weight area/3; it integrates every polynomial of total
degree <= 2 exactly.
"""
from __future__ import annotations

import numpy as np

BARY = np.array([[2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0],
                 [1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0],
                 [1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0]])


def areas(V, T):
    """Triangle areas |(b - a) x (c - a)| / 2."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)


def unit_normals(V, T):
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, c - a)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def centroids(V, T):
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    return (a + b + c) / 3.0


def quad_points(V, T):
    """Quadrature points, shape [N, 3, 3] (triangle, point, xyz).

    Point q of triangle j is a*w0 + b*w1 + c*w2 with (w0, w1, w2) the q-th
    row of BARY, summed left to right.
    """
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    out = np.empty((T.shape[0], 3, 3))
    for q in range(3):
        w0, w1, w2 = BARY[q]
        out[:, q, :] = a * w0 + b * w1 + c * w2
    return out


def quad_weights(V, T):
    """Quadrature weights, shape [N, 3]: area / 3 for every point."""
    A = areas(V, T)
    return np.repeat((A / 3.0)[:, None], 3, axis=1)
