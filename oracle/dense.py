"""Dense direct-quadrature reference of the same scalar operator (oracle).

D_ij = sum_p sum_q (A_i/3)(A_j/3) G_d(k, |r_ip - r_jq|)
       + A_s,NR[i, j]                                  if (i, j) is near,
       + sum_p sum_q (A_i/3)(A_j/3) G_s(|r_ip - r_jq|)  otherwise.

This is the Galerkin matrix with the kernel split of eq. hgfdecomp0: the
singular static part integrated directly where it matters (the near region)
and the smooth dynamic part G_d (eq. hgfd, with G_d(0) = -jk/(4 pi) from
eq. hgfdtaylor) by the 3 x 3 point rule everywhere.  It measures the
approximation error of the grid-accelerated operator (the "direct" matrix of
Sec. IV-B); it is not the parity target of the GPU path.
"""
from __future__ import annotations

import numpy as np

from . import mesh as _mesh
from .green import green_dynamic, green_static


def dense_rows(V, T, k: float, rows, near_static) -> np.ndarray:
    """Rows of D as a dense array [len(rows), N].

    ``near_static`` is a scipy.sparse matrix holding A_s,NR on the near list.
    """
    qp = _mesh.quad_points(V, T)                  # [N, 3, 3]
    w = _mesh.quad_weights(V, T)                  # [N, 3]
    rows = np.asarray(rows, dtype=np.int64)
    N = T.shape[0]
    out = np.zeros((rows.size, N), dtype=np.complex128)
    ns = near_static.tocsr()
    for t, i in enumerate(rows):
        d = qp[i][:, None, None, :] - qp[None, :, :, :]
        # d: [3 (p of i), N, 3 (q of j), 3 xyz]
        R = np.linalg.norm(d, axis=-1)
        ww = w[i][:, None, None] * w[None, :, :]
        dyn = np.sum(ww * green_dynamic(k, R), axis=(0, 2))
        with np.errstate(divide="ignore"):
            st = np.sum(ww * np.where(R > 0, green_static(np.where(R > 0, R, 1.0)), 0.0),
                        axis=(0, 2))
        row = ns.getrow(int(i))
        st[row.indices] = row.data
        out[t] = dyn + st
    return out


def dense_matvec(V, T, k: float, x, near_static, rows=None) -> np.ndarray:
    """(D x) on all rows, or on ``rows`` only."""
    N = T.shape[0]
    rows = np.arange(N) if rows is None else np.asarray(rows)
    x = np.asarray(x, dtype=np.complex128)
    y = np.empty(rows.size, dtype=np.complex128)
    chunk = 64
    for s in range(0, rows.size, chunk):
        y[s:s + chunk] = dense_rows(V, T, k, rows[s:s + chunk], near_static) @ x
    return y


def cluster_block(V, T, k: float, members, near_static) -> np.ndarray:
    """The block of D over a set of triangles (rows and columns ``members``):
    the near-region/block preconditioner of Sec. III-A built from the full
    kernel, i.e. the static near entries with the dynamic part added."""
    members = np.asarray(members, dtype=np.int64)
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    d = qp[members][:, None, :, None, :] - qp[members][None, :, None, :, :]
    R = np.linalg.norm(d, axis=-1)                        # [m, m, 3, 3]
    ww = w[members][:, None, :, None] * w[members][None, :, None, :]
    dyn = np.sum(ww * green_dynamic(k, R), axis=(2, 3))
    with np.errstate(divide="ignore"):
        st = np.sum(ww * np.where(R > 0, green_static(np.where(R > 0, R, 1.0)), 0.0),
                    axis=(2, 3))
    ns = near_static.tocsr()
    for a, i in enumerate(members):
        row = ns.getrow(int(i))
        pos = {int(c): v for c, v in zip(row.indices, row.data)}
        for b, j in enumerate(members):
            if int(j) in pos:
                st[a, b] = pos[int(j)]
    return dyn + st


def nearblock_apply(V, T, k: float, clusters, near_static, x) -> np.ndarray:
    """z = B^{-1} x with B block diagonal over ``clusters`` (lists of
    triangle indices), each block the cluster_block."""
    x = np.asarray(x, dtype=np.complex128)
    z = np.zeros_like(x)
    for members in clusters:
        B = cluster_block(V, T, k, members, near_static)
        z[..., members] = np.linalg.solve(B, x[..., members].T).T
    return z


def self_lin_correction(V, T, k: float) -> np.ndarray:
    """Change of the dense reference's self entries when their linear
    dynamic term k^2 G_lin = -k^2 R/(8 pi) (eq. linterm) is integrated
    directly (closed-form inner integral) instead of by the 3 x 3 point rule
    (the accuracy modification of Sec. III-A): per triangle,
    k^2 (A_lin[i, i] - sum_p sum_q (A_i/3)^2 G_lin(|r_ip - r_iq|))."""
    from .lin import lin_self
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    R = np.linalg.norm(qp[:, :, None, :] - qp[:, None, :, :], axis=-1)   # [N, 3, 3]
    rule = np.sum(w[:, :, None] * w[:, None, :] * (-R / (8.0 * np.pi)), axis=(1, 2))
    return (k * k) * (lin_self(V, T) - rule)
