"""Krylov solvers (oracle): restarted right-preconditioned FGMRES and
mixed-precision-style iterative refinement.

The paper solves its AIMx systems with restarted GMRES to a relative
residual of 1e-4 (Sec. V, results set-up) using diagonal preconditioners
built from the static near-field matrix (Sec. III-A, "Preconditioning").
This is the textbook algorithm (Saad & Schultz 1986; flexible variant,
Saad 1993): Arnoldi with modified Gram-Schmidt in complex128, Givens
rotations on the Hessenberg matrix, right preconditioning z = M(v) with the
preconditioned vectors kept (so M may change between iterations), zero
initial guess unless given, and the stopping test applied to the true
residual ||b - A x|| / ||b|| at every restart.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SolveInfo:
    converged: bool = False
    iters: int = 0
    matvecs: int = 0
    rel_resid: float = np.inf
    history: list = field(default_factory=list)
    breakdown: bool = False
    fallback_used: bool = False


def fgmres(A, b, tol: float = 1e-6, restart: int = 30, max_iter: int = 1000,
           M=None, x0=None):
    """Solve A x = b.  ``A`` and ``M`` are callables on complex128 vectors
    (``M`` defaults to the identity)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    M = (lambda v: v) if M is None else M
    info = SolveInfo()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        info.converged, info.rel_resid = True, 0.0
        return np.zeros(n, dtype=np.complex128), info
    while info.iters < max_iter:
        r = b - A(x)
        info.matvecs += 1
        beta = np.linalg.norm(r)
        info.rel_resid = beta / bnorm
        info.history.append(info.rel_resid)
        if not np.isfinite(beta):
            info.breakdown = True
            return x, info
        if info.rel_resid <= tol:
            info.converged = True
            return x, info
        m = min(restart, max_iter - info.iters)
        Vb = np.zeros((m + 1, n), dtype=np.complex128)
        Z = np.zeros((m, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        Vb[0] = r / beta
        used = 0
        for j in range(m):
            Z[j] = M(Vb[j])
            w = A(Z[j])
            info.matvecs += 1
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.vdot(Vb[i], w)
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = np.linalg.norm(w)
            if not np.all(np.isfinite(H[:j + 2, j])):    # e.g. a non-finite M(v)
                info.breakdown = True
                break
            for i in range(j):                           # earlier rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0.0:
                info.breakdown = True
                break
            if a == 0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            used = j + 1
            info.iters += 1
            info.history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or H[j, j] == 0:
                break
            Vb[j + 1] = w / (np.linalg.norm(w) if np.linalg.norm(w) > 0 else 1.0)
        if used:
            y = np.linalg.solve(np.triu(H[:used, :used]), g[:used])
            x = x + Z[:used].T @ y
        if info.breakdown:
            break
    r = b - A(x)
    info.matvecs += 1
    info.rel_resid = np.linalg.norm(r) / bnorm
    info.converged = info.rel_resid <= tol
    return x, info


def iterative_refinement(A_hi, inner_solve, b, tol: float, max_refine: int = 20):
    """x <- x + inner_solve(b - A_hi x) until ||b - A_hi x|| <= tol ||b||."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    hist = []
    for it in range(max_refine + 1):
        r = b - A_hi(x)
        rel = np.linalg.norm(r) / bnorm
        hist.append(rel)
        if rel <= tol or it == max_refine:
            return x, rel <= tol, hist
        x = x + inner_solve(r)
    return x, False, hist


def gated_fgmres(A, b, M, M_fallback=None, gate: float = 0.7, tol: float = 1e-6,
                 restart: int = 30, max_iter: int = 1000):
    """FGMRES with a gate on an untrusted (learned) preconditioner ``M``.

    Restart cycles run with ``M``.  After every cycle the true relative
    residual must have fallen below ``gate`` times its value at the start of
    the cycle (or below ``tol``); if it has not, or a value is not finite,
    the rest of the solve runs with ``M_fallback`` (identity if None) from
    the last finite iterate, and ``info.fallback_used`` is set."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    rel = 1.0 if bnorm > 0 else 0.0
    total = SolveInfo()
    switch = False
    while total.iters < max_iter and rel > tol:
        xn, info = fgmres(A, b, tol=tol, restart=restart,
                          max_iter=min(restart, max_iter - total.iters), M=M, x0=x)
        total.iters += info.iters
        total.matvecs += info.matvecs
        total.history += info.history
        if info.breakdown or not np.isfinite(info.rel_resid) or not np.all(np.isfinite(xn)):
            switch = True
            break
        x = xn
        if info.rel_resid > tol and info.rel_resid > gate * rel:
            rel = info.rel_resid
            switch = True
            break
        rel = info.rel_resid
    if switch:
        total.fallback_used = True
        x, info = fgmres(A, b, tol=tol, restart=restart,
                         max_iter=max(1, max_iter - total.iters), M=M_fallback, x0=x)
        total.iters += info.iters
        total.matvecs += info.matvecs
        total.history += info.history
        rel = info.rel_resid
    total.rel_resid = float(np.linalg.norm(b - A(x)) / bnorm) if bnorm > 0 else 0.0
    total.converged = total.rel_resid <= tol
    return x, total
