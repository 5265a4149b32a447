"""Modified block BiCGSTAB (Alg. 1 and Alg. 2 of the paper) and its pieces.

Blocks are complex128 arrays of shape (N, L); `A` and `M` are callables
mapping such a block to one of the same shape.  Inner products are
<a, b> = sum conj(a_n) b_n; ||.|| is the Euclidean norm of a column.

Readings where the printed algorithm is silent or garbled:
* the loop runs while max_i ||r_i|| / ||b_i|| > eps (the printed "<=" is a
  typesetting slip; the paper's own prose stops once the ratio is <= eps);
* X starts at 0 unless a guess is given; R~ = R_0 unless given;
* zeta is one complex scalar shared by all columns;
* after the recursive residual converges, the true residual B - A X is
  checked; if it is above eps the iteration restarts from R = B - A X, P = R,
  keeping R~, at most `max_restarts` times.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg


def mgs(P: np.ndarray):
    """Modified Gram-Schmidt QR, P = Q gamma (gamma upper triangular, real
    positive diagonal).  The paper uses MGS for step 4.1 (Sec. 2.1)."""
    Q = np.array(P, dtype=np.complex128, copy=True)
    L = Q.shape[1]
    g = np.zeros((L, L), dtype=np.complex128)
    for j in range(L):
        g[j, j] = np.linalg.norm(Q[:, j])
        Q[:, j] /= g[j, j]
        for k in range(j + 1, L):
            g[j, k] = np.vdot(Q[:, j], Q[:, k])
            Q[:, k] -= g[j, k] * Q[:, j]
    return Q, g


def col_norms(X: np.ndarray) -> np.ndarray:
    return np.sqrt(np.sum(np.abs(X) ** 2, axis=0))


@dataclass
class SolveResult:
    X: np.ndarray
    iterations: int
    restarts: int
    true_res: np.ndarray
    rec_res: np.ndarray
    converged: bool
    history: list = field(default_factory=list)        # max rec. residual per iteration
    true_history: list = field(default_factory=list)   # max true residual (if tracked)
    n_A: int = 0
    n_M: int = 0


def _lu_solve(G: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """LU with partial pivoting (LAPACK getrf/getrs)."""
    return scipy.linalg.lu_solve(scipy.linalg.lu_factor(G), rhs)


def block_bicgstab(A, M, B, tol, maxiter=1000, X0=None, Rt=None, qr=True,
                   max_restarts=3, track_true=False, invariants=None):
    """Alg. 1: modified (QR-stabilised) block BiCGSTAB, right preconditioned.

    Steps per iteration (numbering as in Alg. 1):
      4.1 P = Q gamma, P <- Q       4.2 U = M P        4.3 V = A U
      4.4 (R~^H V) alpha = R~^H R   4.5 T = R - V alpha
      4.6 S = M T                   4.7 Z = A S
      4.8 zeta = Tr(Z^H T) / Tr(Z^H Z)
      4.9 X <- X + U alpha + zeta S 4.10 R = T - zeta Z
      4.11 (R~^H V) beta = -R~^H Z  4.12 P <- R + (P - zeta V) beta
    """
    B = np.asarray(B, dtype=np.complex128)
    bn = col_norms(B)
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.complex128)
    R = B - A(X)
    nA, nM = 1, 0
    P = R.copy()
    Rt = R.copy() if Rt is None else np.asarray(Rt, dtype=np.complex128)
    it, restarts = 0, 0
    hist, thist = [], []
    while True:
        while np.max(col_norms(R) / bn) > tol and it < maxiter:
            if qr:
                P, _ = mgs(P)                                  # 4.1
            U = M(P)                                           # 4.2
            V = A(U)                                           # 4.3
            RtV = Rt.conj().T @ V
            alpha = _lu_solve(RtV, Rt.conj().T @ R)            # 4.4
            T = R - V @ alpha                                  # 4.5
            S = M(T)                                           # 4.6
            Z = A(S)                                           # 4.7
            zeta = np.vdot(Z, T) / np.vdot(Z, Z)               # 4.8 (Tr Z^H T / Tr Z^H Z)
            X = X + U @ alpha + zeta * S                       # 4.9
            Rn = T - zeta * Z                                  # 4.10
            beta = _lu_solve(RtV, -(Rt.conj().T @ Z))          # 4.11
            P = Rn + (P - zeta * V) @ beta                     # 4.12
            if invariants is not None:
                invariants.append({"RtT": Rt.conj().T @ T, "ZR": np.vdot(Z, Rn),
                                   "scale": (np.linalg.norm(Rt) * np.linalg.norm(T),
                                             np.linalg.norm(Z) * np.linalg.norm(Rn))})
            R = Rn
            nA += 2
            nM += 2
            it += 1
            hist.append(float(np.max(col_norms(R) / bn)))
            if track_true:
                thist.append(float(np.max(col_norms(B - A(X)) / bn)))
        true = col_norms(B - A(X)) / bn
        nA += 1
        if np.max(true) <= tol or restarts >= max_restarts or it >= maxiter:
            break
        restarts += 1
        R = B - A(X)
        nA += 1
        P = R.copy()
    rec = col_norms(R) / bn
    return SolveResult(X, it, restarts, true, rec, bool(np.max(true) <= tol),
                       hist, thist, nA, nM)


def block_bicgstab_memsave(A, M, B, tol, maxiter=1000, X0=None, Rt=None,
                           max_restarts=3):
    """Alg. 2: the memory-saving form (T stored in R, X updated in two parts).

      4.1 QR   4.2 U = M P   4.3 V = A U   4.4 alpha   4.5 R <- R - V alpha
      4.6 X <- X + U alpha   4.7 S = M R   4.8 Z = A S
      4.9 zeta = Tr(Z^H R) / Tr(Z^H Z)   4.10 X <- X + zeta S
      4.11 R <- R - zeta Z   4.12 beta from -R~^H Z   4.13 P <- R + (P - zeta V) beta
    """
    B = np.asarray(B, dtype=np.complex128)
    bn = col_norms(B)
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.complex128)
    R = B - A(X)
    P = R.copy()
    Rt = R.copy() if Rt is None else np.asarray(Rt, dtype=np.complex128)
    it, restarts, hist = 0, 0, []
    while True:
        while np.max(col_norms(R) / bn) > tol and it < maxiter:
            P, _ = mgs(P)
            U = M(P)
            V = A(U)
            RtV = Rt.conj().T @ V
            alpha = _lu_solve(RtV, Rt.conj().T @ R)
            R = R - V @ alpha
            X = X + U @ alpha
            S = M(R)
            Z = A(S)
            zeta = np.vdot(Z, R) / np.vdot(Z, Z)
            X = X + zeta * S
            R = R - zeta * Z
            beta = _lu_solve(RtV, -(Rt.conj().T @ Z))
            P = R + (P - zeta * V) @ beta
            it += 1
            hist.append(float(np.max(col_norms(R) / bn)))
        true = col_norms(B - A(X)) / bn
        if np.max(true) <= tol or restarts >= max_restarts or it >= maxiter:
            break
        restarts += 1
        R = B - A(X)
        P = R.copy()
    return SolveResult(X, it, restarts, true, col_norms(R) / bn,
                       bool(np.max(true) <= tol), hist)


def bicgstab(A, M, b, tol, maxiter=1000, x0=None, rt=None):
    """Textbook right-preconditioned BiCGSTAB (van der Vorst 1992), one RHS.

    Written in the usual rho/alpha/omega recurrences, independently of the
    block algorithm; used to check that the block method with L = 1 reduces
    to it.  Returns (x, residual-norm history relative to ||b||).
    """
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128).reshape(-1)
    r = b - A(x[:, None])[:, 0]
    rt = r.copy() if rt is None else np.asarray(rt).reshape(-1)
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    bn = np.linalg.norm(b)
    hist = []
    for _ in range(maxiter):
        if np.linalg.norm(r) / bn <= tol:
            break
        rho = np.vdot(rt, r)
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = M(p[:, None])[:, 0]
        v = A(ph[:, None])[:, 0]
        alpha = rho / np.vdot(rt, v)
        s = r - alpha * v
        sh = M(s[:, None])[:, 0]
        t = A(sh[:, None])[:, 0]
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho_old = rho
        hist.append(float(np.linalg.norm(r) / bn))
    return x, hist
