"""Block Krylov-Schur for a symmetric matrix, FP64 (oracle).

The paper's generic eigen-iteration (its eigensolver algorithm: update the
subspace, solve the projected problem, form Ritz pairs and residuals, test
convergence) with the block extension (b vectors per step, subspace m = b*NB,
so the sparse product is an SpMM).  The specific solver is the block
Krylov-Schur method the paper selects; the paper only cites it, so the steps
below are Stewart's Krylov-Schur specialised to symmetric A (a block
thick-restart Lanczos with full reorthogonalisation).  The readings the paper
does not fix are marked "reading".

State: V (n x k, orthonormal), Q (n x b, orthonormal, Q orthogonal to V),
T (k x k symmetric), B (b x k) with  A V = V T + Q B.

Expand (while k < m):
  V <- [V, Q];  W = A Q                          (sparse product)
  C = CGS2(V, W)                                  (reorthogonalisation: classical
                                                   Gram-Schmidt applied twice)
  W = Q' R                                        (block QR: CholQR2, falling back
                                                   to column-wise CGS2 with random
                                                   refill of dependent columns)
  T[:, new] = C, T[new, :] = C^T;  B = [0 .. 0, R];  Q <- Q'
Rayleigh-Ritz: S = (T + T^T)/2 = Y diag(theta) Y^T, ordered by |theta|
  descending, ties to larger theta (reading: largest magnitude).
Converged: rho_i = ||B y_i||_2 <= tol * max(eps^(2/3), |theta_i|) for i < nev,
  eps the FP64 unit roundoff (reading: ARPACK's convention, relative to the
  Ritz value except for Ritz values near zero).
Restart: keep p = m - b*max(1, floor((m - nev)/(2b))) Ritz vectors (reading):
  V <- V Y[:, :p], T <- diag(theta_1..p), B <- B Y[:, :p], k = p.
Final check: X = V Y[:, :nev], explicit residual
  ||A x_i - theta_i x_i|| / (max(eps^(2/3), |theta_i|) ||x_i||).

Block QR thresholds (reading; the paper does not describe breakdown):
  eta (refill): column j of the new block is dependent when its norm after
  projection against V and the earlier accepted columns is <= eta times its
  norm before projection, or is not finite.  A refill discards that residual
  part, so A V = V T + Q B then holds only up to eta ||A q_j|| <= eta ||A||
  per refilled column, an error the estimates rho do not see (the explicit
  residuals of the final check do).  eta = 1e-10 keeps it far below every
  tolerance used; exact breakdowns (invariant subspaces of closed-form
  graphs) give ratios near the unit roundoff.
  eta_chol (factorisation): Cholesky QR twice is stable only while the
  block's condition number stays well below u^(-1/2) (Yamamoto, Nakatsukasa,
  Yanagisawa and Fukaya, 2015); when some column-wise ratio is below
  eta_chol = 1e-6 the column-wise Gram-Schmidt factors are kept instead.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .rng import refill_column


EPS23 = np.finfo(np.float64).eps ** (2.0 / 3.0)


def ritz_scale(theta: np.ndarray) -> np.ndarray:
    """Denominator of the convergence test and of the reported residuals."""
    return np.maximum(np.abs(theta), EPS23)


def restart_keep(m: int, b: int, nev: int) -> int:
    """Number of Ritz vectors kept at a restart (reading; keeps m - p a multiple of b)."""
    return m - b * max(1, (m - nev) // (2 * b))


@dataclass
class KSResult:
    evals: np.ndarray
    evecs: np.ndarray
    resid: np.ndarray          # explicit ||A x - theta x|| / |theta| per pair
    rho: np.ndarray            # Krylov-Schur residual estimates at the last check
    restarts: int
    spmm_calls: int            # width-b products during the iteration
    converged: bool
    refills: int = 0
    history: list = field(default_factory=list)


def _cgs2(Vk: np.ndarray, W: np.ndarray):
    """Classical Gram-Schmidt twice: W <- (I - Vk Vk^T)^2 W, returns C = C1 + C2."""
    C1 = Vk.T @ W
    W -= Vk @ C1
    C2 = Vk.T @ W
    W -= Vk @ C2
    return C1 + C2


def _chol_upper(G: np.ndarray):
    L = np.linalg.cholesky(G)  # raises LinAlgError if G is not positive definite
    return L.T


def _columnwise(W: np.ndarray, nb: np.ndarray, eta: float):
    """Column-wise CGS2 of W in column order (W already projected against V).

    Column j is dependent when its norm after projection against the earlier
    accepted columns is not above eta * nb[j] (nb = norm before any
    projection), which includes a non-finite column.
    Returns Q (dependent columns zero), R (dependent rows zero), accepted,
    dependent, and the ratio norm-after / norm-before of every column.
    """
    n, b = W.shape
    Q = np.zeros_like(W)
    R = np.zeros((b, b))
    acc, dep = [], []
    ratio = np.zeros(b)
    for j in range(b):
        w = W[:, j].copy()
        if acc:
            Qa = Q[:, acc]
            c1 = Qa.T @ w
            w -= Qa @ c1
            c2 = Qa.T @ w
            w -= Qa @ c2
            R[acc, j] = c1 + c2
        nw = np.sqrt(w @ w)
        ratio[j] = nw / nb[j] if nb[j] > 0 else 0.0
        if not (nw > eta * nb[j]) or nw == 0.0:
            dep.append(j)
        else:
            Q[:, j] = w / nw
            R[j, j] = nw
            acc.append(j)
    return Q, R, acc, dep, ratio


def _block_qr(Vk: np.ndarray, W: np.ndarray, nb: np.ndarray, eta: float, seed: int, step: int,
              eta_chol: float = 1e-6):
    """Orthonormalise W (already projected against Vk).  Returns Q, R, refill count.

    Dependence is decided column by column (reading).  With no dependent
    column and every column-wise ratio >= eta_chol the factorisation is
    CholQR2: R1 = chol(W^T W), W <- W R1^-1, R2 = chol(W^T W), Q = W R2^-1,
    R = R2 R1.  Otherwise the column-wise result is kept; each dependent
    column has R[j, :] = 0 and is replaced, after all independent columns are
    fixed and in column order, by a random vector orthogonalised (twice)
    against Vk and every column defined so far.
    """
    n, b = W.shape
    Qc, Rc, acc, dep, ratio = _columnwise(W, nb, eta)
    if not dep and ratio.min() < eta_chol:
        return Qc, Rc, 0
    if not dep:
        try:
            R1 = _chol_upper(W.T @ W)
            W1 = np.linalg.solve(R1.T, W.T).T  # W R1^-1
            R2 = _chol_upper(W1.T @ W1)
            Q = np.linalg.solve(R2.T, W1.T).T
            return Q, R2 @ R1, 0
        except np.linalg.LinAlgError:
            return Qc, Rc, 0
    Q, R = Qc, Rc
    for j in dep:
        r = refill_column(n, j, step, seed)
        basis = np.concatenate([Vk, Q[:, acc]], axis=1)
        if basis.shape[1]:
            r -= basis @ (basis.T @ r)
            r -= basis @ (basis.T @ r)
        Q[:, j] = r / np.sqrt(r @ r)
        acc.append(j)
    return Q, R, len(dep)


def _ritz_order(theta: np.ndarray) -> np.ndarray:
    # primary key |theta| descending, secondary theta descending
    return np.lexsort((-theta, -np.abs(theta)))


def krylov_schur(spmm, n: int, nev: int, b: int, m: int, tol: float, X0: np.ndarray,
                 max_restarts: int = 500, seed: int = 0, eta: float = 1e-10,
                 eta_chol: float = 1e-6, keep: int = 0) -> KSResult:
    """spmm(X) must return A @ X for an (n, cols) float64 array.  keep: Ritz
    vectors kept at a restart (0: restart_keep(m, b, nev)); a multiple of b
    away from m, at least nev."""
    if m % b or nev > m - b or nev < 1 or tol <= 0 or m + b > n:
        raise ValueError("need m % b == 0, 1 <= nev <= m - b, tol > 0, m + b <= n")
    if keep and (keep < nev or keep > m - b or (m - keep) % b):
        raise ValueError("need nev <= keep <= m - b and (m - keep) % b == 0")
    V = np.zeros((n, m), order="F")
    T = np.zeros((m, m))
    Bk = np.zeros((b, m))
    X0 = np.array(X0, dtype=np.float64, copy=True)
    Q, _, refills = _block_qr(np.zeros((n, 0)), X0, np.sqrt(np.sum(X0 * X0, axis=0)), eta,
                              seed, 0, eta_chol)
    k = 0
    step = 0
    spmm_calls = 0
    restarts = 0
    history = []
    while True:
        while k < m:
            V[:, k:k + b] = Q
            k += b
            W = np.array(spmm(np.ascontiguousarray(Q)), dtype=np.float64)
            spmm_calls += 1
            step += 1
            Vk = V[:, :k]
            nb = np.sqrt(np.sum(W * W, axis=0))
            C = _cgs2(Vk, W)
            Q, R, nref = _block_qr(Vk, W, nb, eta, seed, step, eta_chol)
            refills += nref
            T[:k, k - b:k] = C
            T[k - b:k, :k] = C.T
            Bk = np.zeros((b, m))
            Bk[:, k - b:k] = R
        S = 0.5 * (T + T.T)
        theta, Y = np.linalg.eigh(S)
        order = _ritz_order(theta)
        theta, Y = theta[order], Y[:, order]
        rho = np.sqrt(np.sum((Bk @ Y) ** 2, axis=0))
        scale = ritz_scale(theta)
        conv = rho[:nev] <= tol * scale[:nev]
        history.append((restarts, spmm_calls, float(np.max(rho[:nev] / scale[:nev]))))
        if conv.all() or restarts >= max_restarts:
            break
        p = keep if keep else restart_keep(m, b, nev)
        V[:, :p] = V @ Y[:, :p]
        T = np.zeros((m, m))
        T[np.arange(p), np.arange(p)] = theta[:p]
        Bp = np.zeros((b, m))
        Bp[:, :p] = Bk @ Y[:, :p]
        Bk = Bp
        k = p
        restarts += 1
    X = V @ Y[:, :nev]
    AX = np.asarray(spmm(np.ascontiguousarray(X)), dtype=np.float64)
    Rres = AX - X * theta[:nev]
    resid = np.sqrt(np.sum(Rres * Rres, axis=0)) / (ritz_scale(theta[:nev]) *
                                                     np.sqrt(np.sum(X * X, axis=0)))
    return KSResult(evals=theta[:nev].copy(), evecs=X, resid=resid, rho=rho[:nev] / scale[:nev],
                    restarts=restarts, spmm_calls=spmm_calls, converged=bool(conv.all()),
                    refills=refills, history=history)
