"""Spectral estimates by repeated Lanczos runs (oracle; test infrastructure only).

Follows Sec. 4.2 and Algorithm 6 of the paper: k plain Lanczos steps give A U = U T_k + f_k e_k^T;
the upper bound is b_sup = ||f_k||_2 + max Ritz value of T_k (the bound of Zhou and Li cited
there); n_vec further runs from fresh random vectors give the weighted spectral density of
Eq. (10), whose integral locates mu_{nev+nex}; mu_1 is the smallest Ritz value seen.

Readings where the paper is silent or garbled:
  * "simple Lanczos steps": no reorthogonalisation;
  * the DoS weight of Ritz value i is the squared modulus of the first component of the i-th
    eigenvector of T_k (the weights of one run then sum to one);
  * sigma = 0.25 is measured after mapping [min Ritz value, b_sup] affinely onto [-1, 1];
  * mu_1 is the minimum over the n_vec DoS runs of their smallest Ritz value;
  * the Ritz vectors U z_i interspersed into the start block come from the first DoS run and
    are placed in the leading columns.

Pins: ``lanczos_run`` -- the Lanczos relation A U = U T + f e_k^T and U^H U = I at small k,
exact eigenvalues for k = n on a small diagonal matrix, b_sup >= lambda_max (the invariant the
algorithm needs).  ``dos_measure`` -- the k-point Gauss quadrature property of Lanczos: its
weights and Ritz values reproduce the moments v^H A^p v / v^H v for p < 2k, and at k = n they
are the eigenvalues and the squared spectral components of the start vector.
``dos_estimates`` -- at k = n with start vectors of equal spectral weights and a narrow
Gaussian, the smoothed density integrates to the eigenvalue counting function, so mu_1 is
lambda_1 and mu_{nev+nex} lies just above lambda_{nev+nex}.  ``ritz_vectors_below`` -- the
Galerkin condition U^H (A Y - Y Theta) = 0 and the count of Ritz values below the bound; exact
eigenpairs at k = n.  How well the smoothed density of a few short runs estimates the spectrum
of a large matrix is a heuristic that no closed form fixes.
"""

from __future__ import annotations

import math

import numpy as np


def lanczos_run(A, v0, k: int):
    """k steps of the Hermitian Lanczos process from v0.

    Returns (alpha[k], beta[k], U[n, k]) where T_k has diagonal alpha and off-diagonal
    beta[0..k-2], and beta[k-1] = ||f_k||_2 is the norm of the residual vector f_k.
    """
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    k = min(k, n)
    U = np.zeros((n, k), dtype=np.complex128)
    alpha = np.zeros(k)
    beta = np.zeros(k)
    u = np.asarray(v0, dtype=np.complex128) / np.linalg.norm(v0)
    u_prev = np.zeros(n, dtype=np.complex128)
    b_prev = 0.0
    for j in range(k):
        U[:, j] = u
        w = A @ u - b_prev * u_prev
        alpha[j] = float(np.real(np.vdot(u, w)))
        w = w - alpha[j] * u
        beta[j] = float(np.linalg.norm(w))
        u_prev, b_prev = u, beta[j]
        if beta[j] == 0.0:
            # invariant subspace found; the remaining steps are empty
            U = U[:, : j + 1]
            alpha = alpha[: j + 1]
            beta = beta[: j + 1]
            break
        u = w / beta[j]
    return alpha, beta, U


def tridiagonal(alpha, beta):
    """T_k from the Lanczos coefficients."""
    k = len(alpha)
    T = np.diag(alpha).astype(np.float64)
    if k > 1:
        T += np.diag(beta[: k - 1], 1) + np.diag(beta[: k - 1], -1)
    return T


def upper_bound(alpha, beta):
    """b_sup = ||f_k||_2 + max(Ritz values of T_k) (Alg. 6, the upper bound)."""
    ritz = np.linalg.eigvalsh(tridiagonal(alpha, beta))
    return float(beta[-1] + ritz.max())


def _phi_cdf(x):
    return 0.5 * (1.0 + np.vectorize(math.erf)(np.asarray(x) / math.sqrt(2.0)))


def dos_measure(alpha, beta):
    """Ritz values and weights of one DoS run: the eigenvalues of T_k and the squared moduli of
    the first components of its eigenvectors (the discrete measure behind Eq. (10))."""
    lam, S = np.linalg.eigh(tridiagonal(alpha, beta))
    return lam, np.abs(S[0, :]) ** 2


def dos_estimates(runs, b_sup: float, nev: int, nex: int, n: int, sigma: float = 0.25):
    """mu_1 and mu_{nev+nex} from the averaged spectral density of Eq. (10) (Alg. 6, the DoS estimate).

    ``runs`` is a list of (alpha, beta) pairs, one per DoS Lanczos run.  The integral of the
    Gaussian-smoothed density is a sum of normal CDFs; t with integral (nev+nex)/n is found by
    bisection.
    """
    ritz_all, w_all = [], []
    for alpha, beta in runs:
        lam, w = dos_measure(alpha, beta)
        ritz_all.append(lam)
        w_all.append(w)
    lo = min(float(r.min()) for r in ritz_all)
    mu_1 = lo
    half = 0.5 * (b_sup - lo) if b_sup > lo else 1.0
    s = sigma * half                          # sigma on the [-1, 1] scale, back in matrix units
    lam = np.concatenate(ritz_all)
    w = np.concatenate(w_all) / len(runs)
    target = (nev + nex) / float(n)

    def cdf(t):
        return float(np.sum(w * _phi_cdf((t - lam) / s)))

    a, b = lo - 8.0 * s, b_sup + 8.0 * s
    for _ in range(200):
        mid = 0.5 * (a + b)
        if cdf(mid) < target:
            a = mid
        else:
            b = mid
    mu_nevnex = 0.5 * (a + b)
    return mu_1, mu_nevnex


def ritz_vectors_below(alpha, beta, U, bound: float):
    """Ritz vectors U z_i of one run whose Ritz values lie below ``bound`` (Alg. 6, the vectors it returns)."""
    lam, S = np.linalg.eigh(tridiagonal(alpha, beta))
    sel = lam < bound
    return U[:, : S.shape[0]] @ S[:, sel]


def lanczos_estimates(A, starts, nev: int, nex: int, k: int, approx: bool, sigma: float = 0.25):
    """Alg. 6.  ``starts`` holds 1 + n_vec start vectors as columns (random numbers are inputs).

    Returns dict with b_sup and, when ``approx`` is false, mu_1, mu_nevnex and the Ritz vectors
    to intersperse.
    """
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    a0, b0, _ = lanczos_run(A, starts[:, 0], k)
    ritz0 = np.linalg.eigvalsh(tridiagonal(a0, b0))
    out = {"b_sup": upper_bound(a0, b0), "matvecs": len(a0),
           "norm_lower": float(np.max(np.abs(ritz0)))}
    if approx:
        return out
    runs = []
    first = None
    for j in range(1, starts.shape[1]):
        aj, bj, Uj = lanczos_run(A, starts[:, j], k)
        runs.append((aj, bj))
        out["matvecs"] += len(aj)
        if first is None:
            first = (aj, bj, Uj)
    mu_1, mu_b = dos_estimates(runs, out["b_sup"], nev, nex, n, sigma)
    out["mu_1"], out["mu_nevnex"] = mu_1, mu_b
    out["ritz_vectors"] = ritz_vectors_below(*first, mu_b)
    return out
