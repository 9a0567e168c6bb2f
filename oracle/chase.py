"""The ChASE outer loop (oracle; test infrastructure only).

Algorithm 1 of the paper, step by step, with
  * FILTER          -- ``chebyshev.filter_columns`` (Alg. 4 / Eq. (7), per column);
  * ORTHOGONALIZE   -- Householder QR of [Y V] (``numpy.linalg.qr``; Alg. 1);
  * RAYLEIGH-RITZ   -- Alg. 2 with TSOLVE = ``numpy.linalg.eigh``;
  * residuals       -- Alg. 1, Res_a = ||A v_a - lambda_a v_a||_2;
  * DEFLATION & LOCKING -- Alg. 3;
  * interval update -- Alg. 1 (new mu_1 and mu_{nev+nex}, then c and e);
  * DEGREES         -- Alg. 5 / Eq. (8);
  * sort by degree  -- Alg. 1 (last step of an iteration);
  * LANCZOS         -- Alg. 6 (``lanczos.lanczos_estimates``);
and the sequence driver of Sec. 3.3 / Sec. 6.1 (solution of problem l-1 is the start of l).

Readings (the paper is silent, ambiguous or garbled):
  * Alg. 1 passes Q-hat to RAYLEIGH-RITZ; the active block Q-tilde is meant.
  * Alg. 1's call of DEGREES passes lambda_a; the Ritz value of the active vector is meant (Alg. 5 input).
  * The Rayleigh quotient G is symmetrised, (G + G^H)/2, before TSOLVE.
  * Residual test: relative by default, Res_a <= tol * ||A||_est with ||A||_est the largest
    |Ritz value| of the b_sup Lanczos run, fixed after LANCZOS.  Ritz values lie in
    [lambda_1, lambda_n], so ||A||_est <= ||A||_2 and the test implies Res_a/||A||_2 <= tol.
    The paper's absolute criterion is a flag.
    Alg. 5 then uses tol' = tol * ||A||_est so that degrees and locking agree.
  * Alg. 3 sorts stably by Ritz value and locks while Res_a <= tol (equality locks).
  * Alg. 5 with |t| <= 1 has |rho| = 1 and divides by log 1 = 0; the quotient is taken as
    +infinity so the min() with DEGMAX returns DEGMAX.  A zero residual is treated the same way.
  * The initial degree is rounded up to an even value (the filter's even-degree contract).
  * More than nev pairs may lock; the first nev (ascending) are returned.
  * On maxIter the locked and the active pairs are returned, sorted ascending, with status 1.

Pins (tests/test_oracle_solver.py): prescribed spectrum H = Q diag(lam) Q^H against lam;
brute-force ``eigh`` at n <= 200; orthonormality and residual invariants; Sylvester inertia;
unit cases for Alg. 3 and Alg. 5.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import chebyshev, lanczos


@dataclasses.dataclass
class ChaseParams:
    """Table 1 of the paper (double-precision defaults) plus the readings listed above."""

    nev: int
    nex: int
    tol: float = 1e-10
    max_iter: int = 25
    optim: bool = False
    deg_extra: int = 2
    deg_max: int = 36
    deg: int = 20
    lanczos_iter: int = 25
    num_lanczos: int = 4
    resid_relative: bool = True
    dos_sigma: float = 0.25
    intersperse: bool = True


def degrees(tol: float, res, ritz, c: float, e: float, deg_extra: int, deg_max: int):
    """Algorithm 5 for every active vector (vectorised over a, one formula per vector)."""
    res = np.asarray(res, dtype=np.float64)
    t = (np.asarray(ritz, dtype=np.float64) - c) / e
    root = np.sqrt((t * t - 1.0).astype(np.complex128))
    rho = np.maximum(np.abs(t - root), np.abs(t + root))
    out = np.empty(len(t), dtype=np.int64)
    for a in range(len(t)):
        lr = math.log(rho[a])
        if lr <= 0.0 or res[a] <= 0.0:
            d = deg_max
        else:
            q = abs(math.log(res[a] / tol) / lr)
            d = min(int(math.ceil(q)) + deg_extra, deg_max)
        out[a] = d + d % 2
    return out


def lock(ritz, res, V, tol: float):
    """Algorithm 3: stable sort by Ritz value, then lock the leading run with Res <= tol.

    Returns (n_new, order): the active arrays permuted by ``order`` have the n_new newly locked
    pairs first.
    """
    order = np.argsort(np.asarray(ritz), kind="stable")
    n_new = 0
    for a in order:
        if res[a] > tol:
            break
        n_new += 1
    return n_new, order


def rayleigh_ritz(A, Qt):
    """Algorithm 2 on the active block: G = Q^H A Q, (W, lam) = eigh(G), return (lam, Q W, A Q W)."""
    AQ = A @ Qt
    G = Qt.conj().T @ AQ
    G = 0.5 * (G + G.conj().T)
    lam, Wg = np.linalg.eigh(G)
    return lam, Qt @ Wg, AQ @ Wg


def orthogonalize(Y, Vf):
    """ORTHOGONALIZE of Alg. 1: Householder QR of [Y V], keep the columns after Y."""
    Qh, _ = np.linalg.qr(np.hstack([Y, Vf]), mode="reduced")
    return Qh[:, Y.shape[1]:]


def solve(A, p: ChaseParams, V0, lanczos_starts, approx: bool = False, ritzv0=None,
          mu=None):
    """Algorithm 1.  ``V0``: n x (nev+nex) start block (random numbers are inputs);
    ``lanczos_starts``: n x (1 + num_lanczos) Lanczos start vectors; ``approx``: warm start
    with ``ritzv0`` (min/max give mu_1, mu_{nev+nex}); ``mu``: optional (mu_1, mu_nevnex) pair that
    replaces the DoS estimate on a cold start.

    Returns a dict: ritzv (nev+nex,), resid (nev+nex,), V (n, nev+nex), status (0 converged,
    1 maxIter), nconv, iterations, matvecs, filter_matvecs, b_sup, norm_est.
    """
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    nb = p.nev + p.nex
    V = np.array(V0, dtype=np.complex128, copy=True)
    deg0 = p.deg + (p.deg % 2)
    m = np.full(nb, deg0, dtype=np.int64)                     # Alg. 1: initial degrees

    est = lanczos.lanczos_estimates(A, np.asarray(lanczos_starts), p.nev, p.nex,
                                    p.lanczos_iter, approx or mu is not None, p.dos_sigma)
    b_sup = est["b_sup"]
    matvecs = est["matvecs"]
    if approx:
        r0 = np.asarray(ritzv0, dtype=np.float64)
        mu_1, mu_b = float(r0.min()), float(r0.max())
    elif mu is not None:
        mu_1, mu_b = float(mu[0]), float(mu[1])
    else:
        mu_1, mu_b = est["mu_1"], est["mu_nevnex"]
        if p.intersperse:
            Z = est["ritz_vectors"][:, :nb]
            V[:, : Z.shape[1]] = Z
    norm_est = est["norm_lower"]
    tol_eff = p.tol * norm_est if p.resid_relative else p.tol

    Y = np.zeros((n, 0), dtype=np.complex128)
    Lam = np.zeros(0)
    Ylam_res = np.zeros(0)
    ritz = np.zeros(nb)
    res = np.zeros(nb)
    it = 0
    filter_mv = 0
    while Y.shape[1] < p.nev and it < p.max_iter:             # Alg. 1: outer loop
        it += 1
        nact = V.shape[1]
        Vf = chebyshev.filter_columns(A, V, m, b_sup, mu_1, mu_b)       # FILTER
        filter_mv += int(m.sum())
        Qt = orthogonalize(Y, Vf)                                         # ORTHOGONALIZE
        ritz, V, AV = rayleigh_ritz(A, Qt)                                # RAYLEIGH-RITZ
        matvecs += nact                                                   # H Q (A V = (H Q) W)
        res = np.linalg.norm(AV - V * ritz[None, :], axis=0)             # residuals
        n_new, order = lock(ritz, res, V, tol_eff)                       # DEFLATION & LOCKING
        ritz, res, V = ritz[order], res[order], V[:, order]
        Y = np.hstack([Y, V[:, :n_new]])
        Lam = np.concatenate([Lam, ritz[:n_new]])
        Ylam_res = np.concatenate([Ylam_res, res[:n_new]])
        ritz, res, V = ritz[n_new:], res[n_new:], V[:, n_new:]
        allv = np.concatenate([Lam, ritz])
        mu_1, mu_b = float(allv.min()), float(allv.max())                 # interval
        c, e = chebyshev.filter_interval(b_sup, mu_b)                     # c, e
        if p.optim:                                                       # DEGREES
            m = degrees(tol_eff, res, ritz, c, e, p.deg_extra, p.deg_max)
        else:
            m = np.full(V.shape[1], deg0, dtype=np.int64)
        srt = np.argsort(m, kind="stable")                                # sort by degree
        m, ritz, res, V = m[srt], ritz[srt], res[srt], V[:, srt]
    matvecs += filter_mv

    # assemble the output: locked pairs ascending, then the active ones ascending
    lo = np.argsort(Lam, kind="stable")
    ao = np.argsort(ritz, kind="stable")
    out_lam = np.concatenate([Lam[lo], ritz[ao]])
    out_res = np.concatenate([Ylam_res[lo], res[ao]])
    out_V = np.hstack([Y[:, lo], V[:, ao]])
    nconv = int(Y.shape[1])
    return {
        "ritzv": out_lam[:nb],
        "resid": out_res[:nb],
        "V": out_V[:, :nb],
        "status": 0 if nconv >= p.nev else 1,
        "nconv": nconv,
        "iterations": it,
        "matvecs": matvecs,
        "filter_matvecs": filter_mv,
        "b_sup": b_sup,
        "norm_est": norm_est,
        "tol_eff": tol_eff,
    }


def solve_sequence(As, p: ChaseParams, V0, lanczos_starts_per_problem, mu=None):
    """Sequence driver (Sec. 3.3, Sec. 6.1): problem 1 cold, then the previous nev+nex vectors
    and Ritz values are the warm start (approx = true) of the next problem."""
    results = []
    V, ritz = V0, None
    for k, A in enumerate(As):
        r = solve(A, p, V, lanczos_starts_per_problem[k], approx=(k > 0), ritzv0=ritz,
                  mu=mu if k == 0 else None)
        results.append(r)
        V, ritz = r["V"], r["ritzv"]
    return results
