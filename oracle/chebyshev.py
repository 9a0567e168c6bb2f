"""Chebyshev polynomials and the Chebyshev filter (oracle; test infrastructure only).

Follows Sec. 4.1.1 of the paper: Definition 4.1 with Eq. (2)-(5) for the closed forms, Eq. (7)
for the scaled three-term recurrence, and Algorithm 4 (filter with sorted even degrees).

Pins (tests/test_oracle_chebyshev.py):
  * ``cheb_closed`` against the integer recurrence of Eq. (3) and cos(k*theta) on [-1, 1];
  * ``filter_columns`` on a diagonal H and on H = Q diag(lam) Q^H against the closed form of
    Eq. (5) evaluated at the eigenvalues;
  * ``sigma`` values against C_{m-1}(s)/C_m(s) with s = 1/sigma_1;
  * p_m(mu_1) = 1 (the normalisation of Eq. (5));
  * ``filter_alg4`` (double-buffer transcription) against ``filter_columns`` (per-column);
  * ``product`` against a hand-computed 3 x 3 complex case (beta and gamma nonzero; a transposed
    or conjugated matrix or swapped beta/gamma fails it), and composed with the rows of
    ``filter_scalars`` and Alg. 4's buffer swap against ``filter_columns`` and Eq. (5).

Readings where the paper is silent: (A - cI)X is formed as A@X - c*X (the matrix is never shifted
in place); in Alg. 4 the loop over s stops at the end of the degree array; a column with m_a = i
has received exactly i products.
"""

from __future__ import annotations

import numpy as np


def cheb_closed(m: int, t):
    """C_m(t) from Definition 4.1 / Eq. (2): cos(m acos t) on [-1, 1], cosh(m acosh |t|) with
    the sign (-1)^m for t < -1 outside it (Eq. (4) gives |C_m| = (|rho|^m + |rho|^-m)/2)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(m * np.arccos(t[inside]))
    ao = np.abs(t[~inside])
    sign = np.where(t[~inside] < 0, (-1.0) ** m, 1.0)
    out[~inside] = sign * np.cosh(m * np.arccosh(ao))
    return out


def filter_interval(b_sup: float, mu_nevnex: float):
    """Centre c and half-width e of [mu_{nev+nex}, b_sup] (Alg. 1's interval update, Alg. 4)."""
    c = 0.5 * (b_sup + mu_nevnex)
    e = 0.5 * (b_sup - mu_nevnex)
    return c, e


def p_closed(x, m: int, b_sup: float, mu_1: float, mu_nevnex: float):
    """Scaled filter polynomial of Eq. (5) with gamma = mu_1, alpha = mu_{nev+nex}, beta = b_sup
    (the identification made right after Eq. (5))."""
    c, e = filter_interval(b_sup, mu_nevnex)
    return cheb_closed(m, (np.asarray(x, dtype=np.float64) - c) / e) / cheb_closed(
        m, np.array([(mu_1 - c) / e])
    )[0]


def sigma(m: int, b_sup: float, mu_1: float, mu_nevnex: float):
    """sigma_1 .. sigma_m of Eq. (7): sigma_1 = e / (mu_1 - c), sigma_i = 1/(2/sigma_1 - sigma_{i-1})."""
    c, e = filter_interval(b_sup, mu_nevnex)
    s = [e / (mu_1 - c)]
    for _ in range(1, m):
        s.append(1.0 / (2.0 / s[0] - s[-1]))
    return np.array(s)


def filter_scalars(m_max: int, b_sup: float, mu_1: float, mu_nevnex: float):
    """Per-product coefficients of the filter, one row per product i = 1..m_max.

    Product i computes  OUT <- a_i * A @ X + g_i * X + b_i * Y  with
      i = 1 : a_1 = sigma_1/e,            b_1 = 0,                    g_1 = -a_1*c   (Alg. 4, first step)
      i >= 2: tau = 1/(2/sigma_1 - sigma), a_i = 2*tau/e, b_i = -tau*sigma, g_i = -a_i*c (Alg. 4, recurrence)
    Returned as an (m_max, 3) array of (a_i, b_i, g_i).
    """
    c, e = filter_interval(b_sup, mu_nevnex)
    sig = sigma(max(m_max, 1), b_sup, mu_1, mu_nevnex)
    rows = []
    a1 = sig[0] / e
    rows.append((a1, 0.0, -a1 * c))
    for i in range(2, m_max + 1):
        tau, prev = sig[i - 1], sig[i - 2]
        a = 2.0 * tau / e
        rows.append((a, -tau * prev, -a * c))
    return np.array(rows[:m_max])


def filter_columns(A, V, degrees, b_sup: float, mu_1: float, mu_nevnex: float):
    """Per-column Chebyshev filter: column a of the result is p_{m_a}(A) V[:, a] (Eq. (7)).

    Each column is filtered independently with its own degree, no blocking, no buffers shared
    between columns.  This is the reference for the HIP filter's parity tests.
    """
    A = np.asarray(A, dtype=np.complex128)
    V = np.asarray(V, dtype=np.complex128)
    degrees = np.asarray(degrees, dtype=np.int64)
    c, e = filter_interval(b_sup, mu_nevnex)
    out = np.empty_like(V)
    for a in range(V.shape[1]):
        m = int(degrees[a])
        sig = sigma(max(m, 1), b_sup, mu_1, mu_nevnex)
        prev = V[:, a].copy()                                   # p_0(A) v = v
        cur = (sig[0] / e) * (A @ prev - c * prev)              # p_1(A) v
        if m == 0:
            out[:, a] = prev
            continue
        for i in range(2, m + 1):                               # Eq. (7): p_{i} from p_{i-1}, p_{i-2}
            s_new, s_old = sig[i - 1], sig[i - 2]
            nxt = (2.0 * s_new / e) * (A @ cur - c * cur) - (s_new * s_old) * prev
            prev, cur = cur, nxt
        out[:, a] = cur
    return out


def filter_alg4(A, V, degrees, b_sup: float, mu_1: float, mu_nevnex: float):
    """Algorithm 4 as printed: two buffers swapped after every product, active columns s:end.

    ``degrees`` must be sorted ascending and even (Alg. 5 guarantees evenness, the sort
    closing each iteration of Alg. 1 the order).  Returns the buffer the algorithm returns (W after the last swap).
    """
    Vb = np.array(V, dtype=np.complex128, copy=True)
    m = np.asarray(degrees, dtype=np.int64)
    if np.any(np.diff(m) < 0):
        raise ValueError("degrees must be sorted ascending")
    if np.any(m % 2) or np.any(m < 2):
        raise ValueError("degrees must be even and >= 2")
    A = np.asarray(A, dtype=np.complex128)
    c, e = filter_interval(b_sup, mu_nevnex)
    sigma1 = e / (mu_1 - c)
    Wb = (sigma1 / e) * (A @ Vb - c * Vb)
    sig = sigma1
    s = 0                                  # 0-based index of the first active column
    nb = Vb.shape[1]
    for i in range(2, int(m[-1]) + 1):
        tau = 1.0 / (2.0 / sigma1 - sig)
        Vb[:, s:] = (2.0 * tau / e) * (A @ Wb[:, s:] - c * Wb[:, s:]) - (tau * sig) * Vb[:, s:]
        Vb, Wb = Wb, Vb
        sig = tau
        while s < nb and m[s] <= i:
            s += 1
    return Wb


def product(A, X, Y, alpha: float, beta: float, gamma: float):
    """One product of the recurrence written out: alpha*A@X + gamma*X + beta*Y (Eq. (7) with the
    shift (A - cI) expanded, as in the steps of Alg. 4).  ``Y`` is ignored when beta == 0.

    Pinned by the hand-computed case and the composition test in tests/test_oracle_chebyshev.py."""
    out = alpha * (np.asarray(A) @ np.asarray(X)) + gamma * np.asarray(X)
    if beta != 0.0:
        out = out + beta * np.asarray(Y)
    return out
