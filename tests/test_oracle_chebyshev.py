"""Pins of the oracle's Chebyshev filter against facts fixed by the mathematics (no GPU).

Independent sources used here: NumPy's Chebyshev-series evaluator ``chebval`` (a library
routine for C_m), closed-form eigen-decompositions (diagonal H; H = Q diag(lam) Q^H), and the
normalisation p_m(mu_1) = 1 of Eq. (5).
"""

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import chebyshev as ch
from paper_1805_10121_amd import workloads as wl


def C_lib(m, t):
    coef = np.zeros(m + 1)
    coef[m] = 1.0
    return npcheb.chebval(np.asarray(t, dtype=np.float64), coef)


def p_lib(x, m, b_sup, mu_1, mu_b):
    c, e = 0.5 * (b_sup + mu_b), 0.5 * (b_sup - mu_b)
    return C_lib(m, (np.asarray(x) - c) / e) / C_lib(m, (mu_1 - c) / e)


@pytest.mark.parametrize("m", [0, 1, 2, 3, 7, 20, 36])
def test_cheb_closed_vs_library(m):
    t = np.concatenate([np.linspace(-1, 1, 41), np.linspace(-3, -1.0001, 9), np.linspace(1.0001, 3, 9)])
    ref = C_lib(m, t)
    got = ch.cheb_closed(m, t)
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 5, 10, 36])
def test_cos_k_theta(k):
    th = np.linspace(0, np.pi, 101)
    assert np.allclose(C_lib(k, np.cos(th)), np.cos(k * th), atol=1e-12)
    assert np.allclose(ch.cheb_closed(k, np.cos(th)), np.cos(k * th), atol=1e-12)


def test_sigma_is_ratio_of_chebyshev_values():
    b_sup, mu_1, mu_b = 2.1, -1.05, -0.3
    c, e = 0.5 * (b_sup + mu_b), 0.5 * (b_sup - mu_b)
    s = (mu_1 - c) / e                     # 1/sigma_1
    sig = ch.sigma(20, b_sup, mu_1, mu_b)
    for m in range(1, 21):
        assert sig[m - 1] == pytest.approx(C_lib(m - 1, s) / C_lib(m, s), rel=1e-13)


def test_filter_scalars_reproduce_the_polynomial():
    # Applying the per-product coefficients to a scalar x must give p_m(x) (Eq. (5)).
    b_sup, mu_1, mu_b = 1.7, -1.2, -0.1
    rows = ch.filter_scalars(30, b_sup, mu_1, mu_b)
    xs = np.array([-1.2, -1.0, -0.5, -0.1, 0.4, 1.7])
    prev = np.ones_like(xs)
    a, b, g = rows[0]
    cur = a * xs + g * prev
    for m in range(2, 31):
        a, b, g = rows[m - 1]
        prev, cur = cur, a * xs * cur + g * cur + b * prev
        assert np.allclose(cur, p_lib(xs, m, b_sup, mu_1, mu_b), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("seed", [0, 1])
def test_filter_on_diagonal_matrix(seed):
    g = wl.rng(seed)
    n, nb = 60, 12
    b_sup, mu_1, mu_b = 2.05, -1.0, -0.4
    lam = np.sort(g.uniform(-1.0, 2.0, n))
    lam[0] = mu_1                          # p_m(mu_1) = 1: that component is left unchanged
    A = np.diag(lam).astype(np.complex128)
    V = wl.complex_gaussian(g, n, nb)
    deg = np.sort(2 * g.integers(1, 19, nb))
    out = ch.filter_columns(A, V, deg, b_sup, mu_1, mu_b)
    for a in range(nb):
        ref = p_lib(lam, int(deg[a]), b_sup, mu_1, mu_b) * V[:, a]
        assert np.linalg.norm(out[:, a] - ref) <= 1e-13 * np.linalg.norm(ref)
        assert abs(out[0, a] - V[0, a]) <= 1e-13 * abs(V[0, a])


def test_filter_on_prescribed_spectrum():
    n, nb = 120, 9
    g = wl.rng(7)
    lam = wl.spectrum_uniform(n, g)
    Q = wl.haar_unitary(n, g)
    A = wl.hermitian_from(Q, lam)
    V = wl.complex_gaussian(g, n, nb)
    b_sup, mu_1, mu_b = 1.02, lam[0], lam[20]
    deg = np.array([2, 2, 4, 8, 10, 10, 20, 30, 36])
    out = ch.filter_columns(A, V, deg, b_sup, mu_1, mu_b)
    for a in range(nb):
        ref = Q @ (p_lib(lam, int(deg[a]), b_sup, mu_1, mu_b) * (Q.conj().T @ V[:, a]))
        assert np.linalg.norm(out[:, a] - ref) <= 1e-12 * np.linalg.norm(ref)


def test_filter_rejects_transposed_operand():
    # A^T = conj(A) differs from A for complex Hermitian A; the prescribed-spectrum pin must see it.
    n = 40
    g = wl.rng(3)
    lam = wl.spectrum_uniform(n, g)
    Q = wl.haar_unitary(n, g)
    A = wl.hermitian_from(Q, lam)
    V = wl.complex_gaussian(g, n, 2)
    deg = np.array([4, 4])
    good = ch.filter_columns(A, V, deg, 1.1, lam[0], lam[8])
    bad = ch.filter_columns(A.T, V, deg, 1.1, lam[0], lam[8])
    assert np.linalg.norm(good - bad) > 1e-3 * np.linalg.norm(good)


@pytest.mark.parametrize("seed", [0, 5])
def test_alg4_double_buffer_equals_per_column(seed):
    g = wl.rng(seed)
    n, nb = 80, 17
    lam = wl.spectrum_uniform(n, g)
    A = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    V = wl.complex_gaussian(g, n, nb)
    deg = np.sort(2 * g.integers(1, 19, nb))
    a = ch.filter_alg4(A, V, deg, 1.05, lam[0], lam[10])
    b = ch.filter_columns(A, V, deg, 1.05, lam[0], lam[10])
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


def test_alg4_rejects_odd_or_unsorted():
    A = np.eye(4, dtype=np.complex128)
    V = np.ones((4, 2), dtype=np.complex128)
    with pytest.raises(ValueError):
        ch.filter_alg4(A, V, [3, 4], 2.0, -1.0, 0.0)
    with pytest.raises(ValueError):
        ch.filter_alg4(A, V, [4, 2], 2.0, -1.0, 0.0)


def test_structured_generator_closed_form():
    # The fast device generator's matrix, read column-major, is Qbar diag(lam) Qbar^H with the
    # host-reproducible reflector factors; the filter on it has the closed form of Eq. (5).
    n, nb = 160, 5
    lam = wl.spectrum_uniform(n, wl.rng(8))
    A = wl.hermitian_torch_fast(n, lam, 21, device="cpu").numpy().T
    U, d = wl.structured_unitary(n, 21)
    V = wl.complex_gaussian(wl.rng(9), n, nb)
    deg = np.array([2, 4, 8, 16, 36])
    got = ch.filter_columns(A, V, deg, 1.1, lam[0], lam[15])
    W = wl.apply_colmajor_qh(U, d, V)
    for a in range(nb):
        W[:, a] *= p_lib(lam, int(deg[a]), 1.1, lam[0], lam[15])
    ref = wl.apply_colmajor_q(U, d, W)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_structured_orthogonal_generator_closed_form():
    # The real device generator's matrix is Q diag(lam) Q^T with the host-reproducible factors
    # of structured_orthogonal; the filter on it has the closed form of Eq. (5).
    n, nb = 150, 4
    lam = wl.spectrum_uniform(n, wl.rng(18))
    A = wl.symmetric_torch_fast(n, lam, 23, device="cpu").numpy()
    assert np.max(np.abs(A - A.T)) <= 1e-15
    U, d = wl.structured_orthogonal(n, 23)
    Q = wl.apply_real_q(U, d, np.eye(n))
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13
    assert np.linalg.norm(A - (Q * lam) @ Q.T) <= 1e-13 * n
    V = wl.rng(19).standard_normal((n, nb))
    deg = np.array([2, 6, 14, 36])
    got = ch.filter_columns(A, V, deg, 1.1, lam[0], lam[12])
    W = wl.apply_real_qt(U, d, V)
    for a in range(nb):
        W[:, a] *= p_lib(lam, int(deg[a]), 1.1, lam[0], lam[12])
    ref = wl.apply_real_q(U, d, W)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_filter_on_real_symmetric_matrix():
    # Real symmetric H (the real instance of the method): the oracle's filter of a real block
    # is real and equals Q diag(p_m(lam)) Q^T V.
    n, nb = 90, 6
    g = wl.rng(12)
    lam = wl.spectrum_uniform(n, g)
    Q = wl.haar_orthogonal(n, g)
    A = wl.symmetric_from(Q, lam)
    V = g.standard_normal((n, nb))
    deg = np.array([2, 4, 6, 10, 20, 36])
    out = ch.filter_columns(A, V, deg, 1.05, lam[0], lam[12])
    assert np.max(np.abs(out.imag)) == 0.0
    for a in range(nb):
        ref = Q @ (p_lib(lam, int(deg[a]), 1.05, lam[0], lam[12]) * (Q.T @ V[:, a]))
        assert np.linalg.norm(out[:, a].real - ref) <= 1e-12 * np.linalg.norm(ref)


# ----------------------------------------------------------------------------------------------
# oracle.chebyshev.product: one fused step  alpha*A@X + gamma*X + beta*Y  (Eq. (7) with the shift
# expanded; the steps of Alg. 4).  It is the reference of every single-product GPU test, so it is
# pinned on its own: a hand-computed case, and its composition into the whole filter.

# Hand-computed 3 x 3 case with integer entries: A Hermitian and not real (so A^T = conj(A) != A),
# beta != gamma, both nonzero.  A @ X, worked out by hand:
#   column 0: (4+2j, 5-1j, 3j);  column 1: (2j, 1-1j, 1)
# and with alpha = 2, beta = -3, gamma = 0.5:  2*A@X + 0.5*X - 3*Y  is _OUT below.
_A3 = np.array([[2, 1 + 1j, 0], [1 - 1j, 3, -2j], [0, 2j, 1]], dtype=np.complex128)
_X3 = np.array([[1, 1j], [2, 0], [-1j, 1]], dtype=np.complex128)
_Y3 = np.array([[1, 0], [0, 1], [1j, -1]], dtype=np.complex128)
_OUT = np.array([[5.5 + 4j, 4.5j], [11 - 2j, -1 - 2j], [2.5j, 5.5]], dtype=np.complex128)


def test_product_hand_computed():
    got = ch.product(_A3, _X3, _Y3, 2.0, -3.0, 0.5)
    assert np.array_equal(got, _OUT)
    # beta == 0: Y is not read (NaN there must not reach the result)
    nan_y = np.full_like(_Y3, np.nan)
    got0 = ch.product(_A3, _X3, nan_y, 2.0, 0.0, 0.5)
    assert np.array_equal(got0, _OUT + 3.0 * _Y3)


def test_product_fixture_rejects_plausible_mistakes():
    # The hand-computed case must tell apart a transposed or conjugated A and swapped beta/gamma.
    wrong = [
        ch.product(_A3.T, _X3, _Y3, 2.0, -3.0, 0.5),
        ch.product(_A3.conj(), _X3, _Y3, 2.0, -3.0, 0.5),
        ch.product(_A3, _X3, _Y3, 2.0, 0.5, -3.0),
        ch.product(_A3, _Y3, _X3, 2.0, -3.0, 0.5),
    ]
    for w in wrong:
        assert np.max(np.abs(w - _OUT)) >= 1.0


def _filter_by_products(A, V, degrees, b_sup, mu_1, mu_b):
    """Alg. 4 written with oracle.chebyshev.product and the rows of filter_scalars: product 1 into
    W, then V[:, s:] <- product(A, W[:, s:], V[:, s:], row i) and a swap of the two buffers."""
    m = np.asarray(degrees)
    rows = ch.filter_scalars(int(m[-1]), b_sup, mu_1, mu_b)
    Vb = np.array(V, dtype=np.complex128, copy=True)
    a, b, g = rows[0]
    Wb = ch.product(A, Vb, None, a, b, g)
    s = 0
    for i in range(2, int(m[-1]) + 1):
        a, b, g = rows[i - 1]
        Vb[:, s:] = ch.product(A, Wb[:, s:], Vb[:, s:], a, b, g)
        Vb, Wb = Wb, Vb
        while s < m.size and m[s] <= i:
            s += 1
    return Wb


@pytest.mark.parametrize("kind", ["diagonal", "unitary"])
def test_products_compose_to_the_filter(kind):
    g = wl.rng(31)
    n, nb = 70, 11
    lam = np.sort(g.uniform(-1.0, 2.0, n))
    b_sup, mu_1, mu_b = 2.04, float(lam[0]), float(lam[12])
    if kind == "diagonal":
        Q = np.eye(n, dtype=np.complex128)
        A = np.diag(lam).astype(np.complex128)
    else:
        Q = wl.haar_unitary(n, g)
        A = wl.hermitian_from(Q, lam)
    V = wl.complex_gaussian(g, n, nb)
    deg = np.sort(2 * g.integers(1, 19, nb))
    got = _filter_by_products(A, V, deg, b_sup, mu_1, mu_b)
    per_col = ch.filter_columns(A, V, deg, b_sup, mu_1, mu_b)
    closed = np.empty_like(V)
    for a in range(nb):
        closed[:, a] = Q @ (p_lib(lam, int(deg[a]), b_sup, mu_1, mu_b) * (Q.conj().T @ V[:, a]))
    assert np.linalg.norm(got - per_col) <= 1e-13 * np.linalg.norm(per_col)
    assert np.linalg.norm(got - closed) <= 1e-13 * np.linalg.norm(closed)
