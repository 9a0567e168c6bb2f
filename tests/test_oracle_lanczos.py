"""Pins of the oracle's Lanczos estimates (Algorithm 6) -- no GPU."""

import numpy as np
import pytest

from oracle import lanczos as lz
from paper_1805_10121_amd import workloads as wl


def test_lanczos_relation_and_orthonormality():
    n, k = 200, 12
    g = wl.rng(11)
    lam = wl.spectrum_uniform(n, g)
    A = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    v0 = wl.complex_gaussian(g, n)
    alpha, beta, U = lz.lanczos_run(A, v0, k)
    T = lz.tridiagonal(alpha, beta)
    R = A @ U - U @ T
    assert np.linalg.norm(R[:, : k - 1]) <= 1e-12
    assert np.linalg.norm(R[:, k - 1]) == pytest.approx(beta[k - 1], rel=1e-10)
    assert np.linalg.norm(U.conj().T @ U - np.eye(k)) <= 1e-10


def test_full_lanczos_on_small_diagonal_is_exact():
    lam = np.array([-2.0, -0.5, 0.1, 0.3, 1.0, 4.0])
    A = np.diag(lam).astype(np.complex128)
    v0 = np.ones(6, dtype=np.complex128)
    alpha, beta, _ = lz.lanczos_run(A, v0, 6)
    got = np.linalg.eigvalsh(lz.tridiagonal(alpha, beta))
    assert np.allclose(got, lam, atol=1e-10)
    assert beta[-1] < 1e-8                  # f_n = 0 for a full run


@pytest.mark.parametrize("cfg,seed", [(1, 0), (1, 1), (2, 0), (2, 3)])
def test_upper_bound_is_an_upper_bound(cfg, seed):
    n = 600
    g = wl.rng(100 + seed)
    lam = wl.spectrum_uniform(n, g) if cfg == 1 else wl.spectrum_clustered(n, g, n_clustered=60)
    A = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    for j in range(3):
        alpha, beta, _ = lz.lanczos_run(A, wl.complex_gaussian(g, n), 25)
        b_sup = lz.upper_bound(alpha, beta)
        assert b_sup >= lam.max()
        assert b_sup - lam.max() < 0.5 * (lam.max() - lam.min())


def _hermitian(n, lam, seed):
    g = wl.rng(seed)
    return wl.hermitian_from(wl.haar_unitary(n, g), lam), g


def test_dos_measure_is_gauss_quadrature():
    """k Lanczos steps define the k-point Gauss quadrature of the start vector's spectral
    measure: sum_i w_i theta_i^p = v^H A^p v / v^H v for every p < 2k (the moments are computed
    here by repeated products with A, not through T)."""
    n, k = 150, 6
    lam = np.sort(wl.rng(31).uniform(-1.0, 1.0, n))
    A, g = _hermitian(n, lam, 32)
    v = wl.complex_gaussian(g, n)
    alpha, beta, _ = lz.lanczos_run(A, v, k)
    theta, w = lz.dos_measure(alpha, beta)
    assert len(theta) == k
    x = v / np.linalg.norm(v)
    y = x.copy()
    for p in range(2 * k):
        moment = float(np.real(np.vdot(x, y)))   # x^H A^p x
        assert np.sum(w * theta ** p) == pytest.approx(moment, abs=1e-11), p
        y = A @ y
    # degree 2k is beyond the rule's exactness: the quadrature is not the moment there
    assert abs(np.sum(w * theta ** (2 * k)) - float(np.real(np.vdot(x, y)))) > 1e-8


def test_dos_measure_at_full_length_is_the_spectral_measure():
    """At k = n the Ritz values are the eigenvalues and the weights the squared components of
    the start vector in the eigenbasis."""
    n = 12
    lam = np.linspace(-1.0, 1.0, n)
    g = wl.rng(41)
    Q = wl.haar_unitary(n, g)
    A = wl.hermitian_from(Q, lam)
    v = wl.complex_gaussian(g, n)
    alpha, beta, _ = lz.lanczos_run(A, v, n)
    theta, w = lz.dos_measure(alpha, beta)
    assert np.max(np.abs(theta - lam)) < 1e-10
    c = np.abs(Q.conj().T @ v) ** 2 / np.vdot(v, v).real
    assert np.max(np.abs(w - c)) < 1e-10


def test_dos_estimates_count_eigenvalues():
    """With k = n and start vectors of equal spectral weights, the density is 1/n at each
    eigenvalue, so mu_1 = lambda_1; on equispaced eigenvalues the Gaussians of the neighbours on
    either side of the point halfway between lambda_{nev+nex} and the next eigenvalue cancel
    pairwise by symmetry, so the smoothed integral reaches (nev + nex) / n exactly there.  The
    width (0.3 of the spacing) keeps the integral strictly increasing, so the crossing is
    unique."""
    n, nev, nex = 24, 7, 3
    lam = np.linspace(-1.0, 1.0, n)
    g = wl.rng(51)
    Q = wl.haar_unitary(n, g)
    A = wl.hermitian_from(Q, lam)
    runs = []
    for _ in range(3):
        phases = np.exp(2j * np.pi * g.uniform(0.0, 1.0, n))
        alpha, beta, _ = lz.lanczos_run(A, Q @ phases / np.sqrt(n), n)
        runs.append((alpha, beta))
    b_sup = lz.upper_bound(*runs[0])
    # sigma is measured on [min Ritz value, b_sup] mapped onto [-1, 1], here [-1, 1] itself
    sig = 0.3 * (lam[1] - lam[0])
    mu_1, mu_b = lz.dos_estimates(runs, b_sup, nev, nex, n, sigma=sig)
    m = nev + nex
    assert mu_1 == pytest.approx(lam[0], abs=1e-10)
    assert mu_b == pytest.approx(0.5 * (lam[m - 1] + lam[m]), abs=1e-8)
    # mu_1 is the smallest Ritz value over all runs: a run whose start vector has no component
    # along the lowest eigenvector sees lambda_2 as its smallest, and must not raise mu_1
    c = np.exp(2j * np.pi * g.uniform(0.0, 1.0, n)) / np.sqrt(n - 1)
    c[0] = 0.0
    a_perp, b_perp, _ = lz.lanczos_run(A, Q @ c, n - 1)
    assert lz.dos_estimates([(a_perp, b_perp)], b_sup, nev, nex, n, sig)[0] == \
        pytest.approx(lam[1], abs=1e-10)
    assert lz.dos_estimates([(a_perp, b_perp)] + runs, b_sup, nev, nex, n, sig)[0] == \
        pytest.approx(lam[0], abs=1e-10)
    # the target is (nev + nex) / n, not nev / n: the crossing moves with nex
    _, mu_b2 = lz.dos_estimates(runs, b_sup, nev, nex + 2, n, sigma=sig)
    assert mu_b2 == pytest.approx(0.5 * (lam[m + 1] + lam[m + 2]), abs=1e-8)


def test_ritz_vectors_below_galerkin():
    """The returned vectors are the Ritz vectors U z_i with theta_i below the bound: orthonormal,
    as many as those Ritz values, and satisfying the Galerkin condition U^H (A Y - Y Theta) = 0;
    at k = n they are exact eigenvectors."""
    n, k = 150, 20
    lam = np.sort(wl.rng(61).uniform(-1.0, 1.0, n))
    A, g = _hermitian(n, lam, 62)
    alpha, beta, U = lz.lanczos_run(A, wl.complex_gaussian(g, n), k)
    theta = np.linalg.eigvalsh(lz.tridiagonal(alpha, beta))
    bound = float(np.median(theta))
    Y = lz.ritz_vectors_below(alpha, beta, U, bound)
    sel = theta[theta < bound]
    assert Y.shape == (n, len(sel))
    assert np.linalg.norm(Y.conj().T @ Y - np.eye(len(sel))) < 1e-8
    G = U.conj().T @ (A @ Y - Y * sel[None, :])
    assert np.max(np.abs(G)) < 1e-8
    # full length: exact eigenpairs below the bound
    n2 = 12
    lam2 = np.linspace(-1.0, 1.0, n2)
    A2, g2 = _hermitian(n2, lam2, 63)
    a2, b2, U2 = lz.lanczos_run(A2, wl.complex_gaussian(g2, n2), n2)
    Y2 = lz.ritz_vectors_below(a2, b2, U2, 0.0)
    assert Y2.shape[1] == int(np.sum(lam2 < 0.0))
    assert np.max(np.abs(A2 @ Y2 - Y2 * lam2[lam2 < 0.0][None, :])) < 1e-10


def test_dos_self_consistency():
    # at the bench's scale (k = 25 of n = 800, random starts): weights sum to one, mu_1 is a Ritz
    # value inside the spectrum, mu_{nev+nex} lies in the lower part of the spectrum.
    n = 800
    g = wl.rng(21)
    lam = wl.spectrum_uniform(n, g)
    A = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    starts = wl.complex_gaussian(g, n, 5)
    est = lz.lanczos_estimates(A, starts, 40, 16, 25, approx=False)
    for j in range(1, 5):
        a, b, _ = lz.lanczos_run(A, starts[:, j], 25)
        _, S = np.linalg.eigh(lz.tridiagonal(a, b))
        assert np.sum(np.abs(S[0, :]) ** 2) == pytest.approx(1.0, abs=1e-12)
    assert lam.min() - 1e-12 <= est["mu_1"] <= lam[5]
    assert est["b_sup"] >= lam.max()
    assert lam.min() < est["mu_nevnex"] < np.quantile(lam, 0.25)
    Z = est["ritz_vectors"]
    assert Z.shape[0] == n
    if Z.shape[1]:
        assert np.linalg.norm(Z.conj().T @ Z - np.eye(Z.shape[1])) < 1e-8
