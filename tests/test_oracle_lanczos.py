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


def test_dos_self_consistency():
    # parity unpinned (heuristic): weights sum to one, mu_1 is a Ritz value inside the spectrum,
    # mu_{nev+nex} lies in the lower part of the spectrum.
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
