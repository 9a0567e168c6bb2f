"""GPU single-precision solves (precision = CHASE_FP32: complex64, or float32 with
real_symmetric = 1) against prescribed spectra and the FP64 oracle run at the same tolerance.

Bars, derived from single-precision arithmetic (unit roundoff u = 2^-24 ~ 6e-8):
  - the returned residual norms are <= tol * ||H||_est (the convergence test itself);
  - the residual recomputed in FP64 from the returned FP32 vectors adds the rounding of one FP32
    product, about sqrt(n) u ||H|| (2e-6 ||H|| at n = 1000), so it is checked against 2 tol ||H||;
  - every eigenvalue then lies within that residual of a true one (Hermitian Bauer-Fike), so the
    Ritz values match the prescribed spectrum and the oracle's values within 2 tol ||H||;
  - orthonormality of the returned vectors: ||Y^H Y - I||_F <= 1e-4 (a few hundred u after the
    Cholesky QR passes, with margin).
"""

import numpy as np
import pytest

from oracle import chase as och
from paper_1805_10121_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-5  # Table 1's single-precision tolerance


@pytest.fixture(scope="module")
def ctx():
    from paper_1805_10121_amd import capi

    c = capi.Context(0)
    yield c
    c.close()


def _solve(ctx, H, V0, starts, real, **kw):
    import torch
    from paper_1805_10121_amd import capi

    n, nb = V0.shape
    nev = kw.pop("nev")
    cfg = capi.config_fp32(n, nev, nb - nev, real_symmetric=int(real), **kw)
    dt = torch.float32 if real else torch.complex64
    dS = capi.to_device(starts).to(dt)
    cfg.lanczos_start = dS.data_ptr()
    dH, dV = capi.to_device(H).to(dt), capi.to_device(V0).to(dt)
    ritzv, resid = np.zeros(nb), np.zeros(nb)
    rc, st = ctx.chase_solve(cfg, dH, n, dV, n, ritzv, resid)
    Y = capi.from_device(dV)
    assert Y.dtype == (np.float32 if real else np.complex64)
    return rc, st, ritzv, resid, Y


def _check(H, lam, ritzv, resid, Y, nev, st):
    normH = np.max(np.abs(lam))
    assert np.max(resid[:nev]) <= TOL * st.norm_est * 1.0001
    Yn = Y[:, :nev].astype(np.complex128 if np.iscomplexobj(Y) else np.float64)
    assert np.linalg.norm(Yn.conj().T @ Yn - np.eye(nev)) <= 1e-4
    R = H @ Yn - Yn * ritzv[None, :nev]
    assert np.max(np.linalg.norm(R, axis=0)) <= 2 * TOL * normH
    assert np.max(np.abs(ritzv[:nev] - lam[:nev])) <= 2 * TOL * normH


@pytest.mark.parametrize("real", [False, True])
@pytest.mark.parametrize("optim", [1, 0])
def test_fp32_solve_prescribed_spectrum_and_oracle(ctx, real, optim):
    n, nev, nex = 1000, 50, 20
    g = wl.rng(401 + int(real))
    lam = wl.spectrum_uniform(n, g)
    if real:
        H = wl.symmetric_from(wl.haar_orthogonal(n, g), lam)
        V0, S = g.standard_normal((n, nev + nex)), g.standard_normal((n, 5))
    else:
        H = wl.hermitian_from(wl.haar_unitary(n, g), lam)
        V0, S = wl.complex_gaussian(g, n, nev + nex), wl.complex_gaussian(g, n, 5)
    print(f"fp32 solve real={real} optim={optim}", flush=True)
    rc, st, ritzv, resid, Y = _solve(ctx, H, V0, S, real, nev=nev, optim=optim)
    assert rc == 0 and st.nconv >= nev
    _check(H, lam, ritzv, resid, Y, nev, st)
    p = och.ChaseParams(nev=nev, nex=nex, optim=bool(optim), tol=TOL, deg_max=18, deg=10,
                        lanczos_iter=12)
    ref = och.solve(H, p, V0, S)
    assert np.max(np.abs(ritzv[:nev] - ref["ritzv"][:nev])) <= 2 * TOL * np.max(np.abs(lam))
    # Lanczos bounds: FP32 Lanczos on the same start vectors, so b_sup agrees to FP32 accuracy
    assert st.b_sup == pytest.approx(ref["b_sup"], rel=1e-4)


def test_fp32_solve_ragged_sizes(ctx):
    # odd n (one-element loads, ragged row and K tails) and a block narrower than one tile
    n, nev, nex = 333, 9, 4
    g = wl.rng(409)
    lam = wl.spectrum_uniform(n, g)
    H = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    V0, S = wl.complex_gaussian(g, n, nev + nex), wl.complex_gaussian(g, n, 5)
    rc, st, ritzv, resid, Y = _solve(ctx, H, V0, S, False, nev=nev, optim=1)
    assert rc == 0
    _check(H, lam, ritzv, resid, Y, nev, st)


def test_fp32_householder_fallback(ctx):
    # a zero start column makes the Cholesky factorisations break down
    n, nev, nex = 200, 10, 5
    g = wl.rng(411)
    lam = wl.spectrum_uniform(n, g)
    H = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    V0 = wl.complex_gaussian(g, n, nev + nex)
    V0[:, -1] = 0.0
    rc, st, ritzv, resid, Y = _solve(ctx, H, np.asfortranarray(V0), wl.complex_gaussian(g, n, 5),
                                     False, nev=nev, optim=1, intersperse=0)
    assert rc == 0 and st.qr_fallbacks >= 1
    _check(H, lam, ritzv, resid, Y, nev, st)


def test_fp32_sequence(ctx):
    import torch
    from paper_1805_10121_amd import capi

    n, nev, nex = 600, 30, 10
    g = wl.rng(415)
    lam = wl.spectrum_uniform(n, g)
    H = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    cfg = capi.config_fp32(n, nev, nex, optim=1, seed=7)
    seq = capi.Sequence(ctx, cfg)
    its = []
    for k in range(3):
        if k:
            E = wl.complex_gaussian(g, n, n)
            E = 0.5 * (E + E.conj().T)
            H = H + 1e-3 * E / np.max(np.abs(np.linalg.eigvalsh(E)))
        ev = np.linalg.eigvalsh(H)
        dH = capi.to_device(H).to(torch.complex64)
        ritzv, resid = np.zeros(nev + nex), np.zeros(nev + nex)
        rc, st = seq.chase_seq_solve(dH, n, ritzv, resid)
        torch.cuda.synchronize()
        assert rc == 0
        assert np.max(np.abs(ritzv[:nev] - ev[:nev])) <= 2 * TOL * np.max(np.abs(ev))
        its.append(st.iterations)
    ptr, ld = seq.chase_seq_vectors()
    Y = capi.device_block_to_host(ptr, ld, n, nev + nex, dtype=np.complex64).astype(np.complex128)
    assert np.linalg.norm(Y[:, :nev].conj().T @ Y[:, :nev] - np.eye(nev)) <= 1e-4
    assert its[1] <= its[0] and its[2] <= its[0]
    seq.close()



def test_fp32_config2_full_size(ctx):
    """The order-10000 clustered problem (nev = 500, nex = 100, cold start) solved wholly in
    complex64 with Table 1's single-precision defaults: eigenvalues against the prescribed
    spectrum, residuals recomputed in FP64 on a column sample."""
    import torch
    from paper_1805_10121_amd import capi

    c = wl.WORKLOADS["clustered_n10000"]
    n, nev, nex = c["n"], c["nev"], c["nex"]
    lam = wl.spectrum_for("clustered_n10000")
    print("fp32 config2: generating H", flush=True)
    dH64 = wl.hermitian_torch(n, lam, seed=2001)
    dH = torch.empty((n, n), dtype=torch.complex64, device="cuda")
    assert ctx.chase_convert_c128_to_c64(dH64, n, dH, n, n, n) == 0
    H = capi.from_device(dH64)
    del dH64
    cfg = capi.config_fp32(n, nev, nex, optim=1, seed=2600)
    dV = capi.to_device(wl.start_block(n, nev + nex, 2500)).to(torch.complex64)
    ritzv, resid = np.zeros(nev + nex), np.zeros(nev + nex)
    print("fp32 config2: solving", flush=True)
    rc, st = ctx.chase_solve(cfg, dH, n, dV, n, ritzv, resid)
    print(f"fp32 config2: rc={rc} it={st.iterations} total_ms={st.total_ms:.1f} "
          f"qr_fallbacks={st.qr_fallbacks}", flush=True)
    assert rc == 0
    # the shifted CholeskyQR pass (shift capped at 1e-2 m in single precision) keeps the block
    # orthonormalisable without the Householder fallback
    assert st.qr_fallbacks == 0
    normH = np.max(np.abs(lam))
    assert np.max(resid[:nev]) <= TOL * st.norm_est * 1.0001
    assert np.max(np.abs(ritzv[:nev] - lam[:nev])) <= 2 * TOL * normH
    Y = capi.from_device(dV[:nev]).astype(np.complex128)
    assert np.linalg.norm(Y.conj().T @ Y - np.eye(nev)) <= 1e-4 * max(1.0, nev ** 0.5)
    cols = [0, 99, 100, 250, 499]
    R = H @ Y[:, cols] - Y[:, cols] * ritzv[None, cols]
    assert np.max(np.linalg.norm(R, axis=0)) <= 2 * TOL * normH
