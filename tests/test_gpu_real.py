"""GPU parity of the real symmetric instance (CHASE_REAL_FP64 / CHASE_REAL_FP32 products and
filters, chase_solve with real_symmetric = 1) against the oracle and prescribed spectra.

The oracle computes in complex arithmetic; on a real symmetric problem its results are real
(checked by the oracle pins), so the GPU's real results are compared with their real parts.
Tolerances are those of the complex instance: one FP64 product <= 1e-13 of max |OUT|, FP64
filter <= 1e-12 block-Frobenius, FP32 filter <= 2e-5, eigenvalues <= 1e-10 ||H||.
"""

import numpy as np
import pytest

from oracle import chase as och
from oracle import chebyshev as ch
from paper_1805_10121_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1805_10121_amd import capi

    c = capi.Context(0)
    yield c
    c.close()


def _problem(n, nb, seed):
    g = wl.rng(seed)
    lam = np.sort(g.uniform(-1.0, 2.0, n))
    H = wl.symmetric_from(wl.haar_orthogonal(n, g), lam)
    V = g.standard_normal((n, nb))
    return lam, H, V


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,nb,alpha,beta,gamma", [
    (64, 64, 1.0, 0.0, 0.0),
    (200, 5, 0.7, -0.3, 0.25),      # thin tile (Lanczos block width)
    (333, 17, -1.3, 0.5, 0.1),      # odd n: ragged rows and K tail, one-element loads
    (300, 130, 2.0, 1.0, -0.5),     # even n: two-element loads, partial column tile
    (1000, 257, 1.0, -1.0, 0.0),
])
def test_real_hemm_step(ctx, n, nb, alpha, beta, gamma):
    import torch
    from paper_1805_10121_amd import capi

    print(f"real hemm_step n={n} nb={nb}", flush=True)
    _, H, X = _problem(n, nb, 20 + n)
    Y = wl.rng(6).standard_normal((n, nb))
    ref = ch.product(H, X, Y, alpha, beta, gamma).real
    dH, dX = capi.to_device(H), capi.to_device(X)
    dO = capi.to_device(Y) if beta != 0 else torch.full((nb, n), float("nan"), dtype=torch.float64, device="cuda")
    assert ctx.chase_hemm_step(capi.CHASE_REAL_FP64, dH, n, n, dX, n, dO, n, nb, alpha, beta, gamma) == 0
    torch.cuda.synchronize()
    got = capi.from_device(dO)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_real_hemm_step_leading_dimensions(ctx):
    import torch
    from paper_1805_10121_amd import capi

    n, nb, ldh, ldx, ldo = 150, 40, 163, 157, 170
    _, H, X = _problem(n, nb, 78)
    Hp = np.full((ldh, n), np.nan)
    Hp[:n] = H
    Xp = np.full((ldx, nb), np.nan)
    Xp[:n] = X
    Op = np.full((ldo, nb), 7.0)
    dH, dX, dO = capi.to_device(Hp), capi.to_device(Xp), capi.to_device(Op)
    assert ctx.chase_hemm_step(capi.CHASE_REAL_FP64, dH, ldh, n, dX, ldx, dO, ldo, nb, 1.5, 0.0, -0.5) == 0
    torch.cuda.synchronize()
    got = capi.from_device(dO)
    ref = ch.product(H, X, np.zeros((n, nb)), 1.5, 0.0, -0.5).real
    assert np.max(np.abs(got[:n] - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.all(got[n:] == 7.0)                   # rows past n untouched


@pytest.mark.parametrize("n,nb", [(1000, 70), (333, 41)])
def test_real_filter_fp64_vs_oracle(ctx, n, nb):
    import torch
    from paper_1805_10121_amd import capi

    print(f"real filter fp64 n={n} nb={nb}", flush=True)
    lam, H, V = _problem(n, nb, 30 + n)
    deg = np.sort(2 * wl.rng(n).integers(1, 19, nb)).astype(np.int32)
    b_sup, mu_1, mu_b = 2.02, lam[0], lam[nb]
    ref = ch.filter_columns(H, V, deg, b_sup, mu_1, mu_b)
    assert np.max(np.abs(ref.imag)) == 0.0
    dH, dV = capi.to_device(H), capi.to_device(V)
    dW = torch.empty_like(dV)
    assert ctx.chase_filter(capi.CHASE_REAL_FP64, dH, n, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b) == 0
    torch.cuda.synchronize()
    assert _relerr(capi.from_device(dV), ref.real) <= 1e-12


@pytest.mark.parametrize("n,nb", [(20000, 1200), (60000, 2400)])
def test_real_filter_large_orders_closed_form(ctx, n, nb):
    """The real FP64 filter at the bench's order-20000 shape and at order 60000 (sorted even
    degrees spread over 2..36) on the structured orthogonal generator: the whole filtered block
    against the closed form Q diag(p_m(lam)) Q^T V of Eq. (5), block-relative 1e-12."""
    import torch
    from paper_1805_10121_amd import capi

    print(f"real large-order filter n={n} nb={nb}: generating", flush=True)
    lam = wl.spectrum_for({60000: "sequence_n60000"}.get(n, "sequence_n20000"), n=n)
    dH = wl.symmetric_torch_fast(n, lam, seed=7400 + n)
    U, d = wl.structured_orthogonal(n, 7400 + n)
    V = wl.rng(7401).standard_normal((n, nb))
    deg = wl.optimized_degree_profile(nb, 36)
    b_sup, mu_1, mu_b = float(lam[-1]) + 0.05, float(lam[0]), float(lam[nb - 1])
    dV = capi.to_device(V)
    dW = torch.empty_like(dV)
    print("real large-order filter: running", flush=True)
    ctx.chase_filter(capi.CHASE_REAL_FP64, dH, n, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b)
    torch.cuda.synchronize()
    got = capi.from_device(dV)
    del dH, dV, dW
    torch.cuda.empty_cache()
    Wq = wl.apply_real_qt(U, d, V)
    for m in np.unique(deg):
        cols = deg == m
        Wq[:, cols] *= ch.p_closed(lam, int(m), b_sup, mu_1, mu_b)[:, None]
    ref = wl.apply_real_q(U, d, Wq)
    err = _relerr(got, ref)
    print(f"real large-order filter n={n}: block-relative error {err:.3e}")
    assert err <= 1e-12


def test_real_filter_fp32_vs_oracle(ctx):
    import torch
    from paper_1805_10121_amd import capi

    n, nb = 1000, 60
    lam, H, V = _problem(n, nb, 44)
    deg = np.sort(2 * wl.rng(3).integers(1, 10, nb)).astype(np.int32)
    b_sup, mu_1, mu_b = 2.02, lam[0], lam[nb]
    ref = ch.filter_columns(H, V, deg, b_sup, mu_1, mu_b).real
    dH = capi.to_device(H).to(torch.float32)
    dV = capi.to_device(V).to(torch.float32)
    dW = torch.empty_like(dV)
    assert ctx.chase_filter(capi.CHASE_REAL_FP32, dH, n, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b) == 0
    torch.cuda.synchronize()
    assert _relerr(capi.from_device(dV).astype(np.float64), ref) <= 2e-5


def _real_solve(ctx, H, V0, starts, **kw):
    from paper_1805_10121_amd import capi

    n, nb = V0.shape
    nev = kw.pop("nev")
    ritz_in = kw.pop("ritzv", None)
    cfg = capi.config(n, nev, nb - nev, real_symmetric=1, **kw)
    dS = capi.to_device(starts)
    cfg.lanczos_start = dS.data_ptr()
    dH, dV = capi.to_device(H), capi.to_device(V0)
    ritzv = np.zeros(nb) if ritz_in is None else np.array(ritz_in, dtype=np.float64)
    resid = np.zeros(nb)
    rc, st = ctx.chase_solve(cfg, dH, n, dV, n, ritzv, resid)
    return rc, st, ritzv, resid, capi.from_device(dV)


def _check(H, lam_true, ritzv, Y, nev, tol=1e-10):
    normH = np.max(np.abs(lam_true))
    assert np.max(np.abs(ritzv[:nev] - lam_true[:nev])) <= tol * normH
    Yn = Y[:, :nev]
    assert Yn.dtype == np.float64
    assert np.linalg.norm(Yn.T @ Yn - np.eye(nev)) <= 1e-12 * max(1, nev ** 0.5)
    R = H @ Yn - Yn * ritzv[None, :nev]
    assert np.max(np.linalg.norm(R, axis=0)) <= tol * normH * 1.0001


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_real_solve_prescribed_spectrum_and_oracle(ctx, precision):
    from paper_1805_10121_amd import capi

    n, nev, nex = 1000, 50, 20
    g = wl.rng(81)
    lam = wl.spectrum_uniform(n, g)
    H = wl.symmetric_from(wl.haar_orthogonal(n, g), lam)
    V0, S = g.standard_normal((n, nev + nex)), g.standard_normal((n, 5))
    prec = capi.CHASE_FP64 if precision == "fp64" else capi.CHASE_MIXED
    print(f"real solve {precision}", flush=True)
    rc, st, ritzv, resid, Y = _real_solve(ctx, H, V0, S, nev=nev, optim=1, precision=prec)
    assert rc == 0 and st.nconv >= nev
    _check(H, lam, ritzv, Y, nev)
    if precision == "mixed":
        assert st.fp32_iterations >= 1
    r = och.solve(H, och.ChaseParams(nev=nev, nex=nex, optim=True), V0, S)
    assert np.max(np.abs(ritzv[:nev] - r["ritzv"][:nev])) <= 1e-10 * np.max(np.abs(lam))


def test_real_householder_fallback(ctx):
    n, nev, nex = 200, 10, 5
    g = wl.rng(67)
    lam = wl.spectrum_uniform(n, g)
    H = wl.symmetric_from(wl.haar_orthogonal(n, g), lam)
    V0 = g.standard_normal((n, nev + nex))
    V0[:, -1] = 0.0
    rc, st, ritzv, resid, Y = _real_solve(ctx, H, np.asfortranarray(V0), g.standard_normal((n, 5)),
                                          nev=nev, optim=1, intersperse=0)
    assert rc == 0 and st.qr_fallbacks >= 1
    _check(H, lam, ritzv, Y, nev)


def test_real_warm_start_exact_vectors_one_iteration(ctx):
    n, nev, nex = 150, 8, 4
    g = wl.rng(91)
    lam = wl.spectrum_uniform(n, g)
    Q = wl.haar_orthogonal(n, g)
    H = wl.symmetric_from(Q, lam)
    rc, st, ritzv, resid, Y = _real_solve(ctx, H, np.asfortranarray(Q[:, : nev + nex]),
                                          g.standard_normal((n, 1)), nev=nev, optim=1, approx=1,
                                          ritzv=lam[: nev + nex])
    assert rc == 0 and st.iterations == 1
    _check(H, lam, ritzv, Y, nev)


def test_real_sequence_resident_state(ctx):
    import torch
    from paper_1805_10121_amd import capi

    n, nev, nex = 600, 30, 10
    g = wl.rng(95)
    lam = wl.spectrum_uniform(n, g)
    H = wl.symmetric_from(wl.haar_orthogonal(n, g), lam)
    cfg = capi.config(n, nev, nex, optim=1, real_symmetric=1, seed=5)
    seq = capi.Sequence(ctx, cfg)
    its = []
    for k in range(3):
        if k:
            E = g.standard_normal((n, n))
            E = 0.5 * (E + E.T)
            H = H + 1e-3 * E / np.max(np.abs(np.linalg.eigvalsh(E)))
        ev = np.linalg.eigvalsh(H)
        dH = capi.to_device(H)
        ritzv, resid = np.zeros(nev + nex), np.zeros(nev + nex)
        rc, st = seq.chase_seq_solve(dH, n, ritzv, resid)
        torch.cuda.synchronize()
        assert rc == 0
        assert np.max(np.abs(ritzv[:nev] - ev[:nev])) <= 1e-10 * np.max(np.abs(ev))
        its.append(st.iterations)
    assert its[1] <= its[0] and its[2] <= its[0]
    seq.close()


def test_real_invalid_flag(ctx):
    from paper_1805_10121_amd import capi

    n = 64
    cfg = capi.config(n, 4, 2, real_symmetric=2)
    H = np.eye(n)
    dH, dV = capi.to_device(H), capi.to_device(np.ones((n, 6)))
    with pytest.raises(capi.ChaseError) as e:
        ctx.chase_solve(cfg, dH, n, dV, n, np.zeros(6), np.zeros(6))
    assert "real_symmetric" in str(e.value)
