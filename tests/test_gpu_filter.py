"""GPU parity of the Chebyshev filter (chase_filter, chase_hemm_step) against the oracle.

Tolerances (stated with their derivation in the design notes):
  * FP64, one product: max-element error <= 1e-13 relative to max |OUT| (a K = n FP64
    dot product with 4 real MACs per complex MAC has error ~ sqrt(n) u ||H|| ||x||).
  * FP64 filter: block-Frobenius relative error <= 1e-12 (per-column errors are amplified
    along the dominant direction, see the oracle notes).
  * FP32 filter: block-Frobenius relative error <= 2e-5 (FP32 unit roundoff 6e-8 times
    sqrt(n) accumulation growth and the recurrence's error propagation over <= 18 products).
"""

import numpy as np
import pytest

from oracle import chebyshev as ch
from paper_1805_10121_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401
    from paper_1805_10121_amd import capi

    c = capi.Context(0)
    yield c
    c.close()


def _problem(n, nb, seed, lam_lo=-1.0):
    g = wl.rng(seed)
    lam = np.sort(g.uniform(lam_lo, 2.0, n))
    H = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    V = wl.complex_gaussian(g, n, nb)
    return lam, H, V


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,nb,alpha,beta,gamma", [
    (64, 64, 1.0, 0.0, 0.0),
    (200, 70, 0.7, -0.3, 0.25),
    (333, 17, -1.3, 0.5, 0.1),     # ragged rows, K tail and a partial column tile
    (129, 130, 2.0, 1.0, -0.5),
    (1000, 1, 1.0, -1.0, 0.0),
    (200, 5, 0.9, 0.4, -0.2),       # thin tile (<= 16 columns): Lanczos block width
    (515, 16, -0.6, 1.0, 0.3),      # thin tile, full width, ragged rows and K tail
])
def test_hemm_step_fp64(ctx, n, nb, alpha, beta, gamma):
    import torch
    from paper_1805_10121_amd import capi

    print(f"hemm_step fp64 n={n} nb={nb}", flush=True)
    _, H, X = _problem(n, nb, 10 + n)
    Y = wl.complex_gaussian(wl.rng(5), n, nb)
    ref = ch.product(H, X, Y, alpha, beta, gamma)
    dH, dX = capi.to_device(H), capi.to_device(X)
    dO = capi.to_device(Y) if beta != 0 else torch.full((nb, n), float("nan"), dtype=torch.complex128, device="cuda")
    ctx.chase_hemm_step(capi.CHASE_FP64, dH, n, n, dX, n, dO, n, nb, alpha, beta, gamma)
    torch.cuda.synchronize()
    got = capi.from_device(dO)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_hemm_step_leading_dimensions(ctx):
    import torch
    from paper_1805_10121_amd import capi

    n, nb, ldh, ldx, ldo = 150, 40, 163, 157, 170
    _, H, X = _problem(n, nb, 77)
    Hp = np.zeros((ldh, n), dtype=np.complex128)
    Hp[:n] = H
    Hp[n:] = np.nan                                 # padding must never be read
    Xp = np.full((ldx, nb), np.nan, dtype=np.complex128)
    Xp[:n] = X
    Op = np.full((ldo, nb), 7.0 + 1j, dtype=np.complex128)
    dH, dX, dO = capi.to_device(Hp), capi.to_device(Xp), capi.to_device(Op)
    ctx.chase_hemm_step(capi.CHASE_FP64, dH, ldh, n, dX, ldx, dO, ldo, nb, 1.5, 0.0, -0.5)
    torch.cuda.synchronize()
    got = capi.from_device(dO)
    ref = ch.product(H, X, None, 1.5, 0.0, -0.5)
    assert np.max(np.abs(got[:n] - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.all(got[n:] == 7.0 + 1j)              # rows beyond n untouched


DEGREE_PATTERNS = {
    "equal": lambda nb: np.full(nb, 20),
    "sorted_mixed": lambda nb: wl.optimized_degree_profile(nb, 36),
    "tail_of_one": lambda nb: np.array([2] * (nb - 1) + [36]),
    "two_levels": lambda nb: np.array([4] * (nb // 2) + [10] * (nb - nb // 2)),
}


@pytest.mark.parametrize("pattern", list(DEGREE_PATTERNS))
@pytest.mark.parametrize("n,nb", [(1000, 70), (333, 65), (130, 1), (333, 12)])
def test_filter_fp64_parity(ctx, pattern, n, nb):
    import torch
    from paper_1805_10121_amd import capi

    print(f"filter fp64 n={n} nb={nb} pattern={pattern}", flush=True)
    deg = np.sort(DEGREE_PATTERNS[pattern](nb)).astype(np.int32)
    lam, H, V = _problem(n, nb, 1000 + n + nb)
    b_sup, mu_1, mu_b = 2.02, lam[0], lam[max(1, n // 15)]
    ref = ch.filter_columns(H, V, deg, b_sup, mu_1, mu_b)
    dH, dV = capi.to_device(H), capi.to_device(V)
    dW = torch.empty_like(dV)
    ctx.chase_filter(capi.CHASE_FP64, dH, n, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b)
    torch.cuda.synchronize()
    got = capi.from_device(dV)
    assert _relerr(got, ref) <= 1e-12


def test_filter_fp64_diagonal_closed_form(ctx):
    # p_m(H) on a diagonal H is diag(p_m(lam)); compare with the closed form of Eq. (5).
    import torch
    from paper_1805_10121_amd import capi

    n, nb = 257, 33
    g = wl.rng(3)
    lam = np.sort(g.uniform(-1.0, 2.0, n))
    H = np.diag(lam).astype(np.complex128)
    V = wl.complex_gaussian(g, n, nb)
    deg = np.sort(2 * g.integers(1, 19, nb)).astype(np.int32)
    b_sup, mu_1, mu_b = 2.0, lam[0], 0.0
    dH, dV = capi.to_device(H), capi.to_device(V)
    dW = torch.empty_like(dV)
    ctx.chase_filter(capi.CHASE_FP64, dH, n, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b)
    torch.cuda.synchronize()
    got = capi.from_device(dV)
    for a in range(nb):
        ref = ch.p_closed(lam, int(deg[a]), b_sup, mu_1, mu_b) * V[:, a]
        assert np.linalg.norm(got[:, a] - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,nb", [(1000, 70), (333, 65)])
def test_filter_fp32_parity(ctx, n, nb):
    import torch
    from paper_1805_10121_amd import capi

    deg = wl.optimized_degree_profile(nb, 18)
    lam, H, V = _problem(n, nb, 2000 + n)
    b_sup, mu_1, mu_b = 2.02, lam[0], lam[n // 15]
    ref = ch.filter_columns(H, V, deg, b_sup, mu_1, mu_b)
    dH, dV = capi.to_device(H), capi.to_device(V)
    h32 = torch.empty((n, n), dtype=torch.complex64, device="cuda")
    v32 = torch.empty((nb, n), dtype=torch.complex64, device="cuda")
    w32 = torch.empty_like(v32)
    ctx.chase_convert_c128_to_c64(dH, n, h32, n, n, n)
    ctx.chase_convert_c128_to_c64(dV, n, v32, n, n, nb)
    ctx.chase_filter(capi.CHASE_FP32, h32, n, n, v32, w32, n, nb, deg, b_sup, mu_1, mu_b)
    ctx.chase_convert_c64_to_c128(v32, n, dV, n, n, nb)
    torch.cuda.synchronize()
    err = _relerr(capi.from_device(dV), ref)
    print(f"fp32 filter block-relative error {err:.3e}")
    assert err <= 2e-5


def test_filter_deterministic(ctx):
    import torch
    from paper_1805_10121_amd import capi

    n, nb = 700, 90
    deg = wl.optimized_degree_profile(nb, 36)
    lam, H, V = _problem(n, nb, 4242)
    dH = capi.to_device(H)
    outs = []
    for _ in range(2):
        dV = capi.to_device(V)
        dW = torch.empty_like(dV)
        ctx.chase_filter(capi.CHASE_FP64, dH, n, n, dV, dW, n, nb, deg, 2.02, lam[0], lam[50])
        torch.cuda.synchronize()
        outs.append(dV.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


# per product mode: (precision name, element dtype, H elements per n x n matrix, H dtype)
_MODES = {
    "fp64": ("CHASE_FP64", "complex128", 1, "complex128"),
    "fp64_3m": ("CHASE_FP64_3M", "complex128", 2, "float64"),
    "fp32": ("CHASE_FP32", "complex64", 1, "complex64"),
    "fp32_3m": ("CHASE_FP32_3M", "complex64", 2, "float32"),
    "real_fp64": ("CHASE_REAL_FP64", "float64", 1, "float64"),
    "real_fp32": ("CHASE_REAL_FP32", "float32", 1, "float32"),
}


@pytest.mark.parametrize("mode", list(_MODES))
def test_filter_empty_and_invalid(ctx, mode):
    """Zero columns is a no-op; every malformed call is rejected with CHASE_EINVAL before any
    launch, in every product mode (for the planar 3M modes H spans both planes, so an output
    inside the imaginary plane is an overlap)."""
    import torch
    from paper_1805_10121_amd import capi

    pname, vdt, hmul, hdt = _MODES[mode]
    prec = getattr(capi, pname)
    n = 64
    dH = torch.zeros(hmul * n * n, dtype=getattr(torch, hdt), device="cuda")
    dV = torch.zeros((4, n), dtype=getattr(torch, vdt), device="cuda")
    dW = torch.zeros_like(dV)
    assert ctx.chase_filter(prec, dH, n, n, dV, dW, n, 0, [], 2.0, -1.0, 0.0) == 0
    bad = [
        dict(deg=[2, 3, 4, 4]),                 # odd
        dict(deg=[4, 2, 4, 4]),                 # unsorted
        dict(deg=[0, 2, 2, 2]),                 # below 2
        dict(bounds=(2.0, 0.0, -1.0)),          # mu_nevnex < mu_1
        dict(bounds=(float("nan"), -1.0, 0.0)),
        dict(W=dV),                             # V and W overlap
        dict(ld=n - 1),
        dict(ldh=n - 1),
        dict(W=dH[(hmul * n * n) // 2:]),        # W inside H (its second half)
    ]
    for case in bad:
        deg = case.get("deg", [2, 2, 2, 2])
        bsup, m1, mb = case.get("bounds", (2.0, -1.0, 0.0))
        W = case.get("W", dW)
        ld, ldh = case.get("ld", n), case.get("ldh", n)
        with pytest.raises(capi.ChaseError) as ei:
            ctx.chase_filter(prec, dH, ldh, n, dV, W, ld, 4, deg, bsup, m1, mb)
        assert ei.value.code == capi.CHASE_EINVAL, (mode, case)


@pytest.mark.parametrize("mode", list(_MODES))
def test_hemm_step_empty_and_invalid(ctx, mode):
    """chase_hemm_step: zero columns or order zero is a no-op; bad leading dimensions,
    overlapping operands, a non-finite coefficient and the solver-only precision
    CHASE_MIXED are rejected with CHASE_EINVAL before any launch."""
    import torch
    from paper_1805_10121_amd import capi

    pname, vdt, hmul, hdt = _MODES[mode]
    prec = getattr(capi, pname)
    n = 64
    dH = torch.zeros(hmul * n * n, dtype=getattr(torch, hdt), device="cuda")
    dX = torch.zeros((4, n), dtype=getattr(torch, vdt), device="cuda")
    dO = torch.zeros_like(dX)
    assert ctx.chase_hemm_step(prec, dH, n, n, dX, n, dO, n, 0, 1.0, 0.0, 0.0) == 0
    assert ctx.chase_hemm_step(prec, dH, n, 0, dX, n, dO, n, 4, 1.0, 0.0, 0.0) == 0
    bad = [
        dict(ldh=n - 1),
        dict(ldx=n - 1),
        dict(ldo=n - 1),
        dict(O=dX),                              # X and OUT are the same block
        dict(O=dH[(hmul * n * n) // 2:]),         # OUT inside H
        dict(X=dH[(hmul * n * n) // 2:]),         # X inside H
        dict(coef=(float("inf"), 0.0, 0.0)),
        dict(coef=(1.0, float("nan"), 0.0)),
        dict(prec=capi.CHASE_MIXED),
        dict(ncols=-1),
    ]
    for case in bad:
        a, b, g = case.get("coef", (1.0, 0.0, 0.0))
        with pytest.raises(capi.ChaseError) as ei:
            ctx.chase_hemm_step(case.get("prec", prec), dH, case.get("ldh", n), n,
                                case.get("X", dX), case.get("ldx", n), case.get("O", dO),
                                case.get("ldo", n), case.get("ncols", 4), a, b, g)
        assert ei.value.code == capi.CHASE_EINVAL, (mode, case)


def test_convert_planar64_invalid(ctx):
    """chase_convert_c128_to_planar64: order zero is a no-op; short leading dimensions and
    overlapping source and destination are rejected."""
    import torch
    from paper_1805_10121_amd import capi

    n = 32
    src = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    dst = torch.zeros(2 * n * n, dtype=torch.float64, device="cuda")
    assert ctx.chase_convert_c128_to_planar64(src, n, dst, n, 0) == 0
    for args in [(src, n - 1, dst, n), (src, n, dst, n - 1),
                 (src, n, torch.view_as_real(src).reshape(-1), n)]:
        with pytest.raises(capi.ChaseError) as ei:
            ctx.chase_convert_c128_to_planar64(*args, n)
        assert ei.value.code == capi.CHASE_EINVAL


def _filter_operand(ctx, dH, n, mode):
    """(precision, H operand) for a filter call: the interleaved H itself for the 4M products,
    or its planar copy (made here, H kept) for the 3M products."""
    import torch
    from paper_1805_10121_amd import capi

    if mode == "fp64":
        return capi.CHASE_FP64, dH
    planes = torch.empty(2 * n * n, dtype=torch.float64, device="cuda")
    ctx.chase_convert_c128_to_planar64(dH, n, planes, n, n)
    return capi.CHASE_FP64_3M, planes


@pytest.mark.parametrize("mode", ["fp64", "fp64_3m"])
def test_filter_full_size_sampled(ctx, mode):
    """Config-2 shape (n = 10000, nev + nex = 600) in both product schemes; the 3M one on the
    planar copy of H is the launch configuration the benchmark times.  A sample of columns is
    checked against the oracle column by column."""
    import torch
    from paper_1805_10121_amd import capi

    n, nb = 10000, 600
    print(f"full-size filter ({mode}): generating H on the device", flush=True)
    lam = wl.spectrum_for("clustered_n10000")
    dH = wl.hermitian_torch(n, lam, seed=2001)
    V = wl.start_block(n, nb, 2500)
    deg = wl.optimized_degree_profile(nb, 36)
    b_sup, mu_1, mu_b = 2.05, float(lam[0]), float(lam[nb - 1])
    dV = capi.to_device(V)
    dW = torch.empty_like(dV)
    prec, Hop = _filter_operand(ctx, dH, n, mode)
    print("full-size filter: running", flush=True)
    ctx.chase_filter(prec, Hop, n, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b)
    torch.cuda.synchronize()
    del Hop
    H = capi.from_device(dH)
    cols = [0, 1, 299, 300, 598, 599]
    sub = capi.from_device(dV[cols])
    print("full-size filter: oracle on sampled columns", flush=True)
    ref = ch.filter_columns(H, V[:, cols], deg[cols], b_sup, mu_1, mu_b)
    err = _relerr(sub, ref)
    print(f"full-size filter ({mode}): sampled block-relative error {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("mode", ["fp64", "fp64_3m"])
@pytest.mark.parametrize("n,nb,profile_max", [(10000, 600, 36), (20000, 1200, 36),
                                               (60000, 2400, 36)])
def test_filter_large_orders_closed_form(ctx, n, nb, profile_max, mode):
    """Orders 10000 (600 columns), 20000 (1200 columns) and 60000 (2400 columns), each with
    sorted even degrees spread over 2..36, on the structured generator, with 4M products on H
    and 3M products on its planar copy: the whole filtered block against the closed form
    Qbar diag(p_m(lam)) Qbar^H v (Eq. (5) at the eigenvalues), block-relative 1e-12."""
    import torch
    from paper_1805_10121_amd import capi

    print(f"large-order filter n={n} nb={nb} {mode}: generating", flush=True)
    lam = wl.spectrum_for({60000: "sequence_n60000", 20000: "sequence_n20000"}.get(
        n, "clustered_n10000"), n=n)
    dH = wl.hermitian_torch_fast(n, lam, seed=7000 + n)
    U, d = wl.structured_unitary(n, 7000 + n)
    V = wl.start_block(n, nb, 7100)
    deg = wl.optimized_degree_profile(nb, profile_max)
    b_sup, mu_1, mu_b = float(lam[-1]) + 0.05, float(lam[0]), float(lam[nb - 1])
    dV = capi.to_device(V)
    dW = torch.empty_like(dV)
    prec, Hop = _filter_operand(ctx, dH, n, mode)
    if mode != "fp64":
        del dH  # the planar copy is the only operand from here on
        torch.cuda.empty_cache()
    print("large-order filter: running", flush=True)
    ctx.chase_filter(prec, Hop, n, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b)
    torch.cuda.synchronize()
    del Hop, dW
    dH = None
    got = capi.from_device(dV)
    del dV
    torch.cuda.empty_cache()
    print("large-order filter: closed form", flush=True)
    Wq = wl.apply_colmajor_qh(U, d, V)
    for m in np.unique(deg):
        cols = deg == m
        Wq[:, cols] *= ch.p_closed(lam, int(m), b_sup, mu_1, mu_b)[:, None]
    ref = wl.apply_colmajor_q(U, d, Wq)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"large-order filter n={n} {mode}: block-relative error {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("n,nb", [(20000, 1200), (60000, 2400)])
def test_fp32_3m_filter_large_orders_closed_form(ctx, n, nb):
    """The mixed solver's FP32 stage (3M products on planar complex64 H, FP64 sums of the FP32
    accumulators every 8 K stages) at the order-20000 and order-60000 shapes, degrees 2..18,
    against the FP64 closed form Qbar diag(p_m(lam)) Qbar^H v.  Bar: each product's FP32 sums
    run over 128 terms before they are added into FP64, an error of about sqrt(128) u_32, and at
    most 18 products add up linearly: 18 sqrt(128) u_32 = 1.2e-5, independent of n.  Without the
    promotion (FP32 sums over K = n) the same bound would be 18 sqrt(n) u_32, 1.5e-4 at
    n = 20000, which this bar rejects; measured 6.8e-7 and 7.4e-7."""
    import torch
    from paper_1805_10121_amd import capi

    print(f"fp32 3M large-order filter n={n} nb={nb}: generating", flush=True)
    lam = wl.spectrum_for({60000: "sequence_n60000", 20000: "sequence_n20000"}[n], n=n)
    dH = wl.hermitian_torch_fast(n, lam, seed=7300 + n)
    U, d = wl.structured_unitary(n, 7300 + n)
    V = wl.start_block(n, nb, 7400)
    deg = wl.optimized_degree_profile(nb, 18)
    b_sup, mu_1, mu_b = float(lam[-1]) + 0.05, float(lam[0]), float(lam[nb - 1])
    planes = torch.empty(2 * n * n, dtype=torch.float32, device="cuda")
    ctx.chase_convert_c128_to_planar32(dH, n, planes, n, n)
    del dH
    torch.cuda.empty_cache()
    dV = capi.to_device(V).to(torch.complex64)
    dW = torch.empty_like(dV)
    print("fp32 3M large-order filter: running", flush=True)
    ctx.chase_filter(capi.CHASE_FP32_3M, planes, n, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b)
    torch.cuda.synchronize()
    del planes, dW
    got = capi.from_device(dV).astype(np.complex128)
    del dV
    torch.cuda.empty_cache()
    print("fp32 3M large-order filter: closed form", flush=True)
    Wq = wl.apply_colmajor_qh(U, d, V)
    for m in np.unique(deg):
        cols = deg == m
        Wq[:, cols] *= ch.p_closed(lam, int(m), b_sup, mu_1, mu_b)[:, None]
    ref = wl.apply_colmajor_q(U, d, Wq)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    bar = 18 * np.sqrt(128.0) * 2.0 ** -24
    print(f"fp32 3M large-order filter n={n}: block-relative error {err:.3e} (bar {bar:.2e})")
    assert err <= bar


def test_fp32_4m_filter_large_order_closed_form(ctx):
    """The single-precision 4M filter (CHASE_FP32 on interleaved complex64 H) at the bench's
    order-20000 shape, degrees 2..18, against the FP64 closed form Qbar diag(p_m(lam)) Qbar^H v.
    This tile keeps its FP32 sums over the whole K = n, so each product's error is about
    sqrt(n) u_32 and at most 18 products add up linearly: bar 18 sqrt(n) u_32 = 1.5e-4."""
    import torch
    from paper_1805_10121_amd import capi

    n, nb = 20000, 1200
    print(f"fp32 4M large-order filter n={n} nb={nb}: generating", flush=True)
    lam = wl.spectrum_for("sequence_n20000", n=n)
    dH = wl.hermitian_torch_fast(n, lam, seed=7500 + n)
    U, d = wl.structured_unitary(n, 7500 + n)
    V = wl.start_block(n, nb, 7501)
    deg = wl.optimized_degree_profile(nb, 18)
    b_sup, mu_1, mu_b = float(lam[-1]) + 0.05, float(lam[0]), float(lam[nb - 1])
    h32 = torch.empty((n, n), dtype=torch.complex64, device="cuda")
    ctx.chase_convert_c128_to_c64(dH, n, h32, n, n, n)
    del dH
    torch.cuda.empty_cache()
    dV = capi.to_device(V).to(torch.complex64)
    dW = torch.empty_like(dV)
    print("fp32 4M large-order filter: running", flush=True)
    ctx.chase_filter(capi.CHASE_FP32, h32, n, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b)
    torch.cuda.synchronize()
    del h32, dW
    got = capi.from_device(dV).astype(np.complex128)
    del dV
    torch.cuda.empty_cache()
    Wq = wl.apply_colmajor_qh(U, d, V)
    for m in np.unique(deg):
        cols = deg == m
        Wq[:, cols] *= ch.p_closed(lam, int(m), b_sup, mu_1, mu_b)[:, None]
    ref = wl.apply_colmajor_q(U, d, Wq)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    bar = 18 * np.sqrt(float(n)) * 2.0 ** -24
    print(f"fp32 4M large-order filter n={n}: block-relative error {err:.3e} (bar {bar:.2e})")
    assert err <= bar


@pytest.mark.parametrize("n,ld", [(333, 334), (333, 333), (1001, 1002)])
def test_filter_fp32_ragged_rows_and_leading_dimension(ctx, n, ld):
    """FP32 products use 16-byte loads when pointers and leading dimensions allow it; odd n
    with even ld exercises the per-element tail, odd ld the 8-byte path."""
    import torch
    from paper_1805_10121_amd import capi

    nb = 37
    deg = wl.optimized_degree_profile(nb, 12)
    lam, H, V = _problem(n, nb, 3000 + n + ld)
    b_sup, mu_1, mu_b = 2.02, lam[0], lam[n // 15]
    ref = ch.filter_columns(H, V, deg, b_sup, mu_1, mu_b)
    Hp = np.full((ld, n), np.nan, dtype=np.complex64)
    Hp[:n] = H.astype(np.complex64)
    Vp = np.full((ld, nb), np.nan, dtype=np.complex64)
    Vp[:n] = V.astype(np.complex64)
    dH, dV = capi.to_device(Hp), capi.to_device(Vp)
    dW = torch.zeros_like(dV)
    ctx.chase_filter(capi.CHASE_FP32, dH, ld, n, dV, dW, ld, nb, deg, b_sup, mu_1, mu_b)
    torch.cuda.synchronize()
    got = capi.from_device(dV)[:n].astype(np.complex128)
    err = _relerr(got, ref)
    print(f"fp32 n={n} ld={ld} block-relative error {err:.3e}")
    assert err <= 2e-5


@pytest.mark.parametrize("n,ld", [(1000, 1000), (333, 333), (1024, 1024), (515, 516)])
def test_filter_fp32_3m_parity(ctx, n, ld):
    """3M products on planar complex64 H (three FP32 MFMA products per complex product, FP64
    sums across K stages) against the FP64 oracle."""
    import torch
    from paper_1805_10121_amd import capi

    nb = 70
    deg = wl.optimized_degree_profile(nb, 18)
    lam, H, V = _problem(n, nb, 5000 + n)
    b_sup, mu_1, mu_b = 2.02, lam[0], lam[n // 15]
    ref = ch.filter_columns(H, V, deg, b_sup, mu_1, mu_b)
    Hp = np.zeros((ld, n), dtype=np.complex128)
    Hp[:n] = H
    dH = capi.to_device(Hp)
    planes = torch.empty(2 * ld * n, dtype=torch.float32, device="cuda")
    ctx.chase_convert_c128_to_planar32(dH, ld, planes, ld, n)
    v32 = torch.empty((nb, n), dtype=torch.complex64, device="cuda")
    dV = capi.to_device(V)
    ctx.chase_convert_c128_to_c64(dV, n, v32, n, n, nb)
    w32 = torch.empty_like(v32)
    ctx.chase_filter(capi.CHASE_FP32_3M, planes, ld, n, v32, w32, n, nb, deg, b_sup, mu_1, mu_b)
    ctx.chase_convert_c64_to_c128(v32, n, dV, n, n, nb)
    torch.cuda.synchronize()
    err = _relerr(capi.from_device(dV), ref)
    print(f"fp32 3M n={n} ld={ld} block-relative error {err:.3e}")
    assert err <= 2e-5


def test_hemm_step_3m_single_product(ctx):
    import torch
    from paper_1805_10121_amd import capi

    n, nb = 777, 45
    _, H, X = _problem(n, nb, 99)
    Y = wl.complex_gaussian(wl.rng(7), n, nb)
    ref = ch.product(H, X, Y, 0.9, -0.4, 0.3)
    dH = capi.to_device(H)
    planes = torch.empty(2 * n * n, dtype=torch.float32, device="cuda")
    ctx.chase_convert_c128_to_planar32(dH, n, planes, n, n)
    x32 = capi.to_device(X.astype(np.complex64))
    o32 = capi.to_device(Y.astype(np.complex64))
    ctx.chase_hemm_step(capi.CHASE_FP32_3M, planes, n, n, x32, n, o32, n, nb, 0.9, -0.4, 0.3)
    torch.cuda.synchronize()
    got = capi.from_device(o32).astype(np.complex128)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("mode", ["fp64", "fp64_3m", "fp32", "fp32_3m", "real_fp64", "real_fp32"])
def test_hemm_step_random_shapes(ctx, mode):
    """One product OUT <- alpha H X + gamma X + beta OUT on seeded random shapes: orders 1..599,
    1..199 columns (thin, narrow, slim and wide tiles; data-parallel and stream-K schedules),
    leading dimensions padded by 0..3 (odd and even), beta = 0 with a NaN-filled OUT that must
    not be read, and rows past n of OUT that must stay untouched.  Against the oracle's product
    in FP64; FP32 modes within 5e-5 of max |OUT| (K <= 599 terms of FP32 rounding)."""
    import torch
    from paper_1805_10121_amd import capi

    real = mode.startswith("real")
    prec = {"fp64": capi.CHASE_FP64, "fp64_3m": capi.CHASE_FP64_3M, "fp32": capi.CHASE_FP32,
            "fp32_3m": capi.CHASE_FP32_3M, "real_fp64": capi.CHASE_REAL_FP64,
            "real_fp32": capi.CHASE_REAL_FP32}[mode]
    single = mode in ("fp32", "fp32_3m", "real_fp32")
    tol = 5e-5 if single else 1e-13
    g = wl.rng({"fp64": 1, "fp32": 2, "fp32_3m": 3, "real_fp64": 4, "real_fp32": 5,
                "fp64_3m": 6}[mode] + 7000)
    for case in range(8):
        n, nb = int(g.integers(1, 600)), int(g.integers(1, 200))
        ldh, ldx, ldo = (n + int(p) for p in g.integers(0, 4, 3))
        alpha, beta, gamma = (float(v) for v in g.uniform(-2.0, 2.0, 3))
        if case % 3 == 0:
            beta = 0.0
        print(f"{mode} case {case}: n={n} ncols={nb} ld=({ldh},{ldx},{ldo}) beta={beta:.2f}",
              flush=True)
        if real:
            A = g.standard_normal((n, n))
            H = 0.5 * (A + A.T)
            X, Y = g.standard_normal((n, nb)), g.standard_normal((n, nb))
        else:
            A = wl.complex_gaussian(g, n, n)
            H = 0.5 * (A + A.conj().T)
            X, Y = wl.complex_gaussian(g, n, nb), wl.complex_gaussian(g, n, nb)
        ref = ch.product(H, X, Y, alpha, beta, gamma)
        if real:
            ref = ref.real
        dt = (np.float32 if real else np.complex64) if single else (np.float64 if real else np.complex128)
        Hp = np.full((ldh, n), np.nan, dtype=H.dtype)
        Hp[:n] = H
        Xp = np.full((ldx, nb), np.nan, dtype=X.dtype)
        Xp[:n] = X
        Op = np.full((ldo, nb), 7.0, dtype=Y.dtype)
        Op[:n] = Y if beta != 0.0 else np.nan
        if mode == "fp32_3m":
            dH64 = capi.to_device(Hp)
            dH = torch.empty(2 * ldh * n, dtype=torch.float32, device="cuda")
            ctx.chase_convert_c128_to_planar32(dH64, ldh, dH, ldh, n)
        elif mode == "fp64_3m":
            dH64 = capi.to_device(Hp)
            dH = torch.empty(2 * ldh * n, dtype=torch.float64, device="cuda")
            ctx.chase_convert_c128_to_planar64(dH64, ldh, dH, ldh, n)
        else:
            dH = capi.to_device(Hp.astype(dt))
        dX, dO = capi.to_device(Xp.astype(dt)), capi.to_device(Op.astype(dt))
        assert ctx.chase_hemm_step(prec, dH, ldh, n, dX, ldx, dO, ldo, nb, alpha, beta, gamma) == 0
        torch.cuda.synchronize()
        got = capi.from_device(dO)
        assert np.all(got[n:] == 7.0)
        err = np.max(np.abs(got[:n].astype(ref.dtype) - ref)) / np.max(np.abs(ref))
        assert err <= tol, (mode, case, n, nb, err)


@pytest.mark.parametrize("n,ld", [(1000, 1000), (333, 335), (130, 130)])
def test_filter_fp64_3m_parity(ctx, n, ld):
    """3M products on planar complex128 H (three FP64 MFMA products per complex product) against
    the oracle at the FP64 filter bar (block-relative 1e-12), with sorted even degrees 2..36 so
    that the active range shrinks over 36 products (wide, narrow and thin 3M tiles)."""
    import torch
    from paper_1805_10121_amd import capi

    nb = 70
    deg = wl.optimized_degree_profile(nb, 36)
    lam, H, V = _problem(n, nb, 6000 + n)
    b_sup, mu_1, mu_b = 2.02, lam[0], lam[min(n - 1, nb)]
    ref = ch.filter_columns(H, V, deg, b_sup, mu_1, mu_b)
    Hp = np.zeros((ld, n), dtype=np.complex128)
    Hp[:n] = H
    planes = torch.empty(2 * ld * n, dtype=torch.float64, device="cuda")
    ctx.chase_convert_c128_to_planar64(capi.to_device(Hp), ld, planes, ld, n)
    dV = capi.to_device(V)
    dW = torch.empty_like(dV)
    ctx.chase_filter(capi.CHASE_FP64_3M, planes, ld, n, dV, dW, n, nb, deg, b_sup, mu_1, mu_b)
    torch.cuda.synchronize()
    err = _relerr(capi.from_device(dV), ref)
    print(f"fp64 3M n={n} ld={ld} block-relative error {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("n,nb,pad", [(1, 1, 0), (63, 3, 1), (64, 8, 0), (65, 5, 2), (200, 5, 0),
                                      (300, 6, 0), (513, 7, 2), (640, 4, 0), (777, 1, 3),
                                      (1000, 8, 1), (3000, 5, 0), (4500, 2, 1), (5000, 3, 0)])
def test_hemm_step_lower_triangle(ctx, n, nb, pad):
    """CHASE_FP64_LOWER (one-triangle product for thin blocks) against the oracle's product: the
    upper triangle of H and the padding rows are NaN, so any read of them would show; ragged
    orders cover partial tiles, orders up to 4500 every super-tile edge the launcher picks
    (1 and 2 here, 4 and 8 in the order-10000/20000 test); beta = 0 with a NaN-filled OUT that
    must not be read; a repeat is bitwise equal."""
    import torch
    from paper_1805_10121_amd import capi

    print(f"lower-triangle product n={n} ncols={nb}", flush=True)
    g = wl.rng(9000 + n)
    A = wl.complex_gaussian(g, n, n)
    H = 0.5 * (A + A.conj().T)
    X, Y = wl.complex_gaussian(g, n, nb), wl.complex_gaussian(g, n, nb)
    Hp = np.full((n + pad, n), np.nan + 1j * np.nan, dtype=np.complex128)
    Hp[:n] = np.tril(H)
    Hp[:n][np.triu_indices(n, 1)] = np.nan
    dH = capi.to_device(Hp)
    Xp = np.full((n + pad, nb), np.nan, dtype=np.complex128)
    Xp[:n] = X
    dX = capi.to_device(Xp)
    for alpha, beta, gamma in ((1.0, 0.0, 0.0), (0.7, -0.4, 0.3)):
        ref = ch.product(H, X, Y, alpha, beta, gamma)
        Op = np.full((n + pad, nb), 7.0, dtype=np.complex128)
        Op[:n] = Y if beta != 0.0 else np.nan
        outs = []
        for _ in range(2):
            dO = capi.to_device(Op)
            ctx.chase_hemm_step(capi.CHASE_FP64_LOWER, dH, n + pad, n, dX, n + pad, dO, n + pad, nb,
                                alpha, beta, gamma)
            torch.cuda.synchronize()
            outs.append(capi.from_device(dO))
        got = outs[0]
        assert np.array_equal(outs[0], outs[1])
        assert np.all(got[n:] == 7.0)
        err = np.max(np.abs(got[:n] - ref)) / np.max(np.abs(ref))
        assert err <= 1e-13, (n, nb, alpha, beta, err)


def test_hemm_step_lower_triangle_large_orders(ctx):
    """CHASE_FP64_LOWER at orders 10000 and 20000 (super-tiles of 2 to 8 tiles) against the
    oracle's product on a host copy of H; at order 20000 the partial sums of 8 columns exceed the
    context's product scratch, which the call reports as an invalid argument."""
    import torch
    from paper_1805_10121_amd import capi

    for n, seed, widths in ((10000, 41, (8, 5, 1)), (20000, 42, (5, 2, 1))):
        lam = wl.spectrum_for("sequence_n20000", n=n)
        dH = wl.hermitian_torch_fast(n, lam, seed=seed)
        H = capi.from_device(dH)
        if n == 20000:
            dX = torch.zeros((8, n), dtype=torch.complex128, device="cuda")
            dO = torch.zeros((8, n), dtype=torch.complex128, device="cuda")
            with pytest.raises(capi.ChaseError) as ei:
                ctx.chase_hemm_step(capi.CHASE_FP64_LOWER, dH, n, n, dX, n, dO, n, 8, 1.0, 0.0,
                                    0.0)
            assert ei.value.code == capi.CHASE_EINVAL
            del dX, dO
        for nb in widths:
            print(f"lower-triangle product n={n} ncols={nb}", flush=True)
            X = wl.start_block(n, nb, seed + nb)
            dX = capi.to_device(X)
            dO = torch.full((nb, n), float("nan"), dtype=torch.complex128, device="cuda")
            ctx.chase_hemm_step(capi.CHASE_FP64_LOWER, dH, n, n, dX, n, dO, n, nb, 1.0, 0.0, 0.0)
            torch.cuda.synchronize()
            ref = ch.product(H, X, None, 1.0, 0.0, 0.0)
            err = np.max(np.abs(capi.from_device(dO) - ref)) / np.max(np.abs(ref))
            print(f"  max error {err:.2e} of max |OUT|")
            assert err <= 1e-13
        del dH, H
        torch.cuda.empty_cache()


def test_hemm_step_lower_triangle_order_60000(ctx):
    """CHASE_FP64_LOWER at order 60000 with one column, the widest block whose partial sums fit
    the context's product scratch at this order (two columns are refused).  H holds 7.2e9
    doubles, so element offsets pass 2^31.  Checked against the structured generator's closed
    form H x = Qbar diag(lam) Qbar^H x (no host copy of H)."""
    import torch
    from paper_1805_10121_amd import capi

    n = 60000
    print(f"lower-triangle product n={n}: generating", flush=True)
    lam = wl.spectrum_for("sequence_n60000", n=n)
    dH = wl.hermitian_torch_fast(n, lam, seed=7300)
    U, d = wl.structured_unitary(n, 7300)
    dX2 = torch.zeros((2, n), dtype=torch.complex128, device="cuda")
    dO2 = torch.zeros((2, n), dtype=torch.complex128, device="cuda")
    with pytest.raises(capi.ChaseError) as ei:
        ctx.chase_hemm_step(capi.CHASE_FP64_LOWER, dH, n, n, dX2, n, dO2, n, 2, 1.0, 0.0, 0.0)
    assert ei.value.code == capi.CHASE_EINVAL
    del dX2, dO2
    X = wl.start_block(n, 1, 7301)
    dX = capi.to_device(X)
    dO = torch.full((1, n), float("nan"), dtype=torch.complex128, device="cuda")
    print(f"lower-triangle product n={n} ncols=1", flush=True)
    ctx.chase_hemm_step(capi.CHASE_FP64_LOWER, dH, n, n, dX, n, dO, n, 1, 1.0, 0.0, 0.0)
    torch.cuda.synchronize()
    got = capi.from_device(dO)
    del dH, dX, dO
    torch.cuda.empty_cache()
    ref = wl.apply_colmajor_q(U, d, lam[:, None] * wl.apply_colmajor_qh(U, d, X))
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  max error {err:.2e} of max |OUT|")
    assert err <= 1e-13


def test_lower_triangle_argument_errors(ctx):
    import torch
    from paper_1805_10121_amd import capi

    n = 64
    dH = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    dX = torch.zeros((9, n), dtype=torch.complex128, device="cuda")
    dO = torch.zeros((9, n), dtype=torch.complex128, device="cuda")
    with pytest.raises(capi.ChaseError) as ei:           # more than 8 columns
        ctx.chase_hemm_step(capi.CHASE_FP64_LOWER, dH, n, n, dX, n, dO, n, 9, 1.0, 0.0, 0.0)
    assert ei.value.code == capi.CHASE_EINVAL
    with pytest.raises(capi.ChaseError) as ei:           # products only, not the filter
        ctx.chase_filter(capi.CHASE_FP64_LOWER, dH, n, n, dX, dO, n, 2, [2, 2], 2.0, -1.0, 0.0)
    assert ei.value.code == capi.CHASE_EINVAL
