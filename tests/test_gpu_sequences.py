"""Warm-started sequences (Sec. 3.3, Sec. 6.1) at a reduced size of the order-20000 sequence.

Order 2000, nev = 100, nex = 20 and the clustered spectrum (600 clustered values, the rest in
the bulk), eps = 1e-3 perturbations, 3 problems.  The sequence is solved on the device with the
plain FP64 filter and with the mixed FP32/FP64 filter, state resident between problems
(chase_seq_*), and by the oracle's sequence driver on the same start block and Lanczos start
vectors.  Bars: eigenvalues within 1e-10 * ||H|| of the oracle, of the prescribed spectrum
(problem 1) and of a dense eigensolver (every problem); the difference between the FP64 and the
mixed solves is printed and held to the same bar.
"""

import numpy as np
import pytest

from oracle import chase as och
from paper_1805_10121_amd import workloads as wl

pytestmark = pytest.mark.gpu

N, NEV, NEX, PROBLEMS, EPS = 2000, 100, 20, 3, 1e-3


@pytest.fixture(scope="module")
def problem():
    lam = wl.spectrum_clustered(N, wl.rng(3100), 600)
    Hs = wl.sequence(N, lam, PROBLEMS, EPS, 3101)
    starts = wl.start_block(N, 5, 3103)
    evs = [np.linalg.eigvalsh(H) for H in Hs]
    return lam, Hs, starts, evs


@pytest.fixture(scope="module")
def gpu_runs(problem):
    """Both device solves of the sequence; the start block the library drew is read back so
    the oracle can run on the same inputs."""
    import torch
    from paper_1805_10121_amd import capi

    lam, Hs, starts, _ = problem
    ctx = capi.Context(0)
    dS = capi.to_device(starts)
    dHs = [capi.to_device(H) for H in Hs]
    out = {}
    for name, prec in (("fp64", capi.CHASE_FP64), ("mixed", capi.CHASE_MIXED)):
        cfg = capi.config(N, NEV, NEX, optim=1, seed=3104, precision=prec)
        cfg.lanczos_start = dS.data_ptr()
        seq = capi.Sequence(ctx, cfg)
        ptr, ld = seq.chase_seq_vectors()
        V0 = capi.device_block_to_host(ptr, ld, N, NEV + NEX)
        per = []
        for k, dH in enumerate(dHs):
            print(f"sequence n={N} {name} problem {k + 1}", flush=True)
            ritzv, resid = np.zeros(NEV + NEX), np.zeros(NEV + NEX)
            rc, st = seq.chase_seq_solve(dH, N, ritzv, resid)
            per.append((rc, ritzv.copy(), resid.copy(), st.iterations, st.fp32_iterations))
        ptr, ld = seq.chase_seq_vectors()
        Y = capi.device_block_to_host(ptr, ld, N, NEV + NEX)
        seq.close()
        out[name] = (V0, per, Y)
    torch.cuda.synchronize()
    ctx.close()
    return out


def test_sequence_fp64_and_mixed_against_spectrum(problem, gpu_runs):
    lam, Hs, _, evs = problem
    normH = float(np.max(np.abs(lam)))
    for name in ("fp64", "mixed"):
        _, per, Y = gpu_runs[name]
        for k, (rc, ritzv, resid, it, it32) in enumerate(per):
            assert rc == 0, (name, k)
            err = np.max(np.abs(ritzv[:NEV] - evs[k][:NEV])) / normH
            print(f"{name} problem {k + 1}: {it} iterations ({it32} with FP32 columns), "
                  f"eigenvalue error {err:.2e} x ||H||")
            assert err <= 1e-10
            assert np.max(resid[:NEV]) <= 1e-10 * normH
            if k == 0:
                assert np.max(np.abs(ritzv[:NEV] - lam[:NEV])) <= 1e-10 * normH
        if name == "mixed":
            assert per[0][4] >= 1     # the cold problem filtered some columns in FP32
        # the last problem's eigenvectors: orthonormal, residuals recomputed with a fresh product
        Yn = Y[:, :NEV]
        assert np.linalg.norm(Yn.conj().T @ Yn - np.eye(NEV)) <= 1e-12 * NEV ** 0.5
        R = Hs[-1] @ Yn - Yn * per[-1][1][None, :NEV]
        assert np.max(np.linalg.norm(R, axis=0)) <= 1e-10 * normH * 1.0001
    d = max(np.max(np.abs(a[1][:NEV] - b[1][:NEV]))
            for a, b in zip(gpu_runs["fp64"][1], gpu_runs["mixed"][1])) / normH
    print(f"largest FP64 - mixed eigenvalue difference over the sequence: {d:.2e} x ||H||")
    assert d <= 1e-10


def test_sequence_against_oracle(problem, gpu_runs):
    """The oracle's sequence driver (Alg. 1 per problem, warm start from the previous solution)
    on the start block the FP64 device sequence drew and the same Lanczos start vectors."""
    lam, Hs, starts, _ = problem
    normH = float(np.max(np.abs(lam)))
    V0 = gpu_runs["fp64"][0]
    print("oracle sequence solve", flush=True)
    ref = och.solve_sequence(Hs, och.ChaseParams(nev=NEV, nex=NEX, optim=True), V0,
                             [starts] * PROBLEMS)
    for name in ("fp64", "mixed"):
        for k, r in enumerate(ref):
            assert r["status"] == 0
            got = gpu_runs[name][1][k][1]
            err = np.max(np.abs(got[:NEV] - r["ritzv"][:NEV])) / normH
            print(f"{name} problem {k + 1} vs oracle: {err:.2e} x ||H|| (oracle "
                  f"{r['iterations']} iterations)")
            assert err <= 1e-10
