"""Whole-space solves (nev + nex = n) in FP64, FP32 and mixed precision (pending a GPU run)."""

import numpy as np
import pytest

from paper_1805_10121_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1805_10121_amd import capi

    c = capi.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "mixed"])
def test_search_space_is_the_whole_space(ctx, precision):
    # nev + nex = n: the search space is all of C^n, so after one orthonormalisation the
    # Rayleigh-Ritz step is exact; Lanczos runs k = min(k, n) steps (n = 24 < k = 25)
    import torch
    from paper_1805_10121_amd import capi

    n, nev, nex = 24, 20, 4
    g = wl.rng(97)
    lam = wl.spectrum_uniform(n, g)
    H = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    V0, S = wl.complex_gaussian(g, n, n), wl.complex_gaussian(g, n, 5)
    if precision == "fp32":
        cfg = capi.config_fp32(n, nev, nex, optim=1)
        dt = torch.complex64
        tol = 2e-5
    else:
        cfg = capi.config(n, nev, nex, optim=1,
                          precision=capi.CHASE_MIXED if precision == "mixed" else capi.CHASE_FP64)
        dt = torch.complex128
        tol = 1e-10
    dS = capi.to_device(S).to(dt)
    cfg.lanczos_start = dS.data_ptr()
    dH, dV = capi.to_device(H).to(dt), capi.to_device(V0).to(dt)
    ritzv, resid = np.zeros(n), np.zeros(n)
    rc, st = ctx.chase_solve(cfg, dH, n, dV, n, ritzv, resid)
    assert rc == 0 and st.nconv >= nev
    normH = np.max(np.abs(lam))
    assert np.max(np.abs(ritzv[:nev] - lam[:nev])) <= tol * normH
    Y = capi.from_device(dV).astype(np.complex128)
    assert np.linalg.norm(Y[:, :nev].conj().T @ Y[:, :nev] - np.eye(nev)) <= (1e-4 if precision == "fp32" else 1e-12)
