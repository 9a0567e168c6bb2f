"""Serving (chase_server_*): continuous batching of solves from several sequences of uneven order.

The bar: each request's result is the same alone and in the mix (bitwise: every product runs in
data-parallel tiles whose arithmetic does not depend on the grouping), and every result meets
the solver's accuracy bars against a dense eigensolver.
"""

import numpy as np
import pytest

from paper_1805_10121_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _sequences():
    specs = [(11, 300, 12, 4), (12, 520, 20, 6), (13, 900, 30, 8)]
    out = {}
    for sid, n, nev, nex in specs:
        g = wl.rng(sid)
        lam = wl.spectrum_clustered(n, g, n // 10)
        out[sid] = (n, nev, nex, wl.sequence(n, lam, 3, 1e-3, 500 + sid))
    return out


def _run(seqs, order, precision, filter_3m=1):
    import torch
    from paper_1805_10121_amd import capi

    srv = capi.Server(0, mem_budget_bytes=16 << 30, workers=4)
    dev = {sid: [capi.to_device(H) for H in seqs[sid][3]] for sid in seqs}
    torch.cuda.synchronize()
    tickets = []
    for sid, k in order:
        n, nev, nex, _ = seqs[sid]
        cfg = capi.config(n, nev, nex, optim=1, seed=77 + sid, precision=precision,
                          filter_3m=filter_3m)
        tickets.append((sid, k, srv.chase_server_submit(sid, cfg, dev[sid][k], n)))
    res = {}
    for sid, k, t in tickets:
        rc, ritzv, resid, st, lat = srv.chase_server_poll(t, wait=True)
        res[(sid, k)] = (rc, ritzv, resid, st.iterations)
    vecs = {}
    for sid in {s for s, _ in order}:
        ptr, ld = srv.chase_server_vectors(sid)
        n, nev, nex, _ = seqs[sid]
        vecs[sid] = capi.device_block_to_host(ptr, ld, n, nev + nex)
    info = srv.chase_server_info()
    srv.close()
    return res, vecs, info


@pytest.mark.parametrize("precision_name,filter_3m", [("fp64", 1), ("fp64", 0), ("mixed", 1)])
def test_alone_equals_mix(precision_name, filter_3m):
    """Grouped FP64 products in both schemes (3M on each solve's planar copy of H, the default,
    and 4M on H itself) and the mixed solver's grouped FP32 3M and FP64 3M products."""
    from paper_1805_10121_amd import capi

    precision = capi.CHASE_FP64 if precision_name == "fp64" else capi.CHASE_MIXED
    seqs = _sequences()
    alone_order = [(12, 0), (12, 1), (12, 2)]
    mix_order = [(11, 0), (12, 0), (13, 0), (11, 1), (12, 1), (13, 1), (13, 2), (11, 2), (12, 2)]
    a_res, a_vec, _ = _run(seqs, alone_order, precision, filter_3m)
    m_res, m_vec, info = _run(seqs, mix_order, precision, filter_3m)
    assert info["grouped_products"] > info["grouped_launches"] > 0
    for k in range(3):
        ra, rm = a_res[(12, k)], m_res[(12, k)]
        assert ra[0] == 0 and rm[0] == 0
        assert np.array_equal(ra[1], rm[1]), "Ritz values differ alone vs mix"
        assert np.array_equal(ra[2], rm[2])
    assert np.array_equal(a_vec[12], m_vec[12]), "vectors differ alone vs mix"
    for (sid, k), (rc, ritzv, resid, it) in m_res.items():
        n, nev, nex, Hs = seqs[sid]
        ev = np.linalg.eigvalsh(Hs[k])
        assert rc == 0
        assert np.max(np.abs(ritzv[:nev] - ev[:nev])) <= 1e-10 * np.max(np.abs(ev))


def test_budget_and_sequence_rules():
    import torch
    from paper_1805_10121_amd import capi

    n, nev, nex = 400, 10, 4
    g = wl.rng(5)
    lam = wl.spectrum_uniform(n, g)
    H = capi.to_device(wl.hermitian_from(wl.haar_unitary(n, g), lam))
    cfg = capi.config(n, nev, nex, optim=1)
    need = capi.lib().chase_workspace_bytes(__import__("ctypes").byref(cfg)) + n * (nev + nex) * 16
    # the server's fixed allocations (batcher scratch, per-worker product scratch and handle
    # allowance) are charged at creation and reported as bytes in use
    probe = capi.Server(0, mem_budget_bytes=64 << 30, workers=2)
    fixed = probe.chase_server_info()["bytes_in_use"]
    probe.close()
    assert fixed > 0
    with pytest.raises(capi.ChaseError):                            # budget below the fixed part
        capi.Server(0, mem_budget_bytes=fixed, workers=2)
    srv = capi.Server(0, mem_budget_bytes=fixed + need + (1 << 20), workers=2)
    with pytest.raises(capi.ChaseError) as ei:                      # alone above the budget
        big = capi.config(4 * n, 4 * nev, nex, optim=1)
        srv.chase_server_submit(9, big, H, 4 * n)
    assert ei.value.code == capi.CHASE_EBUSY
    t1 = srv.chase_server_submit(1, cfg, H, n)
    with pytest.raises(capi.ChaseError) as ei:                      # size change in a sequence
        srv.chase_server_submit(1, capi.config(n, nev + 1, nex), H, n)
    assert ei.value.code == capi.CHASE_EINVAL
    rc, ritzv, *_ = srv.chase_server_poll(t1, wait=True)
    assert rc == 0 and np.max(np.abs(ritzv[:nev] - lam[:nev])) <= 1e-10
    # only one sequence state fits: sequence 2 runs after sequence 1 is released
    assert srv.chase_server_end_sequence(1) == 0
    t2 = srv.chase_server_submit(2, cfg, H, n)
    rc, ritzv, *_ = srv.chase_server_poll(t2, wait=True)
    assert rc == 0 and np.max(np.abs(ritzv[:nev] - lam[:nev])) <= 1e-10
    srv.close()
    torch.cuda.synchronize()


def test_real_sequence_in_server_matches_direct():
    # A real symmetric sequence served beside complex ones gives the same Ritz values, bitwise,
    # as the same sequence solved directly with chase_seq_* (real products run on the worker's
    # stream, outside the cross-solve batcher).
    import torch
    from paper_1805_10121_amd import capi

    n, nev, nex = 400, 16, 6
    g = wl.rng(21)
    lam = wl.spectrum_uniform(n, g)
    H0 = wl.symmetric_from(wl.haar_orthogonal(n, g), lam)
    Hs = [H0]
    for _ in range(2):
        E = g.standard_normal((n, n))
        E = 0.5 * (E + E.T)
        Hs.append(Hs[-1] + 1e-3 * E / np.max(np.abs(np.linalg.eigvalsh(E))))
    cfg = capi.config(n, nev, nex, optim=1, seed=31, real_symmetric=1)
    dev = [capi.to_device(H) for H in Hs]
    torch.cuda.synchronize()
    ctx = capi.Context(0)
    seq = capi.Sequence(ctx, cfg)
    direct = []
    for dH in dev:
        r, s = np.zeros(nev + nex), np.zeros(nev + nex)
        seq.chase_seq_solve(dH, n, r, s)
        direct.append(r.copy())
    seq.close()
    ctx.close()
    seqs = _sequences()
    cplx = {sid: [capi.to_device(H) for H in seqs[sid][3]] for sid in (11, 13)}
    torch.cuda.synchronize()
    srv = capi.Server(0, mem_budget_bytes=8 << 30, workers=4)
    tickets = []
    for k in range(3):
        tickets.append(("real", k, srv.chase_server_submit(99, cfg, dev[k], n)))
        for sid in (11, 13):
            cn, cnev, cnex, _ = seqs[sid]
            ccfg = capi.config(cn, cnev, cnex, optim=1, seed=77 + sid)
            tickets.append((sid, k, srv.chase_server_submit(sid, ccfg, cplx[sid][k], cn)))
    served = {}
    for sid, k, t in tickets:
        rc, ritzv, resid, st, lat = srv.chase_server_poll(t, wait=True)
        assert rc == 0
        if sid == "real":
            served[k] = ritzv.copy()
            ev = np.linalg.eigvalsh(Hs[k])
            assert np.max(np.abs(ritzv[:nev] - ev[:nev])) <= 1e-10 * np.max(np.abs(ev))
    ptr, ld = srv.chase_server_vectors(99)
    Y = capi.device_block_to_host(ptr, ld, n, nev + nex, dtype=np.float64)
    srv.close()
    for k in range(3):
        assert np.array_equal(served[k], direct[k])
    Yn = Y[:, :nev]
    assert np.linalg.norm(Yn.T @ Yn - np.eye(nev)) <= 1e-12 * nev ** 0.5


def test_fp32_sequence_in_server_matches_direct():
    # A single-precision (complex64) sequence served beside FP64 ones gives bitwise the Ritz
    # values of the same sequence solved directly; switching its precision is refused.
    import torch
    from paper_1805_10121_amd import capi

    n, nev, nex = 400, 16, 6
    seqs = _sequences()
    g = wl.rng(23)
    lam = wl.spectrum_uniform(n, g)
    Hs = wl.sequence(n, lam, 3, 1e-3, 523)
    cfg = capi.config_fp32(n, nev, nex, optim=1, seed=33)
    dev = [capi.to_device(H).to(torch.complex64) for H in Hs]
    torch.cuda.synchronize()
    ctx = capi.Context(0)
    seq = capi.Sequence(ctx, cfg)
    direct = []
    for dH in dev:
        r, s = np.zeros(nev + nex), np.zeros(nev + nex)
        seq.chase_seq_solve(dH, n, r, s)
        direct.append(r.copy())
    seq.close()
    ctx.close()
    cplx = {sid: [capi.to_device(H) for H in seqs[sid][3]] for sid in (11, 13)}
    torch.cuda.synchronize()
    srv = capi.Server(0, mem_budget_bytes=8 << 30, workers=4)
    tickets = []
    for k in range(3):
        tickets.append(("fp32", k, srv.chase_server_submit(98, cfg, dev[k], n)))
        for sid in (11, 13):
            cn, cnev, cnex, _ = seqs[sid]
            ccfg = capi.config(cn, cnev, cnex, optim=1, seed=77 + sid)
            tickets.append((sid, k, srv.chase_server_submit(sid, ccfg, cplx[sid][k], cn)))
    # the sequence's state is complex64: a complex128 request for it is refused
    with pytest.raises(capi.ChaseError):
        srv.chase_server_submit(98, capi.config(n, nev, nex, optim=1), cplx[13][0], n)
    served = {}
    for sid, k, t in tickets:
        rc, ritzv, resid, st, lat = srv.chase_server_poll(t, wait=True)
        assert rc == 0
        if sid == "fp32":
            served[k] = ritzv.copy()
            ev = np.linalg.eigvalsh(Hs[k])
            assert np.max(np.abs(ritzv[:nev] - ev[:nev])) <= 2e-5 * np.max(np.abs(ev))
    srv.close()
    for k in range(3):
        assert np.array_equal(served[k], direct[k])


def test_config4_sizes_alone_equals_mix():
    """Serving-size solves (orders 2000 and 4000, nev = 5 % of n, nex = 20 % of nev, clustered
    spectrum, eps = 1e-3, mixed filter) beside a small sequence: the order-4000 sequence gives
    bitwise the same Ritz values, residuals and vectors alone and in the mix, and every served
    result meets the 1e-10 * ||H|| bar against a dense eigensolver."""
    from paper_1805_10121_amd import capi

    seqs = {}
    for sid, n in ((21, 2000), (22, 4000)):
        nev = round(0.05 * n)
        nex = round(0.2 * nev)
        lam = wl.spectrum_clustered(n, wl.rng(600 + sid), 600)
        print(f"serving sizes: generating order {n}", flush=True)
        seqs[sid] = (n, nev, nex, wl.sequence(n, lam, 3, 1e-3, 700 + sid))
    seqs[11] = _sequences()[11]
    alone_order = [(22, 0), (22, 1), (22, 2)]
    mix_order = [(21, 0), (22, 0), (11, 0), (22, 1), (21, 1), (11, 1), (21, 2), (22, 2), (11, 2)]
    print("serving sizes: alone", flush=True)
    a_res, a_vec, _ = _run(seqs, alone_order, capi.CHASE_MIXED)
    print("serving sizes: mix", flush=True)
    m_res, m_vec, info = _run(seqs, mix_order, capi.CHASE_MIXED)
    assert info["grouped_products"] > info["grouped_launches"] > 0
    for k in range(3):
        ra, rm = a_res[(22, k)], m_res[(22, k)]
        assert ra[0] == 0 and rm[0] == 0
        assert np.array_equal(ra[1], rm[1]), "Ritz values differ alone vs mix"
        assert np.array_equal(ra[2], rm[2])
    assert np.array_equal(a_vec[22], m_vec[22]), "vectors differ alone vs mix"
    for (sid, k), (rc, ritzv, resid, it) in sorted(m_res.items()):
        n, nev, nex, Hs = seqs[sid]
        ev = np.linalg.eigvalsh(Hs[k])
        err = np.max(np.abs(ritzv[:nev] - ev[:nev])) / np.max(np.abs(ev))
        print(f"served order {n} problem {k + 1}: {it} iterations, error {err:.2e} x ||H||")
        assert rc == 0 and err <= 1e-10
