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


def _run(seqs, order, precision):
    import torch
    from paper_1805_10121_amd import capi

    srv = capi.Server(0, mem_budget_bytes=8 << 30, workers=4)
    dev = {sid: [capi.to_device(H) for H in seqs[sid][3]] for sid in seqs}
    torch.cuda.synchronize()
    tickets = []
    for sid, k in order:
        n, nev, nex, _ = seqs[sid]
        cfg = capi.config(n, nev, nex, optim=1, seed=77 + sid, precision=precision)
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


@pytest.mark.parametrize("precision_name", ["fp64", "mixed"])
def test_alone_equals_mix(precision_name):
    from paper_1805_10121_amd import capi

    precision = capi.CHASE_FP64 if precision_name == "fp64" else capi.CHASE_MIXED
    seqs = _sequences()
    alone_order = [(12, 0), (12, 1), (12, 2)]
    mix_order = [(11, 0), (12, 0), (13, 0), (11, 1), (12, 1), (13, 1), (13, 2), (11, 2), (12, 2)]
    a_res, a_vec, _ = _run(seqs, alone_order, precision)
    m_res, m_vec, info = _run(seqs, mix_order, precision)
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
    srv = capi.Server(0, mem_budget_bytes=need + (1 << 20), workers=2)
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
