"""The C ABI without a GPU: the library loads, exports every symbol the header declares, the
ctypes structures match the C layout, and chase_config_init fills Table 1's defaults."""

import ctypes
import json
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chase.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(chase_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_1805_10121_amd import capi

    L = capi.lib()
    declared = _declared_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(declared) == sorted(capi.exported_symbols())


def test_struct_layout_matches_c():
    from paper_1805_10121_amd import capi

    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "chase.h"
#define F(T, m) printf("%s %zu\n", #m, offsetof(T, m));
int main(void) {
  printf("sizeof_config %zu\nsizeof_stats %zu\n", sizeof(chase_config), sizeof(chase_stats));
  F(chase_config, approx) F(chase_config, tol) F(chase_config, precision)
  F(chase_config, switch_resid) F(chase_config, dos_sigma) F(chase_config, seed)
  F(chase_config, lanczos_start) F(chase_config, have_mu) F(chase_config, mu_nevnex)
  F(chase_config, verbose) F(chase_config, real_symmetric) F(chase_config, filter_3m)
  F(chase_stats, matvecs) F(chase_stats, filter_flops) F(chase_stats, norm_est)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    vals = dict(line.split() for line in out.strip().splitlines())
    assert int(vals["sizeof_config"]) == ctypes.sizeof(capi.chase_config)
    assert int(vals["sizeof_stats"]) == ctypes.sizeof(capi.chase_stats)
    for f in ["approx", "tol", "precision", "switch_resid", "dos_sigma", "seed", "lanczos_start",
              "have_mu", "mu_nevnex", "verbose", "real_symmetric", "filter_3m"]:
        assert int(vals[f]) == getattr(capi.chase_config, f).offset, f
    for f in ["matvecs", "filter_flops", "norm_est"]:
        assert int(vals[f]) == getattr(capi.chase_stats, f).offset, f


def test_config_defaults_are_table1():
    from paper_1805_10121_amd import capi

    with open(os.path.join(ROOT, "tests", "golden", "table1_defaults.json")) as f:
        t1 = json.load(f)["double"]
    cfg = capi.config(1000, 50, 20)
    assert (cfg.n, cfg.nev, cfg.nex) == (1000, 50, 20)
    assert cfg.approx == int(t1["approx"]) and cfg.tol == t1["tol"]
    assert cfg.max_iter == t1["max_iter"] and cfg.optim == int(t1["optim"])
    assert cfg.deg_extra == t1["deg_extra"] and cfg.deg_max == t1["deg_max"] and cfg.deg == t1["deg"]
    assert cfg.lanczos_iter == t1["lanczos_iter"] and cfg.num_lanczos == t1["num_lanczos"]
    assert cfg.deg_max_fp32 == 18 and cfg.dos_sigma == 0.25 and cfg.precision == capi.CHASE_FP64


def test_workspace_bytes_is_pure_host():
    from paper_1805_10121_amd import capi

    cfg = capi.config(10000, 500, 100)
    b = capi.lib().chase_workspace_bytes(ctypes.byref(cfg))
    assert b >= 3 * 10000 * 600 * 16
    # real symmetric data: 8-byte elements, so about half the complex workspace
    cfg.real_symmetric = 1
    br = capi.lib().chase_workspace_bytes(ctypes.byref(cfg))
    assert 3 * 10000 * 600 * 8 <= br < 0.6 * b


def test_config_init_fp32_table1_single_precision():
    # Table 1: the values in parentheses are the single-precision defaults
    from paper_1805_10121_amd import capi

    c = capi.config_fp32(1000, 40, 10)
    d = capi.config(1000, 40, 10)
    assert c.precision == capi.CHASE_FP32
    assert (c.tol, c.deg_max, c.deg, c.lanczos_iter) == (1e-5, 18, 10, 12)
    assert (c.max_iter, c.deg_extra, c.num_lanczos, c.optim, c.approx) == (25, 2, 4, 0, 0)
    for f in ("switch_resid", "deg_max_fp32", "resid_relative", "intersperse", "dos_sigma",
              "seed", "have_mu", "verbose", "real_symmetric"):
        assert getattr(c, f) == getattr(d, f), f
    capi.lib().chase_config_init_fp32(None, 1, 1, 0)  # NULL is ignored


def test_workspace_bytes_planar_copy_for_3m():
    # filter_3m = 1 (default) reserves the planar complex128 copy of H; 0 does not
    from paper_1805_10121_amd import capi

    n = 3000
    on = capi.lib().chase_workspace_bytes(ctypes.byref(capi.config(n, 100, 20)))
    off = capi.lib().chase_workspace_bytes(ctypes.byref(capi.config(n, 100, 20, filter_3m=0)))
    real = capi.lib().chase_workspace_bytes(ctypes.byref(capi.config(n, 100, 20, real_symmetric=1)))
    real_off = capi.lib().chase_workspace_bytes(
        ctypes.byref(capi.config(n, 100, 20, real_symmetric=1, filter_3m=0)))
    assert 16 * n * n <= on - off <= 16 * n * n + 256
    assert real == real_off   # real data has no 3M form


def test_workspace_bytes_fp32_half_of_fp64():
    from paper_1805_10121_amd import capi

    n = 5000
    for real in (0, 1):
        c64 = capi.config(n, 200, 40, lanczos_iter=12, real_symmetric=real)
        c32 = capi.config_fp32(n, 200, 40, real_symmetric=real)
        b64 = capi.lib().chase_workspace_bytes(ctypes.byref(c64))
        b32 = capi.lib().chase_workspace_bytes(ctypes.byref(c32))
        # complex: each holds a planar copy of H for its 3M filter (16 n^2 bytes for complex128,
        # 8 n^2 for complex64)
        p64, p32 = (0, 0) if real else (16 * n * n, 8 * n * n)
        assert 0.45 * (b64 - p64) <= b32 - p32 <= 0.55 * (b64 - p64)


def test_create_without_gpu_fails_cleanly():
    import torch
    from paper_1805_10121_amd import capi

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert capi.lib().chase_create(ctypes.byref(h), 0, None) == capi.CHASE_EDEVICE
    assert not h.value


def test_bench_refuses_more_than_one_gpu():
    # the bench measures one GPU; asking for more exits with status 2 before touching a device
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
