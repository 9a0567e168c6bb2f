"""The library's host-side logic, compiled with g++ on the CPU, against the oracle (no GPU).

Covers the filter's product schedule (Alg. 4 / Eq. (7) scalars and active ranges), Alg. 5
(degrees), the tridiagonal eigensolver used on the Lanczos coefficients and the DoS estimate of
mu_{nev+nex} (Alg. 6).  The C++ and the oracle share no code; this test only compares them.
"""

import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import chase as och
from oracle import chebyshev as ch
from oracle import lanczos as lz
from paper_1805_10121_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_10121_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <string>
#include <vector>
#include "host_logic.h"
using namespace chase;
int main() {
  char mode[32];
  if (scanf("%31s", mode) != 1) return 1;
  std::string m(mode);
  if (m == "schedule") {
    long nc; double b, m1, mb; scanf("%ld %lf %lf %lf", &nc, &b, &m1, &mb);
    std::vector<int32_t> d(nc); for (auto& x : d) scanf("%d", &x);
    for (auto& p : filter_schedule(nc, d.data(), b, m1, mb))
      printf("%d %ld %ld %.17g %.17g %.17g\n", p.from_v ? 1 : 0, (long)p.col0, (long)p.ncols, p.alpha, p.beta, p.gamma);
  } else if (m == "degrees") {
    int k, extra, dmax; double tol, c, e; scanf("%d %lf %lf %lf %d %d", &k, &tol, &c, &e, &extra, &dmax);
    for (int i = 0; i < k; ++i) { double r, l; scanf("%lf %lf", &r, &l); printf("%d\n", degree_of(tol, r, l, c, e, extra, dmax)); }
  } else if (m == "tridiag") {
    int nv, k; scanf("%d %d", &nv, &k);
    std::vector<double> al(nv * k), be(nv * k);
    for (auto& x : al) scanf("%lf", &x);
    for (auto& x : be) scanf("%lf", &x);
    for (int c = 0; c < nv; ++c) {
      LanczosRun r = tridiag_eig(al, be, nv, c, k);
      for (int i = 0; i < r.k; ++i) printf("%.17g %.17g\n", r.ritz[i], r.evecs[0 * r.k + i] * r.evecs[0 * r.k + i]);
    }
  } else if (m == "dos") {
    int nv, k; double bsup, sigma, target; scanf("%d %d %lf %lf %lf", &nv, &k, &bsup, &sigma, &target);
    std::vector<double> al(nv * k), be(nv * k);
    for (auto& x : al) scanf("%lf", &x);
    for (auto& x : be) scanf("%lf", &x);
    std::vector<LanczosRun> runs; double lo = 1e300;
    for (int c = 0; c < nv; ++c) { runs.push_back(tridiag_eig(al, be, nv, c, k)); lo = std::min(lo, runs.back().ritz.front()); }
    printf("%.17g %.17g\n", lo, dos_mu(runs, lo, bsup, sigma, target));
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def exe():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "drv.cpp")
    out = os.path.join(d, "drv")
    open(src, "w").write(DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, src, "-o", out], check=True)
    return out


def _run(exe, text):
    return subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout


def test_filter_schedule_matches_oracle(exe):
    g = wl.rng(1)
    for _ in range(5):
        nc = int(g.integers(1, 40))
        deg = np.sort(2 * g.integers(1, 19, nc)).astype(int)
        b, m1, mb = 2.1, -1.05, float(g.uniform(-0.6, 0.5))
        out = _run(exe, f"schedule {nc} {b!r} {m1!r} {mb!r} " + " ".join(map(str, deg)))
        rows = [ln.split() for ln in out.strip().splitlines()]
        ref = ch.filter_scalars(int(deg.max()), b, m1, mb)
        assert len(rows) == int(deg.max())
        for i, r in enumerate(rows, start=1):
            a, bb, gg = map(float, r[3:])
            assert np.allclose([a, bb, gg], ref[i - 1], rtol=1e-14, atol=0)
            # active columns at product i: degrees >= i; buffers alternate V->W, W->V, ...
            assert int(r[1]) == int(np.searchsorted(deg, i, side="left")) if i > 1 else int(r[1]) == 0
            assert int(r[2]) == nc - int(r[1])
            assert int(r[0]) == (1 if i % 2 == 1 else 0)


def test_degrees_match_oracle(exe):
    g = wl.rng(2)
    k = 300
    res = 10.0 ** g.uniform(-13, 0, k)
    ritz = g.uniform(-1.5, 1.2, k)
    c, e, tol = 0.8, 1.1, 1e-10
    text = f"degrees {k} {tol!r} {c!r} {e!r} 2 36 " + " ".join(f"{float(r)!r} {float(l)!r}" for r, l in zip(res, ritz))
    got = np.array([int(x) for x in _run(exe, text).split()])
    ref = och.degrees(tol, res, ritz, c, e, 2, 36)
    assert np.array_equal(got, ref)


def test_tridiagonal_eigensolver_and_dos_match_oracle(exe):
    n = 500
    g = wl.rng(3)
    lam = wl.spectrum_uniform(n, g)
    A = wl.hermitian_from(wl.haar_unitary(n, g), lam)
    nv, k = 4, 25
    al = np.zeros((k, nv))
    be = np.zeros((k, nv))
    runs = []
    for c in range(nv):
        a, b, _ = lz.lanczos_run(A, wl.complex_gaussian(g, n), k)
        al[:, c], be[:, c] = a, b
        runs.append((a, b))
    flat = " ".join(f"{float(x)!r}" for x in al.ravel()) + " " + " ".join(f"{float(x)!r}" for x in be.ravel())
    out = _run(exe, f"tridiag {nv} {k} " + flat).split()
    vals = np.array(out, dtype=float).reshape(nv, k, 2)
    for c in range(nv):
        ev, S = np.linalg.eigh(lz.tridiagonal(al[:, c], be[:, c]))
        assert np.allclose(vals[c, :, 0], ev, atol=1e-13)
        assert np.allclose(vals[c, :, 1], np.abs(S[0, :]) ** 2, atol=1e-12)
    b_sup = lz.upper_bound(al[:, 0], be[:, 0])
    mu1_ref, mub_ref = lz.dos_estimates(runs, b_sup, 40, 10, n, 0.25)
    lo, mub = map(float, _run(exe, f"dos {nv} {k} {float(b_sup)!r} 0.25 {50 / n!r} " + flat).split())
    assert lo == pytest.approx(mu1_ref, abs=1e-13)
    assert mub == pytest.approx(mub_ref, abs=1e-9)


SCHED_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "host_logic.h"
using namespace chase;
// Exhaustive check of the product kernel's stream-K schedule over many shapes: every unit has
// exactly one owner; each workgroup writes at most one partial per slot; every split tile gets
// exactly one fixup workgroup, whose contributor range [pf, pl] and slot choice match what the
// contributors wrote; tiles finished in place get no fixup; the XCD order is a permutation.
int main() {
  long checked = 0;
  const int nks[] = {1, 2, 3, 7, 16, 63, 625, 1250};
  const long Ps[] = {1, 2, 3, 8, 64, 256, 512, 768, 1024};
  for (long tiles = 1; tiles <= 3000; tiles = tiles < 40 ? tiles + 1 : tiles * 3 / 2 + 1)
    for (int nk : nks)
      for (long P0 : Ps)
        for (int hybrid = 0; hybrid < 2; ++hybrid) {
          const SkPlan pl = sk_plan(tiles, nk, P0, hybrid);
          if (pl.P < 1 || pl.dp_tiles % P0 != 0 || pl.dp_tiles > tiles) return 1;
          if (pl.units != (tiles - pl.dp_tiles) * nk) return 2;
          if (pl.units == 0) continue;
          const long U = pl.units, P = pl.P, T = tiles - pl.dp_tiles;
          std::vector<int> owner(U, -1);
          std::vector<int> contributors(T, 0), written(2 * P, -1);
          for (long p = 0; p < P; ++p) {
            const long u0 = sk_start(p, U, P), u1 = sk_start(p + 1, U, P);
            for (long u = u0; u < u1; ++u) {
              if (owner[u] != -1 || sk_owner(u, U, P) != p) return 3;
              owner[u] = p;
            }
            long u = u0;
            while (u < u1) {
              const SkSegment sg = sk_segment(u, u1, nk);
              if (sg.ka < 0 || sg.kb <= sg.ka || sg.kb > nk) return 4;
              ++contributors[sg.tile];
              if (!(sg.ka == 0 && sg.kb == nk)) {  // partial: one slot per segment
                const int slot = sk_slot(p, sg.tile, U, P, nk);
                if (written[2 * p + slot] != -1) return 5;
                written[2 * p + slot] = static_cast<int>(sg.tile);
              }
              u = sg.tile * nk + sg.kb;
            }
          }
          for (long u = 0; u < U; ++u)
            if (owner[u] == -1) return 6;
          std::vector<int> fixups(T, 0);
          for (long q = 0; q < P; ++q) {
            const long tr = sk_fixup_tile(q, U, P, nk);
            if (tr < 0) continue;
            ++fixups[tr];
            const long pf = sk_owner(tr * nk, U, P), pl2 = sk_owner((tr + 1) * nk - 1, U, P);
            for (long pp = pf; pp <= pl2; ++pp) {
              const long a = sk_start(pp, U, P), b = sk_start(pp + 1, U, P);
              if (a >= b) continue;
              if (written[2 * pp + sk_slot(pp, tr, U, P, nk)] != tr) return 7;
            }
          }
          for (long t = 0; t < T; ++t)
            if ((contributors[t] > 1) != (fixups[t] == 1) || fixups[t] > 1) return 8;
          std::vector<char> seen(P0, 0);
          for (long p = 0; p < P0; ++p) {
            const long q = xcd_order(p, P0);
            if (q < 0 || q >= P0 || seen[q]) return 9;
            seen[q] = 1;
          }
          ++checked;
        }
  printf("%ld\n", checked);
  return 0;
}
"""


def test_stream_k_schedule_exhaustive():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "sched.cpp")
    out = os.path.join(d, "sched")
    open(src, "w").write(SCHED_DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, src, "-o", out], check=True)
    r = subprocess.run([out], capture_output=True, text=True)
    assert r.returncode == 0, f"schedule check {r.returncode}"
    assert int(r.stdout) > 1000


GRAM_DRIVER = r"""
#include <cstdio>
#include "host_logic.h"
using namespace chase;
// The solver's use of the K-sliced Gram product: slices in [1, 16], each at least 256 rows when
// there is more than one, and -- after the solver's cap -- all slices inside the reserved buffer
// for every result shape up to nb x nb (cgs: nlock x nact with nlock + nact = nb).
int main() {
  long checked = 0;
  for (long nb : {1L, 5L, 64L, 70L, 300L, 600L, 1200L, 2400L, 4000L})
    for (long n : {nb, 2 * nb, 1000L, 10000L, 60000L}) {
      if (n < nb) continue;
      const long cap = gram_buffer_elems(nb);
      if (cap < nb * nb) return 1;
      for (long m1 = 1; m1 <= nb; m1 += (nb > 64 ? 7 : 1))
        for (long m2 : {nb - m1 > 0 ? nb - m1 : 1L, m1}) {
          long p = gram_slices(m1, m2, n);
          if (p < 1 || p > 16) return 2;
          if (p > 1 && p * 256 > n) return 3;
          if (p * m1 * m2 > cap) p = cap / (m1 * m2);
          if (p < 1 || p * m1 * m2 > cap) return 4;
          ++checked;
        }
    }
  printf("%ld\n", checked);
  return 0;
}
"""


def test_gram_slices_fit_the_buffer():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "gram.cpp")
    out = os.path.join(d, "gram")
    open(src, "w").write(GRAM_DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, src, "-o", out], check=True)
    r = subprocess.run([out], capture_output=True, text=True)
    assert r.returncode == 0, f"gram slice check {r.returncode}"
    assert int(r.stdout) > 1000


DP_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "host_logic.h"
using namespace chase;
int main() {
  long checked = 0;
  for (long G = 1; G <= 5000; G += (G < 600 ? 1 : 7)) {
    std::vector<char> seen(G, 0);
    for (long b = 0; b < G; ++b) {
      const long t = dp_tile(b, G);
      if (t < 0 || t >= G || seen[t]) return 1;
      seen[t] = 1;
      // inside a full window, the workgroups of one XCD (b % 8) hold kDpChunk consecutive tiles
      const long W = 8 * kDpChunk;
      if ((b / W + 1) * W <= G && t / kDpChunk != (b / W) * 8 + (b % W) % 8) return 2;
    }
    ++checked;
  }
  printf("%ld\n", checked);
  return 0;
}
"""


def test_dp_tile_order_is_a_bijection():
    """The data-parallel grid's XCD-aware tile order visits every tile exactly once, and gives
    each XCD's workgroups of a full window consecutive tiles."""
    d = tempfile.mkdtemp()
    src = os.path.join(d, "dp.cpp")
    out = os.path.join(d, "dp")
    open(src, "w").write(DP_DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, src, "-o", out], check=True)
    r = subprocess.run([out], capture_output=True, text=True)
    assert r.returncode == 0, r.returncode
    assert int(r.stdout) > 1000


GROUP_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "host_logic.h"
using namespace chase;
int main() {
  long checked = 0;
  for (long tm = 1; tm <= 70; ++tm)
    for (long tn = 1; tn <= 40; tn += (tn < 20 ? 1 : 3)) {
      std::vector<char> seen(tm * tn, 0);
      for (long t = 0; t < tm * tn; ++t) {
        const TileMN c = grouped_tile(t, tm, tn);
        if (c.m < 0 || c.m >= tm || c.n < 0 || c.n >= tn || seen[c.m * tn + c.n]) return 1;
        seen[c.m * tn + c.n] = 1;
        // inside a full group, kTileGroupRows consecutive positions are one column tile
        const long g = t / (kTileGroupRows * tn);
        if ((g + 1) * kTileGroupRows <= tm &&
            (c.n != (t % (kTileGroupRows * tn)) / kTileGroupRows ||
             c.m != g * kTileGroupRows + t % kTileGroupRows))
          return 2;
      }
      ++checked;
    }
  printf("%ld\n", checked);
  return 0;
}
"""


def test_grouped_tile_order_is_a_bijection():
    """The product kernels' grouped tile order visits every output tile once, ragged last group
    included, and walks a full group column by column."""
    d = tempfile.mkdtemp()
    src = os.path.join(d, "grp.cpp")
    out = os.path.join(d, "grp")
    open(src, "w").write(GROUP_DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, src, "-o", out], check=True)
    r = subprocess.run([out], capture_output=True, text=True)
    assert r.returncode == 0, r.returncode
    assert int(r.stdout) > 1000
