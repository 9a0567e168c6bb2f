"""HBM traffic per filter product from rocprofv3 counter runs.

Reads four ``rocprofv3 --pmc ... -f csv`` output folders:
  * FETCH_SIZE and WRITE_SIZE over a run of ``bench.py`` (the filter products), and
  * FETCH_SIZE and WRITE_SIZE over ``bench.py --copy-calibration`` (a plain 1 GiB device copy,
    run three times).

Both counters are reported in KiB per dispatch by the tool; the copy runs give the factor that
turns each counter into bytes (bytes copied / counted KiB per copy).  The products counted are
the main-kernel dispatches (``hemm_sk_kernel``, ``hemm_dp_kernel``) among the selected ones; a
stream-K product's fixup dispatch adds its counts to the same product.  The result is the JSON
``bench.py`` reads into ``roofline.traffic``, stamped with the hash of the kernel source it was
measured on (``bench.py`` reports null once the source differs).

Usage (from the repository root):
  python -m paper_1805_10121_amd.pmc_traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR \\
      --select Tile3M --out profiles/traffic_hemm_step_fp64_3m_n20000.json
"""

import argparse
import collections
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCE = os.path.join(ROOT, "paper_1805_10121_amd", "csrc", "filter_kernels.hip")
THIN_TILE = "Tile<double, 128, 16"  # the bench's thin-product dispatches, not filter products
COPY_BYTES = 1 << 30
BENCH_RUN = "--headline-only --steps 1 --warmup 0"
COMMANDS = [
    "cd /tmp && rocprofv3 --pmc FETCH_SIZE --kernel-include-regex hemm -f csv -d "
    "<repo>/gpurun_out/pmc_fetch -o fetch -- python3 <repo>/bench.py " + BENCH_RUN,
    "cd /tmp && rocprofv3 --pmc WRITE_SIZE --kernel-include-regex hemm -f csv -d "
    "<repo>/gpurun_out/pmc_write -o write -- python3 <repo>/bench.py " + BENCH_RUN,
    "cd /tmp && rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'copy|elementwise' -f csv -d "
    "<repo>/gpurun_out/pmc_cfetch -o cfetch -- python3 <repo>/bench.py --copy-calibration",
    "cd /tmp && rocprofv3 --pmc WRITE_SIZE --kernel-include-regex 'copy|elementwise' -f csv -d "
    "<repo>/gpurun_out/pmc_cwrite -o cwrite -- python3 <repo>/bench.py --copy-calibration",
]


def read_counters(folder):
    """Rows of the ``*counter_collection.csv`` file in ``folder``."""
    names = [f for f in os.listdir(folder) if f.endswith("counter_collection.csv")]
    if len(names) != 1:
        raise FileNotFoundError(f"expected one counter_collection.csv in {folder}, found {names}")
    with open(os.path.join(folder, names[0]), newline="") as f:
        return list(csv.DictReader(f))


def per_kernel(rows, select="", exclude=""):
    """{short kernel name: [dispatches, summed counter KiB]} over the selected product kernels."""
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        name = r["Kernel_Name"]
        i = name.find("hemm_")
        if i < 0 or THIN_TILE in name or (select and select not in name) or \
                (exclude and exclude in name):
            continue
        short = name[i:].split("<")[0].split("(")[0]
        agg[short][0] += 1
        agg[short][1] += float(r["Counter_Value"])
    return dict(agg)


def copy_factor(rows):
    """Bytes per counted KiB, from the copy kernel's dispatches of the calibration run."""
    vals = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
    if not vals:
        raise ValueError("no copy dispatches in the calibration run")
    kib = sum(vals) / len(vals)
    return COPY_BYTES / 1024.0 / kib, kib


def traffic(fetch_rows, write_rows, copy_fetch_rows, copy_write_rows, select="", exclude="",
            algorithmic_bytes=None):
    """The traffic record: calibrated fetched and written bytes per product."""
    F = per_kernel(fetch_rows, select, exclude)
    W = per_kernel(write_rows, select, exclude)
    products = sum(v[0] for k, v in F.items() if "fixup" not in k)
    if products == 0:
        raise ValueError("no product dispatches selected")
    if products != sum(v[0] for k, v in W.items() if "fixup" not in k):
        raise ValueError("the FETCH_SIZE and WRITE_SIZE runs count different products")
    ff, fkib = copy_factor(copy_fetch_rows)
    wf, wkib = copy_factor(copy_write_rows)
    fetch_b = sum(v[1] for v in F.values()) * 1024 * ff
    write_b = sum(v[1] for v in W.values()) * 1024 * wf
    out = {
        "products_counted": products,
        "hbm_bytes_per_launch": round((fetch_b + write_b) / products),
        "fetch_bytes_per_launch": round(fetch_b / products),
        "write_bytes_per_launch": round(write_b / products),
        "calibration": {"copy_bytes": COPY_BYTES, "FETCH_SIZE_KiB_per_copy": fkib,
                        "WRITE_SIZE_KiB_per_copy": wkib, "fetch_factor": ff, "write_factor": wf},
        "per_kernel_KiB": {k: {"dispatches": F[k][0], "FETCH_SIZE": F[k][1],
                               "WRITE_SIZE": W.get(k, [0, 0.0])[1]} for k in F},
    }
    if algorithmic_bytes is not None:
        out["algorithmic_bytes_per_launch"] = round(algorithmic_bytes)
    return out


def source_hash(path=KERNEL_SOURCE):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("copy_fetch_dir")
    ap.add_argument("copy_write_dir")
    ap.add_argument("--select", default="", help="keep kernels whose name contains this")
    ap.add_argument("--exclude", default="", help="drop kernels whose name contains this")
    ap.add_argument("--kernel", default="", help="description stored with the record")
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--sum-degrees", type=int, default=22788,
                    help="sum of the filter's degrees (active columns summed over its products)")
    ap.add_argument("--products", type=int, default=36, help="products of one filter call")
    ap.add_argument("--command", action="append", default=None,
                    help="the commands that made the counter runs (stored with the record; "
                         "default: the bench's four standard counter runs)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    # algorithmic bytes of one product: H once (16 n^2) plus the read X, read OUT and written
    # OUT blocks (48 n per active column), averaged over the filter's products
    alg = 16 * a.n ** 2 + 48 * a.n * a.sum_degrees / a.products
    rec = traffic(read_counters(a.fetch_dir), read_counters(a.write_dir),
                  read_counters(a.copy_fetch_dir), read_counters(a.copy_write_dir),
                  a.select, a.exclude, alg)
    kernel = a.kernel or (f"FP64 filter product kernels (hemm_*; select {a.select!r}, exclude "
                          f"{a.exclude!r}), bench.py filter workload, n={a.n}")
    rec = {"kernel": kernel, "kernel_source_sha256_16": source_hash(), **rec,
           "commands": a.command or COMMANDS}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: rec[k] for k in ("products_counted", "hbm_bytes_per_launch")}))


if __name__ == "__main__":
    main()
