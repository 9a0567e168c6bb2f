"""The counter aggregation behind roofline.traffic, on small synthetic rocprofv3 CSV files:
selection of the product kernels, copy calibration, per-product averages, and the checks that
refuse inconsistent runs."""

import csv
import os

import pytest

from paper_1805_10121_amd import pmc_traffic as pt

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
SK3M = "void chase::(anonymous namespace)::hemm_sk_kernel<double, chase::Tile3M<64, 64, 16, 2, 2, 4, 0, double>, 2, false>(double const*)"
FIX3M = "void chase::(anonymous namespace)::hemm_fixup_kernel<double, chase::Tile3M<64, 64, 16, 2, 2, 4, 0, double> >(double const*)"
SK4M = "void chase::(anonymous namespace)::hemm_sk_kernel<double, chase::Tile<double, 64, 64, 16>, 2, false>(double const*)"
THIN = "void chase::(anonymous namespace)::hemm_sk_kernel<double, chase::Tile<double, 128, 16, 16>, 2, false>(double const*)"


def _folder(tmp_path, name, rows, counter):
    d = tmp_path / name
    d.mkdir()
    with open(d / f"{name}_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (k, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": k, "Counter_Name": counter,
                        "Counter_Value": v})
    return str(d)


def _runs(tmp_path, write_products=2):
    fetch = [(SK3M, 1000.0), (FIX3M, 10.0), (SK3M, 3000.0), (FIX3M, 30.0), (SK4M, 9e9), (THIN, 7e9)]
    write = [(SK3M, 100.0), (FIX3M, 1.0), (SK3M, 300.0), (FIX3M, 3.0), (SK4M, 9e9), (THIN, 7e9)]
    if write_products == 1:
        write = write[:2]
    copy_f = [("void at::native::vectorized_elementwise_kernel<4, FillFunctor<double>>", 22.0)] + \
             [("__amd_rocclr_copyBuffer", 524288.0)] * 3
    copy_w = [("__amd_rocclr_copyBuffer", 1048576.0)] * 3
    return (pt.read_counters(_folder(tmp_path, "fetch", fetch, "FETCH_SIZE")),
            pt.read_counters(_folder(tmp_path, "write", write, "WRITE_SIZE")),
            pt.read_counters(_folder(tmp_path, "cfetch", copy_f, "FETCH_SIZE")),
            pt.read_counters(_folder(tmp_path, "cwrite", copy_w, "WRITE_SIZE")))


def test_selected_products_and_calibration(tmp_path):
    F, W, CF, CW = _runs(tmp_path)
    rec = pt.traffic(F, W, CF, CW, select="Tile3M", algorithmic_bytes=123.4)
    # 1 GiB copy counted as 524288 KiB fetched (factor 2) and 1048576 KiB written (factor 1)
    assert rec["calibration"]["fetch_factor"] == 2.0
    assert rec["calibration"]["write_factor"] == 1.0
    assert rec["products_counted"] == 2
    fetch = (1000 + 10 + 3000 + 30) * 1024 * 2.0 / 2
    write = (100 + 1 + 300 + 3) * 1024 * 1.0 / 2
    assert rec["fetch_bytes_per_launch"] == round(fetch)
    assert rec["write_bytes_per_launch"] == round(write)
    assert rec["hbm_bytes_per_launch"] == round(fetch + write)
    assert rec["algorithmic_bytes_per_launch"] == 123
    assert rec["per_kernel_KiB"]["hemm_fixup_kernel"] == {"dispatches": 2, "FETCH_SIZE": 40.0,
                                                          "WRITE_SIZE": 4.0}


def test_exclusion_and_thin_tile(tmp_path):
    F, W, CF, CW = _runs(tmp_path)
    rec = pt.traffic(F, W, CF, CW, exclude="Tile3M")
    # only the 4M dispatch is left: the thin-tile dispatch is never a filter product
    assert rec["products_counted"] == 1
    assert rec["fetch_bytes_per_launch"] == round(9e9 * 1024 * 2.0)


def test_inconsistent_runs_are_refused(tmp_path):
    F, W, CF, CW = _runs(tmp_path, write_products=1)
    with pytest.raises(ValueError):
        pt.traffic(F, W, CF, CW, select="Tile3M")
    sub = tmp_path / "complete"
    sub.mkdir()
    F, W, CF, CW = _runs(sub)
    with pytest.raises(ValueError):
        pt.traffic(F, W, CW[:0], CW, select="Tile3M")      # no copy dispatches
    with pytest.raises(ValueError):
        pt.traffic(F, W, CF, CW, select="no such tile")


def test_hash_is_the_one_the_bench_checks():
    import importlib.util

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert pt.source_hash() == bench.kernel_source_hash()
