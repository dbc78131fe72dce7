"""Host logic of the benchmark's measurement (CPU): the HBM-counter summary and
the algorithmic byte model that the roofline figures come from.

* The counter summary scales FETCH_SIZE and WRITE_SIZE (KiB, summed over the
  L2 channels of a dispatch) by what they read for the calibration copy, and
  averages only the dispatches between the calibration copy and the end marker
  (the timed steps): checked on a synthetic counter file with known values.
* A summary taken on other sources is not used (traffic is reported as null).
* The byte model: the regular-voxel operator moves 2F per load plus one byte of
  material per voxel once per launch plus the enriched gather, linear in the
  number of loads apart from that byte.
"""

import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _write_counters(path, counter, rows):
    """rows: (dispatch id, kernel name, list of per-channel KiB values)."""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for did, name, vals in rows:
            for v in vals:
                w.writerow({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_counter_summary_window_and_scaling(tmp_path):
    b = _bench()
    kib = b.COPY_BYTES / 1024.0
    neg = "void at::native::vectorized_elementwise_kernel<neg_kernel_cuda>"
    reg = "void xfft::(anonymous namespace)::k_regular<float, true, false, false>(OpArgs<float>)"
    fft = "void xfft::(anonymous namespace)::k_fft_z_t<float, 128, 16>(FftArgs)"
    # FETCH reads half the copy's bytes (factor 2), WRITE all of them (factor 1);
    # dispatches 1 and 9 lie outside the window and must not count
    fetch = [(1, reg, [1e9]), (2, neg, [kib / 4, kib / 4]), (3, reg, [100.0, 50.0]), (4, fft, [10.0]),
             (5, reg, [200.0, 100.0]), (8, neg, [1.0]), (9, reg, [1e9])]
    write = [(1, reg, [1e9]), (2, neg, [kib / 2, kib / 2]), (3, reg, [30.0]), (4, fft, [20.0]),
             (5, reg, [60.0]), (8, neg, [1.0]), (9, reg, [1e9])]
    fp, wp = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _write_counters(fp, "FETCH_SIZE", fetch)
    _write_counters(wp, "WRITE_SIZE", write)
    out = b.pmc_summary(str(fp), str(wp))
    assert out["factor_fetch"] == pytest.approx(2.0)
    assert out["factor_write"] == pytest.approx(1.0)
    k = out["kernels"]["regular_voxels/fp32"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes"] == round(2.0 * 1024.0 * (150.0 + 300.0) / 2)
    assert k["write_bytes"] == round(1024.0 * (30.0 + 60.0) / 2)
    assert k["bytes_per_launch"] == k["fetch_bytes"] + k["write_bytes"]
    z = out["kernels"]["fft_z_green/fp32"]
    assert z["dispatches"] == 1 and z["fetch_bytes"] == round(2.0 * 1024.0 * 10.0)


def test_counter_summary_needs_copy_and_marker(tmp_path):
    b = _bench()
    reg = "void xfft::(anonymous namespace)::k_regular<float, true, false, false>(OpArgs<float>)"
    fp, wp = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _write_counters(fp, "FETCH_SIZE", [(3, reg, [1.0])])
    _write_counters(wp, "WRITE_SIZE", [(3, reg, [1.0])])
    with pytest.raises(SystemExit):
        b.pmc_summary(str(fp), str(wp))


def test_traffic_of_other_sources_is_not_used(tmp_path, monkeypatch):
    b = _bench()
    prof = tmp_path / "profiles"
    prof.mkdir()
    data = {"source_sha256": "0" * 64, "kernels": {"regular_voxels/fp32": {"bytes_per_launch": 1}}}
    (prof / "traffic_spheres128.md").write_text("x\n```json\n" + json.dumps(data) + "\n```\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    monkeypatch.setattr(b, "source_digest", lambda: "1" * 64)
    assert b.load_traffic("spheres128") is None
    # the same summary is used while the digest matches
    data["source_sha256"] = "1" * 64
    (prof / "traffic_spheres128.md").write_text("x\n```json\n" + json.dumps(data) + "\n```\n")
    assert b.load_traffic("spheres128")["kernels"]["regular_voxels/fp32"]["bytes_per_launch"] == 1


def test_committed_traffic_summaries_match_the_sources():
    # the summaries in profiles/ were taken on the HIP sources of this tree
    b = _bench()
    for workload in ("spheres128", "ellipsoids256"):
        t = b.load_traffic(workload)
        assert t is not None, workload
        assert t["factor_fetch"] == pytest.approx(2.0, rel=1e-3)
        assert t["factor_write"] == pytest.approx(1.0, rel=1e-3)


def test_algorithmic_bytes_model():
    b = _bench()
    g = dict(N=128 ** 3, nX=1000, n_irregular_voxels=500, n_cut_elements=2000, n0=128, n1=128, n2=128)
    one, six = b.algorithmic_bytes(g, 4, 1), b.algorithmic_bytes(g, 4, 6)
    F = 3 * g["N"] * 4
    gather = g["nX"] * (8 * 4 + 3 * 4)
    assert one["regular_voxels"] == 2 * F + gather + g["N"]
    # per-load parts scale with the loads, the material byte does not
    assert six["regular_voxels"] - g["N"] == 6 * (one["regular_voxels"] - g["N"])
    for k in ("irregular_voxels", "fft_x_forward", "fft_z_green", "fft_x_inverse"):
        assert six[k] == pytest.approx(6 * one[k])
    S = 3 * 128 * 128 * 65 * 2 * 4
    assert one["fft_x_forward"] == 3 * F + S
    assert one["fft_z_green"] == 2 * S + g["nX"] * 3 * 4 * 3
