"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic work model behind the
roofline line, and the lookup of profiled HBM traffic (summed over a timing bucket's template
instances, and withheld once the kernel sources differ from the profiled ones)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus must be 1" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_flops_are_the_closed_forms():
    f = bench.algo_flops()
    n = m = 128
    assert f["hetrd"] == pytest.approx(16.0 / 3.0 * n ** 3)
    assert f["gram"] == 8.0 * m * n * (n + 1) / 2
    assert f["vecs"] == 8.0 * n * n * 64
    assert f["split"] == 8.0 * m * n * 64
    assert f["theta"] == 8.0 * m * n * 64 + 8.0 * 16 * 64 * 64


def test_bucket_kernels_follow_the_dispatch():
    # workload order n = 128, chi = 64: every update kernel contracts on the matrix cores
    assert [bench.bucket_kernel(b, 128, 64, 0) for b in ("theta", "gram", "hetrd", "vecs", "split")] == [
        ("k_theta_gate", "mfma"), ("k_gram_mfma", "mfma"), ("k_hetrd_mfma", "mfma"), ("k_tvecs", "mfma"),
        ("k_split", "mfma")]
    # the autotuner's wave-tile choice, a small order, and orders past the MFMA kernels' limits
    assert bench.bucket_kernel("hetrd", 128, 64, 1) == ("k_hetrd_tile", "alu")
    assert bench.bucket_kernel("gram", 64, 32, 0) == ("k_gram", "alu")
    assert bench.bucket_kernel("hetrd", 192, 96, 0) == ("k_hetrd", "alu")
    assert bench.bucket_kernel("vecs", 192, 96, 0) == ("k_vecs", "alu")


def _rows(path):
    out = {}
    for ln in open(path).read().splitlines():
        if ln.startswith("#") or ln.startswith("kernel ") or not ln.strip():
            continue
        parts = ln.split()
        out[" ".join(parts[:-4])] = (int(parts[-4]), float(parts[-1]))
    return out


def test_profiled_traffic_sums_a_buckets_dispatches(tmp_path, monkeypatch):
    if not os.path.exists(bench.TRAFFIC_PROFILE):
        pytest.skip("no committed traffic summary")
    rows = _rows(bench.TRAFFIC_PROFILE)
    hetrd = [v for k, v in rows.items() if k.replace("void ", "").split("<")[0].strip() == "k_hetrd_mfma"]
    got = bench.profiled_traffic("k_hetrd_mfma")
    if got is None:
        pytest.skip("committed summary was taken with other kernel sources")
    assert len(hetrd) == 2  # head and tail
    # bytes weighted by dispatches, per launch (every chunk has a tail; chunks of order <= 64 no head)
    launches = max(n for n, _ in hetrd)
    assert got == pytest.approx(sum(n * b for n, b in hetrd) / launches)
    assert got <= sum(b for _, b in hetrd)
    assert bench.profiled_traffic("no_such_kernel") is None
    # a summary whose source hash differs is not used
    fake = tmp_path / "traffic.txt"
    text = open(bench.TRAFFIC_PROFILE).read()
    i = text.index("k_update.hip sha256:") + len("k_update.hip sha256:")
    fake.write_text(text[:i] + "0" * 16 + text[i + 16:])
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(fake))
    assert bench.profiled_traffic("k_hetrd_mfma") is None


def test_path_model_matches_the_stated_flop_model():
    # d = 2, chi = 64 (n = 128): Theta 8.39 MF, gate 0.52 MF, reconstruction 8.39 MF on FP32;
    # Gram 16.8 MF and the eigensolve model 28.0 MF on FP64: about 62 MF and 0.68 us per update
    m = bench.path_model(2, 64)
    assert m["flops_per_update"] == pytest.approx(62.04e6, rel=1e-3)
    assert m["t_min_us"] == pytest.approx(0.679, rel=2e-3)
    assert m["bound_updates_per_s"] == pytest.approx(1.0 / (m["t_min_us"] * 1e-6))


def test_per_bond_work_matches_the_square_model_and_counts_edges():
    # a saturated bulk bond (64, 64, 64) is the square workload shape of algo_flops / path_model
    f = bench.item_flops(64, 64, 64, 64)
    assert f == pytest.approx(bench.algo_flops())
    assert bench.item_t_min(64, 64, 64, 64) * 1e6 == pytest.approx(bench.path_model(2, 64)["t_min_us"])
    # L = 8, chi = 4: bonds 0..6 with dims 1 2 4 4 4 4 2 1 -> 7 updates per step, parity 0 first
    dims = [1, 2, 4, 4, 4, 4, 4, 2, 1]
    items = bench.layer_items(dims)
    assert [it[:3] for it in items] == [(1, 2, 4), (4, 4, 4), (4, 4, 4), (4, 2, 1),
                                        (2, 4, 4), (4, 4, 4), (4, 4, 2)]
    work, n, tmin = bench.step_work([dims, dims])
    assert n == 14
    assert work["hetrd"] == pytest.approx(2 * sum(16.0 / 3.0 * (2 * c) ** 3 for _, _, c, _ in items))
    assert tmin == pytest.approx(2 * sum(bench.item_t_min(*it) for it in items))
    # edge bonds are cheaper than bulk ones, so the per-bond count sits below the square count
    work64, n64, _ = bench.step_work([[1] + [min(64, 2 ** min(b, 64 - b)) for b in range(1, 64)] + [1]])
    assert n64 == 63 and work64["hetrd"] < 63 * bench.algo_flops()["hetrd"]


def test_cpu_baseline_runs_the_oracle_in_processes():
    r = bench.cpu_baseline(8, 8, 0.01, 0.5, procs=2)
    assert r["kind"] == "oracle" and r["cores"] == 2
    assert r["value"] > 0 and r["single_core"]["value"] > 0
    assert "2 processes x 1 BLAS thread" in r["sample"]
    assert r["host"]["nproc"] >= 1 and r["host"]["affinity"] >= 1


def test_oracle_check_reports_each_checkpoint():
    # the oracle's own gesdd run, handed in as the device result, has no error; the other LAPACK
    # driver differs from it only by rounding
    import numpy as np
    import tn_inputs
    from oracle import model as M, tebd, stochastic, measure
    L, chi, dt = 8, 8, 0.01
    tensors, lams, _ = tn_inputs.random_isometric_mps(2024, L, chi)
    nz = tn_inputs.normals(7, (5, 8))
    mdl = M.Model(L)
    st = tebd.TNState([t.copy() for t in tensors], [l.copy() for l in lams])
    C = {}
    for k in range(5):
        stochastic.qsd_step(st, mdl.jumps, dt, nz[k][0:4], lambda b, tau: M.gate_heff(mdl, b, tau), chi,
                            bench.SV_CUTOFF["split"], driver="gesdd")
        if k + 1 in (2, 5):
            C[k + 1] = measure.corr_mps(st, normalize=False)[0]
    out = bench.oracle_check(tn_inputs, (tensors, lams), L, chi, dt, nz, C)
    assert sorted(out) == [2, 5]
    for err, spread, e_diag, e_nn in out.values():
        assert err == 0.0 and e_diag == 0.0 and e_nn == 0.0
        assert spread < 1e-12
    out = bench.oracle_check(tn_inputs, (tensors, lams), L, chi, dt, nz, {5: C[5] + 1e-3 * np.abs(C[5]).max()})
    assert abs(out[5][0] - 1e-3) < 1e-9
    # a start with a log-norm scales the unnormalized correlations by exp(2 lognorm)
    out = bench.oracle_check(tn_inputs, (tensors, lams, 0.5 * np.log(2.0)), L, chi, dt, nz, {5: 2.0 * C[5]})
    assert out[5][0] < 1e-12
