"""Benchmark: batched two-site TEBD updates/s on one MI355X.

Workload (one bench step = one output interval of a quantum-state-diffusion batch):
  B trajectories of the boundary-driven free-fermion chain (J = 1, gamma = 0.5, source s+ on
  the first site, sink s- on the last), L = 64 sites, bond dimension chi = 64, SPLIT precision
  (complex64 storage, FP32 MFMA Theta with the gate, FP64 Gram/eigensolver/split/weights/norms);
  per bench step: INNER first-order Trotter steps (dt = 0.01) of exp(-i h^eff dt) gates, each
  followed by the diffusion factors 1 + dW sqrt(gamma) L with complex Gaussian dW, then one
  measurement of C_ij = <c_i^+ c_j> for every trajectory (the output time).
Inputs are synthetic and seeded.  The headline starts from physical checkpoints: a few
trajectories evolved from the Neel state with the library's FP64 path until the middle bonds
saturate chi, copied over the batch.  A second figure starts from right-isometric tensors with
geometric bond weights (sigma_a ~ exp(-a/8)).
Reported: value = two-site updates/s of the batched split path (whole job, timed with kernel
timing off so the captured HIP graphs replay), the plain per-instance and the batched FP64 GPU
paths for comparison, the error against the FP64 oracle after one interval and after 100 steps
with the tolerance, the roofline of the dominant kernel from a separate pass with kernel timing
on and the chunks of a layer on one stream (algorithmic flops of the actual bond shapes over
the HIP-event durations), value against the path's flop-model bound, and the CPU oracle timed
on a bounded sample (one core, and one process per core).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "hbm": 8.0e12}
# rocprofv3 counter summary that holds the HBM bytes per dispatch of each update kernel at this
# workload's launch shape (8192 / 7936 updates per dispatch); it names the sha256 of the kernel
# sources it was taken with, and its figures are used only while the sources still match.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_qsd_B1024_L64_chi64_physical_split.txt")


def bucket_kernel(bucket, n, chi, hetrd_variant):
    """(kernel, bound) of a timing bucket in split precision at Gram order n and bond dimension chi:
    the kernel that runs in it and whether its inner products sit on the matrix cores ("mfma") or
    on the vector FP64 units ("alu").  The Gram uses the MFMA kernel for 64 < n <= 128; for
    n <= 128 the Householder reduction is the autotuner's choice (variant 0: MFMA block columns,
    1: vector wave tiles); the eigenvector kernel with the MFMA back-transformation runs for
    n <= 128 and chi <= 64."""
    if bucket == "gram":
        return ("k_gram_mfma", "mfma") if 64 < n <= 128 else ("k_gram", "alu")
    if bucket == "hetrd":
        if n > 128:
            return ("k_hetrd", "alu")
        return ("k_hetrd_tile", "alu") if hetrd_variant == 1 else ("k_hetrd_mfma", "mfma")
    if bucket == "vecs":
        return ("k_tvecs", "mfma") if (n <= 128 and chi <= 64) else ("k_vecs", "alu")
    return {"theta": ("k_theta_gate", "mfma"), "split": ("k_split", "mfma")}[bucket]


# algorithmic FLOPs per two-site update at the workload shape (m = n = 128, chi_m = k = 64, D = 4)
def algo_flops(n=128, m=128, chim=64, k=64, D=4):
    return {
        "theta": 8.0 * m * n * chim + 8.0 * D * D * (m // 2) * (n // 2),   # Theta GEMM + gate (complex, 8 flops/CMAC)
        "gram": 8.0 * m * n * (n + 1) / 2,                                 # Hermitian Gram (lower half)
        "hetrd": 16.0 / 3.0 * n ** 3,                                      # Householder tridiagonalization
        "vecs": 8.0 * n * n * k,                                           # back-transformation of k vectors
        "split": 8.0 * m * n * k,                                          # Theta~ V
    }


def path_model(d=2, chi=64):
    """Lower-bound time model of one two-site update at bond dimension chi (local dimension d, Gram
    order n = d chi, k = chi kept): Theta, gate and reconstruction at the FP32 matrix peak, the
    Gram matrix (8 n^3) and a Hermitian eigensolve counted as 4 (4/3 + 2) n^3 at the FP64 peak;
    real flops, a complex MAC counted as 8."""
    n, k = d * chi, chi
    f32 = 8.0 * d * d * chi ** 3 + 8.0 * (d * d) ** 2 * chi * chi + 8.0 * n * n * k
    f64 = 8.0 * n ** 3 + 4.0 * (4.0 / 3.0 + 2.0) * n ** 3
    t = f32 / PEAK["fp32"] + f64 / PEAK["fp64"]
    return {"flops_per_update": f32 + f64, "t_min_us": t * 1e6, "bound_updates_per_s": 1.0 / t}


def item_flops(chil, chim, chir, k, d=2):
    """Algorithmic real flops of one two-site update with bond dimensions (chi_l, chi_m, chi_r), k kept
    (Theta is (d chi_l) x (d chi_r), Gram order n = d chi_r), per timing bucket: the closed forms of
    algo_flops at the item's own shape."""
    m, n = d * chil, d * chir
    D = d * d
    return {
        "theta": 8.0 * m * n * chim + 8.0 * D * D * chil * chir,
        "gram": 8.0 * m * n * (n + 1) / 2,
        "hetrd": 16.0 / 3.0 * n ** 3,
        "vecs": 8.0 * n * n * k,
        "split": 8.0 * m * n * k,
    }


def item_t_min(chil, chim, chir, k, d=2):
    """Lower-bound time (s) of one update at its own shape, the model of path_model: Theta, gate and
    reconstruction at the FP32 matrix peak; the Gram matrix (8 m n^2) and the Hermitian eigensolve
    (4 (4/3 + 2) n^3) at the FP64 peak."""
    m, n = d * chil, d * chir
    f32 = 8.0 * m * n * chim + 8.0 * (d * d) ** 2 * chil * chir + 8.0 * m * n * k
    f64 = 8.0 * m * n * n + 4.0 * (4.0 / 3.0 + 2.0) * n ** 3
    return f32 / PEAK["fp32"] + f64 / PEAK["fp64"]


def layer_items(dims):
    """(chi_l, chi_m, chi_r, k) of every two-site update of one first-order Trotter step of one
    instance whose bond dimensions dims (L + 1 entries) hold from step to step (a saturated
    state): parity 0 (bonds 0, 2, ...) then parity 1, each bond keeping its dimension, k = chi_m."""
    L = len(dims) - 1
    return [(int(dims[b]), int(dims[b + 1]), int(dims[b + 2]), int(dims[b + 1]))
            for parity in (0, 1) for b in range(parity, L - 1, 2)]


def step_work(all_dims):
    """Per first-order Trotter step of a batch whose instances have bond dimensions all_dims: the
    algorithmic flops of each timing bucket, the number of updates and the summed t_min (s)."""
    tot = {"theta": 0.0, "gram": 0.0, "hetrd": 0.0, "vecs": 0.0, "split": 0.0}
    n_items, tmin = 0, 0.0
    for dims in all_dims:
        for chil, chim, chir, k in layer_items(dims):
            for key, v in item_flops(chil, chim, chir, k).items():
                tot[key] += v
            tmin += item_t_min(chil, chim, chir, k)
            n_items += 1
    return tot, n_items, tmin


def profiled_traffic(kernel):
    """HBM bytes per launch of the timing bucket whose kernel is `kernel`, from the committed counter
    summary, or None when the summary is missing or was taken with different kernel sources.  A
    launch may be several dispatches (the Householder reduction of a chunk is a head and a tail, and
    chunks of order <= 64 have the tail only), so the bytes of every template instance are weighted
    by its dispatch count and divided by the largest count, which is the number of launches."""
    import hashlib
    try:
        lines = open(TRAFFIC_PROFILE).read().splitlines()
    except OSError:
        return None
    src = [ln for ln in lines if ln.startswith("# sources:")]
    if not src:
        return None
    for item in src[0][len("# sources:"):].split(","):
        name, h = item.strip().split(" sha256:")
        path = os.path.join(ROOT, "paper_2609_18841_amd", "csrc", name)
        if hashlib.sha256(open(path, "rb").read()).hexdigest()[:16] != h:
            return None
    tot, launches = 0.0, 0
    for ln in lines:
        if ln.startswith("#"):
            continue
        parts = ln.split()
        nm = " ".join(parts[:-4]).replace("void ", "").split("<")[0].strip()
        if nm == kernel:
            n = int(parts[-4])
            tot += float(parts[-1]) * n
            launches = max(launches, n)
    return tot / launches if launches else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--chi", type=int, default=64)
    ap.add_argument("--inner", type=int, default=10, help="Trotter steps per output interval")
    ap.add_argument("--dt", type=float, default=0.01)
    ap.add_argument("--workload", choices=["qsd", "mpdo", "qt", "qsd-wide", "purified"], default="qsd",
                    help="qsd: the headline (default); the others time the remaining configurations and "
                         "print their own line (run_workload)")
    ap.add_argument("--pre", type=int, default=-1, help="untimed steps before timing (other workloads)")
    ap.add_argument("--theta-bits", type=int, choices=[32, 64], default=64,
                    help="matrix cores of the Theta contraction in split mode (the other is timed beside it)")
    ap.add_argument("--input", choices=["physical", "synthetic"], default="physical",
                    help="headline input: evolved checkpoints (default) or geometric-spectrum tensors")
    ap.add_argument("--checkpoints", type=int, default=16, help="distinct evolved trajectories copied over the batch")
    ap.add_argument("--ck-dt", type=float, default=0.05, help="time step of the checkpoint evolution (FP64)")
    ap.add_argument("--ck-tmax", type=float, default=20.0, help="longest checkpoint evolution")
    ap.add_argument("--plain-steps", type=int, default=10, help="Trotter steps per timed run of the plain FP64 path")
    ap.add_argument("--fp64-batched-steps", type=int, default=2,
                    help="timed Trotter steps of the batched FP64 path at the full batch (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-clock window of the all-core oracle run (the single-core run takes up to 6 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the second input's throughput")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run every chunk of a layer on the caller's stream in the timed region")
    ap.add_argument("--no-buckets", action="store_true",
                    help="form each layer's chunks from all its bonds in instance order (no bond-size buckets)")
    ap.add_argument("--overlap-measure", action="store_true",
                    help="measure each output from a snapshot, beside the next interval's steps")
    ap.add_argument("--check-trajectories", type=int, default=4,
                    help="trajectories of the check batch compared with the oracle (trajectory 0 also against "
                         "the oracle's other SVD driver and its complex64-rounded start)")
    ap.add_argument("--check-steps", type=int, default=100,
                    help="Trotter steps of the longer oracle comparison (besides one output interval)")
    ap.add_argument("--checkpoint-file", default="",
                    help="npz of the evolved checkpoints: loaded when it exists, else written after evolving")
    ap.add_argument("--profile-only", action="store_true",
                    help="one stream throughout: warmup intervals, then one profiled interval; prints the "
                         "roofline line only (for rocprofv3 runs, whose traces then hold one-stream dispatches)")
    ap.add_argument("--summarize-trace", default="", metavar="DIR",
                    help="print the per-kernel summary of a rocprofv3 --stats --output-format csv run and exit")
    ap.add_argument("--summarize-counters", default="",
                    help="print the per-kernel means of a rocprofv3 --pmc run's counters and exit")
    ap.add_argument("--summarize-pmc", nargs=4, default=None,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="print the per-kernel HBM traffic from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of "
                         "the workload and of --calib-copy 1024, and exit")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration) and exit")
    return ap.parse_args()


# relative singular-value cutoff of the timed state (split precision) and of the FP64 paths
SV_CUTOFF = {"split": 1e-6, "fp64": 1e-12}
# the split path's stated bound on correlations against the FP64 oracle, normwise
# max |dC| / max |C| (the precision pattern's tolerance for FP32 contractions)
ERR_TOLERANCE = 1e-5


def source_hashes():
    """sha256 prefixes of the kernel sources a profile summary was taken with."""
    import hashlib
    out = []
    for name in ("k_update.hip", "k_measure.hip", "k_jumps.hip", "gemm.h"):
        path = os.path.join(ROOT, "paper_2609_18841_amd", "csrc", name)
        out.append(f"{name} sha256:{hashlib.sha256(open(path, 'rb').read()).hexdigest()[:16]}")
    return ", ".join(out)


def _csv_rows(directory, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)):
        with open(path) as f:
            rows.extend(csv.DictReader(f))
    return rows


def summarize_trace(directory):
    """Per-kernel table from rocprofv3's kernel_stats.csv: calls, total, average, min, max (ms)."""
    rows = _csv_rows(directory, "kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"{'kernel':60s} {'calls':>7s} {'total_ms':>10s} {'avg_ms':>9s} {'min_ms':>9s} {'max_ms':>9s} {'pct':>6s}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        n, t = int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6
        lines.append(f"{r['Name'][:60]:60s} {n:7d} {t:10.3f} {t / n:9.4f} {float(r['MinNs']) / 1e6:9.4f} "
                     f"{float(r['MaxNs']) / 1e6:9.4f} {100 * t * 1e6 / tot:6.2f}")
    return lines


def _pmc_means(directory, counter, counts=False):
    """Mean counter value per dispatch, by kernel, from rocprofv3's counter_collection.csv (and, with
    counts, the number of dispatches of each kernel)."""
    acc = {}
    for r in _csv_rows(directory, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        k = r["Kernel_Name"]
        a = acc.setdefault(k, [0.0, 0])
        a[0] += float(r["Counter_Value"])
        a[1] += 1
    means = {k: v / n for k, (v, n) in acc.items()}
    return (means, {k: n for k, (_, n) in acc.items()}) if counts else means


def summarize_counters(directory):
    """Per-kernel mean of every counter of a rocprofv3 --pmc run, per dispatch, with the number of
    dispatches (kernels by total of the first counter)."""
    acc = {}
    names = []
    for r in _csv_rows(directory, "counter_collection.csv"):
        c = r.get("Counter_Name")
        if c not in names:
            names.append(c)
        a = acc.setdefault(r["Kernel_Name"], {}).setdefault(c, [0.0, 0])
        a[0] += float(r["Counter_Value"])
        a[1] += 1
    lines = [f"{'kernel':60s} {'dispatches':>10s} " + " ".join(f"{c:>26s}" for c in names)]
    first = names[0] if names else None
    for k in sorted(acc, key=lambda k: -acc[k].get(first, [0.0, 1])[0]):
        n = max(v[1] for v in acc[k].values())
        vals = " ".join(f"{(acc[k][c][0] / acc[k][c][1]) if c in acc[k] else 0.0:26.4e}" for c in names)
        lines.append(f"{k[:60]:60s} {n:10d} {vals}")
    return lines


def summarize_pmc(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_mib=1024):
    """Per-kernel FETCH_SIZE and WRITE_SIZE (KiB per dispatch) and the HBM bytes they stand for, each
    counter scaled by what it reads for a plain device copy of copy_mib MiB (which reads and writes
    exactly that many bytes)."""
    (fetch, ndisp), write = _pmc_means(fetch_dir, "FETCH_SIZE", counts=True), _pmc_means(write_dir, "WRITE_SIZE")
    cf = max(_pmc_means(cfetch_dir, "FETCH_SIZE").values())
    cw = max(_pmc_means(cwrite_dir, "WRITE_SIZE").values())
    kib = copy_mib * 1024.0
    sf, sw = kib / cf, kib / cw
    lines = [f"# calibration: a {copy_mib} MiB device copy reads FETCH_SIZE {cf:.1f} KiB and WRITE_SIZE {cw:.1f} KiB "
             f"per dispatch -> scale fetch x{sf:.4f}, write x{sw:.4f}",
             f"{'kernel':60s} {'dispatches':>10s} {'FETCH_KiB':>12s} {'WRITE_KiB':>12s} {'hbm_bytes_scaled':>18s}"]
    for k in sorted(fetch, key=lambda k: -(fetch[k] * sf + write.get(k, 0.0) * sw)):
        b = (fetch[k] * sf + write.get(k, 0.0) * sw) * 1024.0
        lines.append(f"{k[:60]:60s} {ndisp[k]:10d} {fetch[k]:12.1f} {write.get(k, 0.0):12.1f} {b:18.4e}")
    return lines


def evolve_checkpoints(api, tn_inputs, L, chi, n, dt, tmax, seed=4242):
    """n quantum-state-diffusion trajectories of the workload's chain evolved from the Neel state with
    the FP64 path (first-order Trotter steps of size dt, each followed by the noise) until chi binds
    on every bond at least 6 sites from both ends also under the split path's cutoff: the bond
    holds chi weights and the smallest is above 10 x SV_CUTOFF["split"] of the largest (from the
    Neel state at dt = 0.05 that is t = 2.5 to 3); or until tmax.  Returns the packed instances
    [(tensors, lams, lognorm)], the time reached and the bond dimensions."""
    model = api.Model.free_fermion(L, 1.0, 0.5)
    st = api.State(api.KIND_MPS, model, n, chi, tn_inputs.neel(L), precision=api.FP64,
                   sv_cutoff=SV_CUTOFF["fp64"])
    nmax = int(round(tmax / dt))
    noise = tn_inputs.normals(seed, (nmax, n * 4))
    k = 0
    while k < nmax:
        st.tebd_step(dt, order=1)
        st.apply_jumps(api.MODE_QSD, dt, noise[k], api.NOISE_GAUSS)
        k += 1
        if k % 5 == 0:
            lam = [st.lams(b) for b in range(n)]
            if all(len(l) == chi and l[-1] > 10 * SV_CUTOFF["split"] * l[0] for x in lam for l in x[5:L - 6]):
                break
    cks = []
    for b in range(n):
        t, lam, ln, _ = st.get_instance(b)
        cks.append((t, lam, ln))
    dims = [st.dims(b).tolist() for b in range(n)]
    st.close()
    return cks, k * dt, dims


def make_state(api, tn_inputs, prec, B, L, chi, cks=None, seed=2024, bits=64):
    """A batch of B trajectories at bond dimension chi: instance b starts from checkpoint b mod
    len(cks), or, without checkpoints, every instance from the geometric-spectrum tensors; in split
    precision Theta is formed on the matrix cores of `bits`.  Returns the state and the FP64 start
    of instance 0 (tensors, lams, lognorm)."""
    model = api.Model.free_fermion(L, 1.0, 0.5)
    st = api.State(api.KIND_MPS, model, B, chi, tn_inputs.neel(L), precision=prec,
                   sv_cutoff=SV_CUTOFF["split"] if prec == api.SPLIT else SV_CUTOFF["fp64"])
    if prec == api.SPLIT:
        st.theta_precision(bits)
    if cks is None:
        tensors, lams, dims = tn_inputs.random_isometric_mps(seed, L, chi)
        st.set_instance(0, tensors, lams, 0.0)
        if B > 1:
            st.replicate(0)
        return st, (tensors, lams, 0.0)
    for b in range(B):
        t, lam, ln = cks[b % len(cks)]
        st.set_instance(b, t, lam, ln)
    return st, cks[0]


def run_interval(api, st, noise, inner, dt, measure=True):
    for k in range(inner):
        st.tebd_step(dt, order=1)
        st.apply_jumps(api.MODE_QSD, dt, noise[k], api.NOISE_GAUSS)
    if measure:
        return st.measure_corr(normalize=0)
    return None


def _oracle_qsd_run(seed, L, chi, dt, budget_s, t_start=None):
    """Oracle QSD steps on one trajectory of the workload for budget_s seconds with BLAS limited to
    one thread; returns (updates, t0, t1) in wall-clock seconds.  With t_start the timed loop
    begins at that wall-clock time (the processes of the all-core run start together)."""
    from threadpoolctl import threadpool_limits
    import tn_inputs
    from oracle import model as M, tebd, stochastic
    with threadpool_limits(limits=1):
        mdl = M.Model(L)
        cache = {}

        def fn(b, tau):
            if (b, tau) not in cache:
                cache[(b, tau)] = M.gate_heff(mdl, b, tau)
            return cache[(b, tau)]
        tensors, lams, _ = tn_inputs.random_isometric_mps(2024, L, chi)
        st = tebd.TNState(tensors, lams)
        noise = tn_inputs.normals(seed, (10 ** 6 // (4 * L) + 8, 4))
        if t_start is not None:
            while time.time() < t_start:
                time.sleep(0.002)
        t0 = time.time()
        steps = 0
        while time.time() - t0 < budget_s:
            stochastic.qsd_step(st, mdl.jumps, dt, noise[steps], fn, chi, SV_CUTOFF["split"])
            steps += 1
        t1 = time.time()
    return steps * (L - 1), t0, t1


def _oracle_qsd_job(job):
    return _oracle_qsd_run(*job)


def _host_info():
    """CPU model, logical CPUs (all, and those this process may run on) and numpy's BLAS/LAPACK."""
    info = {"cpu_model": None, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            info["cpu_model"] = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    try:
        deps = np.show_config(mode="dicts").get("Build Dependencies", {})
        info["numpy_blas"] = {k: f"{v.get('name')} {v.get('version')}" for k, v in deps.items()}
    except Exception:
        info["numpy_blas"] = None
    return info


def cpu_baseline(L, chi, dt, budget_s, procs=None):
    """The oracle (numpy complex128, LAPACK SVD) on the same workload, BLAS one thread per process:
    single-core rate (one trajectory in this process) and all-core throughput (one process per
    core, each evolving its own trajectory, all timed over the same wall-clock window).  value is
    the all-core throughput; cores is the number of processes, one BLAS thread each."""
    import multiprocessing as mp
    if procs is None:
        procs = max(1, min(16, len(os.sched_getaffinity(0))))
    t_single = min(6.0, 0.5 * budget_s)
    upd1, a, b = _oracle_qsd_run(99, L, chi, dt, t_single)
    single = upd1 / (b - a)
    ctx = mp.get_context("spawn")
    t_start = time.time() + 3.0 + 0.1 * procs  # after the workers have imported numpy and scipy
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_qsd_job, [(100 + w, L, chi, dt, budget_s, t_start) for w in range(procs)])
    upd = sum(r[0] for r in res)
    wall = max(r[2] for r in res) - min(r[1] for r in res)
    return {"value": upd / wall, "unit": "two-site updates/s", "cores": procs, "kind": "oracle",
            "single_core": {"value": single, "unit": "two-site updates/s", "updates": upd1},
            "host": _host_info(),
            "sample": f"{procs} processes x 1 BLAS thread, each one L={L} chi={chi} QSD trajectory of the workload "
                      f"(numpy complex128 + LAPACK SVD), {upd} updates in a {wall:.1f} s wall-clock window; "
                      f"single core: {upd1} updates in {b - a:.1f} s"}


def _oracle_corr_run(job):
    """One FP64 oracle trajectory from start (tensors, lams, lognorm) under the given noise rows with
    the given LAPACK driver; {steps: C} at the requested step counts (BLAS one thread).  Driver
    "c64start" is gesdd from the start's tensors rounded to complex64: the spread that storing the
    start in the split path's precision alone causes."""
    start, L, chi, dt, noise, want, driver = job
    if driver == "c64start":
        start = ([t.astype(np.complex64).astype(np.complex128) for t in start[0]],) + tuple(start[1:])
        driver = "gesdd"
    from threadpoolctl import threadpool_limits
    from oracle import model as M, tebd, stochastic, measure
    mdl = M.Model(L)
    cache = {}

    def fn(b, tau):
        if (b, tau) not in cache:
            cache[(b, tau)] = M.gate_heff(mdl, b, tau)
        return cache[(b, tau)]
    tensors, lams = start[0], start[1]
    lognorm = start[2] if len(start) > 2 else 0.0
    out = {}
    with threadpool_limits(limits=1):
        st = tebd.TNState([t.copy() for t in tensors], [l.copy() for l in lams], lognorm)
        for k in range(max(want)):
            stochastic.qsd_step(st, mdl.jumps, dt, noise[k][0:4], fn, chi, SV_CUTOFF["split"], driver=driver)
            if k + 1 in want:
                out[k + 1] = measure.corr_mps(st, normalize=False)[0]
    return out


def oracle_check(tn_inputs, st_init, L, chi, dt, noise, C_gpu0, pool=None, c64start=False):
    """{steps: (err, spread, err_density, err_nn)} for trajectory 0 at each checkpoint of C_gpu0
    ({steps: C}).  err and spread are max |dC| / max |C|: err is the GPU against the FP64 oracle on
    the same input and with the same truncation (chi and the split state's singular-value cutoff);
    spread is the oracle against itself with another LAPACK SVD driver (gesvd instead of gesdd).
    At a binding chi the kept singular vectors depend on rounding inside the SVD, and spread is the
    scale at which two exact FP64 runs already differ.  err_density and err_nn are the GPU's
    elementwise relative errors on the diagonal (densities) and on the first off-diagonal.
    st_init is (tensors, lams) or (tensors, lams, lognorm); pool (a process pool started before
    the GPU was touched) runs the drivers side by side.  With c64start each entry gains a fifth
    figure: the oracle from the start rounded to complex64 against the oracle from the start,
    the part of err that the precision of the stored start alone explains (at a binding chi the
    truncation amplifies any perturbation, and this shows by how much)."""
    jobs = oracle_jobs(st_init, L, chi, dt, noise, C_gpu0, c64start)
    res = pool.map(_oracle_corr_run, jobs) if pool is not None else [_oracle_corr_run(j) for j in jobs]
    return oracle_compare(C_gpu0, res, c64start)


def oracle_jobs(st_init, L, chi, dt, noise, C_gpu0, c64start=False):
    """The oracle runs that oracle_check compares C_gpu0 with (gesdd, gesvd and optionally the
    complex64-rounded start), as jobs for _oracle_corr_run."""
    want = sorted(C_gpu0)
    drivers = ("gesdd", "gesvd", "c64start") if c64start else ("gesdd", "gesvd")
    return [(st_init, L, chi, dt, noise, want, drv) for drv in drivers]


def oracle_compare(C_gpu0, res, c64start=False):
    """oracle_check's figures from the results of its oracle_jobs, in job order."""
    drivers = ("gesdd", "gesvd", "c64start") if c64start else ("gesdd", "gesvd")
    Cs = dict(zip(drivers, res))
    out = {}
    for n, Cg in C_gpu0.items():
        ref = Cs["gesdd"][n]
        scale = np.max(np.abs(ref))
        out[n] = (float(np.max(np.abs(Cg - ref)) / scale), float(np.max(np.abs(Cs["gesvd"][n] - ref)) / scale),
                  _elementwise(np.diag(Cg), np.diag(ref)), _elementwise(np.diag(Cg, 1), np.diag(ref, 1)))
        if c64start:
            out[n] = out[n] + (float(np.max(np.abs(Cs["c64start"][n] - ref)) / scale),)
    return out


def _elementwise(a, b):
    """max_i |a_i - b_i| / |b_i| (the densities C_ii, or the nearest-neighbour terms C_i,i+1)."""
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _profiled_interval(api, st, noise, inner, dt, B):
    """One output interval with kernel timing on and the chunks of a layer on the caller's stream only,
    so that no two launches share the compute units and each HIP-event interval is one dispatch's
    own duration.  Returns ({kernel: {total_ms, launches, avg_ms}}, bond dimensions at the start)."""
    import torch
    dims = [st.dims(b) for b in range(B)]
    st.overlap(False)
    st.prof_enable(True)
    run_interval(api, st, noise, inner, dt)
    torch.cuda.synchronize()
    kt = {}
    for kid, name in enumerate(api.K_NAMES):
        ms, n = st.prof_query(kid)
        kt[name] = {"total_ms": ms, "launches": n, "avg_ms": ms / n if n else 0.0}
    st.prof_enable(False)
    return kt, dims


def roofline_line(api, st, kt, dims, inner, chi):
    """Roofline of the update kernel with the largest profiled time: algorithmic flops of the items it
    processed (every bond at its own (chi_l, chi_m, chi_r), step_work) over its summed HIP-event
    durations, against the FP64 or FP32 matrix peak of its type."""
    work, n_items, tmin = step_work(dims)
    upd = ["theta", "gram", "hetrd", "vecs", "split"]
    dom = max(upd, key=lambda k: kt[k]["total_ms"])
    peak = PEAK["fp32"] if dom == "theta" else PEAK["fp64"]
    flops = work[dom] * inner
    secs = kt[dom]["total_ms"] / 1e3
    achieved = flops / secs
    kname, bound = bucket_kernel(dom, 2 * chi, chi, st.tuning()[0])
    launches = max(1, kt[dom]["launches"])
    return {"bound": bound, "kernel": kname, "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": profiled_traffic(kname),
            "traffic_unit": "bytes per launch", "algo_flops_per_launch": flops / launches,
            "items_per_launch": n_items * inner / launches, "avg_launch_ms": kt[dom]["avg_ms"],
            "launches": kt[dom]["launches"], "streams": 1,
            "basis": "profiled interval: one stream, HIP events per launch; flops of each bond's own shape"}, \
        work, n_items, tmin


def run_workload(args):
    """Throughput of the configurations besides the headline, from the Neel state, with untimed steps
    first so that the bond dimensions have grown (and, for trajectories, spread):
      mpdo      vectorized Lindblad, L = 64, chi = 128 (Theta up to 512 x 512), 2nd order, dt = 0.02:
                split and FP64, with the split result's distance to the FP64 one on the same steps;
      qt        1024 quantum trajectories, L = 32, chi = 64, dt = 0.01, jumps from FP64 uniforms
                (a jumped trajectory skips its Trotter step, so only evolved ones count);
      qsd-wide  4096 QSD trajectories, L = 64, chi = 32, dt = 0.01, one measurement per 10 steps;
      purified  locally purified MPS, L = 32, chi = 64, chi_k = 4, dt = 0.02, Kraus step each step.
    Prints one JSON line."""
    import torch
    import tn_inputs
    from paper_2609_18841_amd import api
    torch.cuda.set_device(0)
    wl = args.workload
    res = {"workload": wl, "unit": "two-site updates/s", "n_gpus": 1, "data": "synthetic", "higher_is_better": True}

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_upd = fn(steps)
        torch.cuda.synchronize()
        return n_upd / (time.perf_counter() - t0), n_upd

    if wl == "mpdo":
        L, chi, dt = 64, 128, 0.02
        pre = 25 if args.pre < 0 else args.pre
        out = {}
        for name, prec in (("split", api.SPLIT), ("fp64", api.FP64)):
            st = api.State(api.KIND_MPDO, api.Model.free_fermion(L), 1, chi, tn_inputs.neel(L), precision=prec,
                           sv_cutoff=SV_CUTOFF["split"] if prec == api.SPLIT else SV_CUTOFF["fp64"])
            if prec == api.SPLIT:
                st.theta_precision(args.theta_bits)
            if args.no_buckets:
                st.buckets(on=0)
            for k in range(pre):
                st.tebd_step(dt, order=2)
                if k % 5 == 4:
                    print(f"# mpdo {name}: untimed step {k + 1}", file=sys.stderr, flush=True)

            def steps(k):
                for i in range(k):
                    st.tebd_step(dt, order=2)
                    print(f"# mpdo {name}: timed step {i + 1}", file=sys.stderr, flush=True)
                return 94 * k
            v, n_upd = timed(steps, args.steps)
            C, _, _, tr = st.measure_corr()
            out[name] = {"value": v, "updates": n_upd, "C": C, "trace": float(tr[0]),
                         "max_bond_dim": int(max(st.dims(0)))}
            st.close()
            print(f"# mpdo {name}: {v:.1f} updates/s", file=sys.stderr, flush=True)
        diff = float(np.max(np.abs(out["split"]["C"] - out["fp64"]["C"])) / np.max(np.abs(out["fp64"]["C"])))
        res.update({"metric": "two-site updates/s, MPDO L=64 chi=128", "value": out["split"]["value"],
                    "fp64": out["fp64"]["value"], "split_over_fp64": out["split"]["value"] / out["fp64"]["value"],
                    "split_vs_fp64_C": diff, "trace_split": out["split"]["trace"], "trace_fp64": out["fp64"]["trace"],
                    "max_bond_dim": out["fp64"]["max_bond_dim"],
                    "config": {"L": L, "chi": chi, "dt": dt, "order": 2, "untimed_steps": pre, "timed_steps": args.steps,
                               "start": "Neel", "theta_bits": args.theta_bits, "buckets": not args.no_buckets}})
    elif wl == "qt":
        L, chi, B, dt = 32, 64, 1024, 0.01
        pre = 400 if args.pre < 0 else args.pre  # t = 4 of the configuration's t <= 5
        st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, tn_inputs.neel(L), precision=api.SPLIT,
                       sv_cutoff=SV_CUTOFF["split"])
        st.theta_precision(args.theta_bits)
        if args.no_buckets:
            st.buckets(on=0)
        us = tn_inputs.uniforms(11, (pre + args.steps, B))
        jumps = [0]

        def qt_steps(k0, k):
            n_upd = 0
            for i in range(k0, k0 + k):
                _, mask = st.apply_jumps(api.MODE_QT, dt, us[i])
                st.tebd_step(dt, order=1, mask=mask)
                n_upd += int(B - mask.sum()) * (L - 1)
                jumps[0] += int(mask.sum())
            return n_upd
        for k0 in range(0, pre, 100):
            qt_steps(k0, min(100, pre - k0))
            print(f"# qt: untimed step {min(pre, k0 + 100)}", file=sys.stderr, flush=True)
        jumps[0] = 0
        v, n_upd = timed(lambda k: qt_steps(pre, k), args.steps)
        mids = np.array([st.dims(b)[L // 2] for b in range(B)])
        res.update({"metric": "two-site updates/s, QT B=1024 L=32 chi<=64", "value": v, "updates": n_upd,
                    "jump_fraction": jumps[0] / (B * args.steps),
                    "middle_bond_dim": {"min": int(mids.min()), "max": int(mids.max()), "mean": float(mids.mean())},
                    "config": {"B": B, "L": L, "chi": chi, "dt": dt, "untimed_steps": pre, "timed_steps": args.steps,
                               "start": "Neel", "theta_bits": args.theta_bits, "buckets": not args.no_buckets}})
        st.close()
    elif wl == "qsd-wide":
        L, chi, B, dt, inner = 64, 32, 4096, 0.01, 10
        pre = 400 if args.pre < 0 else args.pre  # t = 4 of the configuration's t <= 5
        st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, tn_inputs.neel(L), precision=api.SPLIT,
                       sv_cutoff=SV_CUTOFF["split"])
        st.theta_precision(args.theta_bits)
        if args.no_buckets:
            st.buckets(on=0)
        nz = tn_inputs.normals(13, (pre + args.steps * inner, B * 4))
        for k in range(pre):
            st.tebd_step(dt, order=1)
            st.apply_jumps(api.MODE_QSD, dt, nz[k], api.NOISE_GAUSS)
            if k % 100 == 99:
                print(f"# qsd-wide: untimed step {k + 1}", file=sys.stderr, flush=True)

        def intervals(k):
            for r in range(k):
                run_interval(api, st, nz[pre + r * inner:pre + (r + 1) * inner], inner, dt)
            return k * inner * (L - 1) * B
        v, n_upd = timed(intervals, args.steps)
        mids = np.array([st.dims(b)[L // 2] for b in range(0, B, 16)])
        res.update({"metric": "two-site updates/s, QSD B=4096 L=64 chi<=32", "value": v, "updates": n_upd,
                    "middle_bond_dim": {"min": int(mids.min()), "max": int(mids.max()), "mean": float(mids.mean())},
                    "config": {"B": B, "L": L, "chi": chi, "dt": dt, "inner_steps": inner, "untimed_steps": pre,
                               "timed_intervals": args.steps, "start": "Neel", "theta_bits": args.theta_bits, "buckets": not args.no_buckets}})
        st.close()
    else:
        L, chi, chik, dt = 32, 64, 4, 0.02
        pre = 200 if args.pre < 0 else args.pre  # t = 4 of the configuration's t <= 5
        st = api.State(api.KIND_PURIFIED, api.Model.free_fermion(L), 1, chi, tn_inputs.neel(L), chi_k_max=chik,
                       precision=api.SPLIT, sv_cutoff=SV_CUTOFF["split"])
        st.theta_precision(args.theta_bits)
        if args.no_buckets:
            st.buckets(on=0)

        def psteps(k):
            for _ in range(k):
                st.tebd_step(dt, order=1)
                st.apply_jumps(api.MODE_KRAUS, dt)
            return k * (L - 1)
        for k0 in range(0, pre, 50):
            psteps(min(50, pre - k0))
            print(f"# purified: untimed step {min(pre, k0 + 50)}", file=sys.stderr, flush=True)
        v, n_upd = timed(psteps, args.steps)
        C, _, _, _ = st.measure_corr()
        ev = np.linalg.eigvalsh((C + C.conj().T) / 2)
        res.update({"metric": "two-site updates/s, purified L=32 chi=64 chi_k=4", "value": v, "updates": n_upd,
                    "eig_C": [float(ev.min()), float(ev.max())], "max_bond_dim": int(max(st.dims(0))),
                    "config": {"L": L, "chi": chi, "chi_k": chik, "dt": dt, "untimed_steps": pre,
                               "timed_steps": args.steps, "start": "Neel", "theta_bits": args.theta_bits, "buckets": not args.no_buckets}})
        st.close()
    print(json.dumps(res))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per run: --gpus must be 1 (the batch on one GPU is the measured unit)"}))
        sys.exit(2)
    if args.summarize_trace:
        print("\n".join(summarize_trace(args.summarize_trace)))
        return
    if args.summarize_pmc:
        print("\n".join(summarize_pmc(*args.summarize_pmc)))
        return
    if args.summarize_counters:
        print("\n".join(summarize_counters(args.summarize_counters)))
        return
    if args.workload != "qsd":
        run_workload(args)
        return
    # the oracle's CPU work runs in processes started before this process touches the GPU: the
    # timing first, then a pool kept for the accuracy checks
    quick = args.calib_copy > 0 or args.profile_only
    cpu = None if (args.no_cpu or quick) else cpu_baseline(args.L, args.chi, args.dt, args.cpu_seconds)
    pool = None
    if not (args.no_check or quick):
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(6)
    import torch
    import tn_inputs
    from paper_2609_18841_amd import api

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calib_copy > 0:
        # reference traffic for the FETCH_SIZE / WRITE_SIZE counters: each copy reads and writes
        # exactly MIB MiB
        nb = args.calib_copy << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": nb, "copies": 3}))
        return
    B, L, chi, inner, dt = args.batch, args.L, args.chi, args.inner, args.dt
    log = lambda msg: print(f"# {msg}", file=sys.stderr, flush=True)  # noqa: E731

    cks, ck_info = None, None
    if args.input == "physical" or not (args.no_secondary or args.profile_only):
        t0 = time.perf_counter()
        if args.checkpoint_file and os.path.exists(args.checkpoint_file):
            z = np.load(args.checkpoint_file)
            cks = [([z[f"t{b}_{i}"] for i in range(L)], [z[f"l{b}_{i}"] for i in range(L - 1)], float(z["ln"][b]))
                   for b in range(int(z["count"]))]
            t_ck, ck_dims = float(z["t"]), [list(z["dims"][b]) for b in range(int(z["count"]))]
        else:
            cks, t_ck, ck_dims = evolve_checkpoints(api, tn_inputs, L, chi, args.checkpoints, args.ck_dt,
                                                    args.ck_tmax)
            if args.checkpoint_file:
                arrs = {"count": len(cks), "t": t_ck, "dims": np.array(ck_dims), "ln": np.array([c[2] for c in cks])}
                for b, (tt, ll, _) in enumerate(cks):
                    arrs.update({f"t{b}_{i}": x for i, x in enumerate(tt)})
                    arrs.update({f"l{b}_{i}": x for i, x in enumerate(ll)})
                np.savez(args.checkpoint_file, **arrs)
        ck_info = {"count": args.checkpoints, "evolved_to_t": t_ck, "dt": args.ck_dt, "precision": "fp64",
                   "start": "Neel", "max_bond_dim": int(max(max(d) for d in ck_dims)),
                   "saturated_bonds": int(sum(1 for d in ck_dims[0] if d == chi)),
                   "seconds": time.perf_counter() - t0}
        log(f"checkpoints: {args.checkpoints} trajectories evolved to t = {t_ck:.2f}")
    head_cks = cks if args.input == "physical" else None

    bits, other_bits = args.theta_bits, 96 - args.theta_bits
    st, init = make_state(api, tn_inputs, api.SPLIT, B, L, chi, head_cks, bits=bits)
    total_steps = args.warmup + args.steps + 1
    noise = tn_inputs.normals(7, (total_steps * inner, B * 2 * 2))
    log(f"bench: B={B} L={L} chi={chi} inner={inner} warmup={args.warmup} steps={args.steps} input={args.input}")

    overlap = args.overlap_measure
    if overlap:
        st.measure_async_enable()
    if args.no_overlap or args.profile_only:
        st.overlap(False)
    if args.no_buckets:
        st.buckets(on=0)
    if args.profile_only:
        st.tuning(0)  # the autotuner's choice at this shape, without its timing dispatches
        for w in range(args.warmup):
            run_interval(api, st, noise[w * inner:(w + 1) * inner], inner, dt)
        kt, dims0 = _profiled_interval(api, st, noise[args.warmup * inner:], inner, dt, B)
        roof, work, n_items, tmin = roofline_line(api, st, kt, dims0, inner, chi)
        print(json.dumps({"profile_only": True, "config": {"batch": B, "L": L, "chi": chi, "input": args.input,
                                                           "theta_bits": bits, "warmup": args.warmup},
                          "roofline": roof, "kernel_ms_profiled_interval": kt}))
        return

    def interval(i0, pending):
        # the steps of one output interval, then its measurement: with overlap the measurement of
        # a snapshot runs beside the next interval's steps and is collected before the next start
        run_interval(api, st, noise[i0:i0 + inner], inner, dt, measure=not overlap)
        if overlap:
            if pending:
                st.measure_finish()
            st.measure_start(0)
        return overlap

    pending = False
    for w in range(args.warmup):
        pending = interval(w * inner, pending)
        log(f"warmup {w} done")
    if pending:
        st.measure_finish()
        pending = False
    st.stats(reset=True)

    # timed region: kernel timing off, so unmasked Trotter steps replay their captured graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        pending = interval((args.warmup + s_) * inner, pending)
        log(f"step {s_} done")
    if pending:
        st.measure_finish()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    updates = args.steps * inner * (L - 1) * B
    value = updates / el
    fb_items, mgs_items = st.stats()

    # roofline from a separate profiled interval (one stream, HIP events), after the timed region
    kt, dims0 = _profiled_interval(api, st, noise[(args.warmup + args.steps) * inner:], inner, dt, B)
    dims1 = [st.dims(b) for b in range(B)]
    changed = float(np.mean([np.mean(np.asarray(a) != np.asarray(b)) for a, b in zip(dims0, dims1)]))
    roof, work, n_items, tmin = roofline_line(api, st, kt, dims0, inner, chi)
    roof["bond_dims_changed_during_interval"] = changed
    interval_ms = sum(v["total_ms"] for k, v in kt.items())
    pm = path_model(2, chi)
    t_min_avg = tmin / n_items
    path_roof = {"flops_per_update_square": pm["flops_per_update"], "t_min_us_square": pm["t_min_us"],
                 "t_min_us_per_update": t_min_avg * 1e6, "bound_updates_per_s": 1.0 / t_min_avg,
                 "frac": value * t_min_avg,
                 "frac_updates_only": value * t_min_avg / max(1e-9, 1.0 - kt["measure"]["total_ms"] / interval_ms),
                 "measure_share_of_kernel_time": kt["measure"]["total_ms"] / interval_ms,
                 "basis": "value (with the measurement sweep) against the flop model summed over each bond's shape"}
    buckets = None if args.no_buckets else [[n, nb, hv] for n, nb, hv in st.buckets(parity=0)]
    del st
    torch.cuda.empty_cache()

    # plain per-instance FP64 GPU path (one instance per call), same input
    plain = None
    if not args.no_plain:
        pst, _ = make_state(api, tn_inputs, api.FP64, 1, L, chi, head_cks)
        run_interval(api, pst, noise[:1, :4], 1, dt, measure=False)
        rates = []
        for r in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            run_interval(api, pst, noise[r * args.plain_steps:(r + 1) * args.plain_steps, :4], args.plain_steps, dt,
                         measure=False)
            torch.cuda.synchronize()
            rates.append(args.plain_steps * (L - 1) / (time.perf_counter() - t1))
        pv = float(np.mean(rates))
        plain = {"value": pv, "unit": "two-site updates/s", "precision": "fp64", "batch": 1,
                 "steps_timed": 3 * args.plain_steps, "runs": rates, "speedup_split_batched": value / pv}
        del pst
        torch.cuda.empty_cache()
        log("plain fp64 done")

    # batched FP64 at the full batch: separates the batching gain from the precision gain
    fp64b = None
    if args.fp64_batched_steps > 0:
        fst, _ = make_state(api, tn_inputs, api.FP64, B, L, chi, head_cks)
        run_interval(api, fst, noise[:1], 1, dt, measure=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_interval(api, fst, noise[1:1 + args.fp64_batched_steps], args.fp64_batched_steps, dt, measure=False)
        torch.cuda.synchronize()
        fv = args.fp64_batched_steps * (L - 1) * B / (time.perf_counter() - t1)
        fp64b = {"value": fv, "unit": "two-site updates/s", "precision": "fp64", "batch": B,
                 "steps_timed": args.fp64_batched_steps, "measurement": "none (Trotter steps and noise only)",
                 "split_over_fp64_batched": value / fv}
        del fst
        torch.cuda.empty_cache()
        log("batched fp64 done")

    def short_run(start_cks, b, n_int=2):
        """updates/s of a split batch over n_int output intervals after one untimed interval, and the
        eigensolver route counts of the timed ones"""
        sst, _ = make_state(api, tn_inputs, api.SPLIT, B, L, chi, start_cks, bits=b)
        run_interval(api, sst, noise[:inner], inner, dt)
        sst.stats(reset=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for r in range(n_int):
            run_interval(api, sst, noise[(r + 1) * inner:(r + 2) * inner], inner, dt)
        torch.cuda.synchronize()
        v = n_int * inner * (L - 1) * B / (time.perf_counter() - t1)
        f, m = sst.stats()
        sst.close()
        del sst
        torch.cuda.empty_cache()
        return {"value": v, "unit": "two-site updates/s", "steps": n_int, "cluster_items": f,
                "reorthogonalized_items": m, "updates": n_int * inner * (L - 1) * B}

    # the other Theta precision on the headline input
    other = dict(short_run(head_cks, other_bits), theta_bits=other_bits)
    log(f"theta bits {other_bits} done")

    # secondary input: the geometric-spectrum tensors (or the checkpoints when they are not the headline)
    second = None
    if not args.no_secondary:
        alt = None if head_cks is not None else cks
        second = {"input": "synthetic geometric spectrum" if alt is None else "physical checkpoints",
                  "theta_bits": bits, **short_run(alt, bits),
                  "other_theta_bits": dict(short_run(alt, other_bits), theta_bits=other_bits)}
        log("secondary input done")

    ntraj = max(2, args.check_trajectories)

    def gpu_trajectory(start_cks, b):
        """the trajectories of a small split batch (ntraj of them), bucketed like the timed batch
        (a trajectory's result does not depend on the other items of its chunks): their starts, the
        noise the oracle replays, and C of each after one output interval and after check_steps
        Trotter steps"""
        cst, _ = make_state(api, tn_inputs, api.SPLIT, ntraj, L, chi, start_cks, bits=b)
        cst.buckets(on=0 if args.no_buckets else 2)
        nlong = max(inner, args.check_steps)
        nz = tn_inputs.normals(7, (nlong, B * 2 * 2))[:, :ntraj * 2 * 2]
        Cg = {}
        for k in range(nlong):
            cst.tebd_step(dt, order=1)
            cst.apply_jumps(api.MODE_QSD, dt, nz[k], api.NOISE_GAUSS)
            if k + 1 in (inner, nlong):
                Cg[k + 1] = cst.measure_corr(normalize=0, each=True)[2][:ntraj]
        cst.close()
        if start_cks is None:
            t0, l0, _ = tn_inputs.random_isometric_mps(2024, L, chi)
            starts = [(t0, l0, 0.0)] * ntraj
        else:
            starts = [start_cks[t % len(start_cks)] for t in range(ntraj)]
        return starts, nz, Cg

    def summarize(checks):
        return {str(n): dict(zip(["err_vs_fp64_oracle", "oracle_driver_spread", "density_elementwise",
                                  "nearest_neighbour_elementwise", "oracle_c64_start_spread"], v))
                for n, v in sorted(checks.items())}

    checks = checks2 = checks_o = checks2_o = by_traj = None
    err = spread = None
    if not args.no_check:
        # both Theta precisions on each input, against the same oracle runs
        starts = [head_cks] + ([None if head_cks is not None else cks] if second is not None else [])
        runs = []
        for sc in starts:
            st_a, nz_a, Cg_a = gpu_trajectory(sc, bits)
            _, _, Cg_b = gpu_trajectory(sc, other_bits)
            runs.append((st_a, nz_a, Cg_a, Cg_b))
        traj = lambda C, t: {n: c[t] for n, c in C.items()}  # noqa: E731
        # trajectory 0 of each input with three oracle runs, trajectories 1.. of the first input with
        # one (gesdd), all side by side in the pool
        jobs = [j for st_a, z, c, _ in runs for j in oracle_jobs(st_a[0], L, chi, dt, z[:, 0:4], traj(c, 0), c64start=True)]
        st_a, z, c, _ = runs[0]
        extra = [(st_a[t], L, chi, dt, z[:, 4 * t:4 * t + 4], sorted(c), "gesdd") for t in range(1, ntraj)]
        flat = pool.map(_oracle_corr_run, jobs + extra)
        outs = [(oracle_compare(traj(c, 0), flat[3 * r:3 * r + 3], c64start=True),
                 oracle_compare(traj(c2, 0), flat[3 * r:3 * r + 3], c64start=True))
                for r, (_, _, c, c2) in enumerate(runs)]
        checks, checks_o = outs[0]
        if len(outs) > 1:
            checks2, checks2_o = outs[1]
        err, spread = checks[inner][:2]
        ref = [flat[0]] + flat[len(jobs):]
        by_traj = {str(n): [float(np.max(np.abs(c[n][t] - ref[t][n])) / np.max(np.abs(ref[t][n])))
                            for t in range(ntraj)] for n in sorted(c)}
        log("oracle check done")
    if pool is not None:
        pool.close()
        pool.join()

    workload = (f"QSD trajectory batch B={B}, L={L}, chi={chi}, dt={dt}, {inner} Trotter steps + noise per "
                f"output, 1 measurement of C per output; split precision; start: "
                + ("FP64-evolved checkpoints" if head_cks is not None else "geometric-spectrum tensors"))
    res = {
        "metric": "two-site TEBD updates/sec (batched trajectories, L=64 chi=64) vs plain, at stated err",
        "value": value, "unit": "two-site updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64-store/f64-contract/f64-svd" if bits == 64 else "c64-store/f32-contract/f64-svd",
        "data": "synthetic",
        "config": {"workload": workload, "batch": B, "L": L, "chi": chi, "dt": dt, "inner_steps": inner,
                   "input": args.input, "checkpoints": ck_info, "theta_bits": bits,
                   "measurement": "beside the next interval's steps (snapshot)" if overlap else "synchronous",
                   "timing": "kernel timing off; captured HIP graphs replay the Trotter steps",
                   "chunk_streams": 1 if args.no_overlap else 2,
                   "bond_size_buckets": buckets},
        "roofline": roof, "path_roofline": path_roof,
        "cpu_baseline": cpu, "plain_fp64": plain, "fp64_batched": fp64b, "secondary_input": second,
        "eigensolver_routes": {"cluster_items": fb_items, "reorthogonalized_items": mgs_items,
                               "updates": updates},
        "err_vs_fp64_oracle": err, "oracle_driver_spread": spread, "err_tolerance": ERR_TOLERANCE,
        "err_within_tolerance": None if by_traj is None else {n: max(v) <= ERR_TOLERANCE for n, v in by_traj.items()},
        "err_by_trajectory": by_traj,
        "err_by_steps": None if checks is None else summarize(checks),
        "secondary_err_by_steps": None if checks2 is None else summarize(checks2),
        "secondary_err_within_tolerance": None if checks2 is None else {
            str(n): v[0] <= ERR_TOLERANCE for n, v in sorted(checks2.items())},
        "other_theta_bits": dict(other, err_by_steps=None if checks_o is None else summarize(checks_o),
                                 secondary_err_by_steps=None if checks2_o is None else summarize(checks2_o)),
        "kernel_ms_profiled_interval": kt,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
