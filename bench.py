"""Benchmark: batched two-site TEBD updates/s on one MI355X.

Workload (one bench step = one output interval of a quantum-state-diffusion batch):
  B trajectories of the boundary-driven free-fermion chain (J = 1, gamma = 0.5, source s+ on
  the first site, sink s- on the last), L = 64 sites, bond dimension chi = 64, SPLIT precision
  (complex64 MFMA contractions, FP64 Gram/eigensolver/weights/norms); per bench step:
    INNER first-order Trotter steps (dt = 0.01) of exp(-i h^eff dt) gates, each followed by the
    diffusion factors 1 + dW sqrt(gamma) L with complex Gaussian dW, then one measurement of
    C_ij = <c_i^+ c_j> for every trajectory (the output time).
  Inputs are synthetic and seeded: a right-isometric MPS with geometric bond weights
  (sigma_a ~ exp(-a/8)) at chi = 64 on every saturated bond stands in for a pre-evolved state.
Reported: value = two-site updates/s of the batched split path (whole job), the plain
per-instance FP64 GPU path for comparison, the roofline fraction of the dominant kernel
(HIP events on the library stream), value as a fraction of the path's flop-model bound, and the
CPU oracle timed on a bounded sample (one core, and one process per core).
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
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_qsd_B256_L64_chi64_split.txt")


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


def profiled_traffic(kernel):
    """HBM bytes per launch of the timing bucket whose kernel is `kernel` (the sum over its template
    instances: the Householder reduction is a head and a tail dispatch) from the committed counter
    summary, or None when the summary is missing or was taken with different kernel sources."""
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
    tot, found = 0.0, False
    for ln in lines:
        if ln.startswith("#"):
            continue
        parts = ln.split()
        nm = " ".join(parts[:-3]).replace("void ", "").split("<")[0].strip()
        if nm == kernel:
            tot += float(parts[-1])
            found = True
    return tot if found else None


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
    ap.add_argument("--plain-instances", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-clock window of the all-core oracle run (the single-core run takes up to 6 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--overlap-measure", action="store_true",
                    help="measure each output from a snapshot, beside the next interval's steps")
    ap.add_argument("--check-steps", type=int, default=100,
                    help="Trotter steps of the longer oracle comparison (besides one output interval)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration) and exit")
    return ap.parse_args()


# relative singular-value cutoff of the timed state (split precision) and of the FP64 paths
SV_CUTOFF = {"split": 1e-6, "fp64": 1e-12}


def make_state(api, tn_inputs, prec, B, L, chi, seed=2024):
    model = api.Model.free_fermion(L, 1.0, 0.5)
    st = api.State(api.KIND_MPS, model, B, chi, tn_inputs.neel(L), precision=prec,
                   sv_cutoff=SV_CUTOFF["split"] if prec == api.SPLIT else SV_CUTOFF["fp64"])
    tensors, lams, dims = tn_inputs.random_isometric_mps(seed, L, chi)
    st.set_instance(0, tensors, lams, 0.0)
    if B > 1:
        st.replicate(0)
    return st, (tensors, lams)


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


def oracle_check(tn_inputs, st_init, L, chi, dt, noise, C_gpu0):
    """{steps: (err, spread, err_density, err_nn)} for trajectory 0 at each checkpoint of C_gpu0
    ({steps: C}).  err and spread are max |dC| / max |C|: err is the GPU against the FP64 oracle on
    the same input and with the same truncation (chi and the split state's singular-value cutoff);
    spread is the oracle against itself with another LAPACK SVD driver (gesvd instead of gesdd).
    At a binding chi the kept singular vectors depend on rounding inside the SVD, and spread is the
    scale at which two exact FP64 runs already differ.  err_density and err_nn are the GPU's
    elementwise relative errors on the diagonal (densities) and on the first off-diagonal."""
    from threadpoolctl import threadpool_limits
    from oracle import model as M, tebd, stochastic, measure
    mdl = M.Model(L)
    cache = {}

    def fn(b, tau):
        if (b, tau) not in cache:
            cache[(b, tau)] = M.gate_heff(mdl, b, tau)
        return cache[(b, tau)]
    tensors, lams = st_init
    last = max(C_gpu0)
    Cs = {"gesdd": {}, "gesvd": {}}
    with threadpool_limits(limits=1):
        for driver in Cs:
            st = tebd.TNState([t.copy() for t in tensors], [l.copy() for l in lams])
            for k in range(last):
                stochastic.qsd_step(st, mdl.jumps, dt, noise[k][0:4], fn, chi, SV_CUTOFF["split"], driver=driver)
                if k + 1 in C_gpu0:
                    Cs[driver][k + 1] = measure.corr_mps(st, normalize=False)[0]
    out = {}
    for n, Cg in C_gpu0.items():
        ref = Cs["gesdd"][n]
        scale = np.max(np.abs(ref))
        out[n] = (float(np.max(np.abs(Cg - ref)) / scale), float(np.max(np.abs(Cs["gesvd"][n] - ref)) / scale),
                  _elementwise(np.diag(Cg), np.diag(ref)), _elementwise(np.diag(Cg, 1), np.diag(ref, 1)))
    return out


def _elementwise(a, b):
    """max_i |a_i - b_i| / |b_i| (the densities C_ii, or the nearest-neighbour terms C_i,i+1)."""
    return float(np.max(np.abs(a - b) / np.abs(b)))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per run: --gpus must be 1 (the batch on one GPU is the measured unit)"}))
        sys.exit(2)
    # the oracle's CPU timing runs first, before this process touches the GPU (its worker
    # processes start from a process without GPU state)
    cpu = None if (args.no_cpu or args.calib_copy > 0) else cpu_baseline(args.L, args.chi, args.dt, args.cpu_seconds)
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
    st, init = make_state(api, tn_inputs, api.SPLIT, B, L, chi)
    total_steps = args.warmup + args.steps
    noise = tn_inputs.normals(7, (total_steps * inner, B * 2 * 2))
    print(f"# bench: B={B} L={L} chi={chi} inner={inner} warmup={args.warmup} steps={args.steps}", file=sys.stderr,
          flush=True)

    err = spread = None
    overlap = args.overlap_measure
    if overlap:
        st.measure_async_enable()

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
        print(f"# warmup {w} done", file=sys.stderr, flush=True)
    if pending:
        st.measure_finish()
        pending = False

    torch.cuda.synchronize()
    st.prof_enable(True)
    t0 = time.perf_counter()
    for s in range(args.steps):
        pending = interval((args.warmup + s) * inner, pending)
        print(f"# step {s} done", file=sys.stderr, flush=True)
    if pending:
        st.measure_finish()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    updates = args.steps * inner * (L - 1) * B
    value = updates / el
    kt = {}
    for kid, name in enumerate(api.K_NAMES):
        ms, n = st.prof_query(kid)
        kt[name] = {"total_ms": ms, "launches": n, "busy_ms": st.prof_busy(kid)}
    st.prof_enable(False)

    # Roofline of the dominant update kernel (FLOP-bound, FP64 or FP32 peak by kernel type).  The
    # chunks of a layer run on two streams (when a layer spans more than one chunk), so two
    # launches of the same kernel can run at once and each one's duration covers both; the
    # kernel's rate is its algorithmic work over the wall time during which any launch of it
    # runs (union of the launch intervals, HIP events on both streams).  busy_ms_per_launch is
    # that time per launch, comparable with the union of dispatch intervals in the committed
    # rocprofv3 kernel trace; avg_launch_ms is the plain per-launch duration.
    fl = algo_flops(n=2 * chi, m=2 * chi, chim=chi, k=chi)
    upd_kernels = ["theta", "gram", "hetrd", "vecs", "split"]
    dom = max(upd_kernels, key=lambda k: kt[k]["busy_ms"])
    peak = PEAK["fp32"] if dom in ("theta", "split") else PEAK["fp64"]
    launches = max(1, kt[dom]["launches"])
    items_per_launch = updates / launches
    busy_s = kt[dom]["busy_ms"] / 1e3
    achieved = fl[dom] * updates / busy_s if busy_s > 0 else 0.0
    kname, bound = bucket_kernel(dom, 2 * chi, chi, st.tuning()[0])
    roof = {"bound": bound, "kernel": kname,
            "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": profiled_traffic(kname), "traffic_unit": "bytes per launch",
            "algo_flops_per_update": fl[dom], "items_per_launch": items_per_launch,
            "busy_ms_per_launch": kt[dom]["busy_ms"] / launches,
            "avg_launch_ms": kt[dom]["total_ms"] / launches,
            "streams": 2 if kt[dom]["total_ms"] > 1.2 * kt[dom]["busy_ms"] else 1}

    # plain per-instance FP64 GPU path (one instance per call), same workload shape
    plain = None
    if not args.no_plain:
        del st
        torch.cuda.empty_cache()
        pst, _ = make_state(api, tn_inputs, api.FP64, 1, L, chi)
        pst.tebd_step(dt, order=1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.plain_instances):
            pst.tebd_step(dt, order=1)
            pst.apply_jumps(api.MODE_QSD, dt, noise[i][:4], api.NOISE_GAUSS)
        torch.cuda.synchronize()
        pel = time.perf_counter() - t1
        pv = args.plain_instances * (L - 1) / pel
        plain = {"value": pv, "unit": "two-site updates/s", "precision": "fp64",
                 "instances_timed": args.plain_instances, "speedup_split_batched": value / pv}
        del pst
        torch.cuda.empty_cache()

    checks = None
    if not args.no_check:
        # trajectory 0 of a two-trajectory batch against the oracle after one output interval and
        # after check_steps Trotter steps, on the same noise
        cst, init2 = make_state(api, tn_inputs, api.SPLIT, 2, L, chi)
        nlong = max(inner, args.check_steps)
        nz = tn_inputs.normals(7, (nlong, B * 2 * 2))[:, :2 * 2 * 2]
        Cg = {}
        for k in range(nlong):
            cst.tebd_step(dt, order=1)
            cst.apply_jumps(api.MODE_QSD, dt, nz[k], api.NOISE_GAUSS)
            if k + 1 in (inner, nlong):
                Cg[k + 1] = cst.measure_corr(normalize=0, each=True)[2][0]
        checks = oracle_check(tn_inputs, init2, L, chi, dt, nz, Cg)
        err, spread = checks[inner][:2]
        del cst

    pm = path_model(2, chi)
    res = {
        "metric": "two-site TEBD updates/sec (batched trajectories, L=64 chi=64) vs plain, at stated err",
        "value": value, "unit": "two-site updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64-contract/f64-svd", "data": "synthetic",
        "config": {"workload": f"QSD trajectory batch B={B}, L={L}, chi={chi}, dt={dt}, {inner} Trotter steps + "
                               f"noise per output, 1 measurement of C per output; split precision",
                   "batch": B, "L": L, "chi": chi, "dt": dt, "inner_steps": inner,
                   "measurement": "beside the next interval's steps (snapshot)" if overlap else "synchronous"},
        "roofline": roof, "path_roofline": dict(pm, frac=value * pm["t_min_us"] * 1e-6),
        "cpu_baseline": cpu, "plain_fp64": plain,
        "err_vs_fp64_oracle": err, "oracle_driver_spread": spread,
        "err_by_steps": None if checks is None else {
            str(n): {"err_vs_fp64_oracle": e, "oracle_driver_spread": sp, "density_elementwise": ed,
                     "nearest_neighbour_elementwise": en} for n, (e, sp, ed, en) in sorted(checks.items())},
        "kernel_ms": kt,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
