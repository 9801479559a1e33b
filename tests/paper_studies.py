"""The paper's N = 24 studies at its own parameters, run through the library on one GPU.

Not a pytest module (the short trend checks live in test_gpu_studies.py); each run takes minutes:
    python tests/paper_studies.py mpdo      # Sec. 3.1, fig-Algo1a/b: chi 64 (dt 0.01, 0.003), chi 32 (dt 0.01)
    python tests/paper_studies.py mpdo --only 64,0.001 --stop-at 9.5 --save a.npz   # dt 0.001, in two
    python tests/paper_studies.py mpdo --only 64,0.001 --resume a.npz               # sittings
    python tests/paper_studies.py purified  # Sec. 3.2, fig-Algo2a/b: chi 64, chi_k 4, dt 0.003
    python tests/paper_studies.py qt        # Sec. 4.1, fig-Algo3a/b and fig-Algo5: 3000 histories, chi 16
    python tests/paper_studies.py qsd       # Sec. 4.2, fig-Algo4a/b and fig-Algo5: 3000 histories, chi 16
    python tests/paper_studies.py qsd --noise binary   # the same with the paper's eta = +-1 increments
Model (Sec. 2.1): free fermions, J = 1, a source c_1^+ and a sink c_N at rate gamma = 0.5 (the paper
states no rate; this is the configurations' value), the vacuum as initial state, t up to 18.89.
At every output time (every 0.5 and at the end) the density n_i = C_ii and the current
j_i = i (C_{i,i-1} - C_{i-1,i}) are compared with the exact solution (eq. SoleqCorr) by the
root-mean-square deviation the figures plot, sqrt((1/N) sum_i (n_i - n_i^exact)^2) (and over the
N - 1 currents).  Trajectory studies report it for the first 300, 1000 and 3000 histories, with
the statistical error of eq. ErrorCLT of the density (for QSD also the ratio estimator of the
linear unravelling and the spread of the norms), and for fig-Algo5 the density of site 8 in eight
histories.  Results go to a JSON file (--out) and one progress line per output time.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import tn_inputs  # noqa: E402
from oracle import exact, stats  # noqa: E402

N, J, GAMMA, T_END = 24, 1.0, 0.5, 18.89
OCC = [0] * N


def rms(C, Cx):
    n, j = exact.density_current(C)
    nx, jx = exact.density_current(Cx)
    return float(np.sqrt(np.mean((n - nx) ** 2))), float(np.sqrt(np.mean((j - jx) ** 2)))


def schedule(dt):
    """(number of steps, steps between outputs): outputs every 0.5 and at T_END."""
    n = int(round(T_END / dt))
    return n, int(round(0.5 / dt))


def log(msg):
    print(msg, flush=True)


def run_mpdo(api, only=None, stop_at=None, resume=None, save=None):
    """only: one (chi, dt) instead of the three runs; stop_at: end the run at the first output time
    >= stop_at and write the state and the rows so far to `save` (an npz), from which `resume`
    continues (runs longer than one sitting split in two)."""
    out = []
    for chi, dt in ([only] if only else ((64, 0.01), (64, 0.003), (32, 0.01))):
        st = api.State(api.KIND_MPDO, api.Model.free_fermion(N, J, GAMMA), 1, chi, OCC, precision=api.SPLIT,
                       sv_cutoff=1e-6)
        st.theta_precision(64)
        n, every = schedule(dt)
        rows, t0, k0 = [], time.time(), 0
        if resume:
            z = np.load(resume)
            k0 = int(z["k"])
            st.set_instance(0, [z[f"t{i}"] for i in range(N)], [z[f"l{i}"] for i in range(N - 1)], float(z["ln"]))
            rows = json.loads(str(z["rows"]))
            log(f"mpdo chi={chi} dt={dt}: resumed at step {k0} (t = {k0 * dt:.2f})")
        for k in range(k0 + 1, n + 1):
            st.tebd_step(dt, order=2)
            if k % every == 0 or k == n:
                C, _, _, tr = st.measure_corr()
                e_n, e_j = rms(C, exact.c_exact(k * dt, OCC, J, GAMMA))
                rows.append({"t": k * dt, "rms_n": e_n, "rms_j": e_j, "trace": float(tr[0])})
                log(f"mpdo chi={chi} dt={dt} t={k * dt:.2f}: rms n {e_n:.3e} j {e_j:.3e} ({time.time() - t0:.0f} s)")
                if stop_at is not None and k * dt >= stop_at and k < n:
                    tens, lams, ln, _ = st.get_instance(0)
                    arrs = {"k": k, "ln": ln, "rows": json.dumps(rows)}
                    arrs.update({f"t{i}": x for i, x in enumerate(tens)})
                    arrs.update({f"l{i}": x for i, x in enumerate(lams)})
                    np.savez(save, **arrs)
                    log(f"mpdo chi={chi} dt={dt}: stopped at step {k}, state in {save}")
                    st.close()
                    return [{"chi": chi, "dt": dt, "order": 2, "precision": "split (Theta FP64)", "rows": rows,
                             "stopped_at_step": k}]
        out.append({"chi": chi, "dt": dt, "order": 2, "precision": "split (Theta FP64)", "rows": rows})
        st.close()
    return out


def run_purified(api):
    chi, chik, dt = 64, 4, 0.003
    st = api.State(api.KIND_PURIFIED, api.Model.free_fermion(N, J, GAMMA), 1, chi, OCC, chi_k_max=chik,
                   precision=api.SPLIT, sv_cutoff=1e-6)
    st.theta_precision(64)
    n, every = schedule(dt)
    rows, t0 = [], time.time()
    for k in range(1, n + 1):
        st.tebd_step(dt, order=1)
        st.apply_jumps(api.MODE_KRAUS, dt)
        if k % every == 0 or k == n:
            C, _, _, _ = st.measure_corr()
            ev = np.linalg.eigvalsh((C + C.conj().T) / 2)
            e_n, e_j = rms(C, exact.c_exact(k * dt, OCC, J, GAMMA))
            rows.append({"t": k * dt, "rms_n": e_n, "rms_j": e_j, "eig_min": float(ev.min()), "eig_max": float(ev.max())})
            log(f"purified t={k * dt:.2f}: rms n {e_n:.3e} j {e_j:.3e} eig(C) [{ev.min():.2e}, {ev.max():.4f}] "
                f"({time.time() - t0:.0f} s)")
    st.close()
    return [{"chi": chi, "chi_k": chik, "dt": dt, "order": 1, "precision": "split (Theta FP64)", "rows": rows}]


def run_trajectories(api, kind, noise="gauss"):
    chi, dt, B = 16, 0.003, 3000
    st = api.State(api.KIND_MPS, api.Model.free_fermion(N, J, GAMMA), B, chi, OCC, precision=api.SPLIT,
                   sv_cutoff=1e-6)
    st.theta_precision(64)
    n, every = schedule(dt)
    rows, hist, t0 = [], [], time.time()
    block, rnd = None, None
    for k in range(1, n + 1):
        b0 = (k - 1) // every
        if b0 != block:  # random inputs, one seeded block per output interval
            block = b0
            if kind == "qt" or noise == "binary":
                rnd = tn_inputs.uniforms(1000 + b0 if kind == "qt" else 3000 + b0, (every, B * (1 if kind == "qt" else 2)))
            else:
                rnd = tn_inputs.normals(2000 + b0, (every, B * 4))
        r = rnd[(k - 1) % every]
        if kind == "qt":
            _, mask = st.apply_jumps(api.MODE_QT, dt, r)
            st.tebd_step(dt, order=1, mask=mask)
        else:
            st.tebd_step(dt, order=1)
            st.apply_jumps(api.MODE_QSD, dt, r, api.NOISE_BINARY if noise == "binary" else api.NOISE_GAUSS)
        if k % every == 0 or k == n:
            # QT histories are normalized; QSD keeps the linear values (its estimator, Sec. 4.2)
            Cm, var, Ce, nrm = st.measure_corr(normalize=1 if kind == "qt" else 0, each=True)
            Cx = exact.c_exact(k * dt, OCC, J, GAMMA)
            row = {"t": k * dt}
            for nc in (300, 1000, 3000):
                e_n, e_j = rms(stats.batch_mean(Ce[:nc]), Cx)
                row[f"rms_n_{nc}"], row[f"rms_j_{nc}"] = e_n, e_j
                if kind == "qsd":  # the ratio estimator, which divides out the norms' spread
                    e_n, e_j = rms(stats.ratio_mean(Ce[:nc], nrm[:nc]), Cx)
                    row[f"ratio_rms_n_{nc}"], row[f"ratio_rms_j_{nc}"] = e_n, e_j
            row["norm_mean"], row["norm_std"] = float(np.mean(nrm)), float(np.std(nrm))
            err = np.sqrt(np.real(np.diag(var)) / B)
            row["clt_err_n_max"] = float(err.max())
            dens8 = np.real(Ce[:8, 7, 7]) / (1.0 if kind == "qt" else nrm[:8])
            hist.append([k * dt] + [float(x) for x in dens8])
            rows.append(row)
            extra = (f", ratio estimator {row['ratio_rms_n_3000']:.3e}, norms {row['norm_mean']:.3f} +- "
                     f"{row['norm_std']:.3f}" if kind == "qsd" else "")
            log(f"{kind} t={k * dt:.2f}: rms n (300/1000/3000) {row['rms_n_300']:.3e} {row['rms_n_1000']:.3e} "
                f"{row['rms_n_3000']:.3e}, CLT err n <= {err.max():.2e}{extra} ({time.time() - t0:.0f} s)")
    st.close()
    return [{"chi": chi, "dt": dt, "histories": B, "order": 1, "precision": "split (Theta FP64)", "rows": rows,
             "noise": noise if kind == "qsd" else None, "site8_eight_histories": hist}]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["mpdo", "purified", "qt", "qsd"])
    ap.add_argument("--out", default="")
    ap.add_argument("--noise", choices=["gauss", "binary"], default="gauss", help="QSD increments")
    ap.add_argument("--only", default="", help="mpdo: one run, 'chi,dt'")
    ap.add_argument("--stop-at", type=float, default=None, help="mpdo: stop at this time and save the state")
    ap.add_argument("--save", default="", help="mpdo: npz written at --stop-at")
    ap.add_argument("--resume", default="", help="mpdo: npz to continue from")
    args = ap.parse_args()
    import torch
    from paper_2609_18841_amd import api
    torch.cuda.set_device(0)
    only = None
    if args.only:
        c, d = args.only.split(",")
        only = (int(c), float(d))
    res = {"mpdo": lambda a: run_mpdo(a, only, args.stop_at, args.resume or None, args.save or None),
           "purified": run_purified}.get(args.study, lambda a: run_trajectories(a, args.study, args.noise))(api)
    doc = {"study": args.study, "N": N, "J": J, "gamma": GAMMA, "start": "vacuum", "results": res}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(doc, f)
    log("done")


if __name__ == "__main__":
    main()
