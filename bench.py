"""Throughput of batched Ehrenfest mean-field trajectory propagation on one MI355X.

Workload: the asymmetric-top + atom system with j <= 8 (all k, m; N = 969
channels), random smooth Hermitian complex coupling tables on 200 R points,
4096 trajectories in a mid-collision population (R0 uniform in 4-19.5 A,
b uniform in 0-min(12 A, 0.9 R0), E_coll uniform in 100-2000 cm^-1, initial
channel uniform over the 35 channels with j <= 2).  One bench step advances
every trajectory by a window of RK4 steps (dt = 12 a.u.) through the whole hot
path (interval lookup, phases, fused spline + complex matvec, mean-field
force and torque, classical update, final probabilities and diagnostics).
Inputs are synthetic and resident in HBM before timing starts.

Reported: trajectory-steps/s for the FP32-table form (value) and the FP64
form, the roofline position of the step kernel (HBM-bound: algorithmic table
bytes / measured kernel time), the FP32 - FP64 probability difference, and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("trajectory-steps/s × N² (coupling GB/s), FP32 vs FP64 at "
          "ΔP≤1e-4; adjoint s/grad")
HBM_PEAK_GBPS = 8000.0
MFMA_PEAK_TFLOPS = {"C64": 157.3, "C128": 78.6}   # dense FP32 / FP64 matrix peaks

# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs scaled by the same counters on a plain 1 GiB copy (profiles/).
# Valid only for the kernel source file and workload they were taken on.
MEASURED_TRAFFIC = {
    # FETCH_SIZE (x 1.99992, the copy calibration) + WRITE_SIZE of bin_gemm<C64> per
    # launch, taken on this source revision: the N=969 window (mean of the 41 launches
    # of one bench step) and the N=4096 collision (mean of all 40,020 launches)
    ("C64", "binned"): {"source": "binned.hip", "source_sha256_16": "36178d36d14d6324",
                        "bytes": 2.928e9, "window": 10, "trajectories": 4096},
    ("C64", "large"): {"source": "binned.hip", "source_sha256_16": "36178d36d14d6324",
                       "bytes": 1.9866e10, "trajectories": 512},
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--window", type=int, default=10, help="RK4 steps per bench step")
    ap.add_argument("--traj", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", choices=["C64", "C128"], default=None)
    ap.add_argument("--schedule", choices=["gemv", "binned", "both"], default="both")
    ap.add_argument("--adjoint", choices=["on", "off", "only"], default="on",
                    help="time one full gradient on the N=256 two-rotor workload")
    ap.add_argument("--adjoint-traj", type=int, default=1024)
    ap.add_argument("--adjoint-steps", type=int, default=4096)
    ap.add_argument("--adjoint-layout", choices=["dense", "sparse"], default="sparse",
                    help="table layout of the adjoint workload (sparse keeps every structural "
                         "nonzero: the same gradient)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--workload", choices=["headline", "window", "large", "uneven", "at",
                                           "coupling", "coupling_paper", "rates", "paper_at"],
                    default="headline",
                    help="headline (default): the N=4096 collision (512 trajectories x 10,000 RK4 "
                         "steps, binned, FP32 tables), one bench step = 1/--steps of it, with "
                         "the FP32-vs-FP64 adaptive runs, the N=969 windows, the uneven batch and "
                         "the adjoint as variants; "
                         "window: N=969 mid-collision windows; "
                         "large: N=4096, 512 full collisions of 10,000 RK4 steps on the binned "
                         "schedule; uneven: 20,000 trajectories of three systems with adaptive DP5; "
                         "at: decoupled (AT) dynamics, 64 trajectories x 100 initial states; "
                         "coupling: build the N=6825 top + rotor tables (83 terms, 63 knots); "
                         "coupling_paper: screened build for the 206,350-state p-H2O + p-H2 "
                         "basis; "
                         "rates: Eq. 20 and rate coefficients for 1032 levels, 10 energies, "
                         "20 temperatures; "
                         "paper_at: AT dynamics at the paper's size -- the screened 206,350-state "
                         "p-H2O + p-H2 matrices as a coordinate list, one path carrying the 100 "
                         "lowest states, the whole collision in RK4 steps of 10 a.u.")
    ap.add_argument("--large-n", type=int, default=4096)
    ap.add_argument("--large-traj", type=int, default=512)
    ap.add_argument("--large-steps", type=int, default=10000)
    ap.add_argument("--large-window", type=int, default=1000)
    ap.add_argument("--large-integrator", choices=["rk4", "dp5", "both"], default="rk4",
                    help="large workload: fixed RK4 windows, one adaptive DP5 call "
                         "(rtol = atol = 1e-8) on the binned schedule for the whole collision, "
                         "or both (with the largest difference of their final probabilities)")
    ap.add_argument("--large-windows", type=int, default=0,
                    help="run only the first windows of the collision (0: all)")
    ap.add_argument("--scatter-rmin", type=float, default=4.0,
                    help="large scatter population: smallest start radius (A); the start radii "
                         "are uniform up to 19.5 A")
    ap.add_argument("--large-scatter", type=int, default=0,
                    help="large workload: instead of the collision, time --steps windows of this "
                         "many RK4 steps of a scattered mid-collision population (R0 uniform in "
                         "4-19.5 A), the regime where few trajectories share a knot")
    ap.add_argument("--uneven-traj", type=int, default=20000)
    ap.add_argument("--uneven-max-steps", type=int, default=50000,
                    help="accepted-step limit (the workload's step counts range up to 50,000)")
    ap.add_argument("--uneven-schedule", choices=["auto", "queue", "split"], default="auto",
                    help="uneven workload: one call with the library's default split (the N=969 "
                         "class on the binned schedule beside the work list), everything on "
                         "the work list in one call (queue), or two calls one after the other "
                         "(split: the N=969 class binned, then the rest on the work list)")
    ap.add_argument("--headline-only", action="store_true",
                    help="headline workload without the variants (for profiler runs)")
    ap.add_argument("--uneven-layout", choices=["dense", "sparse"], default="sparse",
                    help="sparse: systems whose tables are mostly structural zeros keep only the "
                         "nonzeros (drop_below = 0, the same results)")
    ap.add_argument("--paper-steps", type=int, default=0,
                    help="paper_at workload: RK4 steps to time (0: the whole collision)")
    ap.add_argument("--only-paper", choices=["R32", "R64"], default=None,
                    help="paper_at workload: one storage type only")
    ap.add_argument("--probe-bw", action="store_true",
                    help="only measure streaming-read bandwidth at 2 GB, 200 MB and 8 MB footprints")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.probe_bw:
        print(json.dumps(read_bandwidth_probe()), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(trajectories shard trivially; see the design notes). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import systems as S

    if args.adjoint == "only":
        print(json.dumps(adjoint_timing(args.adjoint_traj, args.adjoint_steps,
                                        layout=args.adjoint_layout)), flush=True)
        return
    if args.workload == "headline":
        print(json.dumps(headline(args)), flush=True)
        return
    if args.workload == "large" and args.large_scatter > 0:
        print(json.dumps(large_scatter(args)), flush=True)
        return
    if args.workload == "large":
        print(json.dumps(large_workload(args)), flush=True)
        return
    if args.workload == "coupling":
        print(json.dumps(coupling_workload(args)), flush=True)
        return
    if args.workload == "rates":
        print(json.dumps(rates_workload(args)), flush=True)
        return
    if args.workload == "coupling_paper":
        print(json.dumps(coupling_paper_workload(args)), flush=True)
        return
    if args.workload == "paper_at":
        print(json.dumps(paper_at_workload(args)), flush=True)
        return
    if args.workload == "uneven":
        print(json.dumps(uneven_workload(args)), flush=True)
        return
    if args.workload == "at":
        print(json.dumps(at_workload(args)), flush=True)
        return
    line = window_workload(args)
    print(json.dumps(line), flush=True)


def window_variants(args, storages=None, gemv_steps=None):
    """The N = 969 mid-collision windows: --traj trajectories, --window RK4 steps of
    12 a.u. per bench step, per-trajectory and binned schedules, FP32 and FP64
    tables.  gemv_steps: fewer timed steps for the per-trajectory schedule."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import systems as S
    t0 = time.time()
    (s,), b = S.config2(n_traj=args.traj, full_collision=False, window_steps=args.window)
    log("generated N=%d K=%d B=%d in %.1fs" % (s.N, s.K, b.B, time.time() - t0))
    N, B, W = s.N, b.B, args.window
    ctx = mq.Context(0)
    dev = ctx.device
    results = {}
    P_of = {}
    if storages is None:
        storages = [args.only] if args.only else ["C64", "C128"]
    schedules = [args.schedule] if args.schedule != "both" else ["gemv", "binned"]
    for storage in storages:
        t0 = time.time()
        sid = ctx.load_system(s, storage=storage)
        torch.cuda.synchronize()
        log("loaded %s tables (%.1f GB) in %.1fs" % (storage, ctx.system_bytes(sid) / 1e9,
                                                     time.time() - t0))
        out = {"P": torch.empty(B * N, dtype=torch.float64, device=dev),
               "classical": torch.empty((B, 6), dtype=torch.float64, device=dev),
               "t_final": torch.empty(B, dtype=torch.float64, device=dev),
               "steps": torch.empty(B, dtype=torch.int64, device=dev),
               "rejects": torch.empty(B, dtype=torch.int64, device=dev),
               "status": torch.empty(B, dtype=torch.int32, device=dev),
               "norm_err": torch.empty(B, dtype=torch.float64, device=dev),
               "energy_err": torch.empty(B, dtype=torch.float64, device=dev),
               "angmom_err": torch.empty(B, dtype=torch.float64, device=dev)}
        sids = np.full(B, sid, np.int32)
        Ns = np.full(B, N, np.int64)
        es = 8 if storage == "C64" else 16
        for sched in schedules:
            n_timed = gemv_steps if (sched == "gemv" and gemv_steps) else args.steps

            def step():
                ctx.run(sids, Ns, init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0,
                        dt=b.dt, n_steps=b.n_steps, out=out, schedule=sched)

            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            stream = torch.cuda.current_stream(dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            ctx.set_profiling(True)
            wall0 = time.time()
            e0.record(stream)
            for _ in range(n_timed):
                step()
            e1.record(stream)
            torch.cuda.synchronize()
            wall = (time.time() - wall0) / n_timed
            kern_ms, kern_n, kern_bytes = ctx.profile_read(with_bytes=True)
            ctx.set_profiling(False)
            ms = e0.elapsed_time(e1) / n_timed
            evals = B * (4 * W + 1)              # RK4 stages + the final diagnostic evaluation
            alg_bytes = evals * 4.0 * N * N * es  # four spline slices of N x N per evaluation
            st = out["status"].cpu().numpy()
            r = {"value": B * W / (ms * 1e-3), "ms_per_step": ms, "wall_ms_per_step": wall * 1e3,
                 # the four spline slices every trajectory's evaluation needs, per second: a
                 # work rate (the binned schedule reads each occupied knot once per stage)
                 "coupling_work_GBps": alg_bytes / (ms * 1e-3) / 1e9,
                 "N2_traj_steps_per_s": B * W * N * N / (ms * 1e-3),
                 "status_nonzero": int(np.count_nonzero(st)),
                 "max_norm_err": float(out["norm_err"].abs().max().item())}
            if sched == "gemv":
                kms = kern_ms / kern_n
                gbps = alg_bytes / (kms * 1e-3) / 1e9
                # algorithmic bytes: the four spline slices of every evaluation.  Trajectories
                # in one interval share those slices through L2 and the last-level cache, so
                # this is a cache-assisted rate that can exceed what HBM delivers; the HBM
                # share is `traffic` (counters), when taken on the current source
                r["roofline"] = {"kernel": "rk4_gemv", "bound": "hbm", "achieved": gbps,
                                 "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                                 "cache_assisted": True, "bytes": "coupling slices per evaluation",
                                 "traffic": None, "alg_bytes_per_launch": alg_bytes,
                                 "launch_ms": kms, "launches_timed": kern_n}
            else:
                # one product launch per stage: 2 knots x 2 slices x (N x 2N) x (2N x 2) real
                # multiply-adds per trajectory = 32 N^2 flops per trajectory and stage
                kms = kern_ms / kern_n
                flops = 32.0 * N * N * B
                peak = MFMA_PEAK_TFLOPS[storage]
                tf = flops / (kms * 1e-3) / 1e12
                r["roofline"] = {"kernel": "bin_gemm", "bound": "mfma", "achieved": tf,
                                 "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
                                 "traffic": None, "alg_flops_per_launch": flops,
                                 "launch_ms": kms, "launches_timed": kern_n,
                                 # the occupied knots' slices, read once per stage
                                 "table_bytes_per_launch": kern_bytes / kern_n,
                                 "table_GBps": kern_bytes / (kern_ms * 1e-3) / 1e9}
            tr = MEASURED_TRAFFIC.get((storage, sched))
            if tr and tr["source_sha256_16"] == _source_hash(tr["source"]) and \
                    tr["window"] == W and tr["trajectories"] == B:
                r["roofline"]["traffic"] = tr["bytes"]
            results[(storage, sched)] = r
            P_of[(storage, sched)] = out["P"].reshape(B, N).cpu().numpy()
            log("%s %s: %.2f ms/step, %.3g traj-steps/s, dominant kernel %.3f ms x %d (%s %.3g %s, "
                "%.1f%% of peak)" % (storage, sched, ms, r["value"], kms, kern_n,
                                    r["roofline"]["kernel"], r["roofline"]["achieved"],
                                    r["roofline"]["unit"], 100 * r["roofline"]["frac"]))
        ctx.free_system(sid)

    out = {"variants": {"%s/%s" % k: v for k, v in results.items()}, "results": results,
           "P_of": P_of, "s": s, "b": b, "W": W}
    if ("C64", "binned") in P_of and ("C128", "binned") in P_of:
        out["fp32_vs_fp64_max_abs_dP"] = float(
            np.max(np.abs(P_of[("C64", "binned")] - P_of[("C128", "binned")])))
    ctx.close()
    return out


def window_workload(args):
    """The N = 969 window workload as its own line."""
    import numpy as np
    wv = window_variants(args)
    results, P_of, s, b, W = wv["results"], wv["P_of"], wv["s"], wv["b"], wv["W"]
    N, B = s.N, b.B
    storages = sorted({k[0] for k in results})

    def best(storage):
        cands = [(k, v) for k, v in results.items() if k[0] == storage]
        return max(cands, key=lambda kv: kv[1]["value"]) if cands else (None, None)

    hk, head = best("C64") if "C64" in storages else best("C128")
    line = {
        "metric": METRIC, "value": head["value"], "unit": "traj-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if hk[0] == "C64" else "f64", "data": "synthetic",
        "config": {"workload": "asymmetric top + atom, j<=8 all k,m (N=969), 200-point "
                               "Hermitian complex tables, %d trajectories mid-collision, "
                               "%d RK4 steps of 12 a.u. per bench step" % (B, W),
                   "N": N, "K": s.K, "trajectories": B, "rk4_steps_per_bench_step": W,
                   "schedule": hk[1], "tables": hk[0]},
        "roofline": head["roofline"],
        "coupling_work_GBps": head["coupling_work_GBps"],
        "N2_traj_steps_per_s": head["N2_traj_steps_per_s"],
        "status_nonzero": head["status_nonzero"],
        "variants": {"%s/%s" % k: {kk: vv for kk, vv in v.items()} for k, v in results.items()},
    }
    if ("C64", hk[1]) in P_of and ("C128", hk[1]) in P_of:
        line["fp32_vs_fp64_max_abs_dP"] = float(
            np.max(np.abs(P_of[("C64", hk[1])] - P_of[("C128", hk[1])])))
        f64 = max((v for k, v in results.items() if k[0] == "C128"), key=lambda v: v["value"])
        line["fp32_speedup_over_fp64"] = head["value"] / f64["value"]
    if ("C64", "gemv") in results and ("C64", "binned") in results:
        line["binned_speedup_over_gemv_fp32"] = (results[("C64", "binned")]["value"] /
                                                 results[("C64", "gemv")]["value"])
    if ("C128", "gemv") in results:
        line["plain_fp64_gemv_value"] = results[("C128", "gemv")]["value"]
        line["speedup_over_plain_fp64"] = head["value"] / results[("C128", "gemv")]["value"]

    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(s, b, W)
    if args.adjoint == "on":
        line["adjoint"] = adjoint_timing(args.adjoint_traj, args.adjoint_steps,
                                         layout=args.adjoint_layout)
    return line




def large_workload(args):
    """N = 4096 random Hermitian tables (54 GB as complex128 values, built on the
    GPU), 512 trajectories from 20 A in lockstep, full collisions of 10,000 RK4
    steps (dt = T/10^4) on the binned schedule, FP32 and FP64 tables.  The
    collision runs as consecutive windows of --large-window steps chained through
    the final amplitudes, classical state and time (one progress line each).
    Also: per-trajectory schedule vs binned on 8 trajectories x 200 steps (FP64)."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import systems as S
    N, B, T, W = args.large_n, args.large_traj, args.large_steps, args.large_window
    t0 = time.time()
    (s,), b = S.config5(n_traj=B, n_steps=T, N=N, build_tables=False)
    ctx = mq.Context(0)
    dev = ctx.device
    Md = S.gp_tables_device(s, dev)
    torch.cuda.synchronize()
    s.labels["gp"] = None
    log("large: N=%d tables built on the device in %.1fs" % (N, time.time() - t0))
    res, finals = {}, {}
    for storage in ([args.only] if args.only else ["C64", "C128"]):
        t1 = time.time()
        sid = ctx.load_system(R_grid=s.R_grid, E=s.E, M=Md, jx=None, mu=s.mu, storage=storage)
        torch.cuda.synchronize()
        log("large: loaded %s (%.1f GB) in %.1fs" % (storage, ctx.system_bytes(sid) / 1e9,
                                                     time.time() - t1))
        sids, Ns = np.full(B, sid, np.int32), np.full(B, N, np.int64)
        if args.large_integrator == "dp5":
            res[storage] = large_dp5(ctx, sid, sids, Ns, b, storage)
            finals[storage] = res[storage].pop("P")
            ctx.free_system(sid)
            continue
        dp5 = large_dp5(ctx, sid, sids, Ns, b, storage) if args.large_integrator == "both" \
            else None
        stream = torch.cuda.current_stream(dev)
        state = None
        ms_tot = 0.0
        kern_ms = kern_n = kern_bytes = 0
        n_win = T // W if args.large_windows <= 0 else min(T // W, args.large_windows)
        for w in range(n_win):
            kw = dict(dt=b.dt, n_steps=np.full(B, W), schedule="binned")
            if state is None:
                kw.update(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0)
            else:
                kw.update(a0=state[0], classical0=state[1], t0=state[2])
            ctx.set_profiling(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            out = ctx.run(sids, Ns, **kw)
            e1.record(stream)
            torch.cuda.synchronize()
            km, kn, kb = ctx.profile_read(with_bytes=True)
            ctx.set_profiling(False)
            kern_ms += km
            kern_n += kn
            kern_bytes += kb
            ms = e0.elapsed_time(e1)
            ms_tot += ms
            state = (out["a_final"].cpu().numpy().reshape(B, N), out["classical"].cpu().numpy(),
                     out["t_final"].cpu().numpy())
            R = state[1][:, 0]
            log("large %s: window %d/%d %.0f ms, R %.1f..%.1f bohr, max|norm-1| %.2e, "
                "bin_gemm %.3f ms x %d, %.1f knots, %.0f GB/s" % (
                    storage, w + 1, n_win, ms, R.min(), R.max(),
                    float(out["norm_err"].abs().max().item()), km / max(kn, 1), kn,
                    kb / max(kn, 1) / (2.0 * N * N * (8 if storage == "C64" else 16)),
                    kb / max(km * 1e-3, 1e-30) / 1e9))
        P = np.abs(state[0]) ** 2
        finals[storage] = P
        flops = 32.0 * N * N * B
        kms = kern_ms / max(kern_n, 1)
        tf = flops / (kms * 1e-3) / 1e12
        peak = MFMA_PEAK_TFLOPS[storage]
        gbps = kern_bytes / (kern_ms * 1e-3) / 1e9
        # mid-collision only a few trajectories share a knot, so the product reads
        # each occupied knot's slices for few columns: report the roof it is nearer
        mf = {"kernel": "bin_gemm", "bound": "mfma", "achieved": tf, "peak": peak,
              "unit": "TFLOP/s", "frac": tf / peak, "traffic": None,
              "alg_flops_per_launch": flops, "launch_ms": kms, "launches_timed": kern_n}
        hb = {"kernel": "bin_gemm", "bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS,
              "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS, "traffic": None,
              "alg_bytes_per_launch": kern_bytes / max(kern_n, 1), "launch_ms": kms,
              "launches_timed": kern_n}
        roof = dict(hb if hb["frac"] > mf["frac"] else mf)
        roof["other_roof"] = {k: (mf if roof["bound"] == "hbm" else hb)[k]
                              for k in ("bound", "achieved", "peak", "unit", "frac")}
        if dp5 is not None:
            Pd = dp5.pop("P")
            dp5["max_abs_dP_vs_rk4"] = float(np.max(np.abs(Pd - P)))
            log("large %s: DP5 vs RK4 (%d steps) max|dP| = %.3e" % (
                storage, T, dp5["max_abs_dP_vs_rk4"]))
        res[storage] = {
            "value": B * W * n_win / (ms_tot * 1e-3), "ms_per_window": ms_tot / n_win,
            "total_s": ms_tot * 1e-3, "windows": n_win,
            "N2_traj_steps_per_s": B * W * n_win * float(N) * N / (ms_tot * 1e-3),
            "roofline": roof,
            "max_norm_err": float(np.max(np.abs(P.sum(1) - 1.0)))}
        if dp5 is not None:
            res[storage]["dp5"] = dp5
        log("large %s: %.3g traj-steps/s, bin_gemm %.3f ms (%.1f TFLOP/s = %.1f%%; %.0f GB/s "
            "of tables = %.1f%%)" % (storage, res[storage]["value"], kms, tf, 100 * tf / peak,
                                     gbps, 100 * gbps / HBM_PEAK_GBPS))
        if storage == "C128":
            # per-trajectory schedule vs binned at full size: 8 trajectories x 200 steps
            sub = np.arange(8)
            kw = dict(init_channel=b.init_channel[sub], E_coll=b.E_coll[sub], b=b.b[sub],
                      R0=b.R0[sub], dt=b.dt[sub], n_steps=np.full(8, 200))
            g1 = ctx.run_host(np.full(8, sid, np.int32), np.full(8, N), schedule="gemv", **kw)
            g2 = ctx.run_host(np.full(8, sid, np.int32), np.full(8, N), schedule="binned", **kw)
            res[storage]["gemv_vs_binned_max_abs_dP_8x200"] = float(np.max(np.abs(g1["P"] - g2["P"])))
            log("large: gemv vs binned (8 x 200 steps) max|dP| = %.3e"
                % res[storage]["gemv_vs_binned_max_abs_dP_8x200"])
        ctx.free_system(sid)
    del Md
    ctx.close()
    head = res.get("C64") or res["C128"]
    if args.large_integrator == "dp5":
        line = {"metric": METRIC, "value": head["value"], "unit": "traj-steps/s", "n_gpus": 1,
                "steps": 1, "warmup": 0, "ms_per_step": head["total_s"] * 1e3,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f32" if "C64" in res else "f64", "data": "synthetic",
                "config": {"workload": "N=%d random Hermitian tables on 200 R points, %d full "
                                       "collisions from 20 A, adaptive DP5 (rtol = atol = 1e-8) "
                                       "on the binned schedule, one call" % (N, B),
                           "N": N, "trajectories": B, "tables": list(res)},
                "roofline": head["roofline"], "variants": res}
        if "C64" in finals and "C128" in finals:
            d = np.abs(finals["C64"] - finals["C128"])
            line["fp32_vs_fp64_dP"] = {"max": float(d.max()), "mean": float(d.mean())}
        return line
    line = {"metric": METRIC, "value": head["value"], "unit": "traj-steps/s", "n_gpus": 1,
            "steps": head["windows"], "warmup": 0, "ms_per_step": head["ms_per_window"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if "C64" in res else "f64", "data": "synthetic",
            "config": {"workload": "N=%d random Hermitian tables on 200 R points, %d full "
                                   "collisions of %d RK4 steps from 20 A, binned schedule, "
                                   "one bench step = %d steps" % (N, B, T, W),
                       "N": N, "trajectories": B, "rk4_steps": T, "tables": list(res)},
            "roofline": head["roofline"], "variants": res}
    if "C64" in finals and "C128" in finals:
        d = np.abs(finals["C64"] - finals["C128"])
        line["fp32_vs_fp64_dP"] = {"max": float(d.max()), "mean": float(d.mean()),
                                   "p99": float(np.percentile(d, 99))}
        line["fp32_speedup_over_fp64"] = res["C64"]["value"] / res["C128"]["value"]
    return line


def system_info():
    """GPU, ROCm and host CPU of the run."""
    import torch
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count()
    return {"gpu": torch.cuda.get_device_name(0), "rocm_hip": torch.version.hip,
            "torch": torch.__version__, "host_cpu": cpu, "host_threads_visible": os.cpu_count(),
            "host_threads_affinity": affinity}


def collision_windows(ctx, sids, Ns, b, n_windows, warmup, total_steps, storage):
    """The N = 4096 collision as n_windows consecutive calls of total_steps / n_windows
    RK4 steps (each continues the stored state of the one before, resume = 1), after
    `warmup` windows of the same collision from its start.  Returns the timed run's
    per-window kernel records and its final probabilities."""
    import numpy as np
    import torch
    B, N = len(sids), int(Ns[0])
    spw = -(-total_steps // n_windows)
    start = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt)
    sizes = [min(spw, total_steps - w * spw) for w in range(n_windows)]
    for w in range(warmup):
        ctx.run(sids, Ns, n_steps=np.full(B, spw), schedule="binned",
                **(start if w == 0 else {}), resume=w > 0)
        torch.cuda.synchronize()
        log("  warm-up window %d of %d done" % (w + 1, warmup))
    stream = torch.cuda.current_stream(ctx.device)
    rec = []
    ctx.set_profiling(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.time()
    e0.record(stream)
    for w, n in enumerate(sizes):
        out = ctx.run(sids, Ns, n_steps=np.full(B, n), schedule="binned",
                      **(start if w == 0 else {}), resume=w > 0)
        km, kn, kb = ctx.profile_read(with_bytes=True)   # waits for the window
        rec.append({"steps": n, "kernel_ms": km, "launches": kn, "table_bytes": kb})
        log("  window %d of %d done at %.1f s" % (w + 1, len(sizes), time.time() - wall0))
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    ctx.set_profiling(False)
    ms = e0.elapsed_time(e1)
    st = out["status"].cpu().numpy()
    P = out["P"].reshape(B, N).cpu().numpy()
    R = out["classical"][:, 0].cpu().numpy()
    for w, r in enumerate(rec):
        flops = 32.0 * N * N * B * r["launches"]
        peak = MFMA_PEAK_TFLOPS[storage] * 1e12
        ideal = max(r["table_bytes"] / (HBM_PEAK_GBPS * 1e9), flops / peak)
        r["knots_per_launch"] = r["table_bytes"] / max(r["launches"], 1) / (
            2.0 * N * N * (8 if storage == "C64" else 16))
        r["GBps"] = r["table_bytes"] / (r["kernel_ms"] * 1e-3) / 1e9
        r["TFLOPs"] = flops / (r["kernel_ms"] * 1e-3) / 1e12
        r["roofline_ms"] = ideal * 1e3
        log("  %s window %2d: %4d steps, bin_gemm %.3f ms x %d, %.1f knots, %5.0f GB/s, "
            "%5.1f TFLOP/s, %.0f%% of its roofline" % (
                storage, w + 1, r["steps"], r["kernel_ms"] / max(r["launches"], 1), r["launches"],
                r["knots_per_launch"], r["GBps"], r["TFLOPs"],
                100 * r["roofline_ms"] / r["kernel_ms"]))
    return {"ms": ms, "wall_s": wall, "windows": rec, "P": P, "status": st,
            "norm_err_max": float(out["norm_err"].abs().max().item()), "R_final": R}


def headline(args):
    """The N = 4096 collision (the largest configuration) as the headline, with
    the other workloads as variants of the same line."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import systems as S
    t_all = time.time()
    info = system_info()
    log("system %s" % json.dumps(info))
    N, B, T = args.large_n, args.large_traj, args.large_steps
    K_win, W = args.steps, args.warmup
    t0 = time.time()
    (s, ), b = S.config5(n_traj=B, n_steps=T, N=N, build_tables=False)
    ctx = mq.Context(0)
    probe = read_bandwidth_probe(ctx=ctx)["read_bandwidth_probe"]
    Md = S.gp_tables_device(s, ctx.device)
    torch.cuda.synchronize()
    log("large: N=%d tables built on the device in %.1fs" % (N, time.time() - t0))
    sids, Ns = np.full(B, 0, np.int32), np.full(B, N, np.int64)
    variants = {}
    finals = {}
    # the headline: FP32 tables, the whole collision of T RK4 steps in K_win windows
    sid = ctx.load_system(R_grid=s.R_grid, E=s.E, M=Md, jx=None, mu=s.mu, storage="C64")
    sids[:] = sid
    cw = collision_windows(ctx, sids, Ns, b, K_win, W, T, "C64")
    rec = cw["windows"]
    kms = sum(r["kernel_ms"] for r in rec)
    kn = sum(r["launches"] for r in rec)
    kb = sum(r["table_bytes"] for r in rec)
    flops = 32.0 * N * N * B * kn
    roof_ms = sum(r["roofline_ms"] for r in rec)
    gbps = kb / (kms * 1e-3) / 1e9
    tf = flops / (kms * 1e-3) / 1e12
    hbm_time, mfma_time = kb / (HBM_PEAK_GBPS * 1e9), flops / (MFMA_PEAK_TFLOPS["C64"] * 1e12)
    head = {"value": B * T / (cw["ms"] * 1e-3), "ms_per_step": cw["ms"] / K_win,
            "total_s": cw["ms"] * 1e-3, "wall_s": cw["wall_s"],
            "N2_traj_steps_per_s": B * T * float(N) * N / (cw["ms"] * 1e-3),
            "status_nonzero": int(np.count_nonzero(cw["status"])),
            "max_norm_err": cw["norm_err_max"]}
    # the product moves between the two roofs during the collision: the bound is the
    # one its ideal time spends longer under, and the mixed fraction compares the
    # ideal time of every window (the larger of its bytes at 8 TB/s and its flops at
    # the matrix peak) with the measured time
    if hbm_time >= mfma_time:
        roof = {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": gbps / HBM_PEAK_GBPS}
        other = {"bound": "mfma", "achieved": tf, "peak": MFMA_PEAK_TFLOPS["C64"],
                 "unit": "TFLOP/s", "frac": tf / MFMA_PEAK_TFLOPS["C64"]}
    else:
        roof = {"bound": "mfma", "achieved": tf, "peak": MFMA_PEAK_TFLOPS["C64"],
                "unit": "TFLOP/s", "frac": tf / MFMA_PEAK_TFLOPS["C64"]}
        other = {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                 "frac": gbps / HBM_PEAK_GBPS}
    roof.update({"kernel": "bin_gemm", "traffic": None,
                 "alg_bytes_per_launch": kb / kn, "alg_flops_per_launch": flops / kn,
                 "launch_ms": kms / kn, "launches_timed": kn,
                 "mixed_frac": roof_ms / kms, "other_roof": other})
    tr = MEASURED_TRAFFIC.get(("C64", "large"))
    if tr and tr["source_sha256_16"] == _source_hash(tr["source"]) and tr["trajectories"] == B:
        roof["traffic"] = tr["bytes"]
    # against the streaming-read rate this GPU reaches with 1 KiB wave loads (2 GB buffer)
    roof["measured_read_peak_GBps"] = probe["2GB"]["GBps"]
    roof["frac_of_measured_read_peak"] = gbps / probe["2GB"]["GBps"]
    head["roofline"] = roof
    head["windows"] = [{k: v for k, v in r.items()} for r in rec]
    finals["C64/rk4"] = cw["P"]
    log("large C64: %.1f s for the collision, %.3g traj-steps/s, bin_gemm %.3f ms x %d: "
        "%.0f GB/s (%.1f%% of HBM), %.1f TFLOP/s (%.1f%%), %.1f%% of the mixed roofline" % (
            head["total_s"], head["value"], kms / kn, kn, gbps, 100 * gbps / HBM_PEAK_GBPS, tf,
            100 * tf / MFMA_PEAK_TFLOPS["C64"], 100 * roof_ms / kms))
    variants["large/C64/binned/rk4"] = {k: v for k, v in head.items() if k != "windows"}
    if not args.headline_only:
        # the same collisions with adaptive steps, FP32 and FP64 tables
        d = large_dp5(ctx, sid, sids, Ns, b, "C64")
        finals["C64/dp5"] = d.pop("P")
        variants["large/C64/binned/dp5"] = d
        ctx.free_system(sid)
        sid = ctx.load_system(R_grid=s.R_grid, E=s.E, M=Md, jx=None, mu=s.mu, storage="C128")
        sids[:] = sid
        d = large_dp5(ctx, sid, sids, Ns, b, "C128")
        finals["C128/dp5"] = d.pop("P")
        variants["large/C128/binned/dp5"] = d
    ctx.free_system(sid)
    del Md
    ctx.close()
    torch.cuda.empty_cache()
    line = {"metric": METRIC, "value": head["value"], "unit": "traj-steps/s", "n_gpus": 1,
            "steps": K_win, "warmup": W, "ms_per_step": head["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "N=%d random Hermitian channels on 200 R points (53.7 GB of "
                                   "FP32 tables), %d trajectories from 20 A, the whole collision "
                                   "of %d RK4 steps of T/%d on the binned schedule; one bench "
                                   "step = %d steps (the %d timed steps cover the collision)"
                                   % (N, B, T, T, -(-T // K_win), K_win),
                       "N": N, "K": s.K, "trajectories": B, "rk4_steps": T,
                       "schedule": "binned", "tables": "C64"},
            "roofline": head["roofline"],
            "N2_traj_steps_per_s": head["N2_traj_steps_per_s"],
            "status_nonzero": head["status_nonzero"], "system": info,
            "read_bandwidth_probe": probe, "windows": head["windows"]}
    if "C128/dp5" in finals:
        dd = np.abs(finals["C64/dp5"] - finals["C128/dp5"])
        line["fp32_vs_fp64_dP"] = {"max": float(dd.max()), "mean": float(dd.mean()),
                                   "p99": float(np.percentile(dd, 99)),
                                   "runs": "whole collision, adaptive DP5 rtol=atol=1e-8, "
                                           "FP32 vs FP64 tables"}
        line["dp5_vs_rk4_fp32_max_dP"] = float(np.max(np.abs(finals["C64/dp5"] -
                                                           finals["C64/rk4"])))
        line["fp32_speedup_over_fp64_dp5"] = (variants["large/C64/binned/dp5"]["value"] /
                                              variants["large/C128/binned/dp5"]["value"])
        log("large: FP32 vs FP64 (DP5) max|dP| %.2e, DP5 vs RK4 (FP32) max|dP| %.2e" % (
            line["fp32_vs_fp64_dP"]["max"], line["dp5_vs_rk4_fp32_max_dP"]))
    if not args.headline_only:
        # the N = 969 mid-collision windows (FP32 and FP64 tables, binned and per trajectory)
        wa = argparse.Namespace(**vars(args))
        wa.steps, wa.warmup, wa.only, wa.schedule = 10, 2, None, "both"
        win = window_variants(wa, storages=["C64", "C128"], gemv_steps=2)
        for k, v in win["variants"].items():
            variants["window/" + k] = v
        line["window_fp32_vs_fp64_max_abs_dP"] = win.get("fp32_vs_fp64_max_abs_dP")
        # the uneven batch, one call
        un = uneven_workload(argparse.Namespace(**dict(vars(args), no_cpu=True)))
        variants["uneven"] = {k: un[k] for k in ("value", "ms_per_step", "config", "per_system",
                                                 "N2_traj_steps_per_s")}
        # the adjoint
        line["adjoint"] = adjoint_timing(args.adjoint_traj, args.adjoint_steps,
                                         layout=args.adjoint_layout)
        # AT dynamics at the paper's size: one path x 100 initial states on the
        # screened 206,350-state matrices, FP32 tables, the whole collision
        pa = paper_at_workload(argparse.Namespace(**dict(vars(args), only_paper="R32",
                                                          paper_steps=0)))
        variants["paper_at/R32/columns"] = dict(pa["variants"]["R32"], config=pa["config"])
    line["variants"] = variants
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_large(s, b)
    log("headline run %.0f s in all" % (time.time() - t_all))
    return line


def cpu_baseline_large(s, b, target_s=15.0):
    """The FP64 oracle on the headline workload: the first trajectories of the batch
    (one per host thread the oracle uses, OpenMP over trajectories) over the first
    steps of their collision (about target_s of propagation), on the knots those
    steps touch; then one trajectory on one thread."""
    import numpy as np
    import oracle
    from synth import systems as S
    t0 = time.time()
    phi, v, H, scale = S.gp_rank_factors(s)
    ks = np.arange(s.K - 6, s.K)
    o = oracle.OracleSystem(s, knots=oracle.rank_q_knot_tables(s.R_grid, phi, v, H, ks, scale))
    log("oracle: %d knots of the N=%d tables in %.1fs" % (len(ks), s.N, time.time() - t0))
    th = oracle.threads()

    def timed(n_traj):
        sub = b.subset(range(n_traj))
        sub.n_steps[:] = 1
        t0 = time.time()
        o.propagate(sub)
        t1 = time.time() - t0
        n = int(max(1, min(40, round(target_s / max(t1, 1e-3)))))
        sub.n_steps[:] = n
        t0 = time.time()
        r = o.propagate(sub)
        dt = time.time() - t0
        assert np.all(r["classical"][:, 0] > s.R_grid[ks[0]])
        log("oracle: %d trajectories x %d steps in %.1fs" % (n_traj, n, dt))
        return n_traj * n / dt, n

    n_all = min(th, b.B)
    v_all, n1 = timed(n_all)
    v_one, n2 = timed(1)
    return {"value": v_all, "unit": "traj-steps/s", "cores": n_all, "kind": "oracle",
            "single_thread_value": v_one,
            "sample": "the first %d of the %d trajectories x the first %d of the %d RK4 steps "
                      "on %d threads (OpenMP over trajectories), and the first trajectory x %d "
                      "steps on one thread (FP64 oracle, N=%d complex tables held at the %d knots "
                      "those steps touch); wall time of the propagation only" % (
                          n_all, b.B, n1, int(b.n_steps[0]), n_all, n2, s.N, len(ks))}


def large_scatter(args):
    """bin_gemm on the N = 4096 tables where it streams: 512 trajectories spread over
    the interaction region (R0 uniform in 4-19.5 A, b uniform below min(12 A, 0.9 R0),
    E_coll 1000 cm^-1), windows of --large-scatter RK4 steps of 10.1 a.u."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import systems as S, units as U
    N, B, W = args.large_n, args.large_traj, args.large_scatter
    t0 = time.time()
    (s,), b = S.config5(n_traj=B, n_steps=10000, N=N, build_tables=False)
    rng = np.random.default_rng(231202322 + 55)
    R0 = U.ang_to_bohr(rng.uniform(args.scatter_rmin, 19.5, B))
    bb = np.minimum(b.b, 0.9 * R0)
    ctx = mq.Context(0)
    dev = ctx.device
    Md = S.gp_tables_device(s, dev)
    torch.cuda.synchronize()
    log("large scatter: N=%d tables built in %.1fs" % (N, time.time() - t0))
    res = {}
    for storage in ([args.only] if args.only else ["C64", "C128"]):
        sid = ctx.load_system(R_grid=s.R_grid, E=s.E, M=Md, jx=None, mu=s.mu, storage=storage)
        sids, Ns = np.full(B, sid, np.int32), np.full(B, N, np.int64)
        kw = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=bb, R0=R0, dt=b.dt,
                  n_steps=np.full(B, W), schedule="binned")
        for _ in range(args.warmup):
            ctx.run(sids, Ns, **kw)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.set_profiling(True)
        e0.record(stream)
        for _ in range(args.steps):
            ctx.run(sids, Ns, **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        km, kn, kb = ctx.profile_read(with_bytes=True)
        ctx.set_profiling(False)
        ms = e0.elapsed_time(e1) / args.steps
        kms = km / kn
        gbps = kb / (km * 1e-3) / 1e9
        tf = 32.0 * N * N * B / (kms * 1e-3) / 1e12
        res[storage] = {"value": B * W / (ms * 1e-3), "ms_per_step": ms, "launch_ms": kms,
                        "launches": kn, "table_bytes_per_launch": kb / kn,
                        "occupied_knots_per_launch": kb / kn / (2.0 * N * N * (8 if storage == "C64" else 16)),
                        "table_GBps": gbps, "hbm_frac": gbps / HBM_PEAK_GBPS, "TFLOPs": tf}
        log("large scatter %s: %.2f ms per window of %d steps, bin_gemm %.3f ms x %d, %.1f knots, "
            "%.0f GB/s (%.1f%% of HBM), %.1f TFLOP/s" % (
                storage, ms, W, kms, kn, res[storage]["occupied_knots_per_launch"], gbps,
                100 * gbps / HBM_PEAK_GBPS, tf))
        ctx.free_system(sid)
    del Md
    ctx.close()
    return {"workload": "N=%d scattered window" % N, "variants": res}


def large_dp5(ctx, sid, sids, Ns, b, storage, rtol=1e-8):
    """The large workload's collisions in one adaptive DP5 call on the binned schedule."""
    import numpy as np
    import torch
    N, B = int(Ns[0]), len(sids)
    dev = ctx.device
    stream = torch.cuda.current_stream(dev)
    ctx.set_profiling(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    out = ctx.run(sids, Ns, init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0,
                  integrator="dp5", rtol=rtol, atol=rtol, max_steps=100000, h_min=1e-6,
                  schedule="binned")
    e1.record(stream)
    torch.cuda.synchronize()
    km, kn, kb = ctx.profile_read(with_bytes=True)
    ctx.set_profiling(False)
    ms = e0.elapsed_time(e1)
    steps = out["steps"].cpu().numpy()
    rej = out["rejects"].cpu().numpy()
    status = out["status"].cpu().numpy()
    kms = km / max(kn, 1)
    gbps = kb / (km * 1e-3) / 1e9
    roof = {"kernel": "bin_gemm", "bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS, "traffic": None,
            "alg_bytes_per_launch": kb / max(kn, 1), "launch_ms": kms, "launches_timed": kn}
    r = {"value": float(steps.sum()) / (ms * 1e-3), "total_s": ms * 1e-3,
         "collisions_per_s": B / (ms * 1e-3),
         "steps_p0_p50_p100": [int(v) for v in np.percentile(steps, [0, 50, 100])],
         "rejects": int(rej.sum()), "exited": int(np.count_nonzero(status & 1)),
         "max_norm_err": float(out["norm_err"].abs().max().item()), "roofline": roof,
         "P": out["P"].cpu().numpy().reshape(B, N)}
    log("large %s dp5: %.1f s for %d collisions, steps p0/p50/p100 %s, %d rejects, %d exited, "
        "bin_gemm %.3f ms x %d (%.0f GB/s of tables)" % (
            storage, r["total_s"], B, r["steps_p0_p50_p100"], r["rejects"], r["exited"], kms, kn,
            gbps))
    return r


def at_workload(args, n_paths=64, n_init=100):
    """Decoupled (AT) dynamics on the N = 969 asymmetric-top system: 64
    trajectories in the mid-collision population of the default workload, each
    carrying the 100 lowest channels as initial states (6400 amplitude columns),
    driven by the isotropic part of the coupling; one bench step = a window of
    RK4 steps of 12 a.u. on the binned schedule, FP32 and FP64 tables."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import systems as S
    W = args.window
    (s,), b0 = S.config2(n_traj=n_paths, full_collision=False, window_steps=W)
    N = s.N
    U = np.real(np.einsum("knn->k", s.M)) / N
    idx = np.repeat(np.arange(n_paths), n_init)
    b = b0.subset(idx)
    b.init_channel = np.tile(np.arange(n_init, dtype=np.int32), n_paths)
    B = b.B
    ctx = mq.Context(0)
    dev = ctx.device
    res = {}
    P_of = {}
    for storage in ([args.only] if args.only else ["C64", "C128"]):
        sid = ctx.load_system(s, storage=storage)
        ctx.set_driver(sid, U)
        sids, Ns = np.full(B, sid, np.int32), np.full(B, N, np.int64)
        kw = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt,
                  n_steps=b.n_steps, schedule="binned", dynamics="at")
        for _ in range(args.warmup):
            out = ctx.run(sids, Ns, **kw)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.set_profiling(True)
        e0.record(stream)
        for _ in range(args.steps):
            out = ctx.run(sids, Ns, **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        km, kn, kb = ctx.profile_read(with_bytes=True)
        ctx.set_profiling(False)
        ms = e0.elapsed_time(e1) / args.steps
        kms = km / kn
        flops = 32.0 * N * N * B
        peak = MFMA_PEAK_TFLOPS[storage]
        tf = flops / (kms * 1e-3) / 1e12
        P_of[storage] = out["P"].reshape(B, N).cpu().numpy()
        cl = out["classical"].reshape(n_paths, n_init, 6)
        res[storage] = {
            "value": B * W / (ms * 1e-3), "ms_per_step": ms,
            "paths_shared_bitwise": bool(torch.all(cl == cl[:, :1, :]).item()),
            "roofline": {"kernel": "bin_gemm", "bound": "mfma", "achieved": tf, "peak": peak,
                         "unit": "TFLOP/s", "frac": tf / peak, "traffic": None,
                         "alg_flops_per_launch": flops, "launch_ms": kms, "launches_timed": kn,
                         "table_bytes_per_launch": kb / kn}}
        log("at %s: %.2f ms/step, %.3g column-steps/s, bin_gemm %.3f ms (%.1f TFLOP/s, %.1f%%)"
            % (storage, ms, res[storage]["value"], kms, tf, 100 * tf / peak))
        ctx.free_system(sid)
    ctx.close()
    head = res.get("C64") or res["C128"]
    line = {"metric": METRIC, "value": head["value"], "unit": "traj-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if "C64" in res else "f64", "data": "synthetic",
            "config": {"workload": "AT dynamics, N=969 asymmetric top + atom, %d mid-collision "
                                   "paths x %d initial states (%d amplitude columns), %d RK4 "
                                   "steps of 12 a.u. per bench step, binned schedule"
                                   % (n_paths, n_init, B, W),
                       "N": N, "paths": n_paths, "initial_states": n_init},
            "roofline": head["roofline"], "variants": res}
    if "C64" in P_of and "C128" in P_of:
        line["fp32_vs_fp64_max_abs_dP"] = float(np.max(np.abs(P_of["C64"] - P_of["C128"])))
    return line


def coupling_workload(args, cpu_rows=256):
    """Coupling-matrix build (Section II, Eqs. 12-18): asymmetric top (H2O constants,
    j1 <= 6, every tau1) + para-H2 (j2 = 0, 2, 4), all j and m: N = 6825 channels;
    83 expansion terms from the ranges of the paper's potential; 63 knots from 3 to
    30 bohr.  One step = one complete build of the FP64 tables [63][N][N] (23.5 GB)
    from the expansion coefficients.  The unit counts the elements between channels
    of equal m (the ones the potential couples), times the knots."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import coupling as CP
    basis, ex = CP.config6()
    N, T, K = basis.N, ex.T, ex.K
    counts = np.bincount(basis.m - basis.m.min()).astype(np.float64)
    elements = float(np.sum(counts ** 2)) * K
    ctx = mq.Context(0)
    for _ in range(args.warmup):
        out = ctx.build_couplings(basis, ex)
        del out
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.time()
    for _ in range(args.steps):
        out = ctx.build_couplings(basis, ex)
        del out
    torch.cuda.synchronize()
    sec = (time.time() - t0) / args.steps
    km, kn, kb = ctx.profile_read(with_bytes=True)
    ctx.set_profiling(False)
    ctx.close()
    kms = km / kn
    written = kb / kn
    gbps = written / (kms * 1e-3) / 1e9
    log("coupling: N=%d T=%d K=%d, %.1f ms per build, zero + fill kernels %.2f ms (%.0f GB/s written, "
        "%.1f%% of HBM)" % (N, T, K, sec * 1e3, kms, gbps, 100 * gbps / HBM_PEAK_GBPS))
    line = {"metric": "coupling-matrix elements/s (equal-m pairs x knots)",
            "value": elements / sec, "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "coupling-matrix build, asymmetric top (j1<=6) + para-H2 "
                                   "(j2<=4), N=%d channels, %d expansion terms, %d knots, FP64 "
                                   "tables [K][N][N]" % (N, T, K),
                       "N": N, "terms": T, "knots": K},
            "roofline": {"kernel": "cpl_zero + cpl_fill", "bound": "hbm", "achieved": gbps,
                         "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                         "traffic": None, "alg_bytes_per_launch": written, "launch_ms": kms,
                         "launches_timed": kn}}
    if not args.no_cpu:
        import oracle
        rows = np.linspace(0, N - 1, cpu_rows).astype(np.int64)
        t0 = time.time()
        oracle.coupling_tables(basis, ex, rows=rows)
        csec = time.time() - t0
        cel = float(np.sum(counts[basis.m[rows] - basis.m.min()])) * K
        line["cpu_baseline"] = {"value": cel / csec, "unit": "elements/s",
                                "cores": oracle.threads(), "kind": "oracle",
                                "sample": "%d of the %d rows (Eq. 17 sums), %.1f s"
                                          % (cpu_rows, N, csec)}
        log("coupling: oracle %.3g elements/s on %d rows (%.1f s, %d threads)"
            % (cel / csec, cpu_rows, csec, oracle.threads()))
    return line


def paper_at_workload(args, n_init=100, U_cm=300.0, b_bohr=2.0, R0_bohr=20.0, dt=10.0):
    """AT-MQCT at the paper's size (Section III): the p-H2O (j1 <= 28) + p-H2 (j2 <= 10)
    basis below 8000 cm^-1 (206,350 states), its screened coupling matrices (elements
    above the threshold at 6.03 or 7.11 bohr, the kept ones on 63 knots from 3 to 30
    bohr) as a coordinate list; one classical path driven by the isotropic term,
    carrying the 100 lowest states as initial states (the paper's 100 initial states
    of water per trajectory); RK4 steps of 10 a.u. (the paper's smallest step) over
    the whole collision from 20 bohr.  FP32 and FP64 tables."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import coupling as CP
    from synth import systems as S
    t0 = time.time()
    basis = CP.para_h2o_para_h2_basis()
    terms = CP.select_terms(CP.expansion_terms(), 83, seed=0)
    Rg = CP.log_grid(63)
    ex = CP.synthetic_expansion(terms, Rg, seed=0)
    vs = CP.synthetic_expansion(terms, np.array(CP.PAPER_SCREEN_R), seed=0).v
    thr = CP.U.cm_to_hartree(CP.PAPER_SCALE_DROP_CM)
    ctx = mq.Context(0)
    out = ctx.build_couplings_sparse(basis, ex, vs, thr)
    nnz = out["n_kept"]
    log("paper_at: N=%d, %d kept elements (built in %.1f s with the basis)" % (
        basis.N, nnz, time.time() - t0))
    iso = [t for t, tm in enumerate(terms) if tuple(tm) == (0, 0, 0, 0)][0]
    Udrv = ex.v[iso] / (2.0 * np.pi)       # the isotropic term is v / (2 pi) times the identity
    mu = CP.U.amu_to_me(1.8)
    E = CP.U.cm_to_hartree(U_cm)
    init = np.argsort(basis.E, kind="stable")[:n_init].astype(np.int32)
    n_steps = int(np.ceil(S.collision_time(R0_bohr, E, mu) / dt))
    if args.paper_steps > 0:
        n_steps = min(n_steps, args.paper_steps)
    B = n_init
    kw = dict(init_channel=init, E_coll=np.full(B, E), b=np.full(B, b_bohr),
              R0=np.full(B, R0_bohr), dt=np.full(B, dt), schedule="columns", dynamics="at")
    res = {}
    for storage in ([args.only_paper] if getattr(args, "only_paper", None) else ["R32", "R64"]):
        t1 = time.time()
        sid = ctx.load_system_coo(R_grid=Rg, E=basis.E, rows=out["rows"], cols=out["cols"],
                                  values=out["values"], mu=mu,
                                  jx=(basis.jx_row, basis.jx_col, basis.jx_val), storage=storage)
        ctx.set_driver(sid, Udrv)
        torch.cuda.synchronize()
        load_s = time.time() - t1
        sids, Ns = np.full(B, sid, np.int32), np.full(B, basis.N, np.int64)
        ctx.run(sids, Ns, n_steps=np.full(B, 4), **kw)           # warm-up
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(ctx.device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g = ctx.run(sids, Ns, n_steps=np.full(B, n_steps), **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        es = 4 if storage == "R32" else 8
        stage_ms = ms / (4.0 * n_steps)
        # per stage: the interval's four slices of every kept element, and the
        # amplitude passes (a0, accumulator, stage input for J_x read; accumulator,
        # next stage input written: complex FP64) plus the phased operand written
        tab = 4.0 * nnz * es
        amp = float(basis.N) * B * (16 * 5 + 2 * es)
        gather = float(nnz) * B * 2 * es
        P = g["P"].reshape(B, basis.N)
        moved = 1.0 - P[torch.arange(B), torch.as_tensor(init, device=P.device).long()]
        r = {"seconds": ms * 1e-3, "rk4_steps": n_steps, "columns": B,
             "column_steps_per_s": B * n_steps / (ms * 1e-3), "stage_ms": stage_ms,
             "load_s": load_s, "table_bytes": ctx.system_bytes(sid),
             "hbm_bytes_per_stage": tab + amp, "hbm_GBps": (tab + amp) / (stage_ms * 1e-3) / 1e9,
             "gather_bytes_per_stage": gather,
             "gather_GBps": gather / (stage_ms * 1e-3) / 1e9,
             "max_norm_err": float(g["norm_err"].abs().max().item()),
             "energy_err": float(g["energy_err"].abs().max().item()),
             "status": int(g["status"].max().item()),
             "R_final": float(g["classical"][0, 0].item()),
             "population_moved_p50_max": [float(moved.median().item()), float(moved.max().item())]}
        log("paper_at %s: %.2f s for %d columns x %d RK4 steps (%.3g column-steps/s), %.3f ms per "
            "stage; HBM %.0f GB/s, gathers %.0f GB/s; max|norm-1| %.2e; moved p50/max %.2e/%.2e" % (
                storage, r["seconds"], B, n_steps, r["column_steps_per_s"], stage_ms, r["hbm_GBps"],
                r["gather_GBps"], r["max_norm_err"], *r["population_moved_p50_max"]))
        res[storage] = r
        if storage == "R32":
            P32 = P.cpu().numpy()
        else:
            res["fp32_vs_fp64_max_abs_dP"] = float(np.max(np.abs(P32 - P.cpu().numpy()))) \
                if "R32" in res else None
        del g, P
        ctx.free_system(sid)
    ctx.close()
    line = {"metric": "column-steps/s (AT, paper-size truncated tables)",
            "value": res[list(res)[0]]["column_steps_per_s"], "unit": "column-steps/s",
            "n_gpus": 1, "steps": n_steps, "warmup": 1,
            "ms_per_step": res[list(res)[0]]["stage_ms"] * 4, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "AT-MQCT, p-H2O + p-H2 below 8000 cm^-1 (N=%d), %d screened "
                                   "couplings on 63 knots, one path (E=%.0f cm^-1, b=%.1f bohr, "
                                   "from %.0f bohr) x %d initial states, %d RK4 steps of %.0f a.u."
                                   % (basis.N, nnz, U_cm, b_bohr, R0_bohr, B, n_steps, dt),
                       "N": basis.N, "kept": nnz, "columns": B},
            "variants": res}
    return line


def coupling_paper_workload(args, cpu_pairs=12):
    """Screened coupling build at the paper's size (Section III): para-H2O (j1 <= 28)
    + para-H2 (j2 <= 10) below 8000 cm^-1, all j and m: 206,350 states, 1.2e9
    elements of equal m; 83 expansion terms; every element evaluated at R = 6.03 and
    7.11 bohr and kept above the threshold, the kept ones computed at 63 knots from
    3 to 30 bohr.  One step = one complete screened build."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import coupling as CP
    basis = CP.para_h2o_para_h2_basis()
    terms = CP.select_terms(CP.expansion_terms(), 83, seed=0)
    ex = CP.synthetic_expansion(terms, CP.log_grid(63), seed=0)
    vs = CP.synthetic_expansion(terms, np.array(CP.PAPER_SCREEN_R), seed=0).v
    thr = CP.U.cm_to_hartree(CP.PAPER_SCALE_DROP_CM)
    counts = np.bincount(basis.m - basis.m.min()).astype(np.float64)
    screened = float(np.sum(counts ** 2))
    ctx = mq.Context(0)
    out = ctx.build_couplings_sparse(basis, ex, vs, thr)        # counts, then builds
    n_kept = out["n_kept"]
    cap = n_kept
    del out
    for _ in range(args.warmup):
        o = ctx.build_couplings_sparse(basis, ex, vs, thr, capacity=cap)
        del o
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        o = ctx.build_couplings_sparse(basis, ex, vs, thr, capacity=cap)
        del o
    torch.cuda.synchronize()
    sec = (time.time() - t0) / args.steps
    ctx.close()
    log("coupling_paper: N=%d, %.3g equal-m elements screened, %d kept (> %.3g cm^-1), "
        "%.3f s per build" % (basis.N, screened, n_kept, CP.PAPER_SCALE_DROP_CM, sec))
    line = {"metric": "equal-m coupling elements screened/s (Eq. 17 at two distances, kept "
                      "ones on the radial grid)", "value": screened / sec,
            "unit": "elements/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "screened coupling build, p-H2O (j1<=28) + p-H2 (j2<=10) "
                                   "below 8000 cm^-1, N=%d states, %d terms, screening at "
                                   "6.03 and 7.11 bohr, %d kept elements on 63 knots"
                                   % (basis.N, len(terms), n_kept),
                       "N": basis.N, "terms": len(terms), "kept": n_kept,
                       "screened": screened}}
    if not args.no_cpu:
        import oracle
        rng = np.random.default_rng(5)
        m0 = basis.m.min()
        pairs = []
        while len(pairs) < cpu_pairs:
            f = int(rng.integers(0, basis.N))
            same = np.where(basis.m == basis.m[f])[0]
            pairs.append((f, int(rng.choice(same))))
        t0 = time.time()
        for f, i in pairs:
            sub = CP.CouplingBasis(basis.j[[f, i]], basis.m[[f, i]], basis.rot1[[f, i]],
                                   basis.j2[[f, i]], basis.rot1_j, basis.rot1_tau, basis.b,
                                   basis.E[[f, i]], np.zeros(0, np.int32), np.zeros(0, np.int32),
                                   np.zeros(0), np.zeros(2, np.int32), 2)
            oracle.coupling_tables(sub, ex)
        csec = time.time() - t0
        line["cpu_baseline"] = {"value": len(pairs) / csec, "unit": "elements/s",
                                "cores": oracle.threads(), "kind": "oracle",
                                "sample": "%d random equal-m elements, Eq. 17 sums at 63 knots, "
                                          "%.1f s" % (len(pairs), csec)}
        log("coupling_paper: oracle %.3g elements/s" % (len(pairs) / csec))
    return line


def rates_workload(args, L=1032, n_T=20, cpu_pairs=600):
    """Post-processing (Section III): 1032 non-degenerate levels (the paper's count for
    an o/p-H2O + p-H2 symmetry), cross sections at the paper's ten collision energies
    (20 - 12000 cm^-1), Eq. 20 symmetrisation, then rate coefficients at 20
    temperatures from 10 to 2000 K: 2.1e7 Maxwell-Boltzmann integrals.  Level
    energies and degeneracies are synthetic (0 - 8000 cm^-1, g = (2j1+1)(2j2+1) with
    j1 <= 28, j2 <= 10); cross sections smooth positive functions of U.  One step =
    Eq. 20 + all rates, inputs and outputs in device memory."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import units as UU
    rng = np.random.default_rng(np.random.SeedSequence([231202322, 7]))
    U = UU.cm_to_hartree(np.array([20.0, 41.28, 84.0, 170.47, 346.41, 703.89, 1430.0, 2906.3,
                                   5906.0, 12000.0]))
    E = np.sort(UU.cm_to_hartree(8000.0 * rng.random(L)))
    g = ((2 * rng.integers(0, 29, L) + 1) * (2 * rng.integers(0, 11, L) + 1)).astype(float)
    A = rng.random((L, L)) * 30.0
    p = 0.2 + 0.6 * rng.random((L, L))
    Uc = UU.cm_to_hartree(3000.0 + 6000.0 * rng.random((L, L)))
    sigma = A[None] * (U[:, None, None] / U[0]) ** p[None] * np.exp(-U[:, None, None] / Uc[None])
    T = np.geomspace(10.0, 2000.0, n_T)
    beta = 3.166811563e-6 * T
    mu = UU.amu_to_me(1.8)
    dev = torch.device("cuda", 0)
    td = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    dU, dE, dg, dsig, db = td(U), td(E), td(g), td(sigma), td(beta)
    dsym = torch.empty_like(dsig)
    dk = torch.empty((n_T, L, L), dtype=torch.float64, device=dev)
    ctx = mq.Context(0)
    L_ = mq.lib()
    P = lambda t: C.c_void_p(t.data_ptr())

    def step():
        ctx._check(L_.mqct_xs_symmetrize(ctx.h, mq.MEM_DEVICE, U.size, L, P(dg), P(dsig), P(dsym),
                                         None))
        ctx._check(L_.mqct_rate_coefficients(ctx.h, mq.MEM_DEVICE, U.size, L, P(dU), P(dE), P(dg),
                                             P(dsym), mu, n_T, P(db), P(dk)))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    ctx.close()
    n_int = n_T * L * L
    log("rates: %d levels, %d temperatures: %.2f ms per step, %.3g rate coefficients/s"
        % (L, n_T, ms, n_int / (ms * 1e-3)))
    line = {"metric": "rate coefficients/s (Maxwell-Boltzmann integrals of Eq. 20 cross "
                      "sections)", "value": n_int / (ms * 1e-3), "unit": "rates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "%d levels x %d collision energies -> Eq. 20 -> rate "
                                   "coefficients at %d temperatures" % (L, U.size, n_T),
                       "levels": L, "energies": int(U.size), "temperatures": n_T}}
    if not args.no_cpu:
        from oracle import postproc as PP
        sym = PP.symmetrize(sigma, g)
        pick = rng.integers(0, L, (cpu_pairs // n_T + 1, 2))
        pairs = [tuple(x) for x in pick]
        t0 = time.time()
        PP.rate_coefficients(U, sym, E, g, mu, beta, pairs=pairs)
        csec = time.time() - t0
        line["cpu_baseline"] = {"value": len(pairs) * n_T / csec, "unit": "rates/s", "cores": 1,
                                "kind": "oracle",
                                "sample": "%d transitions x %d temperatures (scipy quad), %.1f s"
                                          % (len(pairs), n_T, csec)}
    return line


def uneven_workload(args):
    """Three systems in one batch -- rotor + atom (N = 49), rotor + rotor (N = 256),
    asymmetric top + atom (N = 969) -- 60 / 30 / 10 % of --uneven-traj trajectories,
    collision energies log-uniform in 10-5000 cm^-1, adaptive DP5 (rtol = atol =
    1e-8, at most 10^5 steps), FP32 tables, on the work-list schedule.  A warm-up
    batch (the first 4000 trajectories, 50 steps) lets the autotuner pick each
    class's shape; the timed run is the whole batch from start to finish."""
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import systems as S
    t0 = time.time()
    systems, b = S.config3(n_traj=args.uneven_traj)
    log("uneven: generated %s, B=%d in %.1fs" % ([x.N for x in systems], b.B, time.time() - t0))
    ctx = mq.Context(0)
    kinds = ["R32", "R32", "C64"]
    layouts = []
    for x in systems:
        A = np.abs(x.M).max(axis=0)
        kept = float(np.mean((A > 0) | (A.T > 0)))
        layouts.append("sparse" if args.uneven_layout == "sparse" and kept < 0.5 else "dense")
    ids = [ctx.load_system(x, storage=k, layout=l) for x, k, l in zip(systems, kinds, layouts)]
    # table bytes one right-hand side streams: four slices of the stored matrices
    rhs_bytes = [2.0 * ctx.system_bytes(i) / x.K for i, x in zip(ids, systems)]
    sids = np.array([ids[i] for i in b.system_index], np.int32)
    Ns = np.array([systems[i].N for i in b.system_index], np.int64)
    DP = dict(integrator="dp5", rtol=1e-8, atol=1e-8, h_min=1e-6)
    start = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0)
    w = np.arange(min(4000, b.B))
    ctx.run_host(sids[w], Ns[w], init_channel=b.init_channel[w], E_coll=b.E_coll[w], b=b.b[w],
                 R0=b.R0[w], max_steps=50, **DP)
    log("uneven: autotuner %s" % ctx.tuning_report())
    torch.cuda.synchronize()
    parts = {}
    t1 = time.time()
    if args.uneven_schedule == "split":
        big = b.system_index == int(np.argmax([x.N for x in systems]))
        g = {}
        for name, m, sched in (("binned", big, "binned"), ("work_list", ~big, "queue")):
            tp = time.time()
            gp = ctx.run_host(sids[m], Ns[m], max_steps=args.uneven_max_steps, schedule=sched,
                              **{k: v[m] for k, v in start.items()}, **DP)
            parts[name] = time.time() - tp
            log("uneven split: %s part (%d trajectories) %.2f s" % (name, int(m.sum()),
                                                                    parts[name]))
            for k in ("steps", "rejects", "status"):
                if k not in g:
                    g[k] = np.zeros(b.B, gp[k].dtype)
                g[k][m] = gp[k]
    else:
        g = ctx.run_host(sids, Ns, max_steps=args.uneven_max_steps, schedule=args.uneven_schedule,
                         **start, **DP)
    sec = time.time() - t1
    steps, rej = g["steps"], g["rejects"]
    evals = 6 * (steps + rej) + 3          # attempts x 6, the two starting evaluations, the end
    alg_bytes = float(np.sum(evals * np.array([rhs_bytes[i] for i in b.system_index])))
    per = {}
    for si, x in enumerate(systems):
        m = b.system_index == si
        st = steps[m]
        per["N=%d" % x.N] = {"trajectories": int(m.sum()), "storage": kinds[si],
                             "layout": layouts[si],
                             "steps_p0_p50_p90_p100": [int(v) for v in
                                                       np.percentile(st, [0, 50, 90, 100])],
                             "rejects": int(rej[m].sum()),
                             "exited": int(np.count_nonzero(g["status"][m] & 1)),
                             "max_steps_reached": int(np.count_nonzero(g["status"][m] & 2))}
    gbps = alg_bytes / sec / 1e9   # per-trajectory streaming equivalent (the binned share reads less)
    line = {"metric": METRIC, "value": float(steps.sum()) / sec, "unit": "traj-steps/s",
            "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": sec * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "uneven batch of %d trajectories: N=49/256/969 systems "
                                   "60/30/10 %%, E_coll log-uniform 10-5000 cm^-1, DP5 rtol 1e-8, "
                                   "at most %d steps, FP32 tables (%s layout where mostly zero), "
                                   "%s" % (
                                       b.B, args.uneven_max_steps, args.uneven_layout,
                                       {"queue": "one call, work-list schedule",
                                        "split": "two calls: the N=969 class binned, then the "
                                                 "rest on the work list",
                                        "auto": "one call, default schedule: the N=969 class binned on a "
                                                "second stream beside the work list"}[
                                           args.uneven_schedule]),
                       "trajectories": b.B},
            "N2_traj_steps_per_s": float(np.sum(steps * Ns.astype(float) ** 2)) / sec,
            "coupling_work_GBps": gbps,
            "per_system": per, "autotuner": ctx.tuning_report()}
    if parts:
        line["parts_s"] = parts
    log("uneven: %.1f s, %d steps, %.3g traj-steps/s (%s)" % (
        sec, int(steps.sum()), line["value"], json.dumps(per)))
    ctx.close()
    if not args.no_cpu:
        line["cpu_baseline"] = uneven_cpu_baseline(systems, b)
    return line


def uneven_cpu_baseline(systems, b, per_system=8, max_steps=2000):
    """The FP64 oracle's DP5 on 8 trajectories of each system (the first of each in
    batch order), at most 2000 steps each."""
    import numpy as np
    import oracle
    tot_steps, tot_s = 0, 0.0
    th = oracle.threads()
    for si, x in enumerate(systems):
        idx = np.where(b.system_index == si)[0][:per_system]
        o = oracle.OracleSystem(x)
        t0 = time.time()
        r = o.propagate(b.subset(idx), method="dp5", rtol=1e-8, atol=1e-8, max_steps=max_steps,
                        h_min=1e-6)
        tot_s += time.time() - t0
        tot_steps += int(r["steps"].sum())
    log("uneven oracle: %d steps in %.1fs on %d threads" % (tot_steps, tot_s, th))
    return {"value": tot_steps / tot_s, "unit": "traj-steps/s", "cores": th, "kind": "oracle",
            "sample": "%d trajectories of each of the three systems (FP64 oracle DP5, at most "
                      "%d steps each); wall time of the propagation only" % (per_system, max_steps)}


def adjoint_timing(n_traj, n_steps, checkpoint_every=None, layout="sparse"):
    """Seconds per full 96-coefficient gradient of a b-weighted inelastic cross section.

    Two linear rotors, j1, j2 <= 3 (N = 256), potential linear in 96 coefficients,
    n_traj trajectories of n_steps RK4 steps; L = sum_i (2 pi b_max / B) b_i
    sum_{n outside the initial level} P_i(n); discrete adjoint.  checkpoint_every
    None: one segment (every stage state stored by the forward pass, nothing
    recomputed; 67 MB per trajectory at 4096 steps); the same gradient with
    checkpoints every 256 steps is timed beside it.  layout="sparse" stores only
    the structural nonzeros of the tables (drop_below = 0: the gradient of the
    same model).
    """
    import numpy as np
    import torch
    import paper_2312_02322_amd as mq
    from synth import systems as S
    (s,), b = S.config4(n_traj=n_traj, n_steps=n_steps)
    ctx = mq.Context(0)
    sid = ctx.load_system(s, layout=layout)
    ctx.set_params(sid, s.param_radial, s.param_G_index, s.G)
    ctx.set_theta(sid, s.theta)
    lev = s.level_of_channel
    w = np.array([(2 * np.pi * b.b_max / b.B) * b.b[i] * (lev != b.init_level[i])
                  for i in range(b.B)])
    kw = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, dt=b.dt, n_steps=b.n_steps,
              R0=b.R0)
    # the forward propagation of the same batch alone (per-trajectory schedule)
    fwd = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.time()
        ctx.run([sid] * b.B, [s.N] * b.B, schedule="gemv", **kw)
        torch.cuda.synchronize()
        fwd.append(time.time() - t0)
    if checkpoint_every is None:
        checkpoint_every = int(np.max(b.n_steps))
    sec_all = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.time()
        grad, P = ctx.adjoint(sid, s.N, w, checkpoint_every=checkpoint_every, **kw)
        sec_all.append(time.time() - t0)
    sec, fsec = sec_all[-1], fwd[-1]
    torch.cuda.synchronize()
    t0 = time.time()
    g256, _ = ctx.adjoint(sid, s.N, w, checkpoint_every=256, **kw)
    sec256 = time.time() - t0
    same = bool(np.array_equal(g256, grad))
    table_bytes = ctx.system_bytes(sid)
    ctx.close()
    log("adjoint (%s tables): %d trajectories x %d steps, N=%d, %d coefficients: %.2f s/grad "
        "(first call %.2f s; checkpoints every 256 steps %.2f s, same gradient: %s), forward "
        "alone %.2f s (ratio %.1f), |grad| = %.3e" % (
            layout, b.B, n_steps, s.N, grad.shape[0], sec, sec_all[0], sec256, same, fsec,
            sec / fsec, float(np.linalg.norm(grad))))
    return {"s_per_grad": sec, "unit": "s", "first_call_s": sec_all[0], "forward_s": fsec,
            "adjoint_over_forward": sec / fsec, "layout": layout, "table_bytes": table_bytes,
            "trajectories": b.B,
            "rk4_steps": n_steps, "N": s.N,
            "n_coefficients": int(grad.shape[0]), "checkpoint_every": checkpoint_every,
            "s_per_grad_checkpoint_256": sec256, "same_gradient_checkpoint_256": same,
            "L": float(np.sum(w * P)), "grad_norm": float(np.linalg.norm(grad))}


def _source_hash(name):
    import hashlib
    src = os.path.join(ROOT, "paper_2312_02322_amd", "csrc", name)
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def cpu_baseline(s, b, W):
    """The FP64 oracle on a bounded sample of the same workload (rank 0 only).

    The sample is the first n trajectories of the batch over the same window of
    W RK4 steps, with n sized from a short calibration run to take ~12 s.
    """
    import numpy as np
    import oracle
    t0 = time.time()
    o = oracle.OracleSystem(s)
    log("oracle spline prep %.1fs" % (time.time() - t0))
    th = oracle.threads()
    n = max(1, min(b.B, th))
    t0 = time.time()
    o.propagate(b.subset(range(n)), n_steps=np.full(n, W))
    t1 = time.time() - t0
    n = int(min(b.B, max(n, th * round(12.0 / max(t1, 1e-3)))))
    t0 = time.time()
    o.propagate(b.subset(range(n)), n_steps=np.full(n, W))
    dt = time.time() - t0
    log("oracle: %d trajectories x %d steps in %.1fs on %d threads" % (n, W, dt, th))
    return {"value": n * W / dt, "unit": "traj-steps/s", "cores": th, "kind": "oracle",
            "sample": "first %d of the %d trajectories x the same %d RK4 steps (FP64 oracle, "
                      "complex N=969 tables); wall time of the propagation only" % (n, b.B, W)}


def read_bandwidth_probe(reps=20, ctx=None):
    """Achievable streaming-read bandwidth with the library's read kernel (1 KiB
    contiguous wave loads, four workgroups per compute unit) over buffers of 2 GB
    (HBM), 200 MB (fits the 256 MB Infinity Cache) and 8 MB (fits the L2 of the
    dies), `reps` passes each timed with events."""
    import torch
    import paper_2312_02322_amd as mq
    own = ctx is None
    if own:
        ctx = mq.Context(0)
    out = {}
    for name, nbytes in (("2GB", 2 << 30), ("200MB", 200 << 20), ("8MB", 8 << 20)):
        x = torch.ones(nbytes // 4, dtype=torch.float32, device=ctx.device)
        ms = ctx.read_bandwidth(x, reps)
        out[name] = {"bytes": nbytes, "ms": ms, "GBps": nbytes / (ms * 1e-3) / 1e9}
        log("read probe %s: %.4f ms, %.0f GB/s" % (name, ms, out[name]["GBps"]))
        del x
    if own:
        ctx.close()
    torch.cuda.empty_cache()
    return {"read_bandwidth_probe": out}


def copy_probe(nbytes):
    """A plain device-to-device copy of known size, for calibrating byte counters."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reads": nbytes, "writes": nbytes}))


if __name__ == "__main__":
    main()
