"""Throughput of the screened-WKB screen step on one MI355X.

Workload: the smooth random medium (lambda = 1; 200 seeded Gaussian index
bumps; 1000 x 4000 wavelengths; N = 8192 grid points, M = 2048 modes,
400 screens of width 10).  One step = one full propagation across all 400
screens (FFT, ray march, interpolation and superposition per screen), input
field resident on the device.  The mixed-precision path (FP32 march,
interpolation and phase evaluation; FP64 ray-tube variations and phase
bookkeeping) is the reported value; the plain FP64 path is timed beside it
and the mixed result is checked against it.

Prints one JSON line.  --gpus must be 1: the propagation runs on one GPU.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mode×point evals/s; range km/s at 1e-3 rel err vs FP64 plain; p50/p99 latency"

# Algorithmic flops of the ray march (transcendentals, divisions and square
# roots count as one flop each; a fused multiply-add as two):
#   per RK4 stage evaluation of the ray system                      51
#     (35 in the right-hand side, 16 in the stage/step combinations)
#   per evaluation of eps, eps_z/2, eps_zz/2 from the index deviation 7
#   per Gaussian term inside its cutoff (distance, exp, 3 sums)      22
#   per medium value read from the per-screen table (node index and
#     offset 4, cubic and its two derivatives by Horner 12, scaling 2)   18
FLOPS_PER_RHS = 51
FLOPS_PER_MEDIUM = 7
FLOPS_PER_TERM = 22
FLOPS_PER_TABLE = 18
PEAK_FP32_VECTOR = 157.3e12   # MI355X published dense FP32 vector FLOP/s (counts packed FP32)
PEAK_FP64_VECTOR = 78.6e12
PEAK_HBM = 8.0e12            # MI355X published HBM3E bandwidth, bytes/s
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz: the FP32 ceiling of
# code without packed FP32 instructions (this build excludes them)
PEAK_ALU_NONPACKED = 256 * 4 * 16 * 2 * 2.4e9


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("march.hip", "medium.h"):
        with open(os.path.join(ROOT, "paper_2301_03814_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def traffic_from_profiles(precision):
    """HBM bytes per launch of the march kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "march_random_medium_N8192_pmc.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    rec = d.get(precision)
    return None if rec is None else rec.get("hbm_bytes_per_launch")


def bench_serving(torch, np, W, Plan, Server, FP64, MIXED, n_req=64):
    """Serving loop on the first n_req requests of the seeded Poisson stream
    (20 req/s; ducts and random media, N_z 1024..32768, M = N_z/4, ranges as
    in the stream): requests are submitted at their arrival times (wall
    clock) to the library's server (mixed precision, continuous batching),
    latency = completion seen by the host minus arrival.  Baseline: the same
    requests, at the same arrival times, served one after another in arrival
    order with plain FP64 plans (a FIFO server on the wall clock)."""
    reqs = W.serving_stream(seed=5, rate=20.0, duration=60.0)[:n_req]
    dev = torch.device("cuda:0")
    u0s = [W.incident_field(c) for _, c in reqs]
    work = sum(c["n_modes"] * c["n_z"] * c["n_screens"] for _, c in reqs)
    srv = Server(200 << 30, max_active=16, screens_per_round=1, mode_points_per_round=2e9)
    ids, done, nxt = {}, {}, 0
    t0 = time.perf_counter()
    while len(done) < n_req:
        now = time.perf_counter() - t0
        while nxt < n_req and reqs[nxt][0] <= now:
            ids[nxt] = srv.submit(reqs[nxt][1], u0s[nxt], precision=MIXED)
            nxt += 1
        srv.step()
        for i, rid in ids.items():
            if i not in done:
                _, _, field = srv.poll(rid)
                if field is not None:
                    done[i] = (time.perf_counter() - t0 - reqs[i][0], field)
        time.sleep(0.0002)
    wall = time.perf_counter() - t0
    srv.close()
    lat = np.array([done[i][0] for i in range(n_req)])
    # FP64 plain, one request at a time in arrival order, on the wall clock
    service, errs, lat64 = [], [], []
    t0 = time.perf_counter()
    for i, (t_arr, c) in enumerate(reqs):
        now = time.perf_counter() - t0
        if now < t_arr:
            time.sleep(t_arr - now)
        s0 = time.perf_counter()
        p = Plan(c, precision=FP64, device=dev)
        h = p.propagate(torch.from_numpy(u0s[i]).to(dev), 0, c["n_screens"])
        ref = h[-1].cpu().numpy()
        torch.cuda.synchronize()
        t_done = time.perf_counter()
        p.close()
        del p, h
        service.append(t_done - s0)
        lat64.append(t_done - t0 - t_arr)
        errs.append(float(np.linalg.norm(done[i][1] - ref) / np.linalg.norm(ref)))
    lat64 = np.array(lat64)
    end64 = time.perf_counter() - t0
    return {
        "workload": f"first {n_req} requests of the Poisson stream (seed 5, 20 req/s): ducts (1-10 GHz, 200-500 m, "
                    "10-100 km) and random media (1000-4000 wavelengths), N_z 1024-32768, M = N_z/4",
        "requests": n_req, "mode_points": work,
        "mixed_served": {"wall_s": wall, "requests_per_s": n_req / wall, "mode_points_per_s": work / wall,
                         "latency_ms_p50": float(np.percentile(lat, 50)) * 1e3,
                         "latency_ms_p99": float(np.percentile(lat, 99)) * 1e3,
                         "max_active": 16, "mode_points_per_round": 2e9},
        "fp64_serial": {"wall_s": end64, "service_s_sum": float(sum(service)),
                        "requests_per_s": n_req / end64, "mode_points_per_s": work / float(sum(service)),
                        "served": "FIFO on the wall clock, arrivals as for the mixed server",
                        "latency_ms_p50": float(np.percentile(lat64, 50)) * 1e3,
                        "latency_ms_p99": float(np.percentile(lat64, 99)) * 1e3},
        "speedup_throughput": float(sum(service)) / wall,
        "offered_load": {"arrival_span_s": float(reqs[-1][0]), "arrival_rate_per_s": n_req / float(reqs[-1][0]),
                         "note": "arrivals outpace the FP64 server, so its latencies are mostly queueing"},
        "rel_err_mixed_vs_fp64_max": max(errs),
    }


def bench_duct(args, torch, np, W, Plan, FP64, MIXED):
    """Surface duct at 6 GHz (N = 16384, M = 4096, 1000 screens of 100 m,
    Dirichlet ground mirror): an x-invariant medium, so the plan tabulates
    the mode functions once and every screen is FFT + matrix product; beside
    it the plain per-screen step (rays reused, interpolation and sum over
    modes every screen)."""
    B = 16
    cfg = W.with_overrides(W.surface_duct(), max_batch=B)
    N, M, Q = cfg["n_z"], cfg["n_modes"], cfg["n_screens"]
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    srcs = []
    for b in range(B):  # sources at heights 10..85 m
        c = W.with_overrides(cfg)
        c["source"] = dict(cfg["source"], z0=10.0 + 5.0 * b)
        srcs.append(W.incident_field(c))
    U0 = torch.from_numpy(np.stack(srcs)).to(dev)
    out = {"workload": "surface duct: lambda=0.05 m, M-profile -0.3/+0.118 M/m (corner 40 m), 0-300 m, "
                       "N_z=16384, 4096 modes, 1000 screens of 100 m (100 km), Dirichlet ground"}
    hist = {}
    for name, prec in (("mixed", MIXED), ("fp64", FP64)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = Plan(cfg, precision=prec, device=dev)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        h = torch.empty((Q, N), dtype=torch.complex128, device=dev)
        plan.propagate(u0, 0, Q, out=h)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.propagate(u0, 0, Q, out=h)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        hist[name] = h[::50].cpu().numpy()
        del h
        plan.propagate_batch(U0, 0, Q, history=False)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.propagate_batch(U0, 0, Q, history=False)
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0
        out[name] = {"mode_point_evals_per_s": M * N * Q / dt, "ms_per_run": 1e3 * dt,
                     "range_km_per_s": 100.0 / dt, "plan_build_ms": 1e3 * t_plan,
                     "uses_matrix": plan.uses_matrix,
                     f"batch{B}": {"mode_point_evals_per_s": B * M * N * Q / dtb, "ms_per_run": 1e3 * dtb,
                                   "note": f"{B} sources (heights 10-85 m) per screen as one complex matrix product on the matrix cores"}}
        plan.close()
        # the plain per-screen step on the same workload
        plain = Plan(W.with_overrides(cfg, propagator=2, max_batch=1), precision=prec, device=dev)
        h = torch.empty((Q, N), dtype=torch.complex128, device=dev)
        plain.propagate(u0, 0, Q, out=h)  # warm-up (marches the rays once)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain.propagate(u0, 0, Q, out=h)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        hp = h[::50].cpu().numpy()
        del h
        plain.close()
        out[name]["plain_per_screen"] = {
            "mode_point_evals_per_s": M * N * Q / dtp, "ms_per_run": 1e3 * dtp, "range_km_per_s": 100.0 / dtp,
            "rel_diff_vs_matrix_every_50th_screen": float(np.linalg.norm(hp - hist[name]) / np.linalg.norm(hist[name]))}
    out["rel_err_mixed_vs_fp64_every_50th_screen"] = float(
        np.linalg.norm(hist["mixed"] - hist["fp64"]) / np.linalg.norm(hist["fp64"]))
    print(f"[bench] duct: {out}", file=sys.stderr, flush=True)
    return out


def bench_multi(torch, np, W, Plan, Multi, MIXED, n_problems=64, graphs=True):
    """The seeded batch of uneven duct problems (1-10 GHz, duct depth 10-100
    m, 200-500 m high, 10-100 km, N_z 2048-16384, M = N_z/4, mixed): every
    problem one after another through its own plan (HIP graphs), then all of
    them in one group (one launch per stage per screen step), with the
    single-problem launch shapes and autotuned with the step sequence
    replayed as one HIP graph, and the autotuned shapes in one persistent
    launch for the whole run."""
    cfgs = W.duct_batch(seed=4, n_problems=n_problems)
    dev = torch.device("cuda:0")
    mp = sum(c["n_z"] * c["n_modes"] * c["n_screens"] for c in cfgs)
    tbytes = sum(8 * c["n_z"] * c["n_modes"] * c["n_screens"] for c in cfgs)  # complex64 T read per screen
    km = sum(c["n_screens"] * c["dx"] for c in cfgs) / 1e3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans = [Plan(c, precision=MIXED, device=dev) for c in cfgs]
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    u0s = [torch.from_numpy(W.incident_field(c)).to(dev) for c in cfgs]

    def timed(fn):
        fn()  # warm-up (graph capture)
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    for p in plans:
        p.graphs(graphs)
    t_seq = timed(lambda: [p.propagate(u, 0, c["n_screens"], history=False) for p, u, c in zip(plans, u0s, cfgs)])
    seq_fields = [p.field() for p in plans]
    for p in plans:
        p.graphs(False)
    m = Multi(plans)
    t_def = timed(lambda: m.propagate(u0s))
    same = all(bool(torch.equal(p.field(), f)) for p, f in zip(plans, seq_fields))
    t0 = time.perf_counter()
    tun = m.tune(reps=5)
    t_tune = time.perf_counter() - t0
    m.set_tuning(graphs=graphs)
    t_tuned = timed(lambda: m.propagate(u0s))
    dev_max = max(float(torch.linalg.vector_norm(p.field() - f) / torch.linalg.vector_norm(f))
                  for p, f in zip(plans, seq_fields))
    tuned_fields = [p.field() for p in plans]
    # the same tuned shapes in one persistent (cooperative) launch
    m.set_tuning(persistent=True)
    t_pers = timed(lambda: m.propagate(u0s))
    same_pers = all(bool(torch.equal(p.field(), f)) for p, f in zip(plans, tuned_fields))
    m.set_tuning(persistent=False, graphs=graphs)
    out = {
        "workload": f"{n_problems} uneven surface-duct problems (seed 4): 1-10 GHz, duct depth 10-100 m, "
                    f"in-duct slope -0.5..-0.1 M/m, 200-500 m high, 10-100 km in 100 m screens, "
                    f"N_z 2048-16384, M = N_z/4, Dirichlet ground, mixed",
        "mode_points": mp, "screens": sum(c["n_screens"] for c in cfgs), "range_km": km,
        "plan_build_s": round(t_build, 3),
        "one_after_another": {"seconds": t_seq, "mode_point_evals_per_s": mp / t_seq},
        "group_default_shapes": {"seconds": t_def, "mode_point_evals_per_s": mp / t_def,
                                 "bit_identical_to_one_after_another": same},
        "group_autotuned_graph": {"seconds": t_tuned, "mode_point_evals_per_s": mp / t_tuned,
                                  "range_km_per_s": km / t_tuned,
                                  "max_rel_diff_vs_one_after_another": dev_max},
        "group_autotuned_persistent": {"seconds": t_pers, "mode_point_evals_per_s": mp / t_pers,
                                       "range_km_per_s": km / t_pers,
                                       "bit_identical_to_autotuned_graph": same_pers},
        "autotune_s": round(t_tune, 3),
        "tuning": {k: tun[k] for k in ("n_z", "fft_elems", "apply_groups")},
        "speedup_vs_one_after_another": t_seq / t_tuned,
        "matrix_stream": {"bytes": tbytes, "achieved_GBps": tbytes / t_tuned / 1e9,
                          "frac_of_hbm_peak": tbytes / t_tuned / PEAK_HBM,
                          "note": "complex64 mode-function matrices read once per screen over the whole run "
                                  "(FFT, partial sums and epilogue included in the time)"},
    }
    m.close()
    for p in plans:
        p.close()
    print(f"[bench] multi: {out}", file=sys.stderr, flush=True)
    return out


def bench_patches(torch, np, W, Plan, PatchPlan, MIXED, n_patches=8):
    """Tall surface ducts (6 GHz, 1000 screens of 100 m, Dirichlet ground,
    mixed): 0-600 m (N_z = 32768, 8192 modes) by the single-domain step and by
    the overlapping-patch steps (8 patches, partition of unity of scale 1 m,
    margins of 20 m): the paper's Fourier-continuation patches and the
    library's windowed pieces; 0-1200 m (N_z = 65536, 16384 modes: beyond one
    plan's grid) by patches only."""
    from paper_2301_03814_amd import PATCH_FC, PATCH_WINDOWED
    methods = (("fourier_continuation", PATCH_FC), ("windowed", PATCH_WINDOWED))
    dev = torch.device("cuda:0")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    def run_patches(cfg, method):
        Q = cfg["n_screens"]
        u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pp = PatchPlan(cfg, n_patches, 1.0, 20.0, precision=MIXED, method=method)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        info = pp.info()
        pp.graphs(True)
        h = torch.empty((Q, cfg["n_z"]), dtype=torch.complex128, device=dev)
        dt, _ = timed(lambda: pp.propagate(u0, 0, Q, out=h))  # first call captures, the timed one replays
        got = h[::50].cpu().numpy()
        del h
        pp.close()
        work = sum(n * m for _, n, m in info)
        return got, {"seconds": dt, "n_patches": n_patches, "window_m": 1.0, "margin_m": 20.0,
                     "sub_domains": [{"start": a, "n_z": b, "n_modes": c} for a, b, c in info],
                     "mode_points_per_screen": work, "plan_build_s": round(tb, 3),
                     "range_km_per_s": 100.0 / dt,
                     "global_mode_point_evals_per_s": cfg["n_z"] * cfg["n_modes"] * Q / dt, "hip_graph": True}

    cfg = W.surface_duct(n_z=32768, n_modes=8192, height=600.0)
    N, M, Q = cfg["n_z"], cfg["n_modes"], cfg["n_screens"]
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    full = Plan(cfg, precision=MIXED, device=dev)
    torch.cuda.synchronize()
    tb_full = time.perf_counter() - t0
    dt_full, h = timed(lambda: full.propagate(u0, 0, Q, history=True))
    ref = h[::50].cpu().numpy()
    del h
    full.close()
    runs = {name: run_patches(cfg, m) for name, m in methods}
    out = {"workload": "surface ducts: lambda=0.05 m, M-profile -0.3/+0.118 M/m, 1000 screens of 100 m (100 km), "
                       "Dirichlet ground, mixed; 0-600 m with N_z=32768, 8192 modes; 0-1200 m with N_z=65536, "
                       "16384 modes",
           "h600": {"single_domain": {"seconds": dt_full, "mode_points_per_screen": N * M,
                                      "plan_build_s": round(tb_full, 3), "range_km_per_s": 100.0 / dt_full,
                                      "mode_point_evals_per_s": N * M * Q / dt_full},
                    }}
    for name, (got, pat) in runs.items():
        pat["speedup_vs_single_domain"] = dt_full / pat["seconds"]
        pat["rel_diff_vs_single_domain_every_50th_screen"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        out["h600"][f"patches_{name}"] = pat
    cfg2 = W.surface_duct(n_z=65536, n_modes=16384, height=1200.0)
    pat2 = {f"patches_{name}": run_patches(cfg2, m)[1] for name, m in methods}
    out["h1200"] = dict(pat2, single_domain="beyond one plan's grid (n_z <= 32768)")
    print(f"[bench] patches: {out}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-duct", action="store_true", help="skip the surface-duct measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-multi", action="store_true", help="skip the uneven duct batch measurement")
    ap.add_argument("--no-patches", action="store_true", help="skip the overlapping-patch measurement")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the step with per-kernel events (kernels one after another), for rocprofv3")
    ap.add_argument("--only", choices=("duct", "multi", "patches", "serving"), default=None,
                    help="run only that section and print its JSON (for rocprofv3 summaries)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="uneven batch without HIP graphs (for rocprofv3 counter collection)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy kernel over BYTES bytes (HBM counter calibration)")
    args = ap.parse_args()
    if args.profile_only:
        args.steps = 0
    if args.copy_probe:
        import torch
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)  # reads and writes BYTES bytes
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the screened-WKB path is "
              "measured on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2301_03814_amd import FP64, MIXED, Plan

    if args.only == "duct":
        print(json.dumps(bench_duct(args, torch, np, W, Plan, FP64, MIXED)))
        return
    if args.only == "patches":
        from paper_2301_03814_amd import PatchPlan
        print(json.dumps(bench_patches(torch, np, W, Plan, PatchPlan, MIXED)))
        return
    if args.only == "serving":
        from paper_2301_03814_amd import Server
        print(json.dumps(bench_serving(torch, np, W, Plan, Server, FP64, MIXED)))
        return
    if args.only == "multi":
        from paper_2301_03814_amd import Multi
        print(json.dumps(bench_multi(torch, np, W, Plan, Multi, MIXED, graphs=not args.no_graphs)))
        return

    cfg = W.random_medium()
    N, M, Q = cfg["n_z"], cfg["n_modes"], cfg["n_screens"]
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    plans = {"mixed": Plan(cfg, precision=MIXED, device=dev), "fp64": Plan(cfg, precision=FP64, device=dev)}
    hists = {k: torch.empty((Q, N), dtype=torch.complex128, device=dev) for k in plans}
    for p in plans.values():
        # eager launches: on these long x-varying steps the two streams' kernels
        # overlap better than in a replayed HIP graph (timed beside it below)
        p.graphs(False)

    def step(name):
        plans[name].propagate(u0, 0, Q, out=hists[name])

    for _ in range(args.warmup):
        for name in plans:
            step(name)
    torch.cuda.synchronize()

    def roof(r, peak, prec):
        w, p = r["work"], r["prof"]
        flops = FLOPS_PER_RHS * w["rhs_evals"] + FLOPS_PER_MEDIUM * w["medium_evals"] + \
            FLOPS_PER_TERM * w["medium_terms"] + FLOPS_PER_TABLE * w["table_evals"]
        launches = max(1, p["march_launches"])
        avg_s = p["march_ms"] * 1e-3 / launches
        per_launch = flops / launches
        achieved = per_launch / avg_s / 1e12
        t = traffic_from_profiles(prec)
        return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak / 1e12, 1), "unit": "TFLOP/s",
                "frac": round(achieved * 1e12 / peak, 4), "traffic": t,
                "kernel": "march_table_kernel" if w["table_evals"] else
                          f"march_gauss_kernel<{'float' if prec == 'mixed' else 'double'}>",
                "table_share": round(w["table_evals"] / max(1, w["table_evals"] + w["medium_evals"]), 4),
                "peak_nonpacked": round(PEAK_ALU_NONPACKED / 1e12, 1),
                "frac_of_nonpacked": round(achieved * 1e12 / PEAK_ALU_NONPACKED, 4),
                "flops_per_launch": per_launch, "avg_launch_ms": round(avg_s * 1e3, 4),
                "rhs_evals_per_launch": w["rhs_evals"] / launches, "table_evals_per_launch": w["table_evals"] / launches}

    res = {}
    for name, plan in plans.items():
        # timed steps: no per-kernel events
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            step(name)
            e1.record()
            lat.append((e0, e1))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # one more step with HIP events around every kernel: per-kernel times and work counts
        base = plan.diagnostics()
        plan.profile(True)
        plan.profile_read()
        step(name)
        prof = plan.profile_read()
        plan.profile(False)
        diag = plan.diagnostics()
        work = {k: diag[k] - base[k] for k in ("rhs_evals", "medium_evals", "medium_terms", "table_evals",
                                                "screens")}
        res[name] = dict(seconds=t1 - t0, prof=prof, work=work, diag=diag,
                         lat_ms=sorted(a.elapsed_time(b) for a, b in lat))
        if name == "mixed" and not args.profile_only:
            # the same steps replayed from a captured HIP graph (reported beside the value)
            plan.graphs(True)
            step(name)  # capture
            torch.cuda.synchronize()
            tg = time.perf_counter()
            for _ in range(args.steps):
                step(name)
            torch.cuda.synchronize()
            res[name]["graph_ms_per_step"] = 1e3 * (time.perf_counter() - tg) / max(1, args.steps)
            plan.graphs(False)
        print(f"[bench] {name}: {1e3 * (t1 - t0) / max(1, args.steps):.1f} ms/step {prof}", file=sys.stderr,
              flush=True)
    if args.profile_only:
        print(json.dumps({"profile_only": True, "kernel_ms_per_step": {n: r["prof"] for n, r in res.items()},
                          "roofline": roof(res["mixed"], PEAK_FP32_VECTOR, "mixed"),
                          "fp64_roofline": roof(res["fp64"], PEAK_FP64_VECTOR, "fp64")}))
        return

    # four sources through the same random medium: rays marched once per screen
    Bm = 4
    cfgb = W.with_overrides(cfg, max_batch=Bm)
    srcs = []
    for b in range(Bm):
        c = W.with_overrides(cfg)
        c["source"] = dict(cfg["source"], z0=350.0 + 100.0 * b)
        srcs.append(W.incident_field(c))
    U0 = torch.from_numpy(np.stack(srcs)).to(dev)
    pb = Plan(cfgb, precision=MIXED, device=dev)
    pb.propagate_batch(U0, 0, Q, history=False)
    torch.cuda.synchronize()
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        pb.propagate_batch(U0, 0, Q, history=False)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    dtb = sorted(runs)[1]  # median of three runs
    batch_line = {"fields": Bm, "mode_point_evals_per_s": Bm * M * N * Q / dtb, "ms_per_run": 1e3 * dtb,
                  "ms_runs": [round(1e3 * t, 2) for t in runs],
                  "note": "4 sources (heights 350-650) in one propagation: one march per screen, interpolation "
                          "and sin/cos shared by the 4 fields"}
    pb.close()
    del U0

    hm, hd = hists["mixed"].cpu().numpy(), hists["fp64"].cpu().numpy()
    err_mixed = float(np.linalg.norm(hm - hd) / np.linalg.norm(hd))

    mp_per_step = M * N * Q
    rm = res["mixed"]
    ms_step = 1e3 * rm["seconds"] / args.steps
    value = mp_per_step * args.steps / rm["seconds"]
    fp64_ms = 1e3 * res["fp64"]["seconds"] / args.steps

    roof_m = roof(rm, PEAK_FP32_VECTOR, "mixed")
    roof_d = roof(res["fp64"], PEAK_FP64_VECTOR, "fp64")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        threads = oracle.max_threads()
        samples = tuple(range(0, Q, Q // 8))  # 8 screens, about 10 s of oracle work
        # every sampled screen starts from the workload's seeded incident beam,
        # on the GPU (FP64 plan, one screen) and in the oracle alike
        u_in = W.incident_field(cfg)
        p64 = plans["fp64"]
        p64.graphs(False)
        u_in_d = torch.from_numpy(u_in).to(dev)
        gpu_q = {q: p64.propagate(u_in_d, q, q + 1)[0].cpu().numpy() for q in samples}
        t0 = time.perf_counter()
        errs = []
        for q in samples:
            ref, _ = oracle.screen(cfg, q, u_in)
            errs.append(float(np.linalg.norm(gpu_q[q] - ref) / np.linalg.norm(ref)))
        tc = time.perf_counter() - t0
        cpu = {"value": M * N * len(samples) / tc, "unit": "mode-point evals/s", "cores": threads,
               "kind": "oracle",
               "sample": f"screens {list(samples)} of the same workload (FP64 oracle, OpenMP over modes, "
                         f"{threads} threads), each started from the workload's incident beam on that screen",
               "seconds": round(tc, 2), "fp64_gpu_vs_oracle_rel_l2_max": max(errs)}
        # the same oracle on one thread (the paper's timings are single-core), screen 0 only
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.screen(cfg, 0, W.incident_field(cfg))
        t1c = time.perf_counter() - t0
        oracle.set_threads(threads)
        cpu["one_thread"] = {"value": M * N / t1c, "seconds": round(t1c, 2), "sample": "screen 0"}
        cpu["host"] = {"cpu_model": cpu_model(), "logical_cpus": os.cpu_count()}
        # the small case in full (linear caustic: N_z = 512, 128 modes, 32
        # screens): the oracle beside the GPU plans, and their agreement
        c1 = W.linear_caustic()
        u1 = W.incident_field(c1)
        t0 = time.perf_counter()
        ref1, cnt1 = oracle.run(c1, u1)
        t_or = time.perf_counter() - t0
        small = {"workload": "linear caustic: lambda=1, eps=1+0.02z, z in [0,64], N_z=512, 128 modes, 32 screens "
                             "of 8, beam width 4 at z=16 tilted 10 degrees down",
                 "oracle_seconds": round(t_or, 3), "oracle_threads": threads}
        u1d = torch.from_numpy(u1).to(dev)
        for name, prec in (("fp64", FP64), ("mixed", MIXED)):
            pl1 = Plan(c1, precision=prec, device=dev)
            pl1.propagate(u1d, 0, c1["n_screens"])
            d0 = pl1.diagnostics()  # counters of the warm-up run (synchronises)
            t0 = time.perf_counter()
            h1 = pl1.propagate(u1d, 0, c1["n_screens"])
            torch.cuda.synchronize()
            dt1 = time.perf_counter() - t0
            d1 = pl1.diagnostics()
            same = all(d1[k] - d0[k] == cnt1[k] for k in ("caustic_rays", "dead_rays"))
            small[name] = {"seconds": round(dt1, 5),
                           "rel_l2_vs_oracle": float(np.linalg.norm(h1.cpu().numpy() - ref1) / np.linalg.norm(ref1)),
                           "caustic_and_dead_rays_equal_oracle": bool(same)}
            pl1.close()
        cpu["small_case"] = small

    duct = None
    if not args.no_duct:
        duct = bench_duct(args, torch, np, W, Plan, FP64, MIXED)
    multi = None
    if not args.no_multi:
        from paper_2301_03814_amd import Multi
        multi = bench_multi(torch, np, W, Plan, Multi, MIXED)
    patches = None
    if not args.no_patches:
        from paper_2301_03814_amd import PatchPlan
        patches = bench_patches(torch, np, W, Plan, PatchPlan, MIXED)
    serving = None
    if not args.no_serving:
        from paper_2301_03814_amd import Server
        serving = bench_serving(torch, np, W, Plan, Server, FP64, MIXED)
        print(f"[bench] serving: {serving}", file=sys.stderr, flush=True)

    p50 = float(np.percentile(rm["lat_ms"], 50))
    p99 = float(np.percentile(rm["lat_ms"], 99))
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "mode-point evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "random_medium: lambda=1, 200 Gaussian index bumps (seed 2301), 1000x4000 "
                               "wavelengths, N_z=8192, 2048 modes, 400 screens of 10, RK4 S=8, ray stride 8",
                   "n_z": N, "n_modes": M, "n_screens": Q, "rays_per_mode": plans["mixed"].num_rays,
                   "precision": "mixed: FP32 ray state, medium table, interpolation and sin/cos; FP64 ray "
                                "tube (Z_s, Q_s accumulated in FP64 from FP32 RK4 increments) and transport "
                                "amplitude, range phase, FFT and cross-group sums",
                   "hip_graphs": False},
        "range_wavelengths_per_s": 4000.0 * args.steps / rm["seconds"],
        "rel_err_mixed_vs_fp64": err_mixed,
        "latency_ms_p50": p50,
        "latency_ms_p99": p99,
        "graph_replay_ms_per_step": round(res["mixed"]["graph_ms_per_step"], 3),
        "fp64": {"value": mp_per_step * args.steps / res["fp64"]["seconds"], "ms_per_step": fp64_ms,
                 "roofline": roof_d},
        "speedup_mixed_vs_fp64": fp64_ms / ms_step,
        "kernel_ms_per_step": {k: round(v, 3) for k, v in rm["prof"].items() if k.endswith("_ms")},
        "batched_mixed": batch_line,
        "roofline": roof_m,
        "cpu_baseline": cpu,
        "surface_duct": duct,
        "uneven_duct_batch": multi,
        "tall_duct_patches": patches,
        "serving": serving,
    }
    print(json.dumps(line))
    for p in plans.values():
        p.close()


if __name__ == "__main__":
    main()
