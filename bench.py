"""Benchmark of the trajectory engine on one MI355X.

Workload (N=1): the 26-qubit d=5 rotated surface code with the cross-resonance
gate set, complex128 state (the live data register of 2^25 amplitudes,
512 MiB), p = 1e-3 depolarizing noise, per-site over-rotation theta ~
U[0, 0.05) rad (eps = theta/2) drawn once per job, ZZ crosstalk zeta = 0.01,
5 noisy rounds of 24 stabilizer circuits, seed 1; synthetic by construction.

A step is one whole trajectory: logical |0>, 5 rounds (per round one register
pass per X check and one per chain of up to four Z checks, 15 passes for the
24 circuits, each deciding its measurements on the device), the final Z
measurement of the 25 data qubits.  K steps are timed as one sv_run_rounds
call of K trajectories after W warm-up trajectories.

Printed: one JSON line with the round time (ms, lower is better), the
per-circuit algorithmic HBM rate, the roofline of the dominant kernel (the
register pass: one read and one write of the 2^25-amplitude register = 1 GiB
per launch) timed with HIP events on its stream inside the library, and the
oracle timed on the host cores on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# dense matrix-core peaks of MI355X: FP64 (complex128) and FP32 (complex64)
PEAK_MFMA_TFS = {"c128": 78.6, "c64": 157.3}
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_upass_d5_c128_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2204_11404_amd", "csrc", f)
                  for f in ("kernels.hip", "qec_common.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic():
    """HBM bytes per register-pass launch from the committed rocprofv3 counter
    summary, if the pass kernel's sources are unchanged since it was taken."""
    try:
        fields = {}
        with open(TRAFFIC_SUMMARY) as f:
            for line in f:
                if line.startswith("- ") and ": " in line:
                    k, v = line[2:].split(": ", 1)
                    fields[k.strip()] = v.strip().strip("`")
        if fields.get("kernel_sources_sha256") != kernel_source_hash():
            return None
        return int(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


_TUNING_FILE = None
_TUNING_LOADED = False


def tune(qs, d, dtype, gateset="cr"):
    """Launch parameters for (d, dtype): from the --tuning file when it
    existed at start-up, else autotuned (and written to the file)."""
    if _TUNING_LOADED:
        return qs.tuning_get(d, dtype)
    best, _ = qs.autotune(d, dtype, gateset)
    if _TUNING_FILE:
        qs.tuning_save(_TUNING_FILE)
    return best


def cpu_baseline(c, eps, n_blocks):
    """Oracle (complex128, gate by gate on 26 qubits) on the first n_blocks
    noisy circuits of a round; scaled to ms per 24-circuit round."""
    import oracle
    sec, threads = oracle.time_blocks(c["d"], oracle.GATESET_CR, c["seed"], 0, c["p"], n_blocks,
                                      zeta=c["zeta"], eps_site=eps)
    n_stab = c["d"] ** 2 - 1
    ms_round = sec * 1e3 * n_stab / n_blocks
    return {"value": ms_round, "unit": "ms/round", "cores": threads, "kind": "oracle",
            "sample": f"{n_blocks} of the {n_stab} noisy stabilizer circuits of round 1 "
                      f"(26 qubits, complex128, gate by gate), {sec:.1f} s, scaled to one round"}


def copy_calibration(qs, torch, steps):
    """Plain copy of a 2^26-amplitude complex128 register (1 GiB read + 1 GiB
    written per launch) with the library's streaming copy kernel."""
    a, b = qs.State(26, "c128"), qs.State(26, "c128")
    b.copy_from(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        b.copy_from(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                      "copy_ms": ms, "copy_gbs": 2 * (1 << 30) / (ms * 1e-3) / 1e9}), flush=True)


def fused_run(qs, torch, reps=10):
    """Dense k-qubit matrices on the 26-qubit register through sv_apply_fused
    (k = 4, 5 run on the matrix cores).  Per call: one read and one write of
    the register, 8 * 4^k flops per group of 2^k amplitudes; time per call
    from HIP events on the state's stream (each call also uploads its
    matrix, 16 KB at most)."""
    import workloads
    out = []
    stream = torch.cuda.current_stream()
    for dt in ("c128", "c64"):
        s = qs.State(26, dt, stream=stream)
        s.set_basis(0)
        for k, qubits in ((5, [20, 21, 22, 23, 24]), (5, [0, 1, 2, 3, 4]), (4, [20, 21, 22, 23])):
            m = workloads.random_matrix(k, 11)
            s.apply_fused(qubits, m)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                s.apply_fused(qubits, m)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            nbytes = 2 * s.nbytes
            flops = 8 * 4 ** k * (1 << (26 - k))
            peak_tf = PEAK_MFMA_TFS[dt]
            out.append({"dtype": dt, "k": k, "qubits": qubits, "ms_per_call": ms,
                        "gbs": nbytes / (ms * 1e-3) / 1e9, "tflops": flops / (ms * 1e-3) / 1e12,
                        "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                        "mfma_frac": flops / (ms * 1e-3) / 1e12 / peak_tf})
        s.free()
    return out


def gate_run(qs, torch, reps=10):
    """One- and two-qubit gates (sv_apply_gate: one strided-pair or
    quadruple pass over the register) on 26 qubits, on low and high qubits;
    per call one read and one write of the register, time from HIP events on
    the state's stream."""
    import workloads
    out = []
    stream = torch.cuda.current_stream()
    for dt in ("c128", "c64"):
        s = qs.State(26, dt, stream=stream)
        s.set_basis(0)
        for qubits in ([0], [25], [0, 1], [12, 25]):
            m = workloads.random_matrix(len(qubits), 3)
            s.apply_gate(qubits, m)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                s.apply_gate(qubits, m)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = 2 * s.nbytes / (ms * 1e-3) / 1e9
            out.append({"dtype": dt, "qubits": qubits, "ms_per_call": ms, "gbs": gbs,
                        "hbm_frac": gbs / PEAK_HBM_GBS})
        s.free()
    return out


def serving_run(qs, kind, window_s, horizon_s, budget_gib=256):
    """Replay a Poisson job stream against the server in real time; at
    `horizon_s` cancel what is left.  Latency = completion - submission on the
    server clock (queueing included)."""
    import numpy as np
    import workloads
    stream = workloads.serving_stream(window_s, seed=2, companion=(kind == "companion"),
                                      n_sites=lambda d: qs.template_info(d, "cr")[1])
    srv = qs.Server(hbm_budget=budget_gib << 30, big_streams=2, max_batch_traj=65536)
    done, t0 = [], time.perf_counter()
    meta = {}
    for arr, job in stream:
        while time.perf_counter() - t0 < arr:
            done += srv.poll()
            time.sleep(0.0005)
        srv.submit(**job)
        meta[job["tag"]] = job
    while time.perf_counter() - t0 < horizon_s and len(done) < len(stream):
        done += srv.poll()
        time.sleep(0.002)
    stats = srv.stats()
    srv.close(cancel=True)
    ok = [c for c in done if c["status"] == 0]
    lat = np.array([c["t_done"] - c["t_submit"] for c in ok]) * 1e3
    traj_rounds = sum(meta[c["tag"]]["n_traj"] * meta[c["tag"]]["rounds"] for c in ok)
    by_d = {d: int(sum(1 for c in ok if meta[c["tag"]]["d"] == d)) for d in (3, 4, 5)}
    return {"stream": kind, "arrival_window_s": window_s, "horizon_s": horizon_s,
            "jobs_offered": len(stream), "jobs_completed": len(ok), "completed_by_d": by_d,
            "backlog_at_horizon": len(stream) - len(ok),
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "trajectory_rounds_per_s": traj_rounds / horizon_s,
            "launches": stats["launches"], "hbm_high_water_gib": stats["hbm_high_water"] / (1 << 30)}


def batch_run(qs, d, n_traj, dtype, seed=7):
    """One batched launch of the small-distance workload shape: rounds uniform
    on 1..9, p uniform on [5e-4, 5e-3), theta uniform on [0, 0.05) per site."""
    import workloads
    n_stab, n_sites, _ = qs.template_info(d, "cr")
    R, p, eps = workloads.batch_params(n_traj, n_sites, seed)
    tuning = tune(qs, d, dtype)          # untimed: launch parameters for this shape
    qs.run_batch(d, "cr", R[:256], p[:256], seed, eps_site=eps[:256], dtype=dtype)
    g = qs.run_batch(d, "cr", R, p, seed, eps_site=eps, dtype=dtype, max_rounds=9)
    amp = 8 if dtype == "c64" else 16
    alg = (int(R.sum()) * n_stab + n_traj) * 2 * (1 << (d * d)) * amp
    return {"d": d, "trajectories": n_traj, "dtype": dtype, "launch_ms": g["gpu_ms"],
            "trajectories_per_s": n_traj / (g["gpu_ms"] * 1e-3),
            "alg_gbs": alg / (g["gpu_ms"] * 1e-3) / 1e9, "tuning": tuning}


def d3_textbook_run(qs):
    """The d=3 workload: 9 data qubits + 1 ancilla, textbook H/CNOT/CZ
    circuit, complex128, 3 rounds of 8 stabilizers, p = 1e-3 after every gate,
    exp(-i 0.02 X) after each H, 1000 trajectories, seed 0 -- one batched
    launch (registers in LDS).  Algorithmic bytes by the per-circuit model:
    one read and one write of the 2^9-amplitude register per circuit, plus
    the initial write and the final read."""
    import numpy as np
    import workloads
    c = workloads.CONFIGS["d3_textbook_c128"]
    d, R, n = c["d"], c["rounds"], c["n_traj"]
    n_stab = qs.template_info(d, "textbook")[0]
    tuning = tune(qs, d, "c128", "textbook")      # untimed
    rounds = np.full(n, R, dtype=np.int32)
    p = np.full(n, c["p"])
    kw = dict(eps=c["eps"], zeta=c["zeta"], dtype="c128", max_rounds=R)
    qs.run_batch(d, "textbook", rounds, p, c["seed"], traj0=10 ** 6, **kw)   # warm-up
    ms = []
    for _ in range(5):
        ms.append(qs.run_batch(d, "textbook", rounds, p, c["seed"], **kw)["gpu_ms"])
    t = float(np.median(ms))
    alg = (R * n_stab + 1) * 2 * (1 << (d * d)) * 16 * n
    return {"workload": "d3_textbook_c128", "trajectories": n, "launch_ms": t,
            "trajectories_per_s": n / (t * 1e-3), "alg_gbs": alg / (t * 1e-3) / 1e9,
            "frac_of_hbm_peak": alg / (t * 1e-3) / 1e9 / PEAK_HBM_GBS, "tuning": tuning}


def precision_run(qs, n_traj, thetas=(0.01, 0.03, 0.05)):
    """Complex64 amplitudes (FP64 probabilities and renormalisation) against
    complex128 on the same draws: d=5 cross-resonance circuit, p=1e-3,
    zeta=0.01, 5 rounds, every site over-rotated by theta (eps = theta/2).
    Infidelity 1 - |<psi64|psi128>|^2 of the register before the final
    measurement, per trajectory."""
    import numpy as np
    from oracle import decoder
    out = []
    for theta in thetas:
        inf, div = [], 0
        recs = {"c64": [], "c128": []}
        fins = {"c64": [], "c128": []}
        for t in range(n_traj):
            st = {}
            for dt in ("c128", "c64"):
                r = qs.run_rounds(5, "cr", 5, 1, seed=1, p=1e-3, eps=theta / 2, zeta=0.01, dtype=dt,
                                  traj0=t, want_states=True)
                st[dt] = r["states"][0]
                recs[dt].append(r["records"][0])
                fins[dt].append(r["final_bits"][0])
            a = st["c64"].astype(np.complex128)
            b = st["c128"]
            inf.append(1.0 - abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))
            div += int(not np.array_equal(recs["c64"][-1], recs["c128"][-1]))
        pl = {dt: decoder.logical_error_rate(5, 0, np.array(recs[dt]), np.array(fins[dt]))[0]
              for dt in recs}
        out.append({"theta": theta, "trajectories": n_traj, "infidelity_max": float(max(inf)),
                    "infidelity_mean": float(np.mean(inf)), "diverged_trajectories": div,
                    "p_L_c64": pl["c64"], "p_L_c128": pl["c128"], "delta_p_L": pl["c64"] - pl["c128"]})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--cpu-blocks", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-only", action="store_true",
                    help="time only the library's plain register copy (HBM calibration)")
    ap.add_argument("--only", choices=["batch", "serving", "precision", "fused", "gates"], default=None,
                    help="run one side measurement alone and print it (for profiling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-launch, serving and precision measurements")
    ap.add_argument("--precision-traj", type=int, default=4,
                    help="trajectories per angle in the complex64 vs complex128 comparison")
    ap.add_argument("--tuning", default=None,
                    help="launch-parameter file: load it instead of autotuning if it exists, "
                         "else autotune and write it (profiled runs then contain no trials)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2204_11404_amd as qs
    import workloads

    torch.cuda.set_device(0)
    global _TUNING_FILE, _TUNING_LOADED
    _TUNING_FILE = args.tuning
    if args.tuning and os.path.exists(args.tuning):
        qs.tuning_load(args.tuning)
        _TUNING_LOADED = True
    if args.copy_only:
        copy_calibration(qs, torch, args.steps)
        return
    if args.only == "batch":
        print(json.dumps({"d3": d3_textbook_run(qs),
                          "batched": [batch_run(qs, 3, 65536, "c64"), batch_run(qs, 4, 4096, "c64")]}))
        return
    if args.only == "fused":
        print(json.dumps({"fused": fused_run(qs, torch)}))
        return
    if args.only == "gates":
        print(json.dumps({"gates": gate_run(qs, torch)}))
        return
    if args.only == "serving":
        print(json.dumps({"serving": [serving_run(qs, "companion", 5.0, 8.0)]}))
        return
    if args.only == "precision":
        print(json.dumps({"precision": precision_run(qs, args.precision_traj)}))
        return
    c = dict(workloads.CONFIGS["d5_cr_c128"])
    d, R = c["d"], c["rounds"]
    n_stab, n_sites, _ = qs.template_info(d, "cr")
    eps = workloads.eps_sites(n_sites, c["theta"], c["seed"])
    kw = dict(d=d, gateset="cr", rounds=R, seed=c["seed"], p=c["p"], eps_site=eps,
              zeta=c["zeta"], dtype=args.dtype)

    tuning = tune(qs, d, args.dtype)   # untimed: launch parameters for this shape
    if args.warmup > 0:
        qs.run_rounds(n_traj=args.warmup, traj0=1_000_000, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = qs.run_rounds(n_traj=args.steps, traj0=0, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    amp_bytes = 16 if args.dtype == "c128" else 8
    blk_bytes = 2 * (1 << (d * d)) * amp_bytes          # read + write of the live register
    rounds_total = args.steps * R
    ms_round = wall * 1e3 / rounds_total
    alg_gbs = n_stab * blk_bytes / (ms_round * 1e-3) / 1e9
    pass_ms = r["pass_ms"]
    achieved = blk_bytes / (pass_ms * 1e-3) / 1e9   # one read + one write per pass
    out = {
        "metric": "d=5 26q QEC round time (ms) + HBM GB/s; d=3 trajectories/s; p99 latency",
        "value": ms_round,
        "unit": "ms/round",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": "d5_cr_c128: rotated surface code d=5, 26 qubits, cross-resonance "
                               "gates, p=1e-3, theta~U[0,0.05) per site, zeta=0.01, 5 rounds",
                   "state": args.dtype, "trajectories_per_step": 1, "rounds": R,
                   "stabilizers_per_round": n_stab},
        # per-circuit byte model (one read + write of the register per
        # stabilizer circuit); exceeds the bytes moved when passes apply chains
        "hbm_gbs_algorithmic": alg_gbs,
        "tuning": tuning,
        "kernel_sources_sha256": kernel_source_hash(),
        "gpu_ms_device": r["gpu_ms"],
        "trajectories_per_s": args.steps / wall,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": counted_traffic(),
                     "kernel": "k_upass", "bytes_per_launch": blk_bytes,
                     "avg_launch_ms": pass_ms,
                     "passes_per_round": r["passes_per_round"],
                     "circuits_per_pass": n_stab / r["passes_per_round"]},
    }
    if not args.no_extras:
        out["d3"] = d3_textbook_run(qs)
        out["d3_trajectories_per_s"] = out["d3"]["trajectories_per_s"]
        out["batched"] = [batch_run(qs, 3, 65536, "c64"), batch_run(qs, 4, 4096, "c64")]
        out["serving"] = [serving_run(qs, "companion", 5.0, 8.0), serving_run(qs, "spec", 2.0, 4.0)]
        out["p99_latency_ms"] = out["serving"][0]["p99_ms"]
        out["precision"] = precision_run(qs, args.precision_traj)
        out["fused"] = fused_run(qs, torch)
        out["gates"] = gate_run(qs, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, eps, args.cpu_blocks)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
