"""Host timing of the oracle for the benchmark's CPU baseline.

TEST INFRASTRUCTURE ONLY: the benchmark's cpu_baseline leg runs this module
(in a child process, so that the oracle's OpenMP loops are single-threaded and
the parallelism is over trajectories); nothing in the product library uses
it.  Prints one JSON object.

  python -m oracle.timing d3 --threads N   the d=3 textbook workload: 9 data
      qubits + 1 ancilla, H/CNOT/CZ circuits, 3 rounds, p = 1e-3 after every
      gate, exp(-i 0.02 X) after each H, 1000 trajectories, seed 0;
  python -m oracle.timing d4 --threads N   64 trajectories of the batched d=4
      workload (cross-resonance circuit, rounds uniform on 1..9, p uniform on
      [5e-4, 5e-3), theta uniform on [0, 0.05) per site and trajectory).
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _run(jobs, threads):
    """Wall time of the trajectories `jobs` (keyword dicts of run_trajectory)
    on `threads` host threads (the oracle releases the interpreter lock)."""
    import oracle
    t0 = time.perf_counter()
    if threads == 1:
        for j in jobs:
            oracle.run_trajectory(**j)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda j: oracle.run_trajectory(**j), jobs))
    return time.perf_counter() - t0


def d3_jobs():
    import oracle
    import workloads
    c = workloads.CONFIGS["d3_textbook_c128"]
    return [dict(d=c["d"], gateset=oracle.GATESET_TEXTBOOK, rounds=c["rounds"], seed=c["seed"], t=t,
                 p=c["p"], eps=c["eps"]) for t in range(c["n_traj"])]


def d4_jobs(n=64, seed=7):
    import oracle
    import workloads
    n_sites = oracle.template_counts(4, oracle.GATESET_CR)[1]
    R, p, eps = workloads.batch_params(n, n_sites, seed)
    return [dict(d=4, gateset=oracle.GATESET_CR, rounds=int(R[i]), seed=seed, t=i, p=float(p[i]),
                 eps_site=eps[i]) for i in range(n)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["d3", "d4"])
    ap.add_argument("--threads", type=int, default=1)
    a = ap.parse_args()
    import oracle
    oracle.set_threads(1)
    jobs = d3_jobs() if a.workload == "d3" else d4_jobs()
    sec = _run(jobs, a.threads)
    print(json.dumps({"workload": a.workload, "trajectories": len(jobs), "seconds": sec,
                      "trajectories_per_s": len(jobs) / sec, "threads": a.threads,
                      "trajectory_rounds": int(sum(j["rounds"] for j in jobs))}))


if __name__ == "__main__":
    main()
