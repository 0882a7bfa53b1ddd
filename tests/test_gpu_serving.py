"""GPU tests of the serving loop (sv_server): continuous batching with
HBM-budget admission.  Each job's records and final bits must be identical
whether the job runs alone (sv_run_rounds) or merged with other jobs in the
server's batched launches and concurrent streams."""
import numpy as np
import pytest

import paper_2204_11404_amd as qs
import workloads

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def _mix():
    """A mixed set of jobs: distances 3/4/5, both dtypes, uneven rounds."""
    rng = np.random.default_rng(8)
    jobs = []
    for tag in range(14):
        d = [3, 3, 4, 3, 4, 3, 5, 3, 4, 3, 3, 4, 3, 3][tag]
        n_stab, n_sites, _ = qs.template_info(d, "cr")
        jobs.append(dict(tag=tag, d=d, gateset="cr", rounds=int(rng.integers(1, 6)),
                         n_traj=2 if d == 5 else int(rng.integers(5, 60)), seed=100 + tag,
                         p=float(rng.uniform(5e-3, 3e-2)),
                         eps_site=rng.uniform(0, 0.05, n_sites) / 2,
                         zeta=0.0, dtype=["c64", "c128"][tag % 2], traj0=int(rng.integers(0, 1000))))
    return jobs


def test_results_same_alone_and_in_mix():
    jobs = _mix()
    srv = qs.Server(hbm_budget=64 * GiB, big_streams=2, max_batch_traj=4096)
    for j in jobs:
        srv.submit(**j)
    srv.wait_idle(300)
    done = {c["tag"]: c for c in srv.poll()}
    st = srv.stats()
    srv.close()
    assert set(done) == {j["tag"] for j in jobs}
    for j in jobs:
        c = done[j["tag"]]
        assert c["status"] == 0
        assert c["t_submit"] <= c["t_admit"] <= c["t_done"]
        alone = qs.run_rounds(j["d"], j["gateset"], j["rounds"], j["n_traj"], j["seed"], j["p"],
                              eps_site=j["eps_site"], zeta=j["zeta"], dtype=j["dtype"],
                              traj0=j["traj0"])
        assert np.array_equal(c["records"], alone["records"]), j["tag"]
        assert np.array_equal(c["final_bits"], alone["final_bits"]), j["tag"]
    # small jobs were merged: fewer launches than jobs
    assert st["launches"] < len(jobs)
    assert st["hbm_in_use"] == 0


def test_admission_respects_budget():
    jobs = _mix()
    budget = 2 * GiB  # about three d=5 complex128 jobs' worth; forces queueing
    srv = qs.Server(hbm_budget=budget, big_streams=2, max_batch_traj=256)
    for j in jobs:
        srv.submit(**j)
    srv.wait_idle(300)
    done = srv.poll()
    st = srv.stats()
    srv.close()
    assert len(done) == len(jobs) and all(c["status"] == 0 for c in done)
    assert 0 < st["hbm_high_water"] <= budget


def test_job_larger_than_budget_is_rejected():
    srv = qs.Server(hbm_budget=64 << 20, big_streams=1)
    with pytest.raises(qs.SvError) as e:
        srv.submit(tag=1, d=5, gateset="cr", rounds=1, n_traj=1, seed=0, p=1e-3)
    assert e.value.status == qs.SV_ENOMEM
    with pytest.raises(qs.SvError) as e:
        srv.submit(tag=2, d=6, gateset="cr", rounds=1, n_traj=1, seed=0, p=1e-3)
    assert e.value.status == qs.SV_EINVAL
    srv.close()


def test_cancel_ends_queued_and_running_jobs():
    srv = qs.Server(hbm_budget=1 * GiB, big_streams=1)
    for tag in range(6):
        srv.submit(tag=tag, d=5, gateset="cr", rounds=5, n_traj=50, seed=tag, p=1e-3, dtype="c64")
    srv.close(cancel=True)  # returns once every job has ended
    # completions were recorded before the server was freed; a closed server
    # has no handle, so check through a fresh one that submission still works
    srv2 = qs.Server(hbm_budget=4 * GiB, big_streams=1)
    srv2.submit(tag=9, d=3, gateset="cr", rounds=2, n_traj=4, seed=1, p=0.01)
    srv2.wait_idle(60)
    assert [c["status"] for c in srv2.poll()] == [0]
    srv2.close()
