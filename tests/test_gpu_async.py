"""sv_run_rounds_async: two runs enqueued on two streams overlap on the
device and give the results of the synchronous sv_run_rounds (the paper's
workload is many independent trajectories, Sec. III.B)."""
import numpy as np
import pytest

import paper_2204_11404_amd as qs
import workloads

pytestmark = pytest.mark.gpu


def _jobs():
    n5 = qs.template_info(5, "cr")[1]
    n4 = qs.template_info(4, "cr")[1]
    a = dict(d=5, gateset="cr", rounds=3, n_traj=1, seed=4, p=5e-3,
             eps_site=workloads.eps_sites(n5, (0.0, 0.05), 4), zeta=0.01, dtype="c128", want_p1=True)
    b = dict(d=4, gateset="cr", rounds=2, n_traj=6, seed=5, p=1e-2,
             eps_site=workloads.eps_sites(n4, (0.0, 0.05), 5), zeta=0.01, dtype="c64", want_p1=True)
    return a, b


def test_two_streams_match_synchronous_runs(monkeypatch):
    import torch
    # enqueued runs use the plain passes (no speculative units), so does the
    # synchronous reference here
    monkeypatch.setenv("QECSV_SPEC", "0")
    a, b = _jobs()
    ref_a = qs.run_rounds(**a)
    ref_b = qs.run_rounds(**b)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ra = qs.run_rounds_async(stream=sa, **a)
    # three d=5 rounds (45 register passes of 1 GiB) are still running when
    # the call returns: the run was enqueued, not waited for
    still_running = not ra.done()
    rb = qs.run_rounds_async(stream=sb, **b)
    ga, gb = ra.wait(), rb.wait()
    print(f"d=5 run still in flight after the call returned: {still_running}", flush=True)
    assert still_running
    for g, ref in ((ga, ref_a), (gb, ref_b)):
        assert np.array_equal(g["records"], ref["records"])
        assert np.array_equal(g["final_bits"], ref["final_bits"])
        assert np.array_equal(g["p1"], ref["p1"])
        assert g["passes_per_round"] == ref["passes_per_round"]


def test_async_rejects_graph_and_states():
    import torch
    s = torch.cuda.Stream()
    with pytest.raises(qs.SvError):
        job, keep, _ = qs._rounds_job(3, "cr", 1, 1, 0, 0.01, 0.0, None, 0.0, "c128", 0, s, True,
                                      False, False, False, False, False)
        res = qs.Result()
        rec = np.zeros(8, np.uint8)
        fb = np.zeros(9, np.uint8)
        res.records = rec.ctypes.data_as(qs.ctypes.POINTER(qs.ctypes.c_uint8))
        res.final_bits = fb.ctypes.data_as(qs.ctypes.POINTER(qs.ctypes.c_uint8))
        ev = torch.cuda.Event()
        ev.record(s)
        qs._check(qs.lib().sv_run_rounds_async(qs.ctypes.byref(job), qs.ctypes.byref(res),
                                                qs.ctypes.c_void_p(ev.cuda_event)))


def test_async_zero_trajectories_records_the_event():
    import torch
    s = torch.cuda.Stream()
    r = qs.run_rounds_async(3, "cr", 2, 0, 0, 0.01, stream=s)
    g = r.wait()
    assert g["records"].shape == (0, 2, 8)


def test_async_speculative_runs_match_synchronous(monkeypatch):
    """Without the data ZZ layer both the enqueued and the synchronous runs
    use speculative units (predicted outcomes, redone when they fail): the
    same records, final bits and p1 bit for bit."""
    import torch
    monkeypatch.delenv("QECSV_SPEC", raising=False)
    n4 = qs.template_info(4, "cr")[1]
    kw = dict(d=4, gateset="cr", rounds=3, n_traj=5, seed=9, p=5e-3,
              eps_site=workloads.eps_sites(n4, (0.0, 0.05), 9), zeta=0.0, dtype="c128", want_p1=True)
    ref = qs.run_rounds(**kw)
    s = torch.cuda.Stream()
    r = qs.run_rounds_async(stream=s, **kw)
    g = r.wait()
    assert g["passes_per_round"] == ref["passes_per_round"] < 10
    assert np.array_equal(g["records"], ref["records"])
    assert np.array_equal(g["final_bits"], ref["final_bits"])
    assert np.array_equal(g["p1"], ref["p1"])
