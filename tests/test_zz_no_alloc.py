"""sv_run_batch_noalloc (every device buffer in the library's static scratch
array) against sv_run_batch on the same jobs, through the C ABI: two calls in
a row, the second smaller, so stale contents of the first call's records and
tables would show; plus the size limit and the d = 4 refusal."""
import numpy as np
import pytest

import paper_2204_11404_amd as qs
import workloads

pytestmark = pytest.mark.gpu


def _job(d, gateset, n, seed):
    n_sites = qs.template_info(d, gateset)[1]
    R, p, eps = workloads.batch_params(n, n_sites, seed, p=(5e-3, 5e-2))
    return R, p, eps


@pytest.mark.parametrize("d,gateset,dtype", [(3, "cr", "c64"), (3, "textbook", "c128"), (2, "cr", "c128")])
def test_no_alloc_matches_run_batch_twice(d, gateset, dtype):
    for n, seed in ((3000, 71), (700, 72)):  # the second call is smaller
        R, p, eps = _job(d, gateset, n, seed)
        print(f"case no-alloc d={d} {gateset} {dtype} n={n}", flush=True)
        a = qs.run_batch(d, gateset, R, p, seed, eps_site=eps, zeta=0.01, dtype=dtype, max_rounds=9,
                         traj0=5, no_alloc=True)
        b = qs.run_batch(d, gateset, R, p, seed, eps_site=eps, zeta=0.01, dtype=dtype, max_rounds=9,
                         traj0=5)
        assert np.array_equal(a["records"], b["records"])
        assert np.array_equal(a["final_bits"], b["final_bits"])
        assert a["gpu_ms"] > 0


def test_no_alloc_common_angles_then_per_site():
    """One angle for the launch (the shared-table buffer is used), then per-site
    angles with fewer trajectories."""
    n = 500
    R = np.full(n, 3, dtype=np.int32)
    p = np.full(n, 0.02)
    a = qs.run_batch(3, "cr", R, p, 9, eps=0.02, dtype="c64", no_alloc=True)
    b = qs.run_batch(3, "cr", R, p, 9, eps=0.02, dtype="c64")
    assert np.array_equal(a["records"], b["records"]) and np.array_equal(a["final_bits"], b["final_bits"])
    R2, p2, eps2 = _job(3, "cr", 200, 10)
    a = qs.run_batch(3, "cr", R2, p2, 10, eps_site=eps2, dtype="c64", no_alloc=True)
    b = qs.run_batch(3, "cr", R2, p2, 10, eps_site=eps2, dtype="c64")
    assert np.array_equal(a["records"], b["records"]) and np.array_equal(a["final_bits"], b["final_bits"])


def test_no_alloc_limits():
    with pytest.raises(qs.SvError) as e:
        qs.run_batch(4, "cr", [2], [0.01], 0, no_alloc=True)
    assert e.value.status == qs.SV_EINVAL
    # 9 rounds and 56 per-site angles take about 560 B per trajectory: 200 000
    # trajectories need more than the 64 MiB scratch
    R, p, eps = _job(3, "cr", 200000, 73)
    with pytest.raises(qs.SvError) as e:
        qs.run_batch(3, "cr", R, p, 73, eps_site=eps, dtype="c64", max_rounds=9, no_alloc=True)
    assert e.value.status == qs.SV_ENOMEM
    # the scratch still works after the refusal
    R, p, eps = _job(3, "cr", 100, 74)
    a = qs.run_batch(3, "cr", R, p, 74, eps_site=eps, dtype="c64", max_rounds=9, no_alloc=True)
    b = qs.run_batch(3, "cr", R, p, 74, eps_site=eps, dtype="c64", max_rounds=9)
    assert np.array_equal(a["records"], b["records"])
