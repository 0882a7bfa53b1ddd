"""Launch-parameter table and autotuner (sv_tuning_*, sv_autotune).

The CPU tests check the host side (defaults, validation, set/get, save/load);
the GPU tests run the autotuner and check that a tuned configuration computes
the same records as the oracle."""
import os

import numpy as np
import pytest

import oracle
import paper_2204_11404_amd as qs
import workloads

FIELDS = {"zchain", "snake", "batch_waves_per_cu", "lockstep_mib", "pass_wgs_per_cu", "xpair"}
ENV = ("QECSV_ZCHAIN", "QECSV_SNAKE", "QECSV_BATCH_WAVES_PER_CU", "QECSV_LOCKSTEP_MIB",
       "QECSV_PASS_WGS_PER_CU", "QECSV_XPAIR")


@pytest.fixture(autouse=True)
def _restore_tuning():
    saved = {(d, dt): qs.tuning_get(d, dt) for d in (2, 3, 4, 5) for dt in ("c64", "c128")}
    yield
    for (d, dt), t in saved.items():
        qs.tuning_set(d, dt, **t)


def test_defaults_and_roundtrip(monkeypatch):
    for var in ENV:
        monkeypatch.delenv(var, raising=False)
    t = qs.tuning_get(5, "c128")
    assert set(t) == FIELDS and 1 <= t["zchain"] <= 4 and t["xpair"] == 0
    qs.tuning_set(5, "c128", zchain=2, snake=0)
    assert qs.tuning_get(5, "c128")["zchain"] == 2
    assert qs.tuning_get(5, "c128")["snake"] == 0
    assert qs.tuning_get(5, "c64")["zchain"] == t["zchain"]   # per dtype


def test_environment_overrides(monkeypatch):
    qs.tuning_set(4, "c64", zchain=4, xpair=0)
    monkeypatch.setenv("QECSV_ZCHAIN", "1")
    monkeypatch.setenv("QECSV_XPAIR", "1")
    assert qs.tuning_get(4, "c64")["zchain"] == 1
    assert qs.tuning_get(4, "c64")["xpair"] == 1


@pytest.mark.parametrize("bad", [dict(zchain=0), dict(zchain=7), dict(snake=2),
                                 dict(batch_waves_per_cu=0), dict(batch_waves_per_cu=33),
                                 dict(lockstep_mib=0), dict(pass_wgs_per_cu=-1),
                                 dict(pass_wgs_per_cu=65), dict(xpair=2), dict(xpair=-1)])
def test_rejects_out_of_range(bad):
    with pytest.raises(qs.SvError):
        qs.tuning_set(3, "c64", **bad)
    with pytest.raises(qs.SvError):
        qs.tuning_get(6, "c64")


def test_save_load(tmp_path, monkeypatch):
    for var in ENV:
        monkeypatch.delenv(var, raising=False)
    qs.tuning_set(4, "c128", zchain=3, lockstep_mib=1024, xpair=1)
    path = str(tmp_path / "tune.txt")
    qs.tuning_save(path)
    qs.tuning_set(4, "c128", zchain=4, lockstep_mib=4096, xpair=0)
    qs.tuning_load(path)
    t = qs.tuning_get(4, "c128")
    assert t["zchain"] == 3 and t["lockstep_mib"] == 1024 and t["xpair"] == 1
    # a file written before the xpair field (eight fields a line) still loads
    old = str(tmp_path / "old.txt")
    with open(path) as f, open(old, "w") as g:
        for line in f:
            g.write(" ".join(line.split()[:8]) + "\n")
    qs.tuning_load(old)
    assert qs.tuning_get(4, "c128")["xpair"] == 0
    with open(path, "a") as f:
        f.write("garbage line\n")
    with pytest.raises(qs.SvError):
        qs.tuning_load(path)
    with pytest.raises(qs.SvError):
        qs.tuning_load(str(tmp_path / "missing.txt"))


@pytest.mark.gpu
@pytest.mark.parametrize("d,dtype", [(3, "c64"), (4, "c64"), (5, "c128")])
def test_autotune_then_parity(d, dtype, monkeypatch):
    for var in ENV:
        monkeypatch.delenv(var, raising=False)
    print(f"case autotune d={d} {dtype}", flush=True)
    best, ms = qs.autotune(d, dtype)
    assert ms > 0.0
    assert qs.tuning_get(d, dtype) == best
    assert best["xpair"] in (0, 1)
    if d == 5:
        assert best["zchain"] in (2, 3, 4, 5, 6) and best["snake"] in (0, 1)
        assert best["pass_wgs_per_cu"] in (0, 3, 4, 6, 8, 12, 16)
        return
    if d == 4:
        assert best["lockstep_mib"] in (256, 1024, 4096)
    else:
        assert best["batch_waves_per_cu"] in (2, 4, 8, 12, 16)
    n_stab, n_sites, _ = qs.template_info(d, "cr")
    n = 6
    R, p, eps = workloads.batch_params(n, n_sites, 9, p=(5e-3, 3e-2))
    g = qs.run_batch(d, "cr", R, p, 9, eps_site=eps, dtype=dtype, max_rounds=9)
    for i in range(n):
        o = oracle.run_trajectory(d, oracle.GATESET_CR, int(R[i]), 9, i, p[i], eps_site=eps[i])
        assert np.array_equal(g["records"][i, :R[i]], o["records"])
        assert np.array_equal(g["final_bits"][i], o["final_bits"])
