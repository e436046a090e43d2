"""The autotuner's search logic on the CPU: its phases, the refine, coarse-sweep
and pass-form modes and the cache it writes, with the device solve replaced by
a stand-in whose time depends on the options in a known way (so the winner is
known in advance).  The GPU side of the tuner is the same solve the parity
tests and the bench run.
"""
import json

import numpy as np
import pytest

import paper_1403_8105_amd.autotune as A


def fake_solver(calls, fused_lr_faster=False):
    def solve_ms(F, st, h, ptrs, phi, stream, o):
        calls.append(dict(o))
        if o["tol"] == 0.0:
            # capped probe (launch shapes, pass forms): time per iteration
            per_it = 1.0 + 0.5 * o.get("fuse_rb", 0) + (-0.2 if fused_lr_faster else 0.1) * \
                o.get("fuse_lr", 0)
            return per_it * o["max_iters"], {"status": 0, "iterations": o["max_iters"],
                                             "rel": 1.0}
        its = 100
        if (o.get("nu_coarse"), o.get("coarse_from")) == (32, 3):
            its -= 40
        if o.get("nu1") == 3 and o.get("nu2") == 3:
            its -= 10
        return float(its), {"status": 0, "iterations": its, "rel": 1e-7,
                            "nested_iterations": 0}
    return solve_ms


@pytest.fixture
def tuner(monkeypatch):
    calls = []
    monkeypatch.setattr(A, "_device_inputs", lambda st, al, q: ([], [1, 2, 3], 4, 0))
    monkeypatch.setattr(A, "device_arch", lambda device=0: "gfx950")
    return calls


def medium(n=8):
    z = np.zeros((n, n, n))
    return z, z, z, 0.1


def test_full_search_with_coarse_sweeps_and_pass_forms(tuner, monkeypatch, tmp_path):
    monkeypatch.setattr(A, "_solve_ms", fake_solver(tuner))
    path = str(tmp_path / "cache.json")
    st, al, q, h = medium()
    entry = A.tune(st, al, q, h, path=path, log=lambda m: None, coarse=True)
    o = entry["options"]
    # the known optimum: V(3,3), 32 sweeps from level 3, separate passes
    assert (o["nu1"], o["nu2"], o["nu_coarse"], o["coarse_from"]) == (3, 3, 32, 3)
    assert "fuse_rb" not in o and "fuse_lr" not in o
    assert entry["iterations"] == 50
    assert set(entry["pass_ms_per_iteration"]) == {"0,0", "1,0", "0,1", "1,1"}
    # every coarse-sweep candidate was tried, and the pass forms ran capped
    tried = {(c.get("nu_coarse"), c.get("coarse_from")) for c in tuner if c["tol"] > 0}
    assert set(A.COARSE_SWEEPS) <= tried
    assert any(c["tol"] == 0.0 and c.get("fuse_rb") == 1 for c in tuner)
    # the cache holds the entry under the grid's key
    cache = json.load(open(path))
    assert cache[A.cache_key("gfx950", st.shape, "mixed", "lp")]["options"] == o


def test_passes_only_keeps_the_schedule(tuner, monkeypatch, tmp_path):
    path = str(tmp_path / "cache.json")
    st, al, q, h = medium()
    key = A.cache_key("gfx950", st.shape, "mixed", "lp")
    opts = {"nu1": 4, "nu2": 4, "omega_s": 1.15, "restart_growth": 2.0, "corr_scale": 2.0,
            "task_cells0": 8192, "coarse_blocks": 2048, "aa_m": 8}
    json.dump({key: {"options": opts, "ms_to_tol": 1.0, "iterations": 7}}, open(path, "w"))
    monkeypatch.setattr(A, "_solve_ms", fake_solver(tuner, fused_lr_faster=True))
    entry = A.tune(st, al, q, h, path=path, log=lambda m: None, passes_only=True)
    assert entry["options"] == dict(opts, fuse_lr=1)
    assert all(c["tol"] == 0.0 for c in tuner) and len(tuner) == 2 * len(A.PASSES)
    assert json.load(open(path))[key]["options"] == dict(opts, fuse_lr=1)


def test_refine_coarse_starts_from_the_cached_entry(tuner, monkeypatch, tmp_path):
    path = str(tmp_path / "cache.json")
    st, al, q, h = medium()
    key = A.cache_key("gfx950", st.shape, "mixed", "lp")
    opts = {"nu1": 2, "nu2": 2, "omega_s": 1.15, "restart_growth": 2.0, "corr_scale": 2.0,
            "task_cells0": 4096, "coarse_blocks": 2048, "aa_m": 8, "nested_tol": 0.1}
    json.dump({key: {"options": opts, "ms_to_tol": 1.0, "iterations": 7,
                     "shape_ms_per_iteration": {"4096,2048": 1.0}}}, open(path, "w"))
    monkeypatch.setattr(A, "_solve_ms", fake_solver(tuner))
    entry = A.tune(st, al, q, h, path=path, log=lambda m: None, refine=True, coarse=True)
    o = entry["options"]
    assert (o["nu_coarse"], o["coarse_from"], o["nu1"], o["nu2"]) == (32, 3, 3, 3)
    assert o["aa_m"] == 8 and o["nested_tol"] == 0.1
    full = [c for c in tuner if c["tol"] > 0]
    # the cached entry once, the coarse candidates, the sweeps above them, the
    # windows again; no launch-shape probes and no schedule search
    assert full[0]["nu_coarse"] == 0 and full[0]["nu1"] == 2
    assert len(full) == 1 + len(A.COARSE_SWEEPS) + (len(A.FINE_SWEEPS) - 1) + \
        (len(A.AA_WINDOWS) - 1)
