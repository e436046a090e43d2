"""Auxiliary subsystems: the tuner-cache override (CPU), failure injection
and the per-iteration log (GPU)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from synth import media

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tune_cache_override(tmp_path):
    # FLD_TUNE_CACHE names the cache that tuned_options reads
    path = tmp_path / "cache.json"
    key = "gfx950|16x16x16|mixed|lp"
    path.write_text(json.dumps({key: {"options": {"nu1": 3, "nu2": 1, "aa_m": 5}},
                                key + "|tol=1e-10": {"options": {"nu1": 1}}}))
    code = ("import json, paper_1403_8105_amd.autotune as A; "
            "print(json.dumps([A.CACHE, A.tuned_options((16, 16, 16), 'mixed', 'lp', arch='gfx950'), "
            "A.tuned_options((16, 16, 16), 'mixed', 'lp', arch='gfx950', tol=1e-10), "
            "A.tuned_options((16, 16, 16), 'mixed', 'lp', arch='gfx950', tol=1e-8), "
            "A.tuned_options((8, 8, 8), 'mixed', 'lp', arch='gfx950')]))")
    env = dict(os.environ, FLD_TUNE_CACHE=str(path))
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                         text=True, check=True).stdout
    cache, opts, tight, other_tol, missing = json.loads(out.strip().splitlines()[-1])
    assert cache == str(path)
    assert opts == {"nu1": 3, "nu2": 1, "aa_m": 5}
    assert tight == {"nu1": 1}            # the entry tuned for that tolerance
    assert other_tol == opts              # no such entry: the grid's own
    assert missing == {}


@pytest.mark.gpu
@pytest.mark.parametrize("kw", [dict(), dict(precision="mixed", aa_m=4), dict(graph=0)])
def test_nan_injection_ends_in_divergence(kw):
    F = pytest.importorskip("paper_1403_8105_amd")
    st, al, Q, h = media.config("cloud128", n=16)
    s = F.Solver(st.shape, h, tol=0.0, max_iters=50, debug_nan_iter=3, **kw)
    s.set_medium(st, al, Q)
    phi, rep = s.solve(allow=(F.FLD_ERR_DIVERGED,))
    s.close()
    assert rep["status"] == F.FLD_ERR_DIVERGED
    hist = rep["history"]
    # iterations 0..3 have finite residuals, the one after the injection not
    assert len(hist) == 5 and np.all(np.isfinite(hist[:4])) and not np.isfinite(hist[4])


@pytest.mark.gpu
def test_per_iteration_log():
    F = pytest.importorskip("paper_1403_8105_amd")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1403_8105_amd as F\n"
            "from synth import media\n"
            "st, al, Q, h = media.config('cloud128', n=16)\n"
            "s = F.Solver(st.shape, h, tol=0.0, max_iters=6)\n"
            "s.set_medium(st, al, Q)\n"
            "phi, rep = s.solve()\n"
            "print('HIST', list(rep['history']))\n") % ROOT
    env = dict(os.environ, FLD_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, check=True, timeout=120)
    lines = [json.loads(l) for l in r.stderr.splitlines() if l.startswith('{"fld_iteration"')]
    hist = eval(r.stdout.strip().splitlines()[-1][5:])
    assert [l["fld_iteration"] for l in lines] == list(range(7))
    np.testing.assert_array_equal([l["rel"] for l in lines], hist)
