"""Autotuned tiles through the persistent cache on the GPU: a solve with the
tuning table filled by mg_autotune (cold) and one with the table read back
from the cache file (hot) pick the same tiles and give bit-identical results;
a fresh process given MACPROJ_TUNE_CACHE finds the entries for this GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_1910_12979_amd import inputs as I

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _solve(mp, prob, d0):
    d = mp.to_device(prob)
    H = mp.Hierarchy(mp.params_of(prob))
    st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)
    torch.cuda.synchronize()
    tiles = [H.sweep_config(l) for l in range(H.nlevels)]
    H.close()
    return st, {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}, tiles


def test_tuned_tiles_cold_and_hot(mp, tmp_path):
    path = str(tmp_path / "tune.json")
    prob = I.make_problem((128, 96, 64), H=0.15, seed=21)
    mp.tune_cache_clear()
    try:
        st0, out0, tiles0 = _solve(mp, prob, None)                 # per-shape defaults
        d = mp.to_device(prob)
        H = mp.Hierarchy(mp.params_of(prob))
        H.set_coefficients(d.rho, d.beta0_cc, d.beta0_edge)
        H.mg_autotune(reps=3)
        H.close()
        st1, out1, tiles1 = _solve(mp, prob, None)                 # cold: tuned in this process
        n = mp.tune_cache_save(path)
        assert n >= 1
        mp.tune_cache_clear()
        assert mp.tune_cache_load(path) == n
        st2, out2, tiles2 = _solve(mp, prob, None)                 # hot: read back from the file
        print("default tiles", tiles0, "tuned", tiles1)
        assert tiles2 == tiles1
        assert st2["cycles"] == st1["cycles"] and st2["rel_resid"] == st1["rel_resid"]
        for k in ("phi", "u", "v", "w"):
            assert np.array_equal(out2[k], out1[k]), k
        # the tiles do not change the per-cell arithmetic: the same cycles
        # give the same fields as the untuned solve
        assert st1["cycles"] == st0["cycles"]
        for k in ("phi", "u", "v", "w"):
            assert np.array_equal(out1[k], out0[k]), k
        # a fresh process reads the file named by MACPROJ_TUNE_CACHE
        nx, ny, nz = prob.n
        code = ("import sys; sys.path.insert(0, %r)\n"
                "import torch; torch.cuda.set_device(0)\n"
                "from paper_1910_12979_amd import macproj as M\n"
                "print(M.tune_lookup((%d, %d, %d), rho=True, fp64=True))\n") % (ROOT, nx, ny, nz)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           env=dict(os.environ, MACPROJ_TUNE_CACHE=path), timeout=300)
        assert r.returncode == 0, r.stderr
        assert int(r.stdout.strip().splitlines()[-1]) == tiles1[0][3]
    finally:
        mp.tune_cache_clear()
