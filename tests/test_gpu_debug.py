"""Debug checks (environment variable SE2_DEBUG): the same solves with every job table checked
on the host and every launch synchronised give bitwise the same results as without."""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# A pruned OT solve through the queue (two solves, two lanes' worth of launches), a blocking
# pruned solve, a barycenter, and an FP32 matrix-core solve; the outputs go to one .npz file.
SCRIPT = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[2])
from paper_2402_15322_amd import native, synth
native.se2_init()
out = {}
g = synth.Grid(24, 24, 16)
k = native.Kernel(24, 24, 16, False, (1.0, 3.0, 1.0), 0.2, 5)
pairs = []
for i in range(2):
    r = synth.rng_for(9600 + i, 0)
    segs = synth.draw_segments(r, g, 3, 3.0, 8.0)
    mu = synth.splat_segments(g, segs, 1.0, 1e-6)
    nu = synth.splat_segments(g, synth.moved_segments(r, g, segs, 1.0, 0.1), 1.0, 1e-6)
    pairs.append((torch.from_numpy(mu).cuda(), torch.from_numpy(nu).cuda()))
o = native.opts(tol=-1, max_iter=60, check_every=10)
q = native.SolveQueue(hbm_budget_bytes=256 << 20, max_slots=4)
res = []
for mu, nu in pairs:
    f, gg = torch.empty_like(mu), torch.empty_like(mu)
    res.append((q.submit_ot(k, mu, nu, o, f, gg), f, gg))
for i, (t, f, gg) in enumerate(res):
    rep = q.wait(t)
    out[f"q{i}_f"] = f.cpu().numpy(); out[f"q{i}_g"] = gg.cpu().numpy(); out[f"q{i}_err"] = np.array(rep["marg_l1"])
q.close()
mu, nu = pairs[0]
f, gg = torch.empty_like(mu), torch.empty_like(mu)
rep = native.se2_sinkhorn(k, mu, nu, o, f, gg)
out["b_f"] = f.cpu().numpy(); out["b_cost"] = np.array(rep["cost"])
f2, g2 = torch.empty_like(mu), torch.empty_like(mu)
rep = native.se2_sinkhorn(k, mu, nu, native.opts(tol=-1, max_iter=30, check_every=10, prec=native.SE2_F32_MFMA), f2, g2)
out["m_f"] = f2.cpu().numpy(); out["m_fb"] = np.array(rep["fallbacks"])
kb = native.Kernel(24, 24, 16, False, (1.0, 2.0, 1.0), 0.5, 4)
b = torch.empty_like(mu)
native.se2_barycenter(kb, [mu, nu], [0.5, 0.5], native.opts(tol=-1, max_iter=20, check_every=10), b)
out["bar"] = b.cpu().numpy()
np.savez(sys.argv[1], **out)
print("done", flush=True)
"""


def _run(tmp_path, debug: bool):
    path = str(tmp_path / ("debug.npz" if debug else "plain.npz"))
    env = dict(os.environ)
    env.pop("SE2_DEBUG", None)
    if debug:
        env["SE2_DEBUG"] = "1"
    r = subprocess.run([sys.executable, "-c", SCRIPT, path, ROOT], env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    return np.load(path)


def test_debug_checks_leave_results_unchanged(tmp_path):
    plain = _run(tmp_path, False)
    dbg = _run(tmp_path, True)
    assert sorted(plain.files) == sorted(dbg.files)
    for name in plain.files:
        assert np.array_equal(plain[name], dbg[name]), name
