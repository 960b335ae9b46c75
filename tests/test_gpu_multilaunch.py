"""Work lists longer than one dispatch are split over several launches.
PS_MAX_GRID_BLOCKS (read once per process) lowers the per-launch cap, so a
child process with a tiny cap takes the multi-launch path on small problems;
its outputs must equal this process's single-launch outputs bit for bit."""

import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import workloads
from psx import announce, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = textwrap.dedent("""
    import sys, numpy as np, torch
    sys.path.insert(0, {root!r})
    import workloads
    from paper_1705_08210_amd import ps
    def dev(V):
        return torch.from_numpy(np.ascontiguousarray(V)).cuda()
    out = {{}}
    Vf = dev(workloads.sparse_uniform(1100, 700, seed=81))
    out["c2"] = ps.ps2(Vf, tile=2)[0]
    out["c2_split"] = ps.ps2(Vf, acc="blocked", tile=2)[0]
    Vg = dev(workloads.sparse_uniform(300, 900, seed=82))
    out["c3"] = ps.ps3(Vg, tile=2)
    Vh = dev(workloads.sparse_uniform(1100, 200, seed=86))   # whole + edge tile launches
    out["c3_edges"] = ps.ps3(Vh, j_begin=400, j_end=430)
    Vl = dev(workloads.levels(1300, 500, seed=83))
    out["mfma"] = ps.ps2(Vl, path="mfma", levels=3)[0]
    out["fp4"] = ps.ps2(Vl, path="mfma_fp4", levels=3)[0]
    Vm = dev(workloads.levels(600, 300, seed=84))
    out["mfma3"] = ps.ps3(Vm, path="mfma", levels=3)
    Vs = [dev(workloads.exponential(n, 400, seed=85 + n)) for n in (700, 90, 1000)]
    for k, (c, _, _) in enumerate(ps.ps2_batched(Vs, acc="plain", tile=2)):
        out[f"b{{k}}"] = c
    torch.cuda.synchronize()
    np.savez({path!r}, **{{k: v.cpu().numpy() for k, v in out.items()}})
""")


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_multi_launch_equals_single_launch(tmp_path):
    path = str(tmp_path / "out.npz")
    announce("multi-launch child process (PS_MAX_GRID_BLOCKS=64)")
    env = dict(os.environ, PS_MAX_GRID_BLOCKS="64")
    r = subprocess.run([sys.executable, "-c", CASES.format(root=ROOT, path=path)], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    child = np.load(path)
    announce("multi-launch: same cases in this process")
    single_path = str(tmp_path / "single.npz")
    exec(CASES.format(root=ROOT, path=single_path), {})
    single = np.load(single_path)
    assert sorted(child.files) == sorted(single.files)
    for k in child.files:
        assert np.array_equal(child[k].view(np.uint32), single[k].view(np.uint32)), k
