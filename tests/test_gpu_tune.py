"""The tuner (autotune.py) on tiny shapes: it times every alternative through
the C ABI, registers its choices (VALU tile configurations, the AUTO path for
integer levels, the int8 matrix-core tile order), and the library's own
choices then keep parity with the oracle.  The packaged cache is registered
again afterwards."""

import numpy as np
import pytest

import oracle
import workloads
from psx import announce, check_exact_f32, check_rel, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_quick_tune_registers_choices_that_keep_parity(monkeypatch):
    import torch
    from paper_1705_08210_amd import autotune, ps
    # one tiny representative shape per way, in the first n_f and n_v buckets
    monkeypatch.setattr(autotune, "REPS", {2: {(0, 0): (700, 300)}, 3: {(0, 0): (600, 140)}})
    monkeypatch.setattr(autotune, "PATH_REPS", {2: {(0, 0): (900, 400)},
                                                3: {(0, 0): (700, 150)}})
    announce("tune quick tiny")
    try:
        cache = autotune.tune(dtypes=("f32", "u8"), ways=(2, 3, 0), reps=1, log=lambda m: None,
                              batch_count=3)
        kinds = {(e["dtype"], e["way"], e["path"]) for e in cache["entries"]}
        assert {("f32", 2, "valu"), ("f32", 3, "valu"), ("f32", 0, "valu"), ("u8", 2, "auto"),
                ("u8", 3, "auto"), ("u8", 2, "mfma")} <= kinds
        for e in cache["entries"]:
            assert len(e["ms"]) >= 2 and all(t > 0 for t in e["ms"])
            assert e["tile"] == int(np.argmin(e["ms"])) or e["path"] == "auto"
        # the library now runs the registered choices (opts.tile = 0, AUTO)
        V = workloads.sparse_uniform(300, 700, seed=91)
        c2, _ = ps.ps2(to_dev(V))
        check_rel(host(c2), oracle.c2_all(V), 1e-5, "f32 2-way, tuned tile")
        V3 = workloads.sparse_uniform(140, 600, seed=92)
        check_rel(host(ps.ps3(to_dev(V3))), oracle.c3_all(V3), 1e-5, "f32 3-way, tuned tile")
        U = workloads.levels(400, 900, seed=93)
        c2u, _ = ps.ps2(to_dev(U), levels=3)
        check_exact_f32(host(c2u), oracle.c2_all(U), "u8 2-way, tuned path")
        U3 = workloads.levels(150, 700, seed=94)
        check_exact_f32(host(ps.ps3(to_dev(U3), levels=3)), oracle.c3_all(U3),
                        "u8 3-way, tuned path")
        # every matrix-core tile order gives the same bits
        Ud = to_dev(U)
        outs = []
        for idx in range(len(ps.tile_configs(torch.uint8, 2, "mfma"))):
            ps.tune_clear()
            ps.tune_register(torch.uint8, 2, "mfma", (0, 1 << 40), (0, 1 << 40), idx)
            outs.append(host(ps.ps2(Ud, path="mfma", levels=3)[0]))
        for o in outs[1:]:
            assert np.array_equal(o.view(np.uint32), outs[0].view(np.uint32))
    finally:
        ps.tune_clear()
        autotune.load()
