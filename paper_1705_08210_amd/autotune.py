"""Tuner of the library's launch choices.

Times the alternatives through the C ABI on seeded synthetic inputs of
representative shapes and keeps the fastest per (storage type, way, n_f
bucket, n_v bucket) in a JSON cache:
  - the VALU tile configuration (``ps_tile_config``) of 2-way, 3-way and
    batched launches (entries with path "valu");
  - the path AUTO takes for integer levels (VALU, int8 or fp4 matrix cores;
    path "auto", the entry's "tile" is the chosen ps_path code);
  - the tile order of the 2-way int8 matrix-core kernel: block columns
    walked in groups of 2^idx (path "mfma").
``load()`` registers a cache with the library (``ps_tune_register``), after
which the library's own choices (``opts.tile = 0``, ``opts.path = AUTO``)
follow it.  Runs off the timed path.

    python -m paper_1705_08210_amd.autotune [--quick] [--out FILE]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import ps

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

# bucket edges: [lo, hi)
NF_BUCKETS = [(0, 2048), (2048, 8192), (8192, 1 << 40)]
NV_BUCKETS = [(0, 1024), (1024, 4096), (4096, 1 << 40)]
# representative shapes per bucket (n_f, n_v) -- a tile choice depends on
# how many tiles fill the chip and on the depth of the field loop
REPS = {
    2: {(0, 0): (1024, 512), (0, 1): (1024, 2048), (0, 2): (1024, 8192),
        (1, 0): (4096, 512), (1, 1): (4096, 2048), (1, 2): (4096, 8192),
        (2, 0): (16384, 512), (2, 1): (16384, 2048), (2, 2): (16384, 8192)},
    3: {(0, 0): (1024, 256), (1, 0): (4096, 384), (2, 0): (12000, 256),
        (0, 1): (1024, 1024), (1, 1): (4096, 1024), (2, 1): (12000, 1024)},
}
# integer-level shapes for the path and matrix-core tile-order choices
PATH_REPS = {
    2: {(1, 0): (4096, 512), (1, 1): (4096, 2048), (1, 2): (8192, 8192),
        (2, 1): (16384, 2048)},
    3: {(1, 0): (4096, 384), (0, 1): (1024, 1024), (1, 1): (4096, 1024)},
}
LEVELS = 3
DTYPES = {"f32": torch.float32, "f16": torch.float16, "u8": torch.uint8}
PATH_CODES = {"valu": 1, "mfma": 2, "mfma_fp4": 3}


def _input(n_v, n_f, dt, seed=0):
    g = torch.Generator(device="cuda").manual_seed(seed)
    if dt == torch.uint8:
        return torch.randint(0, 4, (n_v, n_f), device="cuda", dtype=torch.uint8, generator=g)
    x = torch.rand((n_v, n_f), device="cuda", generator=g)
    x = torch.where(torch.rand((n_v, n_f), device="cuda", generator=g) < 0.5, 0.0, x)
    return x.to(dt)


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = math.inf
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def _entry(dname, way, path, fb, vb, shape, idx, times):
    return {"dtype": dname, "way": way, "path": path, "nf": list(NF_BUCKETS[fb]),
            "nv": list(NV_BUCKETS[vb]), "shape": list(shape), "tile": idx,
            "ms": [round(t, 4) for t in times]}


def tune_paths(ways=(2, 3), reps=3, quick=False, log=print):
    """For uint8 levels (0..3): the fastest of the VALU, int8 and fp4
    matrix-core paths per bucket (the choice AUTO then takes), and for the
    2-way int8 kernel the fastest tile order."""
    out = []
    dt = torch.uint8
    for way in ways:
        for (fb, vb), (n_f, n_v) in PATH_REPS[way].items():
            if quick and (fb, vb) not in ((1, 1), (1, 0)):
                continue
            V = _input(n_v, n_f, dt)
            s, _ = ps.vector_sums(V, want_bad=False)
            if way == 2:
                c2 = torch.empty(n_v * (n_v - 1) // 2, device="cuda")
                run = (lambda p: ps.ps2(V, s=s, c2=c2, path=p, levels=LEVELS))
            else:
                _, n2 = ps.ps2(V, s=s, want_c2=False, want_n2=True)
                c3 = torch.empty(math.comb(n_v, 3), device="cuda")
                run = (lambda p: ps.ps3(V, s=s, n2=n2, c3=c3, path=p, levels=LEVELS))
            names = list(PATH_CODES)
            times = [_time(lambda p=p: run(p), reps) for p in names]
            best = names[int(np.argmin(times))]
            rec = _entry("u8", way, "auto", fb, vb, (n_f, n_v), PATH_CODES[best], times)
            log(json.dumps(rec))
            out.append(rec)
            if way == 2:   # tile order of the int8 matrix-core kernel
                times = []
                for idx in range(len(ps.tile_configs(dt, 2, "mfma"))):
                    ps.tune_clear()
                    ps.tune_register(dt, 2, "mfma", (0, 1 << 40), (0, 1 << 40), idx)
                    times.append(_time(lambda: run("mfma"), reps))
                ps.tune_clear()
                rec = _entry("u8", 2, "mfma", fb, vb, (n_f, n_v), int(np.argmin(times)), times)
                log(json.dumps(rec))
                out.append(rec)
            del V
            torch.cuda.empty_cache()
    return out


def _batch_inputs(dt, count=24, seed=0):
    """A representative uneven batch: shapes log-uniform like the batched
    workload (n_v in [500, 8000], n_f in [1000, 20000]), scaled down in count."""
    g = np.random.default_rng(seed)
    Vs = []
    for p in range(count):
        n_v = int(math.exp(g.uniform(math.log(500), math.log(8000))))
        n_f = int(math.exp(g.uniform(math.log(1000), math.log(20000))))
        Vs.append(_input(n_v, n_f, dt, seed=seed + p))
    return Vs


def tune_batched(dname, reps=3, log=print, count=24):
    """One entry for batched launches (way 0, any shape): the configuration
    that runs a representative uneven batch fastest as one launch."""
    dt = DTYPES[dname]
    Vs = _batch_inputs(dt, count)
    outs = ps._batch_outputs(Vs)
    ncfg = len(ps.tile_configs(dt, 2))
    times = [_time(lambda i=idx: ps.ps2_batched(Vs, outs=outs, tile=i + 1), reps)
             for idx in range(ncfg)]
    best = int(np.argmin(times))
    rec = {"dtype": dname, "way": 0, "path": "valu", "nf": [0, 1 << 40], "nv": [0, 1 << 40],
           "shape": [len(Vs), "uneven"], "tile": best, "ms": [round(t, 4) for t in times]}
    log(json.dumps(rec))
    del Vs, outs
    torch.cuda.empty_cache()
    return rec


def tune(dtypes=("f32", "f16", "u8"), ways=(2, 3, 0), reps=3, quick=False, log=print,
         batch_count=24):
    ps.tune_clear()    # time the alternatives, not earlier choices
    out = []
    for dname in dtypes:
        if 0 in ways:
            out.append(tune_batched(dname, reps, log, batch_count))
    for dname in dtypes:
        dt = DTYPES[dname]
        ncfg = len(ps.tile_configs(dt, 2))
        for way in (w for w in ways if w != 0):
            for (fb, vb), (n_f, n_v) in REPS[way].items():
                if quick and (fb, vb) not in ((1, 1), (2, 2), (1, 0)):
                    continue
                V = _input(n_v, n_f, dt)
                s, _ = ps.vector_sums(V, want_bad=False)
                if way == 3:
                    _, n2 = ps.ps2(V, s=s, want_c2=False, want_n2=True)
                    c3 = torch.empty(math.comb(n_v, 3), device="cuda")
                else:
                    c2 = torch.empty(n_v * (n_v - 1) // 2, device="cuda")
                times = []
                for idx in range(ncfg):
                    if way == 2:
                        f = (lambda i=idx: ps.ps2(V, s=s, c2=c2, path="valu", tile=i + 1))
                    else:
                        f = (lambda i=idx: ps.ps3(V, s=s, n2=n2, c3=c3, path="valu",
                                                  tile=i + 1))
                    times.append(_time(f, reps))
                rec = _entry(dname, way, "valu", fb, vb, (n_f, n_v), int(np.argmin(times)),
                             times)
                log(json.dumps(rec))
                out.append(rec)
                del V
                torch.cuda.empty_cache()
    if "u8" in dtypes and (2 in ways or 3 in ways):
        out += tune_paths(tuple(w for w in (2, 3) if w in ways), reps, quick, log)
    ps.tune_clear()      # the library now follows the new choices
    for e in out:
        register(e)
    return {"device": torch.cuda.get_device_name(0), "time": time.time(), "entries": out}


def register(e) -> None:
    """One cache entry into the library's tuning table."""
    ps.tune_register(DTYPES[e["dtype"]], e["way"], e.get("path", "valu"), e["nf"], e["nv"],
                     e["tile"])


def save(cache, path=CACHE):
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)


def load(path=CACHE) -> int:
    """Register the cached choices with libps; returns the number registered."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        cache = json.load(f)
    n = 0
    for e in cache.get("entries", []):
        register(e)
        n += 1
    return n


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--dtypes", default="f32,f16,u8")
    ap.add_argument("--ways", default="2,3,0",
                    help="ways to tune; the entries of other ways are kept from --out")
    a = ap.parse_args(argv)
    ways = tuple(int(w) for w in a.ways.split(","))
    dtypes = tuple(a.dtypes.split(","))
    cache = tune(dtypes, ways=ways, reps=a.reps, quick=a.quick)
    if os.path.exists(a.out):    # keep the entries this run did not re-tune
        with open(a.out) as f:
            old = json.load(f)
        kept = [e for e in old.get("entries", [])
                if not (e["way"] in ways and e["dtype"] in dtypes)]
        cache["entries"] = kept + cache["entries"]
    save(cache, a.out)
    print(f"wrote {a.out} ({len(cache['entries'])} entries)")


if __name__ == "__main__":
    main()
