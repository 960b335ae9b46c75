"""Host logic of the 3-way work lists: the flattened (pair row, k column)
tiles of the VALU slices cover every triple of a stage exactly once; the
slab tile sets of the matrix-core slices (whole tiles plus edge tiles, or
every tile) cover each slab rectangle i < j < k exactly once, and the
finish's output ranges cover each slab.  The check is a small host program
compiled against the library's internal header (no GPU)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_slab_tile_sets_cover_each_slab_once(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "tilesets")
    subprocess.run([hipcc, "-O2", "-std=c++17", os.path.join(HERE, "tilesets_check.cpp"), "-o",
                    exe], check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")
