"""GPU smoke test of the autotuner and the tile cache it writes.

The tuner runs for one bucket (d = 2, n <= 256) with the batch objective on
a reduced batch, writing a fresh cache; a new process (the library reads
the cache once per process) pointed at that file must plan exactly the
written tile for a problem in that bucket.  The same process checks that
rows of another architecture are ignored and that the scoped FJOFC_TILE
form applies to its (d, n range) only.
"""
import json
import os
import subprocess
import sys

import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
from paper_1502_03391_amd import fjofc
ctx = fjofc.Context(0)
out = {f"{n},{d}": fjofc.fjofc_tile_choice(ctx, n, d) for n, d in
       [(200, 2), (129, 2), (256, 2), (257, 2), (200, 3), (1000, 3), (20000, 5)]}
ctx.close()
print(json.dumps(out))
"""


def _probe(cache, tile=None):
    env = dict(os.environ, FJOFC_TUNE_TABLE=str(cache))
    env.pop("FJOFC_TILE", None)
    if tile:
        env["FJOFC_TILE"] = tile
    r = subprocess.run([sys.executable, "-c", PROBE, ROOT], env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return {k: tuple(v) for k, v in json.loads(r.stdout.strip().splitlines()[-1]).items()}


def _rows(path):
    out = []
    for line in open(path):
        p = line.partition("#")[0].split()
        if p:
            out.append((p[0], int(p[1]), int(p[2]), int(p[3]), int(p[4])))
    return out


def test_autotune_cache_is_read_back(tmp_path):
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = tmp_path / "cache.txt"
    # a row of another architecture, which the run must keep and the
    # library must ignore
    cache.write_text("gfx000 2 256 512 3   # not this device\n")
    env = dict(os.environ)
    env.pop("FJOFC_TILE", None)
    r = subprocess.run([sys.executable, "-m", "paper_1502_03391_amd.autotune", "--buckets",
                        "256", "--dims", "2", "--batch-count", "96", "--iters", "10",
                        "--out", str(cache)], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
    rows = _rows(cache)
    assert ("gfx000", 2, 256, 512, 3) in rows
    mine = [x for x in rows if x[0] == arch]
    assert len(mine) == 1 and mine[0][1:3] == (2, 256)
    th, var = mine[0][3], mine[0][4]
    rows_per_wave = {4: 4, 5: 2}.get(var, 1) * 8
    th_planned = -(-th // rows_per_wave) * rows_per_wave
    got = _probe(cache)
    # every n of the bucket (and, with no d = 3 rows, d = 3 too: the
    # nearest tabulated d) takes the row; n above it takes the default
    for key in ("200,2", "129,2", "256,2", "200,3"):
        assert got[key] == (th_planned, var), key
    assert got["257,2"] == (256, 5) and got["1000,3"] == (256, 5)
    # scoped override: only d = 2, n in [100, 220]; a later entry for d = 5
    got = _probe(cache, "2:100:220:96:4,5:10000:30000:128:1")
    assert got["200,2"] == (96, 4) and got["129,2"] == (96, 4)
    assert got["256,2"] == (th_planned, var)
    assert got["20000,5"] == (128, 1)
    got = _probe(cache, "64:1")
    assert all(v == (64, 1) for v in got.values())
