"""GPU test of the autotuner's loop: tune one operation at a small size,
store the choice in a cache file, load the package in a fresh process with
that cache, and check that the stored shape is applied there and that the
operation's results under it still equal the oracle's."""
import json
import os
import subprocess
import sys

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


CHILD = r"""
import json, sys
import numpy as np

import torch
sys.path.insert(0, {root!r})
import oracle, workloads
import paper_1910_05109_amd as b64
b64.load()
x = workloads.random_bytes(workloads.SEED_BASE + 360, 40_003)
got = b64.encode(torch.from_numpy(x).cuda()).cpu().numpy()
print(json.dumps({{"shape": list(b64.tune_get("encode", 0)),
                   "other": list(b64.tune_get("encode", 4)),
                   "equal": bool(np.array_equal(got, oracle.encode(x)))}}))
"""


def test_tune_store_reload_apply(b64, oracle, tmp_path):
    from paper_1910_05109_amd import tune
    old = b64.tune_shapes("encode")
    cache = str(tmp_path / "tune.json")
    try:
        say("tune encode bucket 0 on 40 KB")
        r = tune.tune_op("encode", 0, nbytes=40_003, reps=5, unrolls=(1, 2), bpcs=(1, 64),
                         nts=(0, 1), verbose=False)
        best = (r["unroll"], r["blocks_per_cu"], r["nontemporal"])
        assert b64.tune_get("encode", 0) == best
        assert b64.tune_get("encode", 4) == old[4]          # other buckets untouched
        tune.save({"encode": {0: {k: r[k] for k in ("unroll", "blocks_per_cu", "nontemporal")}}},
                  cache)
        with open(cache) as f:
            data = json.load(f)
        assert list(data.values())[0]["encode"]["0"]["unroll"] == best[0]
    finally:
        b64.tune_restore("encode", old)
    say("reload in a child process with the cache")
    env = dict(os.environ, B64HIP_TUNE_CACHE=cache)
    out = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], env=env, cwd=ROOT,
                         capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    res = json.loads(out.stdout.strip().splitlines()[-1])
    assert tuple(res["shape"]) == best
    assert tuple(res["other"]) == old[4]
    assert res["equal"]
    # without the cache the child keeps the library's defaults
    env["B64HIP_TUNE_CACHE"] = "off"
    out = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], env=env, cwd=ROOT,
                         capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    res = json.loads(out.stdout.strip().splitlines()[-1])
    assert tuple(res["shape"]) == old[0] and res["equal"]


def test_malformed_cache_is_refused(b64, tmp_path):
    from paper_1910_05109_amd import tune
    path = str(tmp_path / "bad.json")
    with open(path, "w") as f:
        json.dump({tune.device_key(): {"encode": {"7": {"unroll": 4, "blocks_per_cu": 1}}}}, f)
    old = b64.tune_shapes("encode")
    try:
        with pytest.raises(ValueError):
            tune.apply_cached(path)
    finally:
        b64.tune_restore("encode", old)
