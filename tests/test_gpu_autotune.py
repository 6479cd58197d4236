"""Autotuner (needs an MI355X): the chosen options are valid, exact and cached."""

import os
import subprocess
import sys
from pathlib import Path

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

glop = pytest.importorskip("paper_1704_02278_amd")
from gpu_util import assert_same, gpu_match, oracle_match, say, to_device  # noqa: E402

ROOT = Path(__file__).resolve().parents[1]


@pytest.mark.parametrize("name,n_bytes", [("tiny", 1 << 20), ("medium", 64 << 20), ("large", 32 << 20)])
def test_tuned_options_are_exact(name, n_bytes):
    pats, text, _ = synth.make_workload(name, n_bytes=n_bytes)
    sample = torch.from_numpy(text).cuda()
    say("autotune", name, n_bytes)
    r = glop.autotune(pats, sample)
    assert r["evaluated"] >= 2 and not r["from_cache"]
    assert 0 < r["ms"] <= r["auto_ms"] * 1.0001
    d = glop.Dict(pats, **r["opts"])
    info = d.info()
    for k in ("filter", "stride", "qgram", "bitmap_log2", "probe_bits", "tile_kib"):
        if r["opts"][k]:
            assert info[k] == r["opts"][k], k
    part = text[: 8 << 20]
    assert_same(gpu_match(d, to_device(part, 5)), oracle_match(part, pats), f"{name} tuned {r['opts']}")
    again = glop.autotune(pats, sample)
    assert again["from_cache"] and again["evaluated"] == 0 and again["opts"] == r["opts"]


def test_tune_cache_file_is_shared_between_processes(tmp_path):
    cache = tmp_path / "tune.txt"
    code = (
        "import sys, torch, json; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
        "import synth, paper_1704_02278_amd as glop\n"
        "pats, text, _ = synth.make_workload('tiny')\n"
        "r = glop.autotune(pats, torch.from_numpy(text).cuda())\n"
        "print(json.dumps(r))\n" % (str(ROOT), str(ROOT / "tests"))
    )
    env = dict(os.environ, GLOP_TUNE_CACHE=str(cache))
    outs = []
    for k in range(2):
        say("tune-cache process", k)
        p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        assert p.returncode == 0, p.stderr[-2000:]
        outs.append(p.stdout.strip().splitlines()[-1])
    import json

    a, b = (json.loads(x) for x in outs)
    assert not a["from_cache"] and b["from_cache"] and a["opts"] == b["opts"]
    assert len(cache.read_text().splitlines()) == 1
