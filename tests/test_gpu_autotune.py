"""The kernel-block autotuner (SPSVM_AUTOTUNE=1, choices cached in the JSON file SPSVM_TUNE_CACHE): every variant it
can pick gives the same bits, so a tuned training run returns the untuned run's model bit for bit, and a second
process reads the cached choices; each variant forced in turn (SPSVM_KBLOCK_VARIANT) gives the same bits too. The
environment is read once per process, so the tuned runs are subprocesses."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import datagen
import paper_1404_1066_amd as lib

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_RUN = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
import datagen, paper_1404_1066_amd as lib
X, y = datagen.make_blobs(70001, 300, seed=24, dtype=np.float32)
Xg = torch.tensor(X, device="cuda"); yg = torch.tensor(y, dtype=torch.float32, device="cuda")
J, beta, F = lib.train(Xg, yg, 1.0, 1.0 / 300, 60, seed=2, precision="mixed").get()
B = (np.random.default_rng(5).random((66000, 90)) < 0.2).astype(np.float32)
idx = torch.tensor(np.random.default_rng(6).integers(0, 66000, 300), dtype=torch.int32, device="cuda")
K = lib.rbf_block(torch.tensor(B, device="cuda"), idx, 0.05, "mixed").cpu().numpy()
np.savez(sys.argv[2], J=J, beta=beta, F=np.array([F]), K=K)
"""

VARIANTS = ("rows128", "rows256", "wide", "wide_k32", "wide_half")


def _run(tmp_path, name, env):
    script = tmp_path / "run.py"
    script.write_text(_RUN)
    out = tmp_path / f"{name}.npz"
    e = dict(os.environ)
    e.update(env)
    r = subprocess.run([sys.executable, str(script), ROOT, str(out)], env=e, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return np.load(out)


def test_tuned_training_is_bitwise_the_untuned_one(tmp_path):
    X, y = datagen.make_blobs(70001, 300, seed=24, dtype=np.float32)
    Xg = torch.tensor(X, device="cuda")
    yg = torch.tensor(y, dtype=torch.float32, device="cuda")
    J, beta, F = lib.train(Xg, yg, 1.0, 1.0 / 300, 60, seed=2, precision="mixed").get()
    cache = tmp_path / "tune.json"
    tuned = _run(tmp_path, "tuned", {"SPSVM_AUTOTUNE": "1", "SPSVM_TUNE_CACHE": str(cache)})
    assert np.array_equal(tuned["J"], J) and np.array_equal(tuned["beta"], beta) and tuned["F"][0] == F
    entries = [json.loads(ln) for ln in cache.read_text().splitlines() if ln.strip()]
    assert entries and all(e["variant"] in VARIANTS for e in entries)
    assert any(e["key"].startswith("split=0") for e in entries) and any(e["key"].startswith("split=1") for e in entries)
    cached = _run(tmp_path, "cached", {"SPSVM_TUNE_CACHE": str(cache)})
    assert np.array_equal(cached["J"], J) and np.array_equal(cached["beta"], beta) and cached["F"][0] == F


def test_every_forced_variant_gives_the_same_bits(tmp_path):
    """Training (single-pass candidate blocks, split winners' columns) and a single-pass block of binary rows with
    90 features (a half k chunk for the 64-wide chunk form), each with one variant forced wherever it applies."""
    base = _run(tmp_path, "base", {})
    for v in VARIANTS:
        got = _run(tmp_path, v, {"SPSVM_KBLOCK_VARIANT": v})
        assert np.array_equal(got["J"], base["J"]) and np.array_equal(got["beta"], base["beta"]), v
        assert got["F"][0] == base["F"][0] and np.array_equal(got["K"], base["K"]), v
