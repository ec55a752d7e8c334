"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and rejects bad arguments
before touching the GPU. No compute call needs a GPU here."""

import ctypes
import glob
import os
import re

import numpy as np
import pytest

import paper_1404_1066_amd as lib
from paper_1404_1066_amd import binding
from oracle import rng as orng

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(spsvm_[a-z_0-9]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = lib.load()
    declared = _declared()
    assert len(declared) >= 14
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(binding.EXPORTED)


def test_options_defaults():
    o = lib.options()
    assert o.struct_size == ctypes.sizeof(binding.Options)
    assert (o.kappa, o.growth, o.chunk_cap, o.newton_max_iter) == (59, 0.25, 256, 50)
    assert o.newton_tol == 1e-10 and o.newton_ftol == 1e-14 and o.precision == binding.SPSVM_F32


def test_workspace_sizes_grow_with_problem():
    a = lib.workspace_bytes(1000, 10, 50)
    b = lib.workspace_bytes(2000, 10, 50)
    c = lib.workspace_bytes(1000, 10, 100)
    assert 0 < a < b and a < c
    # the kernel block n x J_max dominates
    big = lib.workspace_bytes(100000, 123, 1000)
    assert big >= 100000 * 1000 * 4
    f64 = lib.workspace_bytes(100000, 123, 1000, precision="f64")
    assert f64 >= 100000 * 1000 * 8
    assert lib.workspace_bytes(1000, 10, 50, fixed=True) < a


def _train_raw(**kw):
    L = lib.load()
    o = lib.options()
    args = dict(X=ctypes.c_void_p(16), xdt=0, y=ctypes.c_void_p(16), n=100, d=3, C=1.0, gamma=1.0, J_max=10,
                opt=ctypes.byref(o), ws=ctypes.c_void_p(256), ws_bytes=1 << 30, stream=None)
    args.update(kw)
    out = ctypes.c_void_p(12345)
    st = L.spsvm_train(args["X"], args["xdt"], args["y"], args["n"], args["d"], args["C"], args["gamma"],
                       args["J_max"], args["opt"], args["ws"], args["ws_bytes"], args["stream"], ctypes.byref(out))
    return st, out.value, L.spsvm_last_error().decode()


@pytest.mark.parametrize("kw, what", [
    (dict(X=None), "device pointers"),
    (dict(C=0.0), "C must"),
    (dict(C=float("inf")), "C must"),
    (dict(gamma=-1.0), "gamma must"),
    (dict(J_max=0), "J_max"),
    (dict(J_max=101), "J_max"),
    (dict(n=0), "n must"),
    (dict(d=0), "d must"),
    (dict(xdt=7), "dtype"),
])
def test_invalid_arguments_rejected_before_gpu_work(kw, what):
    st, out, msg = _train_raw(**kw)
    assert st == 1 and out is None and what in msg


def test_bad_options_rejected():
    L = lib.load()
    o = lib.options()
    o.struct_size = 3
    st, out, msg = _train_raw(opt=ctypes.byref(o))
    assert st == 1 and "struct_size" in msg
    for field, val in [("kappa", 0), ("kappa", 65), ("chunk_cap", 0), ("newton_max_iter", 0), ("precision", 9)]:
        o = lib.options()
        setattr(o, field, val)
        st, out, msg = _train_raw(opt=ctypes.byref(o))
        assert st == 1, field


def test_status_strings_and_free_null():
    L = lib.load()
    for s in range(7):
        assert L.spsvm_status_string(s)
    L.spsvm_model_free(None)


def test_binding_refuses_cpu_tensors():
    import torch

    with pytest.raises(ValueError):
        lib.train(torch.zeros(4, 2), torch.ones(4), 1.0, 1.0, 2)


def test_host_candidate_draw_matches_oracle_generator():
    """The library's C++ sampler and the oracle's Python sampler implement the same published generator
    independently; they must draw the same rows."""
    for seed, t, n in [(0, 0, 2000), (5, 17, 100000), (2**63 + 7, 999, 12345), (1, 3, 7)]:
        a = lib.candidate_draw(seed, t, n)
        b = orng.draw_candidates(seed, t, n, 59, lambda i: False)
        assert a == b
    total = [lib.candidate_draw(3, t, 100) for t in range(200)]
    assert all(len(c) == 59 and len(set(c)) == 59 for c in total)


def test_host_candidate_draw_stream_start_matches_hand_worked_values():
    """The library's sampler against the first indices worked by hand from the published generator outputs."""
    path = os.path.join(ROOT, "tests", "golden", "candidate_stream_start.txt")
    lines = [ln for ln in open(path) if ln.strip() and not ln.startswith("#")]
    for ln in lines:
        seed, t, n, idx = [p.strip() for p in ln.split(";")]
        want = [int(v) for v in idx.split(",")]
        assert lib.candidate_draw(int(seed, 0), int(t), int(n))[:len(want)] == want
