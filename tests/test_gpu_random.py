"""Randomised GPU parity: training on random shapes, data kinds, C, gamma, precisions and with or without the offset,
each against the FP64 oracle. The FP64 path must pick the oracle's basis whenever no step was a near tie (the oracle
records each step's score gap); every path must reach the oracle's optimum at the GPU's basis (both sides of 1e-6)
and match its decision values (1e-4)."""

import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1404_1066_amd as lib
from oracle import spsvm as osp

pytestmark = pytest.mark.gpu


def _case(seed):
    r = np.random.default_rng(9000 + seed)
    n = int(r.integers(40, 2500))
    kind = ["blobs", "binary", "dups"][seed % 3]
    if kind == "binary":
        d = int(r.integers(8, 130))
        X, y = datagen.make_binary_sparse(n, d, seed=seed, ones=max(1, d // 9))
        X = X.astype(np.float64)
    else:
        d = int(r.integers(1, 300))
        X, y = datagen.make_blobs(n, d, seed=seed)
        if kind == "dups":  # a fifth of the rows repeat earlier ones
            k = n // 5
            X[n - k:] = X[:k]
            y[n - k:] = y[:k]
    groups = len(np.unique(X, axis=0))
    J_max = int(r.integers(1, min(groups, 120) + 1))
    C = float(10.0 ** r.uniform(-1, 2))
    gamma = float(10.0 ** r.uniform(-1.5, 0.5)) / max(d, 1)
    prec = ["f64", "f32", "mixed"][int(r.integers(0, 3))]
    bias = int(r.integers(0, 2))
    return X, y, J_max, C, gamma, prec, bias, int(r.integers(0, 1 << 30))


@pytest.mark.parametrize("seed", range(24))
def test_random_training_matches_oracle(seed):
    X, y, J_max, C, gamma, prec, bias, draw = _case(seed)
    n, d = X.shape
    print(f"case {seed}: n={n} d={d} J_max={J_max} C={C:.4g} gamma={gamma:.4g} {prec} bias={bias}")
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd = X if prec == "f64" else X.astype(np.float32).astype(np.float64)  # what the GPU sees
    model = lib.train(torch.tensor(Xd, dtype=dt, device="cuda"), torch.tensor(y, dtype=torch.float32, device="cuda"),
                      C, gamma, J_max, seed=draw, precision=prec, bias=bias)
    J, beta, F = model.get()
    assert len(J) == J_max
    if prec == "f64":
        ref = oracle.train(Xd, y, C, gamma, J_max, seed=draw, bias=bool(bias))
        if min(ref.gaps, default=1.0) > 1e-9:
            assert J.tolist() == ref.J.tolist()
    b_or, F_or, info = osp.solve_fixed_J(Xd, y, C, gamma, J, bias=bool(bias))
    Fo = osp.objective_at(Xd, y, C, gamma, J, beta, b=model.bias)
    assert abs(Fo - F_or) / F_or <= 1e-6, (Fo, F_or)
    dg = model.predict(torch.tensor(Xd, dtype=dt, device="cuda")).cpu().numpy()
    do = oracle.predict(Xd[J], b_or, gamma, Xd, info.bias)
    assert float(np.max(np.abs(dg - do) / np.maximum(1.0, np.abs(do)))) <= 1e-4
