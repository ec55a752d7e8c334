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


@pytest.mark.parametrize("seed", range(8))
def test_random_batch_matches_oracle(seed):
    """Batched Newton solves on a random shared basis: random problem count, labels, C and gamma per problem."""
    r = np.random.default_rng(9500 + seed)
    n, d = int(r.integers(60, 2000)), int(r.integers(2, 120))
    X, _ = datagen.make_blobs(n, d, seed=100 + seed)
    P = int(r.integers(1, 9))
    Y = np.where(r.standard_normal((P, n)) + X[:, :1].T > 0, 1.0, -1.0)
    C = 10.0 ** r.uniform(-1, 2, P)
    gamma = 10.0 ** r.uniform(-1.5, 0.5, P) / d
    m = int(r.integers(1, min(n, 150) + 1))
    J = np.sort(r.choice(n, m, replace=False))
    prec = ["f64", "f32", "mixed"][seed % 3]
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd = X if prec == "f64" else X.astype(np.float32).astype(np.float64)
    models = lib.train_batch(torch.tensor(Xd, dtype=dt, device="cuda"),
                             torch.tensor(Y, dtype=torch.float32, device="cuda"), C, gamma, J, precision=prec)
    for q in range(P):
        _, beta, _ = models[q].get()
        b_or, F_or, _ = osp.solve_fixed_J(Xd, Y[q], C[q], gamma[q], J)
        Fo = osp.objective_at(Xd, Y[q], C[q], gamma[q], J, beta)
        assert abs(Fo - F_or) / F_or <= 1e-6, (q, Fo, F_or)


@pytest.mark.parametrize("seed", range(6))
def test_random_shared_basis_reaches_oracle_objective(seed):
    """A greedily grown shared basis for random problems: every problem at the oracle's optimum on that basis."""
    r = np.random.default_rng(9700 + seed)
    n, d = int(r.integers(100, 1500)), int(r.integers(2, 60))
    X, _ = datagen.make_blobs(n, d, seed=200 + seed)
    P = int(r.integers(1, 6))
    Y = np.where(r.standard_normal((P, n)) + X[:, 1:2].T > 0, 1.0, -1.0)
    C = 10.0 ** r.uniform(-1, 2, P)
    gamma = np.repeat(10.0 ** r.uniform(-1.5, 0.5, 2) / d, (P + 1) // 2)[:P]
    J_max = int(r.integers(1, min(n, 80) + 1))
    prec = ["f64", "f32", "mixed"][seed % 3]
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd = X if prec == "f64" else X.astype(np.float32).astype(np.float64)
    models = lib.train_shared(torch.tensor(Xd, dtype=dt, device="cuda"),
                              torch.tensor(Y, dtype=torch.float32, device="cuda"), C, gamma, J_max,
                              seed=int(r.integers(0, 1 << 30)), precision=prec)
    J0 = models[0].get()[0]
    assert len(J0) == J_max
    for q in range(P):
        J, beta, _ = models[q].get()
        assert J.tolist() == J0.tolist()
        b_or, F_or, _ = osp.solve_fixed_J(Xd, Y[q], C[q], gamma[q], J)
        Fo = osp.objective_at(Xd, Y[q], C[q], gamma[q], J, beta)
        assert abs(Fo - F_or) / F_or <= 1e-6, (q, Fo, F_or)


@pytest.mark.parametrize("seed", range(6))
def test_random_csr_training_reaches_oracle_objective(seed):
    """CSR rows of random size and width, with or without the offset."""
    r = np.random.default_rng(9900 + seed)
    n, d = int(r.integers(200, 6000)), int(r.integers(4, 400))
    ip, ix, v, y = datagen.make_sparse_rows(n, d, seed=300 + seed, mean_nnz=max(2.0, d / 10))
    X = datagen.csr_to_dense(ip, ix, v, d)
    groups = len(np.unique(X, axis=0))
    J_max = int(r.integers(1, min(groups, 100) + 1))
    C, gamma, bias = float(10.0 ** r.uniform(-1, 2)), float(10.0 ** r.uniform(-1.5, 0) * 10 / d), seed % 2
    dev = [torch.tensor(a, device="cuda") for a in (ip, ix, v)]
    model = lib.train_csr(*dev, d, torch.tensor(y, dtype=torch.float32, device="cuda"), C, gamma, J_max,
                          seed=int(r.integers(0, 1 << 30)), bias=bias)
    J, beta, _ = model.get()
    assert len(J) == J_max
    b_or, F_or, _ = osp.solve_fixed_J(X, y, C, gamma, J, bias=bool(bias))
    Fo = osp.objective_at(X, y, C, gamma, J, beta, b=model.bias)
    assert abs(Fo - F_or) / F_or <= 1e-6, (Fo, F_or)
