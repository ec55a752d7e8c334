"""Sparse (CSR) rows: greedy training and prediction against the FP64 oracle on the same rows made dense."""

import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1404_1066_amd as lib
from oracle import spsvm as osp

pytestmark = pytest.mark.gpu


def _dev_csr(ip, ix, v):
    return (torch.tensor(ip, device="cuda"), torch.tensor(ix, device="cuda"), torch.tensor(v, device="cuda"))


def _decision_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))


@pytest.mark.parametrize("n,d,bias", [(20000, 127, 0), (9001, 300, 1)])
def test_csr_training_reaches_oracle_objective(n, d, bias):
    """KDDCup-like rows (about 10% of the features set; 300 features take the sparse block's second feature chunk),
    greedy to |J| = 150: the oracle re-solves at the GPU's basis on the dense rows; decisions of held-out CSR rows
    against the oracle's; the dense prediction of the same model agrees."""
    ip, ix, v, y = datagen.make_sparse_rows(n, d, seed=7)
    X = datagen.csr_to_dense(ip, ix, v, d)
    C, gamma, m = 10.0, 0.1, 150
    model = lib.train_csr(*_dev_csr(ip, ix, v), d, torch.tensor(y, dtype=torch.float32, device="cuda"), C, gamma, m,
                          seed=1, bias=bias)
    J, beta, F = model.get()
    assert len(J) == m and len(set(osp.duplicate_groups(X)[J].tolist())) == m
    b_or, F_or, info = osp.solve_fixed_J(X, y, C, gamma, J, bias=bool(bias))
    Fo = osp.objective_at(X, y, C, gamma, J, beta, b=model.bias)
    print("F_gpu", Fo, "F_oracle", F_or, "rel", (Fo - F_or) / F_or)
    assert abs(Fo - F_or) / F_or <= 1e-6
    ipt, ixt, vt, _ = datagen.make_sparse_rows(3000, d, seed=8)
    Xt = datagen.csr_to_dense(ipt, ixt, vt, d)
    dg = lib.predict_csr(model, *_dev_csr(ipt, ixt, vt)).cpu().numpy()
    do = oracle.predict(X[J], b_or, gamma, Xt, info.bias)
    assert _decision_err(dg, do) <= 1e-4
    dd = model.predict(torch.tensor(Xt, dtype=torch.float32, device="cuda")).cpu().numpy()
    assert _decision_err(dg, dd) <= 1e-5


def test_csr_invalid_indices_rejected():
    ip = np.array([0, 2, 3], dtype=np.int64)
    ix = np.array([3, 1, 0], dtype=np.int32)  # row 0 not increasing
    v = np.ones(3, dtype=np.float32)
    y = torch.tensor([1.0, -1.0], device="cuda")
    with pytest.raises(lib.SpsvmError) as e:
        lib.train_csr(*_dev_csr(ip, ix, v), 5, y, 1.0, 0.5, 1)
    assert e.value.status == 1 and "feature indices" in str(e.value)


def test_csr_with_kxj_in_host_memory_gives_the_same_model():
    """CSR rows with the offset and K_XJ in pinned host memory: bit for bit the model made with K_XJ in the
    workspace (the offset's column of ones is written to host memory too)."""
    ip, ix, v, y = datagen.make_sparse_rows(8000, 127, seed=9)
    args = (*_dev_csr(ip, ix, v), 127, torch.tensor(y, dtype=torch.float32, device="cuda"), 10.0, 0.1, 60)
    a = lib.train_csr(*args, seed=2, bias=1)
    b = lib.train_csr(*args, seed=2, bias=1, kxj_host=1)
    Ja, ba, Fa = a.get()
    Jb, bb, Fb = b.get()
    assert np.array_equal(Ja, Jb) and np.array_equal(ba, bb) and Fa == Fb and a.bias == b.bias
