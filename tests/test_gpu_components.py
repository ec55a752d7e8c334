"""GPU parity of single hot-path steps (kernel block, Cholesky Newton solve) against the FP64 oracle."""

import numpy as np
import pytest
import torch

import oracle
import paper_1404_1066_amd as lib

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


def _kblock_case(n, d, nc, prec, xdtype, seed, binary=False):
    r = np.random.default_rng(seed)
    X = (r.random((n, d)) < 0.2).astype(np.float64) if binary else r.standard_normal((n, d)) * 0.7
    X = X.astype(xdtype).astype(np.float64)  # the values the library actually receives
    idx = r.integers(0, n, size=nc).astype(np.int32)
    gamma = 0.5 / d if not binary else 0.05
    Xg = torch.tensor(X, dtype=torch.float32 if xdtype == np.float32 else torch.float64, device="cuda")
    K = lib.rbf_block(Xg, torch.tensor(idx, device="cuda"), gamma, prec).cpu().numpy().astype(np.float64)
    want = oracle.rbf_block(X, X[idx], gamma)
    return X, idx, gamma, K, want


@pytest.mark.parametrize("n,d,nc", [(1, 1, 1), (1037, 70, 59), (300, 123, 64), (129, 5, 3), (4100, 33, 70),
                                    (257, 200, 130)])
def test_rbf_block_f64_matches_oracle(n, d, nc):
    X, idx, gamma, K, want = _kblock_case(n, d, nc, "f64", np.float64, n * 7 + d)
    assert np.max(np.abs(K - want)) <= 1e-12


@pytest.mark.parametrize("n,d,nc", [(1, 1, 1), (1037, 70, 59), (300, 123, 64), (129, 5, 3), (4100, 33, 70)])
def test_rbf_block_f32_within_rounding_bound(n, d, nc):
    X, idx, gamma, K, want = _kblock_case(n, d, nc, "f32", np.float32, n * 11 + d)
    nx = (X * X).sum(1)
    # |d2 error| <= ~ (d + 2) eps32 (|x|^2 + |z|^2) from FP32 products, sums and norms; exp adds a few ulps
    bound = (d + 4) * EPS32 * gamma * (nx[:, None] + nx[idx][None, :]) * want + 4 * EPS32
    assert np.all(np.abs(K - want) <= bound)


@pytest.mark.parametrize("n,d,nc", [(1037, 70, 59), (300, 123, 64), (129, 5, 3), (4100, 54, 70), (70001, 54, 70),
                                    (66000, 300, 64)])
def test_rbf_block_mixed_within_split_bound(n, d, nc):
    """Split-BF16 products: x = hi + lo with |x - hi - lo| <= 2^-17 |x| and the dropped lo.lo' <= 2^-16 |x||z|
    per term, so |d2 error| <= about 2^-13 (|x|^2 + |z|^2)."""
    X, idx, gamma, K, want = _kblock_case(n, d, nc, "mixed", np.float32, n * 13 + d)
    nx = (X * X).sum(1)
    bound = 2.0 ** -13 * gamma * (nx[:, None] + nx[idx][None, :]) * want + 4 * EPS32
    assert np.all(np.abs(K - want) <= bound)


@pytest.mark.parametrize("n,d,nc,binary", [(70001, 300, 260, False), (66000, 54, 512, False),
                                           (66000, 123, 256, True)])
def test_rbf_block_mixed_wide_tiles(n, d, nc, binary):
    """Blocks of 192 or more columns (with at least 256 tiles) take 256 x 256 tiles. Against the oracle: the split
    bound (exact on binary rows). Against 64-column slices of the same block, which take the 64-column tiles: the
    same products are summed in the same order, so the bits agree."""
    X, idx, gamma, K, want = _kblock_case(n, d, nc, "mixed", np.float32, n * 17 + d, binary=binary)
    if binary:
        # exact distances; the FP32 exponent argument gamma log2(e) d2 carries a relative rounding of ~1 eps,
        # which moves K by |ln K| eps relative, and exp2 adds a few ulps
        assert np.all(np.abs(K - want) <= (2.0 * -np.log(want) + 4.0) * EPS32 * want)
    else:
        nx = (X * X).sum(1)
        bound = 2.0 ** -13 * gamma * (nx[:, None] + nx[idx][None, :]) * want + 4 * EPS32
        assert np.all(np.abs(K - want) <= bound)
    Xg = torch.tensor(X, dtype=torch.float32, device="cuda")
    for c in range(0, nc, 64):
        part = lib.rbf_block(Xg, torch.tensor(idx[c:c + 64], device="cuda"), gamma, "mixed").cpu().numpy()
        assert np.array_equal(part.astype(np.float64), K[:, c:c + 64])


def test_rbf_block_mixed_exact_on_binary_rows():
    X, idx, gamma, K, want = _kblock_case(2000, 123, 64, "mixed", np.float32, 6, binary=True)
    assert np.max(np.abs(K - want) / want) <= 4 * EPS32


def test_rbf_block_binary_rows_exact_distances():
    X, idx, gamma, K, want = _kblock_case(2000, 123, 64, "f32", np.float32, 5, binary=True)
    assert np.max(np.abs(K - want) / want) <= 4 * EPS32


def test_rbf_block_negative_index_leaves_column():
    r = np.random.default_rng(3)
    X = torch.tensor(r.standard_normal((200, 9)), dtype=torch.float32, device="cuda")
    idx = torch.tensor([3, -1, 7], dtype=torch.int32, device="cuda")
    out = torch.full((200, 3), float("nan"), dtype=torch.float32, device="cuda")
    lib.rbf_block(X, idx, 0.3, "f32", out=out)
    o = out.cpu().numpy()
    assert np.all(np.isnan(o[:, 1])) and np.all(np.isfinite(o[:, [0, 2]]))


@pytest.mark.parametrize("m", [1, 5, 63, 64, 65, 130, 500, 1000, 1025, 1100, 2000])
def test_newton_solve_matches_numpy(m):
    r = np.random.default_rng(m)
    A = r.standard_normal((m, m + 7))
    H = A @ A.T / (m + 7) + 0.5 * np.eye(m)
    g = r.standard_normal(m)
    Hd = torch.tensor(H, device="cuda")
    upper = torch.triu(torch.ones(m, m, dtype=torch.bool, device="cuda"), 1)
    Hd[upper] = float("nan")  # the strict upper triangle must not be read
    x = lib.newton_solve(Hd, torch.tensor(g, device="cuda")).cpu().numpy()
    want = -np.linalg.solve(H, g)
    assert np.max(np.abs(x - want)) <= 1e-12 * np.max(np.abs(want)) * 10
    L = np.tril(Hd.cpu().numpy())
    assert np.max(np.abs(L - np.linalg.cholesky(H))) <= 1e-13 * np.max(np.abs(H)) * 10
    assert torch.isnan(Hd[upper]).all()


def test_newton_solve_reports_not_pd():
    H = torch.tensor(np.diag([1.0, -1.0, 2.0]), device="cuda")
    with pytest.raises(lib.SpsvmError) as e:
        lib.newton_solve(H, torch.ones(3, dtype=torch.float64, device="cuda"))
    assert e.value.status == 4
