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
                                           (66000, 123, 256, True), (66000, 90, 300, True)])
def test_rbf_block_mixed_wide_tiles(n, d, nc, binary):
    """Blocks of 192 or more columns (with at least 256 tiles) take 256 x 256 tiles (binary rows are BF16 numbers:
    single-pass products in 64-wide k chunks; 90 features make the last chunk a half one). Against the oracle: the split
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


# 3329, 4000 and 4100 are past the one-workgroup triangular solves (3328): blocked solves, the last block partial
@pytest.mark.parametrize("m", [1, 5, 63, 64, 65, 130, 500, 1000, 1025, 1100, 2000, 3329, 4000, 4100])
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


@pytest.mark.parametrize("bad", [-1.0, 0.0, 1e-310])
def test_newton_solve_reports_not_pd(bad):
    """A pivot that is negative, zero or subnormal (as good as zero at FP64 scale) is reported as not positive
    definite, not turned into an infinite factor."""
    H = torch.tensor(np.diag([1.0, bad, 2.0]), device="cuda")
    with pytest.raises(lib.SpsvmError) as e:
        lib.newton_solve(H, torch.ones(3, dtype=torch.float64, device="cuda"))
    assert e.value.status == 4


# -------------------------------------------------------------------------------------------- scoring
def _scores_vs_oracle(o, y, cols, oc, C):
    """GPU scores of the candidate columns against the oracle's exact one-coefficient minimisation on the same
    values (the columns as the FP32 numbers the GPU reads)."""
    from oracle import spsvm as osp

    Kc = np.ascontiguousarray(np.stack(cols).astype(np.float32))
    res = lib.score_candidates(torch.tensor(o, device="cuda"), torch.tensor(y, dtype=torch.float32, device="cuda"),
                               torch.tensor(Kc, device="cuda"), oc, C)
    a = 1.0 - y * o
    f0 = 0.5 * float(np.sum(np.maximum(a, 0.0) ** 2))
    ref = [osp.score_candidate(a, y * Kc[c].astype(np.float64), 1.0 / C, float(oc[c])) for c in range(len(cols))]
    return res, ref, f0


def _check_scores(res, ref, f0):
    best = max(r[1] for r in ref)
    for c, (s_or, sc_or) in enumerate(ref):
        if res["status"][c] == 1:
            assert abs(res["s"][c] - s_or) <= 1e-9 * (1.0 + abs(s_or)), (c, res["s"][c], s_or)
            assert abs(res["score"][c] - sc_or) <= 1e-11 * f0, (c, res["score"][c], sc_or)
        else:  # dropped: it could not have won
            assert res["status"][c] == 3 and sc_or <= best * (1 + 1e-6)


# 1 100 000 rows: several thousand rows per workgroup of a pass
@pytest.mark.parametrize("n,ncand,C", [(5003, 64, 1.0), (777, 59, 10.0), (1, 3, 1.0), (130, 1, 0.5),
                                       (1100000, 13, 1.0)])
def test_candidate_scores_match_oracle(n, ncand, C):
    r = np.random.default_rng(n + ncand)
    o = r.standard_normal(n) * 0.8
    y = np.where(r.random(n) < 0.5, 1.0, -1.0)
    cols = [np.where(r.random(n) < 0.1, 0.0, r.random(n)) for _ in range(ncand)]
    oc = r.standard_normal(ncand) * 0.5
    res, ref, f0 = _scores_vs_oracle(o, y, cols, oc, C)
    _check_scores(res, ref, f0)
    want = max(range(ncand), key=lambda c: (ref[c][1], -c))
    assert res["winner"] == want


@pytest.mark.parametrize("label", [0.5, 0.0, float("nan")])
def test_candidate_scores_reject_labels_other_than_plus_minus_one(label):
    n = 1000
    y = torch.ones(n, dtype=torch.float32, device="cuda")
    y[n // 2] = label
    o = torch.zeros(n, dtype=torch.float64, device="cuda")
    Kc = torch.rand(3, n, dtype=torch.float32, device="cuda")
    with pytest.raises(lib.SpsvmError) as e:
        lib.score_candidates(o, y, Kc, np.zeros(3), 1.0)
    assert e.value.status == 1


@pytest.mark.parametrize("pad", [0, 1100000])
def test_candidate_score_window_overflow_falls_back_to_full_passes(pad):
    """Two candidates with the same one-dimensional problem psi'(s) = 0.9 s - sum b max(0, a - s b), built from
    row groups: 1000 rows with b = 0.01, a = 1 (breakpoint 100); a group with breakpoint 9.99 and sum b^2 = 1; 10
    rows with breakpoint 5. The first Newton point from s = 0 is 9.98503, just below 9.99, and the root (10) lies
    just above it: both inside the window of |s| / 256 around that point. For candidate 0 the 9.99 group has 100
    rows, more than the 64 a window list holds, so the list is incomplete and the slot must continue with full
    passes (4 in all); for candidate 1 the group has 40 rows and the window walk finishes it after 2 passes. Both
    scores must be the exact minimum. pad: rows with kernel value 0 for both candidates (no effect on either
    problem) appended, so that each workgroup of a pass walks thousands of rows."""
    def block(nc):
        bc = float(np.float32(np.sqrt(1.0 / nc)))
        k = np.concatenate([np.full(1000, 0.01), np.full(nc, bc), np.full(10, 0.02)]).astype(np.float32)
        kd = k.astype(np.float64)
        a = np.concatenate([np.ones(1000), 9.99 * kd[1000:1000 + nc], 5.0 * kd[1000 + nc:]])
        return k, 1.0 - a  # y = +1: a = 1 - o
    k0, o0 = block(100)
    k1, o1 = block(40)
    n0, n1 = k0.size, k1.size
    r = np.random.default_rng(9)
    o = np.concatenate([o0, o1, r.standard_normal(pad)])
    y = np.concatenate([np.ones(n0 + n1), np.where(r.random(pad) < 0.5, 1.0, -1.0)])
    zp = np.zeros(pad, np.float32)
    cols = [np.concatenate([k0, np.zeros(n1, np.float32), zp]), np.concatenate([np.zeros(n0, np.float32), k1, zp])]
    res, ref, f0 = _scores_vs_oracle(o, y, cols, np.zeros(2), 1.0 / 0.9)
    assert list(res["status"]) == [1, 1]
    _check_scores(res, ref, f0)
    assert abs(ref[0][0] - 10.0) < 1e-6 and abs(ref[1][0] - 10.0) < 1e-6
    assert res["passes"][1] == 2
    assert res["passes"][0] >= 3
