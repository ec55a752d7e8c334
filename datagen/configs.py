"""Seeded generators for the SP-SVM workloads.

Five workloads, named by what they are:

=================  =========  =====  ====================================================
name               n          d      shape of the data
=================  =========  =====  ====================================================
``blobs-2k``       2 000      16     2 classes x 4 isotropic Gaussians, FP64
``binary-100k``    100 000    123    {0,1} rows with exactly 14 ones, Zipf(1.1) columns
``onehot-500k``    500 000    54     10 continuous + one-hot groups of 4 and 40
``mnist-60k``      60 000     784    10-class Gaussian mixture clipped to [0, 1]
``dense-2m``       2 000 000  2 000  i.i.d. N(0, 1) features
=================  =========  =====  ====================================================

They imitate the shapes of the paper's data sets (Table 1, section 5: Adult,
Covertype, MNIST8M, Epsilon), which are not available. Labels come from random
"teacher" functions with a fixed fraction of flipped labels, so the problems are
learnable but not separable.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

BLOCK = 65536  # rows per independently seeded generation block


@dataclasses.dataclass
class Problem:
    """One binary training problem: rows X (n x d, C-contiguous), labels y in {-1,+1}."""

    name: str
    X: np.ndarray
    y: np.ndarray  # float64 (+1 / -1)
    C: float
    gamma: float
    J_max: int
    info: dict = dataclasses.field(default_factory=dict)


@dataclasses.dataclass
class BatchProblem:
    """Many binary problems that share X and one basis J (one-vs-rest x (C, gamma) grid)."""

    name: str
    X: np.ndarray
    Y: np.ndarray  # P x n float64 labels
    C: np.ndarray  # P
    gamma: np.ndarray  # P
    J: np.ndarray  # shared basis indices (int64, ascending)
    info: dict = dataclasses.field(default_factory=dict)


def _streams(seed: int, n: int, extra: int = 2):
    """Generators: ``extra`` parameter streams, then one per BLOCK-row block."""
    nblk = max(1, -(-n // BLOCK))
    kids = np.random.SeedSequence(seed).spawn(extra + nblk)
    return [np.random.default_rng(k) for k in kids[:extra]], [np.random.default_rng(k) for k in kids[extra:]]


def _blocks(n: int):
    for b, lo in enumerate(range(0, n, BLOCK)):
        yield b, lo, min(n, lo + BLOCK)


def _flip_exact(rng, y: np.ndarray, count: int) -> np.ndarray:
    idx = rng.choice(y.shape[0], size=count, replace=False)
    y = y.copy()
    y[idx] = -y[idx]
    return y


# ----------------------------------------------------------------------------------------------
def make_blobs(n: int = 2000, d: int = 16, seed: int = 0, comps: int = 4, mean_std: float = 2.0,
               dtype=np.float64) -> tuple[np.ndarray, np.ndarray]:
    """Balanced 2-class mixture: per class ``comps`` means ~ N(0, mean_std^2 I), x = mean + N(0, I)."""
    (gp, gl), blk = _streams(seed, n)
    means = gp.standard_normal((2, comps, d)) * mean_std
    y = np.where(np.arange(n) < n // 2 + (n % 2), 1.0, -1.0)
    y = y[gl.permutation(n)]
    X = np.empty((n, d), dtype=np.float64)
    for b, lo, hi in _blocks(n):
        r = blk[b]
        cls = (y[lo:hi] < 0).astype(np.int64)
        comp = r.integers(0, comps, size=hi - lo)
        X[lo:hi] = means[cls, comp] + r.standard_normal((hi - lo, d))
    return np.ascontiguousarray(X.astype(dtype)), y


def make_binary_sparse(n: int = 100000, d: int = 123, seed: int = 1, ones: int = 14, zipf: float = 1.1,
                       centres: int = 200, teacher_gamma: float = 0.05, flip: float = 0.10):
    """{0,1} rows with exactly ``ones`` ones; column j is picked with weight r_j^-zipf (r a random
    permutation of 1..d), without replacement (Gumbel top-k). Labels: sign of a sum of Gaussian bumps
    around ``centres`` random rows of the same kind, thresholded at its median, then exactly
    floor(flip*n) labels flipped."""
    (gp, gl), blk = _streams(seed, n)
    logw = -zipf * np.log(gp.permutation(d) + 1.0)

    def rows(rng, m):
        keys = logw[None, :] + rng.gumbel(size=(m, d))
        top = np.argpartition(-keys, ones - 1, axis=1)[:, :ones]
        out = np.zeros((m, d), dtype=np.float32)
        np.put_along_axis(out, top, 1.0, axis=1)
        return out

    cen = rows(gp, centres).astype(np.float64)
    amp = gp.standard_normal(centres)
    X = np.empty((n, d), dtype=np.float32)
    s = np.empty(n)
    for b, lo, hi in _blocks(n):
        xb = rows(blk[b], hi - lo)
        X[lo:hi] = xb
        sq = ones + cen.sum(1)[None, :] - 2.0 * (xb.astype(np.float64) @ cen.T)
        s[lo:hi] = np.exp(-teacher_gamma * sq) @ amp
    y = np.where(s - np.median(s) >= 0, 1.0, -1.0)
    y = _flip_exact(gl, y, int(np.floor(flip * n)))
    return X, y


def make_mixed_onehot(n: int = 500000, seed: int = 2, n_cont: int = 10, grp_a: int = 4, grp_b: int = 40,
                      zipf: float = 1.1, classes: int = 7, per_class: int = 30, teacher_gamma: float = 0.5,
                      positive_class: int = 2):
    """10 N(0,1) columns, a one-hot group of ``grp_a`` uniform categories and one of ``grp_b``
    Zipf(zipf) categories. A ``classes``-class teacher (argmax of per-class sums of Gaussian bumps
    around ``per_class`` random rows) is reduced to one-vs-rest for ``positive_class`` (1-based).
    The continuous columns are then standardised over the sample."""
    (gp, gl), blk = _streams(seed, n)
    pb = np.arange(1, grp_b + 1, dtype=np.float64) ** (-zipf)
    pb /= pb.sum()
    d = n_cont + grp_a + grp_b

    def rows(rng, m):
        out = np.zeros((m, d), dtype=np.float64)
        out[:, :n_cont] = rng.standard_normal((m, n_cont))
        out[np.arange(m), n_cont + rng.integers(0, grp_a, size=m)] = 1.0
        out[np.arange(m), n_cont + grp_a + rng.choice(grp_b, size=m, p=pb)] = 1.0
        return out

    cen = rows(gp, classes * per_class)
    amp = gp.standard_normal(classes * per_class)
    cn = (cen * cen).sum(1)
    X = np.empty((n, d), dtype=np.float64)
    cls = np.empty(n, dtype=np.int64)
    for b, lo, hi in _blocks(n):
        xb = rows(blk[b], hi - lo)
        X[lo:hi] = xb
        sq = (xb * xb).sum(1)[:, None] + cn[None, :] - 2.0 * (xb @ cen.T)
        contrib = np.exp(-teacher_gamma * np.maximum(sq, 0.0)) * amp[None, :]
        cls[lo:hi] = contrib.reshape(hi - lo, classes, per_class).sum(2).argmax(1)
    mu = X[:, :n_cont].mean(0)
    sd = X[:, :n_cont].std(0)
    X[:, :n_cont] = (X[:, :n_cont] - mu) / sd
    y = np.where(cls == positive_class - 1, 1.0, -1.0)
    return np.ascontiguousarray(X.astype(np.float32)), y, {"positive_fraction": float((y > 0).mean())}


def make_mnist_like(per_class: int = 6000, d: int = 784, seed: int = 3, classes: int = 10, noise: float = 0.25):
    """10-class mixture: means ~ U[0,1]^d, x = clip(mean + noise * N(0, I), 0, 1); rows shuffled."""
    n = per_class * classes
    (gp, gl), blk = _streams(seed, n)
    means = gp.random((classes, d))
    cls = np.repeat(np.arange(classes), per_class)[gl.permutation(n)]
    X = np.empty((n, d), dtype=np.float32)
    for b, lo, hi in _blocks(n):
        X[lo:hi] = np.clip(means[cls[lo:hi]] + noise * blk[b].standard_normal((hi - lo, d)), 0.0, 1.0)
    return X, cls


def make_large_dense(n: int = 2000000, d: int = 2000, seed: int = 4, waves: int = 16, amp: float = 0.3,
                     flip: float = 0.05, out: Optional[np.ndarray] = None, threads: int = 1):
    """x ~ N(0, I_d) in FP32; y = sign(w.x + amp * sum_k sin(u_k.x)) with w, u_k ~ N(0, I/d), then exactly
    floor(flip*n) labels flipped. ``out`` may be a preallocated (e.g. pinned) n x d float32 array;
    ``threads`` > 1 generates blocks in a thread pool (the result does not depend on it)."""
    (gp, gl), blk = _streams(seed, n)
    w = gp.standard_normal(d) / np.sqrt(d)
    U = gp.standard_normal((waves, d)) / np.sqrt(d)
    X = out if out is not None else np.empty((n, d), dtype=np.float32)
    assert X.shape == (n, d) and X.dtype == np.float32
    s = np.empty(n)

    def one(args):
        b, lo, hi = args
        xb = blk[b].standard_normal((hi - lo, d), dtype=np.float32)
        X[lo:hi] = xb
        x64 = xb.astype(np.float64)
        s[lo:hi] = x64 @ w + amp * np.sin(x64 @ U.T).sum(1)

    jobs = list(_blocks(n))
    if threads > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, jobs))
    else:
        for j in jobs:
            one(j)
    y = np.where(s >= 0, 1.0, -1.0)
    y = _flip_exact(gl, y, int(np.floor(flip * n)))
    return X, y


def make_sparse_rows(n: int = 200000, d: int = 127, seed: int = 5, mean_nnz: float = 12.0, zipf: float = 1.1,
                     centres: int = 100, teacher_gamma: float = 0.2, flip: float = 0.05):
    """Sparse rows shaped like KDDCup99 (about 10% of 127 features set): each row sets 1 + Poisson(mean_nnz - 1)
    distinct features (at most d, some rows empty of all but one), picked with weight r_j^-zipf (r a random
    permutation of 1..d) by Gumbel top-k; a random half of the features are one-hot style (value 1) and the rest
    log-normal counts (exp(N(0, 1)), FP32). Labels: sign of a sum of Gaussian bumps around ``centres`` rows of the same
    kind, thresholded at its median, then exactly floor(flip * n) flipped. Returns CSR arrays (indptr int64, indices
    int32 increasing within a row, values float32) and the labels."""
    (gp, gl), blk = _streams(seed, n)
    logw = -zipf * np.log(gp.permutation(d) + 1.0)
    binary = gp.random(d) < 0.5

    def rows(rng, m):
        k = np.minimum(d, 1 + rng.poisson(mean_nnz - 1.0, size=m))
        keys = logw[None, :] + rng.gumbel(size=(m, d))
        order = np.argsort(-keys, axis=1)
        dense = np.zeros((m, d), dtype=np.float32)
        for i in range(m):
            cols = order[i, :k[i]]
            dense[i, cols] = np.where(binary[cols], 1.0, np.exp(rng.standard_normal(k[i]))).astype(np.float32)
        return dense

    cen = rows(gp, centres).astype(np.float64)
    amp = gp.standard_normal(centres)
    cn = (cen * cen).sum(1)
    indptr = np.zeros(n + 1, dtype=np.int64)
    idx_parts, val_parts = [], []
    s = np.empty(n)
    for b, lo, hi in _blocks(n):
        xb = rows(blk[b], hi - lo)
        x64 = xb.astype(np.float64)
        sq = (x64 * x64).sum(1)[:, None] + cn[None, :] - 2.0 * (x64 @ cen.T)
        s[lo:hi] = np.exp(-teacher_gamma * np.maximum(sq, 0.0)) @ amp
        r, c = np.nonzero(xb)
        idx_parts.append(c.astype(np.int32))
        val_parts.append(xb[r, c])
        indptr[lo + 1:hi + 1] = indptr[lo] + np.cumsum(np.bincount(r, minlength=hi - lo))
    y = np.where(s - np.median(s) >= 0, 1.0, -1.0)
    y = _flip_exact(gl, y, int(np.floor(flip * n)))
    return indptr, np.concatenate(idx_parts), np.concatenate(val_parts), y


def csr_to_dense(indptr, indices, values, d: int) -> np.ndarray:
    """The dense n x d FP64 matrix of CSR rows."""
    n = indptr.shape[0] - 1
    X = np.zeros((n, d))
    rows = np.repeat(np.arange(n), np.diff(indptr))
    X[rows, indices] = values
    return X


# ----------------------------------------------------------------------------------------------
_NAMES = ("blobs-2k", "binary-100k", "onehot-500k", "mnist-60k", "dense-2m")


def config_names():
    return _NAMES


def make_config(name: str, seed: Optional[int] = None, n: Optional[int] = None, J_max: Optional[int] = None):
    """Build a named workload. ``n`` / ``J_max`` shrink it (for tests); ``seed`` overrides the default."""
    if name == "blobs-2k":
        nn = n or 2000
        X, y = make_blobs(nn, 16, 0 if seed is None else seed)
        return Problem(name, X, y, C=1.0, gamma=1.0 / 16, J_max=J_max or 100)
    if name == "binary-100k":
        nn = n or 100000
        X, y = make_binary_sparse(nn, 123, 1 if seed is None else seed)
        return Problem(name, X, y, C=1.0, gamma=0.05, J_max=J_max or 1000)
    if name == "onehot-500k":
        nn = n or 500000
        X, y, info = make_mixed_onehot(nn, 2 if seed is None else seed)
        return Problem(name, X, y, C=10.0, gamma=0.5, J_max=J_max or 3000, info=info)
    if name == "mnist-60k":
        per = (n or 60000) // 10
        s = 3 if seed is None else seed
        X, cls = make_mnist_like(per, 784, s)
        nn = X.shape[0]
        m = J_max or 2000
        basis = np.random.default_rng(np.random.SeedSequence([s, 0xB0515])).choice(nn, size=m, replace=False)
        Cs = np.array([0.1, 1.0, 10.0, 100.0])
        gs = np.array([0.005, 0.01, 0.02, 0.05])
        Y, CC, GG = [], [], []
        for c in range(10):
            for Cv in Cs:
                for gv in gs:
                    Y.append(np.where(cls == c, 1.0, -1.0))
                    CC.append(Cv)
                    GG.append(gv)
        return BatchProblem(name, X, np.stack(Y), np.array(CC), np.array(GG), np.sort(basis).astype(np.int64),
                            info={"classes": cls})
    if name == "dense-2m":
        nn = n or 2000000
        X, y = make_large_dense(nn, 2000, 4 if seed is None else seed)
        return Problem(name, X, y, C=1.0, gamma=1.0 / 2000, J_max=J_max or 4000)
    raise ValueError(f"unknown workload {name!r}; known: {_NAMES}")
