"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks one part of the oracle against a closed form, a published value, a brute-force
enumeration, the dual problem, or a derivative-free search. The helpers return an error measure so
that ``test_oracle_mutations.py`` can plant mistakes in the oracle and check that these pins catch them.
"""

import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import rng as orng
from oracle import spsvm as osp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.strip() for ln in fh if ln.strip() and not ln.startswith("#")]


# ------------------------------------------------------------------------------------------------ kernel
def rbf_closed_form_error():
    err = 0.0
    for ln in _golden_lines("rbf_closed_form.txt"):
        xs, zs, g, d2 = [p.strip() for p in ln.split(";")]
        x = np.array([float(v) for v in xs.split(",")])
        z = np.array([float(v) for v in zs.split(",")])
        want = math.exp(-float(g) * float(d2))
        got = oracle.rbf_block(x[None], z[None], float(g))[0, 0]
        err = max(err, abs(got - want) / want)
    return err


def test_rbf_closed_form():
    assert rbf_closed_form_error() < 1e-15


def test_rbf_diagonal_and_symmetry():
    r = np.random.default_rng(0)
    X = r.standard_normal((37, 11))
    K = oracle.rbf_block(X, X, 0.3)
    assert np.array_equal(np.diag(K), np.ones(37))
    assert np.array_equal(K, K.T)
    assert np.all((K > 0) & (K <= 1))


def test_rbf_c_and_numpy_agree():
    from oracle.kernel import rbf_block_numpy

    r = np.random.default_rng(1)
    X = r.standard_normal((50, 13))
    Z = r.standard_normal((7, 13))
    a = oracle.rbf_block(X, Z, 0.2)
    b = rbf_block_numpy(X, Z, 0.2)
    assert np.max(np.abs(a - b)) < 1e-15


# ------------------------------------------------------------------------------------------------ RNG
def test_splitmix64_published_outputs():
    want = [int(v, 16) for v in _golden_lines("splitmix64_seed0.txt")]
    assert orng.splitmix64_stream(0, len(want)) == want


def test_candidate_draw_rules():
    n, kappa = 1000, 59
    blocked = set(range(0, 1000, 3))
    c = orng.draw_candidates(7, 5, n, kappa, lambda i: i in blocked)
    assert len(c) == kappa and len(set(c)) == kappa
    assert all(0 <= i < n and i not in blocked for i in c)
    # the same step of the same seed draws the same indices; another step draws others
    assert c == orng.draw_candidates(7, 5, n, kappa, lambda i: i in blocked)
    assert c != orng.draw_candidates(7, 6, n, kappa, lambda i: i in blocked)
    # few rows available: fewer than kappa candidates, after at most 64 kappa attempts
    c2 = orng.draw_candidates(7, 5, 10, kappa, lambda i: i != 3)
    assert c2 == [3]


def stream_start_mismatches():
    """First candidate indices of an addition step against the values worked by hand from the published
    generator (golden file): pins where a step's stream starts (seed XOR (t 2^32 + 1) GOLDEN)."""
    bad = 0
    for ln in _golden_lines("candidate_stream_start.txt"):
        seed, t, n, idx = [p.strip() for p in ln.split(";")]
        want = [int(v) for v in idx.split(",")]
        got = orng.draw_candidates(int(seed, 0), int(t), int(n), len(want), lambda i: False)
        bad += int(got != want)
    return bad


def test_candidate_stream_start():
    assert stream_start_mismatches() == 0


def consecutive_step_overlap(seeds=(0, 1, 12345), steps=12, n=10**9, kappa=59):
    """Largest number of candidates two consecutive steps share. Section 4 draws a fresh random subset at each
    step; among 10^9 rows two independent draws of 59 share one with probability below 4e-6."""
    worst = 0
    for seed in seeds:
        prev = None
        for t in range(steps):
            cur = set(orng.draw_candidates(seed, t, n, kappa, lambda i: False))
            if prev is not None:
                worst = max(worst, len(cur & prev))
            prev = cur
    return worst


def test_consecutive_steps_draw_fresh_subsets():
    assert consecutive_step_overlap() == 0


def test_candidate_index_is_high_bits_scaled():
    # index = floor(hi32(z) * n / 2^32): check against exact rational arithmetic on the published stream
    z = orng.splitmix64_stream(0, 1)[0]
    for n in (1, 2, 123, 100000, 2**31 + 11):
        assert orng.scaled_index(z, n) == (z >> 32) * n // 2**32
        assert 0 <= orng.scaled_index(z, n) < n


def test_stage_schedule():
    want = [int(v) for v in _golden_lines("stage_schedule_jmax100.txt")[0].split()]
    got, J = [], 0
    while J < 100:
        c = orng.stage_size(J, 100)
        got.append(c)
        J += c
    assert got == want


# --------------------------------------------------------------------------------- one-dimensional solves
def _golden_section(fun, lo, hi, iters=200):
    g = (math.sqrt(5) - 1) / 2
    a, b = lo, hi
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = fun(c), fun(d)
    for _ in range(iters):
        if fc <= fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = fun(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = fun(d)
    return 0.5 * (a + b)


def _phi(a, b, lam, c1, c2, t):
    return lam * (t * c1 + 0.5 * t * t * c2) + 0.5 * float(np.sum(np.maximum(0.0, a - t * b) ** 2))


def line_search_error(seeds=range(20)):
    """max over random piecewise-quadratics of |t* - t_golden| / (1 + t) and of the decrease mismatch."""
    worst = 0.0
    for sd in seeds:
        r = np.random.default_rng(100 + sd)
        n = int(r.integers(5, 200))
        a = r.standard_normal(n) * 2
        b = r.standard_normal(n)
        lam = float(r.uniform(0.01, 3))
        c2 = float(r.uniform(0.1, 5))
        c1 = float(r.standard_normal()) * 3
        if lam * c1 - float(np.sum(b * np.maximum(0, a))) >= 0:
            c1 = -abs(c1) - float(np.sum(np.abs(b) * np.maximum(0, a))) / lam - 1.0  # force a descent direction
        t, dec = osp.exact_line_search(a, b, lam, c1, c2)
        # a dense grid brackets the minimiser, golden section refines it
        hi = 1.0
        while _phi(a, b, lam, c1, c2, hi) < _phi(a, b, lam, c1, c2, hi / 2):
            hi *= 2
        grid = np.linspace(0, hi, 20001)
        vals = np.array([_phi(a, b, lam, c1, c2, v) for v in grid])
        k = int(np.argmin(vals))
        tg = _golden_section(lambda v: _phi(a, b, lam, c1, c2, v), grid[max(k - 1, 0)], grid[min(k + 1, grid.size - 1)])
        worst = max(worst, abs(t - tg) / (1 + abs(tg)))
        direct = _phi(a, b, lam, c1, c2, 0.0) - _phi(a, b, lam, c1, c2, t)
        worst = max(worst, abs(dec - direct) / (1 + abs(direct)))
    return worst


def test_line_search_matches_grid_and_golden_section():
    assert line_search_error() < 1e-7


def test_line_search_no_descent_gives_zero():
    a = np.array([1.0, -1.0])
    b = np.array([-1.0, 1.0])
    assert osp.exact_line_search(a, b, 1.0, 5.0, 1.0) == (0.0, 0.0)


def test_line_search_closed_form_without_breakpoints():
    # every term stays active on [0, t*]: t* = (sum a b - lam c1) / (lam c2 + sum b^2)
    a = np.array([10.0, 12.0, 9.0])
    b = np.array([0.5, 0.25, 1.0])
    lam, c1, c2 = 0.5, -1.0, 2.0
    t, _ = osp.exact_line_search(a, b, lam, c1, c2)
    want = (a @ b - lam * c1) / (lam * c2 + b @ b)
    assert np.all(a - want * b > 0)
    assert abs(t - want) < 1e-15 * want


def score_error(seeds=range(20)):
    worst = 0.0
    for sd in seeds:
        r = np.random.default_rng(200 + sd)
        n = int(r.integers(5, 150))
        a = r.standard_normal(n) * 2
        b = r.standard_normal(n) * r.uniform(0.1, 2)
        lam = float(r.uniform(0.01, 3))
        oc = float(r.standard_normal())

        def psi(s):
            return lam * (s * oc + 0.5 * s * s) + 0.5 * float(np.sum(np.maximum(0.0, a - s * b) ** 2))

        s, dl = osp.score_candidate(a, b, lam, oc)
        R = 1.0
        while psi(R) < psi(R / 2) or psi(-R) < psi(-R / 2):
            R *= 2
        grid = np.linspace(-R, R, 40001)
        vals = np.array([psi(v) for v in grid])
        k = int(np.argmin(vals))
        sg = _golden_section(psi, grid[max(k - 1, 0)], grid[min(k + 1, grid.size - 1)])
        worst = max(worst, abs(s - sg) / (1 + abs(sg)))
        worst = max(worst, abs(dl - (psi(0) - psi(s))) / (1 + abs(dl)))
        assert dl >= 0
    return worst


def test_candidate_score_matches_grid_and_golden_section():
    assert score_error() < 1e-7


# -------------------------------------------------------------------------------------- Newton, fixed J
def _tiny(n, d, seed, dup=False):
    r = np.random.default_rng(seed)
    X = r.standard_normal((n, d))
    y = np.where(r.standard_normal(n) + X[:, 0] > 0, 1.0, -1.0)
    if dup:
        X[1] = X[0]
    return X, y


def violator_enumeration_error(seeds=range(6)):
    """For tiny n, the optimum at fixed J is the unique self-consistent violator set's solution."""
    worst = 0.0
    for sd in seeds:
        n, d = 10, 3
        X, y = _tiny(n, d, 300 + sd)
        J = np.array([0, 3, 7, 8])
        C, gamma = [0.5, 2.0, 10.0][sd % 3], 0.4
        K = oracle.rbf_block(X, X[J], gamma)
        KJJ = K[J]
        lam = 1 / C
        consistent = []
        for mask in itertools.product([False, True], repeat=n):
            I = np.array(mask)
            H = lam * KJJ + K[I].T @ K[I]
            beta = np.linalg.solve(H, K[I].T @ y[I])
            if np.array_equal(y * (K @ beta) < 1, I):
                consistent.append(beta)
        assert len(consistent) == 1
        beta, F, _ = osp.solve_fixed_J(X, y, C, gamma, J)
        worst = max(worst, float(np.max(np.abs(beta - consistent[0])) / (1 + np.max(np.abs(consistent[0])))))
    return worst


def test_newton_matches_violator_enumeration():
    assert violator_enumeration_error() < 1e-9


def dual_qp_error(seeds=range(5)):
    """J = all points is Chapelle's primal (Eq. 3). Its optimum equals the L2-SVM dual
    max_{alpha >= 0} sum alpha - 1/2 alpha^T Q alpha - |alpha|^2 / (2C), Q = (y y^T) * K, solved by
    enumerating supports; beta = y * alpha and primal = dual."""
    worst = 0.0
    for sd in seeds:
        n = 9
        X, y = _tiny(n, 2, 400 + sd)
        C, gamma = [0.7, 3.0, 20.0, 1.0, 5.0][sd], 0.6
        K = oracle.rbf_block(X, X, gamma)
        Q = np.outer(y, y) * K
        found = []
        for mask in itertools.product([False, True], repeat=n):
            S = np.array(mask)
            alpha = np.zeros(n)
            if S.any():
                alpha[S] = np.linalg.solve(Q[np.ix_(S, S)] + np.eye(S.sum()) / C, np.ones(S.sum()))
            if np.any(alpha[S] < 0):
                continue
            if np.any((Q @ alpha)[~S] < 1):
                continue
            found.append(alpha)
        assert len(found) == 1
        alpha = found[0]
        dual = alpha.sum() - 0.5 * alpha @ Q @ alpha - alpha @ alpha / (2 * C)
        beta, F, _ = osp.solve_fixed_J(X, y, C, gamma, np.arange(n))
        worst = max(worst, abs(F - dual) / abs(dual))
        worst = max(worst, float(np.max(np.abs(beta - y * alpha)) / (1 + np.max(np.abs(alpha)))))
    return worst


def test_full_basis_matches_dual_qp():
    assert dual_qp_error() < 1e-10


def kernel_ridge_error():
    """With a tiny C every point stays a violator and the optimum is a ridge solve."""
    X, y = _tiny(60, 4, 500)
    J = np.arange(0, 60, 4)
    C, gamma = 1e-3, 0.3
    K = oracle.rbf_block(X, X[J], gamma)
    lam = 1 / C
    want = np.linalg.solve(lam * K[J] + K.T @ K, K.T @ y)
    assert np.all(y * (K @ want) < 1)
    beta, F, _ = osp.solve_fixed_J(X, y, C, gamma, J)
    Kf = oracle.rbf_block(X, X, gamma)
    full = np.linalg.solve(lam * Kf + Kf @ Kf, Kf @ y)  # J = all points: (lam I + K) beta = y when K is PD
    assert np.all(y * (Kf @ full) < 1)
    betaf, _, _ = osp.solve_fixed_J(X, y, C, gamma, np.arange(60))
    return max(float(np.max(np.abs(beta - want)) / np.max(np.abs(want))),
               float(np.max(np.abs(betaf - full)) / np.max(np.abs(full))))


def test_kernel_ridge_special_case():
    assert kernel_ridge_error() < 1e-9


def test_gradient_vanishes_at_solution_exact_sum():
    X, y = _tiny(300, 5, 600)
    J = np.arange(0, 300, 10)
    C, gamma = 4.0, 0.25
    beta, F, info = osp.solve_fixed_J(X, y, C, gamma, J)
    K = oracle.rbf_block(X, X[J], gamma)
    o = [math.fsum(K[i, k] * beta[k] for k in range(J.size)) for i in range(300)]
    a = [1 - y[i] * o[i] for i in range(300)]
    g = [math.fsum([o[J[k]] / C] + [-y[i] * a[i] * K[i, k] for i in range(300) if a[i] > 0]) for k in range(J.size)]
    scale = math.fsum(abs(y[i] * a[i] * K[i, k]) for k in range(J.size) for i in range(300) if a[i] > 0)
    assert max(abs(v) for v in g) <= 1e-12 * scale


# ------------------------------------------------------------------------------------- selection, train
def selection_bruteforce_mismatches(n=40, steps=12, seed=700):
    """Replays the oracle's first additions: for each drawn candidate set, the best candidate by a direct
    search (append the column, minimise the full objective over the new coefficient by golden section)
    must be the one the oracle picked, with the same objective."""
    X, y = _tiny(n, 3, seed)
    C, gamma = 2.0, 0.5
    lam = 1 / C
    res = osp.train(X, y, C, gamma, J_max=steps, seed=3, kappa=6)
    J, beta = [], np.zeros(0)
    mism = 0
    groups = osp.duplicate_groups(X)
    t = 0
    # replay the first stages (|J| < 8 gives one addition per stage)
    for step in range(min(steps, 8)):
        used = set(groups[j] for j in J)
        cands = orng.draw_candidates(3, t, n, 6, lambda i: groups[i] in used)
        best = None
        for c in cands:
            Jc = J + [c]
            K = oracle.rbf_block(X, X[Jc], gamma)

            def f(s):
                return osp.objective(K, K[Jc], y, np.append(beta, s), lam)

            R = 1.0
            while f(R) < f(R / 2) or f(-R) < f(-R / 2):
                R *= 2
            grid = np.linspace(-R, R, 4001)
            k = int(np.argmin([f(v) for v in grid]))
            s = _golden_section(f, grid[max(k - 1, 0)], grid[min(k + 1, 4000)])
            val = f(s)
            if best is None or val < best[0] - 1e-12 or (abs(val - best[0]) <= 1e-12 and c < best[1]):
                best = (val, c, s)
        J.append(best[1])
        if best[1] != res.J[step]:
            mism += 1
        # Newton after the stage, from the greedy coefficient
        K = oracle.rbf_block(X, X[J], gamma)
        beta, _ = osp.newton_solve(K, K[J], y, lam, np.append(beta, best[2]))
        t += 1
    return mism


def test_selection_matches_bruteforce():
    assert selection_bruteforce_mismatches() == 0


def test_train_monotone_and_consistent():
    X, y = _tiny(400, 4, 800)
    res = osp.train(X, y, 1.0, 0.5, J_max=40, seed=1)
    ft = np.array(res.f_trace)
    assert np.all(np.diff(ft) <= 1e-12 * ft[0])
    assert len(res.J) == 40 and len(set(res.J.tolist())) == 40
    assert sum(res.stages) == 40
    # the returned objective equals the objective recomputed from (J, beta)
    F = osp.objective_at(X, y, 1.0, 0.5, res.J, res.beta)
    assert abs(F - res.F) <= 1e-12 * F
    # the final beta is the optimum for its J
    beta2, F2, _ = osp.solve_fixed_J(X, y, 1.0, 0.5, res.J)
    assert abs(F2 - res.F) <= 1e-10 * F2


def test_duplicate_rows_never_share_the_basis():
    r = np.random.default_rng(900)
    base = r.standard_normal((30, 3))
    X = np.concatenate([base, base, base[:10]])  # 70 rows, 30 distinct
    y = np.where(X[:, 0] + 0.3 * r.standard_normal(70) > 0, 1.0, -1.0)
    y[30:60] = y[:30]
    y[60:] = y[:10]
    res = osp.train(X, y, 1.0, 0.5, J_max=30, seed=2, kappa=8)
    g = osp.duplicate_groups(X)
    assert len(set(g[res.J].tolist())) == len(res.J)
    with pytest.raises(ValueError):
        osp.train(X, y, 1.0, 0.5, J_max=31)


def test_argument_validation():
    X, y = _tiny(20, 2, 1)
    with pytest.raises(ValueError):
        osp.train(X, y, 0.0, 0.5, 5)
    with pytest.raises(ValueError):
        osp.train(X, y, 1.0, -1.0, 5)
    bad = y.copy()
    bad[3] = 0.5
    with pytest.raises(ValueError):
        osp.train(X, bad, 1.0, 0.5, 5)
    Xn = X.copy()
    Xn[2, 1] = np.nan
    with pytest.raises(ValueError):
        osp.train(Xn, y, 1.0, 0.5, 5)


def _indefinite(lam_min, seed=0):
    """H = Q diag(120, 80, 40, 20, 10, lam_min) Q^T with a random orthogonal Q: mean diagonal (270 + lam_min) / 6,
    about 45, and one eigenvalue lam_min < 0 far above the rounding of the entries (~1e-14)."""
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.standard_normal((6, 6)))
    H = (Q * np.array([120.0, 80.0, 40.0, 20.0, 10.0, lam_min])) @ Q.T
    return 0.5 * (H + H.T)


def jitter_error():
    """The retry adds mu * mean(diag H) to the diagonal, mu = 1e-14, 1e-12, 1e-10, 1e-8 in turn. With the smallest
    eigenvalue -1e-9 and mean diagonal ~45 the shifts are 4.5e-13, 4.5e-11 (still indefinite) and 4.5e-9 (PD), so
    the factor must reproduce H + 1e-10 mean(diag H) I; with -1e-7 only the last shift (4.5e-7) succeeds. Returns
    the largest deviation of L L^T from those matrices, relative to the largest entry of H."""
    worst = 0.0
    for lam_min, mu in ((-1e-9, 1e-10), (-1e-7, 1e-8)):
        H = _indefinite(lam_min)
        with pytest.raises(np.linalg.LinAlgError):
            np.linalg.cholesky(H)  # the retry path is taken
        L = osp.cholesky_jitter(H)
        want = H + mu * (np.trace(H) / 6) * np.eye(6)
        worst = max(worst, float(np.max(np.abs(L @ L.T - want)) / np.max(np.abs(H))))
    return worst


def test_cholesky_jitter_scale_and_order():
    assert jitter_error() < 1e-13


def test_cholesky_jitter_gives_up():
    with pytest.raises(osp.NotPositiveDefinite):
        osp.cholesky_jitter(_indefinite(-1e-5))  # the largest shift, 4.5e-7, leaves it indefinite
    with pytest.raises(osp.NotPositiveDefinite):
        osp.cholesky_jitter(np.array([[1.0, 0.0], [0.0, -1.0]]))
    H = np.array([[4.0, 2.0], [2.0, 3.0]])  # PD: no jitter at all
    assert np.array_equal(osp.cholesky_jitter(H), np.linalg.cholesky(H))


# ----------------------------------------------------------------------------- stages of several additions
def _dup_groups(X):
    """Row groups by exact equality of the feature vectors, computed here rather than by the oracle."""
    seen, out = {}, np.empty(X.shape[0], dtype=np.int64)
    for i, row in enumerate(map(tuple, np.asarray(X, dtype=np.float64))):
        out[i] = seen.setdefault(row, len(seen))
    return out


def stage_replay(n=45, J_max=14, kappa=12, growth=1.0, draw_seed=4, data_seed=710):
    """Brute-force replay of the oracle's greedy growth over stages that add several vectors (growth 1 gives
    stages of 1, 1, 2, 4, 6 additions). Every row has two exact duplicates. Per stage: candidates are drawn with
    J as it stood at the stage start blocked (members and their duplicates); a drawn row whose duplicate group
    won earlier in the same stage is skipped; each remaining candidate is appended and the full objective is
    minimised over its coefficient by golden section, the lowest value winning (lower row on ties); Newton
    after the stage. Returns (mismatching additions, additions made in stages of 2 or more, same-stage
    duplicates skipped)."""
    r = np.random.default_rng(data_seed)
    base = r.standard_normal((n // 3, 3))
    X = np.concatenate([base, base, base])
    y = np.where(X[:, 0] + 0.4 * r.standard_normal(n) > 0, 1.0, -1.0)
    C, gamma = 2.0, 0.5
    lam = 1 / C
    res = osp.train(X, y, C, gamma, J_max=J_max, seed=draw_seed, kappa=kappa, growth=growth)
    grp = _dup_groups(X)
    J, beta, t = [], np.zeros(0), 0
    multi = skipped = mism = 0
    while len(J) < J_max:
        cs = min(J_max - len(J), max(1, int(math.floor(growth * len(J)))))
        frozen = {grp[j] for j in J}
        for q in range(cs):
            cands = orng.draw_candidates(draw_seed, t + q, n, kappa, lambda i: grp[i] in frozen)
            best = None
            for c in cands:
                if grp[c] in {grp[j] for j in J}:
                    assert grp[c] not in frozen
                    skipped += 1
                    continue
                Jc = J + [c]
                K = oracle.rbf_block(X, X[Jc], gamma)

                def f(s):
                    return osp.objective(K, K[Jc], y, np.append(beta, s), lam)

                R = 1.0
                while f(R) < f(R / 2) or f(-R) < f(-R / 2):
                    R *= 2
                grid = np.linspace(-R, R, 4001)
                k = int(np.argmin([f(v) for v in grid]))
                s = _golden_section(f, grid[max(k - 1, 0)], grid[min(k + 1, 4000)])
                val = f(s)
                if best is None or val < best[0] - 1e-12 or (abs(val - best[0]) <= 1e-12 and c < best[1]):
                    best = (val, c, s)
            # exact duplicates give identical columns, and their scores differ only by rounding of o (the
            # oracle's products may round identical rows differently): the pick must be the same group, and
            # the replay goes on with the oracle's row
            k = len(J)
            if k >= len(res.J) or grp[res.J[k]] != grp[best[1]]:
                mism += 1
                J.append(best[1])
            else:
                J.append(int(res.J[k]))
            beta = np.append(beta, best[2])
            multi += int(cs >= 2)
        K = oracle.rbf_block(X, X[J], gamma)
        beta, _ = osp.newton_solve(K, K[J], y, lam, beta)
        t += cs
    return mism + abs(len(J) - len(res.J)), multi, skipped


def test_multi_addition_stages_match_bruteforce_replay():
    mism, multi, skipped = stage_replay()
    assert multi >= 8 and skipped >= 1  # the stage-level rules are exercised
    assert mism == 0


# ------------------------------------------------------------------------------------ offset b (Eq. 4 with bias)
def dual_qp_bias_error(seeds=range(5)):
    """J = all points with the offset b: Eq. 3 with b. Its dual is the L2-SVM dual of the previous pin with the
    equality constraint sum y_i alpha_i = 0, whose multiplier is b. Supports S are enumerated: on S,
    (Q_SS + I / C) alpha_S + y_S b = 1 and y_S^T alpha_S = 0; accepted when alpha_S > 0 and every i outside S has
    (Q alpha)_i + y_i b >= 1. At the optimum beta = y * alpha, the offsets agree and primal = dual."""
    worst = 0.0
    for sd in seeds:
        n = 9
        X, y = _tiny(n, 2, 450 + sd)
        C, gamma = [0.7, 3.0, 20.0, 1.0, 5.0][sd], 0.6
        K = oracle.rbf_block(X, X, gamma)
        Q = np.outer(y, y) * K
        found = []
        for mask in itertools.product([False, True], repeat=n):
            S = np.array(mask)
            k = int(S.sum())
            if k == 0 or abs(int(np.sum(y[S]))) == k:  # both classes are needed for sum y alpha = 0 with alpha > 0
                continue
            M = np.zeros((k + 1, k + 1))
            M[:k, :k] = Q[np.ix_(S, S)] + np.eye(k) / C
            M[:k, k] = y[S]
            M[k, :k] = y[S]
            sol = np.linalg.solve(M, np.concatenate([np.ones(k), [0.0]]))
            alpha = np.zeros(n)
            alpha[S] = sol[:k]
            b = sol[k]
            if np.any(alpha[S] <= 0) or np.any((Q @ alpha + y * b)[~S] < 1):
                continue
            found.append((alpha, b))
        assert len(found) == 1
        alpha, b = found[0]
        dual = alpha.sum() - 0.5 * alpha @ Q @ alpha - alpha @ alpha / (2 * C)
        beta, F, info = osp.solve_fixed_J(X, y, C, gamma, np.arange(n), bias=True)
        worst = max(worst, abs(F - dual) / abs(dual), abs(info.bias - b) / (1 + abs(b)))
        worst = max(worst, float(np.max(np.abs(beta - y * alpha)) / (1 + np.max(np.abs(alpha)))))
    return worst


def test_full_basis_with_offset_matches_dual_qp():
    assert dual_qp_bias_error() < 1e-10


def selection_bias_mismatches(n=40, steps=8, seed=705):
    """The oracle's first additions with the offset: for each drawn candidate set, the best candidate by a direct
    search (append the column, minimise the full objective over the new coefficient with b and the other
    coefficients fixed) must be the one the oracle picked; Newton on (b, beta) after each stage."""
    X, y = _tiny(n, 3, seed)
    y = np.where(np.arange(n) % 4 == 0, 1.0, y)  # unbalanced classes, so b matters
    C, gamma = 2.0, 0.5
    lam = 1 / C
    res = osp.train(X, y, C, gamma, J_max=steps, seed=3, kappa=6, bias=True)
    J, th, mism, t = [], np.zeros(1), 0, 0
    grp = _dup_groups(X)
    for step in range(steps):
        used = {grp[j] for j in J}
        cands = orng.draw_candidates(3, t, n, 6, lambda i: grp[i] in used)
        best = None
        for c in cands:
            Jc = J + [c]
            A, R = osp._with_offset(oracle.rbf_block(X, X[Jc], gamma), oracle.rbf_block(X[Jc], X[Jc], gamma))

            def f(s):
                return osp.objective(A, R, y, np.append(th, s), lam)

            Rr = 1.0
            while f(Rr) < f(Rr / 2) or f(-Rr) < f(-Rr / 2):
                Rr *= 2
            grid = np.linspace(-Rr, Rr, 4001)
            k = int(np.argmin([f(v) for v in grid]))
            s = _golden_section(f, grid[max(k - 1, 0)], grid[min(k + 1, 4000)])
            if best is None or f(s) < best[0] - 1e-12 or (abs(f(s) - best[0]) <= 1e-12 and c < best[1]):
                best = (f(s), c, s)
        J.append(best[1])
        mism += int(best[1] != res.J[step])
        A, R = osp._with_offset(oracle.rbf_block(X, X[J], gamma), oracle.rbf_block(X[J], X[J], gamma))
        th, _ = osp.newton_solve(A, R, y, lam, np.append(th, best[2]))
        t += 1
    return mism + int(abs(th[0] - res.b) > 1e-8 * (1 + abs(res.b)))


def test_selection_with_offset_matches_bruteforce():
    assert selection_bias_mismatches() == 0


# ------------------------------------------------------------------------------------------ stopping rule
def stop_rule_mismatches():
    """The stopping rule (section 4, implementation paragraph; eps = 5e-6 in section 5, larger here for a short
    trace) on two recorded runs: a steadily improving one (binary rows, eps 3e-3: it stops after a stage of two
    additions whose decrease, 17 rows of 3000, is 2.8e-3 per added vector but 5.7e-3 in all) and one whose error
    rises at a stage (blobs, eps 1e-3). The training error after each stage is
    recomputed outside the training loop, from the model a run with J_max at that stage's basis size returns
    (decision values by the prediction routine, errors y_i o_i <= 0, 1 at o = 0), and the run must stop exactly at
    the first stage whose decrease per added vector is below eps."""
    import datagen

    bad = 0
    p = datagen.make_config("binary-100k", n=3000)
    Xb, yb = datagen.make_blobs(600, 6, seed=17)
    for X, y, C, gamma, eps in ((p.X, p.y, p.C, p.gamma, 3e-3), (Xb, yb, 1.0, 1 / 6, 1e-3)):
        X = np.asarray(X, dtype=np.float64)
        run = osp.train(X, y, C, gamma, 300, seed=2, bias=True, eps_stop=eps)
        sizes = np.cumsum(run.stages)
        errs, prev, stop_at = [], 1.0, None
        for k, m in enumerate(sizes):
            r = osp.train(X, y, C, gamma, int(m), seed=2, bias=True)
            e = float(np.mean(y * oracle.predict(X[r.J], r.beta, gamma, X, r.b) <= 0))
            errs.append(e)
            if stop_at is None and (prev - e) / run.stages[k] < eps:
                stop_at = k
            prev = e
        bad += int(run.stop != "eps" or stop_at != len(run.stages) - 1)
        bad += int(np.max(np.abs(np.array(errs) - np.array(run.errors))) > 1.0 / X.shape[0])
    return bad


def test_stopping_rule_on_recorded_traces():
    assert stop_rule_mismatches() == 0


# ---------------------------------------------------------------------------------- one-vs-one multiclass
def ovo_vote_mismatches():
    bad = 0
    for ln in _golden_lines("ovo_votes.txt"):
        K, dec, want = [p.strip() for p in ln.split(";")]
        d = np.array([[float(v) for v in dec.split(",")]])
        bad += int(osp.ovo_vote(d, int(K))[0] != int(want))
    return bad


def test_ovo_voting_matches_hand_worked_cases():
    assert ovo_vote_mismatches() == 0


def ovo_subset_mismatches():
    """Each pairwise classifier is greedy training on exactly the rows of its two classes (extracted here row by row,
    labels +1 for the first class): same basis (as rows of X) and coefficients; with two classes the one pair is
    the binary problem itself."""
    import datagen

    X, cls = datagen.make_mnist_like(per_class=40, d=6, seed=11, classes=4)
    X = X.astype(np.float64)
    bad = 0
    models = osp.train_ovo(X, cls, 4, 2.0, 0.5, 12, seed=1, kappa=10)
    for (res, rows), (a, b) in zip(models, osp.ovo_pairs(4)):
        sub = [i for i in range(X.shape[0]) if cls[i] in (a, b)]
        ys = np.array([1.0 if cls[i] == a else -1.0 for i in sub])
        ref = osp.train(X[sub], ys, 2.0, 0.5, 12, seed=1, kappa=10)
        bad += int(list(rows) != sub or ref.J.tolist() != res.J.tolist() or not np.array_equal(ref.beta, res.beta))
    two = osp.train_ovo(X, np.minimum(cls, 1), 2, 2.0, 0.5, 12, seed=1, kappa=10)
    ref = osp.train(X, np.where(np.minimum(cls, 1) == 0, 1.0, -1.0), 2.0, 0.5, 12, seed=1, kappa=10)
    bad += int(two[0][0].J.tolist() != ref.J.tolist())
    return bad


def test_ovo_pairs_train_on_their_rows():
    assert ovo_subset_mismatches() == 0


# ----------------------------------------------------------------------------- shared basis for a batch of problems
def shared_single_mismatches():
    """One problem, and two identical copies of it: the shared growth is the single-problem growth (same basis,
    same coefficients; two equal decreases add up exactly to twice one, so the order of the sums is unchanged)."""
    X, y = _tiny(60, 3, 720)
    a = osp.train(X, y, 2.0, 0.5, 12, seed=3, kappa=6)
    bad = 0
    for Y in (y[None], np.stack([y, y])):
        b = osp.train_shared(X, Y, 2.0, 0.5, 12, seed=3, kappa=6)
        bad += int(not np.array_equal(a.J, b.J))
        bad += sum(int(not np.array_equal(a.beta, row)) for row in b.beta)
        bad += sum(int(F != a.F) for F in b.F)
    return bad


def _shared_tiny(n, seed):
    r = np.random.default_rng(seed)
    X = r.standard_normal((n, 3))
    Y = np.stack([np.where(X[:, 0] + 0.3 * r.standard_normal(n) > 0, 1.0, -1.0),
                  np.where(X[:, 1] - 0.5 * X[:, 2] > 0.2, 1.0, -1.0),
                  np.where(X[:, 0] * X[:, 1] > 0, 1.0, -1.0)])
    return X, Y, np.array([2.0, 0.5, 8.0]), np.array([0.5, 0.5, 1.5])


def shared_replay(n=40, steps=8, seed=725, growth=0.25):
    """Brute-force replay of the shared growth of three problems (own labels, C and gamma): each drawn candidate is
    appended to every problem, each problem's full objective is minimised over its new coefficient by golden
    section, and the candidate with the largest sum of the problems' decreases must be the oracle's pick; the
    winner enters every problem with that problem's coefficient, and every problem is re-optimised by Newton after
    the stage (growth 0.25: one addition per stage here; growth 1: stages of 1, 1, 2, 4, ..., whose later picks
    depend on the coefficients of the earlier ones). Draws block J as it stood at the stage start; a drawn row
    already in J is skipped. Returns (mismatches, steps at which the problems' own best candidates differ)."""
    X, Y, C, gamma = _shared_tiny(n, seed)
    lam = 1.0 / C
    res = osp.train_shared(X, Y, C, gamma, J_max=steps, seed=3, kappa=6, growth=growth)
    groups = _dup_groups(X)
    J, betas = [], [np.zeros(0) for _ in range(3)]
    mism = disagree = 0
    t = 0
    while len(J) < steps:
        cs = min(steps - len(J), max(1, int(math.floor(growth * len(J)))))
        frozen = {groups[j] for j in J}
        for q in range(cs):
            cands = orng.draw_candidates(3, t + q, n, 6, lambda i: groups[i] in frozen)
            best, own = None, [None] * 3
            for c in cands:
                if groups[c] in {groups[j] for j in J}:
                    continue
                Jc = J + [c]
                total, ss = 0.0, []
                for p in range(3):
                    K = oracle.rbf_block(X, X[Jc], gamma[p])

                    def f(s):
                        return osp.objective(K, K[Jc], Y[p], np.append(betas[p], s), lam[p])

                    R = 1.0
                    while f(R) < f(R / 2) or f(-R) < f(-R / 2):
                        R *= 2
                    grid = np.linspace(-R, R, 2001)
                    k = int(np.argmin([f(v) for v in grid]))
                    s = _golden_section(f, grid[max(k - 1, 0)], grid[min(k + 1, 2000)])
                    dec = f(0.0) - f(s)
                    total += dec
                    ss.append(s)
                    if own[p] is None or dec > own[p][0] + 1e-12:
                        own[p] = (dec, c)
                if best is None or total > best[0] + 1e-12 or (abs(total - best[0]) <= 1e-12 and c < best[1]):
                    best = (total, c, ss)
            disagree += int(len({o[1] for o in own}) > 1)
            k = len(J)
            if k >= len(res.J) or best[1] != res.J[k]:
                mism += 1
            J.append(best[1])
            for p in range(3):
                betas[p] = np.append(betas[p], best[2][p])
        for p in range(3):
            K = oracle.rbf_block(X, X[J], gamma[p])
            betas[p], _ = osp.newton_solve(K, K[J], Y[p], lam[p], betas[p])
        t += cs
    for p in range(3):
        mism += int(not np.allclose(betas[p], res.beta[p], rtol=1e-8, atol=1e-10))
    return mism, disagree


def test_shared_basis_single_problem_is_plain_training():
    assert shared_single_mismatches() == 0


def test_shared_basis_matches_bruteforce_replay():
    mism, disagree = shared_replay()
    assert disagree >= 2  # the problems' own best candidates differ: the sum decides
    assert mism == 0


def test_shared_basis_multi_addition_stages_match_bruteforce_replay():
    mism, disagree = shared_replay(n=36, steps=12, seed=731, growth=1.0)
    assert disagree >= 2
    assert mism == 0
