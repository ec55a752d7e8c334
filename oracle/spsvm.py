"""SP-SVM in plain FP64 NumPy: the oracle the GPU library is checked against (test infrastructure only).

Problem (section 4, "Sparse primal optimization", Eq. 4, with the bias omitted as section 2 allows):

    F(beta) = 1/2 beta^T K_JJ beta + C/2 sum_i max(0, 1 - y_i o_i)^2,    o = K_XJ beta,

where K_XJ[i, k] = k(x_i, x_{J_k}) with the RBF kernel of section 2 and K_JJ = K_XJ[J, :]. The code
works with f = F / C, i.e. with lambda = 1 / C on the regulariser:

    f(beta) = lambda/2 beta^T K_JJ beta + 1/2 sum_i max(0, a_i)^2,   a_i = 1 - y_i o_i.

The squared hinge and unconstrained beta are the two relaxations of section 4 ("Primal optimization",
Eq. 3) that make Newton's method applicable. Training alternates greedy basis selection and Newton
re-optimisation of Eq. 4 on the grown basis, as section 4 describes.

Readings of what the paper leaves open (the details are in Keerthi et al., which is not reproduced):

* Bias: b = 0 by default, as section 2 allows; ``bias=True`` fits the offset of Eq. 4 as an unregularised
  coordinate (its kernel column all ones).
* Stopping: J grows to J_max; ``eps_stop`` > 0 adds the rule of section 4 (training-error decrease per added
  vector below eps_stop after a re-optimisation).
* Candidate score: the exact decrease of f when only the new coefficient is optimised, the other
  coefficients held fixed (a one-dimensional convex piecewise-quadratic problem, solved exactly).
* Argmax ties: a strictly larger score wins; equal scores go to the lower training-row index.
* A new basis member enters with its one-dimensional optimum as coefficient; Newton starts from there.
* Duplicate rows (identical feature vectors) give identical kernel columns and a singular K_JJ, so a
  row whose duplicate group already has a basis member is never drawn (as J stood at the start of the
  stage) and scores -inf (as J stands at the time of scoring).
* Newton direction d = -H^{-1} grad f with the generalised Hessian H = lambda K_JJ + K_I^T K_I over the
  violators I = {i : y_i o_i < 1}; step length by exact minimisation of f along d (t >= 0).
  H is re-formed only when I changes. Stop when ||grad f|| <= tol * max(1, ||grad f at entry||), when
  the exact step decreases f by no more than ftol * f, when no descent is possible, or after max_iter
  iterations.
* Cholesky failure: retry with H + mu * mean(diag H) * I for mu in (1e-14, 1e-12, 1e-10, 1e-8), then
  give up (NotPositiveDefinite).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.linalg

from .kernel import rbf_block
from .rng import draw_candidates, stage_size

JITTER = (1e-14, 1e-12, 1e-10, 1e-8)


class NotPositiveDefinite(RuntimeError):
    pass


# ------------------------------------------------------------------------------------------------ objective
def objective(KXJ: np.ndarray, KJJ: np.ndarray, y: np.ndarray, beta: np.ndarray, lam: float) -> float:
    """f(beta) = lambda/2 beta^T K_JJ beta + 1/2 sum max(0, 1 - y_i o_i)^2 (Eq. 4 divided by C)."""
    if beta.size == 0:
        return 0.5 * float(y.shape[0])
    o = KXJ @ beta
    a = 1.0 - y * o
    return 0.5 * lam * float(beta @ (KJJ @ beta)) + 0.5 * float(np.sum(np.maximum(0.0, a) ** 2))


def gradient(KXJ: np.ndarray, KJJ: np.ndarray, y: np.ndarray, beta: np.ndarray, lam: float) -> np.ndarray:
    """grad f = lambda K_JJ beta - sum_{i in I} y_i a_i k_i, with k_i row i of K_XJ."""
    o = KXJ @ beta
    a = 1.0 - y * o
    act = a > 0
    return lam * (KJJ @ beta) - KXJ[act].T @ (y[act] * a[act])


def cholesky_jitter(H: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor of H, with the jitter retry schedule on failure."""
    try:
        return np.linalg.cholesky(H)
    except np.linalg.LinAlgError:
        pass
    scale = float(np.mean(np.diag(H)))
    for mu in JITTER:
        try:
            return np.linalg.cholesky(H + mu * scale * np.eye(H.shape[0]))
        except np.linalg.LinAlgError:
            continue
    raise NotPositiveDefinite("H is not positive definite after the jitter schedule")


# ------------------------------------------------------------------------------------- 1-D exact minimisers
def _segment_root(a, b, lam_c1, lam_c2, rep):
    """Root of the linear piece of the derivative on the segment holding ``rep`` (active set fixed there)."""
    act = a - rep * b > 0
    return (float(np.sum(a[act] * b[act])) - lam_c1) / (lam_c2 + float(np.sum(b[act] * b[act])))


def exact_line_search(a: np.ndarray, b: np.ndarray, lam: float, c1: float, c2: float):
    """Minimise phi(t) = lambda (t c1 + t^2 c2 / 2) + 1/2 sum max(0, a_i - t b_i)^2 over t >= 0.

    With a_i = 1 - y_i o_i, b_i = y_i delta_i (delta = K_XJ d), c1 = beta^T K_JJ d, c2 = d^T K_JJ d this is
    f(beta + t d) up to a constant. phi' is continuous, piecewise linear and increasing. The breakpoints
    a_i / b_i are sorted, the segment holding the root is found by bisection over them (phi' evaluated by
    a full sum each time), and the root is solved on that segment.
    Returns (t*, phi(0) - phi(t*)).
    """
    def dphi(t):
        return lam * (c1 + t * c2) - float(np.sum(b * np.maximum(0.0, a - t * b)))

    if dphi(0.0) >= 0.0:
        return 0.0, 0.0
    nz = b != 0
    bp = a[nz] / b[nz]
    bp = np.unique(bp[bp > 0])
    lo, hi = 0, bp.size
    while lo < hi:  # first breakpoint where phi' >= 0
        mid = (lo + hi) // 2
        if dphi(bp[mid]) >= 0.0:
            hi = mid
        else:
            lo = mid + 1
    left = bp[lo - 1] if lo > 0 else 0.0
    right = bp[lo] if lo < bp.size else math.inf
    rep = 0.5 * (left + right) if math.isfinite(right) else left + 1.0
    t = _segment_root(a, b, lam * c1, lam * c2, rep)
    t = min(max(t, left), right)
    return t, _decrease(a, b, t, lam * c1, lam * c2)


def _decrease(a, b, t, lam_c1, lam_c2):
    """phi(0) - phi(t) summed term by term (no cancellation between two large totals)."""
    a0 = np.maximum(0.0, a)
    at = np.maximum(0.0, a - t * b)
    return 0.5 * float(np.sum((a0 - at) * (a0 + at))) - (t * lam_c1 + 0.5 * t * t * lam_c2)


def score_candidate(a: np.ndarray, b: np.ndarray, lam: float, o_c: float):
    """Exact decrease of f from adding one basis point c with coefficient s, others fixed.

    psi(s) - f = lambda (s o_c + s^2 / 2) + 1/2 sum [max(0, a_i - s b_i)^2 - max(0, a_i)^2],
    with a_i = 1 - y_i o_i, b_i = y_i k(x_i, x_c), o_c = (K_XJ beta)_c and k(x_c, x_c) = 1.
    s ranges over all reals. Returns (s*, Delta = psi(0) - psi(s*) >= 0).
    """
    def dpsi(s):
        return lam * (o_c + s) - float(np.sum(b * np.maximum(0.0, a - s * b)))

    nz = b != 0
    bp = np.unique(a[nz] / b[nz])
    lo, hi = 0, bp.size
    while lo < hi:
        mid = (lo + hi) // 2
        if dpsi(bp[mid]) >= 0.0:
            hi = mid
        else:
            lo = mid + 1
    left = bp[lo - 1] if lo > 0 else -math.inf
    right = bp[lo] if lo < bp.size else math.inf
    if math.isfinite(left) and math.isfinite(right):
        rep = 0.5 * (left + right)
    elif math.isfinite(left):
        rep = left + 1.0
    elif math.isfinite(right):
        rep = right - 1.0
    else:
        rep = 0.0
    s = _segment_root(a, b, lam * o_c, lam, rep)
    s = min(max(s, left), right)
    return s, _decrease(a, b, s, lam * o_c, lam)


# ------------------------------------------------------------------------------------------------- Newton
@dataclasses.dataclass
class NewtonInfo:
    bias: float = 0.0  # the fitted offset b (solve_fixed_J with bias=True)
    iterations: int = 0
    factorizations: int = 0
    grad_norm0: float = 0.0
    grad_norm: float = 0.0
    f_trace: list = dataclasses.field(default_factory=list)
    steps: list = dataclasses.field(default_factory=list)


def newton_solve(KXJ: np.ndarray, KJJ: np.ndarray, y: np.ndarray, lam: float, beta: np.ndarray,
                 tol: float = 1e-10, ftol: float = 1e-14, max_iter: int = 50):
    """Minimise f over beta for a fixed basis (the re-optimisation of Eq. 4), from ``beta``.

    Each iteration: o = K_XJ beta, I = {a_i > 0}, g = grad f; H = lambda K_JJ + K_I^T K_I (re-formed when I
    changed), d = -H^{-1} g by Cholesky, exact line search along d.
    """
    beta = np.array(beta, dtype=np.float64, copy=True)
    info = NewtonInfo()
    if beta.size == 0:
        return beta, info
    fact_act = None
    L = None
    for it in range(max_iter):
        o = KXJ @ beta
        a = 1.0 - y * o
        act = a > 0
        g = gradient(KXJ, KJJ, y, beta, lam)
        gn = float(np.linalg.norm(g))
        if it == 0:
            info.grad_norm0 = gn
        info.grad_norm = gn
        f_now = 0.5 * lam * float(beta @ (KJJ @ beta)) + 0.5 * float(np.sum(np.maximum(0.0, a) ** 2))
        info.f_trace.append(f_now)
        if gn <= tol * max(1.0, info.grad_norm0):
            break
        if fact_act is None or not np.array_equal(fact_act, act):
            H = lam * KJJ + KXJ[act].T @ KXJ[act]
            L = cholesky_jitter(H)
            fact_act = act
            info.factorizations += 1
        d = -scipy.linalg.cho_solve((L, True), g)
        delta = KXJ @ d
        t, dec = exact_line_search(a, y * delta, lam, float(beta @ (KJJ @ d)), float(d @ (KJJ @ d)))
        info.iterations = it + 1
        info.steps.append((t, dec))
        if t == 0.0:
            break
        beta = beta + t * d
        if dec <= ftol * f_now:
            info.f_trace.append(f_now - dec)
            break
    return beta, info


# ------------------------------------------------------------------------------------------- selection
def duplicate_groups(X: np.ndarray) -> np.ndarray:
    """Group id per row: rows with identical feature vectors share an id."""
    _, inv = np.unique(np.asarray(X, dtype=np.float64), axis=0, return_inverse=True)
    return np.asarray(inv).reshape(-1)


@dataclasses.dataclass
class TrainResult:
    J: np.ndarray
    beta: np.ndarray
    F: float  # paper-scale objective C * f
    f_trace: list  # f after every addition and every Newton iterate (must not increase)
    gaps: list  # per addition step: (best - second best) / best score
    stages: list  # number of additions per stage
    newton_iters: list
    b: float = 0.0  # offset of Eq. 4 (0 unless trained with bias=True)
    errors: list = dataclasses.field(default_factory=list)  # training error after each re-optimisation (eps_stop)
    stop: str = "J_max"  # "J_max", "eps" (the stopping rule fired), "blocked" (no candidate left) or "max_steps"


def training_error(y: np.ndarray, o: np.ndarray) -> float:
    """Fraction of rows the decision values misclassify (y_i o_i <= 0; a zero output counts as an error)."""
    return float(np.mean(y * o <= 0.0))


def stage_stops(err_prev: float, err: float, added: int, eps_stop: float) -> bool:
    """The stopping rule of section 4: the decrease of the training error over the last re-optimisation, per basis
    vector its stage added, is below eps_stop (an unchanged or larger error stops too)."""
    return (err_prev - err) / added < eps_stop


def _with_offset(KXJ: np.ndarray, KJJ: np.ndarray):
    """Design and regulariser matrices of Eq. 4 with the offset b as an extra coordinate (first): its kernel column
    is all ones, its regulariser row and column are zero, so f(b, beta) keeps the form of the objective above."""
    n, m = KXJ.shape
    A = np.concatenate([np.ones((n, 1)), KXJ], axis=1)
    R = np.zeros((m + 1, m + 1))
    R[1:, 1:] = KJJ
    return A, R


def _validate(X, y, C, gamma, J_max, groups):
    if not (np.isfinite(C) and C > 0 and np.isfinite(gamma) and gamma > 0):
        raise ValueError("C and gamma must be finite and positive")
    if not np.all((y == 1.0) | (y == -1.0)):
        raise ValueError("labels must be exactly +1 or -1")
    if not np.all(np.isfinite(X)):
        raise ValueError("X holds NaN or Inf")
    if not (1 <= J_max <= int(groups.max()) + 1):
        raise ValueError("J_max must lie in [1, number of distinct rows]")


def train(X: np.ndarray, y: np.ndarray, C: float, gamma: float, J_max: int, seed: int = 0, kappa: int = 59,
          growth: float = 0.25, cap: int = 256, tol: float = 1e-10, ftol: float = 1e-14, max_iter: int = 50,
          max_steps: Optional[int] = None, bias: bool = False, eps_stop: float = 0.0) -> TrainResult:
    """Greedy basis growth with Newton re-optimisation after each stage (section 4).

    ``max_steps`` (timing samples only) stops after that many addition steps, skipping the final Newton.
    ``bias``: fit the offset b of Eq. 4 (o_i = k_i^T beta + b, b not regularised). The Newton solves treat it as one
    more coordinate (see ``_with_offset``); a selection step keeps it fixed, so a candidate's regulariser cross term
    uses (K beta)_c = o_c - b.
    ``eps_stop`` > 0: the stopping rule of section 4 ("Sparse primal optimization", implementation paragraph), with
    the value 5e-6 of section 5: after each re-optimisation, stop when the decrease of the training error since the
    previous re-optimisation, divided by the number of basis vectors the stage added, is below eps_stop. Training
    error: the fraction of rows with y_i o_i <= 0 (1 at o = 0, before the first stage); a stage that leaves the
    error unchanged or raises it stops training. J_max stays an upper bound.
    """
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = X.shape[0]
    groups = duplicate_groups(X)
    _validate(X, y, C, gamma, J_max, groups)
    lam = 1.0 / C
    J: list[int] = []
    beta = np.zeros(0)
    b = 0.0
    KXJ = np.zeros((n, 0))
    o = np.zeros(n)
    used_groups: set = set()
    f_trace = [0.5 * n]
    gaps, stages, newton_iters, errors = [], [], [], []
    err_prev = training_error(y, o)
    stop = "J_max"
    t = 0
    while len(J) < J_max:
        cs = stage_size(len(J), J_max, growth, cap)
        frozen = set(used_groups)
        draws = [draw_candidates(seed, t + q, n, kappa, lambda i: groups[i] in frozen) for q in range(cs)]
        added = 0
        new_cols = []
        for q in range(cs):
            best = None  # (score, index, s, column)
            second = -math.inf
            a = 1.0 - y * o
            for c in draws[q]:
                if groups[c] in used_groups:
                    continue
                k = rbf_block(X, X[c:c + 1], gamma)[:, 0]
                s, dl = score_candidate(a, y * k, lam, float(o[c]) - b)
                if best is None or dl > best[0] or (dl == best[0] and c < best[1]):
                    if best is not None:
                        second = max(second, best[0])
                    best = (dl, c, s, k)
                else:
                    second = max(second, dl)
            if best is None:
                continue
            dl, c, s, k = best
            gaps.append((dl - second) / dl if dl > 0 and math.isfinite(second) else math.inf)
            J.append(c)
            used_groups.add(groups[c])
            beta = np.append(beta, s)
            o = o + s * k
            new_cols.append(k)
            f_trace.append(f_trace[-1] - dl)
            added += 1
        t += cs
        stages.append(added)
        if added == 0:
            stop = "blocked"
            break
        KXJ = np.concatenate([KXJ, np.stack(new_cols, axis=1)], axis=1)
        if max_steps is not None and t >= max_steps:
            stop = "max_steps"
            break
        KJJ = KXJ[J, :]
        if bias:
            A, R = _with_offset(KXJ, KJJ)
            th, info = newton_solve(A, R, y, lam, np.concatenate([[b], beta]), tol=tol, ftol=ftol, max_iter=max_iter)
            b, beta = float(th[0]), th[1:]
            o = A @ th
        else:
            beta, info = newton_solve(KXJ, KJJ, y, lam, beta, tol=tol, ftol=ftol, max_iter=max_iter)
            o = KXJ @ beta
        newton_iters.append(info.iterations)
        f_trace.extend(info.f_trace[1:])
        if eps_stop > 0.0:
            err = training_error(y, o)
            errors.append(err)
            if stage_stops(err_prev, err, added, eps_stop):
                stop = "eps"
                break
            err_prev = err
    KJJ = KXJ[J, :]
    if bias:
        A, R = _with_offset(KXJ, KJJ)
        F = C * objective(A, R, y, np.concatenate([[b], beta]), lam)
    else:
        F = C * objective(KXJ, KJJ, y, beta, lam)
    return TrainResult(np.array(J, dtype=np.int64), beta, F, f_trace, gaps, stages, newton_iters, b, errors, stop)


@dataclasses.dataclass
class SharedResult:
    J: np.ndarray  # the shared basis
    beta: np.ndarray  # P x |J|, one coefficient row per problem
    F: np.ndarray  # paper-scale objective C_p f_p of each problem
    totals: list  # per addition step: the winner's summed score
    stages: list  # number of additions per stage


def _shared_total(decreases) -> float:
    """Score of a candidate for the shared basis: the problems' decreases of f_p added in problem order."""
    total = 0.0
    for dl in decreases:
        total += dl
    return total


def _candidate_columns(X: np.ndarray, c: int, gamma) -> list:
    """Kernel column of row c for each problem (computed once per distinct gamma)."""
    kg = {}
    for g in gamma:
        if g not in kg:
            kg[g] = rbf_block(X, X[c:c + 1], g)[:, 0]
    return [kg[g] for g in gamma]


def train_shared(X: np.ndarray, Y: np.ndarray, C, gamma, J_max: int, seed: int = 0, kappa: int = 59,
                 growth: float = 0.25, cap: int = 256, tol: float = 1e-10, ftol: float = 1e-14,
                 max_iter: int = 50) -> SharedResult:
    """Greedy growth of one basis shared by P problems on the same rows (labels Y[p], C[p], gamma[p]), with Newton
    re-optimisation of every problem after each stage: the selection of section 4 applied to the batch.

    The candidates of a step are drawn as for one problem (same stream, J frozen at the stage start, duplicates of
    members skipped). A candidate's score is the sum over the problems, in problem order, of each problem's exact
    one-coefficient decrease of f_p = F_p / C_p (its own kernel column, coefficients and outputs); the largest sum
    wins (lower row on ties), and every problem takes the winner with its own one-dimensional optimum as the
    coefficient. Without the bias and the stopping rule.
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
    P, n = Y.shape
    C = np.broadcast_to(np.asarray(C, dtype=np.float64), (P,))
    gamma = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (P,))
    groups = duplicate_groups(X)
    for q in range(P):
        _validate(X, Y[q], C[q], gamma[q], J_max, groups)
    lam = 1.0 / C
    J: list[int] = []
    beta = [np.zeros(0) for _ in range(P)]
    o = np.zeros((P, n))
    cols = [[] for _ in range(P)]  # kernel columns of the basis, per problem
    used_groups: set = set()
    totals, stages = [], []
    t = 0
    while len(J) < J_max:
        cs = stage_size(len(J), J_max, growth, cap)
        frozen = set(used_groups)
        draws = [draw_candidates(seed, t + q, n, kappa, lambda i: groups[i] in frozen) for q in range(cs)]
        added = 0
        for q in range(cs):
            best = None  # (summed score, index, coefficients, columns)
            for c in draws[q]:
                if groups[c] in used_groups:
                    continue
                ks = _candidate_columns(X, c, gamma)
                ss, dls = [], []
                for p in range(P):
                    sp, dl = score_candidate(1.0 - Y[p] * o[p], Y[p] * ks[p], lam[p], float(o[p, c]))
                    ss.append(sp)
                    dls.append(dl)
                total = _shared_total(dls)
                if best is None or total > best[0] or (total == best[0] and c < best[1]):
                    best = (total, c, ss, ks)
            if best is None:
                continue
            total, c, ss, ks = best
            totals.append(total)
            J.append(c)
            used_groups.add(groups[c])
            for p in range(P):
                beta[p] = np.append(beta[p], ss[p])
                o[p] = o[p] + ss[p] * ks[p]
                cols[p].append(ks[p])
            added += 1
        t += cs
        stages.append(added)
        if added == 0:
            break
        for p in range(P):
            KXJ = np.stack(cols[p], axis=1)
            beta[p], _ = newton_solve(KXJ, KXJ[J, :], Y[p], lam[p], beta[p], tol=tol, ftol=ftol, max_iter=max_iter)
            o[p] = KXJ @ beta[p]
    F = np.zeros(P)
    for p in range(P):
        if J:
            KXJ = np.stack(cols[p], axis=1)
            F[p] = C[p] * objective(KXJ, KXJ[J, :], Y[p], beta[p], lam[p])
        else:
            F[p] = C[p] * 0.5 * n
    return SharedResult(np.array(J, dtype=np.int64), np.array(beta), F, totals, stages)


def solve_fixed_J(X: np.ndarray, y: np.ndarray, C: float, gamma: float, J, beta0=None, tol: float = 1e-10,
                  ftol: float = 1e-14, max_iter: int = 50, bias: bool = False):
    """Newton re-optimisation of Eq. 4 on a given basis J, from beta0 (default 0; with ``bias`` the offset starts
    at 0 and is returned in info.bias).

    Returns (beta, F, info) with F the paper-scale objective at the returned beta (and offset).
    """
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    J = np.asarray(J, dtype=np.int64)
    KXJ = rbf_block(X, X[J], gamma)
    KJJ = KXJ[J, :]
    lam = 1.0 / C
    b0 = np.zeros(J.size) if beta0 is None else np.asarray(beta0, dtype=np.float64)
    if bias:
        A, R = _with_offset(KXJ, KJJ)
        th, info = newton_solve(A, R, y, lam, np.concatenate([[0.0], b0]), tol=tol, ftol=ftol, max_iter=max_iter)
        info.bias = float(th[0])
        return th[1:], C * objective(A, R, y, th, lam), info
    beta, info = newton_solve(KXJ, KJJ, y, lam, b0, tol=tol, ftol=ftol, max_iter=max_iter)
    return beta, C * objective(KXJ, KJJ, y, beta, lam), info


def objective_at(X: np.ndarray, y: np.ndarray, C: float, gamma: float, J, beta, b: float = 0.0) -> float:
    """Paper-scale F(beta, b) on basis J, everything recomputed in FP64 from X."""
    X = np.asarray(X, dtype=np.float64)
    J = np.asarray(J, dtype=np.int64)
    KXJ = rbf_block(X, X[J], gamma)
    beta = np.asarray(beta, np.float64)
    yd = np.asarray(y, dtype=np.float64)
    if b != 0.0:
        A, R = _with_offset(KXJ, KXJ[J, :])
        return C * objective(A, R, yd, np.concatenate([[b], beta]), 1.0 / C)
    return C * objective(KXJ, KXJ[J, :], yd, beta, 1.0 / C)


def predict(X_basis: np.ndarray, beta: np.ndarray, gamma: float, Xt: np.ndarray, b: float = 0.0) -> np.ndarray:
    """Decision values sum_k beta_k k(x, x_{J_k}) + b for each row x of Xt."""
    return rbf_block(Xt, X_basis, gamma) @ np.asarray(beta, dtype=np.float64) + b


# ------------------------------------------------------------------------------------------ one-vs-one
def ovo_pairs(K: int):
    """The class pairs (a, b), a < b, in the order (0, 1), (0, 2), ..., (K - 2, K - 1)."""
    return [(a, b) for a in range(K) for b in range(a + 1, K)]


def train_ovo(X: np.ndarray, classes: np.ndarray, K: int, C: float, gamma: float, J_max: int, **kw):
    """One-vs-one multiclass training, as section 5 trains MNIST8M (one classifier per pair of classes, each on the
    rows of its two classes only): for each pair (a, b) greedy training on the rows of classes a (label +1) and b
    (label -1), keeping their order. Returns one (TrainResult, rows) per pair in ovo_pairs order, where rows are the
    pair's training rows (indices into X) and result.J indexes them; ``kw`` as for ``train``."""
    X = np.asarray(X, dtype=np.float64)
    classes = np.asarray(classes)
    out = []
    for a, b in ovo_pairs(K):
        rows = np.flatnonzero((classes == a) | (classes == b))
        y = np.where(classes[rows] == a, 1.0, -1.0)
        out.append((train(X[rows], y, C, gamma, J_max, **kw), rows))
    return out


def ovo_vote(decisions: np.ndarray, K: int) -> np.ndarray:
    """Class of each row from the pairwise decision values (one column per pair, ovo_pairs order): a positive value
    is a vote for a, any other for b; the class with the most votes wins, the lowest class on ties."""
    votes = np.zeros((decisions.shape[0], K), dtype=np.int64)
    for p, (a, b) in enumerate(ovo_pairs(K)):
        pos = decisions[:, p] > 0
        votes[pos, a] += 1
        votes[~pos, b] += 1
    return np.argmax(votes, axis=1)  # the first maximum: the lowest class on ties


def predict_ovo(X: np.ndarray, models, gamma: float, Xt: np.ndarray, K: int) -> np.ndarray:
    """Classes of the rows of Xt by one-vs-one voting over the models of ``train_ovo``."""
    X = np.asarray(X, dtype=np.float64)
    dec = np.stack([predict(X[rows][res.J], res.beta, gamma, Xt, res.b) for res, rows in models], axis=1)
    return ovo_vote(dec, K)
