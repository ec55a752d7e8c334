"""GPU parity of SP-SVM training (greedy selection + Newton) and prediction against the FP64 oracle.

Bars: identical basis on the FP64 path; objective F(beta_gpu) within 1e-6 relative of the oracle's optimum
for the same basis (both evaluated by the oracle in FP64); decision values within 1e-4 of the oracle's,
relative to max(1, |value|).
"""

import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1404_1066_amd as lib
from oracle import spsvm as osp

pytestmark = pytest.mark.gpu


def _dev(X, y):
    dt = torch.float64 if X.dtype == np.float64 else torch.float32
    return torch.tensor(X, dtype=dt, device="cuda"), torch.tensor(y, dtype=torch.float32, device="cuda")


def _decision_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))


def test_blobs_full_pipeline_identical_basis_f64():
    p = datagen.make_config("blobs-2k")
    ref = oracle.train(p.X, p.y, p.C, p.gamma, p.J_max, seed=0)
    Xg, yg = _dev(p.X, p.y)
    model = lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=0, precision="f64")
    J, beta, F = model.get()
    print("stats", model.stats())
    assert J.tolist() == ref.J.tolist()
    Fo = osp.objective_at(p.X, p.y, p.C, p.gamma, J, beta)
    assert abs(Fo - ref.F) <= 1e-6 * ref.F
    assert abs(F - Fo) <= 1e-9 * Fo
    Xt, _ = datagen.make_blobs(1500, 16, seed=77)
    dg = model.predict(torch.tensor(Xt, device="cuda")).cpu().numpy()
    do = oracle.predict(p.X[ref.J], ref.beta, p.gamma, Xt)
    assert _decision_err(dg, do) <= 1e-4


def test_wide_rows_identical_basis_f64():
    """Rows of 300 features (several k chunks per tile, a ragged last chunk): the FP64 path must pick the
    oracle's basis, step for step."""
    X, y = datagen.make_blobs(2500, 300, seed=21)
    C, gamma, m = 1.0, 1.0 / 300, 60
    ref = oracle.train(X, y, C, gamma, m, seed=5)
    Xg, yg = _dev(X, y)
    model = lib.train(Xg, yg, C, gamma, m, seed=5, precision="f64")
    J, beta, F = model.get()
    assert J.tolist() == ref.J.tolist()
    Fo = osp.objective_at(X, y, C, gamma, J, beta)
    assert abs(Fo - ref.F) <= 1e-6 * ref.F


@pytest.mark.parametrize("kappa", [64, 33, 1])
def test_grouped_candidate_launches_identical_basis_f64(kappa):
    """300 features: candidate steps share kernel-block launches that take only the drawn candidates, each written
    to its own slot (kappa = 64: every slot in use, 48 steps fill 3072 columns; kappa = 33: up to 52 steps, 1716
    columns; kappa = 1: 52 one-candidate steps in one 64-column tile). Stages of 1, 1, 2, .., 64 and 2 steps: the
    64-step stage takes two launches (48 + 16 or 52 + 12 steps). The FP64 path must still pick the oracle's basis,
    step for step."""
    X, y = datagen.make_blobs(2200, 300, seed=26)
    C, gamma, m = 1.0, 1.0 / 300, 130
    ref = oracle.train(X, y, C, gamma, m, seed=8, kappa=kappa, growth=1.0)
    Xg, yg = _dev(X, y)
    model = lib.train(Xg, yg, C, gamma, m, seed=8, precision="f64", kappa=kappa, growth=1.0)
    J, beta, F = model.get()
    assert J.tolist() == ref.J.tolist()
    Fo = osp.objective_at(X, y, C, gamma, J, beta)
    assert abs(Fo - ref.F) <= 1e-6 * ref.F


@pytest.mark.parametrize("prec", ["f32", "mixed"])
def test_wide_rows_f32_mixed_reach_oracle_objective(prec):
    X, y = datagen.make_blobs(3001, 333, seed=22, dtype=np.float32)
    C, gamma, m = 2.0, 1.0 / 333, 90
    Xg, yg = _dev(X, y)
    model = lib.train(Xg, yg, C, gamma, m, seed=6, precision=prec)
    J, beta, F = model.get()
    assert len(set(J.tolist())) == m
    b_or, F_or, _ = osp.solve_fixed_J(X, y, C, gamma, J)
    Fo = osp.objective_at(X, y, C, gamma, J, beta)
    assert abs(Fo - F_or) / F_or <= 1e-6


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fixed_basis_ragged_matches_oracle(prec):
    X, y = datagen.make_blobs(5003, 37, seed=11, dtype=np.float32 if prec == "f32" else np.float64)
    r = np.random.default_rng(5)
    J = np.sort(r.choice(5003, size=203, replace=False))
    C, gamma = 2.0, 1.0 / 37
    Xg, yg = _dev(X, y)
    model = lib.train_fixed_basis(Xg, yg, C, gamma, J, precision=prec)
    Jg, beta, F = model.get()
    assert Jg.tolist() == J.tolist()
    b_or, F_or, _ = osp.solve_fixed_J(X, y, C, gamma, J)
    Fo = osp.objective_at(X, y, C, gamma, J, beta)
    tol = 1e-6 if prec == "f32" else 1e-11
    assert abs(Fo - F_or) / F_or <= tol
    assert Fo >= F_or * (1 - 1e-12)
    dg = model.predict(Xg).cpu().numpy()
    do = oracle.predict(X[J], b_or, gamma, X)
    assert _decision_err(dg, do) <= (1e-4 if prec == "f32" else 1e-9)


def test_greedy_f32_ragged_matches_oracle_at_gpu_basis():
    X, y = datagen.make_blobs(3001, 21, seed=12, dtype=np.float32)
    C, gamma, m = 1.0, 1.0 / 21, 150
    Xg, yg = _dev(X, y)
    model = lib.train(Xg, yg, C, gamma, m, seed=3)
    J, beta, F = model.get()
    assert len(J) == m and len(set(J.tolist())) == m
    b_or, F_or, _ = osp.solve_fixed_J(X, y, C, gamma, J)
    Fo = osp.objective_at(X, y, C, gamma, J, beta)
    assert abs(Fo - F_or) / F_or <= 1e-6
    assert abs(F - Fo) <= 1e-5 * Fo
    Xt, _ = datagen.make_blobs(1000, 21, seed=13, dtype=np.float32)
    dg = model.predict(torch.tensor(Xt, device="cuda")).cpu().numpy()
    do = oracle.predict(X[J], b_or, gamma, Xt)
    assert _decision_err(dg, do) <= 1e-4


@pytest.mark.parametrize("refactor_frac", [0.0, 0.05])
def test_newton_matrix_reuse_and_updates_keep_parity(refactor_frac):
    """Refactorising at every change of the violator set (0.0) or reusing the factor until 5% of it changed
    must both reach the oracle's optimum at the GPU's basis."""
    X, y = datagen.make_blobs(6000, 10, seed=31, dtype=np.float32)
    C, gamma, m = 4.0, 0.1, 300
    Xg, yg = _dev(X, y)
    model = lib.train(Xg, yg, C, gamma, m, seed=2, refactor_frac=refactor_frac)
    J, beta, F = model.get()
    st = model.stats()
    assert st["incremental_factorizations"] > 0
    b_or, F_or, _ = osp.solve_fixed_J(X, y, C, gamma, J)
    Fo = osp.objective_at(X, y, C, gamma, J, beta)
    assert abs(Fo - F_or) / F_or <= 1e-6


@pytest.mark.parametrize("prec", ["mixed", "f32"])
def test_onehot_mixed_precision_reaches_oracle_objective(prec):
    """Split-BF16 kernel block (mixed) on data shaped like the one-hot workload: the FP64 objective of the
    GPU's beta is within 1e-6 of the oracle's optimum at the GPU's basis."""
    p = datagen.make_config("onehot-500k", n=20000, J_max=300)
    Xg, yg = _dev(p.X, p.y)
    model = lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=1, precision=prec)
    J, beta, F = model.get()
    b_or, F_or, _ = osp.solve_fixed_J(p.X, p.y, p.C, p.gamma, J)
    Fo = osp.objective_at(p.X, p.y, p.C, p.gamma, J, beta)
    print(prec, "objective rel", (Fo - F_or) / F_or)
    assert abs(Fo - F_or) / F_or <= 1e-6
    rows = np.arange(0, 20000, 7)
    dg = model.predict(Xg[torch.tensor(rows, device="cuda")]).cpu().numpy()
    do = oracle.predict(p.X[J], b_or, p.gamma, p.X[rows])
    assert _decision_err(dg, do) <= 1e-4


@pytest.mark.parametrize("d", [54, 300])
def test_mixed_tall_blocks_reach_oracle_objective(d):
    """Mixed precision at n >= 65536: short rows (d = 54) keep the 128-row tiles; long rows (d = 300) take
    256-row tiles for single candidate steps, whose fused first scoring pass writes two 128-row records per tile
    (later stages group steps into 256 x 256 tiles)."""
    if d == 54:
        p = datagen.make_config("onehot-500k", n=70001, J_max=150)
        X, y, C, gamma, m = p.X, p.y, p.C, p.gamma, p.J_max
    else:
        X, y = datagen.make_blobs(70001, d, seed=24, dtype=np.float32)
        C, gamma, m = 1.0, 1.0 / d, 60
    Xg, yg = _dev(X, y)
    model = lib.train(Xg, yg, C, gamma, m, seed=2, precision="mixed")
    J, beta, F = model.get()
    b_or, F_or, _ = osp.solve_fixed_J(X, y, C, gamma, J)
    Fo = osp.objective_at(X, y, C, gamma, J, beta)
    assert abs(Fo - F_or) / F_or <= 1e-6


@pytest.mark.parametrize("binary", [False, True])
def test_mixed_grouped_wide_tiles_reach_oracle_objective(binary):
    """300 features: candidate steps share kernel-block launches (whole stages of up to 24 steps here, 1416
    columns), which the split-BF16 block runs in 256 x 256 tiles with the fused first scoring pass in its first
    64 columns."""
    n, d = 40000, 300
    if binary:
        r = np.random.default_rng(31)
        X = (r.random((n, d)) < 0.05).astype(np.float32)
        s = X @ r.standard_normal(d) + 0.3 * r.standard_normal(n)
        y = np.where(s > np.median(s), 1.0, -1.0).astype(np.float32)
    else:
        X, y = datagen.make_blobs(n, d, seed=23, dtype=np.float32)
    C, gamma, m = 1.0, 1.0 / d, 120
    Xg, yg = _dev(X, y)
    model = lib.train(Xg, yg, C, gamma, m, seed=7, precision="mixed")
    J, beta, F = model.get()
    assert len(set(J.tolist())) == m
    b_or, F_or, _ = osp.solve_fixed_J(X, y, C, gamma, J)
    Fo = osp.objective_at(X, y, C, gamma, J, beta)
    assert abs(Fo - F_or) / F_or <= 1e-6


def test_mixed_on_bf16_exact_data_equals_fp32_bitwise():
    """0/1 features are exact in BF16, so the split's lo parts vanish and the mixed kernel block issues only
    hi.hi'; its integer dot products equal the FP32 path's, so the whole training run must agree bit for bit."""
    p = datagen.make_config("binary-100k", n=12000, J_max=200)
    Xg, yg = _dev(p.X, p.y)
    runs = [lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=4, precision=prec).get() for prec in ("f32", "mixed")]
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    assert runs[0][2] == runs[1][2]


def test_batch_equals_fixed_basis_and_oracle():
    """Batched one-vs-rest x (C, gamma) problems on one shared basis, solved in lockstep: each model matches
    the single-problem fixed-basis solve (the batched SYRK splits its rows differently, so agreement is to
    rounding), reaches the oracle's optimum, and does not depend on which other problems share the batch."""
    p = datagen.make_config("mnist-60k", n=3000, J_max=150)
    sel = [0, 5, 18, 23, 37, 42]  # classes 0-2, several (C, gamma) pairs
    Xg = torch.tensor(p.X, device="cuda")
    Yg = torch.tensor(p.Y[sel], dtype=torch.float32, device="cuda").contiguous()
    models = lib.train_batch(Xg, Yg, p.C[sel], p.gamma[sel], p.J)
    assert len(models) == len(sel)
    sub = lib.train_batch(Xg, Yg[[4, 1]].contiguous(), p.C[[sel[4], sel[1]]], p.gamma[[sel[4], sel[1]]], p.J)
    for q, s_ in enumerate(sel):
        Jb, bb, Fb = models[q].get()
        assert Jb.tolist() == p.J.tolist()
        single = lib.train_fixed_basis(Xg, Yg[q].contiguous(), p.C[s_], p.gamma[s_], p.J)
        J1, b1, F1 = single.get()
        assert abs(Fb - F1) <= 1e-11 * F1
        assert np.max(np.abs(bb - b1)) <= 1e-6 * max(1.0, np.max(np.abs(b1)))
        if q < 2:
            b_or, F_or, _ = osp.solve_fixed_J(p.X, p.Y[s_], p.C[s_], p.gamma[s_], p.J)
            Fo = osp.objective_at(p.X, p.Y[s_], p.C[s_], p.gamma[s_], p.J, bb)
            assert abs(Fo - F_or) / F_or <= 1e-6
    for k, q in enumerate([4, 1]):
        assert np.array_equal(sub[k].get()[1], models[q].get()[1]) and sub[k].get()[2] == models[q].get()[2]


def test_batch_large_basis_matches_oracle():
    """Six problems on a shared basis of 900 rows: the batched Cholesky's trailing update right of the first
    256-column outer panel (644 rows) takes the 128 x 128 tiles with all 256 panel columns, the next one the
    64 x 64 tiles (the triangular solves of this size run one workgroup per problem); each model reaches the
    oracle's optimum."""
    p = datagen.make_config("mnist-60k", n=3000, J_max=900)
    sel = [1, 5, 9, 13, 17, 21]  # one gamma: a lockstep group of six
    Xg = torch.tensor(p.X, device="cuda")
    Yg = torch.tensor(p.Y[sel], dtype=torch.float32, device="cuda").contiguous()
    models = lib.train_batch(Xg, Yg, p.C[sel], p.gamma[sel], p.J)
    for q, s_ in enumerate(sel[:3]):
        _, bb, _ = models[q].get()
        b_or, F_or, _ = osp.solve_fixed_J(p.X, p.Y[s_], p.C[s_], p.gamma[s_], p.J)
        Fo = osp.objective_at(p.X, p.Y[s_], p.C[s_], p.gamma[s_], p.J, bb)
        assert abs(Fo - F_or) / F_or <= 1e-6


def test_batch_more_problems_than_slots():
    """70 problems (more than the 64 lockstep slots): the second round of slots solves the rest; every model
    reaches the oracle's optimum at the shared basis and matches the same problem solved in a small batch."""
    p = datagen.make_config("mnist-60k", n=1500, J_max=60)
    idx = [i % p.Y.shape[0] for i in range(70)]
    g = float(p.gamma[0])  # one gamma: all 70 problems form one lockstep group
    Cs = p.C[idx]
    Xg = torch.tensor(p.X, device="cuda")
    Yg = torch.tensor(p.Y[idx], dtype=torch.float32, device="cuda").contiguous()
    models = lib.train_batch(Xg, Yg, Cs, np.full(70, g), p.J)
    assert len(models) == 70
    for q in (0, 63, 64, 69):
        alone = lib.train_batch(Xg, Yg[[q]].contiguous(), Cs[[q]], [g], p.J)[0]
        assert np.array_equal(alone.get()[1], models[q].get()[1])
        b_or, F_or, _ = osp.solve_fixed_J(p.X, p.Y[idx[q]], Cs[q], g, p.J)
        Fo = osp.objective_at(p.X, p.Y[idx[q]], Cs[q], g, p.J, models[q].get()[1])
        assert abs(Fo - F_or) / F_or <= 1e-6


def test_training_is_deterministic():
    X, y = datagen.make_blobs(4000, 12, seed=21, dtype=np.float32)
    Xg, yg = _dev(X, y)
    a = lib.train(Xg, yg, 1.0, 0.1, 80, seed=9).get()
    b = lib.train(Xg, yg, 1.0, 0.1, 80, seed=9).get()
    assert a[0].tolist() == b[0].tolist()
    assert np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_duplicate_rows_never_share_the_basis():
    r = np.random.default_rng(4)
    base = r.standard_normal((300, 4)).astype(np.float32)
    X = np.concatenate([base, base, base[:100]])
    y = np.where(X[:, 0] + 0.5 * r.standard_normal(700) > 0, 1.0, -1.0)
    y[300:600] = y[:300]
    y[600:] = y[:100]
    Xg, yg = _dev(X, y)
    J, beta, F = lib.train(Xg, yg, 1.0, 0.5, 120, seed=1, kappa=20).get()
    g = osp.duplicate_groups(X)
    assert len(set(g[J].tolist())) == len(J) == 120
    with pytest.raises(lib.SpsvmError) as e:
        lib.train(Xg, yg, 1.0, 0.5, 301)
    assert e.value.status == 1
    with pytest.raises(lib.SpsvmError):
        lib.train_fixed_basis(Xg, yg, 1.0, 0.5, [0, 300])


def test_invalid_inputs_detected_on_device():
    X, y = datagen.make_blobs(500, 3, seed=1, dtype=np.float32)
    Xg, yg = _dev(X, y)
    bad = yg.clone()
    bad[17] = 0.5
    with pytest.raises(lib.SpsvmError) as e:
        lib.train(Xg, bad, 1.0, 0.5, 10)
    assert e.value.status == 1 and "labels" in str(e.value)
    Xn = Xg.clone()
    Xn[3, 1] = float("nan")
    with pytest.raises(lib.SpsvmError) as e:
        lib.train(Xn, yg, 1.0, 0.5, 10)
    assert e.value.status == 1 and "NaN" in str(e.value)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(lib.SpsvmError) as e:
        lib.train(Xg, yg, 1.0, 0.5, 10, workspace=small)
    assert e.value.status == 6 and "workspace" in str(e.value)


def test_predict_empty_and_single_basis():
    X, y = datagen.make_blobs(300, 4, seed=2, dtype=np.float32)
    Xg, yg = _dev(X, y)
    model = lib.train(Xg, yg, 1.0, 0.25, 1)
    J, beta, F = model.get()
    assert len(J) == 1
    out = model.predict(Xg[:0])
    assert out.numel() == 0
    dg = model.predict(Xg).cpu().numpy()
    do = oracle.predict(X[J], beta, 0.25, X)
    assert _decision_err(dg, do) <= 1e-5


@pytest.mark.slow
def test_binary_100k_full_size_f32():
    """The 100k x 123 binary workload at its full size (|J| = 1000), in the configuration the benchmark
    times. The oracle re-solves Eq. 4 at the GPU's basis and checks the objective; decision values are
    checked on 2000 sampled rows."""
    p = datagen.make_config("binary-100k")
    Xg, yg = _dev(p.X, p.y)
    model = lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=0)
    J, beta, F = model.get()
    print("stats", model.stats())
    assert len(J) == p.J_max and len(set(osp.duplicate_groups(p.X)[J].tolist())) == p.J_max
    b_or, F_or, info = osp.solve_fixed_J(p.X, p.y, p.C, p.gamma, J)
    Fo = osp.objective_at(p.X, p.y, p.C, p.gamma, J, beta)
    print("F_gpu", Fo, "F_oracle", F_or, "rel", (Fo - F_or) / F_or, "oracle newton", info.iterations)
    assert abs(Fo - F_or) / F_or <= 1e-6
    rows = np.random.default_rng(0).choice(p.X.shape[0], 2000, replace=False)
    dg = model.predict(Xg[torch.tensor(rows, device="cuda")]).cpu().numpy()
    do = oracle.predict(p.X[J], b_or, p.gamma, p.X[rows])
    assert _decision_err(dg, do) <= 1e-4


@pytest.mark.slow
def test_mnist_60k_full_batch_f32():
    """The batched workload at its full size, as the benchmark's batched mode runs it: 160 one-vs-rest x
    (C, gamma) problems on 60000 x 784 rows with a shared basis of 2000 rows, one call. The oracle re-solves
    three of them (the first, a large-C one and the last) at that basis and checks their objectives; decision
    values of one model are checked on 1000 sampled rows."""
    p = datagen.make_config("mnist-60k")
    P = p.Y.shape[0]
    Xg = torch.tensor(p.X, dtype=torch.float32, device="cuda")
    Yg = torch.tensor(p.Y, dtype=torch.float32, device="cuda")
    models = lib.train_batch(Xg, Yg, p.C, p.gamma, p.J)
    assert len(models) == P
    big_c = int(np.flatnonzero(p.C == p.C.max())[0])
    for q in (0, big_c, P - 1):
        Jq, bq, Fq = models[q].get()
        assert Jq.tolist() == p.J.tolist()
        b_or, F_or, _ = osp.solve_fixed_J(p.X, p.Y[q], p.C[q], p.gamma[q], p.J)
        Fo = osp.objective_at(p.X, p.Y[q], p.C[q], p.gamma[q], p.J, bq)
        print("problem", q, "C", p.C[q], "gamma", p.gamma[q], "F_gpu", Fo, "F_oracle", F_or, "rel", (Fo - F_or) / F_or)
        assert abs(Fo - F_or) / F_or <= 1e-6
    rows = np.random.default_rng(1).choice(p.X.shape[0], 1000, replace=False)
    _, bq, _ = models[P - 1].get()
    dg = models[P - 1].predict(Xg[torch.tensor(rows, device="cuda")]).cpu().numpy()
    do = oracle.predict(p.X[p.J], bq, p.gamma[P - 1], p.X[rows])
    assert _decision_err(dg, do) <= 1e-4


def _oracle_at_basis(X, y, C, gamma, J, beta):
    """The oracle's optimum at basis J (Newton from beta = 0) and the FP64 objective of the GPU's beta there, from
    one oracle kernel block (what solve_fixed_J and objective_at compute, without forming the block twice)."""
    K = oracle.rbf_block(X, X[J], gamma)
    lam, yd = 1.0 / C, np.asarray(y, dtype=np.float64)
    b_or, info = osp.newton_solve(K, K[J], yd, lam, np.zeros(len(J)))
    F_or = C * osp.objective(K, K[J], yd, b_or, lam)
    Fo = C * osp.objective(K, K[J], yd, np.asarray(beta, dtype=np.float64), lam)
    return b_or, F_or, Fo, info


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_jitter_retry_on_near_duplicate_basis_rows(prec):
    """Twelve basis rows have a twin that differs by ~1e-14 relative (distinct values, so both may be in J). With
    C = 1000 the Newton matrix at beta = 0 is singular to FP64 rounding: the oracle's first Cholesky fails and it
    retries with a diagonal shift (checked here). The library must take its jitter retries as well (FP64) and
    reach the oracle's objective at the same basis."""
    X, y = datagen.make_blobs(2000, 5, seed=41)
    r = np.random.default_rng(3)
    J0 = np.sort(r.choice(2000, 60, replace=False))
    twins = X[J0[:12]] * (1 + 1e-14 * r.standard_normal((12, 5)))
    X2, y2 = np.concatenate([X, twins]), np.concatenate([y, y[J0[:12]]])
    J = np.concatenate([J0, np.arange(2000, 2012)])
    assert np.unique(X2[J], axis=0).shape[0] == J.size
    C, gamma = 1000.0, 0.2
    K = oracle.rbf_block(X2, X2[J], gamma)
    with pytest.raises(np.linalg.LinAlgError):
        np.linalg.cholesky(K[J] / C + K.T @ K)  # the oracle's first factorisation takes the retry path
    Xg = torch.tensor(X2, device="cuda")  # FP64 rows in both modes; f32 forms the kernel values in FP32 from them
    yg = torch.tensor(y2, dtype=torch.float32, device="cuda")
    model = lib.train_fixed_basis(Xg, yg, C, gamma, J, precision=prec)
    _, beta, F = model.get()
    st = model.stats()
    if prec == "f64":
        assert st["jitter_retries"] >= 1
    b_or, F_or, Fo, info = _oracle_at_basis(X2, y2, C, gamma, J, beta)
    print(prec, "jitter retries", st["jitter_retries"], "F_gpu", Fo, "F_oracle", F_or)
    assert abs(Fo - F_or) / F_or <= 1e-6


def test_offset_X_view_trains_in_queried_workspace():
    """X starting 4 bytes past a 16-byte boundary (d a multiple of 4): FP32 training copies it to aligned rows
    inside a workspace of exactly the queried size and returns the model of the aligned X, bit for bit."""
    X, y = datagen.make_blobs(3000, 12, seed=8, dtype=np.float32)
    n, d = X.shape
    buf = torch.zeros(n * d + 1, dtype=torch.float32, device="cuda")
    Xv = buf[1:].view(n, d)
    Xv.copy_(torch.tensor(X, device="cuda"))
    assert Xv.data_ptr() % 16 != 0
    Xg, yg = _dev(X, y)
    ws = torch.empty(lib.workspace_bytes(n, d, 100), dtype=torch.uint8, device="cuda")
    a = lib.train(Xv, yg, 1.0, 1.0 / 12, 100, seed=3, workspace=ws).get()
    b = lib.train(Xg, yg, 1.0, 1.0 / 12, 100, seed=3).get()
    assert a[0].tolist() == b[0].tolist() and np.array_equal(a[1], b[1]) and a[2] == b[2]


@pytest.mark.slow
@pytest.mark.parametrize("prec,n", [("mixed", 100000), ("f32", 50000)])
def test_dense_2m_rows_full_basis_reach_oracle_objective(prec, n):
    """Rows of the dense-2m workload (2000 i.i.d. N(0, 1) features, gamma = 1/2000, C = 1) at reduced n, greedy to
    its |J| = 4000: the split-BF16 256 x 256 tiles and 16-step grouped candidate blocks (mixed) or the FP32 grouped
    blocks, and Newton solves past the one-workgroup size (blocked triangular solves, a partial last block). The
    oracle re-solves at the GPU's basis; decisions on 2000 sampled rows."""
    p = datagen.make_config("dense-2m", n=n)
    Xg, yg = _dev(p.X, p.y)
    model = lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=0, precision=prec)
    J, beta, F = model.get()
    assert len(J) == p.J_max == 4000
    b_or, F_or, Fo, info = _oracle_at_basis(p.X, p.y, p.C, p.gamma, J, beta)
    print(prec, n, "F_gpu", Fo, "F_oracle", F_or, "rel", (Fo - F_or) / F_or, "stats", model.stats())
    assert abs(Fo - F_or) / F_or <= 1e-6
    rows = np.random.default_rng(0).choice(n, 2000, replace=False)
    dg = model.predict(Xg[torch.tensor(rows, device="cuda")]).cpu().numpy()
    do = oracle.predict(p.X[J], b_or, p.gamma, p.X[rows])
    assert _decision_err(dg, do) <= 1e-4


@pytest.mark.slow
def test_onehot_200k_full_basis_mixed_reaches_oracle_objective():
    """The one-hot workload (54 features, C = 10, gamma = 0.5) at n = 200 000 with its full |J| = 3000, mixed
    precision: the oracle re-solves at the GPU's basis; decisions on 2000 sampled rows."""
    p = datagen.make_config("onehot-500k", n=200000)
    Xg, yg = _dev(p.X, p.y)
    model = lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=0, precision="mixed")
    J, beta, F = model.get()
    assert len(J) == p.J_max == 3000
    b_or, F_or, Fo, info = _oracle_at_basis(p.X, p.y, p.C, p.gamma, J, beta)
    print("F_gpu", Fo, "F_oracle", F_or, "rel", (Fo - F_or) / F_or, "stats", model.stats())
    assert abs(Fo - F_or) / F_or <= 1e-6
    rows = np.random.default_rng(0).choice(p.X.shape[0], 2000, replace=False)
    dg = model.predict(Xg[torch.tensor(rows, device="cuda")]).cpu().numpy()
    do = oracle.predict(p.X[J], b_or, p.gamma, p.X[rows])
    assert _decision_err(dg, do) <= 1e-4


def test_offset_and_stopping_rule_identical_to_oracle_f64():
    """Eq. 4 with the offset b and the training-error stopping rule of section 4 (here eps = 2e-3 so that it stops
    after about a dozen stages), FP64 path: the same basis, hence the same stopping stage, the same b and objective
    as the oracle; the reported training error is the oracle's last one. Decision values: two separately converged
    Newton solves (each stops at ||grad f|| <= 1e-10 ||grad f_0||), so they agree to that times the conditioning of
    the Newton matrix, here a few 1e-9; the bar is 1e-7, against 1e-4 for parity."""
    p = datagen.make_config("binary-100k", n=3000)
    X = p.X.astype(np.float64)
    ref = oracle.train(X, p.y, p.C, p.gamma, 300, seed=2, bias=True, eps_stop=2e-3)
    assert ref.stop == "eps" and len(ref.J) < 300
    Xg, yg = _dev(X, p.y)
    model = lib.train(Xg, yg, p.C, p.gamma, 300, seed=2, precision="f64", bias=1, eps_stop=2e-3)
    J, beta, F = model.get()
    st = model.stats()
    assert J.tolist() == ref.J.tolist()
    assert st["stop_reason"] == 1
    assert abs(model.bias - ref.b) <= 1e-8 * (1 + abs(ref.b))
    Fo = osp.objective_at(X, p.y, p.C, p.gamma, J, beta, b=model.bias)
    assert abs(Fo - ref.F) <= 1e-9 * ref.F and abs(F - Fo) <= 1e-9 * Fo
    assert abs(st["train_error"] - ref.errors[-1]) <= 1.0 / X.shape[0]
    dg = model.predict(Xg).cpu().numpy()
    do = oracle.predict(X[ref.J], ref.beta, p.gamma, X, ref.b)
    assert _decision_err(dg, do) <= 1e-7


def test_offset_blobs_identical_basis_f64():
    p = datagen.make_config("blobs-2k")
    y = np.where(np.arange(2000) % 3 == 0, 1.0, -1.0)  # one class in three: the offset is far from 0
    ref = oracle.train(p.X, y, p.C, p.gamma, p.J_max, seed=0, bias=True)
    Xg, yg = _dev(p.X, y)
    model = lib.train(Xg, yg, p.C, p.gamma, p.J_max, seed=0, precision="f64", bias=1)
    J, beta, F = model.get()
    assert J.tolist() == ref.J.tolist()
    assert abs(model.bias - ref.b) <= 1e-8 * (1 + abs(ref.b)) and abs(ref.b) > 0.05
    Fo = osp.objective_at(p.X, y, p.C, p.gamma, J, beta, b=model.bias)
    assert abs(Fo - ref.F) <= 1e-9 * ref.F


@pytest.mark.parametrize("prec", ["f32", "mixed"])
def test_offset_greedy_reaches_oracle_objective(prec):
    X, y = datagen.make_blobs(3001, 21, seed=14, dtype=np.float32)
    y = np.where(X[:, 0] + 0.5 * X[:, 1] > 1.5, 1.0, -1.0)  # unbalanced classes: the offset matters
    C, gamma, m = 2.0, 1.0 / 21, 120
    Xg, yg = _dev(X, y)
    model = lib.train(Xg, yg, C, gamma, m, seed=3, precision=prec, bias=1)
    J, beta, F = model.get()
    b_or, F_or, info = osp.solve_fixed_J(X, y, C, gamma, J, bias=True)
    Fo = osp.objective_at(X, y, C, gamma, J, beta, b=model.bias)
    assert abs(Fo - F_or) / F_or <= 1e-6
    dg = model.predict(Xg).cpu().numpy()
    do = oracle.predict(X[J], b_or, gamma, X, info.bias)
    assert _decision_err(dg, do) <= 1e-4


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_offset_fixed_basis_and_batch_match_oracle(prec):
    """The offset in a fixed-basis solve and in a batch of one-vs-rest problems on one basis (FP32 and FP64 kernel
    values): each model reaches the oracle's optimum of Eq. 4 with b at the same basis."""
    p = datagen.make_config("mnist-60k", n=2000, J_max=120)
    sel = [0, 5, 18]
    Xg = torch.tensor(p.X, device="cuda")
    Yg = torch.tensor(p.Y[sel], dtype=torch.float32, device="cuda").contiguous()
    models = lib.train_batch(Xg, Yg, p.C[sel], p.gamma[sel], p.J, precision=prec, bias=1)
    for q, s_ in enumerate(sel):
        _, bb, _ = models[q].get()
        b_or, F_or, info = osp.solve_fixed_J(p.X, p.Y[s_], p.C[s_], p.gamma[s_], p.J, bias=True)
        Fo = osp.objective_at(p.X, p.Y[s_], p.C[s_], p.gamma[s_], p.J, bb, b=models[q].bias)
        assert abs(Fo - F_or) / F_or <= (1e-6 if prec == "f32" else 1e-10)
        single = lib.train_fixed_basis(Xg, Yg[q].contiguous(), p.C[s_], p.gamma[s_], p.J, precision=prec, bias=1)
        assert abs(single.bias - models[q].bias) <= 1e-6 * (1 + abs(info.bias))
        assert abs(single.bias - info.bias) <= 1e-4 * (1 + abs(info.bias))


def test_ovo_identical_to_oracle_f64():
    """One-vs-one multiclass (4 classes, 6 pairs), FP64 path: every pair's model has the oracle's basis (as rows of
    X) and objective, and the voted classes of held-out rows equal the oracle's votes."""
    X, cls = datagen.make_mnist_like(per_class=300, d=10, seed=21, classes=4, noise=0.3)
    X = X.astype(np.float64)
    C, gamma, m = 2.0, 0.5, 25
    ref = oracle.train_ovo(X, cls, 4, C, gamma, m, seed=3)
    Xg = torch.tensor(X, device="cuda")
    models = lib.train_ovo(Xg, torch.tensor(cls, dtype=torch.int32, device="cuda"), 4, C, gamma, m, seed=3,
                           precision="f64")
    assert len(models) == 6
    for (res, rows), md in zip(ref, models):
        J, beta, F = md.get()
        assert J.tolist() == rows[res.J].tolist()
        assert abs(F - res.F) <= 1e-9 * res.F
    Xt, _ = datagen.make_mnist_like(per_class=100, d=10, seed=22, classes=4, noise=0.3)
    Xt = Xt.astype(np.float64)
    got = lib.predict_ovo(models, 4, torch.tensor(Xt, device="cuda")).cpu().numpy()
    want = oracle.predict_ovo(X, ref, gamma, Xt, 4)
    assert np.array_equal(got, want)


def test_ovo_f32_pairs_reach_oracle_objective():
    """One-vs-one in FP32 on 3 classes of 784-feature rows: each pair's objective within 1e-6 of the oracle's optimum
    at that pair's basis."""
    X, cls = datagen.make_mnist_like(per_class=700, d=784, seed=23, classes=3)
    C, gamma, m = 10.0, 0.02, 80
    models = lib.train_ovo(torch.tensor(X, device="cuda"), torch.tensor(cls, dtype=torch.int32, device="cuda"), 3, C,
                           gamma, m, seed=4)
    for (a, b), md in zip(oracle.ovo_pairs(3), models):
        rows = np.flatnonzero((cls == a) | (cls == b))
        J, beta, F = md.get()
        local = np.searchsorted(rows, J)
        assert np.array_equal(rows[local], J)
        y = np.where(cls[rows] == a, 1.0, -1.0)
        b_or, F_or, _ = osp.solve_fixed_J(X[rows], y, C, gamma, local)
        Fo = osp.objective_at(X[rows], y, C, gamma, local, beta)
        assert abs(Fo - F_or) / F_or <= 1e-6


# ------------------------------------------------------------------------------ one greedy basis for a batch
def _shared_case(P=4, n_per=300, d=20):
    X, cls = datagen.make_mnist_like(per_class=n_per, d=d, seed=31, classes=5)
    Y = np.stack([np.where(cls == c, 1.0, -1.0) for c in range(P)])
    C = np.array([1.0, 10.0, 1.0, 10.0, 3.0, 0.5])[:P]
    gamma = np.array([0.1, 0.1, 0.3, 0.3, 0.1, 0.3])[:P]
    return X.astype(np.float64), Y, C, gamma


def test_shared_basis_identical_to_oracle_f64():
    """Four one-vs-rest problems (two C, two gamma) grow one basis: the FP64 path picks the oracle's basis step for
    step and reaches each problem's objective."""
    X, Y, C, gamma = _shared_case()
    ref = osp.train_shared(X, Y, C, gamma, 40, seed=2, kappa=20)
    Xg = torch.tensor(X, device="cuda")
    Yg = torch.tensor(Y, dtype=torch.float32, device="cuda")
    models = lib.train_shared(Xg, Yg, C, gamma, 40, seed=2, kappa=20, precision="f64")
    for p, md in enumerate(models):
        J, beta, F = md.get()
        assert J.tolist() == ref.J.tolist()
        assert abs(F - ref.F[p]) <= 1e-9 * ref.F[p]
        assert np.max(np.abs(beta - ref.beta[p])) <= 1e-6 * max(1.0, np.max(np.abs(ref.beta[p])))


@pytest.mark.parametrize("prec", ["f32", "mixed"])
def test_shared_basis_reaches_oracle_objective(prec):
    """F32 and MIXED: every problem's coefficients reach the oracle's optimum at the shared basis the GPU chose (both
    sides of 1e-6), and its decision values match the oracle's there."""
    X, Y, C, gamma = _shared_case(P=6)
    Xf = X.astype(np.float32)
    Xg = torch.tensor(Xf, device="cuda")
    Yg = torch.tensor(Y, dtype=torch.float32, device="cuda")
    models = lib.train_shared(Xg, Yg, C, gamma, 60, seed=4, kappa=24, precision=prec)
    J0 = models[0].get()[0]
    Xt, _ = datagen.make_mnist_like(per_class=60, d=20, seed=32, classes=5)
    for p, md in enumerate(models):
        J, beta, F = md.get()
        assert J.tolist() == J0.tolist() and len(J) == 60
        X64 = Xf.astype(np.float64)
        b_or, F_or, _ = osp.solve_fixed_J(X64, Y[p], C[p], gamma[p], J)
        Fo = osp.objective_at(X64, Y[p], C[p], gamma[p], J, beta)
        assert abs(Fo - F_or) / F_or <= 1e-6, (p, Fo, F_or)
        dg = md.predict(torch.tensor(Xt, device="cuda")).cpu().numpy()
        do = oracle.predict(X64[J], b_or, gamma[p], Xt.astype(np.float64))
        assert _decision_err(dg, do) <= 1e-4


def test_shared_basis_one_problem_is_plain_training():
    X, Y, C, gamma = _shared_case(P=1)
    Xg = torch.tensor(X, device="cuda")
    Yg = torch.tensor(Y, dtype=torch.float32, device="cuda")
    sh = lib.train_shared(Xg, Yg, C, gamma, 30, seed=7, kappa=16, precision="f64")[0].get()
    one = lib.train(Xg, Yg[0].contiguous(), C[0], gamma[0], 30, seed=7, kappa=16, precision="f64").get()
    assert sh[0].tolist() == one[0].tolist()
    assert abs(sh[2] - one[2]) <= 1e-12 * one[2]


def test_shared_basis_rejects_offset_and_stop_rule():
    X, Y, C, gamma = _shared_case(P=2)
    Xg = torch.tensor(X, device="cuda")
    Yg = torch.tensor(Y, dtype=torch.float32, device="cuda")
    for kw in ({"bias": 1}, {"eps_stop": 1e-3}):
        with pytest.raises(lib.SpsvmError):
            lib.train_shared(Xg, Yg, C, gamma, 10, **kw)


@pytest.mark.parametrize("prec", ["f32", "mixed"])
def test_kxj_in_host_memory_gives_the_same_model(prec):
    """K_XJ held in pinned host memory (kxj_host = 1: every pass over it streams it over the host link) runs the same
    kernels on the same values, so greedy training and a fixed-basis solve return bit for bit the models made with
    K_XJ in the workspace, and the workspace shrinks by the block."""
    n, d, m = 20001, 40, 150
    X, y = datagen.make_blobs(n, d, seed=33, dtype=np.float32)
    Xg, yg = _dev(X, y)
    a = lib.train(Xg, yg, 1.0, 1.0 / d, m, seed=3, precision=prec).get()
    b = lib.train(Xg, yg, 1.0, 1.0 / d, m, seed=3, precision=prec, kxj_host=1).get()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    fa = lib.train_fixed_basis(Xg, yg, 1.0, 1.0 / d, a[0], precision=prec).get()
    fb = lib.train_fixed_basis(Xg, yg, 1.0, 1.0 / d, a[0], precision=prec, kxj_host=1).get()
    assert np.array_equal(fa[1], fb[1]) and fa[2] == fb[2]
    wa = lib.workspace_bytes(n, d, m, precision=prec)
    wb = lib.workspace_bytes(n, d, m, precision=prec, kxj_host=1)
    assert wa - wb >= n * 152 * 4 - 256  # the block (ldk = 152), less the 256 bytes every sub-buffer takes at least


def test_shared_basis_more_problems_than_slots_f64():
    """66 problems, 65 of them on one gamma (more than the 64 Newton slots: that group is solved in two rounds of
    slots) and one on another: the FP64 shared basis equals the oracle's step for step, and the objectives match."""
    X, cls = datagen.make_mnist_like(per_class=80, d=6, seed=41, classes=5)
    X = X.astype(np.float64)
    P = 66
    Y = np.stack([np.where(cls == (q % 5), 1.0, -1.0) for q in range(P)])
    C = np.array([0.5 + 0.25 * (q % 7) for q in range(P)])
    gamma = np.array([1.5 if q == 40 else 0.5 for q in range(P)])
    ref = osp.train_shared(X, Y, C, gamma, 12, seed=6, kappa=8)
    models = lib.train_shared(torch.tensor(X, device="cuda"), torch.tensor(Y, dtype=torch.float32, device="cuda"),
                              C, gamma, 12, seed=6, kappa=8, precision="f64")
    assert len(models) == P
    for q in (0, 1, 40, 63, 64, 65):
        J, beta, F = models[q].get()
        assert J.tolist() == ref.J.tolist()
        assert abs(F - ref.F[q]) <= 1e-9 * ref.F[q]
