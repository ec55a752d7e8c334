"""Planted mistakes in the oracle (on the CPU) must be caught by the pins.

Each test replaces one piece of the oracle with a plausible wrong version (a dropped term, a wrong
factor, a wrong sign, a wrong constant) and checks that at least one pin in ``test_oracle_pins`` then
reports a large error. This shows the pins are sensitive to the mistakes they are meant to catch.
"""

import numpy as np

import oracle
from oracle import kernel as okern
from oracle import rng as orng
from oracle import spsvm as osp

import test_oracle_pins as pins  # noqa: E402


def test_dropped_linear_term_in_segment_root_is_caught(monkeypatch):
    real = osp._segment_root

    def wrong(a, b, lam_c1, lam_c2, rep):
        return real(a, b, 0.0, lam_c2, rep)

    monkeypatch.setattr(osp, "_segment_root", wrong)
    assert pins.line_search_error(range(5)) > 1e-3
    assert pins.score_error(range(5)) > 1e-3


def test_wrong_regulariser_factor_in_objective_is_caught(monkeypatch):
    def wrong(KXJ, KJJ, y, beta, lam):
        o = KXJ @ beta
        return lam * float(beta @ (KJJ @ beta)) + 0.5 * float(np.sum(np.maximum(0.0, 1 - y * o) ** 2))

    monkeypatch.setattr(osp, "objective", wrong)
    assert pins.dual_qp_error(range(2)) > 1e-3


def test_wrong_regularisation_weight_in_newton_is_caught(monkeypatch):
    # lambda taken as 2 / C instead of 1 / C moves the optimum
    real = osp.newton_solve

    def wrong(KXJ, KJJ, y, lam, beta, **kw):
        return real(KXJ, KJJ, y, 2.0 * lam, beta, **kw)

    monkeypatch.setattr(osp, "newton_solve", wrong)
    assert pins.violator_enumeration_error(range(2)) > 1e-3
    assert pins.dual_qp_error(range(2)) > 1e-3


def test_wrong_sign_of_loss_term_in_gradient_is_caught(monkeypatch):
    # a sign error in the loss term of the gradient sends Newton to a wrong point
    def wrong(KXJ, KJJ, y, beta, lam):
        o = KXJ @ beta
        a = 1.0 - y * o
        act = a > 0
        return lam * (KJJ @ beta) + KXJ[act].T @ (y[act] * a[act])

    monkeypatch.setattr(osp, "gradient", wrong)
    assert pins.violator_enumeration_error(range(2)) > 1e-3


def test_wrong_kernel_width_is_caught(monkeypatch):
    real = okern.rbf_block

    def wrong(X, Z, gamma, use_c=True):
        return real(X, Z, 0.5 * gamma, use_c)

    monkeypatch.setattr(oracle, "rbf_block", wrong)
    assert pins.rbf_closed_form_error() > 1e-3


def test_wrong_mixer_constant_is_caught(monkeypatch):
    def wrong(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & orng.MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EA) & orng.MASK64
        return z ^ (z >> 31)

    monkeypatch.setattr(orng, "_mix", wrong)
    want = [int(v, 16) for v in pins._golden_lines("splitmix64_seed0.txt")]
    assert orng.splitmix64_stream(0, 3) != want


def test_score_without_regulariser_changes_selection(monkeypatch):
    real = osp.score_candidate

    def wrong(a, b, lam, o_c):
        return real(a, b, lam, 0.0)

    monkeypatch.setattr(osp, "score_candidate", wrong)
    assert pins.selection_bruteforce_mismatches() > 0


def _jitter_fails():
    try:
        return pins.jitter_error() > 1e-11
    except osp.NotPositiveDefinite:  # the planted schedule gave up where the right one succeeds
        return True


def test_jitter_without_diagonal_scale_is_caught(monkeypatch):
    def wrong(H):
        try:
            return np.linalg.cholesky(H)
        except np.linalg.LinAlgError:
            pass
        for mu in osp.JITTER:  # mu alone, not mu * mean(diag H)
            try:
                return np.linalg.cholesky(H + mu * np.eye(H.shape[0]))
            except np.linalg.LinAlgError:
                continue
        raise osp.NotPositiveDefinite("H")

    monkeypatch.setattr(osp, "cholesky_jitter", wrong)
    assert _jitter_fails()


def test_jitter_schedule_out_of_order_is_caught(monkeypatch):
    monkeypatch.setattr(osp, "JITTER", (1e-14, 1e-12, 1e-8, 1e-10))
    assert _jitter_fails()


def test_stream_started_at_step_instead_of_next_is_caught(monkeypatch):
    monkeypatch.setattr(orng, "step_state", lambda seed, t: (seed ^ ((t * orng.GOLDEN) & orng.MASK64)) & orng.MASK64)
    assert pins.stream_start_mismatches() > 0


def test_stream_steps_one_draw_apart_is_caught(monkeypatch):
    # each step starting one state after the previous one: seed 0 then draws a sliding window of candidates
    monkeypatch.setattr(orng, "step_state", lambda seed, t: (seed ^ (((t + 1) * orng.GOLDEN) & orng.MASK64)) & orng.MASK64)
    assert pins.stream_start_mismatches() > 0
    assert pins.consecutive_step_overlap() > 0


def test_stream_seed_added_instead_of_xored_is_caught(monkeypatch):
    monkeypatch.setattr(orng, "step_state", lambda seed, t: (seed + (t + 1) * orng.GOLDEN) & orng.MASK64)
    assert pins.stream_start_mismatches() > 0


def _replay_fails():
    try:
        return pins.stage_replay()[0] > 0
    except osp.NotPositiveDefinite:  # a duplicate entered the basis and made H singular
        return True


def test_draw_ignoring_the_stage_start_basis_is_caught(monkeypatch):
    real = osp.draw_candidates
    monkeypatch.setattr(osp, "draw_candidates", lambda seed, t, n, kappa, blocked: real(seed, t, n, kappa, lambda i: False))
    assert _replay_fails()


def test_duplicates_of_winners_not_blocked_is_caught(monkeypatch):
    monkeypatch.setattr(osp, "duplicate_groups", lambda X: np.arange(np.asarray(X).shape[0]))
    assert _replay_fails()


def test_regularised_offset_is_caught(monkeypatch):
    real = osp._with_offset

    def wrong(KXJ, KJJ):
        A, R = real(KXJ, KJJ)
        R[0, 0] = 1.0  # b treated like a basis coefficient with unit kernel value
        return A, R

    monkeypatch.setattr(osp, "_with_offset", wrong)
    assert pins.dual_qp_bias_error(range(2)) > 1e-3


def test_stop_rule_on_absolute_change_is_caught(monkeypatch):
    monkeypatch.setattr(osp, "stage_stops", lambda ep, e, added, eps: abs(ep - e) / added < eps)
    assert pins.stop_rule_mismatches() > 0


def test_stop_rule_without_per_vector_scaling_is_caught(monkeypatch):
    monkeypatch.setattr(osp, "stage_stops", lambda ep, e, added, eps: (ep - e) < eps)
    assert pins.stop_rule_mismatches() > 0


def test_training_error_with_strict_sign_is_caught(monkeypatch):
    monkeypatch.setattr(osp, "training_error", lambda y, o: float(np.mean(y * o < 0.0)))
    assert pins.stop_rule_mismatches() > 0


def test_ovo_ties_to_highest_class_is_caught(monkeypatch):
    def wrong(decisions, K):
        votes = np.zeros((decisions.shape[0], K), dtype=np.int64)
        for p, (a, b) in enumerate(osp.ovo_pairs(K)):
            pos = decisions[:, p] > 0
            votes[pos, a] += 1
            votes[~pos, b] += 1
        return K - 1 - np.argmax(votes[:, ::-1], axis=1)

    monkeypatch.setattr(osp, "ovo_vote", wrong)
    assert pins.ovo_vote_mismatches() > 0


def test_ovo_zero_decision_voting_for_first_class_is_caught(monkeypatch):
    def wrong(decisions, K):
        votes = np.zeros((decisions.shape[0], K), dtype=np.int64)
        for p, (a, b) in enumerate(osp.ovo_pairs(K)):
            pos = decisions[:, p] >= 0
            votes[pos, a] += 1
            votes[~pos, b] += 1
        return np.argmax(votes, axis=1)

    monkeypatch.setattr(osp, "ovo_vote", wrong)
    assert pins.ovo_vote_mismatches() > 0


def _shared_fails(**kw):
    mism, _ = pins.shared_replay(**kw)
    return mism > 0


def test_shared_score_from_first_problem_only_is_caught(monkeypatch):
    monkeypatch.setattr(osp, "_shared_total", lambda dls: dls[0])
    assert _shared_fails(steps=8)


def test_shared_score_as_maximum_is_caught(monkeypatch):
    monkeypatch.setattr(osp, "_shared_total", lambda dls: max(dls))
    assert _shared_fails(steps=8)


def test_shared_columns_with_one_gamma_are_caught(monkeypatch):
    def wrong(X, c, gamma):
        k = oracle.rbf_block(X, X[c:c + 1], gamma[0])[:, 0]
        return [k for _ in gamma]

    monkeypatch.setattr(osp, "_candidate_columns", wrong)
    assert _shared_fails(steps=6)


def test_shared_coefficient_of_first_problem_for_all_is_caught(monkeypatch):
    real = osp.score_candidate
    first = {}

    def wrong(a, b, lam, o_c):
        # the first problem's coefficient (recognised by its lambda) is handed to every problem of the step
        s, dl = real(a, b, lam, o_c)
        if lam == 0.5:
            first["s"] = s
        return first.get("s", s), dl

    monkeypatch.setattr(osp, "score_candidate", wrong)
    assert _shared_fails(n=36, steps=12, seed=731, growth=1.0)
