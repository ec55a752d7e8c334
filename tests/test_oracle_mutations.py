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
