"""FP64 CPU oracle for SP-SVM training (sparse primal SVM, section 4 of the paper, Eq. 4).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import, call or link anything in this package. The GPU library never uses it, and it
uses nothing of the GPU library: the two share no code. The only common dependency is ``datagen``,
which draws inputs and holds none of the method's arithmetic.

It is written to be checked by eye against the paper, not to be fast:

* ``kernel``  - the RBF kernel of section 2, k(x, z) = exp(-gamma ||x - z||^2), by explicit differences.
* ``rng``     - the candidate sampler (SplitMix64 counter streams) and the stage schedule.
* ``spsvm``   - Eq. 4 objective, its gradient and generalised Hessian, the Newton re-optimisation with an
  exact line search, the one-coefficient candidate score, greedy basis growth, prediction.

Readings of points the paper leaves open (candidate count, the score, stage sizes, stop rules, ties,
duplicate rows, jitter) are stated in each function's docstring.

Parity status: every function here is pinned by tests in ``tests/test_oracle_*.py`` against values
that do not come from the oracle itself (closed forms, brute-force enumeration, the dual QP, a
published SplitMix64 output, grid and golden-section searches).
"""

from .kernel import rbf_block, rbf_column, have_c_kernel  # noqa: F401
from .rng import splitmix64_stream, draw_candidates, stage_size, GOLDEN  # noqa: F401
from .spsvm import (  # noqa: F401
    NotPositiveDefinite,
    TrainResult,
    objective,
    gradient,
    exact_line_search,
    score_candidate,
    newton_solve,
    solve_fixed_J,
    train,
    SharedResult,
    train_shared,
    predict,
    duplicate_groups,
    ovo_pairs,
    train_ovo,
    ovo_vote,
    predict_ovo,
)
