"""SP-SVM training on AMD Instinct MI355X (gfx950): a C-ABI library of HIP kernels plus a thin binding.

The method is the sparse primal SVM of section 4 of "Parallel Support Vector Machines in Practice"
(greedy basis growth and Newton re-optimisation of Eq. 4, RBF kernel of section 2). See include/spsvm.h.
"""

from .binding import (  # noqa: F401
    Model,
    SpsvmError,
    load,
    options,
    train,
    train_fixed_basis,
    train_batch,
    train_shared,
    train_ovo,
    train_csr,
    predict_csr,
    predict_ovo,
    rbf_block,
    newton_solve,
    newton_solve_noalloc,
    candidate_draw,
    score_candidates,
    workspace_bytes,
    EXPORTED,
    LIB_PATH,
)
