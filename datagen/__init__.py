"""Seeded synthetic inputs for SP-SVM training runs.

This package only draws data. It holds none of the training method's arithmetic
(no kernel blocks, no objective, no Newton steps), so that both the FP64 oracle and
the GPU library can consume the same inputs without sharing any code.

Every generator is deterministic in its seed. Large row counts are generated in
blocks of ``BLOCK`` rows, each block from its own child of
``numpy.random.SeedSequence(seed)``, so generation can run in parallel and any
block can be regenerated on its own.

The workloads stand in for the datasets of the paper's Table 1 (section 5), which
are not available here: only their shapes (n, d), value ranges and label structure
are imitated.
"""

from .configs import (  # noqa: F401
    BLOCK,
    Problem,
    BatchProblem,
    make_config,
    make_blobs,
    make_binary_sparse,
    make_mixed_onehot,
    make_mnist_like,
    make_large_dense,
    make_sparse_rows,
    csr_to_dense,
    config_names,
)
