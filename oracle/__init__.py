"""FP64 CPU oracle for the exterior NMF (eNMF) hot path.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference that the HIP path is checked against.  Only the test
suite, the package smoke check and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the HIP path (no kernels, headers,
helpers or constants) and never imports the product package.

Every function follows one passage of the paper ("An Exterior Method for
Nonnegative Matrix Factorization"), cited in its docstring by section,
equation or algorithm.  Where the paper is silent the docstring states
the reading taken; the full list of readings is kept with the design
notes of the repository.

Parity status: all functions are pinned by the CPU tests in
``tests/test_oracle_pins.py``, ``tests/test_oracle_enmc.py`` and
``tests/test_oracle_sparse.py`` and ``tests/test_oracle_grot.py`` except the global optimality of the ADMM
rotation for r > 2 (an NP-hard problem; parity unpinned).
"""

from .enmf_ref import (  # noqa: F401
    EXT, HALS,
    objective, objective_expanded, relerr, gradients,
    svd_init_exact, svd_init_randomized, fix_signs, balance,
    prox_h, procrustes, rotate, negativity_mass,
    resolve_steps, push_negatives, pbcd, fixed_row_step, hals_half, ext_half,
    kkt, iterate, enmf,
)
from .enmc_ref import (  # noqa: F401
    masked_objective, masked_gradients, masked_relerr, softimpute_als, enmc_init,
    masked_pbcd, masked_kkt, enmc_iterate, enmc,
)
from .sparse_ref import (  # noqa: F401
    csr_to_dense, csr_rows_times, csr_cols_times, csr_sumsq,
)
from .grot_ref import (  # noqa: F401
    rotate_general, lambda_update, lambda_objective, update_w1, update_w2,
)
