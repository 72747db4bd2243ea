"""CPU oracle for tree-GP fitness evaluation -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import, call or run anything in this package. The
device library never depends on it, and it depends on nothing of the
device library.

Pins (what the oracle is checked against, other than itself) live in
tests/test_oracle_*.py; the one function with no external pin is listed in
the module docstring of tgp_oracle as "parity unpinned" (none at present).
"""

from .tgp_oracle import *  # noqa: F401,F403
from .tgp_oracle import (  # noqa: F401
    decode, plan, eval_stack, eval_recursive, eval_shadow32, mse, mse_shadow32, mse_tree,
    mse_tree_shadow32, predict, grad, grad_tree, fd_grad_const, fd_grad_x, adam_reference,
    apply_op, op_partials, length_bucket,
)
from .exchange_oracle import (  # noqa: F401
    subtree_exchange, exchange_tree, ancestors, pick_node,
    X_OK, X_TOO_LONG, X_BAD_OLD, X_BAD_DONOR, OLD_UNIFORM, NEW_UNIFORM,
)
from .generate_oracle import (  # noqa: F401
    generate, philox4x32_10, to_unit, GROW, FULL, RAMPED,
)
from .classify_oracle import accuracy, accuracy_bounds, classes  # noqa: F401
from . import envelope  # noqa: F401  (float32 envelopes for the comparison protocol)
