"""Seeded synthetic inputs for tree-GP fitness evaluation.

This package produces random tree populations in the NaN-padded prefix
encoding (types, values, subtree sizes; paper §III-A), input matrices,
noise vectors and hidden target trees. It evaluates nothing: a target
that is defined by a hidden tree is assembled by the caller from that
tree's encoding and the noise returned here, using whatever evaluator the
caller owns. The package therefore holds no fitness arithmetic and can be
shared by the CPU oracle and the device path alike.
"""

from .trees import (  # noqa: F401
    TYPE_VAR, TYPE_CONST, TYPE_FUNC, TYPE_MODI0, ARITY, F4, F11,
    depth_limited, exact_length, pad_rows,
)
from .workloads import Workload, workload, WORKLOADS  # noqa: F401
