"""MI355X (gfx950) fitness evaluation for tensorized tree genetic programming.

The device library libtgp.so (include/tgp.h) evaluates a population of
expression trees in the paper's NaN-padded prefix encoding on every data
point and reduces to one mean squared error per tree; it also produces
multi-output predictions and gradients, and builds the next population's
trees by subtree exchange (crossover and mutation) and draws random trees. This package is a thin binding:
torch provides device memory and streams, the HIP kernels do all the work.
"""

from ._lib import (  # noqa: F401
    MODE_AUTO, MODE_TREE_MAJOR, MODE_POINT_MAJOR, MODE_PERSISTENT, FLAG_NO_TAIL_CHECK, TgpError, load,
    status_str, LIB_PATH, XCHG_OK, XCHG_TOO_LONG, XCHG_BAD_OLD, XCHG_BAD_DONOR,
)
from .api import (  # noqa: F401
    Population, Workspace, cfg, workspace_bytes, plan, eval_mse, eval_mse_noalloc, eval_multi_output, eval_accuracy,
    eval_mse_grad, autotune, autotune_cached, op_apply, autotune_cache_load, autotune_cache_save, GraphedCall,
    subtree_exchange, crossover, mutation, generate, TreeMSE,
)
