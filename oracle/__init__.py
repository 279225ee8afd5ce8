"""FP64 CPU oracle of the CFG-pair similarity (TEST INFRASTRUCTURE).

Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of
`bench.py` may import or call anything in this package.  The product path
(the HIP library and its Python binding) never touches it, and this package
imports nothing from the product.  See `oracle/cfsim_ref.py` for the
readings of the paper it implements, `oracle/bf16_model.py` for the
model of the BF16 matrix-core variant and `oracle/distances.py` for the
elementwise distances of Table 1 and `oracle/damped.py` for the damped
IsoRank measure (Table 1's full form), `oracle/assign.py` for the
optimal-assignment matching and `oracle/ward.py` for Ward's clustering.
"""
from .cfsim_ref import (  # noqa: F401
    CONVERGED, HIT_MAX_ITER, DEGENERATE, INVALID_INPUT,
    transition_matrix, transition_matrix_sparse, resize_bilinear,
    apply_operator, coupled_iteration, greedy_match, score_pair,
    backward, edge_gradients, topk, PairResult,
)
from .bf16_model import round_bf16, coupled_iteration_bf16  # noqa: F401
from .distances import NAMES as DISTANCE_NAMES, scaled_pair, elementwise_distances, pair_distances  # noqa: F401
from .damped import column_sums, apply_normalised, damped_iteration, score_pair_damped  # noqa: F401
from .assign import optimal_assignment  # noqa: F401
from .ward import squared_distances, ward_linkage  # noqa: F401
