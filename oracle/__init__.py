"""FP64 CPU oracle for the tensor-network contraction path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this; only
the tests, the smoke check and the benchmark's CPU-baseline leg may call it.
It shares no code with the GPU library: it reads plain numpy arrays that the
tests pass in and returns float64 numpy arrays.

Every function states the definition it writes out and the passage of
"TensorNetwork: A Library for Physics and Machine Learning" (arXiv:1905.01330)
it follows.  A library matmul is allowed as a step; nothing is blocked, fused
or reordered beyond what the definition says.
"""
from .contract import (  # noqa: F401
    tensordot,
    contract_between,
    trace_edge,
    outer_product,
    contract_network,
    feature_map,
)
from .mps import (  # noqa: F401
    mps_inner,
    mps_inner_value,
    left_canonicalize,
    env_sweep,
    env_left_step,
    env_right_step,
    mps_to_dense,
    mpo_to_dense,
)
from .classifier import (  # noqa: F401
    classifier_forward,
    classifier_loss,
    classifier_loss_and_grad,
)
from .precision import bf16_round, split3, emulate_split_gemm  # noqa: F401
from .split import split_node, split_node_full_svd, truncation_rank  # noqa: F401
from .dmrg import heff_apply, heff_dense, two_site_update, dmrg  # noqa: F401
from .complex import tensordot_c, mps_inner_c, mps_to_dense_c  # noqa: F401
