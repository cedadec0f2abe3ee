"""MI355X (gfx950) tensor-network contraction library.

Python entry points mirror the C ABI in include/tn.h; the arithmetic runs in
libtn.so (hand-written HIP kernels).  Importing the package does not load
the library; the first call does, and fails loudly if it is not built.
"""
from .api import (  # noqa: F401
    BatchedInner,
    ClassifierFunction,
    MPSClassifier,
    EnvSweep,
    Graph,
    contract_between,
    contract_network,
    dmrg,
    dmrg_apply_heff,
    dmrg_eigensolve,
    dmrg_two_site_update,
    mps_env_sweep,
    mps_inner,
    mps_inner_batched,
    mps_inner_complex,
    mps_left_canonicalize,
    network_order,
    outer_product,
    softmax_xent,
    split_node,
    split_node_full_svd,
    tensordot,
    trace_edge,
    tune,
    tune_force_config,
    tune_force_grouped_config,
    tune_last_choice,
    tune_num_configs,
    measure_split_mfma_rate,
    tune_set_level,
)

from ._lib import TNError  # noqa: F401

__version__ = "0.1.0"
