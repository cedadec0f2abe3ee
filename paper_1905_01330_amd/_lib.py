"""ctypes loader for libtn.so and the tn_tensor descriptor.

Argument marshalling only: every arithmetic step runs in the HIP library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtn.so")
MAX_RANK = 8

F32, F64, C64 = 0, 1, 2
PREC = {"fp32": 0, "bf16": 1, "split_bf16": 2, "split_bf16_3p": 3}

STATUS = {
    0: "ok", -1: "invalid argument", -2: "shape mismatch", -3: "unsupported",
    -4: "workspace too small", -5: "aliasing", -6: "device error",
}


class TnTensor(C.Structure):
    _fields_ = [
        ("data", C.c_void_p),
        ("dtype", C.c_int32),
        ("rank", C.c_int32),
        ("shape", C.c_int64 * MAX_RANK),
        ("stride", C.c_int64 * MAX_RANK),
    ]


class TNError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None

P = C.c_void_p
# bytes of scratch that enable the split rank-0/1 sums (TN_REDUCE_WORKSPACE_BYTES)
REDUCE_WORKSPACE_BYTES = 32768
I32 = C.c_int32
SZ = C.c_size_t
TP = C.POINTER(TnTensor)
I32P = C.POINTER(C.c_int32)

_PROTOS = {
    "tn_status_string": (C.c_char_p, [I32]),
    "tn_last_error": (C.c_char_p, []),
    "tn_version": (C.c_char_p, []),
    "tn_contract_between": (I32, [TP, TP, I32, I32P, I32P, TP, P, SZ, I32, P]),
    "tn_contract_between_c64_workspace": (I32, [TP, C.POINTER(SZ)]),
    "tn_contract_between_c64": (I32, [TP, TP, I32, I32P, I32P, I32, I32, TP, P, SZ, I32, P]),
    "tn_mps_inner_c64_workspace": (I32, [I32, TP, TP, C.POINTER(SZ)]),
    "tn_mps_inner_c64": (I32, [I32, TP, TP, P, P, SZ, I32, P]),
    "tn_trace_edge": (I32, [TP, I32, I32, TP, P]),
    "tn_outer_product": (I32, [TP, TP, TP, P]),
    "tn_contract_network_workspace": (I32, [I32, TP, I32P, I32P, I32, I32P, C.POINTER(SZ)]),
    "tn_contract_network": (I32, [I32, TP, I32P, I32P, I32, I32P, TP, P, SZ, I32, P]),
    "tn_contract_network_noalloc": (I32, [I32, TP, I32P, I32P, I32, I32P, TP, I32, P]),
    "tn_network_order": (I32, [I32, TP, I32P, I32P, I32, I32P, I32P, C.POINTER(C.c_double)]),
    "tn_mps_inner_workspace": (I32, [I32, TP, TP, C.POINTER(SZ)]),
    "tn_mps_inner": (I32, [I32, TP, TP, P, P, SZ, I32, P]),
    "tn_mps_inner_batched_workspace": (I32, [I32, I32P, TP, TP, C.POINTER(SZ)]),
    "tn_mps_inner_batched": (I32, [I32, I32P, TP, TP, P, P, SZ, I32, P]),
    "tn_mps_inner_batched_upload": (I32, [I32, I32P, TP, TP, P, SZ, P]),
    "tn_mps_inner_batched_launch": (I32, [I32, I32P, TP, TP, P, P, SZ, I32, P]),
    "tn_mps_env_sweep_workspace": (I32, [I32, TP, TP, C.POINTER(SZ)]),
    "tn_mps_env_sweep": (I32, [I32, TP, TP, TP, TP, P, I32, P, SZ, I32, P]),
    "tn_mps_left_canonicalize_workspace": (I32, [I32, TP, C.POINTER(SZ)]),
    "tn_mps_left_canonicalize": (I32, [I32, TP, P, P, SZ, P]),
    "tn_mps_classifier_ckpt_shape": (I32, [I32, I32, I32, I32, I32, C.POINTER(C.c_int64)]),
    "tn_mps_classifier_workspace": (I32, [I32, I32, I32, I32, I32, I32, C.POINTER(SZ)]),
    "tn_mps_classifier_forward": (I32, [I32, I32, I32, TP, TP, TP, P, I32, P, SZ, I32, P]),
    "tn_mps_classifier_backward": (I32, [I32, I32, I32, TP, TP, P, I32, TP, TP, P, SZ, I32, P]),
    "tn_softmax_xent": (I32, [TP, P, I32, P, TP, P, SZ, P]),
    "tn_split_node_workspace": (I32, [TP, I32, C.POINTER(SZ)]),
    "tn_split_node_decompose": (I32, [TP, I32, I32, C.c_double, I32P, I32P, P, SZ, P]),
    "tn_split_node": (I32, [TP, I32, I32, TP, TP, TP, P, SZ, P]),
    "tn_split_node_full_svd": (I32, [TP, I32, I32, TP, TP, TP, TP, P, SZ, P]),
    "tn_dmrg_workspace": (I32, [TP, TP, TP, TP, TP, I32, C.POINTER(SZ)]),
    "tn_dmrg_apply_heff": (I32, [TP, TP, TP, TP, TP, TP, P, SZ, I32, P]),
    "tn_dmrg_eigensolve": (I32, [TP, TP, TP, TP, TP, I32, I32, P, P, SZ, I32, P]),
    "tn_tune": (I32, [C.c_char_p, I32]),
    "tn_tune_set_level": (I32, [I32]),
    "tn_tune_last_choice": (I32, []),
    "tn_tune_force_config": (I32, [I32]),
    "tn_tune_force_grouped_config": (I32, [I32]),
    "tn_tune_num_configs": (I32, []),
    "tn_measure_split_mfma_rate": (I32, [I32, I32, P, P]),
}


def lib():
    """Load libtn.so (built by paper_1905_01330_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -m paper_1905_01330_amd.build` "
                "(there is no CPU fallback)")
        lb = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(lb, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lb
    return _lib


def check(code: int):
    if code != 0:
        raise TNError(code, lib().tn_last_error().decode(errors="replace"))


def tensor_desc(t, dtype=None) -> TnTensor:
    """tn_tensor view of a torch tensor (device pointer, shape, element strides)."""
    import torch

    d = TnTensor()
    if t.dim() > MAX_RANK:
        raise ValueError(f"rank {t.dim()} exceeds {MAX_RANK}")
    d.data = t.data_ptr()
    if dtype is None:
        if t.dtype == torch.float32:
            dtype = F32
        elif t.dtype == torch.float64:
            dtype = F64
        elif t.dtype == torch.complex64:
            dtype = C64
        else:
            raise TypeError(f"unsupported dtype {t.dtype}")
    d.dtype = dtype
    d.rank = t.dim()
    for i, (s, st) in enumerate(zip(t.shape, t.stride())):
        d.shape[i] = s
        d.stride[i] = st
    return d


def tensor_array(ts):
    arr = (TnTensor * max(1, len(ts)))()
    for i, t in enumerate(ts):
        arr[i] = tensor_desc(t)
    return arr


def int_array(xs):
    xs = list(xs)
    arr = (C.c_int32 * max(1, len(xs)))()
    for i, x in enumerate(xs):
        arr[i] = int(x)
    return arr


def stream_ptr(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def prec_code(prec) -> int:
    if isinstance(prec, int):
        return prec
    return PREC[prec]
