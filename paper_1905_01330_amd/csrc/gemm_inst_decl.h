// Declarations of the contraction GEMM instantiation tables.
#pragma once

#include "internal.h"

namespace tn {
typedef void (*GemmFn)(const GemmDesc);
typedef void (*GroupedFn)(const Gemm2D*, const int32_t*, int32_t);
GemmFn gemm_fn_prec(int prec, int cfg, int variant);
GroupedFn grouped_fn_prec(int prec, int cfg, int variant);
// lean-stage split-BF16 kernels (gemm_split.hip): kind 1..3, bmode LOAD_KVEC or LOAD_MNVEC
GemmFn split_fn(int kind, int bmode);
}  // namespace tn
