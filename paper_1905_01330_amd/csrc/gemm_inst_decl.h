// Declarations of the contraction GEMM instantiation tables.
#pragma once

#include "internal.h"

namespace tn {
typedef void (*GemmFn)(const GemmDesc);
typedef void (*GroupedFn)(const Gemm2D*, const int32_t*, int32_t);
GemmFn gemm_fn_prec(int prec, int cfg, int variant);
GroupedFn grouped_fn_prec(int prec, int cfg, int variant);
}  // namespace tn
