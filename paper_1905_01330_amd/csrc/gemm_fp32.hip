// Contraction GEMM instantiations for fp32 operands.
#include "gemm_inst.h"

namespace tn {
GemmFn gemm_fn_fp32(int cfg, int variant) { return gemm_fn<P_FP32>(cfg, variant); }
GroupedFn grouped_fn_fp32(int cfg, int variant) { return grouped_fn<P_FP32>(cfg, variant); }
}  // namespace tn
