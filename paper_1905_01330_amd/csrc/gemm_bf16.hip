// Contraction GEMM instantiations for bf16 operands.
#include "gemm_inst.h"

namespace tn {
GemmFn gemm_fn_bf16(int cfg, int variant) { return gemm_fn<P_BF16>(cfg, variant); }
GroupedFn grouped_fn_bf16(int cfg, int variant) { return grouped_fn<P_BF16>(cfg, variant); }
}  // namespace tn
