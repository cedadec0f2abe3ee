// Contraction GEMM instantiations for x3 operands.
#include "gemm_inst.h"

namespace tn {
GemmFn gemm_fn_x3(int cfg, int variant) { return gemm_fn<P_X3>(cfg, variant); }
GroupedFn grouped_fn_x3(int cfg, int variant) { return grouped_fn<P_X3>(cfg, variant); }
}  // namespace tn
