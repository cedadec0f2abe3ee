// Contraction GEMM instantiations for x3 operands.
#include "gemm_inst.h"

namespace tn {
GemmFn gemm_fn_x3(int cfg) { return gemm_fn<P_X3>(cfg); }
GroupedFn grouped_fn_x3(int cfg) { return grouped_fn<P_X3>(cfg); }
}  // namespace tn
