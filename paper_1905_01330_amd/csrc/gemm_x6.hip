// Contraction GEMM instantiations for x6 operands.
#include "gemm_inst.h"

namespace tn {
GemmFn gemm_fn_x6(int cfg, int variant) { return gemm_fn<P_X6>(cfg, variant); }
GroupedFn grouped_fn_x6(int cfg, int variant) { return grouped_fn<P_X6>(cfg, variant); }
}  // namespace tn
