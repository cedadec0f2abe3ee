// Precision dispatch of the contraction GEMM instantiation tables.
#include "gemm_inst_decl.h"

namespace tn {
GemmFn gemm_fn_fp32(int cfg, int variant);
GemmFn gemm_fn_bf16(int cfg, int variant);
GemmFn gemm_fn_x6(int cfg, int variant);
GemmFn gemm_fn_x3(int cfg, int variant);
GroupedFn grouped_fn_fp32(int cfg, int variant);
GroupedFn grouped_fn_bf16(int cfg, int variant);
GroupedFn grouped_fn_x6(int cfg, int variant);
GroupedFn grouped_fn_x3(int cfg, int variant);

GemmFn gemm_fn_prec(int prec, int cfg, int variant) {
  switch (prec) {
    case TN_PREC_FP32: return gemm_fn_fp32(cfg, variant);
    case TN_PREC_BF16: return gemm_fn_bf16(cfg, variant);
    case TN_PREC_SPLIT_BF16: return gemm_fn_x6(cfg, variant);
    default: return gemm_fn_x3(cfg, variant);
  }
}

GroupedFn grouped_fn_prec(int prec, int cfg, int variant) {
  switch (prec) {
    case TN_PREC_FP32: return grouped_fn_fp32(cfg, variant);
    case TN_PREC_BF16: return grouped_fn_bf16(cfg, variant);
    case TN_PREC_SPLIT_BF16: return grouped_fn_x6(cfg, variant);
    default: return grouped_fn_x3(cfg, variant);
  }
}
}  // namespace tn
