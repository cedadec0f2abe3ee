// Instantiation table of the lean-stage split-BF16 contraction kernels.
#include "gemm_inst_decl.h"
#include "gemm_split_kernel.h"

namespace tn {

// kind 1: both operands split into LDS, 160 x 256 tile, eight waves;
// kind 2: B private to each wave, 160 x 256, eight waves;
// kind 3: B private, 160 x 128 tile in two k groups of four waves.
GemmFn split_fn(int kind, int bmode) {
  const bool mn = bmode == LOAD_MNVEC;
  switch (kind) {
    case 1: return mn ? split_gemm_kernel<160, 256, 8, LOAD_MNVEC> : split_gemm_kernel<160, 256, 8, LOAD_KVEC>;
    case 2: return mn ? split_gemm_p_kernel<160, 256, LOAD_MNVEC, 1> : split_gemm_p_kernel<160, 256, LOAD_KVEC, 1>;
    default: return mn ? split_gemm_p_kernel<160, 128, LOAD_MNVEC, 2> : split_gemm_p_kernel<160, 128, LOAD_KVEC, 2>;
  }
}

}  // namespace tn
