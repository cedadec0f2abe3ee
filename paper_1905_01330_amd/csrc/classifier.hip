// MPS classifier (section IV.A) -- entry points.
#include "internal.h"

using namespace tn;

extern "C" {

int32_t tn_mps_classifier_ckpt_shape(int32_t, int32_t, int32_t, int32_t, int32_t, int64_t*) {
  return fail(TN_ERR_UNSUPPORTED, "classifier not built yet");
}
int32_t tn_mps_classifier_workspace(int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, size_t*) {
  return fail(TN_ERR_UNSUPPORTED, "classifier not built yet");
}
int32_t tn_mps_classifier_forward(int32_t, int32_t, int32_t, const tn_tensor*, const tn_tensor*, tn_tensor*, float*,
                                  int32_t, void*, size_t, int32_t, void*) {
  return fail(TN_ERR_UNSUPPORTED, "classifier not built yet");
}
int32_t tn_mps_classifier_backward(int32_t, int32_t, int32_t, const tn_tensor*, const tn_tensor*, const float*,
                                   int32_t, const tn_tensor*, tn_tensor*, void*, size_t, int32_t, void*) {
  return fail(TN_ERR_UNSUPPORTED, "classifier not built yet");
}
}
