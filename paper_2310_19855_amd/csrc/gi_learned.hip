// Learned surrogate of the world cache (placeholder until the kernels land).
#include <hip/hip_runtime.h>

#include "gi_host.hpp"

namespace gi {

struct LearnedState {
  int unused;
};

hipError_t learned_create(gi_context* c) {
  c->learned = nullptr;
  return hipErrorNotSupported;
}
void learned_destroy(gi_context* c) {
  delete c->learned;
  c->learned = nullptr;
}
hipError_t learned_train(gi_context*, hipStream_t) { return hipErrorNotSupported; }
hipError_t learned_infer_rays(gi_context*, hipStream_t) { return hipErrorNotSupported; }
hipError_t learned_query(gi_context*, const float4*, const float4*, uint32_t, float4*, hipStream_t) {
  return hipErrorNotSupported;
}
size_t learned_blob_size(gi_context*) { return 0; }
hipError_t learned_save(gi_context*, void*) { return hipErrorNotSupported; }
hipError_t learned_load(gi_context*, const void*) { return hipErrorNotSupported; }
void learned_stats(gi_context*, float* out8) {
  for (int i = 0; i < 8; ++i) out8[i] = 0.0f;
}

}  // namespace gi
