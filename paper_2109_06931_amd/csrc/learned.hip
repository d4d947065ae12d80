// A7: learned interval index (placeholder until the model is built).
#include "hpa_internal.h"

namespace hpa {

struct LearnedModel {};

void learned_train(hpa_structure_map*, hipStream_t) {
  fail(HPA_E_UNSUPPORTED, "learned index not built in this library yet");
}

void launch_lookup_learned(const hpa_structure_map*, const uint64_t*, uint64_t, uint32_t*, hipStream_t) {
  fail(HPA_E_UNSUPPORTED, "learned index not built in this library yet");
}

void learned_free(LearnedModel* lm) { delete lm; }

}  // namespace hpa
