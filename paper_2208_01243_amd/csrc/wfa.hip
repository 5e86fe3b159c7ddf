// Gap-affine wavefront alignment (placeholder until the kernel lands).
#include "aim_internal.h"

namespace aim {

int64_t wfa_slot_words(int32_t max_len, const Scoring &P) { return 64; }

hipError_t launch_wfa(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                      int32_t *arena, int64_t slot_words, int32_t max_len, int32_t nslots,
                      hipStream_t s) {
  return hipErrorNotSupported;
}

}  // namespace aim
