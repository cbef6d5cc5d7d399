// Learned initial-guess proposer (placeholder until the network lands).
#include "ctx.h"

namespace ndtm {
int guess_mlp(ndtm_ctx* c, const std::vector<double>&, const std::vector<HalfField>&, int, double, const HalfField&,
              const std::vector<double>&, std::vector<double>*, double*, double*, hipStream_t) {
  return fail(c, NDTM_ESTATE, "guess network: not loaded");
}
}  // namespace ndtm

extern "C" void ndtm_mlp_free(ndtm_ctx*) {}
