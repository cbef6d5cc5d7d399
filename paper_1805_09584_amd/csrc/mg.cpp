// Multigrid driver (placeholder until the aggregation multigrid lands).
#include "ctx.h"

namespace ndtm {
int solve_mg_shifts(ndtm_ctx* c, const std::vector<double>&, int, std::vector<HalfField>&, const HalfField&,
                    const ndtm_solve_params*, ndtm_solve_report*, hipStream_t) {
  return fail(c, NDTM_ESTATE, "multigrid shifts: not available");
}
}  // namespace ndtm

using namespace ndtm;
extern "C" {
void ndtm_mg_free(ndtm_ctx*) {}
void ndtm_mlp_free(ndtm_ctx*) {}
void ndtm_mg_default_params(ndtm_mg_params* p) {
  if (!p) return;
  p->block[0] = p->block[1] = p->block[2] = p->block[3] = 4;
  p->n_vec = 24;
  p->setup_iters = 6;
  p->setup_smooth = 4;
  p->smooth_iters = 2;
  p->coarse_iters = 16;
  p->coarse_mu_factor = 1.0;
  p->seed = 32;
  p->precision = NDTM_PREC_F64;
}
int ndtm_mg_setup(ndtm_ctx* c, const ndtm_mg_params*, const void*, void*) { return fail(c, NDTM_ESTATE, "mg: not available"); }
long long ndtm_mg_coarse_volume(const ndtm_ctx*) { return 0; }
int ndtm_mg_restrict(ndtm_ctx* c, void*, const void*, void*) { return fail(c, NDTM_ESTATE, "mg: not available"); }
int ndtm_mg_prolong(ndtm_ctx* c, void*, const void*, void*) { return fail(c, NDTM_ESTATE, "mg: not available"); }
int ndtm_mg_coarse_apply(ndtm_ctx* c, void*, const void*, double, void*) { return fail(c, NDTM_ESTATE, "mg: not available"); }
}
