#include "context.hpp"

using namespace expint;

extern "C" {

int expint_batch_create(int32_t, const expint_grid*, const expint_dfield*, const double*, expint_bc,
                        const expint_opts*, expint_batch** out) {
  if (out) *out = nullptr;
  return set_error(EXPINT_EUNSUPPORTED, "batch not available in this build");
}
int expint_batch_advance(expint_batch*, void* const*, int32_t) {
  return set_error(EXPINT_EUNSUPPORTED, "batch not available in this build");
}
int expint_batch_get_plan(const expint_batch*, int32_t, int32_t*, int32_t*, double*) {
  return set_error(EXPINT_EUNSUPPORTED, "batch not available in this build");
}
void expint_batch_destroy(expint_batch*) {}

}  // extern "C"
