#include "context.hpp"

using namespace expint;

extern "C" {

int expint_grad(expint_ctx*, const void*, int32_t, const void*, int32_t, double*, void*, double*, double*) {
  return set_error(EXPINT_EUNSUPPORTED, "adjoint not available in this build");
}

int expint_vjp(expint_ctx*, const void*, int32_t, const void*, int32_t, void*, double*, double*) {
  return set_error(EXPINT_EUNSUPPORTED, "adjoint not available in this build");
}

}  // extern "C"
