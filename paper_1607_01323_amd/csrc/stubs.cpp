// Entry points whose implementation lives in later translation units.
#include "internal.h"
using namespace dgmf;
extern "C" {
dgmf_status dgmf_convective_create(dgmf_mesh, const dgmf_conv_desc*, dgmf_op*) {
  return fail(DGMF_UNSUPPORTED, "convective not built");
}
dgmf_status dgmf_convective_apply(dgmf_op, const double*, double*, hipStream_t) {
  return fail(DGMF_UNSUPPORTED, "convective not built");
}
dgmf_status dgmf_convective_vjp(dgmf_op, const double*, const double*, double*, hipStream_t) {
  return fail(DGMF_UNSUPPORTED, "convective not built");
}
}
