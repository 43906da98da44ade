// Entry points whose implementation lives in later translation units.
#include "internal.h"
using namespace dgmf;
extern "C" {
dgmf_status dgmf_cg_workspace_bytes(dgmf_op, const dgmf_cg_params*, size_t*) {
  return fail(DGMF_UNSUPPORTED, "cg not built");
}
dgmf_status dgmf_cg_solve(dgmf_op, const double*, double*, const dgmf_cg_params*, void*, size_t, hipStream_t,
                          dgmf_cg_result*) {
  return fail(DGMF_UNSUPPORTED, "cg not built");
}
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
