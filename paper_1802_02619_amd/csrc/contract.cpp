// Contraction orchestration (Section 5.2's three steps) -- placeholder until the multiply kernels land.
#include "lco_internal.h"

namespace lco {

lco_tensor contract_run(lco_ctx ctx, const lco_tensor_s* a, const lco_tensor_s* b, const ContractDetail& d) {
  (void)a; (void)b;
  if (d.empty) return new_tensor(ctx, d.order_c, d.c_dims, 0);
  fail(LCO_E_UNSUPPORTED, "contract: not built yet");
}

}  // namespace lco
