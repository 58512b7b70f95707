// Contraction orchestration, following the three steps of Section 5.2:
// (1) map each LCO operand to a matrix, permuting it only if its lexicographical
// order does not already give the layout the chosen algorithm needs;
// (2) build the multiplication datatype and multiply (row engine or SOP);
// (3) map the product back: permute it into the output label order if needed.
#include "rows.h"

namespace lco {

namespace {

struct Owned {  // a temporary tensor released on scope exit
  lco_tensor t = nullptr;
  ~Owned() {
    if (t) lco_destroy(t);
  }
};

lco_tensor permuted(lco_ctx ctx, const lco_tensor_s* in, const int* perm) {
  RpDetail plan = plan_permute(in->order, in->dims, perm, in->nnz, default_digit_cap());
  lco_tensor t = new_tensor(ctx, in->order, plan.new_dims, in->nnz);
  try {
    permute_storage(ctx, in, plan, t->livs, t->vals);
  } catch (...) {
    lco_destroy(t);
    throw;
  }
  return t;
}

}  // namespace

lco_tensor contract_run(lco_ctx ctx, const lco_tensor_s* a, const lco_tensor_s* b, const ContractDetail& d) {
  if (d.empty) return new_tensor(ctx, d.order_c, d.c_dims, 0);
  Owned ta, tb;
  const lco_tensor_s* A = a;
  const lco_tensor_s* B = b;
  if (d.pub.permute_a) A = ta.t = permuted(ctx, a, d.perm_a);
  if (d.pub.permute_b) B = tb.t = permuted(ctx, b, d.perm_b);
  const uint64_t m = d.pub.m, k = d.pub.k, n = d.pub.n;
  Owned natural;
  switch (d.pub.algo) {
    case LCO_ALG_CSR:
    case LCO_ALG_DCSR:
    case LCO_ALG_CSRNA:
      natural.t = row_engine(ctx, A, B, m, k, n, d.pub.algo != LCO_ALG_DCSR, d.pub.algo != LCO_ALG_CSRNA,
                             d.order_c, d.natural_dims);
      break;
    case LCO_ALG_CSC:
    case LCO_ALG_DCSC:
    case LCO_ALG_CSCNA:
      // column by column: C^T = B^T A^T row by row over the same arrays
      natural.t = row_engine(ctx, B, A, n, k, m, d.pub.algo != LCO_ALG_DCSC, d.pub.algo != LCO_ALG_CSCNA,
                             d.order_c, d.natural_dims);
      break;
    case LCO_ALG_SOP:
      natural.t = sop_engine(ctx, A, B, d);
      break;
    default:
      fail(LCO_E_ARG, "contract: unknown algorithm");
  }
  if (d.pub.permute_c) return permuted(ctx, natural.t, d.perm_c);
  lco_tensor out = natural.t;
  natural.t = nullptr;
  return out;
}

}  // namespace lco
