// LCO oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded CPU implementation of what the HIP library
// computes: construction of linearised-coordinate (LCO) tensors, permutation
// of their modes, sparse tensor contraction and sparse tensor addition.  Only
// the test-suite, the smoke check and the benchmark's CPU-baseline leg may load
// this library.  It
// shares no code, header or table with the HIP library: it is written straight
// from the definitions in Harrison & Joseph, "High Performance Rearrangement
// and Multiplication Routines for Sparse Tensor Arithmetic" (SISC), using
// coordinate lists, std::stable_sort and std::map.
//
// Conventions (readings of the paper, listed in the design notes):
//  * Default lexicographical order: the first mode is the least significant,
//    LIV = c0 + n0*(c1 + n1*(c2 + ...))  (Section 3.1, the LIV formula for a_ijk).
//  * LIVs are unsigned 64-bit; the product of the dimensions may be at most 2^64.
//  * Permutation uses transpose semantics: output mode r is input mode perm[r];
//    the output is sorted in the default order of the permuted dimensions.
//  * Contraction follows Einstein notation (Section 2, y_ij = a_ijkl x_kl):
//    labels shared by the operands and absent from the output are summed; a
//    label in both operands and in the output is entrywise (the product is
//    taken only between entries that agree on it, and it is not summed); each
//    output entry accumulates its products in ascending order of the first
//    operand's LIV, and for each first-operand entry in ascending order of the
//    second operand's LIV, starting from 0.0.  Every structural non-zero (any
//    output position reached by at least one product) is kept, whatever its value.
//
// Status codes returned (kept numerically equal to the library's status enum
// by convention, not by a shared header): 0 ok, 1 bad argument, 2 index
// overflow, 3 shape mismatch, 4 unsorted input, 5 duplicate, 7 unsupported.
//
// Parity pins: see tests/test_oracle_pins.py (worked LIV example of the paper's
// Table on CO/LCO formats, dense brute force, closed-form stencils, involutions).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

namespace {

enum { ORA_OK = 0, ORA_E_ARG = 1, ORA_E_OVERFLOW = 2, ORA_E_SHAPE = 3, ORA_E_UNSORTED = 4,
       ORA_E_DUPLICATE = 5, ORA_E_UNSUPPORTED = 7 };

struct Result {
  int status = ORA_OK;
  int order = 0;
  std::vector<uint64_t> dims;
  std::vector<uint64_t> livs;
  std::vector<double> vals;
  std::vector<double> absum;  // sum of |products| per output entry (contraction only)
};

// Product of the dimensions must fit the LIV range [0, 2^64).  (Section 3.1:
// the paper limits itself to 63 bits; unsigned LIVs extend that to 2^64.)
bool dims_fit(int order, const uint64_t* dims) {
  unsigned __int128 p = 1;
  for (int r = 0; r < order; ++r) {
    if (dims[r] == 0) return false;
    p *= dims[r];
    if (p > ((unsigned __int128)1 << 64)) return false;
  }
  return true;
}

// LIV of one coordinate tuple in the default order (Section 3.1):
// LIV = c0 + n0*(c1 + n1*(c2 + ...)).
uint64_t linearise(int order, const uint64_t* dims, const uint64_t* c) {
  uint64_t liv = 0;
  for (int r = order - 1; r >= 0; --r) liv = liv * dims[r] + c[r];
  return liv;
}

// Inverse of linearise: repeated division by the dimensions in significance order.
void delinearise(int order, const uint64_t* dims, uint64_t liv, uint64_t* c) {
  for (int r = 0; r < order; ++r) {
    if (r == order - 1) {
      c[r] = liv;
    } else {
      c[r] = liv % dims[r];
      liv /= dims[r];
    }
  }
}

bool is_permutation(int order, const int* perm) {
  std::vector<int> seen(order, 0);
  for (int r = 0; r < order; ++r) {
    if (perm[r] < 0 || perm[r] >= order || seen[perm[r]]) return false;
    seen[perm[r]] = 1;
  }
  return true;
}

}  // namespace

extern "C" {

// ---- accessors -----------------------------------------------------------
int ora_status(void* h) { return static_cast<Result*>(h)->status; }
int64_t ora_nnz(void* h) { return (int64_t) static_cast<Result*>(h)->livs.size(); }
int ora_order(void* h) { return static_cast<Result*>(h)->order; }
void ora_copy(void* h, uint64_t* dims, uint64_t* livs, double* vals, double* absum) {
  Result* r = static_cast<Result*>(h);
  if (dims && r->order) std::memcpy(dims, r->dims.data(), sizeof(uint64_t) * r->order);
  if (livs && !r->livs.empty()) std::memcpy(livs, r->livs.data(), sizeof(uint64_t) * r->livs.size());
  if (vals && !r->vals.empty()) std::memcpy(vals, r->vals.data(), sizeof(double) * r->vals.size());
  if (absum && !r->absum.empty()) std::memcpy(absum, r->absum.data(), sizeof(double) * r->absum.size());
}
void ora_free(void* h) { delete static_cast<Result*>(h); }

// ---- LIV codec (Section 3.1) ----------------------------------------------
// coords: nnz rows of `order` coordinates.  Returns a status.
int ora_linearise(int order, const uint64_t* dims, int64_t nnz, const uint64_t* coords, uint64_t* livs) {
  if (order < 0 || nnz < 0) return ORA_E_ARG;
  if (!dims_fit(order, dims)) return ORA_E_OVERFLOW;
  for (int64_t i = 0; i < nnz; ++i) {
    const uint64_t* c = coords + (size_t)i * order;
    for (int r = 0; r < order; ++r)
      if (c[r] >= dims[r]) return ORA_E_ARG;
    livs[i] = linearise(order, dims, c);
  }
  return ORA_OK;
}

int ora_delinearise(int order, const uint64_t* dims, int64_t nnz, const uint64_t* livs, uint64_t* coords) {
  if (order < 0 || nnz < 0) return ORA_E_ARG;
  if (!dims_fit(order, dims)) return ORA_E_OVERFLOW;
  for (int64_t i = 0; i < nnz; ++i) delinearise(order, dims, livs[i], coords + (size_t)i * order);
  return ORA_OK;
}

// ---- construction (Section 3: an LCO tensor is a LIV list sorted in the
// lexicographical order, with a parallel value list) ------------------------
// Entries are sorted by LIV with a stable sort; with sum_dups, equal LIVs are
// summed left to right in input order (starting from the first value); without
// it a repeated LIV is an error.  Explicit zero values are kept.
void* ora_create(int order, const uint64_t* dims, int64_t nnz, const uint64_t* coords,
                 const double* vals, int sum_dups) {
  Result* res = new Result;
  res->order = order;
  if (order < 0 || nnz < 0) { res->status = ORA_E_ARG; return res; }
  res->dims.assign(dims, dims + order);
  if (!dims_fit(order, dims)) { res->status = ORA_E_OVERFLOW; return res; }
  std::vector<std::pair<uint64_t, double>> ent((size_t)nnz);
  for (int64_t i = 0; i < nnz; ++i) {
    const uint64_t* c = coords + (size_t)i * order;
    for (int r = 0; r < order; ++r)
      if (c[r] >= dims[r]) { res->status = ORA_E_ARG; return res; }
    ent[i] = {linearise(order, dims, c), vals[i]};
  }
  std::stable_sort(ent.begin(), ent.end(),
                   [](const std::pair<uint64_t, double>& a, const std::pair<uint64_t, double>& b) {
                     return a.first < b.first;
                   });
  for (size_t i = 0; i < ent.size(); ++i) {
    if (!res->livs.empty() && res->livs.back() == ent[i].first) {
      if (!sum_dups) { res->status = ORA_E_DUPLICATE; res->livs.clear(); res->vals.clear(); return res; }
      res->vals.back() += ent[i].second;
    } else {
      res->livs.push_back(ent[i].first);
      res->vals.push_back(ent[i].second);
    }
  }
  return res;
}

// ---- permutation (Section 4: rearranging already sorted data into another
// lexicographical order) -----------------------------------------------------
// The plain definition: decode every LIV to coordinates, move coordinate
// perm[r] to position r, re-linearise over the permuted dimensions, and sort.
// Input LIVs must be strictly increasing and in range.
void* ora_permute(int order, const uint64_t* dims, int64_t nnz, const uint64_t* livs,
                  const double* vals, const int* perm) {
  Result* res = new Result;
  res->order = order;
  if (order < 0 || nnz < 0 || !is_permutation(order, perm)) { res->status = ORA_E_ARG; return res; }
  if (!dims_fit(order, dims)) { res->status = ORA_E_OVERFLOW; return res; }
  std::vector<uint64_t> nd(order);
  for (int r = 0; r < order; ++r) nd[r] = dims[perm[r]];
  res->dims = nd;
  unsigned __int128 total = 1;
  for (int r = 0; r < order; ++r) total *= dims[r];
  std::vector<std::pair<uint64_t, double>> ent((size_t)nnz);
  std::vector<uint64_t> c(order), cp(order);
  for (int64_t i = 0; i < nnz; ++i) {
    if ((unsigned __int128)livs[i] >= total || (i > 0 && livs[i] <= livs[i - 1])) {
      res->status = ORA_E_UNSORTED;
      return res;
    }
    delinearise(order, dims, livs[i], c.data());
    for (int r = 0; r < order; ++r) cp[r] = c[perm[r]];
    ent[i] = {linearise(order, nd.data(), cp.data()), vals[i]};
  }
  std::sort(ent.begin(), ent.end(),
            [](const std::pair<uint64_t, double>& a, const std::pair<uint64_t, double>& b) {
              return a.first < b.first;
            });
  res->livs.resize(ent.size());
  res->vals.resize(ent.size());
  for (size_t i = 0; i < ent.size(); ++i) { res->livs[i] = ent[i].first; res->vals[i] = ent[i].second; }
  return res;
}

// ---- contraction (Section 2 Einstein notation; Section 5.2 product) --------
// mode 0: std::map accumulation (the plainest form).
// mode 1: the same products in the same generation order collected into a
//         list, stable-sorted by output LIV and summed left to right -- the
//         identical arithmetic, usable when the output is too large for a map.
void* ora_contract(int oa, const uint64_t* da, int64_t na, const uint64_t* la, const double* va, const int* laba,
                   int ob, const uint64_t* db, int64_t nb, const uint64_t* lb, const double* vb, const int* labb,
                   int oc, const int* labc, int mode) {
  Result* res = new Result;
  res->order = oc;
  if (oa < 0 || ob < 0 || oc < 0 || na < 0 || nb < 0) { res->status = ORA_E_ARG; return res; }
  if (!dims_fit(oa, da) || !dims_fit(ob, db)) { res->status = ORA_E_OVERFLOW; return res; }
  // label bookkeeping
  auto find = [](int n, const int* lab, int x) {
    for (int i = 0; i < n; ++i) if (lab[i] == x) return i;
    return -1;
  };
  for (int i = 0; i < oa; ++i) if (find(i, laba, laba[i]) >= 0) { res->status = ORA_E_UNSUPPORTED; return res; }
  for (int i = 0; i < ob; ++i) if (find(i, labb, labb[i]) >= 0) { res->status = ORA_E_UNSUPPORTED; return res; }
  for (int i = 0; i < oc; ++i) if (find(i, labc, labc[i]) >= 0) { res->status = ORA_E_ARG; return res; }
  // output sources: (operand, mode); an entrywise label is read from the first operand
  std::vector<int> src_op(oc), src_mode(oc);
  std::vector<int> ea, eb;  // entrywise labels: mode in a, mode in b
  std::vector<uint64_t> ed;
  res->dims.resize(oc);
  for (int r = 0; r < oc; ++r) {
    int ia = find(oa, laba, labc[r]), ib = find(ob, labb, labc[r]);
    if (ia < 0 && ib < 0) { res->status = ORA_E_ARG; return res; }
    if (ia >= 0 && ib >= 0) {
      if (da[ia] != db[ib]) { res->status = ORA_E_SHAPE; return res; }
      ea.push_back(ia); eb.push_back(ib); ed.push_back(da[ia]);
    }
    src_op[r] = ia >= 0 ? 0 : 1;
    src_mode[r] = ia >= 0 ? ia : ib;
    res->dims[r] = ia >= 0 ? da[ia] : db[ib];
  }
  if (!dims_fit(oc, res->dims.data())) { res->status = ORA_E_OVERFLOW; return res; }
  // contracted labels, in the order they appear in the first operand
  std::vector<int> ka, kb;
  std::vector<uint64_t> kd;
  for (int i = 0; i < oa; ++i) {
    if (find(oc, labc, laba[i]) >= 0) continue;
    int j = find(ob, labb, laba[i]);
    if (j < 0) { res->status = ORA_E_UNSUPPORTED; return res; }  // summed free label
    if (da[i] != db[j]) { res->status = ORA_E_SHAPE; return res; }
    ka.push_back(i); kb.push_back(j); kd.push_back(da[i]);
  }
  for (int j = 0; j < ob; ++j)
    if (find(oc, labc, labb[j]) < 0 && find(oa, laba, labb[j]) < 0) { res->status = ORA_E_UNSUPPORTED; return res; }
  // the join key: contracted labels (in a's order), then entrywise labels
  for (size_t t = 0; t < ea.size(); ++t) { ka.push_back(ea[t]); kb.push_back(eb[t]); kd.push_back(ed[t]); }
  const int nk = (int)ka.size();
  // index the second operand by its join coordinates; entries are pushed in
  // ascending LIV order, so each list is ascending
  std::map<uint64_t, std::vector<int64_t>> bidx;
  std::vector<uint64_t> bco((size_t)nb * ob);
  std::vector<uint64_t> kc(nk);
  for (int64_t j = 0; j < nb; ++j) {
    uint64_t* c = bco.data() + (size_t)j * ob;
    delinearise(ob, db, lb[j], c);
    for (int t = 0; t < nk; ++t) kc[t] = c[kb[t]];
    bidx[linearise(nk, kd.data(), kc.data())].push_back(j);
  }
  std::map<uint64_t, double> acc, aab;
  std::vector<std::pair<uint64_t, double>> prods;
  std::vector<uint64_t> ca(oa), cc(oc);
  for (int64_t i = 0; i < na; ++i) {
    delinearise(oa, da, la[i], ca.data());
    for (int t = 0; t < nk; ++t) kc[t] = ca[ka[t]];
    auto it = bidx.find(linearise(nk, kd.data(), kc.data()));
    if (it == bidx.end()) continue;
    for (int64_t j : it->second) {
      const uint64_t* cb = bco.data() + (size_t)j * ob;
      for (int r = 0; r < oc; ++r) cc[r] = src_op[r] == 0 ? ca[src_mode[r]] : cb[src_mode[r]];
      const uint64_t out = linearise(oc, res->dims.data(), cc.data());
      const double p = va[i] * vb[j];
      if (mode == 0) {
        acc[out] += p;
        aab[out] += std::fabs(p);
      } else {
        prods.push_back({out, p});
      }
    }
  }
  if (mode == 0) {
    res->livs.reserve(acc.size());
    for (auto& kv : acc) { res->livs.push_back(kv.first); res->vals.push_back(kv.second); }
    for (auto& kv : aab) res->absum.push_back(kv.second);
  } else {
    std::stable_sort(prods.begin(), prods.end(),
                     [](const std::pair<uint64_t, double>& a, const std::pair<uint64_t, double>& b) {
                       return a.first < b.first;
                     });
    for (size_t t = 0; t < prods.size(); ++t) {
      if (t == 0 || prods[t].first != prods[t - 1].first) {
        res->livs.push_back(prods[t].first);
        res->vals.push_back(0.0);
        res->absum.push_back(0.0);
      }
      res->vals.back() += prods[t].second;
      res->absum.back() += std::fabs(prods[t].second);
    }
  }
  return res;
}

// ---- addition (Section 2; the sum of the two terms of the combinatorial
// Laplacian, whose second term must first be re-sorted, Section 3.2) ---------
// The plain definition: decode every entry of either operand to coordinates,
// map them to the output's modes through the labels, re-linearise, and
// accumulate in a std::map: first alpha*a for every entry of a, then beta*b for
// every entry of b (added to alpha*a when the position already holds it).
// Input LIVs must be strictly increasing and in range.
void* ora_add(int order, const uint64_t* da, int64_t na, const uint64_t* la, const double* va, const int* laba,
              const uint64_t* db, int64_t nb, const uint64_t* lb, const double* vb, const int* labb,
              const int* labc, double alpha, double beta) {
  Result* res = new Result;
  res->order = order;
  if (order < 0 || na < 0 || nb < 0) { res->status = ORA_E_ARG; return res; }
  auto find = [](int n, const int* lab, int x) {
    for (int i = 0; i < n; ++i) if (lab[i] == x) return i;
    return -1;
  };
  // the three label lists must name the same set of distinct labels
  for (int i = 0; i < order; ++i) {
    if (find(i, laba, laba[i]) >= 0 || find(i, labb, labb[i]) >= 0 || find(i, labc, labc[i]) >= 0) {
      res->status = ORA_E_ARG;
      return res;
    }
  }
  std::vector<int> from_a(order), from_b(order);  // output mode r is a's mode from_a[r], b's mode from_b[r]
  res->dims.resize(order);
  for (int r = 0; r < order; ++r) {
    from_a[r] = find(order, laba, labc[r]);
    from_b[r] = find(order, labb, labc[r]);
    if (from_a[r] < 0 || from_b[r] < 0) { res->status = ORA_E_ARG; return res; }
    if (da[from_a[r]] != db[from_b[r]]) { res->status = ORA_E_SHAPE; return res; }
    res->dims[r] = da[from_a[r]];
  }
  if (!dims_fit(order, da)) { res->status = ORA_E_OVERFLOW; return res; }
  unsigned __int128 total = 1;
  for (int r = 0; r < order; ++r) total *= da[r];
  std::map<uint64_t, double> acc;
  std::vector<uint64_t> c(order), cc(order);
  for (int64_t i = 0; i < na; ++i) {
    if ((unsigned __int128)la[i] >= total || (i > 0 && la[i] <= la[i - 1])) { res->status = ORA_E_UNSORTED; return res; }
    delinearise(order, da, la[i], c.data());
    for (int r = 0; r < order; ++r) cc[r] = c[from_a[r]];
    acc[linearise(order, res->dims.data(), cc.data())] = alpha * va[i];
  }
  for (int64_t j = 0; j < nb; ++j) {
    if ((unsigned __int128)lb[j] >= total || (j > 0 && lb[j] <= lb[j - 1])) { res->status = ORA_E_UNSORTED; return res; }
    delinearise(order, db, lb[j], c.data());
    for (int r = 0; r < order; ++r) cc[r] = c[from_b[r]];
    const uint64_t out = linearise(order, res->dims.data(), cc.data());
    auto it = acc.find(out);
    if (it == acc.end()) acc[out] = beta * vb[j];
    else it->second = it->second + beta * vb[j];
  }
  res->livs.reserve(acc.size());
  res->vals.reserve(acc.size());
  for (auto& kv : acc) { res->livs.push_back(kv.first); res->vals.push_back(kv.second); }
  return res;
}

}  // extern "C"
