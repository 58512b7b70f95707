// Host planning logic: radix-permutation plan (Section 4.1), sparsity
// classification, the multiplication table and operand orientation (Section 5.2).
// Pure functions of shapes; no device work.
#include <algorithm>
#include <cstring>

#include "lco_internal.h"

namespace lco {

namespace {

typedef unsigned __int128 u128;
const u128 kTwo64 = (u128)1 << 64;

u128 product(int order, const uint64_t* dims) {
  u128 p = 1;
  for (int r = 0; r < order; ++r) {
    p *= dims[r];
    if (p > kTwo64) return kTwo64 + 1;
  }
  return p;
}

void check_dims(int order, const uint64_t* dims, const char* what) {
  if (order < 0 || order > LCO_MAX_ORDER) fail(LCO_E_ARG, std::string(what) + ": order out of range");
  if (order && !dims) fail(LCO_E_ARG, std::string(what) + ": dims is NULL");
  for (int r = 0; r < order; ++r)
    if (dims[r] == 0) fail(LCO_E_ARG, std::string(what) + ": zero dimension");
  if (product(order, dims) > kTwo64) fail(LCO_E_OVERFLOW, std::string(what) + ": product of dimensions exceeds 2^64");
}

int bits_of_range(u128 range) {  // bits needed for values in [0, range)
  if (range <= 1) return 0;
  const u128 mx = range - 1;
  const uint64_t hi = (uint64_t)(mx >> 64), lo = (uint64_t)mx;
  return hi ? 64 + bits_for(hi) : bits_for(lo);
}

}  // namespace

// Single-tile LDS sort capacity of the permutation kernels (elements).
constexpr int64_t kSingleTileCap = 8192;

RpDetail plan_permute(int order, const uint64_t* dims, const int* perm, int64_t nnz, int digit_cap) {
  check_dims(order, dims, "permute");
  if (order && !perm) fail(LCO_E_ARG, "permute: perm is NULL");
  int newpos[LCO_MAX_ORDER];
  bool seen[LCO_MAX_ORDER] = {};
  for (int r = 0; r < order; ++r) {
    if (perm[r] < 0 || perm[r] >= order || seen[perm[r]]) fail(LCO_E_ARG, "permute: perm is not a permutation");
    seen[perm[r]] = true;
    newpos[perm[r]] = r;
  }
  RpDetail d;
  std::memset(&d, 0, sizeof(d));
  d.order = order;
  for (int r = 0; r < order; ++r) d.new_dims[r] = dims[perm[r]];
  // weights of the new order: W'_r = prod_{s<r} n'_s (mod 2^64; a weight of 2^64
  // can only multiply a coordinate of a size-1 mode, which is always 0)
  uint64_t wnew[LCO_MAX_ORDER];
  uint64_t w = 1;
  for (int r = 0; r < order; ++r) { wnew[r] = w; w *= d.new_dims[r]; }
  for (int q = 0; q < order; ++q) d.new_weight_of_input_mode[q] = wnew[newpos[q]];

  // Rearrangement indices (Section 4.1): mode x must be re-sorted iff it moves
  // above a mode y that was originally more significant.  Size-1 modes carry no
  // information and are ignored.
  uint32_t rearr = 0;
  for (int x = 0; x < order; ++x) {
    if (dims[x] <= 1) continue;
    for (int y = x + 1; y < order; ++y)
      if (dims[y] > 1 && newpos[y] < newpos[x]) { rearr |= 1u << x; break; }
  }
  // leading resting modes shared by both orders (the top of both orders agree)
  std::vector<int> old_eff, new_eff;
  for (int q = 0; q < order; ++q) if (dims[q] > 1) old_eff.push_back(q);
  for (int r = 0; r < order; ++r) if (dims[perm[r]] > 1) new_eff.push_back(perm[r]);
  int p = 0;
  while (p < (int)old_eff.size() && old_eff[old_eff.size() - 1 - p] == new_eff[new_eff.size() - 1 - p]) ++p;
  int hi_pos = order;  // new positions >= hi_pos form the segment prefix
  if (p > 0) hi_pos = newpos[new_eff[new_eff.size() - p]];
  int lo_pos = order;  // least significant new position of a rearrangement index
  for (int x = 0; x < order; ++x)
    if (rearr & (1u << x)) lo_pos = std::min(lo_pos, newpos[x]);

  lco_rp_plan& pub = d.pub;
  pub.rearrangement = rearr;
  pub.prefix = p;
  pub.full_bits = bits_of_range(product(order, dims));
  if (rearr == 0) {
    pub.identity = 1;
    pub.method = 0;
    pub.suffix = order;
    pub.key_div = 1;
    pub.key_range = 1;
    pub.seg_div = 1;
    d.sort_bits = 0;
    return d;
  }
  pub.suffix = lo_pos;
  u128 kdiv = 1, krange = 1, above = 1, nseg = 1;
  for (int r = 0; r < lo_pos; ++r) kdiv *= d.new_dims[r];
  for (int r = lo_pos; r < hi_pos; ++r) krange *= d.new_dims[r];
  for (int r = lo_pos; r < order; ++r) above *= d.new_dims[r];
  for (int r = hi_pos; r < order; ++r) nseg *= d.new_dims[r];
  u128 sdiv = 1;  // old-LIV divisor of the segment id: product of the non-prefix dims
  for (int r = 0; r < hi_pos; ++r) sdiv *= d.new_dims[r];
  pub.key_div = (uint64_t)kdiv;  // < 2^64: a rearrangement mode lies above
  pub.key_range = krange >= kTwo64 ? ~0ull : (uint64_t)krange;
  pub.seg_div = sdiv >= kTwo64 ? ~0ull : (uint64_t)sdiv;
  pub.key_bits = bits_of_range(krange);
  pub.seg_bits = bits_of_range(nseg);
  if (nnz <= kSingleTileCap) {
    pub.method = 1;
    d.sort_bits = bits_of_range(above);
  } else if (p == 0) {
    pub.method = 2;
    d.sort_bits = pub.key_bits;
  } else {
    pub.method = 3;  // falls back to 4 at run time when a segment exceeds a tile
    d.sort_bits = bits_of_range(above);
    d.avg_segment = (double)nnz / (double)nseg;
  }
  if (digit_cap < 1) digit_cap = 8;
  pub.passes = d.sort_bits ? (d.sort_bits + digit_cap - 1) / digit_cap : 0;
  pub.digit_bits = pub.passes ? (d.sort_bits + pub.passes - 1) / pub.passes : 0;
  if (d.sort_bits == 0) {  // every keyed mode has size 1: order unchanged
    pub.identity = 1;
    pub.method = 0;
  }
  return d;
}

// ---------------------------------------------------------------- selector

int classify(uint64_t rows, uint64_t cols, int64_t nnz) {
  // Section 5.2: hyper-sparse along a dimension when dimension / nnz > 3.
  const u128 lim = (u128)3 * (u128)(nnz > 0 ? nnz : 0);
  const bool row_sp = (u128)rows > lim;
  const bool col_sp = (u128)cols > lim;
  return row_sp && col_sp ? LCO_INDEX_SPARSE : row_sp ? LCO_ROW_SPARSE : col_sp ? LCO_COL_SPARSE : LCO_SPARSE;
}

// The paper's table (rows: class of A; columns: class of B), indexed by lco_sparsity.
static const int kTable[4][4][2] = {
    /* A sparse     */ {{LCO_ALG_CSC, LCO_ALG_CSR}, {LCO_ALG_CSC, LCO_ALG_CSC},
                        {LCO_ALG_CSC, LCO_ALG_CSC}, {LCO_ALG_CSC, LCO_ALG_CSC}},
    /* A row-sparse */ {{LCO_ALG_CSR, LCO_ALG_CSR}, {LCO_ALG_DCSR, LCO_ALG_DCSR},
                        {LCO_ALG_CSCNA, LCO_ALG_CSRNA}, {LCO_ALG_CSCNA, LCO_ALG_CSCNA}},
    /* A col-sparse */ {{LCO_ALG_CSR, LCO_ALG_CSR}, {LCO_ALG_DCSC, LCO_ALG_DCSR},
                        {LCO_ALG_DCSC, LCO_ALG_DCSC}, {LCO_ALG_DCSC, LCO_ALG_DCSC}},
    /* A idx-sparse */ {{LCO_ALG_CSR, LCO_ALG_CSR}, {LCO_ALG_DCSR, LCO_ALG_DCSR},
                        {LCO_ALG_CSRNA, LCO_ALG_CSRNA}, {LCO_ALG_SOP, LCO_ALG_SOP}},
};

static int family(int algo) {  // 0: column-by-column, 1: row-by-row, 2: outer product
  switch (algo) {
    case LCO_ALG_CSC: case LCO_ALG_DCSC: case LCO_ALG_CSCNA: return 0;
    case LCO_ALG_CSR: case LCO_ALG_DCSR: case LCO_ALG_CSRNA: return 1;
    default: return 2;
  }
}

namespace {

struct Layouts {
  int pa[2 * LCO_MAX_ORDER], pb[2 * LCO_MAX_ORDER];  // operand modes, least significant first
  int natural[LCO_MAX_ORDER];  // natural product layout as a list of C positions
  int na, nb, nc;              // layout lengths (an operand with entrywise modes lists them twice)
  int dup = 0;                 // 1: A is block diagonal (entrywise modes twice), 2: B
  uint64_t em = 0, ek = 0, en = 0;
  int cost;
  bool need_a, need_b, need_c;
};

bool is_identity(const int* p, int n) {
  for (int i = 0; i < n; ++i) if (p[i] != i) return false;
  return true;
}

}  // namespace

ContractDetail plan_contract(int oa, const uint64_t* da, const int* la, int64_t na, int ob, const uint64_t* db,
                             const int* lb, int64_t nb, int oc, const int* lc, uint32_t flags,
                             const Selector* sel) {
  check_dims(oa, da, "contract operand a");
  check_dims(ob, db, "contract operand b");
  if (oc < 0 || oc > LCO_MAX_ORDER) fail(LCO_E_ARG, "contract: output order out of range");
  if ((oa && !la) || (ob && !lb) || (oc && !lc)) fail(LCO_E_ARG, "contract: labels are NULL");
  if (na < 0 || nb < 0) fail(LCO_E_ARG, "contract: negative nnz");
  const uint32_t force = flags & LCO_FORCE_MASK;
  if (force > LCO_ALG_SOP) fail(LCO_E_ARG, "contract: unknown forced algorithm");
  auto find = [](int n, const int* l, int x) {
    for (int i = 0; i < n; ++i) if (l[i] == x) return i;
    return -1;
  };
  for (int i = 0; i < oa; ++i) if (find(i, la, la[i]) >= 0) fail(LCO_E_ARG, "contract: label repeated within a");
  for (int i = 0; i < ob; ++i) if (find(i, lb, lb[i]) >= 0) fail(LCO_E_ARG, "contract: label repeated within b");
  for (int i = 0; i < oc; ++i) if (find(i, lc, lc[i]) >= 0) fail(LCO_E_ARG, "contract: label repeated in output");

  ContractDetail d;
  std::memset(&d, 0, sizeof(d));
  d.order_a = oa; d.order_b = ob; d.order_c = oc;
  // output modes: free in a, free in b, or entrywise (in a, b and the output)
  int fa_c[LCO_MAX_ORDER], fb_c[LCO_MAX_ORDER];  // operand mode index, in C order
  int fa_cpos[LCO_MAX_ORDER], fb_cpos[LCO_MAX_ORDER];
  int ea_c[LCO_MAX_ORDER], eb_c[LCO_MAX_ORDER], e_cpos[LCO_MAX_ORDER];
  int nfa = 0, nfb = 0, ne = 0;
  u128 cprod = 1;
  for (int r = 0; r < oc; ++r) {
    const int ia = find(oa, la, lc[r]), ib = find(ob, lb, lc[r]);
    if (ia < 0 && ib < 0) fail(LCO_E_ARG, "contract: output label not found in a or b");
    if (ia >= 0 && ib >= 0) {
      if (da[ia] != db[ib]) fail(LCO_E_SHAPE, "contract: entrywise modes differ in dimension");
      ea_c[ne] = ia; eb_c[ne] = ib; e_cpos[ne++] = r; d.c_dims[r] = da[ia];
    } else if (ia >= 0) {
      fa_cpos[nfa] = r; fa_c[nfa++] = ia; d.c_dims[r] = da[ia];
    } else {
      fb_cpos[nfb] = r; fb_c[nfb++] = ib; d.c_dims[r] = db[ib];
    }
    cprod *= d.c_dims[r];
    if (cprod > kTwo64) fail(LCO_E_OVERFLOW, "contract: output dimension product exceeds 2^64");
  }
  // contracted labels, in a's order and in b's order
  int ka_a[LCO_MAX_ORDER], ka_b[LCO_MAX_ORDER], nk = 0;  // kappa_A: (a index, b index)
  for (int i = 0; i < oa; ++i) {
    if (find(oc, lc, la[i]) >= 0) continue;
    const int j = find(ob, lb, la[i]);
    if (j < 0) fail(LCO_E_UNSUPPORTED, "contract: free label of a missing from the output");
    if (da[i] != db[j]) fail(LCO_E_SHAPE, "contract: contracted modes differ in dimension");
    ka_a[nk] = i; ka_b[nk] = j; ++nk;
  }
  for (int j = 0; j < ob; ++j)
    if (find(oc, lc, lb[j]) < 0 && find(oa, la, lb[j]) < 0)
      fail(LCO_E_UNSUPPORTED, "contract: free label of b missing from the output");
  int kb_a[LCO_MAX_ORDER], kb_b[LCO_MAX_ORDER];  // kappa_B order
  {
    int t = 0;
    for (int j = 0; j < ob; ++j) {
      const int i = find(oa, la, lb[j]);
      if (i >= 0 && find(oc, lc, lb[j]) < 0) { kb_a[t] = i; kb_b[t] = j; ++t; }
    }
  }
  // entrywise modes in a's order and in b's order: (mode in a, mode in b, output position)
  int eo_a[3][LCO_MAX_ORDER], eo_b[3][LCO_MAX_ORDER];
  {
    int t = 0;
    for (int i = 0; i < oa; ++i)
      for (int e = 0; e < ne; ++e)
        if (ea_c[e] == i) { eo_a[0][t] = ea_c[e]; eo_a[1][t] = eb_c[e]; eo_a[2][t++] = e_cpos[e]; }
    t = 0;
    for (int j = 0; j < ob; ++j)
      for (int e = 0; e < ne; ++e)
        if (eb_c[e] == j) { eo_b[0][t] = ea_c[e]; eo_b[1][t] = eb_c[e]; eo_b[2][t++] = e_cpos[e]; }
  }
  // Matricised sizes.  With entrywise modes the product is block diagonal, one
  // block per entrywise index: A is (free a x E) by (contracted x E), B is
  // (contracted x E) by (free b x E).
  u128 m = 1, k = 1, n = 1, h = 1, mf = 1, nf = 1;
  for (int t = 0; t < nfa; ++t) mf *= da[fa_c[t]];
  for (int t = 0; t < nk; ++t) k *= da[ka_a[t]];
  for (int t = 0; t < nfb; ++t) nf *= db[fb_c[t]];
  for (int e = 0; e < ne; ++e) h *= da[ea_c[e]];
  m = mf * h;
  n = nf * h;
  k = k * h;
  if (m >= kTwo64 || k >= kTwo64 || n >= kTwo64)
    fail(LCO_E_UNSUPPORTED, "contract: a matricised side of 2^64 or more");
  lco_plan& pub = d.pub;
  pub.m = (uint64_t)m; pub.k = (uint64_t)k; pub.n = (uint64_t)n;
  pub.nnz_a = na; pub.nnz_b = nb;
  pub.num_contracted = nk;
  pub.num_entrywise = ne;
  pub.a_class = classify(pub.m, pub.k, na);
  pub.b_class = classify(pub.k, pub.n, nb);
  d.n_free_a = nfa; d.n_free_b = nfb; d.n_contracted = nk; d.n_entrywise = ne;

  // Layout of each family for a given contracted order, and its rearrangement
  // cost.  The operand that plays the engine's row side holds the entrywise
  // modes twice (once with its rows, once with its columns, so that it is block
  // diagonal); the other holds them once, after the contracted modes.
  auto layouts = [&](int fam, const int* kap_a, const int* kap_b) {
    Layouts L;
    L.nc = oc;
    int ia = 0, ib = 0, ic = 0;
    const int(*eo)[LCO_MAX_ORDER] = fam == 0 ? eo_a : eo_b;  // entrywise order: that of the plain operand
    if (fam == 0) {  // column by column: A (free, contracted, E) plain; B (contracted, E, free, E)
      for (int t = 0; t < nfa; ++t) L.pa[ia++] = fa_c[t];
      for (int t = 0; t < nk; ++t) L.pa[ia++] = kap_a[t];
      for (int e = 0; e < ne; ++e) L.pa[ia++] = eo[0][e];
      for (int t = 0; t < nk; ++t) L.pb[ib++] = kap_b[t];
      for (int e = 0; e < ne; ++e) L.pb[ib++] = eo[1][e];
      for (int t = 0; t < nfb; ++t) L.pb[ib++] = fb_c[t];
      if (ne) for (int e = 0; e < ne; ++e) L.pb[ib++] = eo[1][e];
      for (int t = 0; t < nfa; ++t) L.natural[ic++] = fa_cpos[t];
      for (int t = 0; t < nfb; ++t) L.natural[ic++] = fb_cpos[t];
      L.dup = ne ? 2 : 0;
      L.em = (uint64_t)n; L.ek = (uint64_t)k; L.en = (uint64_t)mf;
    } else if (fam == 1) {  // row by row: A (contracted, E, free, E); B (free, contracted, E) plain
      for (int t = 0; t < nk; ++t) L.pa[ia++] = kap_a[t];
      for (int e = 0; e < ne; ++e) L.pa[ia++] = eo[0][e];
      for (int t = 0; t < nfa; ++t) L.pa[ia++] = fa_c[t];
      if (ne) for (int e = 0; e < ne; ++e) L.pa[ia++] = eo[0][e];
      for (int t = 0; t < nfb; ++t) L.pb[ib++] = fb_c[t];
      for (int t = 0; t < nk; ++t) L.pb[ib++] = kap_b[t];
      for (int e = 0; e < ne; ++e) L.pb[ib++] = eo[1][e];
      for (int t = 0; t < nfb; ++t) L.natural[ic++] = fb_cpos[t];
      for (int t = 0; t < nfa; ++t) L.natural[ic++] = fa_cpos[t];
      L.dup = ne ? 1 : 0;
      L.em = (uint64_t)m; L.ek = (uint64_t)k; L.en = (uint64_t)nf;
    } else {  // outer product: A (free and E in a's order, contracted, E); B (free, contracted, E) plain
      for (int i = 0; i < oa; ++i) if (find(oc, lc, la[i]) >= 0) L.pa[ia++] = i;
      for (int t = 0; t < nk; ++t) L.pa[ia++] = kap_a[t];
      for (int e = 0; e < ne; ++e) L.pa[ia++] = eo[0][e];
      for (int j = 0; j < ob; ++j) if (find(oc, lc, lb[j]) >= 0 && find(oa, la, lb[j]) < 0) L.pb[ib++] = j;
      for (int t = 0; t < nk; ++t) L.pb[ib++] = kap_b[t];
      for (int e = 0; e < ne; ++e) L.pb[ib++] = eo[1][e];
      for (int r = 0; r < oc; ++r) L.natural[r] = r;  // the sort key is the output LIV itself
      L.dup = ne ? 1 : 0;
      L.em = (uint64_t)m; L.ek = (uint64_t)k; L.en = (uint64_t)nf;
    }
    for (int e = 0; e < ne && fam != 2; ++e) L.natural[ic++] = eo[2][e];  // in the layout's entrywise order
    L.na = ia;
    L.nb = ib;
    L.need_a = L.dup == 1 || !is_identity(L.pa, oa);
    L.need_b = L.dup == 2 || !is_identity(L.pb, ob);
    L.need_c = !is_identity(L.natural, oc);
    L.cost = (int)L.need_a + (int)L.need_b + (int)L.need_c;
    return L;
  };
  // Fewest rearrangements first; the contracted order of a wins ties, which keeps
  // the order of summation that of the first operand's LIVs.
  auto best = [&](int fam) {
    Layouts x = layouts(fam, ka_a, ka_b);
    Layouts y = layouts(fam, kb_a, kb_b);
    return y.cost < x.cost ? y : x;
  };

  int algo;
  if (force) {
    algo = (int)force;
  } else {
    const int* cell = kTable[pub.a_class][pub.b_class];
    algo = cell[0];
    if (cell[0] != cell[1]) {
      // Section 5.2.2: choose the orientation that needs fewer extra sorts; otherwise
      // the column-by-column variant iff n > m.
      const int c0 = best(family(cell[0])).cost, c1 = best(family(cell[1])).cost;
      if (c1 < c0) algo = cell[1];
      else if (c0 == c1) algo = (pub.n > pub.m) ? cell[0] : cell[1];
    }
    if (sel) {
      // Measured crossovers: the cell's specialised algorithm gives way to the
      // singly compressed accumulator one while the operand is only mildly
      // hyper-sparse (the cell and its orientation stay the paper's).  The
      // index-sparse cell's SOP may give way to the doubly compressed
      // accumulator algorithms above that, oriented like the singly
      // compressed ones (fewest rearrangements, then n > m).
      const double* cross = sel->cross;
      auto ratio = [](uint64_t dim, int64_t nz) { return nz > 0 ? (long double)dim / (long double)nz : 0.0L; };
      const long double s_dc = algo == LCO_ALG_DCSC ? ratio(pub.k, na) : ratio(pub.k, nb);
      const long double s_na = algo == LCO_ALG_CSCNA ? ratio(pub.m, na) : ratio(pub.n, nb);
      const long double s_op = std::min(std::min(ratio(pub.m, na), ratio(pub.k, na)),
                                        std::min(ratio(pub.k, nb), ratio(pub.n, nb)));
      if ((algo == LCO_ALG_DCSC || algo == LCO_ALG_DCSR) && s_dc <= cross[0])
        algo = algo == LCO_ALG_DCSC ? LCO_ALG_CSC : LCO_ALG_CSR;
      else if ((algo == LCO_ALG_CSCNA || algo == LCO_ALG_CSRNA) && s_na <= cross[1])
        algo = algo == LCO_ALG_CSCNA ? LCO_ALG_CSC : LCO_ALG_CSR;
      else if (algo == LCO_ALG_SOP && (s_op <= cross[2] || sel->index_dc)) {
        const int c0 = best(0).cost, c1 = best(1).cost;
        const bool by_col = c0 < c1 || (c0 == c1 && pub.n > pub.m);
        if (s_op <= cross[2]) algo = by_col ? LCO_ALG_CSC : LCO_ALG_CSR;
        else algo = by_col ? LCO_ALG_DCSC : LCO_ALG_DCSR;
      }
    }
  }
  pub.algo = algo;
  const int fam = family(algo);
  Layouts L = best(fam);
  d.em = L.em; d.ek = L.ek; d.en = L.en;
  d.dup = L.dup;
  if (L.dup) {
    // the block-diagonal operand: weight of each of its modes in its matricised LIV
    const int* lay = L.dup == 1 ? L.pa : L.pb;
    const int len = L.dup == 1 ? L.na : L.nb;
    const uint64_t* dd = L.dup == 1 ? da : db;
    u128 w = 1;
    for (int r = 0; r < len; ++r) {
      d.dup_weight[lay[r]] += (uint64_t)w;
      w *= dd[lay[r]];
      if (w > kTwo64) fail(LCO_E_UNSUPPORTED, "contract: block-diagonal form of an operand exceeds 2^64");
    }
    d.dup_bits = bits_of_range(w);
    d.dup_dims[0] = (uint64_t)k;
    d.dup_dims[1] = (uint64_t)(w / k);
  } else {
    std::memcpy(d.perm_a, L.pa, sizeof(int) * oa);
    std::memcpy(d.perm_b, L.pb, sizeof(int) * ob);
  }
  if (L.dup == 2) std::memcpy(d.perm_a, L.pa, sizeof(int) * oa);
  if (L.dup == 1) std::memcpy(d.perm_b, L.pb, sizeof(int) * ob);
  pub.permute_a = L.need_a;
  pub.permute_b = L.need_b;
  pub.permute_c = L.need_c;
  // natural layout dims and the permutation natural -> output
  for (int s = 0; s < oc; ++s) d.natural_dims[s] = d.c_dims[L.natural[s]];
  for (int r = 0; r < oc; ++r)
    for (int s = 0; s < oc; ++s)
      if (L.natural[s] == r) d.perm_c[r] = s;
  if (fam == 2) {
    // output-LIV weights of the free (and entrywise) modes of A and the free modes of B
    uint64_t wc[LCO_MAX_ORDER];
    uint64_t w = 1;
    for (int r = 0; r < oc; ++r) { wc[r] = w; w *= d.c_dims[r]; }
    int t = 0;
    bool simple = true;
    int expect = 0;
    for (int i = 0; i < oa; ++i) {
      const int r = find(oc, lc, la[L.pa[i]]);
      if (r < 0) continue;
      d.free_a_dims[t] = da[L.pa[i]];
      d.free_a_cweight[t++] = wc[r];
      if (r != expect++) simple = false;
    }
    d.n_free_a = t;
    t = 0;
    for (int j = 0; j < nfb; ++j) {
      const int r = find(oc, lc, lb[L.pb[j]]);
      d.free_b_dims[t] = db[L.pb[j]];
      d.free_b_cweight[t++] = wc[r];
      if (r != expect++) simple = false;
    }
    d.sop_simple_key = simple;
  }
  d.empty = (na == 0 || nb == 0);
  return d;
}

AddDetail plan_add(int oa, const uint64_t* da, const int* la, int ob, const uint64_t* db, const int* lb,
                   const int* lc) {
  check_dims(oa, da, "add operand a");
  check_dims(ob, db, "add operand b");
  if (oa != ob) fail(LCO_E_ARG, "add: operands of different orders");
  if (oa && (!la || !lb || !lc)) fail(LCO_E_ARG, "add: labels are NULL");
  auto find = [](int n, const int* l, int x) {
    for (int i = 0; i < n; ++i) if (l[i] == x) return i;
    return -1;
  };
  for (int i = 0; i < oa; ++i) {
    if (find(i, la, la[i]) >= 0 || find(i, lb, lb[i]) >= 0 || find(i, lc, lc[i]) >= 0)
      fail(LCO_E_ARG, "add: repeated label");
  }
  AddDetail d;
  d.order = oa;
  for (int r = 0; r < oa; ++r) {
    const int ia = find(oa, la, lc[r]), ib = find(ob, lb, lc[r]);
    if (ia < 0 || ib < 0) fail(LCO_E_ARG, "add: the label lists name different sets of modes");
    if (da[ia] != db[ib]) fail(LCO_E_SHAPE, "add: modes with the same label differ in dimension");
    d.perm_a[r] = ia;
    d.perm_b[r] = ib;
    d.c_dims[r] = da[ia];
    d.permute_a |= ia != r;
    d.permute_b |= ib != r;
  }
  return d;
}

}  // namespace lco

// ---------------------------------------------------------------- C-ABI (host-only)
using namespace lco;

namespace lco {
lco_status set_error(const Error& e);
lco_status set_error_msg(lco_status s, const char* msg);
void clear_error();
}  // namespace lco

extern "C" lco_status lco_classify(uint64_t rows, uint64_t cols, int64_t nnz, int* cls) {
  if (!cls || nnz < 0) return set_error_msg(LCO_E_ARG, "lco_classify: bad argument");
  *cls = classify(rows, cols, nnz);
  return LCO_OK;
}

extern "C" lco_status lco_select(int a_class, int b_class, int* first, int* second) {
  if (a_class < 0 || a_class > 3 || b_class < 0 || b_class > 3 || !first || !second)
    return set_error_msg(LCO_E_ARG, "lco_select: bad argument");
  *first = kTable[a_class][b_class][0];
  *second = kTable[a_class][b_class][1];
  return LCO_OK;
}

extern "C" lco_status lco_plan_contract(int a_order, const uint64_t* a_dims, const int* a_labels, int64_t a_nnz,
                                        int b_order, const uint64_t* b_dims, const int* b_labels, int64_t b_nnz,
                                        int c_order, const int* c_labels, uint32_t flags, lco_plan* out) {
  try {
    if (!out) fail(LCO_E_ARG, "lco_plan_contract: out is NULL");
    ContractDetail d = plan_contract(a_order, a_dims, a_labels, a_nnz, b_order, b_dims, b_labels, b_nnz, c_order,
                                     c_labels, flags);
    *out = d.pub;
    return LCO_OK;
  } catch (const Error& e) {
    return set_error(e);
  }
}

extern "C" lco_status lco_plan_permute(int order, const uint64_t* dims, const int* perm, int64_t nnz,
                                       lco_rp_plan* out) {
  try {
    if (!out) fail(LCO_E_ARG, "lco_plan_permute: out is NULL");
    RpDetail d = plan_permute(order, dims, perm, nnz, 8);
    *out = d.pub;
    return LCO_OK;
  } catch (const Error& e) {
    return set_error(e);
  }
}

extern "C" lco_status lco_fastdiv_host(uint64_t d, int64_t count, const uint64_t* num, uint64_t* quot,
                                       uint64_t* rem) {
  if (d == 0 || count < 0 || (count && (!num || !quot || !rem)))
    return set_error_msg(LCO_E_ARG, "lco_fastdiv_host: bad argument");
  const FastDiv f = make_fastdiv(d);
  for (int64_t i = 0; i < count; ++i) quot[i] = fd_divmod(f, num[i], rem[i]);
  return LCO_OK;
}
