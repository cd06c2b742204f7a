// CPU oracle for the filter -> PK-FK hash join -> hash group-by pipeline.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
// calls this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark do. It shares no code, header, table or constant with
// the GPU library: only the generated input columns are common.
//
// What it computes is the plain relational definition of the query whose
// kernels the paper profiles (hash join build / count / retrieve and
// shared-memory group-by, Section 7 and Table 9):
//
//   SELECT g, SUM(price_cents), SUM(qty), COUNT(*)
//   FROM fact JOIN dim ON fact.fk = dim.pk
//   WHERE fact.day < T
//   GROUP BY g
//
// with g one of (dim.prio, fact.flag), fact.fk, or dim.grp. Sums and counts
// are 64-bit integers that wrap modulo 2^64. Only non-empty groups are
// returned, sorted ascending by key. The data layout is columnar, one plain
// array per column (the Arrow-compatible layout of Section 2.3).
//
// Implementation: single-threaded textbook code. std::unordered_map for the
// join (pk -> dim row) and for the grouping (key -> running sums), then
// std::sort. A second, independent brute-force implementation (nested loop
// over fact x dim, linear-scan group list) pins the first on tiny inputs.
//
// Join output can also be materialised: the gather out[i] = in[map[i]] of
// selected fact and dim columns through the probe's row pairs.
//
// The planner's sketch (HyperLogLog registers of Flajolet, Fusy, Gandouet and
// Meunier, AofA 2007, and the 40 sample statistics) is also here, so the GPU
// sketch can be compared register by register.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

enum GroupBy : int32_t { GB_PRIO_FLAG = 0, GB_FK = 1, GB_DIM_GRP = 2 };
enum CmpOp : int32_t { OP_LT = 0, OP_LE = 1, OP_GT = 2, OP_GE = 3, OP_EQ = 4, OP_NE = 5 };

constexpr int64_t ERR_DUPLICATE_KEY = -1;
constexpr int64_t ERR_CAPACITY = -2;
constexpr int64_t ERR_INVALID = -3;

struct Agg {
  uint64_t sum_price = 0;
  uint64_t sum_qty = 0;
  uint64_t count = 0;
};

bool cmp(int32_t v, int32_t op, int32_t lit) {
  switch (op) {
    case OP_LT: return v < lit;
    case OP_LE: return v <= lit;
    case OP_GT: return v > lit;
    case OP_GE: return v >= lit;
    case OP_EQ: return v == lit;
    case OP_NE: return v != lit;
  }
  return false;
}

// (prio, flag) as one ordered integer: prio * 256 + flag read as an unsigned byte.
int64_t prio_flag_key(int8_t prio, int8_t flag) { return (int64_t)prio * 256 + (int64_t)(uint8_t)flag; }

int64_t emit_sorted(std::vector<std::pair<int64_t, Agg>>& groups, int64_t* out_key, int64_t* out_sp, int64_t* out_sq,
                    int64_t* out_cnt, int64_t out_cap) {
  std::sort(groups.begin(), groups.end(),
            [](const std::pair<int64_t, Agg>& a, const std::pair<int64_t, Agg>& b) { return a.first < b.first; });
  if ((int64_t)groups.size() > out_cap) return ERR_CAPACITY;
  for (size_t g = 0; g < groups.size(); ++g) {
    out_key[g] = groups[g].first;
    out_sp[g] = (int64_t)groups[g].second.sum_price;
    out_sq[g] = (int64_t)groups[g].second.sum_qty;
    out_cnt[g] = (int64_t)groups[g].second.count;
  }
  return (int64_t)groups.size();
}

}  // namespace

extern "C" {

// The whole query. stats (nullable) receives {rows_passed, join_matches, groups}.
// Returns the number of groups, or ERR_DUPLICATE_KEY / ERR_CAPACITY / ERR_INVALID.
int64_t or_filter_join_agg(int64_t n, const int32_t* fk, const int64_t* price, const int32_t* qty, const int32_t* day,
                           const int8_t* flag, int64_t m, const int32_t* pk, const int8_t* prio, const int32_t* grp,
                           int32_t day_lt, int32_t group_by, int64_t* out_key, int64_t* out_sp, int64_t* out_sq,
                           int64_t* out_cnt, int64_t out_cap, int64_t* stats) {
  if (n < 0 || m < 0) return ERR_INVALID;
  if (group_by == GB_DIM_GRP && grp == nullptr && m > 0) return ERR_INVALID;
  // Build: pk -> dim row.
  std::unordered_map<int32_t, int64_t> dim_row;
  dim_row.reserve((size_t)m);
  for (int64_t j = 0; j < m; ++j) {
    if (!dim_row.emplace(pk[j], j).second) return ERR_DUPLICATE_KEY;
  }
  // Filter, probe, aggregate.
  std::unordered_map<int64_t, Agg> acc;
  acc.reserve((size_t)std::min<int64_t>(n, std::max<int64_t>(m, 1)));
  int64_t passed = 0, matched = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!(day[i] < day_lt)) continue;
    ++passed;
    auto it = dim_row.find(fk[i]);
    if (it == dim_row.end()) continue;  // inner join drops unmatched rows
    ++matched;
    const int64_t j = it->second;
    int64_t key;
    if (group_by == GB_PRIO_FLAG) key = prio_flag_key(prio[j], flag[i]);
    else if (group_by == GB_FK) key = fk[i];
    else key = grp[j];
    Agg& a = acc[key];
    a.sum_price += (uint64_t)price[i];
    a.sum_qty += (uint64_t)(int64_t)qty[i];
    a.count += 1;
  }
  std::vector<std::pair<int64_t, Agg>> groups(acc.begin(), acc.end());
  const int64_t ng = emit_sorted(groups, out_key, out_sp, out_sq, out_cnt, out_cap);
  if (stats) {
    stats[0] = passed;
    stats[1] = matched;
    stats[2] = (int64_t)groups.size();
  }
  return ng;
}

// Independent brute force: nested loop over every (fact, dim) pair and a
// group list searched linearly. Quadratic; tiny inputs only.
int64_t or_brute_filter_join_agg(int64_t n, const int32_t* fk, const int64_t* price, const int32_t* qty,
                                 const int32_t* day, const int8_t* flag, int64_t m, const int32_t* pk,
                                 const int8_t* prio, const int32_t* grp, int32_t day_lt, int32_t group_by,
                                 int64_t* out_key, int64_t* out_sp, int64_t* out_sq, int64_t* out_cnt, int64_t out_cap,
                                 int64_t* stats) {
  if (n < 0 || m < 0) return ERR_INVALID;
  for (int64_t a = 0; a < m; ++a)
    for (int64_t b = a + 1; b < m; ++b)
      if (pk[a] == pk[b]) return ERR_DUPLICATE_KEY;
  std::vector<int64_t> keys;
  std::vector<Agg> aggs;
  int64_t passed = 0, matched = 0;
  for (int64_t i = 0; i < n; ++i) {
    const bool pass = day[i] < day_lt;
    passed += pass;
    for (int64_t j = 0; j < m; ++j) {
      if (!pass || fk[i] != pk[j]) continue;
      ++matched;
      int64_t key = group_by == GB_PRIO_FLAG ? prio_flag_key(prio[j], flag[i])
                    : group_by == GB_FK      ? (int64_t)fk[i]
                                             : (int64_t)grp[j];
      size_t g = 0;
      while (g < keys.size() && keys[g] != key) ++g;
      if (g == keys.size()) {
        keys.push_back(key);
        aggs.push_back(Agg());
      }
      aggs[g].sum_price += (uint64_t)price[i];
      aggs[g].sum_qty += (uint64_t)(int64_t)qty[i];
      aggs[g].count += 1;
    }
  }
  std::vector<std::pair<int64_t, Agg>> groups;
  for (size_t g = 0; g < keys.size(); ++g) groups.emplace_back(keys[g], aggs[g]);
  const int64_t ng = emit_sorted(groups, out_key, out_sp, out_sq, out_cnt, out_cap);
  if (stats) {
    stats[0] = passed;
    stats[1] = matched;
    stats[2] = (int64_t)groups.size();
  }
  return ng;
}

// Selection vector: ascending row ids i with cmp(col[i], op, literal).
int64_t or_filter_compact(int64_t n, const int32_t* col, int32_t op, int32_t literal, int32_t* out_idx,
                          int64_t out_cap) {
  if (n < 0 || op < OP_LT || op > OP_NE) return ERR_INVALID;
  int64_t c = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!cmp(col[i], op, literal)) continue;
    if (c >= out_cap) return ERR_CAPACITY;
    out_idx[c++] = (int32_t)i;
  }
  return c;
}

// Join probe: for each probe position k (row = sel ? sel[k] : k) whose fk
// matches a pk, one pair (row, payload of the matching dim row). payload
// nullable: then the dim row id. Pairs come out ordered by position k.
int64_t or_join_probe(int64_t n, const int32_t* fk, const int32_t* sel, int64_t m, const int32_t* pk,
                      const int32_t* payload, int32_t* out_fact_idx, int32_t* out_payload, int64_t out_cap) {
  if (n < 0 || m < 0) return ERR_INVALID;
  std::unordered_map<int32_t, int32_t> table;
  table.reserve((size_t)m);
  for (int64_t j = 0; j < m; ++j) {
    if (!table.emplace(pk[j], payload ? payload[j] : (int32_t)j).second) return ERR_DUPLICATE_KEY;
  }
  int64_t c = 0;
  for (int64_t k = 0; k < n; ++k) {
    const int64_t row = sel ? sel[k] : k;
    auto it = table.find(fk[row]);
    if (it == table.end()) continue;
    if (c >= out_cap) return ERR_CAPACITY;
    out_fact_idx[c] = (int32_t)row;
    out_payload[c] = it->second;
    ++c;
  }
  return c;
}

// General selection predicate: row i passes when every term holds for it. A
// term compares its column's value (integers widened to int64, floating point
// to double) with its literals: <, <=, >, >=, ==, != against one literal,
// BETWEEN lo and hi (both inclusive), or IN a list of up to 16 values (the
// selection of the compute-column step, Section 7, over typed columns).
struct OrPredTerm {
  int32_t column, dtype, op, n_values;  // dtype: i8 i16 i32 i64 f32 f64; op: lt le gt ge eq ne between in
  int64_t iv[16];
  double fv[16];
};

static bool or_term_holds(const OrPredTerm& t, const void* col, int64_t r) {
  bool fp = false;
  int64_t x = 0;
  double y = 0.0;
  switch (t.dtype) {
    case 0: x = static_cast<const int8_t*>(col)[r]; break;
    case 1: x = static_cast<const int16_t*>(col)[r]; break;
    case 2: x = static_cast<const int32_t*>(col)[r]; break;
    case 3: x = static_cast<const int64_t*>(col)[r]; break;
    case 4: fp = true; y = static_cast<const float*>(col)[r]; break;
    default: fp = true; y = static_cast<const double*>(col)[r]; break;
  }
  auto cmp = [&](int op, int j) {
    switch (op) {
      case 0: return fp ? y < t.fv[j] : x < t.iv[j];
      case 1: return fp ? y <= t.fv[j] : x <= t.iv[j];
      case 2: return fp ? y > t.fv[j] : x > t.iv[j];
      case 3: return fp ? y >= t.fv[j] : x >= t.iv[j];
      case 4: return fp ? y == t.fv[j] : x == t.iv[j];
      default: return fp ? y != t.fv[j] : x != t.iv[j];
    }
  };
  if (t.op <= 5) return cmp(t.op, 0);
  if (t.op == 6) return cmp(3, 0) && cmp(1, 1);
  for (int j = 0; j < t.n_values; ++j)
    if (cmp(4, j)) return true;
  return false;
}

int64_t or_pred_filter(int64_t n, const void* const* cols, int32_t ncols, const OrPredTerm* terms, int32_t nterms,
                       int32_t* out, int64_t out_cap) {
  if (n < 0 || nterms < 1) return ERR_INVALID;
  for (int32_t i = 0; i < nterms; ++i) {
    const OrPredTerm& t = terms[i];
    if (t.column < 0 || t.column >= ncols || !cols[t.column] || t.dtype < 0 || t.dtype > 5 || t.op < 0 || t.op > 7 ||
        t.n_values < 1 || t.n_values > 16)
      return ERR_INVALID;
  }
  int64_t c = 0;
  for (int64_t r = 0; r < n; ++r) {
    bool ok = true;
    for (int32_t i = 0; i < nterms && ok; ++i) ok = or_term_holds(terms[i], cols[terms[i].column], r);
    if (!ok) continue;
    if (c >= out_cap) return ERR_CAPACITY;
    out[c++] = (int32_t)r;
  }
  return c;
}

// Materialisation of join output (the gather out[i] = in[map[i]] of the
// transform kernel, Section 7): dst[i] = src[idx[i]] for i in [0, n), elements
// of elem_bytes bytes copied as bytes. An index outside [0, src_rows) is an
// error (ERR_INVALID), as is an element size other than 1, 2, 4 or 8.
int64_t or_join_gather(int64_t n, const int32_t* idx, const void* src, int64_t src_rows, int32_t elem_bytes,
                       void* dst) {
  if (n < 0 || src_rows < 0 || (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8))
    return ERR_INVALID;
  const unsigned char* s = static_cast<const unsigned char*>(src);
  unsigned char* d = static_cast<unsigned char*>(dst);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t row = idx[i];
    if (row < 0 || row >= src_rows) return ERR_INVALID;
    std::memcpy(d + i * elem_bytes, s + row * elem_bytes, (size_t)elem_bytes);
  }
  return n;
}

// Hash group-by over the rows sel[0..n) (or 0..n-1): key, SUM(price), SUM(qty), COUNT.
int64_t or_groupby_agg(int64_t n, const int64_t* key, const int64_t* price, const int32_t* qty, const int32_t* sel,
                       int64_t* out_key, int64_t* out_sp, int64_t* out_sq, int64_t* out_cnt, int64_t out_cap) {
  if (n < 0) return ERR_INVALID;
  std::unordered_map<int64_t, Agg> acc;
  for (int64_t k = 0; k < n; ++k) {
    const int64_t row = sel ? sel[k] : k;
    Agg& a = acc[key[row]];
    a.sum_price += (uint64_t)price[row];
    a.sum_qty += (uint64_t)(int64_t)qty[row];
    a.count += 1;
  }
  std::vector<std::pair<int64_t, Agg>> groups(acc.begin(), acc.end());
  return emit_sorted(groups, out_key, out_sp, out_sq, out_cnt, out_cap);
}

// ---------------------------------------------------------------------------------------------------------------------
// Planner sketch.
//
// HyperLogLog (Flajolet et al. 2007) with m = 64 registers (p = 6 index bits).
// Hash of an int32 key v: the first output of SplitMix64 seeded with the key,
// i.e. the SplitMix64 finaliser applied to (uint32 v) + 0x9E3779B97F4A7C15.
// Register index = the top 6 bits of the hash; rho = 1 + the number of leading
// zeros of the remaining 58 bits (59 when they are all zero). Each register
// keeps the maximum rho seen.

static uint64_t hll_hash(int32_t v) {
  uint64_t z = (uint64_t)(uint32_t)v + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The 64-bit hash of one key, exported so that tests can compare it with
// SplitMix64's published output sequence.
uint64_t or_hll_hash(int32_t v) { return hll_hash(v); }

void or_hll_registers(int64_t n, const int32_t* keys, uint8_t* regs /*64*/) {
  for (int r = 0; r < 64; ++r) regs[r] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t h = hll_hash(keys[i]);
    const int idx = (int)(h >> 58);
    const uint64_t w = h << 6;  // remaining 58 bits, left-aligned
    int rho = 1;
    while (rho <= 58 && !(w & (1ull << (64 - rho)))) ++rho;  // position of the leftmost 1, or 59
    if (rho > regs[idx]) regs[idx] = (uint8_t)rho;
  }
}

// Raw estimate alpha_m m^2 / sum 2^-M[j] with alpha_64 = 0.709, replaced by
// linear counting m ln(m / V) when the raw estimate is at most 5m/2 and V > 0
// registers are zero.
double or_hll_estimate(const uint8_t* regs) {
  const double mm = 64.0;
  double z = 0.0;
  int zeros = 0;
  for (int r = 0; r < 64; ++r) {
    z += std::ldexp(1.0, -(int)regs[r]);
    zeros += regs[r] == 0;
  }
  double e = 0.709 * mm * mm / z;
  if (e <= 2.5 * mm && zeros > 0) e = mm * std::log(mm / (double)zeros);
  return e;
}

// The planner's 40 input features. fact_sample / dim_sample are row indices
// drawn by the caller (with replacement); grp nullable. Layout:
//  0 log2(1+N)  1 log2(1+M)  2 log2((1+N)/(1+M))  3 sample selectivity
//  4..6 one-hot group mode (fk, dim_grp, prio_flag)
//  7..10 sampled fk: distinct, singletons, doubletons, max frequency (each / k)
//  11 fraction of sampled fk inside [min, max] of sampled pk
//  12 log2(1 + range of sampled fk)  13 log2(1 + range of sampled pk)
//  14..16 sampled grp: distinct / k, singletons / k, log2(1 + range)
//  17..20 HLL(fk): log2(1+estimate), zero-register fraction, mean register / 16, max register / 64
//  21..36 histogram of the 64 fk registers, value v in bin min(v, 15), as fractions
//  37..38 HLL(grp): log2(1+estimate), zero-register fraction
//  39 Pearson correlation of (day, fk) over the fact sample (0 if degenerate)
void or_sketch_features(int64_t n, const int32_t* fk, const int32_t* day, int64_t m, const int32_t* pk,
                        const int32_t* grp, int32_t day_lt, int32_t group_by, int64_t k, const int64_t* fact_sample,
                        const int64_t* dim_sample, const uint8_t* hll_fk, const uint8_t* hll_grp, double* f /*40*/) {
  for (int i = 0; i < 40; ++i) f[i] = 0.0;
  f[0] = std::log2(1.0 + (double)n);
  f[1] = std::log2(1.0 + (double)m);
  f[2] = std::log2((1.0 + (double)n) / (1.0 + (double)m));
  f[4] = group_by == GB_FK;
  f[5] = group_by == GB_DIM_GRP;
  f[6] = group_by == GB_PRIO_FLAG;
  const double kk = (double)k;
  if (n > 0 && k > 0) {
    std::vector<int32_t> s_fk, s_day;
    int64_t pass = 0;
    for (int64_t t = 0; t < k; ++t) {
      s_fk.push_back(fk[fact_sample[t]]);
      s_day.push_back(day[fact_sample[t]]);
      pass += day[fact_sample[t]] < day_lt;
    }
    f[3] = (double)pass / kk;
    std::unordered_map<int32_t, int64_t> freq;
    for (int32_t v : s_fk) ++freq[v];
    int64_t f1 = 0, f2 = 0, mx = 0;
    for (auto& kv : freq) {
      f1 += kv.second == 1;
      f2 += kv.second == 2;
      mx = std::max(mx, kv.second);
    }
    f[7] = (double)freq.size() / kk;
    f[8] = (double)f1 / kk;
    f[9] = (double)f2 / kk;
    f[10] = (double)mx / kk;
    const int32_t fmin = *std::min_element(s_fk.begin(), s_fk.end());
    const int32_t fmax = *std::max_element(s_fk.begin(), s_fk.end());
    f[12] = std::log2(1.0 + ((double)fmax - (double)fmin));
    if (m > 0) {
      int32_t pmin = pk[dim_sample[0]], pmax = pmin;
      for (int64_t t = 0; t < k; ++t) {
        pmin = std::min(pmin, pk[dim_sample[t]]);
        pmax = std::max(pmax, pk[dim_sample[t]]);
      }
      int64_t inside = 0;
      for (int32_t v : s_fk) inside += (v >= pmin && v <= pmax);
      f[11] = (double)inside / kk;
      f[13] = std::log2(1.0 + ((double)pmax - (double)pmin));
    }
    // Pearson correlation, two-pass.
    double md = 0, mf = 0;
    for (int64_t t = 0; t < k; ++t) {
      md += s_day[t];
      mf += s_fk[t];
    }
    md /= kk;
    mf /= kk;
    double sdd = 0, sff = 0, sdf = 0;
    for (int64_t t = 0; t < k; ++t) {
      const double a = s_day[t] - md, b = s_fk[t] - mf;
      sdd += a * a;
      sff += b * b;
      sdf += a * b;
    }
    f[39] = (sdd > 0 && sff > 0) ? sdf / std::sqrt(sdd * sff) : 0.0;
  }
  if (grp != nullptr && m > 0 && k > 0) {
    std::unordered_map<int32_t, int64_t> freq;
    int32_t gmin = grp[dim_sample[0]], gmax = gmin;
    for (int64_t t = 0; t < k; ++t) {
      const int32_t v = grp[dim_sample[t]];
      ++freq[v];
      gmin = std::min(gmin, v);
      gmax = std::max(gmax, v);
    }
    int64_t f1 = 0;
    for (auto& kv : freq) f1 += kv.second == 1;
    f[14] = (double)freq.size() / kk;
    f[15] = (double)f1 / kk;
    f[16] = std::log2(1.0 + ((double)gmax - (double)gmin));
  }
  {
    int zeros = 0, mx = 0;
    double sum = 0;
    for (int r = 0; r < 64; ++r) {
      zeros += hll_fk[r] == 0;
      mx = std::max(mx, (int)hll_fk[r]);
      sum += hll_fk[r];
      f[21 + std::min<int>(hll_fk[r], 15)] += 1.0 / 64.0;
    }
    f[17] = std::log2(1.0 + or_hll_estimate(hll_fk));
    f[18] = zeros / 64.0;
    f[19] = sum / 64.0 / 16.0;
    f[20] = mx / 64.0;
  }
  if (grp != nullptr) {
    int zeros = 0;
    for (int r = 0; r < 64; ++r) zeros += hll_grp[r] == 0;
    f[37] = std::log2(1.0 + or_hll_estimate(hll_grp));
    f[38] = zeros / 64.0;
  }
}

}  // extern "C"
