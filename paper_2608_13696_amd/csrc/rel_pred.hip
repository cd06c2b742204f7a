// General selection predicates: a conjunction of typed terms, compiled or
// interpreted (declared in rel.h).
//
// Both modes are one program text built with hipRTC for the device it runs
// on: a single-pass stable compaction (Merrill and Garland's decoupled
// look-back by one wave, four consecutive tiles per ticket so every awaited
// tile belongs to a running workgroup, as in rel_filter.hip) around a function that yields, for one
// thread's run of consecutive rows (32 compiled, 16 interpreted), the bit mask
// of the rows that pass. The
// selected row numbers of a tile are staged in LDS and written out by
// consecutive lanes.
//   * compiled: the mask function is generated for the predicate. Each term
//     reads its column's elements, 16 at a time, with 16-byte loads and compares them
//     against literals written into the code; no branch depends on the term
//     list.
//   * interpreted: the mask function walks a term list in device memory for
//     every row, dispatching on the column type and the operator (the
//     expression-interpretation scheme Section 7 measures in cuDF).
#include <hip/hiprtc.h>

#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "rel_host.h"

namespace {

// Rows per thread, written in front of the program text: 32 for generated
// masks (two groups of 16-byte loads per column), 16 for the interpreter,
// whose rows are evaluated one after another.
// Rows per thread. Compiled: 32 when the predicate reads at most 8 bytes per
// row, else 16 (a thread's loads for 32 rows of wide columns hold so many
// registers that fewer waves fit; measured on 60M rows: the 4-term predicate
// over 17 B per row 0.370 ms at 32, 0.316 ms at 16; day < 1200 alone 0.104 ms
// at 32, 0.117 ms at 16). The interpreter evaluates its rows one after
// another and keeps 16.
int rows_per_thread(int32_t mode, int bytes_per_row) {
  return mode == REL_PRED_COMPILED && bytes_per_row <= 8 ? 32 : 16;
}

// Bytes of one element of a rel_dtype (I8, I16, I32, I64, F32, F64).
int dtype_bytes(int dt) {
  static const int kBytes[] = {1, 2, 4, 8, 4, 8};
  return dt >= 0 && dt < 6 ? kBytes[dt] : 8;
}

// The kernel's name in each mode (profiles tell the two apart by it).
const char* kernel_name(int32_t mode) { return mode == REL_PRED_COMPILED ? "k_pred_compiled" : "k_pred_interpreted"; }

// The compaction around the mask function `tile_bits`, which the program text
// defines after it.
const char* kSkeleton = R"SKEL(
typedef struct {
  int column, dtype, op, n_values;
  long long iv[16];
  double fv[16];
} Term;
typedef struct { const void* c[8]; } Cols;

#define BLOCK 256
#define TILE (BLOCK * IPT)
#define FLAG_AGG (1ull << 62)
#define FLAG_INCL (2ull << 62)
#define VAL_MASK ((1ull << 62) - 1)

// 16 consecutive elements of T from a 16-byte aligned address.
template <class T>
__device__ __forceinline__ void load16(const T* p, T (&v)[16]) {
  const uint4* q = reinterpret_cast<const uint4*>(p);
  uint4 w[sizeof(T)];
#pragma unroll
  for (int j = 0; j < (int)sizeof(T); ++j) w[j] = q[j];
  __builtin_memcpy(v, w, sizeof(w));
}

__device__ __forceinline__ unsigned tile_bits(const Cols& cols, long long r0, long long n, const Term* terms, int nterms);

extern "C" __global__ __launch_bounds__(BLOCK) void PRED_KERNEL(Cols cols, long long n, int* out,
                                                                  unsigned long long* state, long long* ticket,
                                                                  long long* d_count, long long ngroups,
                                                                  const Term* terms, int nterms) {
  // a ticket is a group of TILES_PER_TICKET consecutive tiles: all their rows
  // are tested, the group's count is published and looked back once, then
  // the tiles are staged and written in turn; per-thread counts of the tiles
  // travel packed, 16 bits a tile, in one word
  __shared__ long long s_group;
  __shared__ long long s_excl;
  __shared__ unsigned long long s_wave[BLOCK / 64];
  __shared__ int s_rows[TILE];
  if (threadIdx.x == 0) s_group = (long long)atomicAdd((unsigned long long*)ticket, 1ull);
  __syncthreads();
  const long long group = s_group;
  const long long t0 = group * TILES_PER_TICKET;
  unsigned bits[TILES_PER_TICKET];
  unsigned long long c = 0;
#pragma unroll
  for (int g = 0; g < TILES_PER_TICKET; ++g) {
    const long long r0 = (t0 + g) * TILE + (long long)threadIdx.x * IPT;
    bits[g] = r0 < n ? tile_bits(cols, r0, n, terms, nterms) : 0u;
    c |= (unsigned long long)__popc(bits[g]) << (16 * g);
  }
  const unsigned lane = __lane_id(), wave = threadIdx.x / 64;
  unsigned long long incl = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_up(incl, o, 64);
    if (lane >= (unsigned)o) incl += t;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  unsigned long long wave_off = 0, total = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) {
    const unsigned long long t = s_wave[w];
    wave_off += (unsigned)w < wave ? t : 0ull;
    total += t;
  }
  const unsigned long long my_off = wave_off + incl - c;
  unsigned group_total = 0;
#pragma unroll
  for (int g = 0; g < TILES_PER_TICKET; ++g) group_total += (unsigned)(total >> (16 * g)) & 0xFFFFu;
  // publish, then look back with the first wave: each round reads the states
  // of the 64 nearest predecessors not yet summed
  if (wave == 0) {
    if (lane == 0)
      __hip_atomic_store(&state[group], (group == 0 ? FLAG_INCL : FLAG_AGG) | (unsigned long long)group_total,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long acc = 0;
    long long p = group - 1;
    while (p >= 0) {
      const long long q = p - (long long)lane;
      const unsigned long long st =
          q >= 0 ? __hip_atomic_load(&state[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : FLAG_INCL;
      const unsigned long long flag = st & ~VAL_MASK;
      const unsigned long long inclb = __ballot(flag == FLAG_INCL);
      const unsigned long long wait = __ballot(flag == 0);
      const int fi = inclb ? __ffsll((long long)inclb) - 1 : 64;
      const int fw = wait ? __ffsll((long long)wait) - 1 : 64;
      const int take = fw < fi ? fw : (fi < 64 ? fi + 1 : 64);
      unsigned long long v = (int)lane < take ? (st & VAL_MASK) : 0ull;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      acc += v;
      if (fi < fw) break;
      p -= take;
      if (fw < 64) __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) {
      if (group > 0)
        __hip_atomic_store(&state[group], FLAG_INCL | (acc + group_total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_excl = (long long)acc;
      if (group == ngroups - 1) *d_count = s_excl + group_total;
    }
  }
  // selected rows go through LDS so that the workgroup writes them with consecutive lanes
  unsigned before = 0;
#pragma unroll
  for (int g = 0; g < TILES_PER_TICKET; ++g) {
    const long long r0 = (t0 + g) * TILE + (long long)threadIdx.x * IPT;
    const unsigned tile_total = (unsigned)(total >> (16 * g)) & 0xFFFFu;
    unsigned o = (unsigned)(my_off >> (16 * g)) & 0xFFFFu;
    for (int k = 0; k < IPT; ++k)
      if (bits[g] & (1u << k)) s_rows[o++] = (int)(r0 + k);
    __syncthreads();
    const long long base = s_excl + before;
    for (unsigned j = threadIdx.x; j < tile_total; j += BLOCK) out[base + j] = s_rows[j];
    before += tile_total;
    __syncthreads();  // s_rows is reused by the next tile
  }
}
)SKEL";

// The interpreter's mask function: one row at a time, the term list walked per row.
const char* kInterpreter = R"INTERP(
__device__ __forceinline__ bool interp_term(const Term& t, const Cols& cols, long long r) {
  long long iv = 0;
  double fv = 0.0;
  const bool fp = t.dtype >= 4;
  switch (t.dtype) {
    case 0: iv = ((const signed char*)cols.c[t.column])[r]; break;
    case 1: iv = ((const short*)cols.c[t.column])[r]; break;
    case 2: iv = ((const int*)cols.c[t.column])[r]; break;
    case 3: iv = ((const long long*)cols.c[t.column])[r]; break;
    case 4: fv = (double)((const float*)cols.c[t.column])[r]; break;
    default: fv = ((const double*)cols.c[t.column])[r]; break;
  }
  switch (t.op) {
    case 0: return fp ? fv < t.fv[0] : iv < t.iv[0];
    case 1: return fp ? fv <= t.fv[0] : iv <= t.iv[0];
    case 2: return fp ? fv > t.fv[0] : iv > t.iv[0];
    case 3: return fp ? fv >= t.fv[0] : iv >= t.iv[0];
    case 4: return fp ? fv == t.fv[0] : iv == t.iv[0];
    case 5: return fp ? fv != t.fv[0] : iv != t.iv[0];
    case 6: return fp ? (fv >= t.fv[0] && fv <= t.fv[1]) : (iv >= t.iv[0] && iv <= t.iv[1]);
    default:
      for (int j = 0; j < t.n_values; ++j)
        if (fp ? fv == t.fv[j] : iv == t.iv[j]) return true;
      return false;
  }
}

__device__ __forceinline__ unsigned tile_bits(const Cols& cols, long long r0, long long n, const Term* terms, int nterms) {
  unsigned bits = 0;
  for (int k = 0; k < IPT; ++k) {
    const long long r = r0 + k;
    if (r >= n) break;
    bool ok = true;
    for (int t = 0; t < nterms && ok; ++t) ok = interp_term(terms[t], cols, r);
    bits |= (unsigned)ok << k;
  }
  return bits;
}
)INTERP";

const char* kTypeName[6] = {"signed char", "short", "int", "long long", "float", "double"};

std::string int_literal(int64_t v) {
  if (v == INT64_MIN) return "(-9223372036854775807LL - 1)";
  char b[32];
  std::snprintf(b, sizeof b, "%" PRId64 "LL", v);
  return b;
}

std::string fp_literal(double v) {
  if (std::isnan(v)) return "__builtin_nan(\"\")";
  if (std::isinf(v)) return v > 0 ? "__builtin_inf()" : "(-__builtin_inf())";
  char b[64];
  std::snprintf(b, sizeof b, "%a", v);  // hexadecimal: the exact double
  return b;
}

// The comparison of element expression `x` (already converted to long long or
// double) for one term.
std::string term_expr(const rel_pred_term& t, const std::string& x) {
  const bool fp = t.dtype >= REL_DT_F32;
  auto lit = [&](int j) { return fp ? fp_literal(t.fvalues[j]) : int_literal(t.ivalues[j]); };
  static const char* cmp[6] = {"<", "<=", ">", ">=", "==", "!="};
  if (t.op <= REL_OP_NE) return "(" + x + " " + cmp[t.op] + " " + lit(0) + ")";
  if (t.op == REL_OP_BETWEEN) return "(" + x + " >= " + lit(0) + " && " + x + " <= " + lit(1) + ")";
  std::string e = "(";
  for (int j = 0; j < t.n_values; ++j) e += (j ? " || " : "") + x + " == " + lit(j);
  return e + ")";
}

std::string compiled_mask(const rel_pred_term* terms, int32_t n_terms) {
  std::string s =
      "__device__ __forceinline__ unsigned tile_bits(const Cols& cols, long long r0, long long n, const Term*, int) {\n"
      "  unsigned bits = 0xffffffffu;\n"
      "  const bool full = r0 + IPT <= n;\n";
  for (int32_t i = 0; i < n_terms; ++i) {
    const rel_pred_term& t = terms[i];
    const std::string T = kTypeName[t.dtype];
    const std::string conv = t.dtype >= REL_DT_F32 ? "(double)" : "(long long)";
    s += "  {\n    const " + T + "* p = (const " + T + "*)cols.c[" + std::to_string(t.column) + "];\n";
    s += "    unsigned m = 0;\n";
    s += "    if (full) {\n#pragma unroll\n      for (int g = 0; g < IPT / 16; ++g) {\n        " + T + " v[16];\n";
    s += "        load16<" + T + ">(p + r0 + 16 * g, v);\n";
    s += "#pragma unroll\n        for (int k = 0; k < 16; ++k) m |= (unsigned)" + term_expr(t, conv + "v[k]") + " << (16 * g + k);\n      }\n";
    s += "    } else {\n      for (int k = 0; k < IPT; ++k)\n";
    s += "        if (r0 + k < n) m |= (unsigned)" + term_expr(t, conv + "p[r0 + k]") + " << k;\n    }\n";
    s += "    bits &= m;\n  }\n";
  }
  s += "  if (r0 + IPT > n) bits &= (1u << (unsigned)(n - r0)) - 1u;\n  return bits;\n}\n";
  return s;
}

}  // namespace

struct rel_pred {
  rel_ctx* ctx = nullptr;
  int mode = 0;
  int n_terms = 0;
  int max_column = -1;
  std::vector<int> col_dtype;  // dtype each used column must have (-1: unused)
  hipModule_t module = nullptr;
  hipFunction_t fn = nullptr;
  void* d_terms = nullptr;  // the term list, for the interpreter
  int tiles_per_ticket = 4;  // consecutive tiles per ticket (one look-back per group of them)
  int ipt = 16;              // rows per thread
};

namespace {

void free_pred(rel_pred* p) {
  if (!p) return;
  if (p->module) (void)hipModuleUnload(p->module);
  if (p->d_terms) (void)hipFree(p->d_terms);
  delete p;
}

rel_status compile(rel_ctx* ctx, const std::string& src, const char* kernel, hipModule_t* mod, hipFunction_t* fn) {
  hipDeviceProp_t prop;
  REL_HIP_CHECK(ctx, hipGetDeviceProperties(&prop, ctx->device));
  const std::string arch = std::string("--offload-arch=") + prop.gcnArchName;
  const char* opts[] = {arch.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "rel_pred.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return relh::fail(ctx, REL_HIP, "rel_pred_create: hiprtcCreateProgram failed");
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    return relh::fail(ctx, REL_HIP, "rel_pred_create: compilation failed: %.900s", log.c_str());
  }
  size_t size = 0;
  hiprtcGetCodeSize(prog, &size);
  std::vector<char> code(size);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  REL_HIP_CHECK(ctx, hipModuleLoadData(mod, code.data()));
  REL_HIP_CHECK(ctx, hipModuleGetFunction(fn, *mod, kernel));
  return REL_OK;
}

}  // namespace

extern "C" {

rel_status rel_pred_create(rel_ctx* ctx, const rel_pred_term* terms, int32_t n_terms, int32_t mode, rel_pred** out) {
  if (!ctx || !terms || !out || n_terms < 1 || n_terms > REL_PRED_MAX_TERMS ||
      (mode != REL_PRED_COMPILED && mode != REL_PRED_INTERPRETED))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_pred_create: bad argument");
  std::vector<int> col_dtype;
  for (int32_t i = 0; i < n_terms; ++i) {
    const rel_pred_term& t = terms[i];
    const bool ok_n = t.op <= REL_OP_NE ? t.n_values == 1 : t.op == REL_OP_BETWEEN ? t.n_values == 2
                                                                                 : t.n_values >= 1 && t.n_values <= REL_PRED_MAX_VALUES;
    if (t.column < 0 || t.column >= 8 || t.dtype < REL_DT_I8 || t.dtype > REL_DT_F64 || t.op < REL_OP_LT ||
        t.op > REL_OP_IN || !ok_n)
      return relh::fail(ctx, REL_INVALID_ARG, "rel_pred_create: term %d invalid", i);
    if ((int)col_dtype.size() <= t.column) col_dtype.resize(t.column + 1, -1);
    if (col_dtype[t.column] != -1 && col_dtype[t.column] != t.dtype)
      return relh::fail(ctx, REL_INVALID_ARG, "rel_pred_create: column %d given two types", t.column);
    col_dtype[t.column] = t.dtype;
  }
  rel_pred* p = new rel_pred();
  p->ctx = ctx;
  p->mode = mode;
  p->n_terms = n_terms;
  p->col_dtype = col_dtype;
  p->max_column = (int)col_dtype.size() - 1;
  // Tiles per ticket: a predicate that reads few bytes per row finishes its
  // tiles fast enough for the ticket's cache line to be the limit (atomics on
  // one line serialise at about 12 ns each), so it takes four tiles per ticket
  // (one look-back per group of four); one reading more keeps one tile per
  // ticket, where grouping cost it occupancy. Measured on 60M rows: day < 1200
  // alone (4 B per row) 0.129 ms with one tile, 0.104 ms with four; a 4-term
  // conjunction over 17 B per row 0.371 ms with one, 0.408 ms with four.
  int bytes_per_row = 0;
  for (size_t c = 0; c < col_dtype.size(); ++c)
    if (col_dtype[c] >= 0) bytes_per_row += dtype_bytes(col_dtype[c]);
  p->tiles_per_ticket = bytes_per_row <= 8 ? 4 : 1;
  p->ipt = rows_per_thread(mode, bytes_per_row);
  const std::string src = "#define IPT " + std::to_string(p->ipt) + "\n#define TILES_PER_TICKET " +
                          std::to_string(p->tiles_per_ticket) + "\n#define PRED_KERNEL " +
                          kernel_name(mode) + "\n" + kSkeleton +
                          (mode == REL_PRED_COMPILED ? compiled_mask(terms, n_terms) : std::string(kInterpreter));
  rel_status s = compile(ctx, src, kernel_name(mode), &p->module, &p->fn);
  if (s == REL_OK && mode == REL_PRED_INTERPRETED) {
    hipError_t e = hipMalloc(&p->d_terms, sizeof(rel_pred_term) * n_terms);
    if (e == hipSuccess) e = hipMemcpy(p->d_terms, terms, sizeof(rel_pred_term) * n_terms, hipMemcpyHostToDevice);
    if (e != hipSuccess) s = relh::hip_fail(ctx, e, "rel_pred_create: term list");
  }
  if (s != REL_OK) {
    free_pred(p);
    return s;
  }
  *out = p;
  return REL_OK;
}

rel_status rel_pred_filter(rel_pred* p, const void* const* columns, int32_t n_columns, int64_t n, int32_t* out_idx,
                           int64_t out_cap, int64_t* d_out_count) {
  if (!p) return REL_INVALID_ARG;
  rel_ctx* ctx = p->ctx;
  if (!columns || n < 0 || !d_out_count || (n > 0 && !out_idx) || n_columns <= p->max_column || n_columns > 8)
    return relh::fail(ctx, REL_INVALID_ARG, "rel_pred_filter: bad argument");
  if (n >= (1ll << 31)) return relh::fail(ctx, REL_UNSUPPORTED, "rel_pred_filter: n >= 2^31");
  if (out_cap < n) return relh::fail(ctx, REL_CAPACITY, "rel_pred_filter: out_cap < n");
  struct {
    const void* c[8];
  } cols{};
  for (int c = 0; c < n_columns; ++c) {
    const bool used = c < (int)p->col_dtype.size() && p->col_dtype[c] >= 0;
    if (used && n > 0 && (!columns[c] || !relh::aligned16(columns[c])))
      return relh::fail(ctx, REL_INVALID_ARG, "rel_pred_filter: column %d null or not 16-byte aligned", c);
    cols.c[c] = columns[c];
  }
  rel_status s = relh::ensure_counters(ctx);
  if (s != REL_OK) return s;
  if (n == 0) return relh::fill_u64(ctx, d_out_count, 1, 0);
  const int64_t tile_rows = 256 * (int64_t)p->ipt;
  const long long ntiles = (n + tile_rows - 1) / tile_rows;
  long long ngroups = (ntiles + p->tiles_per_ticket - 1) / p->tiles_per_ticket;
  void* st;
  if ((s = relh::scratch(ctx, SCR_SCAN_STATE, (size_t)ngroups * 8, &st)) != REL_OK) return s;
  int64_t* ticket = relh::counters(ctx) + CNT_TICKET;
  if ((s = relh::fill_u64(ctx, st, (size_t)ngroups, 0)) != REL_OK) return s;
  if ((s = relh::fill_u64(ctx, ticket, 1, 0)) != REL_OK) return s;
  long long nn = n;
  int* out = out_idx;
  unsigned long long* state = (unsigned long long*)st;
  long long* tk = (long long*)ticket;
  long long* dc = (long long*)d_out_count;
  const void* terms = p->d_terms;
  int nterms = p->n_terms;
  void* args[] = {&cols, &nn, &out, &state, &tk, &dc, &ngroups, &terms, &nterms};
  relh::KernelTimer kt(ctx, p->mode == REL_PRED_COMPILED ? "pred_compiled" : "pred_interpreted");
  REL_HIP_CHECK(ctx, hipModuleLaunchKernel(p->fn, (unsigned)ngroups, 1, 1, 256, 1, 1, 0, ctx->stream, args, nullptr));
  return REL_OK;
}

rel_status rel_pred_destroy(rel_pred* p) {
  if (!p) return REL_INVALID_ARG;
  (void)hipStreamSynchronize(p->ctx->stream);
  free_pred(p);
  return REL_OK;
}

}  // extern "C"
