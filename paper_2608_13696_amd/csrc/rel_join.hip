// Hash join: build (insert_if_n analogue) and probe (count + retrieve
// analogue, fused into one pass because a PK-FK probe emits at most one pair
// per probe row, so no counting pass is needed to size the output).
#include "rel_device.h"
#include "rel_host.h"
#include "rel_ops.h"

namespace {

using namespace rel;
using relh::PAY_I32;
using relh::PAY_I8;
using relh::PAY_ROW_ID;

// Insert (pk[j], payload) with one 64-bit CAS per attempted slot. Consecutive
// threads take consecutive rows, so the key and payload reads are coalesced
// and each thread keeps its CAS independent of the others.
template <int PK>
__global__ __launch_bounds__(256) void k_join_build(const int32_t* __restrict__ pk, const void* __restrict__ payload,
                                                    int64_t m, uint64_t* __restrict__ slots, uint32_t mask,
                                                    uint32_t shift, uint32_t* __restrict__ status) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; j < m; j += stride) {
    const int32_t key = pk[j];
    const int32_t pl = PK == PAY_ROW_ID ? (int32_t)j
                       : PK == PAY_I32  ? ((const int32_t*)payload)[j]
                                        : (int32_t)((const int8_t*)payload)[j];
    join_insert(slots, mask, shift, key, pl, status);
  }
}

// ---- join index (dense array or hash table) ----------------------------------------------------------------------------

// Minimum and maximum of the build keys, order-encoded so that both are
// maxima over unsigned words that start at 0 (see JoinIndex::mm). Few, large
// workgroups with two 16-byte loads in flight per thread; each writes its pair
// to part[2b], part[2b + 1], and the clearing kernel that follows combines
// them (no atomics, and no word to zero first).
constexpr int kIdxBlock = 256;
constexpr int kMinMaxBlock = 512;
constexpr int kMinMaxGrid = relh::kKeyMinMaxParts;
__device__ __forceinline__ void minmax_add(int32_t k, uint32_t& lo, uint32_t& hi) {
  const uint32_t o = (uint32_t)k ^ 0x80000000u;
  lo = max(lo, ~o);
  hi = max(hi, o);
}

__global__ __launch_bounds__(kMinMaxBlock) void k_key_minmax(const int32_t* __restrict__ pk, int64_t m, uint32_t* part) {
  __shared__ uint32_t s_lo[kMinMaxBlock / kWave], s_hi[kMinMaxBlock / kWave];
  uint32_t lo = 0, hi = 0;  // max of ~(key ^ 2^31), max of (key ^ 2^31)
  const int64_t nq = m / 4;  // whole 16-byte quads (pk is 16-byte aligned)
  const int4* q = reinterpret_cast<const int4*>(pk);
  constexpr int kQ = 4;  // quads in flight per thread
  const int64_t stride = (int64_t)gridDim.x * kMinMaxBlock * kQ;
  for (int64_t i = blockIdx.x * (int64_t)kMinMaxBlock * kQ + threadIdx.x; i < nq; i += stride) {
    int4 v[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      const int64_t j = i + (int64_t)k * kMinMaxBlock;
      v[k] = q[j < nq ? j : i];
    }
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      minmax_add(v[k].x, lo, hi); minmax_add(v[k].y, lo, hi); minmax_add(v[k].z, lo, hi); minmax_add(v[k].w, lo, hi);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < (m & 3)) minmax_add(pk[nq * 4 + threadIdx.x], lo, hi);
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    lo = max(lo, (uint32_t)__shfl_xor((int)lo, d, kWave));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, kWave));
  }
  if (lane_id() == 0) {
    s_lo[threadIdx.x / kWave] = lo;
    s_hi[threadIdx.x / kWave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kMinMaxBlock / kWave; ++w) {
      lo = max(lo, s_lo[w]);
      hi = max(hi, s_hi[w]);
    }
    part[2 * blockIdx.x] = lo;
    part[2 * blockIdx.x + 1] = hi;
  }
}

// Combines the min/max pairs of k_key_minmax (every workgroup for itself;
// workgroup 0 also stores the result in x.mm for the kernels that follow),
// then clears whichever structure the keys' range selects: the 16-byte words
// that hold the dense entries in use, or the whole hash table; and zeroes the
// caller's spans of 64-bit words.
__global__ __launch_bounds__(kIdxBlock) void k_index_clear(JoinIndex x, int64_t hash_words, const uint32_t* __restrict__ part,
                                                           int32_t nparts, relh::ZeroSpans z) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  __shared__ uint32_t s_mm[2];
  if (threadIdx.x < kWave) {
    uint32_t lo = 0, hi = 0;
    for (int i = threadIdx.x; i < nparts; i += kWave) {
      lo = max(lo, part[2 * i]);
      hi = max(hi, part[2 * i + 1]);
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      lo = max(lo, (uint32_t)__shfl_xor((int)lo, d, kWave));
      hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, kWave));
    }
    if (threadIdx.x == 0) {
      s_mm[0] = lo;
      s_mm[1] = hi;
      if (blockIdx.x == 0) {
        uint32_t* mm = const_cast<uint32_t*>(x.mm);
        mm[0] = lo;
        mm[1] = hi;
      }
    }
  }
  __syncthreads();
  const DenseRange r = dense_range_of(x, s_mm[0], s_mm[1]);
  const int64_t stride = (int64_t)gridDim.x * kIdxBlock;
  const int64_t tid = blockIdx.x * (int64_t)kIdxBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < 2; ++k)
    for (int64_t i = tid; i < z.n[k]; i += stride) z.p[k][i] = 0;
  int64_t i = tid;
  if (r.dense) {
    const int64_t words = dense_words(x, r);
    for (; i < words; i += stride) reinterpret_cast<v4u*>(x.dense)[i] = v4u{0u, 0u, 0u, 0u};
  } else {
    uint64_t* slots = const_cast<uint64_t*>(x.hash.slots);
    for (; i < hash_words; i += stride) slots[i] = kJoinEmpty;
  }
}

// Dense: plain stores (a repeated key is found by counting the entries, which
// the probing kernel does). A thread loads kBuildQuads 16-byte quads of keys
// (and their payloads) before it stores any entry, so its random stores do
// not wait on one load at a time. (Cutting the key range into one slice per
// XCD, so that each L2 takes the stores of its own slice only, measured
// slower on 1.5M keys: 26 us against 17, each XCD then reading every key.)
// Hash: one 64-bit CAS per attempted slot.
constexpr int kBuildQuads = 4;

template <int PK>
__global__ __launch_bounds__(kIdxBlock) void k_index_build(const int32_t* __restrict__ pk, int64_t m, JoinIndex x,
                                                           uint32_t* __restrict__ status) {
  const DenseRange r = dense_range(x);
  if (r.dense) {
    const int64_t nq = (m + 3) / 4;
    const int4* q = reinterpret_cast<const int4*>(pk);
    const int64_t step = (int64_t)gridDim.x * kIdxBlock;
    for (int64_t i0 = blockIdx.x * (int64_t)kIdxBlock + threadIdx.x; i0 < nq; i0 += step * kBuildQuads) {
      int32_t key[kBuildQuads * 4];
#pragma unroll
      for (int u = 0; u < kBuildQuads; ++u) {
        const int64_t i = i0 + u * step;
        if (4 * i + 4 <= m) {
          const int4 v = q[i];
          key[4 * u] = v.x; key[4 * u + 1] = v.y; key[4 * u + 2] = v.z; key[4 * u + 3] = v.w;
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) key[4 * u + c] = 4 * i + c < m ? pk[4 * i + c] : 0;
        }
      }
      uint32_t e[kBuildQuads * 4];
#pragma unroll
      for (int u = 0; u < kBuildQuads; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t j = 4 * (i0 + u * step) + c;
          e[4 * u + c] = j < m ? dense_encode(x, j) : 0u;
        }
#pragma unroll
      for (int u = 0; u < kBuildQuads; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t j = 4 * (i0 + u * step) + c;
          if (j < m) dense_store(x, (int64_t)key[4 * u + c] - r.kmin, e[4 * u + c]);
        }
    }
    return;
  }
  const int64_t stride = (int64_t)gridDim.x * kIdxBlock;
  for (int64_t j = blockIdx.x * (int64_t)kIdxBlock + threadIdx.x; j < m; j += stride) {
    const int32_t key = pk[j];
    const int32_t pl = PK == PAY_ROW_ID ? (int32_t)j
                       : PK == PAY_I32  ? ((const int32_t*)x.payload)[j]
                                        : (int32_t)((const int8_t*)x.payload)[j];
    join_insert(const_cast<uint64_t*>(x.hash.slots), x.hash.mask, x.hash.shift, key, pl, status);
  }
}

// The dense index's duplicate check on its own, for calls whose probing
// kernel does not run (no probe rows): one workgroup counts the entries. A
// no-op for a hash table.
constexpr int kVerifyBlock = 1024;
__global__ __launch_bounds__(kVerifyBlock) void k_index_verify(JoinIndex x, uint32_t* __restrict__ status) {
  __shared__ uint64_t s_red[kVerifyBlock / kWave];
  const DenseRange r = dense_range(x);
  if (!r.dense) return;
  const uint64_t c = block_sum_u64<kVerifyBlock>(dense_count_entries<kVerifyBlock>(x, 0, dense_words(x, r)), s_red);
  if (threadIdx.x == 0 && c != (uint64_t)x.m) set_status(status, kDevDupKey);
}

// Probe: a wave takes 8 x 64 consecutive probe rows per step, one row of each
// 64 per lane. Every lane issues the first-slot loads of its eight rows
// together (the random table reads are the cost, so eight are in flight per
// lane instead of one), then finishes each probe. A wave runs kProbeGroup
// steps, keeping each row's match in registers, and then reserves output
// space for all of them with one atomic: the count is one word, and atomics
// on one cache line serialise on this chip at about 12 ns each, so one per
// step (512 rows) bounded the kernel. Matches are compacted with one ballot
// per row group. Output order is therefore unspecified.
// On 28.15M probes into a 15M-key table: 0.78 ms with eight rows per lane and
// one atomic per step, 1.40 ms with four, 5.31 ms with one; sixteen spill the
// ballot masks.
constexpr int kProbeRows = 8;
constexpr int kProbeGroup = 4;

__global__ __launch_bounds__(256) void k_join_probe(JoinView t, const int32_t* __restrict__ fk,
                                                    const int32_t* __restrict__ sel, int64_t n,
                                                    int32_t* __restrict__ out_fact, int32_t* __restrict__ out_payload,
                                                    int64_t* __restrict__ d_count) {
  constexpr int64_t kStep = (int64_t)kWave * kProbeRows;
  const int64_t wave_global = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const uint32_t lane = lane_id();
  for (int64_t base0 = wave_global * kStep * kProbeGroup; base0 < n; base0 += n_waves * kStep * kProbeGroup) {
    int32_t hrow[kProbeGroup][kProbeRows];  // the matching fact row, or -1
    int32_t hpl[kProbeGroup][kProbeRows];
    uint32_t total = 0;
#pragma unroll
    for (int g = 0; g < kProbeGroup; ++g) {
      const int64_t base = base0 + g * kStep;
      int32_t row[kProbeRows], key[kProbeRows];
      uint64_t first[kProbeRows];
#pragma unroll
      for (int k = 0; k < kProbeRows; ++k) {
        const int64_t i = base + k * kWave + lane;
        row[k] = i < n ? (sel ? sel[i] : (int32_t)i) : -1;
      }
#pragma unroll
      for (int k = 0; k < kProbeRows; ++k) key[k] = row[k] >= 0 ? fk[row[k]] : 0;
#pragma unroll
      for (int k = 0; k < kProbeRows; ++k) first[k] = row[k] >= 0 ? t.slots[join_first_index(t, key[k])] : kJoinEmpty;
#pragma unroll
      for (int k = 0; k < kProbeRows; ++k) {
        hpl[g][k] = 0;
        const bool hit = row[k] >= 0 && join_finish(t, key[k], first[k], &hpl[g][k]);
        hrow[g][k] = hit ? row[k] : -1;
        total += (uint32_t)__popcll(wave_ballot(hit));
      }
    }
    if (total == 0) continue;
    int64_t off = 0;
    if (lane == 0) off = dev_add_ret<unsigned long long>((unsigned long long*)d_count, (unsigned long long)total);
    off = __shfl(off, 0, kWave);
#pragma unroll
    for (int g = 0; g < kProbeGroup; ++g) {
#pragma unroll
      for (int k = 0; k < kProbeRows; ++k) {
        const uint64_t b = wave_ballot(hrow[g][k] >= 0);
        if (hrow[g][k] >= 0) {
          const int64_t o = off + mask_rank(b);
          out_fact[o] = hrow[g][k];
          out_payload[o] = hpl[g][k];
        }
        off += __popcll(b);
      }
    }
  }
}

}  // namespace

namespace relh {

rel_status join_build_into(rel_ctx* ctx, const int32_t* pk, const void* payload, int payload_kind, int64_t m,
                           uint64_t* slots, uint32_t log2cap) {
  const uint64_t cap = 1ull << log2cap;
  rel_status s;
  {
    KernelTimer kt(ctx, "join_table_init");
    s = fill_u64(ctx, slots, cap + 1, rel::kJoinEmpty);
  }
  if (s != REL_OK) return s;
  if (m == 0) return REL_OK;
  const unsigned grid = grid_for(ctx, m, 256 * 4, 8);
  const uint32_t mask = (uint32_t)(cap - 1), shift = 32u - log2cap;
  KernelTimer kt(ctx, "join_build");
  if (payload_kind == PAY_I32)
    hipLaunchKernelGGL(k_join_build<PAY_I32>, dim3(grid), dim3(256), 0, ctx->stream, pk, payload, m, slots, mask, shift,
                       ctx->d_status);
  else if (payload_kind == PAY_I8)
    hipLaunchKernelGGL(k_join_build<PAY_I8>, dim3(grid), dim3(256), 0, ctx->stream, pk, payload, m, slots, mask, shift,
                       ctx->d_status);
  else
    hipLaunchKernelGGL(k_join_build<PAY_ROW_ID>, dim3(grid), dim3(256), 0, ctx->stream, pk, payload, m, slots, mask,
                       shift, ctx->d_status);
  REL_LAUNCH_CHECK(ctx, "join_build");
  return REL_OK;
}

rel_status join_index_build(rel_ctx* ctx, const int32_t* pk, const void* payload, int payload_kind, int64_t m,
                            uint32_t* mm, const ZeroSpans& zero, rel::JoinIndex* out) {
  const uint32_t jl = join_log2cap(m, nullptr);
  void *jt, *dt;
  rel_status s;
  if ((s = scratch(ctx, SCR_JOIN_TABLE, ((size_t)8 << jl) + 8, &jt)) != REL_OK) return s;
  const int64_t dcap = 2 * (m > 8 ? m : 8);
  if ((s = scratch(ctx, SCR_DENSE, (size_t)dcap * 4 + 16, &dt)) != REL_OK) return s;
  void* part;
  if ((s = scratch(ctx, SCR_MINMAX, (size_t)kMinMaxGrid * 8, &part)) != REL_OK) return s;
  rel::JoinIndex x{};
  x.hash = rel::JoinView{(const uint64_t*)jt, (uint32_t)((1ull << jl) - 1), 32u - jl};
  x.dense = dt;
  x.mm = mm;
  x.dense_cap = dcap;
  x.payload = payload;
  x.pkind = payload_kind;
  x.narrow = payload_kind == PAY_I8;
  x.m = m;
  int64_t gm = (m + kMinMaxBlock * 16 - 1) / (kMinMaxBlock * 16);
  if (gm > kMinMaxGrid) gm = kMinMaxGrid;
  {
    KernelTimer kt(ctx, "key_minmax");
    if (m > 0)
      hipLaunchKernelGGL(k_key_minmax, dim3((unsigned)gm), dim3(kMinMaxBlock), 0, ctx->stream, pk, m, (uint32_t*)part);
  }
  {
    KernelTimer kt(ctx, "join_table_init");
    const int64_t words = (int64_t)(1ull << jl) + 1;
    const int64_t most = dcap > words ? dcap : words;
    hipLaunchKernelGGL(k_index_clear, dim3(grid_for(ctx, most, kIdxBlock * 8, 4)), dim3(kIdxBlock), 0, ctx->stream, x, words,
                       (const uint32_t*)part, (int32_t)gm, zero);
  }
  REL_LAUNCH_CHECK(ctx, "join index clear");
  if (m > 0) {
    const unsigned grid = grid_for(ctx, m, kIdxBlock * 4, 8);
    {
      KernelTimer kt(ctx, "join_build");
      if (payload_kind == PAY_I32)
        hipLaunchKernelGGL(k_index_build<PAY_I32>, dim3(grid), dim3(kIdxBlock), 0, ctx->stream, pk, m, x, ctx->d_status);
      else if (payload_kind == PAY_I8)
        hipLaunchKernelGGL(k_index_build<PAY_I8>, dim3(grid), dim3(kIdxBlock), 0, ctx->stream, pk, m, x, ctx->d_status);
      else
        hipLaunchKernelGGL(k_index_build<PAY_ROW_ID>, dim3(grid), dim3(kIdxBlock), 0, ctx->stream, pk, m, x, ctx->d_status);
    }
    REL_LAUNCH_CHECK(ctx, "join index build");
  }
  *out = x;
  return REL_OK;
}

int32_t key_minmax_partials(rel_ctx* ctx, const int32_t* pk, int64_t m, uint32_t* part) {
  int64_t gm = (m + kMinMaxBlock * 16 - 1) / (kMinMaxBlock * 16);
  if (gm > kMinMaxGrid) gm = kMinMaxGrid;
  if (m > 0) {
    KernelTimer kt(ctx, "key_minmax");
    hipLaunchKernelGGL(k_key_minmax, dim3((unsigned)gm), dim3(kMinMaxBlock), 0, ctx->stream, pk, m, part);
  }
  return (int32_t)gm;
}

rel_status join_index_verify(rel_ctx* ctx, const rel::JoinIndex& x) {
  if (x.m == 0) return REL_OK;
  KernelTimer kt(ctx, "join_index_verify");
  hipLaunchKernelGGL(k_index_verify, dim3(1), dim3(kVerifyBlock), 0, ctx->stream, x, ctx->d_status);
  REL_LAUNCH_CHECK(ctx, "join index verify");
  return REL_OK;
}

uint32_t join_log2cap(int64_t m, const rel_table_opts* opts) {
  double load = (opts && opts->max_load > 0.f) ? (double)opts->max_load : 0.5;
  if (load > 0.9) load = 0.9;
  int64_t want = (int64_t)((double)(m > 0 ? m : 1) / load) + 1;
  if (opts && opts->capacity_hint > want) want = opts->capacity_hint;
  uint32_t l = log2_ceil((uint64_t)want);
  if (l < 4) l = 4;
  return l;
}

}  // namespace relh

extern "C" {

rel_status rel_join_build(rel_ctx* ctx, const int32_t* pk, const int32_t* payload, int64_t m,
                          const rel_table_opts* opts, rel_join_table** out) {
  if (!ctx || !out || m < 0 || (m > 0 && !pk)) return relh::fail(ctx, REL_INVALID_ARG, "rel_join_build: bad argument");
  if (m >= (1ll << 30)) return relh::fail(ctx, REL_UNSUPPORTED, "rel_join_build: m >= 2^30");
  if (opts && opts->placement != REL_PLACE_AUTO && opts->placement != REL_PLACE_GLOBAL)
    return relh::fail(ctx, REL_UNSUPPORTED, "rel_join_build: standalone tables live in device memory");
  const uint32_t l = relh::join_log2cap(m, opts);
  if (l > 31) return relh::fail(ctx, REL_UNSUPPORTED, "rel_join_build: capacity above 2^31");
  rel_join_table* t = new rel_join_table();
  t->ctx = ctx;
  t->log2cap = l;
  t->m = m;
  hipError_t e = hipMalloc(&t->slots, (sizeof(uint64_t) << l) + sizeof(uint64_t));
  if (e != hipSuccess) {
    delete t;
    (void)hipGetLastError();
    return relh::fail(ctx, REL_OOM, "rel_join_build: table allocation failed");
  }
  rel_status s = relh::join_build_into(ctx, pk, payload, payload ? relh::PAY_I32 : relh::PAY_ROW_ID, m, t->slots, l);
  if (s != REL_OK) {
    (void)hipFree(t->slots);
    delete t;
    return s;
  }
  *out = t;
  return REL_OK;
}

rel_status rel_join_table_destroy(rel_join_table* t) {
  if (!t) return REL_INVALID_ARG;
  if (t->ctx) (void)hipStreamSynchronize(t->ctx->stream);
  if (t->slots) (void)hipFree(t->slots);
  delete t;
  return REL_OK;
}

rel_status rel_join_probe(rel_ctx* ctx, const rel_join_table* t, const int32_t* fk, const int32_t* sel, int64_t n,
                          int32_t* out_fact_idx, int32_t* out_payload, int64_t out_cap, int64_t* d_out_count) {
  if (!ctx || !t || n < 0 || !d_out_count || (n > 0 && (!fk || !out_fact_idx || !out_payload)))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_join_probe: bad argument");
  if (t->ctx != ctx) return relh::fail(ctx, REL_INVALID_ARG, "rel_join_probe: table belongs to another context");
  if (n >= (1ll << 31)) return relh::fail(ctx, REL_UNSUPPORTED, "rel_join_probe: n >= 2^31");
  if (out_cap < n) return relh::fail(ctx, REL_CAPACITY, "rel_join_probe: out_cap %lld < n %lld", (long long)out_cap, (long long)n);
  rel_status s = relh::fill_u64(ctx, d_out_count, 1, 0);
  if (s != REL_OK || n == 0) return s;
  rel::JoinView v{t->slots, (uint32_t)((1ull << t->log2cap) - 1), 32u - t->log2cap};
  const unsigned grid = relh::grid_for(ctx, n, 256 * kProbeRows, 8);
  relh::KernelTimer kt(ctx, "join_probe");
  hipLaunchKernelGGL(k_join_probe, dim3(grid), dim3(256), 0, ctx->stream, v, fk, sel, n, out_fact_idx, out_payload,
                     d_out_count);
  REL_LAUNCH_CHECK(ctx, "join_probe");
  return REL_OK;
}

}  // extern "C"
