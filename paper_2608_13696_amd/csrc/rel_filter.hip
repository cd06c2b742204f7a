// Stable stream compaction (the filter + prefix-sum pair of Table 9) in one
// pass: single-pass prefix scan with decoupled look-back (Merrill and
// Garland, 2016).
//
// Groups of four consecutive tiles are handed out by an atomic ticket, not by
// blockIdx, so every group a workgroup waits on belongs to a workgroup that is
// already running and that publishes its own count before it looks back: the
// wait always ends. The first wave does the look-back, reading 64 predecessor
// states per round.
//
// A thread tests 32 consecutive rows (eight 16-byte loads); the tile's
// selected row numbers are staged in LDS in output order and written out by
// consecutive lanes, so the stores are contiguous rather than one 4-byte
// store per selected row scattered across a thread's output run.
#include <mutex>

#include "rel_device.h"
#include "rel_host.h"

namespace {

using namespace rel;

constexpr int kBlock = 256;
constexpr int kIPT = 32;  // rows per thread: eight 16-byte loads
constexpr int64_t kTile = (int64_t)kBlock * kIPT;
// Consecutive tiles a workgroup takes with one ticket. Every ticket is an
// atomic on one cache line, and atomics on one line serialise on this chip
// at about 12 ns each; four tiles per ticket keep that line out of the way.
constexpr int64_t kTilesPerTicket = 4;

template <int OP>
__device__ __forceinline__ bool pred(int32_t v, int32_t lit) {
  if (OP == REL_LT) return v < lit;
  if (OP == REL_LE) return v <= lit;
  if (OP == REL_GT) return v > lit;
  if (OP == REL_GE) return v >= lit;
  if (OP == REL_EQ) return v == lit;
  return v != lit;
}

// Row bits of one thread for one tile: bit k = row r0 + k passes.
template <int OP>
__device__ __forceinline__ uint32_t tile_bits(const int32_t* __restrict__ col, int64_t n, int32_t lit, int64_t r0) {
  uint32_t bits = 0;
  if (r0 + kIPT <= n) {
#pragma unroll
    for (int v = 0; v < kIPT / 4; ++v) {
      const int4 x = *reinterpret_cast<const int4*>(col + r0 + 4 * v);
      bits |= (uint32_t)pred<OP>(x.x, lit) << (4 * v);
      bits |= (uint32_t)pred<OP>(x.y, lit) << (4 * v + 1);
      bits |= (uint32_t)pred<OP>(x.z, lit) << (4 * v + 2);
      bits |= (uint32_t)pred<OP>(x.w, lit) << (4 * v + 3);
    }
  } else {
    for (int k = 0; k < kIPT; ++k)
      if (r0 + k < n) bits |= (uint32_t)pred<OP>(col[r0 + k], lit) << k;
  }
  return bits;
}

// One workgroup per ticket, and a ticket is kTilesPerTicket consecutive
// tiles (a group): the group's rows are all tested first, its count is
// published and looked back once (the look-back state is per group, so no
// group waits on the end of another group's writes), then its tiles are
// staged and written one after another. Per-thread counts of the group's
// tiles travel packed in one 64-bit word, 16 bits per tile (a tile holds at
// most 8192 rows), so one scan serves them all.
template <int OP>
__global__ __launch_bounds__(kBlock) void k_filter_compact(const int32_t* __restrict__ col, int64_t n, int32_t lit,
                                                           int32_t* __restrict__ out, uint64_t* __restrict__ state,
                                                           int64_t* __restrict__ ticket, int64_t* __restrict__ d_count,
                                                           int64_t ngroups) {
  static_assert(kTile < (1 << 16) && kTilesPerTicket * 16 <= 64, "packed per-tile counts");
  __shared__ int64_t s_group;
  __shared__ int64_t s_excl;
  __shared__ uint64_t s_wave[kBlock / kWave];
  __shared__ int32_t s_rows[kTile];
  if (threadIdx.x == 0) s_group = (int64_t)dev_add_ret<unsigned long long>((unsigned long long*)ticket, 1ull);
  __syncthreads();
  const int64_t group = s_group;
  const int64_t t0 = group * kTilesPerTicket;
  uint32_t bits[kTilesPerTicket];
  uint64_t c = 0;
#pragma unroll
  for (int g = 0; g < kTilesPerTicket; ++g) {
    const int64_t r0 = (t0 + g) * kTile + (int64_t)threadIdx.x * kIPT;
    bits[g] = r0 < n ? tile_bits<OP>(col, n, lit, r0) : 0u;
    c |= (uint64_t)__popc(bits[g]) << (16 * g);
  }

  // Exclusive scan of the packed counts over the workgroup: wave scan, then wave totals.
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  uint64_t incl = c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t t = (uint64_t)__shfl_up((unsigned long long)incl, o, kWave);
    if (lane >= (uint32_t)o) incl += t;
  }
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint64_t wave_off = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    const uint64_t t = s_wave[w];
    wave_off += (uint32_t)w < wave ? t : 0ull;
    total += t;
  }
  const uint64_t my_off = wave_off + incl - c;
  uint32_t group_total = 0;
#pragma unroll
  for (int g = 0; g < kTilesPerTicket; ++g) group_total += (uint32_t)(total >> (16 * g)) & 0xFFFFu;

  // Publish, then look back (the first wave).
  if (wave == 0) {
    const uint64_t excl = lookback_prefix(state, group, group_total);
    if (threadIdx.x == 0) {
      s_excl = (int64_t)excl;
      if (group == ngroups - 1) *d_count = s_excl + group_total;
    }
  }
  uint32_t before = 0;  // rows of the group's earlier tiles
#pragma unroll
  for (int g = 0; g < kTilesPerTicket; ++g) {
    const int64_t r0 = (t0 + g) * kTile + (int64_t)threadIdx.x * kIPT;
    const uint32_t tile_total = (uint32_t)(total >> (16 * g)) & 0xFFFFu;
    uint32_t o = (uint32_t)(my_off >> (16 * g)) & 0xFFFFu;
    for (int k = 0; k < kIPT; ++k)
      if (bits[g] & (1u << k)) s_rows[o++] = (int32_t)(r0 + k);
    __syncthreads();
    int32_t* dst = out + s_excl + before;
    for (uint32_t j = threadIdx.x; j < tile_total; j += kBlock) dst[j] = s_rows[j];
    before += tile_total;
    __syncthreads();  // s_rows is reused by the next tile
  }
}

template <int OP>
void launch(hipStream_t stream, const int32_t* col, int64_t n, int32_t lit, int32_t* out, uint64_t* state,
            int64_t* ticket, int64_t* d_count, int64_t ntiles) {
  const int64_t ngroups = (ntiles + kTilesPerTicket - 1) / kTilesPerTicket;
  hipLaunchKernelGGL(k_filter_compact<OP>, dim3((unsigned)ngroups), dim3(kBlock), 0, stream, col, n, lit, out, state,
                     ticket, d_count, ngroups);
}

void launch_op(hipStream_t stream, rel_cmp op, const int32_t* col, int64_t n, int32_t lit, int32_t* out,
               uint64_t* state, int64_t* ticket, int64_t* d_count, int64_t ntiles) {
  switch (op) {
    case REL_LT: launch<REL_LT>(stream, col, n, lit, out, state, ticket, d_count, ntiles); break;
    case REL_LE: launch<REL_LE>(stream, col, n, lit, out, state, ticket, d_count, ntiles); break;
    case REL_GT: launch<REL_GT>(stream, col, n, lit, out, state, ticket, d_count, ntiles); break;
    case REL_GE: launch<REL_GE>(stream, col, n, lit, out, state, ticket, d_count, ntiles); break;
    case REL_EQ: launch<REL_EQ>(stream, col, n, lit, out, state, ticket, d_count, ntiles); break;
    case REL_NE: launch<REL_NE>(stream, col, n, lit, out, state, ticket, d_count, ntiles); break;
  }
}

// ---- the allocation-free variant ---------------------------------------------------------------------------------------
//
// Its look-back tile states and its ticket live in a fixed device array: word
// 0 is the ticket, words 1.. the states of up to kNoAllocTiles tiles (1 MiB),
// so it compacts at most kNoAllocTiles * kTile = 2^30 rows. Every device that
// runs the library holds its own copy until the process ends. In host code
// the array's name is not a device address; the address is looked up once
// per device (noalloc_scratch_init, from rel_ctx_create) and kept here.
constexpr int64_t kNoAllocTiles = 1 << 17;
constexpr int64_t kNoAllocMaxRows = kNoAllocTiles * kTile;
static __device__ __align__(256) uint64_t scratch[1 + kNoAllocTiles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace relh {

// Looks up this device's copy of the fixed scratch array (the device must be
// current). Called by rel_ctx_create; later calls for the same device return
// at once.
rel_status noalloc_scratch_init(rel_ctx* ctx, int device) {
  if (device < 0 || device >= kMaxDevices) return fail(ctx, REL_UNSUPPORTED, "device index %d above %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return REL_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch));
  if (e != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    return fail(ctx, REL_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  }
  g_scratch_ptr[device] = p;
  return REL_OK;
}

}  // namespace relh

extern "C" rel_status rel_filter_compact(rel_ctx* ctx, const int32_t* col, int64_t n, rel_cmp op, int32_t literal,
                                         int32_t* out_idx, int64_t out_cap, int64_t* d_out_count) {
  if (!ctx || n < 0 || !d_out_count || (n > 0 && (!col || !out_idx)) || op < REL_LT || op > REL_NE)
    return relh::fail(ctx, REL_INVALID_ARG, "rel_filter_compact: bad argument");
  if (col && !relh::aligned16(col)) return relh::fail(ctx, REL_INVALID_ARG, "rel_filter_compact: column not 16-byte aligned");
  if (n >= (1ll << 31)) return relh::fail(ctx, REL_UNSUPPORTED, "rel_filter_compact: n >= 2^31");
  if (out_cap < n) return relh::fail(ctx, REL_CAPACITY, "rel_filter_compact: out_cap < n");
  rel_status s = relh::ensure_counters(ctx);
  if (s != REL_OK) return s;
  if (n == 0) return relh::fill_u64(ctx, d_out_count, 1, 0);
  const int64_t ntiles = (n + kTile - 1) / kTile;
  void* st;
  s = relh::scratch(ctx, SCR_SCAN_STATE, (size_t)ntiles * 8, &st);
  if (s != REL_OK) return s;
  int64_t* ticket = relh::counters(ctx) + CNT_TICKET;
  if ((s = relh::fill_u64(ctx, st, (size_t)ntiles, 0)) != REL_OK) return s;
  if ((s = relh::fill_u64(ctx, ticket, 1, 0)) != REL_OK) return s;
  uint64_t* state = (uint64_t*)st;
  relh::KernelTimer kt(ctx, "filter_compact");
  launch_op(ctx->stream, op, col, n, literal, out_idx, state, ticket, d_out_count, ntiles);
  REL_LAUNCH_CHECK(ctx, "filter_compact");
  return REL_OK;
}

// rel_filter_compact with its scratch in the fixed array: no allocation, only
// two fill kernels and the compaction kernel on the context's stream.
extern "C" rel_status rel_filter_compact_noalloc(rel_ctx* ctx, const int32_t* col, int64_t n, rel_cmp op,
                                                 int32_t literal, int32_t* out_idx, int64_t out_cap,
                                                 int64_t* d_out_count) {
  if (!ctx || n < 0 || !d_out_count || (n > 0 && (!col || !out_idx)) || op < REL_LT || op > REL_NE)
    return relh::fail(ctx, REL_INVALID_ARG, "rel_filter_compact_noalloc: bad argument");
  if (n > kNoAllocMaxRows)
    return relh::fail(ctx, REL_UNSUPPORTED, "rel_filter_compact_noalloc: n = %lld above the maximum of %lld rows",
                      (long long)n, (long long)kNoAllocMaxRows);
  if (col && !relh::aligned16(col))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_filter_compact_noalloc: column not 16-byte aligned");
  if (out_cap < n) return relh::fail(ctx, REL_CAPACITY, "rel_filter_compact_noalloc: out_cap < n");
  void* base = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch_ptr[ctx->device] : nullptr;
  if (!base) return relh::fail(ctx, REL_HIP, "rel_filter_compact_noalloc: scratch address of device %d unknown", ctx->device);
  if (n == 0) return relh::fill_u64(ctx, d_out_count, 1, 0);
  const int64_t ntiles = (n + kTile - 1) / kTile;
  uint64_t* words = (uint64_t*)base;
  // the ticket and this call's tile states start at zero (the array keeps the last call's contents)
  rel_status s = relh::fill_u64(ctx, words, (size_t)(1 + ntiles), 0);
  if (s != REL_OK) return s;
  launch_op(ctx->stream, op, col, n, literal, out_idx, words + 1, (int64_t*)words, d_out_count, ntiles);
  REL_LAUNCH_CHECK(ctx, "filter_compact_noalloc");
  return REL_OK;
}
