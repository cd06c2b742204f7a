// Host-side internals of librel: the context, its scratch arena, error
// plumbing and launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rel.h"

struct ScratchBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  size_t clean = 0;  // leading bytes known to hold an empty group table (SCR_GROUP_CLEAN)
};

// Scratch slots a context keeps between calls (each grows on demand, never shrinks).
enum ScratchId : int {
  SCR_JOIN_TABLE = 0,  // fused pipeline's join table
  SCR_GROUP_TABLE,     // fused pipeline's group table / per-dim-row aggregates
  SCR_COUNTERS,        // small device counters
  SCR_SCAN_STATE,      // decoupled look-back tile states
  SCR_PART_A,          // partitioned pipeline buffers
  SCR_PART_B,
  SCR_PART_C,
  SCR_PART_D,
  SCR_PART_E,
  SCR_SKETCH,
  SCR_MLP,
  SCR_DENSE,           // dense join index entries
  SCR_WG_COUNTS,       // per-workgroup counts of a streaming kernel
  SCR_GROUP_CLEAN,     // plain path's group table, left empty by its finalize
  SCR_STAGE,           // per-workgroup staged groups for the merge kernel
  SCR_MINMAX,          // per-workgroup key minimum and maximum of the join index build
  SCR_COUNT
};

// Device counter words inside SCR_COUNTERS (int64 each).
enum CounterId : int {
  CNT_ROWS_PASSED = 0,
  CNT_JOIN_MATCHES,
  CNT_TICKET,
  CNT_GROUPS,
  CNT_AUX0,
  CNT_AUX1,
  CNT_AUX2,
  CNT_AUX3,
  CNT_WORDS = 16
};

// Per-kernel timing with HIP events recorded on the context's stream around
// each launch (enabled on request; used by the benchmark to time the dominant
// kernel inside the timed region).
struct KernelTiming {
  std::string name;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double total_ms = 0.0;
  int64_t launches = 0;
};

struct rel_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 256;
  size_t lds_per_block = 65536;
  // Device status words (64 x u32, one allocation). Word 0 is the sticky word
  // rel_ctx_sync reads; word 1 belongs to a synchronising fused call, which
  // clears it first and reads it at its end, so that bits left by earlier
  // calls are neither charged to it nor dropped. d_status is the word that
  // kernels launched now report to.
  uint32_t* d_status_words = nullptr;
  uint32_t* d_status = nullptr;
  std::string err;
  ScratchBuf scratch[SCR_COUNT];
  bool timing = false;
  std::vector<KernelTiming> timings;
  std::vector<hipEvent_t> event_pool;
  // A second stream of the library's own (default priority) for work that can
  // run beside the caller's stream, with the fork / join events; made on first use.
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

struct rel_join_table {
  rel_ctx* ctx = nullptr;
  uint64_t* slots = nullptr;
  uint32_t log2cap = 0;
  int64_t m = 0;
};

namespace relh {

rel_status fail(rel_ctx* ctx, rel_status s, const char* fmt, ...);
rel_status hip_fail(rel_ctx* ctx, hipError_t e, const char* what);
// Device buffer of at least `bytes` in scratch slot `id` (contents undefined).
rel_status scratch(rel_ctx* ctx, int id, size_t bytes, void** out);
int64_t* counters(rel_ctx* ctx);  // valid after ensure_counters
rel_status ensure_counters(rel_ctx* ctx);

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

inline uint32_t log2_ceil(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

// Grid for a grid-stride kernel over `items` work items with `per_block` items per block.
inline unsigned grid_for(const rel_ctx* ctx, int64_t items, int64_t per_block, int blocks_per_cu = 8) {
  int64_t g = (items + per_block - 1) / per_block;
  const int64_t cap = (int64_t)ctx->num_cus * blocks_per_cu;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Fill helpers (plain kernels, so that the calls stay legal inside a captured graph).
rel_status fill_u64(rel_ctx* ctx, void* p, size_t n_u64, uint64_t v);
// Address of this device's fixed scratch array for the allocation-free entry
// point (rel_filter.hip); the device must be current.
rel_status noalloc_scratch_init(rel_ctx* ctx, int device);
rel_status fill_u32(rel_ctx* ctx, void* p, size_t n_u32, uint32_t v);

// Records a start event on construction and a stop event on destruction when
// the context's timing is enabled; otherwise does nothing.
// aux_fork orders the auxiliary stream after the work already on ctx->stream
// (creating it on first use); aux_join makes ctx->stream wait for everything
// enqueued on the auxiliary stream since.
rel_status aux_fork(rel_ctx* ctx);
rel_status aux_join(rel_ctx* ctx);

class KernelTimer {
 public:
  KernelTimer(rel_ctx* ctx, const char* name);
  ~KernelTimer();

 private:
  rel_ctx* ctx_;
  int slot_ = -1;
  hipEvent_t start_ = nullptr;
};

}  // namespace relh

#define REL_HIP_CHECK(ctx, expr)                                 \
  do {                                                           \
    hipError_t e_ = (expr);                                      \
    if (e_ != hipSuccess) return relh::hip_fail((ctx), e_, #expr); \
  } while (0)

#define REL_LAUNCH_CHECK(ctx, what)                                 \
  do {                                                              \
    hipError_t e_ = hipGetLastError();                              \
    if (e_ != hipSuccess) return relh::hip_fail((ctx), e_, (what)); \
  } while (0)
