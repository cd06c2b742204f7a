// Device-side building blocks shared by librel's kernels: hashing, wave64
// ballot/prefix helpers, the packed join-table slot and the group-table slot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rel {

constexpr int kWave = 64;
constexpr uint64_t kJoinEmpty = ~0ull;                // packed join slot: key in bits 0..31, payload in 32..63
constexpr int64_t kGroupEmpty = (int64_t)0x8000000000000000ull;  // group-table key sentinel (INT64_MIN)

constexpr uint32_t kDevOverflow = 0x1u;
constexpr uint32_t kDevDupKey = 0x2u;
constexpr uint32_t kDevBadArg = 0x4u;

// Multiplicative (Fibonacci) hash of a 32-bit key: the top `bits` bits of
// key * floor(2^32 / golden ratio). Only the high product bits are used, so
// the lower bits of the key reach every output bit.
__device__ __forceinline__ uint32_t hash32(int32_t key, uint32_t shift) {
  return ((uint32_t)key * 2654435769u) >> shift;
}

// 64-bit keys: fold the high word in, then the 32-bit hash.
__device__ __forceinline__ uint32_t hash64(int64_t key, uint32_t shift) {
  const uint64_t k = (uint64_t)key;
  const uint32_t x = (uint32_t)k ^ ((uint32_t)(k >> 32) * 0x85EBCA6Bu);
  return (x * 2654435769u) >> shift;
}

// Non-temporal loads, for the partitioning kernels' reads of data that one
// kernel reads exactly once (input columns, first-level runs). Measured on
// the 60M-row workload: the level-1 histogram 126 -> 102 us, the level-1
// scatter 378 -> 368 us. Not a general rule on this chip: the same loads in
// the filter (0.10 -> 0.16 ms), the compiled predicate, the fused streaming
// kernel and the groupjoin made each of them slower, so they keep ordinary
// loads. Stores stay ordinary everywhere: non-temporal stores are not merged
// in L2 with their neighbours, and the scatters, whose runs share cache lines
// at their ends, ran twice as long with them.
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef long long v2l_t __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ T ld_once(const T* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int4 ld_once(const int4* p) {
  const v4i_t v = __builtin_nontemporal_load(reinterpret_cast<const v4i_t*>(p));
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 ld_once(const uint4* p) {
  const v4i_t v = __builtin_nontemporal_load(reinterpret_cast<const v4i_t*>(p));
  return make_uint4((uint32_t)v.x, (uint32_t)v.y, (uint32_t)v.z, (uint32_t)v.w);
}
__device__ __forceinline__ longlong2 ld_once(const longlong2* p) {
  const v2l_t v = __builtin_nontemporal_load(reinterpret_cast<const v2l_t*>(p));
  return make_longlong2(v.x, v.y);
}

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2. This bijection on [0, G) hands XCD x (the workgroups b
// with b % 8 == x) one contiguous range of tiles, so the writes of adjacent
// tiles, which meet inside the same cache lines, are merged in one L2 instead
// of being written back as partial lines by two. Correctness never depends
// on the dispatch order; only locality does.
constexpr uint32_t kNumXcd = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t G) {
  const uint32_t x = b % kNumXcd, i = b / kNumXcd;
  const uint32_t q = G / kNumXcd, r = G % kNumXcd;
  return x * q + (x < r ? x : r) + i;
}

// Number of set bits of a wave mask below this lane.
__device__ __forceinline__ uint32_t mask_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ void set_status(uint32_t* status, uint32_t bits) {
  __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ void dev_add(T* p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ T dev_add_ret(T* p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ T dev_cas(T* p, T expected, T desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value found
}

// ---- workgroup scan and decoupled look-back ----------------------------------------------------------------------------

// Exclusive prefix sum of v over a workgroup of NT threads (NT a multiple of
// 64, at most 1024); *total receives the workgroup sum. Uses `scratch`
// (NT/64 words of LDS) and synchronises the workgroup twice.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* scratch, uint32_t* total) {
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, kWave);
    if (lane >= (uint32_t)o) incl += t;
  }
  __syncthreads();
  if (lane == kWave - 1) scratch[wave] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) {
    const uint32_t t = scratch[w];
    off += (uint32_t)w < wave ? t : 0u;
    tot += t;
  }
  *total = tot;
  return off + incl - v;
}

constexpr uint64_t kLbAgg = 1ull << 62;   // a tile's own count is published
constexpr uint64_t kLbIncl = 2ull << 62;  // a tile's inclusive prefix is published
constexpr uint64_t kLbVal = (1ull << 62) - 1;

// ---- join table -------------------------------------------------------------------------------------------------------

// Slots [0, capacity) hold packed {key, payload}; an in-table key is never
// 0xFFFFFFFF, so the all-ones word is free to mean "empty". The key -1 lives in
// the extra slot [capacity], stored as the zero-extended payload.
struct JoinView {
  const uint64_t* slots;  // capacity + 1 words
  uint32_t mask;          // capacity - 1
  uint32_t shift;         // 32 - log2(capacity)
};

// Linear-probing lookup. The table always keeps at least one empty slot, so the
// walk ends; the step bound only guards a corrupted table.
__device__ __forceinline__ bool join_lookup(const JoinView& t, int32_t key, int32_t* payload) {
  if (key == -1) {
    const uint64_t s = t.slots[(size_t)t.mask + 1];
    *payload = (int32_t)(uint32_t)s;
    return s != kJoinEmpty;
  }
  uint32_t h = hash32(key, t.shift);
  for (uint32_t step = 0; step <= t.mask; ++step) {
    const uint64_t s = t.slots[h];
    if (s == kJoinEmpty) return false;
    if ((uint32_t)s == (uint32_t)key) {
      *payload = (int32_t)(s >> 32);
      return true;
    }
    h = (h + 1) & t.mask;
  }
  return false;
}

// Split form of join_lookup for several independent probes per thread: the
// first slot of every probe is loaded together (join_first), then each probe
// is finished from its loaded slot (join_finish), walking on only when the
// first slot holds another key.
__device__ __forceinline__ size_t join_first_index(const JoinView& t, int32_t key) {
  return key == -1 ? (size_t)t.mask + 1 : (size_t)hash32(key, t.shift);
}

__device__ __forceinline__ bool join_finish(const JoinView& t, int32_t key, uint64_t s, int32_t* payload) {
  if (key == -1) {
    *payload = (int32_t)(uint32_t)s;
    return s != kJoinEmpty;
  }
  uint32_t h = hash32(key, t.shift);
  for (uint32_t step = 0; step <= t.mask; ++step) {
    if (s == kJoinEmpty) return false;
    if ((uint32_t)s == (uint32_t)key) {
      *payload = (int32_t)(s >> 32);
      return true;
    }
    h = (h + 1) & t.mask;
    s = t.slots[h];
  }
  return false;
}

// ---- join index: dense array or hash table --------------------------------------------------------------------------
//
// When the build keys span a range no wider than the index's dense capacity
// (surrogate keys numbered from some base, as dimension keys usually are),
// entry key - kmin of a plain array identifies the key's dim row, and a probe
// is one read at a computed address; otherwise the hash table above is used.
// The choice is made on the device, from the keys' minimum and maximum, so no
// host round trip is needed. An entry is 0 (no key) or, with an int8 payload,
// the 16-bit 0x100 | payload byte (half the bytes, so that more of the array
// stays in the L2 caches while fact rows probe it); otherwise the 32-bit dim
// row j + 1. Entries are written with plain stores, so a repeated key is
// detected by counting: m distinct keys fill exactly m entries, a repeated key
// fewer (dense_count_entries).
struct JoinIndex {
  JoinView hash;
  void* dense;         // dense_cap entries (16-byte aligned, padded to whole 16-byte words)
  const uint32_t* mm;  // {max of ~(key ^ 2^31), max of (key ^ 2^31)}: the keys' min and max, order-encoded
  int64_t dense_cap;
  const void* payload;  // the dim payload column (int32 or int8), or null for row ids
  int32_t pkind;        // relh::PayloadKind
  int32_t narrow;       // 16-bit entries (int8 payload)
  int64_t m;            // build rows
};

struct DenseRange {
  int32_t kmin;
  int64_t range;  // kmax - kmin + 1 (not positive when there are no keys)
  bool dense;
};

// From the two order-encoded words (see JoinIndex::mm).
__device__ __forceinline__ DenseRange dense_range_of(const JoinIndex& x, uint32_t w0, uint32_t w1) {
  DenseRange r;
  r.kmin = (int32_t)(~w0 ^ 0x80000000u);
  const int32_t kmax = (int32_t)(w1 ^ 0x80000000u);
  r.range = (int64_t)kmax - (int64_t)r.kmin + 1;
  r.dense = r.range <= x.dense_cap;
  return r;
}

__device__ __forceinline__ DenseRange dense_range(const JoinIndex& x) { return dense_range_of(x, x.mm[0], x.mm[1]); }

// 16-byte words that hold the range's entries (the last one padded with
// entries that the clearing kernel zeroes too).
__device__ __forceinline__ int64_t dense_words(const JoinIndex& x, const DenseRange& r) {
  if (r.range <= 0) return 0;
  return (r.range * (x.narrow ? 2 : 4) + 15) / 16;
}

// The dense entry of a key: 0 when the key is outside the range or absent.
__device__ __forceinline__ uint32_t dense_entry(const JoinIndex& x, const DenseRange& r, int32_t key) {
  const int64_t off = (int64_t)key - r.kmin;
  if (off < 0 || off >= r.range) return 0u;
  return x.narrow ? (uint32_t)((const uint16_t*)x.dense)[off] : ((const uint32_t*)x.dense)[off];
}

// The entry dim row j stores.
__device__ __forceinline__ uint32_t dense_encode(const JoinIndex& x, int64_t j) {
  if (x.narrow) return 0x100u | (uint32_t)(uint8_t)((const int8_t*)x.payload)[j];
  return (uint32_t)(j + 1);
}

__device__ __forceinline__ void dense_store(const JoinIndex& x, int64_t off, uint32_t e) {
  if (x.narrow) ((uint16_t*)x.dense)[off] = (uint16_t)e;
  else ((uint32_t*)x.dense)[off] = e;
}

// Payload of a non-zero dense entry (PayloadKind values: 0 row id, 1 int32, 2 int8).
__device__ __forceinline__ int32_t dense_payload(const JoinIndex& x, uint32_t e) {
  if (x.narrow) return (int32_t)(int8_t)(e & 0xFFu);
  const uint32_t j = e - 1u;
  if (x.pkind == 1) return ((const int32_t*)x.payload)[j];
  if (x.pkind == 2) return (int32_t)((const int8_t*)x.payload)[j];
  return (int32_t)j;
}

// Non-zero entries among the 16-byte words [w0, w1) of a dense index, counted
// by NT threads (the sum over all words is compared with m).
template <int NT>
__device__ __forceinline__ uint64_t dense_count_entries(const JoinIndex& x, int64_t w0, int64_t w1) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  const v4u* w = reinterpret_cast<const v4u*>(x.dense);
  uint64_t c = 0;
  for (int64_t i = w0 + threadIdx.x; i < w1; i += NT) {
    const v4u v = w[i];
    if (x.narrow) {
      c += ((v.x & 0xFFFFu) != 0) + ((v.x >> 16) != 0) + ((v.y & 0xFFFFu) != 0) + ((v.y >> 16) != 0) +
           ((v.z & 0xFFFFu) != 0) + ((v.z >> 16) != 0) + ((v.w & 0xFFFFu) != 0) + ((v.w >> 16) != 0);
    } else {
      c += (v.x != 0) + (v.y != 0) + (v.z != 0) + (v.w != 0);
    }
  }
  return c;
}

// Insert (key, payload) into a join table with one 64-bit CAS per attempted
// slot; a repeated key sets kDevDupKey, a full table kDevOverflow.
__device__ __forceinline__ void join_insert(uint64_t* slots, uint32_t mask, uint32_t shift, int32_t key, int32_t pl,
                                            uint32_t* status) {
  if (key == -1) {
    const uint64_t old = dev_cas<uint64_t>(&slots[(size_t)mask + 1], kJoinEmpty, (uint64_t)(uint32_t)pl);
    if (old != kJoinEmpty) set_status(status, kDevDupKey);
    return;
  }
  const uint64_t want = (uint64_t)(uint32_t)key | ((uint64_t)(uint32_t)pl << 32);
  uint32_t h = hash32(key, shift);
  for (uint32_t step = 0; step <= mask; ++step) {
    const uint64_t old = dev_cas<uint64_t>(&slots[h], kJoinEmpty, want);
    if (old == kJoinEmpty) return;
    if ((uint32_t)old == (uint32_t)key) {
      set_status(status, kDevDupKey);
      return;
    }
    h = (h + 1) & mask;
  }
  set_status(status, kDevOverflow);
}

// ---- group table ------------------------------------------------------------------------------------------------------

// One group: key and the three running aggregates. A slot is occupied exactly
// when count != 0 (whoever claims a key adds its count right away). The slot at
// index `capacity` is reserved for the key INT64_MIN, the empty sentinel.
struct alignas(32) GroupSlot {
  int64_t key;
  uint64_t sum_price;
  uint64_t sum_qty;
  uint64_t count;
};

struct GroupView {
  GroupSlot* slots;  // capacity + 1 slots
  uint32_t mask;
  uint32_t shift;
  uint32_t* status;
  uint32_t max_probe;  // longest probe walk before the table counts as overflowed
};

// Find or claim the slot of `key` in a device-memory table; -1 when full.
__device__ __forceinline__ int64_t group_slot(const GroupView& t, int64_t key) {
  if (key == kGroupEmpty) return (int64_t)t.mask + 1;
  uint32_t h = hash64(key, t.shift);
  for (uint32_t step = 0; step < t.max_probe; ++step) {
    const int64_t k = t.slots[h].key;  // hint; the CAS below decides
    if (k == key) return h;
    if (k == kGroupEmpty) {
      const int64_t old = dev_cas<int64_t>(&t.slots[h].key, kGroupEmpty, key);
      if (old == kGroupEmpty || old == key) return h;
    }
    h = (h + 1) & t.mask;
  }
  return -1;
}

__device__ __forceinline__ void group_add(const GroupView& t, int64_t key, uint64_t sp, uint64_t sq, uint64_t cnt) {
  const int64_t s = group_slot(t, key);
  if (s < 0) {
    set_status(t.status, kDevOverflow);
    return;
  }
  GroupSlot* g = &t.slots[s];
  dev_add<uint64_t>(&g->sum_price, sp);
  dev_add<uint64_t>(&g->sum_qty, sq);
  dev_add<uint64_t>(&g->count, cnt);
}

// Sum of a 64-bit value over the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, o, kWave);
  return v;
}

// Sum of a 64-bit value over a workgroup of NT threads, valid in thread 0.
// Every thread must call it; s is NT / 64 words of LDS that no thread touches
// until the workgroup's next barrier.
// Kernels add their totals to a device counter once per workgroup, never once
// per wave: thousands of atomics on one cache line at a kernel's end
// serialise on this chip (about 12 ns each) and hold up its completion.
template <int NT>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* s) {
  v = wave_sum_u64(v);
  if (lane_id() == 0) s[threadIdx.x / kWave] = v;
  __syncthreads();
  uint64_t t = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) t += s[w];
  }
  return t;
}

// Decoupled look-back (Merrill and Garland 2016) by one whole wave of tile
// `tile`, whose own count is `count`: publishes the count, sums predecessors
// and returns the exclusive prefix (the same value on every lane). Each round
// reads the states of the 64 nearest predecessors not yet summed, so a walk
// costs one round trip per 64 tiles rather than one per tile. Tiles must be
// numbered in the order their workgroups started (a ticket), so every awaited
// predecessor is running and publishes without waiting on this tile.
__device__ __forceinline__ uint64_t lookback_prefix(uint64_t* state, int64_t tile, uint64_t count) {
  const uint32_t lane = lane_id();
  if (lane == 0)
    __hip_atomic_store(&state[tile], (tile == 0 ? kLbIncl : kLbAgg) | count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint64_t acc = 0;
  int64_t p = tile - 1;  // nearest predecessor not yet summed
  while (p >= 0) {
    const int64_t q = p - (int64_t)lane;
    // before tile 0 reads as an inclusive prefix of 0
    const uint64_t st = q >= 0 ? __hip_atomic_load(&state[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kLbIncl;
    const uint64_t flag = st & ~kLbVal;
    const uint64_t incl = wave_ballot(flag == kLbIncl);
    const uint64_t wait = wave_ballot(flag == 0);
    const int fi = incl ? __ffsll((long long)incl) - 1 : kWave;  // nearest inclusive prefix
    const int fw = wait ? __ffsll((long long)wait) - 1 : kWave;  // nearest tile not yet published
    // sum up to the first unpublished tile, or through the first inclusive prefix
    const int take = fw < fi ? fw : (fi < kWave ? fi + 1 : kWave);
    acc += wave_sum_u64((int)lane < take ? (st & kLbVal) : 0ull);
    if (fi < fw) break;
    p -= take;
    if (fw < kWave) __builtin_amdgcn_s_sleep(1);
  }
  if (lane == 0 && tile > 0)
    __hip_atomic_store(&state[tile], kLbIncl | (acc + count), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return acc;
}

// Lanes sharing a key before a wave pre-sums them (below this the extra
// shuffles cost more than the atomics they save).
constexpr int kWaveCombineMin = 4;

// group_add for one row per active lane, called by every lane of the wave.
// Lanes whose key equals the first active lane's key are summed across the
// wave first, so a hot key (a skewed join) costs one set of device atomics per
// wave instead of one per row.
__device__ __forceinline__ void group_add_wave(const GroupView& t, bool active, int64_t key, uint64_t sp, uint64_t sq) {
  const uint64_t act = wave_ballot(active);
  if (act == 0) return;
  const int first = __ffsll((long long)act) - 1;
  const int64_t k0 = __shfl(key, first, kWave);
  const bool mine = active && key == k0;
  const uint64_t same = wave_ballot(mine);
  if (__popcll(same) >= kWaveCombineMin) {
    const uint64_t s1 = wave_sum_u64(mine ? sp : 0);
    const uint64_t s2 = wave_sum_u64(mine ? sq : 0);
    if ((int)lane_id() == first) group_add(t, k0, s1, s2, (uint64_t)__popcll(same));
    active = active && !mine;
  }
  if (active) group_add(t, key, sp, sq, 1ull);
}

// group_add_wave for partial aggregates: each active lane adds (sp, sq, cnt).
__device__ __forceinline__ void group_add_wave_n(const GroupView& t, bool active, int64_t key, uint64_t sp, uint64_t sq,
                                                 uint64_t cnt) {
  const uint64_t act = wave_ballot(active);
  if (act == 0) return;
  const int first = __ffsll((long long)act) - 1;
  const int64_t k0 = __shfl(key, first, kWave);
  const bool mine = active && key == k0;
  const uint64_t same = wave_ballot(mine);
  if (__popcll(same) >= kWaveCombineMin) {
    const uint64_t s1 = wave_sum_u64(mine ? sp : 0);
    const uint64_t s2 = wave_sum_u64(mine ? sq : 0);
    const uint64_t s3 = wave_sum_u64(mine ? cnt : 0);
    if ((int)lane_id() == first) group_add(t, k0, s1, s2, s3);
    active = active && !mine;
  }
  if (active) group_add(t, key, sp, sq, cnt);
}

// Per-dim-row aggregates of the groupjoin (group key == join key).
struct alignas(8) RowAgg {
  uint64_t sum_price;
  uint64_t sum_qty;
  uint64_t count;
};

// ---- LDS group table ------------------------------------------------------------------------------------------------

template <int SLOTS>
struct LdsGroups {
  int64_t key[SLOTS];
  uint64_t sum_price[SLOTS];
  uint64_t sum_qty[SLOTS];
  uint64_t count[SLOTS];

  __device__ void init(int tid, int nthreads) {
    for (int s = tid; s < SLOTS; s += nthreads) {
      key[s] = kGroupEmpty;
      sum_price[s] = 0;
      sum_qty[s] = 0;
      count[s] = 0;
    }
  }

  // Slot of key, or -1 when the probe budget is spent (caller goes to device memory).
  __device__ __forceinline__ int find(int64_t k, int max_probe) {
    uint32_t h = hash64(k, 32 - __builtin_ctz(SLOTS)) & (SLOTS - 1);
    for (int step = 0; step < max_probe; ++step) {
      const int64_t cur = key[h];
      if (cur == k) return (int)h;
      if (cur == kGroupEmpty) {
        const int64_t old = atomicCAS((unsigned long long*)&key[h], (unsigned long long)kGroupEmpty,
                                      (unsigned long long)k);
        if ((int64_t)old == kGroupEmpty || (int64_t)old == k) return (int)h;
      }
      h = (h + 1) & (SLOTS - 1);
    }
    return -1;
  }

  __device__ __forceinline__ void add(int s, uint64_t sp, uint64_t sq, uint64_t cnt) {
    atomicAdd((unsigned long long*)&sum_price[s], (unsigned long long)sp);
    atomicAdd((unsigned long long*)&sum_qty[s], (unsigned long long)sq);
    atomicAdd((unsigned long long*)&count[s], (unsigned long long)cnt);
  }

  // Push every occupied LDS slot into the device-memory table.
  __device__ void flush(const GroupView& g, int tid, int nthreads) {
    for (int s = tid; s < SLOTS; s += nthreads)
      if (count[s] != 0) group_add(g, key[s], sum_price[s], sum_qty[s], count[s]);
  }
};

}  // namespace rel
