// The fused filter -> probe -> aggregate pipeline (build, one streaming
// kernel, finalize) and the standalone hash group-by.
//
// The streaming kernel reads the fact columns once with 16-byte vector loads,
// several rows per thread (the paper's Recommendation 1: overlap latency with
// instruction-level parallelism), evaluates the compiled predicate, probes the
// join table and updates the group state:
//   * few groups: a per-workgroup LDS table (the shared-memory aggregation of
//     Section 7); a workgroup that ends with few groups stages them with plain
//     stores and one workgroup merges the stages, else it flushes its table
//     to device memory;
//   * many groups: a device-memory table updated with device-scope atomics;
//   * group key == join key (GROUP BY fk): a groupjoin, aggregating straight
//     into per-dim-row accumulators so no second hash table exists.
#include "rel_device.h"
#include "rel_host.h"
#include "rel_ops.h"

namespace {

using namespace rel;

enum Mode : int { M_PRIO_FLAG = REL_GROUP_PRIO_FLAG, M_FK = REL_GROUP_FK, M_DIM_GRP = REL_GROUP_DIM_GRP };
enum GPlace : int { G_LDS = 0, G_GLOBAL = 1, G_ROWAGG = 2 };

constexpr int kBlock = 256;
constexpr int kLdsBlock = 1024;  // fused kernel with an LDS group table: one workgroup per CU
constexpr int kIPT = 4;  // rows per thread per tile: one 16-byte load per int32 column
constexpr int kLdsSlots = 1024;
constexpr int kLdsProbe = 32;
constexpr int kLdsCacheProbe = 4;
// A table sized from a prediction gives up after this many probe steps (at a
// load of 0.5 linear probing practically never walks that far), so that an
// undersized table reports overflow instead of degrading to a linear scan.
constexpr uint32_t kPlannedProbe = 256;
// Groups a workgroup of the LDS variant may stage for the merge kernel (more
// and it adds them to the device table itself).
constexpr int kStageMax = 32;

struct FusedArgs {
  const int32_t* fk;
  const int64_t* price;
  const int32_t* qty;
  const int32_t* day;
  const int8_t* flag;
  int64_t n;
  int32_t day_lt;
  JoinIndex join;
  GroupView groups;
  RowAgg* row_agg;
  uint64_t* wg_counts;  // per workgroup: rows passed, join matches, dense index entries
  // LDS variant: kStageMax group slots per workgroup (unused ones zero), and
  // a word set when any row or group went to the device table instead
  GroupSlot* stage;
  uint32_t* touched;
  int32_t lds_probe;  // LDS probe budget before a row goes to device memory
};

template <int MODE>
__device__ __forceinline__ int64_t group_key(int32_t payload, int32_t fk, int8_t flag) {
  if (MODE == M_PRIO_FLAG) return (int64_t)payload * 256 + (int64_t)(uint8_t)flag;
  if (MODE == M_DIM_GRP) return (int64_t)payload;
  return (int64_t)fk;
}

// One thread's rows of a tile: kIPT consecutive rows, loaded with 16-byte loads.
struct FusedRows {
  int32_t d[kIPT], f[kIPT], q[kIPT];
  int64_t p[kIPT];
  uint32_t fl;  // the four flag bytes
  int nv;       // rows in range
};

template <int MODE>
__device__ __forceinline__ void load_fused(const FusedArgs& a, int64_t r0, FusedRows& r) {
  if (r0 + kIPT <= a.n) {
    r.nv = kIPT;
    const int4 dv = *reinterpret_cast<const int4*>(a.day + r0);
    const int4 fv = *reinterpret_cast<const int4*>(a.fk + r0);
    const int4 qv = *reinterpret_cast<const int4*>(a.qty + r0);
    const longlong2 p01 = *reinterpret_cast<const longlong2*>(a.price + r0);
    const longlong2 p23 = *reinterpret_cast<const longlong2*>(a.price + r0 + 2);
    r.d[0] = dv.x; r.d[1] = dv.y; r.d[2] = dv.z; r.d[3] = dv.w;
    r.f[0] = fv.x; r.f[1] = fv.y; r.f[2] = fv.z; r.f[3] = fv.w;
    r.q[0] = qv.x; r.q[1] = qv.y; r.q[2] = qv.z; r.q[3] = qv.w;
    r.p[0] = p01.x; r.p[1] = p01.y; r.p[2] = p23.x; r.p[3] = p23.y;
    r.fl = MODE == M_PRIO_FLAG ? *reinterpret_cast<const uint32_t*>(a.flag + r0) : 0u;
  } else {
    r.nv = r0 < a.n ? (int)(a.n - r0) : 0;
    r.fl = 0;
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
      const bool ok = k < r.nv;
      r.d[k] = ok ? a.day[r0 + k] : 0;
      r.f[k] = ok ? a.fk[r0 + k] : 0;
      r.q[k] = ok ? a.qty[r0 + k] : 0;
      r.p[k] = ok ? a.price[r0 + k] : 0;
      if (MODE == M_PRIO_FLAG && ok) r.fl |= (uint32_t)(uint8_t)a.flag[r0 + k] << (8 * k);
    }
  }
}

// End of the LDS variant, one LDS slot per thread: a table holding at most
// kStageMax groups is compacted into the workgroup's stage (the rest of the
// stage zeroed); a fuller one goes to the device table with atomics. Few
// groups shared by every workgroup would otherwise mean hundreds of
// workgroups adding into the same few device slots at the kernel's end, and
// atomics on one cache line serialise (about 12 ns each on this chip).
template <int NT>
__device__ void stage_or_flush(LdsGroups<kLdsSlots>& lds, const FusedArgs& a, uint64_t dev_rows) {
  static_assert(NT == kLdsSlots, "one LDS slot per thread");
  __shared__ uint32_t s_wcnt[NT / kWave];
  __shared__ uint64_t s_red[NT / kWave];
  const int t = threadIdx.x;
  const bool occ = lds.count[t] != 0;
  const uint64_t ball = wave_ballot(occ);
  const uint32_t wave = t / kWave;
  if (lane_id() == 0) s_wcnt[wave] = (uint32_t)__popcll(ball);
  dev_rows = block_sum_u64<NT>(dev_rows, s_red);  // (its barrier also publishes s_wcnt)
  uint32_t total = 0, before = 0;
#pragma unroll
  for (uint32_t w = 0; w < NT / kWave; ++w) {
    const uint32_t c = s_wcnt[w];
    before += w < wave ? c : 0u;
    total += c;
  }
  GroupSlot* st = a.stage + (int64_t)blockIdx.x * kStageMax;
  if (total <= (uint32_t)kStageMax) {
    if (occ) st[before + mask_rank(ball)] = GroupSlot{lds.key[t], lds.sum_price[t], lds.sum_qty[t], lds.count[t]};
    if (t >= (int)total && t < kStageMax) st[t] = GroupSlot{kGroupEmpty, 0, 0, 0};
  } else {
    if (occ) group_add(a.groups, lds.key[t], lds.sum_price[t], lds.sum_qty[t], lds.count[t]);
    if (t < kStageMax) st[t] = GroupSlot{kGroupEmpty, 0, 0, 0};
  }
  if (t == 0 && (dev_rows != 0 || total > (uint32_t)kStageMax)) *a.touched = 1u;
}

// Persistent: each workgroup walks tiles with a grid stride and loads its next
// tile while it probes and aggregates the current one. With an LDS group
// table there is one large workgroup per CU, so the table is flushed to device
// memory once per CU (few groups means few, heavily shared device slots).
template <int MODE, int GP, int NT>
__global__ __launch_bounds__(NT) void k_fused(FusedArgs a) {
  __shared__ LdsGroups<GP == G_LDS ? kLdsSlots : 1> lds;
  if (GP == G_LDS) {
    lds.init(threadIdx.x, NT);
    __syncthreads();
  }
  uint64_t passed = 0, matched = 0, dev_rows = 0;
  const DenseRange dr = dense_range(a.join);
  constexpr int64_t tile_rows = (int64_t)NT * kIPT;
  const int64_t ntiles = (a.n + tile_rows - 1) / tile_rows;
  int64_t tile = blockIdx.x;
  FusedRows cur, nxt;
  if (tile < ntiles) load_fused<MODE>(a, tile * tile_rows + (int64_t)threadIdx.x * kIPT, cur);
  // this workgroup's share of the dense index's duplicate check (a count of
  // its entries), while its first tile loads
  uint64_t entries = 0;
  if (dr.dense) {
    const int64_t words = dense_words(a.join, dr);
    const int64_t per = (words + gridDim.x - 1) / gridDim.x;
    const int64_t w0 = (int64_t)blockIdx.x * per;
    entries = dense_count_entries<NT>(a.join, w0, min(words, w0 + per));
  }
  for (; tile < ntiles; tile += gridDim.x) {
    const int64_t tn = tile + gridDim.x;
    if (tn < ntiles) load_fused<MODE>(a, tn * tile_rows + (int64_t)threadIdx.x * kIPT, nxt);
    // every row's first join read (its dense entry, or its first hash slot)
    // is issued before any is examined, so the tile's random reads overlap
    // instead of following one another
    bool pass[kIPT];
    uint64_t first[kIPT];
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
      pass[k] = k < cur.nv && cur.d[k] < a.day_lt;
      if (dr.dense) first[k] = pass[k] ? dense_entry(a.join, dr, cur.f[k]) : 0u;
      else first[k] = pass[k] ? a.join.hash.slots[join_first_index(a.join.hash, cur.f[k])] : kJoinEmpty;
    }
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
      // no early exits: the device-memory update below is a wave-wide call
      passed += pass[k];
      int32_t pl = 0;
      bool hit;
      if (dr.dense) {
        hit = first[k] != 0;
        if (hit) pl = dense_payload(a.join, (uint32_t)first[k]);
      } else {
        hit = pass[k] && join_finish(a.join.hash, cur.f[k], first[k], &pl);
      }
      matched += hit;
      const uint64_t sp = (uint64_t)cur.p[k], sq = (uint64_t)(int64_t)cur.q[k];
      if (GP == G_ROWAGG) {
        if (hit) {
          RowAgg* r = &a.row_agg[pl];
          dev_add<uint64_t>(&r->sum_price, sp);
          dev_add<uint64_t>(&r->sum_qty, sq);
          dev_add<uint64_t>(&r->count, 1ull);
        }
      } else {
        const int64_t key = hit ? group_key<MODE>(pl, cur.f[k], (int8_t)(cur.fl >> (8 * k))) : 0;
        bool global = hit;
        if (GP == G_LDS && hit) {
          const int s = lds.find(key, a.lds_probe);
          if (s >= 0) {
            lds.add(s, sp, sq, 1ull);
            global = false;
          }
        }
        if (GP == G_LDS) dev_rows += global;
        group_add_wave(a.groups, global, key, sp, sq);
      }
    }
    cur = nxt;
  }
  if constexpr (GP == G_LDS) {
    __syncthreads();
    stage_or_flush<NT>(lds, a, dev_rows);
  }
  // the totals go out with plain stores, one triple per workgroup; the merge
  // or finalize kernel adds them up
  __shared__ uint64_t s_red[3][NT / kWave];
  passed = block_sum_u64<NT>(passed, s_red[0]);
  matched = block_sum_u64<NT>(matched, s_red[1]);
  entries = block_sum_u64<NT>(entries, s_red[2]);
  if (threadIdx.x == 0) {
    a.wg_counts[3 * blockIdx.x] = passed;
    a.wg_counts[3 * blockIdx.x + 1] = matched;
    a.wg_counts[3 * blockIdx.x + 2] = entries;
  }
}

// One workgroup merges the stages of the LDS variant in its own LDS table.
// When nothing went to the device table and every merged group found an LDS
// slot, it writes the output itself (groups, their number, the two counters)
// and sets `done`, and the finalize kernel returns at once; otherwise it adds
// its groups to the device table and the finalize kernel scans that.
constexpr int kMergeUnroll = 8;

struct MergeArgs {
  const GroupSlot* stage;  // n_wg * kStageMax
  const uint32_t* touched;
  int64_t n_wg;
  const uint64_t* wg_counts;
  int64_t* counters;
  GroupView groups;
  uint32_t* done;
  JoinIndex join;  // for the dense index's entry count
};

// The per-workgroup counts summed by NT threads (valid in thread 0): rows
// passed and join matches into counters[0] and [1]; a dense index with fewer
// entries than build rows had a repeated key.
template <int NT>
__device__ void sum_wg_counts(const uint64_t* wg, int64_t n_wg, const JoinIndex& jx, int64_t* counters,
                              uint32_t* status) {
  __shared__ uint64_t s_red[3][NT / kWave];
  uint64_t p = 0, q = 0, e = 0;
  for (int64_t i = threadIdx.x; i < n_wg; i += NT) {
    p += wg[3 * i];
    q += wg[3 * i + 1];
    e += wg[3 * i + 2];
  }
  p = block_sum_u64<NT>(p, s_red[0]);
  q = block_sum_u64<NT>(q, s_red[1]);
  e = block_sum_u64<NT>(e, s_red[2]);
  if (threadIdx.x == 0) {
    counters[0] = (int64_t)p;
    counters[1] = (int64_t)q;
    if (jx.mm != nullptr && dense_range(jx).dense && e != (uint64_t)jx.m) set_status(status, kDevDupKey);
  }
}

struct OutArgs;
__global__ __launch_bounds__(kLdsBlock) void k_group_merge(MergeArgs m, OutArgs o);

// Standalone group-by over key[row], row = sel ? sel[k] : k.
template <int GP>
__global__ __launch_bounds__(kBlock) void k_groupby(const int64_t* __restrict__ key, const int64_t* __restrict__ price,
                                                    const int32_t* __restrict__ qty, const int32_t* __restrict__ sel,
                                                    int64_t n, GroupView g) {
  __shared__ LdsGroups<GP == G_LDS ? kLdsSlots : 1> lds;
  if (GP == G_LDS) {
    lds.init(threadIdx.x, kBlock);
    __syncthreads();
  }
  int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (; k < n; k += stride) {
    const int64_t row = sel ? (int64_t)sel[k] : k;
    const int64_t kv = key[row];
    const uint64_t sp = (uint64_t)price[row], sq = (uint64_t)(int64_t)qty[row];
    int s = -1;
    if (GP == G_LDS && kv != kGroupEmpty) s = lds.find(kv, kLdsProbe);
    if (s >= 0) lds.add(s, sp, sq, 1ull);
    else group_add(g, kv, sp, sq, 1ull);
  }
  if (GP == G_LDS) {
    __syncthreads();
    lds.flush(g, threadIdx.x, kBlock);
  }
}

__global__ void k_init_groups(GroupSlot* __restrict__ slots, int64_t nslots) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < nslots; i += stride) {
    GroupSlot s;
    s.key = kGroupEmpty;
    s.sum_price = 0;
    s.sum_qty = 0;
    s.count = 0;
    slots[i] = s;
  }
}

struct OutArgs {
  int64_t* key;
  int64_t* sum_price;
  int64_t* sum_qty;
  int64_t* count;
  int64_t cap;
  int64_t* d_n;
  uint32_t* status;
  // the streaming kernel's per-workgroup (rows passed, join matches), summed
  // into counters[0] and [1] by the first group of tiles; n_wg = 0: none
  const uint64_t* wg_counts;
  int64_t n_wg;
  int64_t* counters;
  const uint32_t* done;  // set: the merge kernel wrote the output (may be null)
  JoinIndex join;        // for the dense index's entry count (mm null: none)
};

__global__ __launch_bounds__(kLdsBlock) void k_group_merge(MergeArgs m, OutArgs o) {
  __shared__ LdsGroups<kLdsSlots> lds;
  __shared__ uint32_t s_lost;  // a group went to the device table here
  __shared__ uint32_t s_wcnt[kLdsBlock / kWave];
  const int t = threadIdx.x;
  lds.init(t, kLdsBlock);
  if (t == 0) s_lost = 0;
  __syncthreads();
  const int64_t nflat = m.n_wg * kStageMax;
  for (int64_t f0 = 0; f0 < nflat; f0 += (int64_t)kLdsBlock * kMergeUnroll) {
    GroupSlot e[kMergeUnroll];
#pragma unroll
    for (int u = 0; u < kMergeUnroll; ++u) {
      const int64_t f = f0 + (int64_t)u * kLdsBlock + t;
      if (f < nflat) e[u] = m.stage[f];
      else e[u].count = 0;
    }
#pragma unroll
    for (int u = 0; u < kMergeUnroll; ++u) {
      if (e[u].count == 0) continue;
      const int s = lds.find(e[u].key, kLdsProbe);
      if (s >= 0) {
        lds.add(s, e[u].sum_price, e[u].sum_qty, e[u].count);
      } else {
        group_add(m.groups, e[u].key, e[u].sum_price, e[u].sum_qty, e[u].count);
        s_lost = 1;
      }
    }
  }
  // the streaming kernel's per-workgroup counts (the barriers inside also end
  // the merge)
  sum_wg_counts<kLdsBlock>(m.wg_counts, m.n_wg, m.join, m.counters, o.status);
  const bool occ = lds.count[t] != 0;
  if (*m.touched != 0 || s_lost != 0) {
    if (occ) group_add(m.groups, lds.key[t], lds.sum_price[t], lds.sum_qty[t], lds.count[t]);
    return;
  }
  const uint64_t ball = wave_ballot(occ);
  const uint32_t wave = t / kWave;
  if (lane_id() == 0) s_wcnt[wave] = (uint32_t)__popcll(ball);
  __syncthreads();
  uint32_t total = 0, before = 0;
#pragma unroll
  for (uint32_t w = 0; w < kLdsBlock / kWave; ++w) {
    const uint32_t c = s_wcnt[w];
    before += w < wave ? c : 0u;
    total += c;
  }
  if (occ) {
    const int64_t pos = before + mask_rank(ball);
    if (pos < o.cap) {
      o.key[pos] = lds.key[t];
      o.sum_price[pos] = (int64_t)lds.sum_price[t];
      o.sum_qty[pos] = (int64_t)lds.sum_qty[t];
      o.count[pos] = (int64_t)lds.count[t];
    } else {
      set_status(o.status, kDevOverflow);
    }
  }
  if (t == 0) {
    *o.d_n = (int64_t)total;
    *m.done = 1u;
  }
}

// Group finalization: stream compaction of the occupied slots into the
// output. Each workgroup takes a group of kFinTilesPerTicket consecutive
// tiles by ticket, counts the group's occupied slots (per tile, packed 16
// bits a tile in one word for a single scan),
// and finds its output offset by decoupled look-back, so no single output
// counter is contended. A thread's slots are kBlock apart, so each count read
// of a wave covers consecutive slots; the groups come out in tile order and,
// inside a tile, thread by thread (the output order is unspecified).
constexpr int kFinIPT = 8;
constexpr int64_t kFinTile = (int64_t)kBlock * kFinIPT;
// Consecutive tiles per ticket (one look-back per group of them): tickets
// are atomics on one cache line, which serialise on this chip at about 12 ns
// each.
constexpr int64_t kFinTilesPerTicket = 4;

// Group table; the last slot holds the key INT64_MIN. With `clean` each slot
// read is emptied again, so that the table needs no clearing before its next
// use (only occupied slots are written, instead of the whole table).
struct SlotSource {
  GroupSlot* slots;
  int64_t side;
  bool clean;
  __device__ bool occupied(int64_t i) const { return slots[i].count != 0; }
  __device__ void get(int64_t i, int64_t* key, uint64_t* sp, uint64_t* sq, uint64_t* cnt) const {
    const GroupSlot g = slots[i];
    *key = i == side ? kGroupEmpty : g.key;
    *sp = g.sum_price;
    *sq = g.sum_qty;
    *cnt = g.count;
    if (clean) slots[i] = GroupSlot{kGroupEmpty, 0, 0, 0};
  }
};

struct RowAggSource {  // groupjoin accumulators; the key is the dim row's pk
  const RowAgg* agg;
  const int32_t* pk;
  __device__ bool occupied(int64_t i) const { return agg[i].count != 0; }
  __device__ void get(int64_t i, int64_t* key, uint64_t* sp, uint64_t* sq, uint64_t* cnt) const {
    const RowAgg r = agg[i];
    *key = pk[i];
    *sp = r.sum_price;
    *sq = r.sum_qty;
    *cnt = r.count;
  }
};

template <class Src>
__global__ __launch_bounds__(kBlock) void k_finalize(Src src, int64_t nitems, OutArgs o, uint64_t* __restrict__ state,
                                                     int64_t* __restrict__ ticket, int64_t ngroups) {
  static_assert(kFinTile < (1 << 16) && kFinTilesPerTicket * 16 <= 64, "packed per-tile counts");
  __shared__ int64_t s_group;
  __shared__ uint64_t s_excl;
  __shared__ uint64_t s_wave[kBlock / kWave];
  if (o.done != nullptr && *o.done != 0) return;
  if (threadIdx.x == 0) s_group = (int64_t)dev_add_ret<unsigned long long>((unsigned long long*)ticket, 1ull);
  __syncthreads();
  const int64_t group = s_group;
  const int64_t t0 = group * kFinTilesPerTicket;
  uint32_t bits[kFinTilesPerTicket];
  uint64_t c = 0;
#pragma unroll
  for (int g = 0; g < kFinTilesPerTicket; ++g) {
    const int64_t i0 = (t0 + g) * kFinTile + (int64_t)threadIdx.x;  // slot of bit k: i0 + k * kBlock
    bits[g] = 0;
#pragma unroll
    for (int k = 0; k < kFinIPT; ++k) {
      const int64_t i = i0 + (int64_t)k * kBlock;
      if (i < nitems && src.occupied(i)) bits[g] |= 1u << k;
    }
    c |= (uint64_t)__popc(bits[g]) << (16 * g);
  }
  const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
  uint64_t incl = c;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint64_t t = (uint64_t)__shfl_up((unsigned long long)incl, d, kWave);
    if (lane >= (uint32_t)d) incl += t;
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
  for (int g = 0; g < kFinTilesPerTicket; ++g) group_total += (uint32_t)(total >> (16 * g)) & 0xFFFFu;
  if (wave == 0) {
    const uint64_t excl = lookback_prefix(state, group, group_total);
    if (threadIdx.x == 0) {
      s_excl = excl;
      if (group == ngroups - 1) *o.d_n = (int64_t)(excl + group_total);
    }
  }
  __syncthreads();
  int64_t before = 0;  // groups of the earlier tiles of this ticket
#pragma unroll
  for (int g = 0; g < kFinTilesPerTicket; ++g) {
    const int64_t i0 = (t0 + g) * kFinTile + (int64_t)threadIdx.x;
    int64_t pos = (int64_t)s_excl + before + (int64_t)((my_off >> (16 * g)) & 0xFFFFu);
    for (int k = 0; k < kFinIPT; ++k) {
      if (!(bits[g] & (1u << k))) continue;
      if (pos < o.cap) {
        int64_t key;
        uint64_t sp, sq, cnt;
        src.get(i0 + (int64_t)k * kBlock, &key, &sp, &sq, &cnt);
        o.key[pos] = key;
        o.sum_price[pos] = (int64_t)sp;
        o.sum_qty[pos] = (int64_t)sq;
        o.count[pos] = (int64_t)cnt;
      } else {
        set_status(o.status, kDevOverflow);
      }
      ++pos;
    }
    before += (total >> (16 * g)) & 0xFFFFu;
  }
  // (as the merge kernel does when there is one)
  if (group == 0 && o.n_wg > 0) sum_wg_counts<kBlock>(o.wg_counts, o.n_wg, o.join, o.counters, o.status);
}

// Tiles of the finalize kernel over nitems slots (with no items, one empty
// tile still sums the per-workgroup counts), and its look-back state.
int64_t finalize_tiles(int64_t nitems) { return nitems > 0 ? (nitems + kFinTile - 1) / kFinTile : 1; }

rel_status finalize_state(rel_ctx* ctx, int64_t nitems, uint64_t** st) {
  void* p;
  rel_status s = relh::scratch(ctx, SCR_SCAN_STATE, (size_t)finalize_tiles(nitems) * 8, &p);
  *st = (uint64_t*)p;
  return s;
}

// zeroed: the look-back state (finalize_state) and the ticket counter are
// already zero (an earlier kernel of the call cleared them), else they are
// cleared here.
template <class Src>
rel_status finalize(rel_ctx* ctx, const Src& src, int64_t nitems, const OutArgs& o, bool zeroed = false) {
  // (when the kernel runs, its last group of tiles writes the group count)
  if (nitems == 0 && o.n_wg == 0) return relh::fill_u64(ctx, o.d_n, 1, 0);
  rel_status s;
  const int64_t ntiles = finalize_tiles(nitems);
  uint64_t* st;
  if ((s = finalize_state(ctx, nitems, &st)) != REL_OK) return s;
  int64_t* ticket = relh::counters(ctx) + CNT_TICKET;
  if (!zeroed) {
    if ((s = relh::fill_u64(ctx, st, (size_t)ntiles, 0)) != REL_OK) return s;
    if ((s = relh::fill_u64(ctx, ticket, 1, 0)) != REL_OK) return s;
  }
  relh::KernelTimer kt(ctx, "finalize");
  const int64_t ngroups = (ntiles + kFinTilesPerTicket - 1) / kFinTilesPerTicket;
  hipLaunchKernelGGL(k_finalize<Src>, dim3((unsigned)ngroups), dim3(kBlock), 0, ctx->stream, src, nitems, o,
                     (uint64_t*)st, ticket, ngroups);
  REL_LAUNCH_CHECK(ctx, "finalize");
  return REL_OK;
}

rel_status init_groups(rel_ctx* ctx, GroupSlot* slots, int64_t nslots) {
  const unsigned grid = relh::grid_for(ctx, nslots, 256 * 4, 4);
  relh::KernelTimer kt(ctx, "group_table_init");
  hipLaunchKernelGGL(k_init_groups, dim3(grid), dim3(256), 0, ctx->stream, slots, nslots);
  REL_LAUNCH_CHECK(ctx, "init_groups");
  return REL_OK;
}

bool out_ok(const rel_groups_out* out) {
  return out && out->key && out->sum_price && out->sum_qty && out->count && out->d_n_groups && out->cap >= 0;
}

OutArgs out_args(rel_ctx* ctx, const rel_groups_out* out) {
  return OutArgs{out->key, out->sum_price, out->sum_qty, out->count, out->cap, out->d_n_groups, ctx->d_status,
                 nullptr, 0, nullptr, nullptr, JoinIndex{}};
}

// Group-table capacity (power of two) for `expected` distinct keys at load `load`.
uint32_t group_log2cap(int64_t expected, double load) {
  if (expected < 1) expected = 1;
  uint32_t l = relh::log2_ceil((uint64_t)((double)expected / load) + 1);
  return l < 4 ? 4 : l;
}

template <int MODE>
rel_status launch_fused(rel_ctx* ctx, int gp, const FusedArgs& a, unsigned grid) {
  relh::KernelTimer kt(ctx, "probe_agg");
  if (gp == G_LDS)
    hipLaunchKernelGGL((k_fused<MODE, G_LDS, kLdsBlock>), dim3(grid), dim3(kLdsBlock), 0, ctx->stream, a);
  else if (gp == G_GLOBAL)
    hipLaunchKernelGGL((k_fused<MODE, G_GLOBAL, kBlock>), dim3(grid), dim3(kBlock), 0, ctx->stream, a);
  else
    hipLaunchKernelGGL((k_fused<MODE, G_ROWAGG, kBlock>), dim3(grid), dim3(kBlock), 0, ctx->stream, a);
  REL_LAUNCH_CHECK(ctx, "fused");
  return REL_OK;
}

#define TRY(x)                      \
  do {                              \
    rel_status s_ = (x);            \
    if (s_ != REL_OK) return s_;    \
  } while (0)

// Fact tables at least this large take the radix-partitioned path unless a
// plan says otherwise ...
constexpr int64_t kPartitionMinRows = 1 << 20;
// ... and, grouping by a dim attribute, at least this many dim rows. Below
// it the plain path's join index (a dense array of 4 B per key when the keys
// are dense, 16 MB at this size) stays in the caches.
constexpr int64_t kPartitionMinDim = 1 << 22;

rel_status sync_stats(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, const rel_query* q, const rel_plan* plan,
                      rel_groups_out* out, rel_stats* stats, int64_t* cnt, int64_t join_cap, int64_t group_cap,
                      int join_place, int group_place);

}  // namespace

extern "C" {

rel_status rel_groupby_agg(rel_ctx* ctx, const int64_t* key, const int64_t* price, const int32_t* qty,
                           const int32_t* sel, int64_t n, const rel_table_opts* opts, rel_groups_out* out) {
  if (!ctx || n < 0 || !out_ok(out) || (n > 0 && (!key || !price || !qty)))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_groupby_agg: bad argument");
  if (n >= (1ll << 31)) return relh::fail(ctx, REL_UNSUPPORTED, "rel_groupby_agg: n >= 2^31");
  const double load = (opts && opts->max_load > 0.f) ? (opts->max_load > 0.9f ? 0.9 : opts->max_load) : 0.5;
  int64_t expected = (opts && opts->capacity_hint > 0) ? opts->capacity_hint : (n < (1ll << 30) ? n : (1ll << 30));
  int placement = opts ? opts->placement : REL_PLACE_AUTO;
  if (placement == REL_PLACE_PARTITIONED) return relh::fail(ctx, REL_UNSUPPORTED, "rel_groupby_agg: partitioned placement");
  if (placement == REL_PLACE_AUTO) placement = expected <= kLdsSlots / 2 ? REL_PLACE_LDS : REL_PLACE_GLOBAL;
  const uint32_t l = group_log2cap(expected, load);
  if (l > 31) return relh::fail(ctx, REL_UNSUPPORTED, "rel_groupby_agg: capacity above 2^31");
  const int64_t nslots = (1ll << l) + 1;
  void* tbl;
  TRY(relh::scratch(ctx, SCR_GROUP_TABLE, (size_t)nslots * sizeof(GroupSlot), &tbl));
  TRY(init_groups(ctx, (GroupSlot*)tbl, nslots));
  const uint32_t probe = (opts && opts->capacity_hint > 0) ? kPlannedProbe : (uint32_t)(1ull << l);
  GroupView g{(GroupSlot*)tbl, (uint32_t)((1ull << l) - 1), 32u - l, ctx->d_status, probe};
  if (n > 0) {
    const unsigned grid = relh::grid_for(ctx, n, kBlock * 4, placement == REL_PLACE_LDS ? 2 : 8);
    relh::KernelTimer kt(ctx, "groupby");
    if (placement == REL_PLACE_LDS)
      hipLaunchKernelGGL(k_groupby<G_LDS>, dim3(grid), dim3(kBlock), 0, ctx->stream, key, price, qty, sel, n, g);
    else
      hipLaunchKernelGGL(k_groupby<G_GLOBAL>, dim3(grid), dim3(kBlock), 0, ctx->stream, key, price, qty, sel, n, g);
    REL_LAUNCH_CHECK(ctx, "groupby");
  }
  return finalize(ctx, SlotSource{(GroupSlot*)tbl, nslots - 1, false}, nslots, out_args(ctx, out));
}

rel_status rel_filter_join_agg(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, const rel_query* q,
                               const rel_plan* plan, rel_groups_out* out, rel_stats* stats) {
  if (!ctx || !fact || !dim || !q || !out_ok(out)) return relh::fail(ctx, REL_INVALID_ARG, "rel_filter_join_agg: null argument");
  const int64_t n = fact->n, m = dim->m;
  const int gb = q->group_by;
  if (n < 0 || m < 0 || gb < REL_GROUP_PRIO_FLAG || gb > REL_GROUP_DIM_GRP)
    return relh::fail(ctx, REL_INVALID_ARG, "rel_filter_join_agg: bad size or group_by");
  if (n > 0 && (!fact->fk || !fact->price_cents || !fact->qty || !fact->day || (gb == REL_GROUP_PRIO_FLAG && !fact->flag)))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_filter_join_agg: missing fact column");
  if (m > 0 && (!dim->pk || (gb == REL_GROUP_PRIO_FLAG && !dim->prio) || (gb == REL_GROUP_DIM_GRP && !dim->grp)))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_filter_join_agg: missing dim column");
  const void* cols[] = {fact->fk, fact->price_cents, fact->qty, fact->day, fact->flag, dim->pk, dim->prio, dim->grp};
  for (const void* c : cols)
    if (c && !relh::aligned16(c)) return relh::fail(ctx, REL_INVALID_ARG, "rel_filter_join_agg: column not 16-byte aligned");
  if (n >= (1ll << 31) || m >= (1ll << 30)) return relh::fail(ctx, REL_UNSUPPORTED, "rel_filter_join_agg: table too large");
  TRY(relh::ensure_counters(ctx));
  int64_t* cnt = relh::counters(ctx);
  const bool planned = plan && plan->group_capacity > 0;
  // A call that synchronises reports through its own status word, cleared
  // here; the others leave their bits in the sticky word for rel_ctx_sync.
  struct StatusScope {
    rel_ctx* c;
    uint32_t* saved;
    ~StatusScope() { c->d_status = saved; }
  } scope{ctx, ctx->d_status};
  if (stats != nullptr || (planned && plan->allow_fallback)) {
    ctx->d_status = ctx->d_status_words + 1;
    TRY(relh::fill_u32(ctx, ctx->d_status, 1, 0));
  } else {
    ctx->d_status = ctx->d_status_words;  // also inside a synchronising call's fallback run
  }

  // Radix partitioning of both sides: asked for, or chosen for large inputs
  // (for a dim-attribute group key only when the dim side is large enough that
  // its join table would not stay in L2).
  const int jp = plan ? plan->join_placement : REL_PLACE_AUTO;
  const bool part = jp == REL_PLACE_PARTITIONED ||
                    (jp == REL_PLACE_AUTO && n >= kPartitionMinRows && (gb == REL_GROUP_FK || m >= kPartitionMinDim));
  if (part && gb == REL_GROUP_FK) {
    // with fact rows, the partitioning's first kernel clears the two counters
    if (n == 0) TRY(relh::fill_u64(ctx, cnt, 2, 0));
    TRY(relh::partitioned_groupjoin(ctx, fact, dim, q->day_lt, out, cnt));
    return sync_stats(ctx, fact, dim, q, plan, out, stats, cnt, m, m, REL_PLACE_PARTITIONED, REL_PLACE_PARTITIONED);
  }

  FusedArgs a{};
  a.fk = fact->fk;
  a.price = fact->price_cents;
  a.qty = fact->qty;
  a.day = fact->day;
  a.flag = fact->flag;
  a.n = n;
  a.day_lt = q->day_lt;

  int gp;
  int64_t group_cap = 0;
  uint32_t gl = 0;
  void* gt = nullptr;
  size_t clean_after = 0;
  if (gb == REL_GROUP_FK) {
    gp = G_ROWAGG;  // group key == join key: per-dim-row accumulators
    group_cap = m;
    TRY(relh::scratch(ctx, SCR_GROUP_TABLE, (size_t)(m > 0 ? m : 1) * sizeof(RowAgg), &gt));
    {
      relh::KernelTimer kt(ctx, "group_table_init");
      TRY(relh::fill_u64(ctx, gt, (size_t)m * 3, 0));
    }
    a.row_agg = (RowAgg*)gt;
  } else {
    const int64_t ub = gb == REL_GROUP_PRIO_FLAG ? (n < 65536 ? n : 65536) : (n < m ? n : m);
    const int64_t expected = planned ? plan->group_capacity : ub;
    int placement = plan ? plan->group_placement : REL_PLACE_AUTO;
    if (placement == REL_PLACE_PARTITIONED) return relh::fail(ctx, REL_UNSUPPORTED, "rel_filter_join_agg: partitioned group-by");
    if (placement == REL_PLACE_AUTO) placement = (gb == REL_GROUP_PRIO_FLAG || expected <= kLdsSlots / 2) ? REL_PLACE_LDS : REL_PLACE_GLOBAL;
    gp = placement == REL_PLACE_LDS ? G_LDS : G_GLOBAL;
    // With more groups than the LDS table holds, LDS acts as a cache in front of
    // the device-memory table (it keeps the keys each workgroup meets first,
    // which under skew are the hot ones); a short probe budget bounds the cost
    // of rows whose key is not cached.
    a.lds_probe = expected <= relh::kLdsGroupCap ? kLdsProbe : kLdsCacheProbe;
    gl = group_log2cap(expected, 0.5);
    if (gl > 31) return relh::fail(ctx, REL_UNSUPPORTED, "rel_filter_join_agg: group table above 2^31 slots");
    group_cap = 1ll << gl;
    const size_t gbytes = (size_t)(group_cap + 1) * sizeof(GroupSlot);
    if (part) {
      TRY(relh::scratch(ctx, SCR_GROUP_TABLE, gbytes, &gt));
      TRY(init_groups(ctx, (GroupSlot*)gt, group_cap + 1));
    } else {
      // the plain path's table is emptied again by the kernel that reads it,
      // so only its first use (or a larger one) clears it
      TRY(relh::scratch(ctx, SCR_GROUP_CLEAN, gbytes, &gt));
      ScratchBuf& sb = ctx->scratch[SCR_GROUP_CLEAN];
      clean_after = sb.clean > gbytes ? sb.clean : gbytes;
      if (sb.clean < gbytes) TRY(init_groups(ctx, (GroupSlot*)gt, group_cap + 1));
      sb.clean = 0;  // until this call's finalize kernel is enqueued
    }
    a.groups = GroupView{(GroupSlot*)gt, (uint32_t)(group_cap - 1), 32u - gl, ctx->d_status,
                         planned ? kPlannedProbe : (uint32_t)group_cap};
  }

  if (part) {
    // the same group table behind a per-workgroup LDS table (probe budget 0:
    // none); grouping by dim.grp with more groups than LDS holds aggregates per
    // dim key first
    TRY(relh::fill_u64(ctx, cnt, CNT_AUX2 + 1, 0));
    const bool eager = gb == REL_GROUP_DIM_GRP && (gp != G_LDS || a.lds_probe != kLdsProbe);
    TRY(relh::partitioned_join_agg(ctx, fact, dim, q->day_lt, gb, gt, gl, a.groups.max_probe,
                                   gp == G_LDS ? a.lds_probe : 0, eager, cnt));
    TRY(finalize(ctx, SlotSource{(GroupSlot*)gt, group_cap, false}, group_cap + 1, out_args(ctx, out)));
    return sync_stats(ctx, fact, dim, q, plan, out, stats, cnt, m, group_cap, REL_PLACE_PARTITIONED,
                      gp == G_LDS ? REL_PLACE_LDS : REL_PLACE_GLOBAL);
  }

  // Join index: a dense array when the dim keys span at most 2m values, else
  // a hash table of plain sizing (2m rounded up to a power of two); both in
  // device memory, the choice made on the device. Its clearing kernel also
  // zeroes the counter words (rows passed, join matches, the finalize ticket,
  // the merge kernel's two flags) and the finalize kernel's look-back state.
  const int64_t fin_items = gp == G_ROWAGG ? m : group_cap + 1;
  uint64_t* fin_state;
  TRY(finalize_state(ctx, fin_items, &fin_state));
  const relh::ZeroSpans zero{{(uint64_t*)cnt, fin_state}, {CNT_AUX2, finalize_tiles(fin_items)}};
  const uint32_t jl = relh::join_log2cap(m, nullptr);
  const void* payload = gb == REL_GROUP_PRIO_FLAG ? (const void*)dim->prio : gb == REL_GROUP_DIM_GRP ? (const void*)dim->grp : nullptr;
  const int pkind = gb == REL_GROUP_PRIO_FLAG ? relh::PAY_I8 : gb == REL_GROUP_DIM_GRP ? relh::PAY_I32 : relh::PAY_ROW_ID;
  JoinIndex jx{};
  TRY(relh::join_index_build(ctx, dim->pk, payload, pkind, m, (uint32_t*)(cnt + CNT_AUX2), zero, &jx));
  a.join = jx;

  OutArgs oa = out_args(ctx, out);
  if (n > 0) {
    const unsigned grid = gp == G_LDS ? relh::grid_for(ctx, n, kLdsBlock * kIPT, 1) : relh::grid_for(ctx, n, kBlock * kIPT, 8);
    void* wc;
    TRY(relh::scratch(ctx, SCR_WG_COUNTS, (size_t)grid * 24, &wc));
    a.wg_counts = (uint64_t*)wc;
    oa.wg_counts = a.wg_counts;
    oa.n_wg = grid;
    oa.counters = cnt;
    oa.join = jx;
    uint32_t* flags = (uint32_t*)(cnt + CNT_AUX1);  // [0] touched, [1] done
    if (gp == G_LDS) {
      void* stage;
      TRY(relh::scratch(ctx, SCR_STAGE, (size_t)grid * kStageMax * sizeof(GroupSlot), &stage));
      a.stage = (GroupSlot*)stage;
      a.touched = flags;
    }
    if (gb == REL_GROUP_PRIO_FLAG) TRY(launch_fused<M_PRIO_FLAG>(ctx, gp, a, grid));
    else if (gb == REL_GROUP_FK) TRY(launch_fused<M_FK>(ctx, gp, a, grid));
    else TRY(launch_fused<M_DIM_GRP>(ctx, gp, a, grid));
    if (gp == G_LDS) {
      MergeArgs mg{a.stage, flags, (int64_t)grid, a.wg_counts, cnt, a.groups, flags + 1, jx};
      oa.n_wg = 0;  // the merge kernel sums the counts
      oa.done = flags + 1;
      relh::KernelTimer kt(ctx, "group_merge");
      hipLaunchKernelGGL(k_group_merge, dim3(1), dim3(kLdsBlock), 0, ctx->stream, mg, oa);
      REL_LAUNCH_CHECK(ctx, "group_merge");
    }
  } else {
    TRY(relh::join_index_verify(ctx, jx));  // (no probing kernel runs)
  }

  if (gp == G_ROWAGG) {
    TRY(finalize(ctx, RowAggSource{(const RowAgg*)gt, dim->pk}, m, oa, true));
  } else {
    TRY(finalize(ctx, SlotSource{(GroupSlot*)gt, group_cap, true}, group_cap + 1, oa, true));
    ctx->scratch[SCR_GROUP_CLEAN].clean = clean_after;
  }
  return sync_stats(ctx, fact, dim, q, plan, out, stats, cnt, (int64_t)1 << jl, group_cap, REL_PLACE_GLOBAL,
                    gp == G_LDS ? REL_PLACE_LDS : REL_PLACE_GLOBAL);
}

}  // extern "C"

namespace {

// Common tail of the fused pipeline: when the caller wants statistics or a
// planned table may need the fallback, synchronise, read the counters and the
// status word, and rerun with plain sizing if a planned table overflowed.
rel_status sync_stats(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, const rel_query* q, const rel_plan* plan,
                      rel_groups_out* out, rel_stats* stats, int64_t* cnt, int64_t join_cap, int64_t group_cap,
                      int join_place, int group_place) {
  const int64_t n = fact->n;
  const bool planned = plan && plan->group_capacity > 0;
  const bool want_sync = stats != nullptr || (planned && plan->allow_fallback);
  if (!want_sync) return REL_OK;
  REL_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  int64_t hc[2] = {0, 0}, ng = 0;
  uint32_t bits = 0;
  REL_HIP_CHECK(ctx, hipMemcpy(hc, cnt, sizeof hc, hipMemcpyDeviceToHost));
  REL_HIP_CHECK(ctx, hipMemcpy(&ng, out->d_n_groups, sizeof ng, hipMemcpyDeviceToHost));
  // this call's own word (cleared at its start)
  REL_HIP_CHECK(ctx, hipMemcpy(&bits, ctx->d_status, sizeof bits, hipMemcpyDeviceToHost));
  if (bits & kDevDupKey) return relh::fail(ctx, REL_DUPLICATE_KEY, "rel_filter_join_agg: duplicate pk");
  const bool overflow = (bits & kDevOverflow) != 0;
  if (overflow && ng > out->cap) return relh::fail(ctx, REL_CAPACITY, "rel_filter_join_agg: %lld groups > cap", (long long)ng);
  if (overflow && planned) {
    if (!plan->allow_fallback) return relh::fail(ctx, REL_OVERFLOW, "rel_filter_join_agg: planned table overflowed");
    rel_status s = rel_filter_join_agg(ctx, fact, dim, q, nullptr, out, stats);
    if (s == REL_OK && stats) {
      stats->overflowed = 1;
      stats->fell_back = 1;
    }
    return s;
  }
  if (overflow) return relh::fail(ctx, REL_OVERFLOW, "rel_filter_join_agg: table overflow");
  if (stats) {
    stats->rows_in = n;
    stats->rows_passed = hc[0];
    stats->join_matches = hc[1];
    stats->groups = ng;
    stats->join_capacity = join_cap;
    stats->group_capacity = group_cap;
    stats->join_placement = join_place;
    stats->group_placement = group_place;
    stats->overflowed = 0;
    stats->fell_back = 0;
  }
  return REL_OK;
}

}  // namespace
