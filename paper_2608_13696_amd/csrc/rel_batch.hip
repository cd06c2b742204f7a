// Batched execution of many independent fused queries.
//
// A small query alone cannot fill 256 CUs (the paper's undersaturation
// finding, Section 6.1); thousands of them issued one by one pay a launch and
// a dependency gap per kernel. Here every instance's build, probe/aggregate
// and finalize become work items of three persistent kernels (one per phase
// and size bucket), workgroups pull items largest-first from a ticket
// counter, and the whole sequence is captured once into a HIP graph so that a
// run is one graph launch.
//
// Per-bucket configuration (rows per thread, workgroup size, LDS or
// device-memory group table, LDS or device-memory join table, rows per work
// item) comes from a tuning table that the autotuner measures.
#include <algorithm>
#include <numeric>

#include "rel_device.h"
#include "rel_host.h"
#include "rel_ops.h"

namespace {

using namespace rel;

constexpr int kBLdsSlots = 1024;
constexpr int kBLdsProbe = 32;
// Instances with more groups than the LDS table holds still use it as a
// cache in front of their device-memory table: the first keys a workgroup
// meets stay in LDS (one set of device atomics per key and work item instead
// of one per row), and a short probe budget bounds the cost for the others.
constexpr int kBLdsCacheProbe = 4;
constexpr int64_t kFinItemSlots = 8192;
// LDS join table: 2048 packed slots (and the side slot of key -1, as in the
// device-memory table), for instances of at most 1024 dim keys (load <= 0.5).
constexpr int kBLdsJoinBits = 11;
constexpr int kBLdsJoinSlots = 1 << kBLdsJoinBits;
constexpr uint32_t kHintProbe = 256;

// Device view of one instance (all pointers device memory).
struct BInst {
  const int32_t* fk;
  const int64_t* price;
  const int32_t* qty;
  const int32_t* day;
  const int8_t* flag;
  const int32_t* pk;
  const int8_t* prio;
  const int32_t* grp;
  int64_t n, m;
  int32_t day_lt, group_by;
  uint64_t* jslots;
  uint32_t jmask, jshift;
  GroupSlot* gslots;
  uint32_t gmask, gshift, gprobe;
  int32_t lds;    // aggregate through the workgroup's LDS table first
  int32_t ljoin;  // probe a join table built in the workgroup's LDS for each work item
  int64_t* out_key;
  int64_t* out_sp;
  int64_t* out_sq;
  int64_t* out_cnt;
  int64_t out_cap;
  int64_t* d_n;
  int64_t* stats;  // [rows passed, join matches, groups]
};

struct BItem {
  int32_t inst;
  int32_t pad;
  int64_t lo, hi;
};

// The join payload of dim row j (the group attribute, or the row id for GROUP BY fk).
__device__ __forceinline__ int32_t batch_payload(const BInst& I, int64_t j) {
  return I.group_by == REL_GROUP_PRIO_FLAG ? (int32_t)I.prio[j] : I.group_by == REL_GROUP_DIM_GRP ? I.grp[j] : (int32_t)j;
}

__global__ void k_batch_zero_outputs(const BInst* __restrict__ inst, int32_t k) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) *inst[i].d_n = 0;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch_build(const BInst* __restrict__ inst, const BItem* __restrict__ items,
                                                       int64_t n_items, int64_t* __restrict__ ticket,
                                                       uint32_t* __restrict__ status) {
  __shared__ int64_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int64_t)dev_add_ret<unsigned long long>((unsigned long long*)ticket, 1ull);
    __syncthreads();
    const int64_t it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const BItem w = items[it];
    const BInst& I = inst[w.inst];
    for (int64_t j = w.lo + threadIdx.x; j < w.hi; j += BLOCK) {
      join_insert(I.jslots, I.jmask, I.jshift, I.pk[j], batch_payload(I, j), status);
    }
  }
}

__device__ __forceinline__ int64_t batch_key(const BInst& I, int32_t pl, int32_t fk, int8_t flag) {
  if (I.group_by == REL_GROUP_PRIO_FLAG) return (int64_t)pl * 256 + (int64_t)(uint8_t)flag;
  if (I.group_by == REL_GROUP_DIM_GRP) return (int64_t)pl;
  return (int64_t)fk;
}

// An instance's join table in LDS, in the packed format of the device-memory
// table (key in the low word, payload in the high word, key -1 in the side
// slot). The workgroup builds it from the dim columns at the start of each
// work item of a small-dim instance, so the probes of the item's rows are LDS
// reads instead of device-memory reads. A repeated key is reported by the
// instance's device-memory build, which every instance still runs.
struct LdsJoin {
  uint64_t slot[kBLdsJoinSlots + 1];

  __device__ void init(int tid, int nthreads) {
    for (int s = tid; s <= kBLdsJoinSlots; s += nthreads) slot[s] = kJoinEmpty;
  }
  // At most kBLdsJoinSlots / 2 keys, so a free slot always exists.
  __device__ void insert(int32_t key, int32_t pl) {
    if (key == -1) {
      atomicCAS((unsigned long long*)&slot[kBLdsJoinSlots], (unsigned long long)kJoinEmpty, (unsigned long long)(uint32_t)pl);
      return;
    }
    const uint64_t want = (uint64_t)(uint32_t)key | ((uint64_t)(uint32_t)pl << 32);
    uint32_t h = hash32(key, 32 - kBLdsJoinBits);
    for (int step = 0; step < kBLdsJoinSlots; ++step) {
      const uint64_t old = atomicCAS((unsigned long long*)&slot[h], (unsigned long long)kJoinEmpty, (unsigned long long)want);
      if (old == kJoinEmpty || (uint32_t)old == (uint32_t)key) return;
      h = (h + 1) & (kBLdsJoinSlots - 1);
    }
  }
  __device__ __forceinline__ bool lookup(int32_t key, int32_t* pl) const {
    if (key == -1) {
      const uint64_t s = slot[kBLdsJoinSlots];
      *pl = (int32_t)(uint32_t)s;
      return s != kJoinEmpty;
    }
    uint32_t h = hash32(key, 32 - kBLdsJoinBits);
    for (int step = 0; step < kBLdsJoinSlots; ++step) {
      const uint64_t s = slot[h];
      if (s == kJoinEmpty) return false;
      if ((uint32_t)s == (uint32_t)key) {
        *pl = (int32_t)(s >> 32);
        return true;
      }
      h = (h + 1) & (kBLdsJoinSlots - 1);
    }
    return false;
  }
};

// LJ: the instance of the kernel that carries the LDS join table (16 KB more
// LDS per workgroup); only buckets whose tuning enables it launch it.
template <bool LJ>
struct LdsJoinStore {
  LdsJoin t;
};
template <>
struct LdsJoinStore<false> {};

template <int BLOCK, int IPT, bool LJ>
__global__ __launch_bounds__(BLOCK) void k_batch_probe(const BInst* __restrict__ inst, const BItem* __restrict__ items,
                                                       int64_t n_items, int64_t* __restrict__ ticket,
                                                       uint32_t* __restrict__ status) {
  __shared__ LdsGroups<kBLdsSlots> lds;
  __shared__ LdsJoinStore<LJ> ljs;
  __shared__ int64_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int64_t)dev_add_ret<unsigned long long>((unsigned long long*)ticket, 1ull);
    __syncthreads();
    const int64_t it = s_item;
    if (it >= n_items) break;
    const BItem w = items[it];
    const BInst& I = inst[w.inst];
    const int lds_probe = I.lds != 0 ? kBLdsProbe : kBLdsCacheProbe;
    const JoinView jv{I.jslots, I.jmask, I.jshift};
    const GroupView gv{I.gslots, I.gmask, I.gshift, status, I.gprobe};
    bool lj = false;  // uniform over the workgroup (one item)
    if constexpr (LJ) {
      lj = I.ljoin != 0;
      if (lj) {
        ljs.t.init(threadIdx.x, BLOCK);
        __syncthreads();
        for (int64_t j = threadIdx.x; j < I.m; j += BLOCK) ljs.t.insert(I.pk[j], batch_payload(I, j));
      }
    }
    lds.init(threadIdx.x, BLOCK);
    __syncthreads();
    uint64_t passed = 0, matched = 0;
    for (int64_t r0 = w.lo + threadIdx.x; r0 < w.hi; r0 += (int64_t)BLOCK * IPT) {
      int32_t d[IPT], f[IPT], q[IPT];
      int64_t p[IPT];
      int8_t fl[IPT];
#pragma unroll
      for (int k = 0; k < IPT; ++k) {  // all loads first; strided rows keep each load coalesced
        const int64_t r = r0 + (int64_t)k * BLOCK;
        const bool ok = r < w.hi;
        d[k] = ok ? I.day[r] : 0;
        f[k] = ok ? I.fk[r] : 0;
        q[k] = ok ? I.qty[r] : 0;
        p[k] = ok ? I.price[r] : 0;
        fl[k] = (ok && I.group_by == REL_GROUP_PRIO_FLAG) ? I.flag[r] : 0;
      }
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        if (r0 + (int64_t)k * BLOCK >= w.hi || !(d[k] < I.day_lt)) continue;
        ++passed;
        int32_t pl;
        bool hit;
        if constexpr (LJ) hit = lj ? ljs.t.lookup(f[k], &pl) : join_lookup(jv, f[k], &pl);
        else hit = join_lookup(jv, f[k], &pl);
        if (!hit) continue;
        ++matched;
        const int64_t key = batch_key(I, pl, f[k], fl[k]);
        const uint64_t sp = (uint64_t)p[k], sq = (uint64_t)(int64_t)q[k];
        const int s = key != kGroupEmpty ? lds.find(key, lds_probe) : -1;
        if (s >= 0) lds.add(s, sp, sq, 1ull);
        else group_add(gv, key, sp, sq, 1ull);
      }
    }
    __syncthreads();
    lds.flush(gv, threadIdx.x, BLOCK);
    passed = wave_sum(passed);
    matched = wave_sum(matched);
    if (lane_id() == 0) {
      if (passed) dev_add<unsigned long long>((unsigned long long*)&I.stats[0], passed);
      if (matched) dev_add<unsigned long long>((unsigned long long*)&I.stats[1], matched);
    }
    __syncthreads();
  }
}

// Emit the occupied group slots of each instance: one atomic per wave on the
// instance's own output counter (instances are small, so it is not contended).
__global__ __launch_bounds__(256) void k_batch_finalize(const BInst* __restrict__ inst, const BItem* __restrict__ items,
                                                        int64_t n_items, int64_t* __restrict__ ticket,
                                                        uint32_t* __restrict__ status) {
  __shared__ int64_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int64_t)dev_add_ret<unsigned long long>((unsigned long long*)ticket, 1ull);
    __syncthreads();
    const int64_t it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const BItem w = items[it];
    const BInst& I = inst[w.inst];
    const int64_t side = (int64_t)I.gmask + 1;
    // wave-uniform trip count, so ballots see every lane
    for (int64_t base = w.lo + (threadIdx.x / kWave) * kWave; base < w.hi; base += 256) {
      const int64_t s = base + lane_id();
      bool occ = false;
      GroupSlot g{};
      if (s < w.hi) {
        g = I.gslots[s];
        occ = g.count != 0;
        if (s == side) g.key = kGroupEmpty;
      }
      const uint64_t b = wave_ballot(occ);
      if (b == 0) continue;
      int64_t pos = 0;
      if (lane_id() == 0) {
        pos = (int64_t)dev_add_ret<unsigned long long>((unsigned long long*)I.d_n, (unsigned long long)__popcll(b));
        dev_add<unsigned long long>((unsigned long long*)&I.stats[2], (unsigned long long)__popcll(b));
      }
      pos = __shfl(pos, 0, kWave) + mask_rank(b);
      if (!occ) continue;
      if (pos < I.out_cap) {
        I.out_key[pos] = g.key;
        I.out_sp[pos] = (int64_t)g.sum_price;
        I.out_sq[pos] = (int64_t)g.sum_qty;
        I.out_cnt[pos] = (int64_t)g.count;
      } else {
        set_status(status, kDevOverflow);
      }
    }
  }
}

__global__ void k_batch_init_groups(GroupSlot* __restrict__ slots, int64_t nslots) {
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

__global__ void k_batch_fill(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

const rel_batch_tuning kDefaultTuning[] = {
    {12, 4, 256, 512, 1024, 0},
    {16, 4, 256, 512, 8192, 0},
    {20, 4, 256, 512, 16384, 0},
    {31, 4, 256, 512, 65536, 0},
};

bool tuning_ok(const rel_batch_tuning& t) {
  const bool ipt = t.items_per_thread == 1 || t.items_per_thread == 2 || t.items_per_thread == 4 || t.items_per_thread == 8;
  const bool blk = t.block == 64 || t.block == 128 || t.block == 256 || t.block == 512;
  return ipt && blk && t.lds_groups_max >= 0 && t.lds_groups_max <= kBLdsSlots / 2 && t.lds_join_max >= 0 &&
         t.lds_join_max <= kBLdsJoinSlots / 2 && t.rows_per_item > 0 &&
         t.rows_per_item % (t.block * t.items_per_thread) == 0 && t.log2_rows_below > 0 && t.log2_rows_below <= 31;
}

}  // namespace

struct BucketPlan {
  rel_batch_tuning t;
  int64_t build_lo = 0, build_n = 0;  // item ranges inside the item arrays
  int64_t probe_lo = 0, probe_n = 0;
};

struct rel_batch {
  rel_ctx* ctx = nullptr;
  int32_t k = 0;
  std::vector<BucketPlan> buckets;
  void* mem = nullptr;
  BInst* d_inst = nullptr;
  BItem* d_items = nullptr;
  int64_t* d_tickets = nullptr;
  int64_t* d_stats = nullptr;
  uint32_t* d_status = nullptr;  // this batch's status word, cleared at the start of every run
  uint64_t* d_join = nullptr;
  size_t join_words = 0;
  GroupSlot* d_groups = nullptr;
  size_t group_slots = 0;
  int64_t fin_lo = 0, fin_n = 0;
  size_t zero_words = 0;  // tickets + stats + status word
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

template <int BLOCK, bool LJ>
void launch_probe(hipStream_t s, unsigned grid, int ipt, const BInst* inst, const BItem* items, int64_t n,
                  int64_t* ticket, uint32_t* status) {
  switch (ipt) {
    case 1: hipLaunchKernelGGL((k_batch_probe<BLOCK, 1, LJ>), dim3(grid), dim3(BLOCK), 0, s, inst, items, n, ticket, status); break;
    case 2: hipLaunchKernelGGL((k_batch_probe<BLOCK, 2, LJ>), dim3(grid), dim3(BLOCK), 0, s, inst, items, n, ticket, status); break;
    case 4: hipLaunchKernelGGL((k_batch_probe<BLOCK, 4, LJ>), dim3(grid), dim3(BLOCK), 0, s, inst, items, n, ticket, status); break;
    default: hipLaunchKernelGGL((k_batch_probe<BLOCK, 8, LJ>), dim3(grid), dim3(BLOCK), 0, s, inst, items, n, ticket, status); break;
  }
}

void launch_build(hipStream_t s, unsigned grid, int block, const BInst* inst, const BItem* items, int64_t n,
                  int64_t* ticket, uint32_t* status) {
  switch (block) {
    case 64: hipLaunchKernelGGL(k_batch_build<64>, dim3(grid), dim3(64), 0, s, inst, items, n, ticket, status); break;
    case 128: hipLaunchKernelGGL(k_batch_build<128>, dim3(grid), dim3(128), 0, s, inst, items, n, ticket, status); break;
    case 256: hipLaunchKernelGGL(k_batch_build<256>, dim3(grid), dim3(256), 0, s, inst, items, n, ticket, status); break;
    default: hipLaunchKernelGGL(k_batch_build<512>, dim3(grid), dim3(512), 0, s, inst, items, n, ticket, status); break;
  }
}

template <bool LJ>
void launch_probe_blk(hipStream_t s, unsigned grid, int block, int ipt, const BInst* inst, const BItem* items,
                      int64_t n, int64_t* ticket, uint32_t* status) {
  switch (block) {
    case 64: launch_probe<64, LJ>(s, grid, ipt, inst, items, n, ticket, status); break;
    case 128: launch_probe<128, LJ>(s, grid, ipt, inst, items, n, ticket, status); break;
    case 256: launch_probe<256, LJ>(s, grid, ipt, inst, items, n, ticket, status); break;
    default: launch_probe<512, LJ>(s, grid, ipt, inst, items, n, ticket, status); break;
  }
}

void launch_probe_any(hipStream_t s, unsigned grid, int block, int ipt, bool lj, const BInst* inst,
                      const BItem* items, int64_t n, int64_t* ticket, uint32_t* status) {
  if (lj) launch_probe_blk<true>(s, grid, block, ipt, inst, items, n, ticket, status);
  else launch_probe_blk<false>(s, grid, block, ipt, inst, items, n, ticket, status);
}

// Workgroups for a persistent kernel: enough to fill the chip, never more than the items.
unsigned persistent_grid(const rel_ctx* ctx, int64_t items, int block) {
  const int64_t per_cu = block >= 512 ? 2 : block >= 256 ? 4 : 8;
  int64_t g = (int64_t)ctx->num_cus * per_cu;
  if (g > items) g = items;
  return (unsigned)(g < 1 ? 1 : g);
}

void free_batch(rel_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->mem) (void)hipFree(b->mem);
  delete b;
}

}  // namespace

extern "C" {

rel_status rel_batch_create(rel_ctx* ctx, const rel_batch_item* items, int32_t k, const rel_batch_tuning* tuning,
                            int32_t n_tuning, rel_batch** out) {
  if (!ctx || !out || k < 0 || (k > 0 && !items) || n_tuning < 0 || (n_tuning > 0 && !tuning))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_batch_create: bad argument");
  std::vector<rel_batch_tuning> tun;
  if (n_tuning > 0) tun.assign(tuning, tuning + n_tuning);
  else tun.assign(std::begin(kDefaultTuning), std::end(kDefaultTuning));
  for (size_t i = 0; i < tun.size(); ++i) {
    if (!tuning_ok(tun[i])) return relh::fail(ctx, REL_INVALID_ARG, "rel_batch_create: tuning entry %zu invalid", i);
    if (i > 0 && tun[i].log2_rows_below <= tun[i - 1].log2_rows_below)
      return relh::fail(ctx, REL_INVALID_ARG, "rel_batch_create: tuning buckets must ascend");
  }
  // validate instances
  for (int32_t i = 0; i < k; ++i) {
    const rel_batch_item& it = items[i];
    const int64_t n = it.fact.n, m = it.dim.m;
    const int gb = it.q.group_by;
    if (n < 0 || m < 0 || gb < REL_GROUP_PRIO_FLAG || gb > REL_GROUP_DIM_GRP || it.group_capacity < 0 ||
        !it.out.key || !it.out.sum_price || !it.out.sum_qty || !it.out.count || !it.out.d_n_groups || it.out.cap < 0)
      return relh::fail(ctx, REL_INVALID_ARG, "rel_batch_create: instance %d invalid", i);
    if ((n > 0 && (!it.fact.fk || !it.fact.price_cents || !it.fact.qty || !it.fact.day ||
                   (gb == REL_GROUP_PRIO_FLAG && !it.fact.flag))) ||
        (m > 0 && (!it.dim.pk || (gb == REL_GROUP_PRIO_FLAG && !it.dim.prio) || (gb == REL_GROUP_DIM_GRP && !it.dim.grp))))
      return relh::fail(ctx, REL_INVALID_ARG, "rel_batch_create: instance %d misses a column", i);
    if (n >= (1ll << 31) || m >= (1ll << 30)) return relh::fail(ctx, REL_UNSUPPORTED, "rel_batch_create: instance %d too large", i);
  }

  rel_batch* b = new rel_batch();
  b->ctx = ctx;
  b->k = k;
  auto bucket_of = [&](int64_t n) {
    for (size_t t = 0; t < tun.size(); ++t)
      if (n < (1ll << tun[t].log2_rows_below)) return (int)t;
    return (int)tun.size() - 1;
  };

  // table sizes and offsets
  std::vector<BInst> hinst(k);
  std::vector<size_t> joff(k), goff(k);
  size_t jw = 0, gs = 0;
  for (int32_t i = 0; i < k; ++i) {
    const rel_batch_item& it = items[i];
    const int64_t n = it.fact.n, m = it.dim.m;
    const uint32_t jl = relh::join_log2cap(m, nullptr);
    int64_t ub = it.q.group_by == REL_GROUP_PRIO_FLAG ? std::min<int64_t>(n, 65536) : std::min(n, m);
    const bool hinted = it.group_capacity > 0 && it.group_capacity < ub;
    if (hinted) ub = it.group_capacity;
    uint32_t gl = relh::log2_ceil((uint64_t)(std::max<int64_t>(ub, 1) * 2) + 1);
    if (gl < 4) gl = 4;
    const rel_batch_tuning& t = tun[bucket_of(n)];
    BInst& I = hinst[i];
    I.fk = it.fact.fk;
    I.price = it.fact.price_cents;
    I.qty = it.fact.qty;
    I.day = it.fact.day;
    I.flag = it.fact.flag;
    I.pk = it.dim.pk;
    I.prio = it.dim.prio;
    I.grp = it.dim.grp;
    I.n = n;
    I.m = m;
    I.day_lt = it.q.day_lt;
    I.group_by = it.q.group_by;
    I.jmask = (uint32_t)((1ull << jl) - 1);
    I.jshift = 32u - jl;
    I.gmask = (uint32_t)((1ull << gl) - 1);
    I.gshift = 32u - gl;
    I.gprobe = hinted ? kHintProbe : (uint32_t)(1ull << gl);
    I.lds = (t.lds_groups_max > 0 && ub <= t.lds_groups_max) ? 1 : 0;
    I.ljoin = (t.lds_join_max > 0 && m <= t.lds_join_max) ? 1 : 0;
    I.out_key = it.out.key;
    I.out_sp = it.out.sum_price;
    I.out_sq = it.out.sum_qty;
    I.out_cnt = it.out.count;
    I.out_cap = it.out.cap;
    I.d_n = it.out.d_n_groups;
    joff[i] = jw;
    jw += (1ull << jl) + 1;
    goff[i] = gs;
    gs += (1ull << gl) + 1;
  }

  // work items, largest instance first inside each bucket
  std::vector<int32_t> order(k);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return items[x].fact.n > items[y].fact.n; });
  std::vector<BItem> hitems;
  b->buckets.resize(tun.size());
  for (size_t t = 0; t < tun.size(); ++t) {
    BucketPlan& bp = b->buckets[t];
    bp.t = tun[t];
    bp.build_lo = (int64_t)hitems.size();
    for (int32_t i : order) {
      if (bucket_of(items[i].fact.n) != (int)t) continue;
      const int64_t m = items[i].dim.m, step = std::max<int64_t>(tun[t].rows_per_item / 4, 256);
      for (int64_t lo = 0; lo < m; lo += step) hitems.push_back(BItem{i, 0, lo, std::min(m, lo + step)});
    }
    bp.build_n = (int64_t)hitems.size() - bp.build_lo;
    bp.probe_lo = (int64_t)hitems.size();
    for (int32_t i : order) {
      if (bucket_of(items[i].fact.n) != (int)t) continue;
      const int64_t n = items[i].fact.n, step = tun[t].rows_per_item;
      for (int64_t lo = 0; lo < n; lo += step) hitems.push_back(BItem{i, 0, lo, std::min(n, lo + step)});
    }
    bp.probe_n = (int64_t)hitems.size() - bp.probe_lo;
  }
  b->fin_lo = (int64_t)hitems.size();
  for (int32_t i : order) {
    const int64_t ns = (int64_t)(hinst[i].gmask) + 2;
    for (int64_t lo = 0; lo < ns; lo += kFinItemSlots) hitems.push_back(BItem{i, 0, lo, std::min(ns, lo + kFinItemSlots)});
  }
  b->fin_n = (int64_t)hitems.size() - b->fin_lo;

  // one device allocation: instances, items, tickets + stats, join tables, group tables
  const size_t n_tickets = 2 * tun.size() + 1;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_inst = 0;
  const size_t o_items = al(o_inst + sizeof(BInst) * (size_t)std::max(k, 1));
  const size_t o_zero = al(o_items + sizeof(BItem) * std::max<size_t>(hitems.size(), 1));
  // tickets, per-instance stats, and the batch's own status word (all cleared at the start of every run)
  b->zero_words = n_tickets + 3 * (size_t)k + 1;
  const size_t o_join = al(o_zero + 8 * b->zero_words);
  const size_t o_groups = al(o_join + 8 * jw);
  const size_t total = al(o_groups + sizeof(GroupSlot) * gs);
  hipError_t e = hipMalloc(&b->mem, total);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    free_batch(b);
    return relh::fail(ctx, REL_OOM, "rel_batch_create: %zu bytes of device memory", total);
  }
  char* base = (char*)b->mem;
  b->d_inst = (BInst*)(base + o_inst);
  b->d_items = (BItem*)(base + o_items);
  b->d_tickets = (int64_t*)(base + o_zero);
  b->d_stats = b->d_tickets + n_tickets;
  b->d_status = (uint32_t*)(b->d_stats + 3 * (size_t)k);
  b->d_join = (uint64_t*)(base + o_join);
  b->join_words = jw;
  b->d_groups = (GroupSlot*)(base + o_groups);
  b->group_slots = gs;
  for (int32_t i = 0; i < k; ++i) {
    hinst[i].jslots = b->d_join + joff[i];
    hinst[i].gslots = b->d_groups + goff[i];
    hinst[i].stats = b->d_stats + 3 * (size_t)i;
  }
  rel_status st = REL_OK;
  auto hip = [&](hipError_t x, const char* what) {
    if (x != hipSuccess && st == REL_OK) st = relh::hip_fail(ctx, x, what);
  };
  if (k > 0) hip(hipMemcpy(b->d_inst, hinst.data(), sizeof(BInst) * k, hipMemcpyHostToDevice), "copy instances");
  if (!hitems.empty()) hip(hipMemcpy(b->d_items, hitems.data(), sizeof(BItem) * hitems.size(), hipMemcpyHostToDevice), "copy items");
  hip(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream");
  if (st != REL_OK) {
    free_batch(b);
    return st;
  }

  // capture: reset, build, probe, finalize
  hip(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st == REL_OK) {
    hipStream_t s = b->cap;
    const unsigned fg = (unsigned)ctx->num_cus * 4;
    hipLaunchKernelGGL(k_batch_fill, dim3(fg), dim3(256), 0, s, (uint64_t*)b->d_tickets, (int64_t)b->zero_words, 0ull);
    if (jw) hipLaunchKernelGGL(k_batch_fill, dim3(fg), dim3(256), 0, s, b->d_join, (int64_t)jw, kJoinEmpty);
    if (gs) hipLaunchKernelGGL(k_batch_init_groups, dim3(fg), dim3(256), 0, s, b->d_groups, (int64_t)gs);
    if (k) hipLaunchKernelGGL(k_batch_zero_outputs, dim3((k + 255) / 256), dim3(256), 0, s, (const BInst*)b->d_inst, k);
    for (size_t t = 0; t < b->buckets.size(); ++t) {
      const BucketPlan& bp = b->buckets[t];
      if (bp.build_n)
        launch_build(s, persistent_grid(ctx, bp.build_n, bp.t.block), bp.t.block, b->d_inst, b->d_items + bp.build_lo,
                     bp.build_n, b->d_tickets + 2 * t, b->d_status);
    }
    for (size_t t = 0; t < b->buckets.size(); ++t) {
      const BucketPlan& bp = b->buckets[t];
      if (bp.probe_n)
        launch_probe_any(s, persistent_grid(ctx, bp.probe_n, bp.t.block), bp.t.block, bp.t.items_per_thread,
                         bp.t.lds_join_max > 0, b->d_inst, b->d_items + bp.probe_lo, bp.probe_n,
                         b->d_tickets + 2 * t + 1, b->d_status);
    }
    if (b->fin_n)
      hipLaunchKernelGGL(k_batch_finalize, dim3(persistent_grid(ctx, b->fin_n, 256)), dim3(256), 0, s, b->d_inst,
                         b->d_items + b->fin_lo, b->fin_n, b->d_tickets + 2 * tun.size(), b->d_status);
    hip(hipGetLastError(), "batch kernels");
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(s, &g);
    hip(ee, "end capture");
    b->graph = g;
    if (st == REL_OK) hip(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate graph");
  }
  if (st != REL_OK) {
    free_batch(b);
    return st;
  }
  *out = b;
  return REL_OK;
}

rel_status rel_batch_run(rel_batch* b) {
  if (!b) return REL_INVALID_ARG;
  relh::KernelTimer kt(b->ctx, "batch_graph");
  REL_HIP_CHECK(b->ctx, hipGraphLaunch(b->exec, b->ctx->stream));
  return REL_OK;
}

rel_status rel_batch_sync(rel_batch* b, rel_stats* stats) {
  if (!b) return REL_INVALID_ARG;
  rel_ctx* ctx = b->ctx;
  REL_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  uint32_t bits = 0;  // the last run's own status word
  REL_HIP_CHECK(ctx, hipMemcpy(&bits, b->d_status, sizeof bits, hipMemcpyDeviceToHost));
  if (stats && b->k > 0) {
    std::vector<int64_t> h(3 * (size_t)b->k);
    REL_HIP_CHECK(ctx, hipMemcpy(h.data(), b->d_stats, 8 * h.size(), hipMemcpyDeviceToHost));
    std::vector<BInst> hi(b->k);
    REL_HIP_CHECK(ctx, hipMemcpy(hi.data(), b->d_inst, sizeof(BInst) * b->k, hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < b->k; ++i) {
      rel_stats& s = stats[i];
      s.rows_in = hi[i].n;
      s.rows_passed = h[3 * i];
      s.join_matches = h[3 * i + 1];
      s.groups = h[3 * i + 2];
      s.join_capacity = (int64_t)hi[i].jmask + 1;
      s.group_capacity = (int64_t)hi[i].gmask + 1;
      s.join_placement = hi[i].ljoin ? REL_PLACE_LDS : REL_PLACE_GLOBAL;
      s.group_placement = hi[i].lds ? REL_PLACE_LDS : REL_PLACE_GLOBAL;
      s.overflowed = 0;
      s.fell_back = 0;
    }
  }
  if (bits & kDevDupKey) return relh::fail(ctx, REL_DUPLICATE_KEY, "rel_batch_sync: duplicate pk");
  if (bits & kDevOverflow) return relh::fail(ctx, REL_OVERFLOW, "rel_batch_sync: a table or output overflowed");
  return REL_OK;
}

rel_status rel_batch_destroy(rel_batch* b) {
  if (!b) return REL_INVALID_ARG;
  (void)hipStreamSynchronize(b->ctx->stream);
  free_batch(b);
  return REL_OK;
}

}  // extern "C"
