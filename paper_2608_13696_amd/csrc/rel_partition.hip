// Radix-partitioned groupjoin for large build sides (GROUP BY fk with fk = pk).
//
// A device-memory table updated with device-scope atomics costs one atomic
// per aggregate per joined row, and those atomics run at a fixed device-wide
// rate far below what the streaming reads allow. Partitioning both sides by
// the key's hash makes every partition's dim keys fit a workgroup's LDS, so
// the build, the probe and all aggregate updates become LDS operations
// (the paper's Recommendation 2: use the on-chip memories), and device memory
// sees only sequential partition reads and writes.
//
// Passes (each side; fact rows are filtered by the predicate in pass 1):
//   1. histogram of the top B1 bits of each key's position in the key order
//      per input tile; column scan; scatter into 2^B1 partitions (long runs
//      per tile, so writes coalesce);
//   2. per first-level partition, the same on the next B2 bits.
// The key order is a multiplicative hash, or, for GROUP BY fk over dim keys
// that span a narrow enough range, a bijection of that range (KeyMap), which
// turns every unit's table into a direct-mapped one.
// Then one work unit per (partition, or 2^merge consecutive partitions in
// the dense order; chunk of dim keys), ordered by decreasing fact-row count,
// builds an LDS table, streams the unit's fact rows through it, and appends
// its groups to the output with one atomic offset reservation per unit. In
// the dense order the dim side stops after its first level and hands the
// units a presence bitmap over the key positions instead of its keys. The same partitions and units
// serve grouping by a dim attribute: k_part_join_agg (few groups, an LDS
// group table per workgroup) and k_part_join_eager (many groups, partials per
// dim key added to a device-memory table at the end of each unit).
#include "rel_device.h"
#include "rel_host.h"
#include "rel_ops.h"

namespace {

using namespace rel;

constexpr int kBlk = 256;         // histogram and scan kernels
constexpr int kSBlk = 512;        // scatter kernels
// One 4096-row tile per 512-thread workgroup at both levels (68 KB of LDS, two
// workgroups per CU), so one workgroup's loads overlap another's sort and
// stores; tiles this long leave runs per partition long enough that few cache
// lines are written partly.
constexpr int64_t kTile1 = 4096;
constexpr int64_t kTile = 4096;
constexpr int kMaxBins = 256;
constexpr int kJBlock = 256;
constexpr int kJSlotBits = 11;
constexpr int kJSlots = 1 << kJSlotBits;
constexpr int kJChunk = 1400;  // dim keys per unit: LDS load factor <= 0.69
constexpr int kCombineMin = 8; // lanes sharing a slot before a wave pre-sums them

// LDS slot: an independent multiplicative hash, so slot bits do not repeat the partition bits.
__device__ __forceinline__ uint32_t slot_hash(int32_t key) { return ((uint32_t)key * 0x85EBCA6Bu) >> (32 - kJSlotBits); }

// The key order of the partition passes: bin bits are the top bits of
// ((key - sub) * mul) << sh.
//
// Hash order (sub 0, mul = 2^32 / golden ratio, sh 0): the multiplicative hash.
//
// Dense order, for GROUP BY fk when the dim keys span at most 2^(P + 11)
// values (P the partition bits; kmin the smallest dim key, L = max(P,
// ceil(log2(range)))): key -> (key - kmin) * mul mod 2^L with mul odd is a
// bijection of [0, 2^L), so a partition (its top P bits) holds exactly the
// keys whose low L - P = `slot_bits` bits differ, and those bits index a
// direct-mapped LDS table: no hashing, probing or key compares in the
// groupjoin. mul is the golden-ratio fraction of 2^L, so consecutive keys
// (the hot ranks of a Zipf key column) fall in far-apart partitions.
struct KeyMap {
  uint32_t sub, mul, sh;
  uint32_t dense;      // 1: dense order
  uint32_t slot_bits;  // dense: slot bits per partition (<= kJSlotBits)
  uint32_t range;      // dense: kmax - kmin + 1 (fact keys outside it match nothing)
  uint32_t merge;      // dense: log2 of the partitions per groupjoin unit
  uint32_t lbits;      // dense: L, the key positions are [0, 2^L)
  uint32_t inv;        // dense: mul^-1 mod 2^32 (key - kmin = position * inv mod 2^L)
};

__device__ __forceinline__ uint32_t key_hash(uint32_t sub, uint32_t mul, uint32_t sh, int32_t key) {
  return (((uint32_t)key - sub) * mul) << sh;
}

// ---- narrow second-level rows --------------------------------------------------------------------------------------
//
// In the dense order the groupjoin needs of a fact row only its slot in the
// unit (a function of the key), whether the key lies in the dim keys' range,
// its price and its quantity. When the passing rows' prices and quantities
// span few enough values, the second level writes each row as one 64-bit
// word instead of 16 bytes: bits 0-10 the slot, bit 11 in-range, then the
// quantity minus the smallest quantity (qb bits), then the price minus a
// lower bound of the prices (the rest). Sums stay exact: price = bound +
// field, added mod 2^64 like the 64-bit sums themselves. The bounds come from
// 32-bit minima and maxima (cheap to reduce across a wave): of the
// quantities, and of the prices' high words (price >> 32), so the price field
// takes 32 bits plus those of the high words' spread. They are the
// first-level scatter's per-wave values, combined by the second-level scan;
// signed values are kept order-encoded (sign bit flipped) so that unsigned
// atomics order them.
constexpr uint32_t kSignFlip = 0x80000000u;
constexpr int kRngWaves = 8;  // waves of a first-level scatter workgroup
static_assert(kRngWaves == kSBlk / kWave, "one range entry per wave of a first-level scatter workgroup");
constexpr uint32_t kNarrowSlotBits = 11;  // >= kJSlotBits
constexpr uint32_t kNarrowFieldBits = 64 - kNarrowSlotBits - 1;
__device__ __forceinline__ uint32_t order_enc(int32_t v) { return (uint32_t)v ^ kSignFlip; }
__device__ __forceinline__ int32_t order_dec(uint32_t u) { return (int32_t)(u ^ kSignFlip); }
__device__ __forceinline__ uint32_t bits_of(uint64_t x) { return x ? 64u - (uint32_t)__clzll((long long)x) : 0u; }

struct Narrow {
  uint32_t on;      // rows are 64-bit words
  uint32_t qb;      // quantity field bits
  int64_t pmin, qmin;
};
// rng: {min, max} of the order-encoded price high words, then of the
// quantities. Prices lie in [hmin * 2^32, (hmax + 1) * 2^32), a span below
// 2^(32 + bits(hmax - hmin)).
__device__ __forceinline__ Narrow narrow_of(const KeyMap* km, const uint32_t* rng, uint32_t enabled) {
  Narrow n{0u, 0u, 0, 0};
  if (!enabled || !km->dense || rng[0] > rng[1]) return n;
  const int32_t hmin = order_dec(rng[0]), hmax = order_dec(rng[1]);
  n.pmin = (int64_t)hmin * 4294967296ll;
  n.qmin = order_dec(rng[2]);
  const uint32_t pb = 32u + bits_of((uint64_t)((int64_t)hmax - hmin));
  n.qb = bits_of((uint64_t)((int64_t)order_dec(rng[3]) - n.qmin));
  n.on = pb + n.qb <= kNarrowFieldBits;
  return n;
}

// What the second-level scatter needs to write narrow rows.
struct NarrowPack {
  Narrow n;
  uint32_t sub, mul, range, smask;
};
__device__ __forceinline__ NarrowPack narrow_pack(const KeyMap* km, const uint32_t* rng, uint32_t enabled) {
  NarrowPack np{narrow_of(km, rng, enabled), 0u, 0u, 0u, 0u};
  if (np.n.on) {
    np.sub = km->sub;
    np.mul = km->mul;
    np.range = km->range;
    np.smask = (1u << (km->slot_bits + km->merge)) - 1u;
  }
  return np;
}

// Minima (even entries) and maxima (odd entries) of four values over the wave
// (every lane gets them) or over the workgroup (thread 0 gets them); every
// lane or thread must call it.
__device__ __forceinline__ void wave_minmax4(uint32_t (&v)[4]) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t u = (uint32_t)__shfl_xor((int)v[i], o, kWave);
      v[i] = (i & 1) ? max(u, v[i]) : min(u, v[i]);
    }
  }
}
template <int NT>
__device__ __forceinline__ void block_minmax4(uint32_t (&v)[4], uint32_t (*sm)[NT / kWave]) {
  wave_minmax4(v);
  if (lane_id() == 0)
#pragma unroll
    for (int i = 0; i < 4; ++i) sm[i][threadIdx.x / kWave] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < NT / kWave; ++w)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (i & 1) ? max(sm[i][w], v[i]) : min(sm[i][w], v[i]);
}

// Bin of a key at a level: `shift` drops the low bits of the key's position
// in the key order, `mask` keeps the level's bits.
struct BinOf {
  uint32_t sub, mul, sh, shift, mask;
  __device__ BinOf(const KeyMap* km, uint32_t shift_, uint32_t mask_)
      : sub(km->sub), mul(km->mul), sh(km->sh), shift(shift_), mask(mask_) {}
  __device__ uint32_t operator()(int32_t key) const { return (key_hash(sub, mul, sh, key) >> shift) & mask; }
};

// One wave: combines the key min/max pairs of the dim keys (nparts of them;
// none for grouping other than by fk) and writes the key map.
__global__ __launch_bounds__(kWave) void k_keymap(const uint32_t* __restrict__ part, int32_t nparts, uint32_t pbits,
                                                  KeyMap* __restrict__ km) {
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
  if (threadIdx.x != 0) return;
  KeyMap k{0u, 2654435769u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  if (nparts > 0) {
    const int64_t kmin = (int32_t)(~lo ^ 0x80000000u), kmax = (int32_t)(hi ^ 0x80000000u);
    const int64_t range = kmax - kmin + 1;  // >= 1
    uint32_t L = 0;
    while (((int64_t)1 << L) < range) ++L;
    if (L < pbits) L = pbits;
    if (L - pbits <= (uint32_t)kJSlotBits) {
      k.sub = (uint32_t)kmin;
      k.mul = (uint32_t)(2654435769ull >> (32 - L)) | 1u;
      k.sh = 32 - L;
      k.dense = 1;
      k.slot_bits = L - pbits;
      k.range = (uint32_t)range;
      k.merge = min((uint32_t)kJSlotBits - k.slot_bits, pbits);
      k.lbits = L;
      uint32_t x = k.mul;  // Newton's iteration for the inverse of an odd number mod 2^32: 3, 6, 12, 24, 48 bits
      for (int i = 0; i < 4; ++i) x *= 2u - k.mul * x;
      k.inv = x;
    }
  }
  *km = k;
}

struct PartSide {
  // first-level inputs
  const int32_t* key;
  const int32_t* day;      // fact only
  const int64_t* price;    // fact only
  const int32_t* qty;      // fact only
  const int8_t* flag;      // fact only, and only when the group key needs it (else null)
  const void* payload;     // dim only (PayloadKind)
  int pkind;
  int32_t day_lt;
  int64_t n;
  // first-level outputs / second-level inputs
  int32_t* key1;
  int64_t* price1;
  int32_t* qty1;
  int8_t* flag1;
  int32_t* pay1;
  // second-level outputs
  int32_t* key2;
  int64_t* price2;
  int32_t* qty2;
  int8_t* flag2;
  int32_t* pay2;
  // bookkeeping
  uint32_t* hist1;   // [ntiles1][nb1]
  uint32_t* tot1;    // [nb1]
  uint32_t* pass1;   // fact only: bit r of word r / 32 set when row r passes the filter (the histogram writes it)
  uint32_t* rng_part;  // fact only, nullable: per wave of a first-level tile, the passing rows' encoded ranges (narrow_of)
  uint32_t* rng;       // fact only: those ranges over all tiles
  uint32_t narrow;     // fact only: the second level may write narrow rows (GROUP BY fk)
  uint32_t* hist2;   // [max tiles2][nb2]
  uint32_t* pstart;  // [nb1 * nb2]
  uint32_t* pcount;  // [nb1 * nb2]
  uint4* tdesc2;     // [max tiles2] second-level tile: {first-level partition, row lo, row hi, 0}
  int64_t* ntiles2;  // number of second-level tiles
  int64_t* zero2;    // nullable: two int64 counters that the first-level histogram clears
  const KeyMap* km;  // the key order of the bins
  uint32_t dense_stop;  // dim side of GROUP BY fk: in the dense order, no second level (see k_dim_bitmap)
  uint32_t b1, b2;
};

// ---- tile walks -------------------------------------------------------------------------------------------------------
//
// The scatter and second-level kernels are persistent: a fixed grid (a
// multiple of 8) walks the tiles, each workgroup loading its next tile while
// it sorts and writes the current one. XCD x (= blockIdx % 8, the hardware's
// round-robin dispatch) takes the contiguous tile range [x T / 8, (x + 1) T / 8)
// with its workgroups interleaved inside it, so the tiles an XCD holds at one
// time are neighbours: their runs in each partition are adjacent in memory and
// meet in that XCD's L2 before they are written back.
struct TileWalk {
  int64_t next, hi, step;
  __device__ TileWalk(int64_t T) {
    const uint32_t x = blockIdx.x % kNumXcd, i = blockIdx.x / kNumXcd;
    step = gridDim.x / kNumXcd;
    next = T * x / kNumXcd + i;
    hi = T * (x + 1) / kNumXcd;
  }
  __device__ int64_t take() {
    const int64_t t = next < hi ? next : -1;
    next += step;
    return t;
  }
};

// ---- skew-tolerant LDS counters ------------------------------------------------------------------------------------
//
// Under key skew most of a wave's rows can fall in one bin, and atomics of
// many lanes on one LDS address execute one after another. The lanes that
// share the first active lane's bin are therefore served by one atomic when
// there are enough of them; the others use their own.
constexpr int kBinCombineMin = 4;

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// ctr[bin] += 1 for every active lane. Every lane of the wave must call it.
__device__ __forceinline__ void lds_count(uint32_t* ctr, uint32_t bin, bool active) {
  const uint64_t act = wave_ballot(active);
  if (act == 0) return;
  const int leader = __ffsll((long long)act) - 1;
  const uint32_t b0 = readlane_u32(bin, leader);
  const bool mine = active && bin == b0;
  const uint64_t same = wave_ballot(mine);
  const int c = __popcll(same);
  if (c >= kBinCombineMin) {
    if ((int)lane_id() == leader) atomicAdd(&ctr[b0], (uint32_t)c);
    active = active && !mine;
  }
  if (active) atomicAdd(&ctr[bin], 1u);
}

// The same, returning each lane's rank in its bin (the counter's value before
// the lane's own increment; lanes combined by one atomic rank in lane order).
__device__ __forceinline__ uint32_t lds_rank(uint32_t* ctr, uint32_t bin, bool active) {
  const uint64_t act = wave_ballot(active);
  if (act == 0) return 0;
  const int leader = __ffsll((long long)act) - 1;
  const uint32_t b0 = readlane_u32(bin, leader);
  const bool mine = active && bin == b0;
  const uint64_t same = wave_ballot(mine);
  const int c = __popcll(same);
  uint32_t rank = 0;
  if (c >= kBinCombineMin) {
    uint32_t base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(&ctr[b0], (uint32_t)c);
    if (active && !mine) rank = atomicAdd(&ctr[bin], 1u);
    base = readlane_u32(base, leader);
    if (mine) rank = base + mask_rank(same);
  } else if (active) {
    rank = atomicAdd(&ctr[bin], 1u);
  }
  return rank;
}

// ---- first level -------------------------------------------------------------------------------------------------------

template <bool FACT>
__device__ __forceinline__ bool row_passes(const PartSide& s, int64_t r) {
  return !FACT || s.day[r] < s.day_lt;
}

template <bool FACT>
__global__ __launch_bounds__(kBlk) void k_p1_hist(PartSide s) {
  __shared__ uint32_t h[kMaxBins];
  const uint32_t nb1 = 1u << s.b1;
  const BinOf bin_of(s.km, 32u - s.b1, nb1 - 1);
  if (s.zero2 && blockIdx.x == 0 && threadIdx.x == 0) {  // for the kernels that follow
    s.zero2[0] = 0;
    s.zero2[1] = 0;
  }
  if (FACT && s.rng_part && blockIdx.x == 0 && threadIdx.x < 4) s.rng[threadIdx.x] = (threadIdx.x & 1) ? 0u : ~0u;
  for (uint32_t b = threadIdx.x; b < nb1; b += kBlk) h[b] = 0;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t r0 = tile * kTile1;
  const int64_t r1 = r0 + kTile1 < s.n ? r0 + kTile1 : s.n;
  constexpr int V = (int)(kTile1 / (4 * kBlk));  // 16-byte loads per column per thread
  if (r1 - r0 == kTile1) {
    // full tile: every load first, then the counting
    int4 kv[V], dv[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const int64_t r = r0 + 4 * (threadIdx.x + (int64_t)k * kBlk);
      kv[k] = ld_once(reinterpret_cast<const int4*>(s.key + r));
      dv[k] = FACT ? ld_once(reinterpret_cast<const int4*>(s.day + r)) : make_int4(0, 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const int32_t ks[4] = {kv[k].x, kv[k].y, kv[k].z, kv[k].w};
      const int32_t ds[4] = {dv[k].x, dv[k].y, dv[k].z, dv[k].w};
      uint32_t nib = 0;  // this thread's four rows' pass bits
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (!FACT || ds[e] < s.day_lt) {
          atomicAdd(&h[bin_of(ks[e])], 1u);
          nib |= 1u << e;
        }
      if (FACT) {
        // eight consecutive lanes hold the 32 rows of one word
        uint32_t w = nib << (4 * (lane_id() & 7));
        w |= (uint32_t)__shfl_xor((int)w, 1, kWave);
        w |= (uint32_t)__shfl_xor((int)w, 2, kWave);
        w |= (uint32_t)__shfl_xor((int)w, 4, kWave);
        if ((lane_id() & 7) == 0) s.pass1[(r0 + 4 * (threadIdx.x + (int64_t)k * kBlk)) >> 5] = w;
      }
    }
  } else {
    __syncthreads();
    // rows q .. q + 63 of a wave start on a multiple of 64 (tiles are multiples of 256 rows)
    for (int64_t q0 = r0 + (threadIdx.x & ~(kWave - 1)); q0 < r1; q0 += kBlk) {
      const int64_t q = q0 + lane_id();
      const bool pass = q < r1 && row_passes<FACT>(s, q);
      if (pass) atomicAdd(&h[bin_of(s.key[q])], 1u);
      if (FACT) {
        const uint64_t b = wave_ballot(pass);
        if (lane_id() == 0) {
          s.pass1[q0 >> 5] = (uint32_t)b;
          if (q0 + 32 < r1) s.pass1[(q0 >> 5) + 1] = (uint32_t)(b >> 32);
        }
      }
    }
  }
  __syncthreads();
  // bin-major [nb1][ntiles], so that each bin's column scan reads contiguously
  for (uint32_t b = threadIdx.x; b < nb1; b += kBlk) s.hist1[(size_t)b * gridDim.x + tile] = h[b];
}

// Column b of hist1 (one bin over all tiles) -> exclusive prefix in place;
// tot1[b] = column sum; also clears bin b's second-level counters. The column goes through LDS in chunks so that global
// reads and writes are coalesced while each thread scans a contiguous run.
constexpr int kColPer = 16;
__global__ __launch_bounds__(kBlk) void k_p1_colscan(uint32_t* __restrict__ hist1, int64_t ntiles, uint32_t nb1,
                                                     uint32_t* __restrict__ tot1, int64_t* __restrict__ passed,
                                                     uint32_t* __restrict__ pcount, uint32_t nb2) {
  for (uint32_t b = threadIdx.x; b < nb2; b += kBlk) pcount[blockIdx.x * nb2 + b] = 0;  // for k_p2_hist
  __shared__ uint32_t buf[kBlk * kColPer];
  __shared__ uint32_t scr[kBlk / kWave];
  uint32_t* col = hist1 + (size_t)blockIdx.x * ntiles;
  uint32_t carry = 0;
  for (int64_t c0 = 0; c0 < ntiles; c0 += kBlk * kColPer) {
    const int64_t len = ntiles - c0 < kBlk * kColPer ? ntiles - c0 : kBlk * kColPer;
    uint32_t v[kColPer];
#pragma unroll
    for (int k = 0; k < kColPer; ++k) {
      const int64_t j = threadIdx.x + k * kBlk;
      v[k] = j < len ? col[c0 + j] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kColPer; ++k) buf[threadIdx.x + k * kBlk] = v[k];
    __syncthreads();
    uint32_t run[kColPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kColPer; ++k) {
      run[k] = sum;
      sum += buf[threadIdx.x * kColPer + k];
    }
    uint32_t tot;
    const uint32_t off = block_excl_scan<kBlk>(sum, scr, &tot);
#pragma unroll
    for (int k = 0; k < kColPer; ++k) buf[threadIdx.x * kColPer + k] = carry + off + run[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kColPer; ++k) {
      const int64_t j = threadIdx.x + k * kBlk;
      if (j < len) col[c0 + j] = buf[j];
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tot1[blockIdx.x] = carry;
    if (passed) dev_add<unsigned long long>((unsigned long long*)passed, (unsigned long long)carry);
  }
}

// ---- LDS-staged scatter ------------------------------------------------------------------------------------------------
//
// Writing each row straight to its partition from the lane that holds it puts
// 64 lanes' stores on up to 64 different cache lines; partly written lines
// are then evicted and written back several times over. Instead a tile's rows
// are first counting-sorted by partition in LDS, then each partition's run is
// written by consecutive lanes to consecutive addresses.

template <bool FACT, int TILE>
struct Stage {
  uint32_t lcnt[kMaxBins];   // rows per bin in this tile; zero between tiles
  uint32_t lbase[kMaxBins];  // first LDS row of each bin
  uint32_t delta[kMaxBins];  // gbase - lbase (mod 2^32): output position = delta[bin] + LDS row
  uint32_t gbase[kMaxBins];  // this tile's start in each bin's output run
  uint32_t total;            // rows staged in this tile
  uint32_t scr[kSBlk / kWave];
  int2 kv[TILE];             // {key, qty (fact) or payload (dim)}
  int64_t price[FACT ? TILE : 1];
  int8_t flag[FACT ? TILE : 1];  // fact flag (when carried)
};

// The rows one thread holds for one tile. valid: bit k set when row k is in
// range; with PASS (fact rows at the first level) the filter's outcome comes
// from the pass bits that the histogram pass stored (one bit per row read
// instead of the 4-byte day), applied only when the rows are used, so a
// prefetched tile's loads are not waited for early.
template <bool FACT, bool PASS, int R>
struct TileRows {
  int32_t key[R];
  int32_t val[R];
  int64_t price[FACT ? R : 1];
  uint32_t pass[PASS ? R : 1];  // the word of pass bits that holds row k's (bit threadIdx.x % 32)
  uint32_t flags[FACT ? (R + 3) / 4 : 1];  // fact flag bytes, four per word (when carried)
  uint32_t valid;
};


// Sorts the workgroup's rows by bin in LDS and writes each to its bin's output
// run at gbase[bin] + rank within the bin. Three barriers per tile:
//   ranks (LDS atomics) | wave 0 scans the counts and clears them for the next
//   tile | rows move to their LDS rows | written out in LDS order.
// Callers write st.gbase before the call (it is read after the first barrier)
// and clear st.lcnt once before the first tile. No barrier at the end: the
// next tile's first barrier orders its scan after this tile's write-out.
template <bool FACT, bool PASS, int NT, int TILE>
__device__ __forceinline__ void stage_and_write(Stage<FACT, TILE>& st, TileRows<FACT, PASS, TILE / NT>& r,
                                                BinOf bin_of, uint32_t nb, bool with_val, int32_t* dkey,
                                                int64_t* dprice, int32_t* dval, int8_t* dflag, const NarrowPack& np) {
  constexpr int R = TILE / NT;
  if (PASS) {
#pragma unroll
    for (int k = 0; k < R; ++k)
      if (((r.pass[k] >> (threadIdx.x & 31)) & 1u) == 0) r.valid &= ~(1u << k);
  }
  uint32_t rank[R];
#pragma unroll
  for (int k = 0; k < R; ++k) rank[k] = lds_rank(st.lcnt, bin_of(r.key[k]), (r.valid >> k) & 1u);
  __syncthreads();
  if (threadIdx.x < kWave) {
    // wave 0: exclusive scan of the counts, four bins per lane (nb <= 256)
    constexpr int kPerLane = kMaxBins / kWave;
    const uint32_t lane = threadIdx.x;
    uint32_t c[kPerLane], sum = 0;
#pragma unroll
    for (int k = 0; k < kPerLane; ++k) {
      const uint32_t b = lane * kPerLane + k;
      c[k] = b < nb ? st.lcnt[b] : 0u;
      sum += c[k];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o, kWave);
      if (lane >= (uint32_t)o) incl += t;
    }
    uint32_t run = incl - sum;
#pragma unroll
    for (int k = 0; k < kPerLane; ++k) {
      const uint32_t b = lane * kPerLane + k;
      if (b < nb) {
        st.lbase[b] = run;
        st.delta[b] = st.gbase[b] - run;
        st.lcnt[b] = 0;
      }
      run += c[k];
    }
    if (lane == kWave - 1) st.total = incl;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (!((r.valid >> k) & 1u)) continue;
    const uint32_t slot = st.lbase[bin_of(r.key[k])] + rank[k];
    st.kv[slot] = make_int2(r.key[k], r.val[k]);
    if (FACT) st.price[slot] = r.price[k];
    if (FACT && dflag) st.flag[slot] = (int8_t)(r.flags[k / 4] >> (8 * (k % 4)));
  }
  __syncthreads();
  const uint32_t total = st.total;
  for (uint32_t j = threadIdx.x; j < total; j += NT) {
    const int2 kv = st.kv[j];
    const uint32_t pos = st.delta[bin_of(kv.x)] + j;
    if (FACT && np.n.on) {  // one 64-bit word per row, in the price column's place
      const uint32_t off = (uint32_t)kv.x - np.sub;
      const uint64_t w = (uint64_t)((off * np.mul) & np.smask) | ((uint64_t)(off < np.range) << kNarrowSlotBits) |
                         ((uint64_t)((int64_t)kv.y - np.n.qmin) << (kNarrowSlotBits + 1)) |
                         (((uint64_t)(st.price[j] - np.n.pmin) << (kNarrowSlotBits + 1)) << np.n.qb);
      reinterpret_cast<uint64_t*>(dprice)[pos] = w;
      continue;
    }
    dkey[pos] = kv.x;
    if (FACT) {
      dprice[pos] = st.price[j];
      dval[pos] = kv.y;
      if (dflag) dflag[pos] = st.flag[j];
    } else if (with_val) {
      dval[pos] = kv.y;
    }
  }
}

constexpr int kR1 = (int)(kTile1 / kSBlk);  // rows per thread at the first level
using Rows1F = TileRows<true, true, kR1>;

// One row of a first-level tile (q < s.n).
template <bool FACT>
__device__ __forceinline__ void load_p1_row(const PartSide& s, int64_t q, int k, TileRows<FACT, FACT, kR1>& r) {
  r.key[k] = ld_once(s.key + q);
  if (FACT) {
    r.val[k] = ld_once(s.qty + q);
    r.price[k] = ld_once(s.price + q);
    r.pass[k] = s.pass1[q >> 5];  // q % 32 == threadIdx.x % 32
    if (s.flag) r.flags[k / 4] |= (uint32_t)(uint8_t)s.flag[q] << (8 * (k % 4));
  } else {
    r.val[k] = s.pkind == relh::PAY_ROW_ID ? (int32_t)q
             : s.pkind == relh::PAY_I32    ? ((const int32_t*)s.payload)[q]
             : s.pkind == relh::PAY_I8     ? (int32_t)((const int8_t*)s.payload)[q]
                                           : 0;
  }
}

// One first-level tile per workgroup (tiles of one XCD contiguous, xcd_tile).
template <bool FACT>
__global__ __launch_bounds__(kSBlk) void k_p1_scatter(PartSide s) {
  __shared__ Stage<FACT, (int)kTile1> st;
  const uint32_t nb1 = 1u << s.b1;
  const BinOf bin_of(s.km, 32u - s.b1, nb1 - 1);
  const int64_t ntiles = gridDim.x;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  TileRows<FACT, FACT, kR1> r;
  if (FACT)
#pragma unroll
    for (int w = 0; w < (kR1 + 3) / 4; ++w) r.flags[w] = 0;
  const int64_t r0 = (int64_t)tile * kTile1 + threadIdx.x;
  if ((int64_t)tile * kTile1 + kTile1 <= s.n) {  // full tile: unconditional loads, issued back to back
#pragma unroll
    for (int k = 0; k < kR1; ++k) load_p1_row<FACT>(s, r0 + (int64_t)k * kSBlk, k, r);
    r.valid = (1u << kR1) - 1;
  } else {
    r.valid = 0;
#pragma unroll
    for (int k = 0; k < kR1; ++k) {
      const int64_t q = r0 + (int64_t)k * kSBlk;
      if (q < s.n) {
        load_p1_row<FACT>(s, q, k, r);
        r.valid |= 1u << k;
      } else {
        r.key[k] = 0;
        r.val[k] = 0;
        if (FACT) {
          r.price[k] = 0;
          r.pass[k] = 0;
        }
      }
    }
  }
  const uint32_t h = threadIdx.x < nb1 ? s.hist1[(size_t)threadIdx.x * ntiles + tile] : 0u;
  // partition starts: exclusive scan of the bin totals (nb1 <= kSBlk)
  uint32_t tot;
  const uint32_t pbase = block_excl_scan<kSBlk>(threadIdx.x < nb1 ? s.tot1[threadIdx.x] : 0u, st.scr, &tot);
  if (threadIdx.x < kMaxBins) st.lcnt[threadIdx.x] = 0;
  if (threadIdx.x < nb1) st.gbase[threadIdx.x] = pbase + h;
  // the tile's passing rows: ranges of price and quantity (narrow second-level
  // rows), per thread here, per wave after the write-out
  int32_t pmn = INT32_MAX, pmx = INT32_MIN, qmn = INT32_MAX, qmx = INT32_MIN;  // price high words, quantities
  if constexpr (FACT) {
    if (s.rng_part) {
#pragma unroll
      for (int k = 0; k < kR1; ++k)
        if (((r.valid >> k) & 1u) && ((r.pass[k] >> (threadIdx.x & 31)) & 1u)) {
          const int32_t ph = (int32_t)(r.price[k] >> 32);
          pmn = min(pmn, ph);
          pmx = max(pmx, ph);
          qmn = min(qmn, r.val[k]);
          qmx = max(qmx, r.val[k]);
        }
    }
  }
  __syncthreads();
  stage_and_write<FACT, FACT, kSBlk, (int)kTile1>(st, r, bin_of, nb1, s.pkind != relh::PAY_NONE, s.key1,
                                                  s.price1, FACT ? s.qty1 : s.pay1, FACT ? s.flag1 : nullptr,
                                                  NarrowPack{});
  if constexpr (FACT) {
    if (s.rng_part) {
      uint32_t v[4] = {order_enc(pmn), order_enc(pmx), order_enc(qmn), order_enc(qmx)};
      wave_minmax4(v);
      if (lane_id() == 0)
        reinterpret_cast<uint4*>(s.rng_part)[(size_t)tile * kRngWaves + threadIdx.x / kWave] = make_uint4(v[0], v[1], v[2], v[3]);
    }
  }
}

// ---- second level ------------------------------------------------------------------------------------------------------
//
// Second-level tiles cut each first-level partition into kTile-row pieces;
// tile ids run over the partitions in order. Every workgroup derives the tile
// table from the first-level totals once, in LDS.

struct L2Map {
  uint32_t start[kMaxBins];  // first row of partition p in the first-level arrays
  uint32_t cnt[kMaxBins];    // rows of partition p
  uint32_t tbase[kMaxBins];  // first tile id of partition p
  uint32_t ntiles;           // tiles over all partitions
};

template <int NT>
__device__ void build_l2map(const PartSide& s, L2Map& mp, uint32_t* scr) {
  const uint32_t nb1 = 1u << s.b1;
  const uint32_t c = threadIdx.x < nb1 ? s.tot1[threadIdx.x] : 0u;
  const uint32_t nt = (uint32_t)((c + kTile - 1) / kTile);
  uint32_t tot, ntot;
  const uint32_t start = block_excl_scan<NT>(c, scr, &tot);
  const uint32_t tb = block_excl_scan<NT>(nt, scr, &ntot);
  if (threadIdx.x < nb1) {
    mp.start[threadIdx.x] = start;
    mp.cnt[threadIdx.x] = c;
    mp.tbase[threadIdx.x] = tb;
  }
  if (threadIdx.x == 0) mp.ntiles = ntot;
  __syncthreads();
}

struct Tile2 {
  uint32_t p;
  int64_t lo, hi;  // rows [lo, hi) of the first-level arrays
};

// The partition holding tile t: the last p with tbase[p] <= t (partitions
// without tiles share their successor's tbase, so the last one is never empty).
__device__ __forceinline__ Tile2 find_tile(const L2Map& mp, uint32_t nb1, int64_t t) {
  uint32_t lo = 0, hi = nb1 - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    if ((int64_t)mp.tbase[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  Tile2 r;
  r.p = lo;
  r.lo = (int64_t)mp.start[lo] + (t - (int64_t)mp.tbase[lo]) * kTile;
  const int64_t end = (int64_t)mp.start[lo] + mp.cnt[lo];
  r.hi = r.lo + kTile < end ? r.lo + kTile : end;
  return r;
}

// Per second-level tile: histogram of the next b2 hash bits. Persistent.
//
// A tile's start inside each bin's run of its partition is the prefix of the
// counts of the partition's earlier tiles (k_p2_scan). That keeps the runs of
// neighbouring tiles, which neighbouring workgroups of one XCD scatter at the
// same time, adjacent in memory, so the cache lines they share are completed
// in that XCD's L2. A scan over a partition's tiles is sequential, though: for
// a partition of more than kScanTilesMax tiles (key skew) the tiles instead
// take their starts with device atomics on the bin counters (pcount, zeroed
// by k_p1_colscan) in the order they get there.
constexpr int kHR = (int)(kTile / kBlk);
constexpr uint32_t kScanTilesMax = 128;
__global__ __launch_bounds__(kBlk) void k_p2_hist(PartSide s) {
  if (s.dense_stop && s.km->dense) return;
  __shared__ L2Map mp;
  __shared__ uint32_t scr[kBlk / kWave];
  __shared__ uint32_t h[kMaxBins];
  build_l2map<kBlk>(s, mp, scr);
  const uint32_t nb1 = 1u << s.b1, nb2 = 1u << s.b2;
  const BinOf bin_of(s.km, 32u - s.b1 - s.b2, nb2 - 1);
  TileWalk w(mp.ntiles);
  int64_t t = w.take();
  int32_t cur[kHR], nxt[kHR];
  Tile2 tc{}, tn2{};
  auto load = [&](const Tile2& x, int32_t(&keys)[kHR]) {
#pragma unroll
    for (int k = 0; k < kHR; ++k) {
      const int64_t q = x.lo + threadIdx.x + (int64_t)k * kBlk;
      keys[k] = q < x.hi ? s.key1[q] : 0;
    }
  };
  if (t >= 0) {
    tc = find_tile(mp, nb1, t);
    load(tc, cur);
  }
  while (t >= 0) {
    const int64_t tn = w.take();
    if (tn >= 0) {
      tn2 = find_tile(mp, nb1, tn);
      load(tn2, nxt);
    }
    for (uint32_t b = threadIdx.x; b < nb2; b += kBlk) h[b] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kHR; ++k) lds_count(h, bin_of(cur[k]), tc.lo + threadIdx.x + (int64_t)k * kBlk < tc.hi);
    __syncthreads();
    if ((mp.cnt[tc.p] + kTile - 1) / kTile > kScanTilesMax) {
      // a long partition: the tile's start inside each bin's run, taken in the
      // order the counts arrive (rows of a partition need no particular order)
      for (uint32_t b = threadIdx.x; b < nb2; b += kBlk) {
        const uint32_t c = h[b];
        s.hist2[(size_t)t * nb2 + b] = c ? dev_add_ret<uint32_t>(&s.pcount[tc.p * nb2 + b], c) : 0u;
      }
    } else {
      for (uint32_t b = threadIdx.x; b < nb2; b += kBlk) s.hist2[(size_t)t * nb2 + b] = h[b];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kHR; ++k) cur[k] = nxt[k];
    tc = tn2;
    t = tn;
  }
}

// One workgroup per first-level partition p: per second-level bin, prefix over
// p's tiles (in place; unless k_p2_hist placed them) and the partition
// starts and counts; then p's entries of the tile table.
constexpr int kScanBatch = 8;
__global__ __launch_bounds__(kBlk) void k_p2_scan(PartSide s) {
  if (s.dense_stop && s.km->dense) return;
  __shared__ L2Map mp;
  __shared__ uint32_t scr[kBlk / kWave];
  build_l2map<kBlk>(s, mp, scr);
  const uint32_t nb2 = 1u << s.b2;
  const uint32_t p = blockIdx.x;
  const uint32_t tb = mp.tbase[p], nt = (uint32_t)((mp.cnt[p] + kTile - 1) / kTile);
  uint32_t bin_tot = 0;
  if (threadIdx.x < nb2) {
    if (nt > kScanTilesMax) {
      bin_tot = s.pcount[p * nb2 + threadIdx.x];
    } else {
      for (uint32_t k0 = 0; k0 < nt; k0 += kScanBatch) {
        uint32_t v[kScanBatch];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k)
          v[k] = k0 + k < nt ? s.hist2[(size_t)(tb + k0 + k) * nb2 + threadIdx.x] : 0u;
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
          if (k0 + k < nt) s.hist2[(size_t)(tb + k0 + k) * nb2 + threadIdx.x] = bin_tot;
          bin_tot += v[k];
        }
      }
    }
  }
  uint32_t tot;
  const uint32_t ex = block_excl_scan<kBlk>(threadIdx.x < nb2 ? bin_tot : 0u, scr, &tot);
  if (threadIdx.x < nb2) {
    s.pstart[p * nb2 + threadIdx.x] = mp.start[p] + ex;
    s.pcount[p * nb2 + threadIdx.x] = bin_tot;
  }
  // the scatter's tile table: this partition's tiles, and (once) their total
  for (uint32_t k = threadIdx.x; k < nt; k += kBlk) {
    const uint32_t lo = mp.start[p] + k * (uint32_t)kTile;
    const uint32_t end = mp.start[p] + mp.cnt[p];
    s.tdesc2[tb + k] = make_uint4(p, lo, lo + (uint32_t)kTile < end ? lo + (uint32_t)kTile : end, 0u);
  }
  if (p == 0 && threadIdx.x == 0) *s.ntiles2 = mp.ntiles;
  if (s.rng_part) {
    // the first-level tiles' ranges, workgroup p taking a 1 / gridDim share
    __shared__ uint32_t s_rng[4][kBlk / kWave];
    const int64_t T = (s.n + kTile1 - 1) / kTile1 * kRngWaves;  // one entry per wave of each first-level tile
    uint32_t v[4] = {~0u, 0u, ~0u, 0u};
    for (int64_t t = T * p / gridDim.x + threadIdx.x; t < T * (p + 1) / gridDim.x; t += kBlk) {
      const uint4 u = reinterpret_cast<const uint4*>(s.rng_part)[t];
      v[0] = min(v[0], u.x);
      v[1] = max(v[1], u.y);
      v[2] = min(v[2], u.z);
      v[3] = max(v[3], u.w);
    }
    block_minmax4<kBlk>(v, s_rng);
    if (threadIdx.x == 0 && v[0] <= v[1]) {
      atomicMin(&s.rng[0], v[0]);
      atomicMax(&s.rng[1], v[1]);
      atomicMin(&s.rng[2], v[2]);
      atomicMax(&s.rng[3], v[3]);
    }
  }
}

constexpr int kR2 = (int)(kTile / kSBlk);  // rows per thread at the second level

template <bool FACT>
__device__ __forceinline__ void load_p2(const PartSide& s, const Tile2& x, bool pay, TileRows<FACT, false, kR2>& r) {
  const int64_t r0 = x.lo + threadIdx.x;
  if (FACT)
#pragma unroll
    for (int w = 0; w < (kR2 + 3) / 4; ++w) r.flags[w] = 0;
  if (x.lo + kTile <= x.hi) {  // full tile: unconditional loads, issued back to back
#pragma unroll
    for (int k = 0; k < kR2; ++k) {
      const int64_t q = r0 + (int64_t)k * kSBlk;
      r.key[k] = ld_once(s.key1 + q);
      if (FACT) r.price[k] = ld_once(s.price1 + q);
      r.val[k] = FACT ? ld_once(s.qty1 + q) : pay ? ld_once(s.pay1 + q) : 0;
      if (FACT && s.flag1) r.flags[k / 4] |= (uint32_t)(uint8_t)s.flag1[q] << (8 * (k % 4));
    }
    r.valid = (1u << kR2) - 1;
  } else {
    r.valid = 0;
#pragma unroll
    for (int k = 0; k < kR2; ++k) {
      const int64_t q = r0 + (int64_t)k * kSBlk;
      const bool in = q < x.hi;
      r.key[k] = in ? s.key1[q] : 0;
      if (FACT) r.price[k] = in ? s.price1[q] : 0;
      r.val[k] = !in ? 0 : FACT ? s.qty1[q] : pay ? s.pay1[q] : 0;
      if (FACT && s.flag1 && in) r.flags[k / 4] |= (uint32_t)(uint8_t)s.flag1[q] << (8 * (k % 4));
      r.valid |= (uint32_t)in << k;
    }
  }
}

// One second-level tile per workgroup, from the tile table; the grid is an
// upper bound and the surplus workgroups leave at once. Workgroup b takes tile
// xcd_tile(b, tiles), so each XCD holds a contiguous range of tiles.
template <bool FACT>
__global__ __launch_bounds__(kSBlk) void k_p2_scatter(PartSide s) {
  if (s.dense_stop && s.km->dense) return;
  __shared__ Stage<FACT, (int)kTile> st;
  const int64_t ntiles = *s.ntiles2;
  if ((int64_t)blockIdx.x >= ntiles) return;
  const uint32_t t = xcd_tile(blockIdx.x, (uint32_t)ntiles);
  const uint4 td = s.tdesc2[t];
  const uint32_t nb2 = 1u << s.b2;
  const BinOf bin_of(s.km, 32u - s.b1 - s.b2, nb2 - 1);
  const bool pay = !FACT && s.pkind != relh::PAY_NONE;
  Tile2 x;
  x.p = td.x;
  x.lo = td.y;
  x.hi = td.z;
  TileRows<FACT, false, kR2> r;
  load_p2<FACT>(s, x, pay, r);
  if (threadIdx.x < kMaxBins) st.lcnt[threadIdx.x] = 0;
  if (threadIdx.x < nb2) st.gbase[threadIdx.x] = s.pstart[x.p * nb2 + threadIdx.x] + s.hist2[(size_t)t * nb2 + threadIdx.x];
  __syncthreads();
  const NarrowPack np = FACT ? narrow_pack(s.km, s.rng, s.narrow) : NarrowPack{};
  stage_and_write<FACT, false, kSBlk, (int)kTile>(st, r, bin_of, nb2, pay, s.key2, s.price2, FACT ? s.qty2 : s.pay2,
                                                  FACT ? s.flag2 : nullptr, np);
}

// ---- dense order: the dim side's presence bitmap ---------------------------------------------------------------------
//
// In the dense order a groupjoin unit is a range of key positions, and all it
// needs from the dim side is which positions hold a dim key. One workgroup per
// first-level partition sets those bits in LDS (a bit already set is a
// repeated key) and stores the partition's words of a bitmap over all 2^L
// positions; the dim side stops after its first level. With fewer than 32
// positions per partition, one workgroup builds the whole (small) bitmap.
constexpr int kBmBlock = 1024;
constexpr int kBmRows = 8;  // keys per thread per step
__global__ __launch_bounds__(kBmBlock) void k_dim_bitmap(PartSide s, uint32_t* __restrict__ bitmap,
                                                         uint32_t* __restrict__ status) {
  HIP_DYNAMIC_SHARED(uint32_t, lb)
  __shared__ uint32_t s_red[kBmBlock / kWave];
  if (!s.km->dense) return;
  const uint32_t sub = s.km->sub, mul = s.km->mul, L = s.km->lbits;
  const uint32_t lmask = L >= 32 ? ~0u : (1u << L) - 1u;
  const uint32_t pbw = L - s.b1;  // position bits inside a first-level partition
  const uint32_t tid = threadIdx.x;
  if (pbw < 5) {
    if (blockIdx.x != 0) return;
    const uint32_t nw = ((1u << L) + 31) / 32;
    for (uint32_t w = tid; w < nw; w += kBmBlock) lb[w] = 0u;
    __syncthreads();
    for (int64_t j = tid; j < s.n; j += kBmBlock) {
      const uint32_t kp = (((uint32_t)s.key1[j] - sub) * mul) & lmask, bit = 1u << (kp & 31);
      if (atomicOr(&lb[kp >> 5], bit) & bit) set_status(status, kDevDupKey);
    }
    __syncthreads();
    for (uint32_t w = tid; w < nw; w += kBmBlock) bitmap[w] = lb[w];
    return;
  }
  const uint32_t p = blockIdx.x, nw = 1u << (pbw - 5), pmask = (1u << pbw) - 1u;
  for (uint32_t w = tid; w < nw; w += kBmBlock) lb[w] = 0u;
  // the partition's first row: the totals of the partitions before it (nb1 <= kBmBlock)
  uint32_t before = tid < p ? s.tot1[tid] : 0u;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) before += (uint32_t)__shfl_xor((int)before, o, kWave);
  if (lane_id() == 0) s_red[tid / kWave] = before;
  __syncthreads();
  uint32_t start = 0;
#pragma unroll
  for (int w = 0; w < kBmBlock / kWave; ++w) start += s_red[w];
  const uint32_t cnt = s.tot1[p];
  const int32_t* const keys = s.key1 + start;
  for (uint32_t j0 = tid; j0 < cnt; j0 += kBmBlock * kBmRows) {  // kBmRows keys in flight per thread
    int32_t kv[kBmRows];
#pragma unroll
    for (int r = 0; r < kBmRows; ++r) {
      const uint32_t j = j0 + r * kBmBlock;
      kv[r] = j < cnt ? keys[j] : 0;
    }
#pragma unroll
    for (int r = 0; r < kBmRows; ++r) {
      if (j0 + r * kBmBlock >= cnt) break;
      const uint32_t kp = (((uint32_t)kv[r] - sub) * mul) & pmask, bit = 1u << (kp & 31);
      if (atomicOr(&lb[kp >> 5], bit) & bit) set_status(status, kDevDupKey);
    }
  }
  __syncthreads();
  for (uint32_t w = tid; w < nw; w += kBmBlock) bitmap[(size_t)p * nw + w] = lb[w];
}

// ---- work units -----------------------------------------------------------------------------------------------------------
//
// A unit is (partition, chunk of at most kJChunk dim keys, range of the
// partition's fact rows). Units are ordered by decreasing size class of their
// fact-row count, largest first, so long units start early.
//
// Key skew (Zipf) concentrates fact rows in the few partitions that hold the
// hottest keys; one workgroup streaming such a partition alone would set the
// kernel's length. A single-chunk partition with more than max(kSplitMin,
// 4 x the mean) fact rows is therefore split into sub-units of kSubRows fact
// rows. Each sub-unit builds the same LDS table, adds its partial sums into a
// per-chunk device accumulator, and the sub-unit that finishes last emits the
// chunk's groups from it (and clears it for the next call).

constexpr uint32_t kSubRows = 8192;
constexpr uint32_t kSplitMin = 3 * kSubRows / 2;
constexpr uint32_t kMaxSplit = 256;  // split chunks per call (more are processed whole)
constexpr uint32_t kNoSplit = ~0u;

struct SplitAcc {
  uint64_t sp, sq, cnt;
};

__device__ __forceinline__ uint32_t size_class(uint32_t rows) { return 32 - __clz(rows); }

// Adds v to ctr[key] for every active lane with one LDS atomic per distinct
// key in the wave, and returns each lane's exclusive position in what its key
// received (the old value plus the v of lower lanes with the same key). Every
// lane of the wave must call it.
__device__ __forceinline__ uint32_t wave_grouped_add(uint32_t* ctr, uint32_t key, uint32_t v, bool active) {
  const uint32_t lane = lane_id();
  uint32_t result = 0;
  uint64_t todo = wave_ballot(active);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const uint32_t k = __shfl(key, leader, kWave);
    const bool mine = active && key == k;
    const uint32_t x = mine ? v : 0u;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o, kWave);
      if (lane >= (uint32_t)o) incl += t;
    }
    const uint32_t total = __shfl(incl, kWave - 1, kWave);
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(&ctr[k], total);
    base = __shfl(base, leader, kWave);
    if (mine) result = base + incl - x;
    todo &= ~wave_ballot(mine);
  }
  return result;
}

// Unit lists in two kernels of one thread per partition. k_unit_count:
// decides the splits and counts units per size class in each workgroup.
// k_unit_emit: every workgroup derives its own start in each class from
// those counts (classes in descending order, workgroups in order) and writes
// its units. desc[u] = {dlo, dhi, flo, fhi}; split[u] = {split id + 1,
// sub-units of the chunk} for a sub-unit of a split chunk, {0, end of the
// partition's dim keys} for a whole chunk.
constexpr int kUBlk = 256;
constexpr int kClasses = 33;
constexpr int kMaxUnitWgs = (1 << 16) / kUBlk;  // partitions never exceed 2^16

struct UnitArgs {
  const uint32_t* dstart;
  const uint32_t* dcount;
  const uint32_t* fstart;
  const uint32_t* fcount;
  uint32_t nparts;
  const int64_t* rows_passed;  // fact rows that passed the predicate (all partitions)
  uint32_t* split_ctr;         // split ids handed out; zero between calls
  uint32_t* sbase;             // [nparts] split id or kNoSplit
  uint32_t* wg_cls;            // [workgroups][kClasses]
  uint4* desc;
  uint2* split;
  int64_t* n_units;
  int64_t* ticket;  // the join kernel's unit ticket: zeroed here
  int64_t* out_n;   // nullable: the output group count, zeroed here
  const KeyMap* km;
};

// A unit covers 2^merge consecutive partitions. In the dense key order their
// key ranges are consecutive, so together they index one direct-mapped table
// of 2^(slot_bits + merge) <= kJSlots slots, and the unit reads its dim side
// from the presence bitmap (one chunk, whatever the dim keys). Hash order: one
// partition, at most kJChunk keys per chunk (table load <= 0.69).
struct UnitShape {
  uint32_t merge, chunk;
};
__device__ __forceinline__ UnitShape unit_shape(const KeyMap* km) {
  return km->dense ? UnitShape{km->merge, (uint32_t)kJSlots} : UnitShape{0u, (uint32_t)kJChunk};
}

struct UnitGroup {
  uint32_t fc, dc, fs, ds;  // fact rows, dim keys and their first positions
};
// Dense order: the dim side has no second level, so a unit's dim "range" is
// its own index (the groupjoin reads the unit's positions from the presence
// bitmap) and every unit with fact rows is live.
__device__ __forceinline__ UnitGroup unit_group(const UnitArgs& a, uint32_t q, uint32_t merge, bool dense) {
  const uint32_t p0 = q << merge, p1 = p0 + (1u << merge);
  UnitGroup g{0u, dense ? 1u : 0u, a.fstart[p0], dense ? q : a.dstart[p0]};
  for (uint32_t p = p0; p < p1; ++p) {
    g.fc += a.fcount[p];
    if (!dense) g.dc += a.dcount[p];
  }
  return g;
}

__global__ __launch_bounds__(kUBlk) void k_unit_count(UnitArgs a) {
  __shared__ uint32_t cls_n[kClasses];
  if (threadIdx.x < kClasses) cls_n[threadIdx.x] = 0;
  __syncthreads();
  const UnitShape us = unit_shape(a.km);
  const uint32_t ngroups = a.nparts >> us.merge;
  const uint32_t q = blockIdx.x * kUBlk + threadIdx.x;
  const UnitGroup g = q < ngroups ? unit_group(a, q, us.merge, a.km->dense != 0) : UnitGroup{0u, 0u, 0u, 0u};
  const uint32_t fc = g.fc, dc = g.dc;
  const uint64_t mean4 = 4 * (uint64_t)*a.rows_passed / ngroups;
  const uint32_t thr = mean4 > kSplitMin ? (uint32_t)(mean4 < 0xffffffffull ? mean4 : 0xffffffffull) : kSplitMin;
  const bool live = fc != 0 && dc != 0;
  uint32_t sb = kNoSplit, units = 0, cls = 0;
  if (live) {
    const uint32_t chunks = (dc + us.chunk - 1) / us.chunk;
    uint32_t nsub = 1;
    if (chunks == 1 && fc > thr) {
      const uint32_t id = dev_add_ret<uint32_t>(a.split_ctr, 1u);
      if (id < kMaxSplit) {
        sb = id;
        nsub = (fc + kSubRows - 1) / kSubRows;
      }
    }
    units = chunks * nsub;
    cls = size_class(nsub > 1 ? kSubRows : fc);
  }
  wave_grouped_add(cls_n, cls, units, live);
  if (q < ngroups) a.sbase[q] = sb;
  __syncthreads();
  if (threadIdx.x < kClasses) a.wg_cls[blockIdx.x * kClasses + threadIdx.x] = cls_n[threadIdx.x];
}

__global__ __launch_bounds__(kUBlk) void k_unit_emit(UnitArgs a) {
  __shared__ uint32_t tab[kMaxUnitWgs * kClasses];
  __shared__ uint32_t tot[kClasses];
  __shared__ uint32_t bef[kClasses];
  __shared__ uint32_t cur[kClasses];
  const uint32_t nwg = gridDim.x;
  for (uint32_t i = threadIdx.x; i < nwg * kClasses; i += kUBlk) tab[i] = a.wg_cls[i];  // coalesced, all in flight
  __syncthreads();
  if (threadIdx.x < kClasses) {
    uint32_t before = 0, total = 0;
    for (uint32_t w = 0; w < nwg; ++w) {
      const uint32_t v = tab[w * kClasses + threadIdx.x];
      before += w < blockIdx.x ? v : 0u;
      total += v;
    }
    tot[threadIdx.x] = total;
    bef[threadIdx.x] = before;
  }
  __syncthreads();
  if (threadIdx.x < kClasses) {
    uint32_t start = 0;  // classes in descending order: class c follows every larger class
    for (int c = kClasses - 1; c > (int)threadIdx.x; --c) start += tot[c];
    cur[threadIdx.x] = start + bef[threadIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *a.n_units = (int64_t)start + tot[0];
      *a.split_ctr = 0;  // k_unit_count has finished with it: clear it for the next call
      *a.ticket = 0;     // counters the join kernel that follows starts from
      if (a.out_n) *a.out_n = 0;
    }
  }
  __syncthreads();
  const UnitShape us = unit_shape(a.km);
  const uint32_t q = blockIdx.x * kUBlk + threadIdx.x;
  const bool in = q < (a.nparts >> us.merge);
  const UnitGroup g = in ? unit_group(a, q, us.merge, a.km->dense != 0) : UnitGroup{0u, 0u, 0u, 0u};
  const uint32_t fc = g.fc, dc = g.dc, ds = g.ds, fs = g.fs, sb = in ? a.sbase[q] : kNoSplit;
  const bool live = fc != 0 && dc != 0;
  const bool splitp = sb != kNoSplit;
  const uint32_t chunks = (dc + us.chunk - 1) / us.chunk;
  const uint32_t nsub = splitp ? (fc + kSubRows - 1) / kSubRows : 1u;
  const uint32_t cls = size_class(splitp ? kSubRows : fc);
  const uint32_t pos = wave_grouped_add(cur, cls, live ? chunks * nsub : 0u, live);
  // A split partition can have hundreds of sub-units: the wave writes each
  // such partition's list together.
  const uint32_t lane = lane_id();
  for (uint64_t todo = wave_ballot(live && splitp); todo != 0; todo &= todo - 1) {
    const int l = __ffsll((long long)todo) - 1;
    const uint32_t lfs = readlane_u32(fs, l), lend = lfs + readlane_u32(fc, l);
    const uint32_t lds = readlane_u32(ds, l), lde = lds + readlane_u32(dc, l);
    const uint32_t lpos = readlane_u32(pos, l), lns = readlane_u32(nsub, l), lsb = readlane_u32(sb, l);
    for (uint32_t j = lane; j < lns; j += kWave) {
      const uint32_t flo = lfs + j * kSubRows;
      a.desc[lpos + j] = make_uint4(lds, lde, flo, flo + kSubRows < lend ? flo + kSubRows : lend);
      a.split[lpos + j] = make_uint2(lsb + 1, lns);
    }
  }
  if (!live || splitp) return;
  for (uint32_t c = 0; c < chunks; ++c) {
    const uint32_t dlo = ds + c * us.chunk;
    a.desc[pos + c] = make_uint4(dlo, dlo + us.chunk < ds + dc ? dlo + us.chunk : ds + dc, fs, fs + fc);
    a.split[pos + c] = make_uint2(0, ds + dc);
  }
}

// ---- partitioned groupjoin -------------------------------------------------------------------------------------------

struct JoinArgs {
  const uint4* unit_desc;
  const uint2* unit_split;
  const int64_t* n_units;
  const int32_t* dkey;
  const int32_t* fkey;
  const int64_t* fprice;
  const int32_t* fqty;
  SplitAcc* split_acc;    // [kMaxSplit][kJSlots], zero between calls
  uint32_t* split_done;   // [kMaxSplit], zero between calls
  int64_t* ticket;
  int64_t* matched;
  uint32_t* status;
  int64_t* out_key;
  int64_t* out_sp;
  int64_t* out_sq;
  int64_t* out_cnt;
  int64_t out_cap;
  int64_t* d_n;
  const KeyMap* km;
  const uint32_t* bitmap;  // dense order: the dim keys' presence bits over all key positions
  uint32_t zero;  // 0 at run time; see take_ticket
  const uint32_t* rng;    // the fact rows' price and quantity ranges (narrow_of)
  uint32_t narrow;        // narrow rows allowed
  const uint64_t* fpack;  // narrow rows (in the second-level price column's place)
};

constexpr uint64_t kLdsEmpty = ~0ull;
constexpr int kJR = 4;                                   // fact rows per thread per step (dim-attribute kernels)
constexpr int kGR = 4;                                   // fact rows per thread per step (groupjoin)
constexpr int kJDK = (kJChunk + kJBlock - 1) / kJBlock;  // dim keys per thread
constexpr int kJPer = kJSlots / kJBlock;                 // LDS slots per thread at emission

// An offset of zero that the compiler cannot prove uniform (zero is a
// run-time 0), for the address of an atomic issued by one thread: a
// uniform-address atomic would be rewritten into a wave-wide one whose result
// is broadcast at once, stalling the wave on the round trip; this way the wave
// waits only where the result is used.
// The offset is rebuilt at each call (the empty asm keeps the compiler from
// hoisting it out of the unit loop): a loop-invariant address would hold two
// registers for the whole loop, and when spilled its reload waits for every
// memory operation in flight.
__device__ __forceinline__ uint32_t unhoisted_zero_offset(uint32_t zero) {
  uint32_t z = zero;
  asm volatile("" : "+v"(z));
  return threadIdx.x * z;
}

// Workgroup b takes units b, b + G, b + 2G, ... (G workgroups). The list is
// ordered largest first, so each workgroup's share mixes the size classes
// alike. (Units by atomic ticket would balance the tail better, but every
// ticket is an atomic on one cache line, and atomics on one line serialise on
// this chip at about 12 ns each: tens of thousands of units per launch make
// that line a bottleneck.)
__device__ __forceinline__ int64_t take_ticket(const JoinArgs& a, int64_t& seq) {
  (void)a;
  seq += gridDim.x;
  return seq;
}

// The groupjoin's fact rows of one step (kGR per thread, kGR * kJBlock per
// workgroup): keys, and the prices and quantities that the updates use.
struct KeyRegs {
  int32_t key[kGR];
};
struct PayRegs {
  int32_t qty[kGR];
  uint64_t sp[kGR];
};

// Row indices are clamped into the (never empty) range [.., fhi): the loads
// carry no branch, so their number is fixed; lanes past the range hold copies
// that the probe skips.
__device__ __forceinline__ void load_keys(const JoinArgs& a, uint32_t i0, uint32_t fhi, KeyRegs& r) {
#pragma unroll
  for (int k = 0; k < kGR; ++k) {
    const uint32_t i = i0 + k * kJBlock;
    r.key[k] = a.fkey[i < fhi ? i : fhi - 1];
  }
}

// Narrow rows: one 64-bit word per row (in r.sp).
__device__ __forceinline__ void load_packed(const JoinArgs& a, uint32_t i0, uint32_t fhi, PayRegs& r) {
#pragma unroll
  for (int k = 0; k < kGR; ++k) {
    const uint32_t i = i0 + k * kJBlock;
    r.sp[k] = a.fpack[i < fhi ? i : fhi - 1];
  }
}

__device__ __forceinline__ void load_payload(const JoinArgs& a, uint32_t i0, uint32_t fhi, PayRegs& r) {
#pragma unroll
  for (int k = 0; k < kGR; ++k) {
    uint32_t i = i0 + k * kJBlock;
    i = i < fhi ? i : fhi - 1;
    r.sp[k] = (uint64_t)a.fprice[i];
    r.qty[k] = a.fqty[i];
  }
}

// The next unit's dim keys and its first step of fact rows (keys, prices and
// quantities), loaded while the current unit emits its groups.
__device__ __forceinline__ void prefetch_unit(const JoinArgs& a, uint4 u, int32_t (&dk)[kJDK], KeyRegs& r, PayRegs& p) {
#pragma unroll
  for (int k = 0; k < kJDK; ++k) {
    const uint32_t j = u.x + threadIdx.x + k * kJBlock;
    dk[k] = a.dkey[j < u.y ? j : u.y - 1];
  }
  load_keys(a, u.z + threadIdx.x, u.w, r);
  load_payload(a, u.z + threadIdx.x, u.w, p);
}

// Output room for `total` groups. The address is not provably uniform (see
// unhoisted_zero_offset), so the wave waits for the result only where it is
// used.
__device__ __forceinline__ int64_t reserve_nowait(const JoinArgs& a, uint32_t total) {
  unsigned long long* p = (unsigned long long*)a.d_n + unhoisted_zero_offset(a.zero);
  return (int64_t)__hip_atomic_fetch_add(p, (unsigned long long)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reserve room for `mine` groups of this thread (block-wide scan, one atomic
// per call) and return this thread's first output row.
__device__ __forceinline__ int64_t reserve_out(const JoinArgs& a, uint32_t mine, uint32_t* scr, uint64_t* s_excl) {
  uint32_t total;
  const uint32_t off = block_excl_scan<kJBlock>(mine, scr, &total);
  if (threadIdx.x == 0)
    *s_excl = total ? dev_add_ret<unsigned long long>((unsigned long long*)a.d_n, (unsigned long long)total) : 0;
  __syncthreads();
  return (int64_t)*s_excl + off;
}

__device__ __forceinline__ void put_group(const JoinArgs& a, int64_t o, int64_t key, uint64_t sp, uint64_t sq, uint64_t c) {
  if (o < a.out_cap) {
    a.out_key[o] = key;
    a.out_sp[o] = (int64_t)sp;
    a.out_sq[o] = (int64_t)sq;
    a.out_cnt[o] = (int64_t)c;
  } else {
    set_status(a.status, kDevOverflow);
  }
}

// A partition of more than kJChunk dim keys is processed as several chunk
// units, and a key repeated in two chunks would meet no other copy in either
// unit's table. Each chunk unit therefore also looks up the keys of the
// partition's later chunks, [from, to), in its own table.
template <int NT>
__device__ __forceinline__ void check_later_chunks(const uint64_t* tkey, const int32_t* dkey, uint32_t from, uint32_t to,
                                                   uint32_t* status) {
  for (uint32_t j = from + threadIdx.x; j < to; j += NT) {
    const int32_t key = dkey[j];
    uint32_t h = slot_hash(key);
    for (int step = 0; step < kJSlots; ++step) {
      const uint64_t c = tkey[h];
      if (c == kLdsEmpty) break;
      if ((uint32_t)c == (uint32_t)key) {
        set_status(status, kDevDupKey);
        break;
      }
      h = (h + 1) & (kJSlots - 1);
    }
  }
}


// A slot is one 64-bit word {key, count}: the key in the low half, the rows
// matched so far in the high half (for a sub-unit of a split chunk, the key's
// position in its chunk sits above bit kPosShift of that half: sub-units have
// at most kSubRows rows); all ones = empty. 48 KB of LDS per workgroup, so
// three 256-thread workgroups fit on a CU. (The dense key order's units are
// in groupjoin_dense below; one kernel holds both and takes the one the key
// map names, a branch on one word that is uniform over the grid.)
constexpr uint32_t kPosShift = 20;

// The groupjoin's LDS, shared by both key orders' code (one kernel holds both).
struct GroupjoinLds {
  union {
    uint64_t tkc[kJSlots];  // hash order: {key, count} words
    struct {
      uint32_t cnt[kJSlots];       // dense order: rows per slot
      uint32_t own[kJSlots / 32];  // dense order: slots owned by a dim key of the unit
    } d;
  } t;
  uint64_t tsp[kJSlots];
  uint64_t tsq[kJSlots];
  uint32_t scr[kJBlock / kWave];
  uint32_t s_wk[kJPer][kJBlock / kWave];  // occupied slots per (slot round, wave)
  uint64_t s_excl;
  uint4 s_desc;
  uint2 s_split;
  int64_t s_u;
  uint32_t s_last;
  uint64_t s_matched[kJBlock / kWave];
};

// The groupjoin in the hash order.
__device__ __forceinline__ void groupjoin_units(const JoinArgs& a, GroupjoinLds& sh) {
  uint64_t* const tkc = sh.t.tkc;
  uint64_t* const tsp = sh.tsp;
  uint64_t* const tsq = sh.tsq;
  uint32_t* const scr = sh.scr;
  auto& s_wk = sh.s_wk;
  uint64_t& s_excl = sh.s_excl;
  uint4& s_desc = sh.s_desc;
  uint2& s_split = sh.s_split;
  int64_t& s_u = sh.s_u;
  uint32_t& s_last = sh.s_last;
  const int64_t n_units = *a.n_units;
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  uint64_t matched = 0;
  // Units come from the largest-first list in static round robin (see
  // take_ticket). Thread 0 runs a unit ahead: at the start of a unit it reads
  // the next unit's descriptor and publishes it after the probe, so the read
  // never delays a unit. Every thread then issues the next unit's dim-key and
  // first fact-row loads.
  int64_t t_ahead = 0;  // thread 0: the next unit
  int64_t seq = blockIdx.x;
  if (tid == 0) {
    const int64_t t = blockIdx.x;  // first unit without a round trip
    t_ahead = take_ticket(a, seq);
    s_u = t;
    if (t < n_units) {
      s_desc = a.unit_desc[t];
      s_split = a.unit_split[t];
    }
  }
  // The table starts empty once; after that each unit's emission leaves the
  // slots it read empty again, and an insert zeroes its slot's sums, so no
  // unit spends a phase and a barrier clearing it.
  for (int s = tid; s < kJSlots; s += kJBlock) tkc[s] = kLdsEmpty;
  __syncthreads();
  int64_t u = s_u;
  uint4 d = s_desc;
  uint2 sp = s_split;
  int32_t dkeys[kJDK];
  KeyRegs ck, nk;  // this step's keys; the next step's (or the next unit's first step's)
  PayRegs pay, npay;
  if (u < n_units) prefetch_unit(a, d, dkeys, nk, npay);
  while (u < n_units) {
    const uint32_t dlo = d.x, dhi = d.y, flo = d.z, fhi = d.w;
    int64_t t_req = 0;
    uint4 nd = make_uint4(0, 0, 0, 0);
    uint2 ns = make_uint2(0, 0);
    if (tid == 0) {
      if (t_ahead < n_units) {
        nd = a.unit_desc[t_ahead];
        ns = a.unit_split[t_ahead];
      }
      t_req = take_ticket(a, seq);
    }
    // build: at most kJChunk unique keys into kJSlots slots, so a free slot
    // always exists. Every key's first compare-and-swap is issued before any
    // result is examined (one LDS round trip for most keys); keys whose home
    // slot was taken walk on one slot at a time.
    {
      uint32_t h[kJDK];
      uint64_t old[kJDK];
#pragma unroll
      for (int k = 0; k < kJDK; ++k) {
        const uint32_t pos = tid + k * kJBlock;
        h[k] = slot_hash(dkeys[k]);
        old[k] = kLdsEmpty;
        if (dlo + pos < dhi) {
          const uint64_t want = (uint64_t)(uint32_t)dkeys[k] | (sp.x != 0 ? (uint64_t)pos << (32 + kPosShift) : 0ull);
          old[k] = atomicCAS((unsigned long long*)&tkc[h[k]], (unsigned long long)kLdsEmpty, (unsigned long long)want);
        }
      }
#pragma unroll
      for (int k = 0; k < kJDK; ++k) {
        const uint32_t pos = tid + k * kJBlock;
        if (dlo + pos >= dhi) continue;
        const int32_t key = dkeys[k];
        const uint64_t want = (uint64_t)(uint32_t)key | (sp.x != 0 ? (uint64_t)pos << (32 + kPosShift) : 0ull);
        uint32_t hh = h[k];
        uint64_t o = old[k];
        for (int step = 0; step < kJSlots; ++step) {
          if (o == kLdsEmpty) {
            tsp[hh] = 0;
            tsq[hh] = 0;
            break;
          }
          if ((uint32_t)o == (uint32_t)key) {
            set_status(a.status, kDevDupKey);
            break;
          }
          hh = (hh + 1) & (kJSlots - 1);
          o = atomicCAS((unsigned long long*)&tkc[hh], (unsigned long long)kLdsEmpty, (unsigned long long)want);
        }
      }
    }
    __syncthreads();
    if (sp.x == 0 && sp.y > dhi) check_later_chunks<kJBlock>(tkc, a.dkey, dhi, sp.y, a.status);
    int32_t ndkeys[kJDK];
    // probe and aggregate in LDS; long units stream further steps through nxt
    const uint32_t nrows = fhi - flo;
    const uint32_t iters = (nrows + kGR * kJBlock - 1) / (kGR * kJBlock);  // uniform over the workgroup
    // The next unit's descriptor is published at the end of the probe (so no
    // thread waits at the build barrier for thread 0's read of it); its loads
    // go out then and travel during the emission.
    const bool combine = sp.x != 0;
    for (uint32_t it = 0; it < iters; ++it) {
      const uint32_t i0 = flo + it * (kGR * kJBlock) + tid;
      ck = nk;
      pay = npay;
      if (it + 1 < iters) {  // the next step's rows travel during this step's updates
        load_keys(a, i0 + kGR * kJBlock, fhi, nk);
        load_payload(a, i0 + kGR * kJBlock, fhi, npay);
      }
      // find every row's slot first, then update: all rows' home slots are
      // read before any is examined (one LDS round trip for most rows), so
      // the finds are not a chain of dependent reads; rows whose home slot
      // holds another key walk on. The updates follow, not queued behind
      // the finds.
      bool fnd[kGR];
      int slt[kGR];
      {
        uint64_t c[kGR];
#pragma unroll
        for (int k = 0; k < kGR; ++k) {
          slt[k] = (int)slot_hash(ck.key[k]);
          c[k] = tkc[slt[k]];
        }
#pragma unroll
        for (int k = 0; k < kGR; ++k) {
          fnd[k] = false;
          if (i0 + k * kJBlock >= fhi) continue;
          uint32_t h = (uint32_t)slt[k];
          uint64_t cc = c[k];
          for (int step = 0; step < kJSlots; ++step) {
            if (cc == kLdsEmpty) break;
            if ((uint32_t)cc == (uint32_t)ck.key[k]) {
              fnd[k] = true;
              break;
            }
            h = (h + 1) & (kJSlots - 1);
            cc = tkc[h];
          }
          slt[k] = (int)h;
        }
      }
#pragma unroll
      for (int k = 0; k < kGR; ++k) {
        bool found = fnd[k];
        const int slot = slt[k];
        matched += found;
        // Hot keys: when many lanes of the wave hit one slot, pre-sum them so the
        // LDS sees one update instead of a serialised run of same-address atomics.
        // Only sub-units of split chunks check: the hottest keys are what makes
        // a chunk split, and elsewhere the check costs more than it saves.
        if (combine) {
        const uint64_t act = wave_ballot(found);
        if (act == 0) continue;
        const int first = __ffsll((long long)act) - 1;
        const int s0 = __shfl(slot, first, kWave);
        const uint64_t same = wave_ballot(found && slot == s0);
        if (__popcll(same) >= kCombineMin) {
          const bool mine = found && slot == s0;
          const uint64_t tsum_p = wave_sum_u64(mine ? pay.sp[k] : 0);
          const uint64_t tsum_q = wave_sum_u64(mine ? (uint64_t)(int64_t)pay.qty[k] : 0);
          if ((int)lane == first) {
            atomicAdd((unsigned long long*)&tsp[s0], (unsigned long long)tsum_p);
            atomicAdd((unsigned long long*)&tsq[s0], (unsigned long long)tsum_q);
            atomicAdd((unsigned long long*)&tkc[s0], (unsigned long long)__popcll(same) << 32);
          }
          found = found && !mine;
        }
        }
        if (found) {
          atomicAdd((unsigned long long*)&tsp[slot], (unsigned long long)pay.sp[k]);
          atomicAdd((unsigned long long*)&tsq[slot], (unsigned long long)(int64_t)pay.qty[k]);
          atomicAdd((unsigned long long*)&tkc[slot], 1ull << 32);
        }
      }
    }
    if (tid == 0) {  // the next unit, read by everyone after the barrier
      s_u = t_ahead;
      s_desc = nd;
      s_split = ns;
    }
    __syncthreads();
    const int64_t un = s_u;
    const uint4 dn = s_desc;
    const uint2 sn = s_split;
    // past the last unit the loads read the current unit again (discarded)
    const uint4 pd = un < n_units ? dn : d;
    if (sp.x == 0) {
      // Whole unit: emit its groups. Output room is reserved with one atomic
      // per unit, taken when the unit finishes, so no unit waits on another.
      // The next unit's loads are issued after the atomic and travel while
      // thread 0 waits for it. Slots go out in round-major order (round k
      // holds slots k * kJBlock + thread), so each wave's stores of a round
      // land on consecutive output rows.
      constexpr int kRounds = kJPer;
      uint32_t occ[kRounds];
      uint64_t bal[kRounds];
      int sl[kRounds];
#pragma unroll
      for (int k = 0; k < kRounds; ++k) {
        sl[k] = k * kJBlock + tid;
        const uint64_t c = tkc[sl[k]];
        occ[k] = c == kLdsEmpty ? 0u : (uint32_t)(c >> 32);
        bal[k] = wave_ballot(occ[k] != 0);
        if (lane == 0) s_wk[k][wave] = (uint32_t)__popcll(bal[k]);
      }
      __syncthreads();
      uint32_t total = 0, base[kRounds];
#pragma unroll
      for (int k = 0; k < kRounds; ++k) {
#pragma unroll
        for (int w = 0; w < kJBlock / kWave; ++w) {
          if (w == (int)wave) base[k] = total;
          total += s_wk[k][w];
        }
      }
      int64_t resv = 0;
      if (tid == 0 && total) resv = reserve_nowait(a, total);
      prefetch_unit(a, pd, ndkeys, nk, npay);
      if (tid == 0) s_excl = (uint64_t)resv;
      __syncthreads();
      const int64_t o0 = (int64_t)s_excl;
#pragma unroll
      for (int k = 0; k < kRounds; ++k) {
        const int s = sl[k];
        if (occ[k] != 0)
          put_group(a, o0 + base[k] + mask_rank(bal[k]), (int64_t)(int32_t)(uint32_t)tkc[s], tsp[s], tsq[s], occ[k]);
        tkc[s] = kLdsEmpty;
      }
    } else {
      // Sub-unit of a split chunk: add the partial sums into the chunk's
      // accumulator; the last sub-unit to finish emits and clears it.
      prefetch_unit(a, pd, ndkeys, nk, npay);
      SplitAcc* acc = a.split_acc + (size_t)(sp.x - 1) * kJSlots;
#pragma unroll
      for (int k = 0; k < kJPer; ++k) {
        const int s = tid * kJPer + k;
        const uint64_t w = tkc[s];
        tkc[s] = kLdsEmpty;
        if (w == kLdsEmpty) continue;
        const uint32_t c = (uint32_t)(w >> 32) & ((1u << kPosShift) - 1);
        if (c == 0) continue;
        SplitAcc* e = acc + (uint32_t)(w >> (32 + kPosShift));
        dev_add<uint64_t>(&e->sp, tsp[s]);
        dev_add<uint64_t>(&e->sq, tsq[s]);
        dev_add<uint64_t>(&e->cnt, (uint64_t)c);
      }
      __threadfence();
      __syncthreads();
      if (tid == 0) s_last = dev_add_ret<uint32_t>(&a.split_done[sp.x - 1], 1u) + 1 == sp.y;
      __syncthreads();
      if (s_last) {
        __threadfence();
        // a count fits 32 bits (fewer than 2^31 fact rows); the sums are read again when written
        uint32_t vc[kJDK];
        uint32_t mine = 0;
#pragma unroll
        for (int k = 0; k < kJDK; ++k) {
          const uint32_t pos = tid + k * kJBlock;
          vc[k] = dlo + pos < dhi ? (uint32_t)__hip_atomic_load(&acc[pos].cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
          mine += vc[k] != 0;
        }
        if (tid == 0) a.split_done[sp.x - 1] = 0;
        int64_t o = reserve_out(a, mine, scr, &s_excl);
#pragma unroll
        for (int k = 0; k < kJDK; ++k) {
          if (vc[k] == 0) continue;
          SplitAcc* e = acc + tid + k * kJBlock;
          const uint64_t vp = __hip_atomic_load(&e->sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint64_t vq = __hip_atomic_load(&e->sq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          put_group(a, o++, (int64_t)dkeys[k], vp, vq, vc[k]);
          e->sp = 0;
          e->sq = 0;
          e->cnt = 0;
        }
      }
    }
    __syncthreads();  // the table, s_excl and s_last are reused by the next unit
    t_ahead = t_req;  // (thread 0) the atomic has had the whole unit to return
    u = un;
    d = dn;
    sp = sn;
#pragma unroll
    for (int k = 0; k < kJDK; ++k) dkeys[k] = ndkeys[k];
  }
  matched = block_sum_u64<kJBlock>(matched, sh.s_matched);
  if (threadIdx.x == 0 && matched) dev_add<unsigned long long>((unsigned long long*)a.matched, (unsigned long long)matched);
}

// The groupjoin in the dense key order. A unit is 2^ubits consecutive key
// positions (ubits = slot bits + merge <= kJSlotBits) and slot s of its
// direct-mapped table is position (unit << ubits) | s; the dim side gives
// only the unit's bitmap words (which positions hold a dim key), so a unit
// loads one word per 32 slots instead of its dim keys, and emission walks the
// slots, computing each group's key back from its position (key = kmin +
// position * mul^-1 mod 2^L). Counts and sums of every slot start at zero and
// emission leaves them so; fact rows outside the key range match nothing and
// are skipped, rows at a position no dim key holds are counted into its slot
// and never emitted. Otherwise the unit loop is the hash order's below
// (prefetch, tickets, reservation, split sub-units).
__device__ __forceinline__ void groupjoin_dense(const JoinArgs& a, GroupjoinLds& sh) {
  const uint32_t sub = a.km->sub, mul = a.km->mul, inv = a.km->inv, range = a.km->range;
  const uint32_t ubits = a.km->slot_bits + a.km->merge, L = a.km->lbits;
  const uint32_t lmask = L >= 32 ? ~0u : (1u << L) - 1u;
  const uint32_t nslots = 1u << ubits, smask = nslots - 1u;
  const uint32_t nw = ubits >= 5 ? nslots >> 5 : 1u;  // bitmap words of a unit
  const Narrow nar = narrow_of(a.km, a.rng, a.narrow);
  const uint64_t qmask = (1ull << nar.qb) - 1ull;  // qb <= kNarrowFieldBits < 64
  uint32_t* const cnt = sh.t.d.cnt;
  uint32_t* const own = sh.t.d.own;
  uint64_t* const tsp = sh.tsp;
  uint64_t* const tsq = sh.tsq;
  uint32_t* const scr = sh.scr;
  auto& s_wk = sh.s_wk;
  uint64_t& s_excl = sh.s_excl;
  uint4& s_desc = sh.s_desc;
  uint2& s_split = sh.s_split;
  int64_t& s_u = sh.s_u;
  uint32_t& s_last = sh.s_last;
  const int64_t n_units = *a.n_units;
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  uint64_t matched = 0;
  int64_t t_ahead = 0;  // thread 0: the next unit
  int64_t seq = blockIdx.x;
  if (tid == 0) {
    const int64_t t = blockIdx.x;
    t_ahead = take_ticket(a, seq);
    s_u = t;
    if (t < n_units) {
      s_desc = a.unit_desc[t];
      s_split = a.unit_split[t];
    }
  }
  for (int s = tid; s < kJSlots; s += kJBlock) {
    cnt[s] = 0u;
    tsp[s] = 0;
    tsq[s] = 0;
  }
  __syncthreads();
  int64_t u = s_u;
  uint4 d = s_desc;
  uint2 sp = s_split;
  uint32_t own_w = 0;  // threads < nw: a bitmap word of the unit (then of the next unit)
  KeyRegs ck, nk;
  PayRegs pay, npay;
  // a unit's bitmap words and its first step of fact rows (d.x is the unit's index)
  auto load_rows = [&](uint32_t i0, uint32_t hi) {
    if (nar.on) {
      load_packed(a, i0, hi, npay);
    } else {
      load_keys(a, i0, hi, nk);
      load_payload(a, i0, hi, npay);
    }
  };
  auto prefetch = [&](uint4 x) {
    if (tid < nw) own_w = a.bitmap[((x.x << ubits) >> 5) + tid];
    load_rows(x.z + tid, x.w);
  };
  if (u < n_units) prefetch(d);
  while (u < n_units) {
    const uint32_t kbase = d.x << ubits, flo = d.z, fhi = d.w;
    int64_t t_req = 0;
    uint4 nd = make_uint4(0, 0, 0, 0);
    uint2 ns = make_uint2(0, 0);
    if (tid == 0) {
      if (t_ahead < n_units) {
        nd = a.unit_desc[t_ahead];
        ns = a.unit_split[t_ahead];
      }
      t_req = take_ticket(a, seq);
    }
    if (tid < nw) own[tid] = own_w;
    // Every thread has read s_u, s_desc and s_split for this unit before
    // thread 0 overwrites them at the end of the probe.
    __syncthreads();
    const uint32_t nrows = fhi - flo;
    const uint32_t iters = (nrows + kGR * kJBlock - 1) / (kGR * kJBlock);
    const bool combine = sp.x != 0;
    for (uint32_t it = 0; it < iters; ++it) {
      const uint32_t i0 = flo + it * (kGR * kJBlock) + tid;
      ck = nk;
      pay = npay;
      if (it + 1 < iters) load_rows(i0 + kGR * kJBlock, fhi);  // the next step's rows travel during this step's updates
#pragma unroll
      for (int k = 0; k < kGR; ++k) {
        bool found;
        int slot;
        uint64_t pv, qv;  // price and quantity (as 64-bit two's complement)
        if (nar.on) {
          const uint64_t w = pay.sp[k], f = w >> (kNarrowSlotBits + 1);
          found = i0 + k * kJBlock < fhi && ((w >> kNarrowSlotBits) & 1u) != 0;
          slot = (int)(w & smask);
          pv = (uint64_t)nar.pmin + (f >> nar.qb);
          qv = (uint64_t)nar.qmin + (f & qmask);
        } else {
          const uint32_t off = (uint32_t)ck.key[k] - sub;
          found = i0 + k * kJBlock < fhi && off < range;
          slot = (int)((off * mul) & smask);
          pv = pay.sp[k];
          qv = (uint64_t)(int64_t)pay.qty[k];
        }
        // hot keys (split sub-units): lanes of the wave on one slot are summed first
        if (combine) {
          const uint64_t act = wave_ballot(found);
          if (act == 0) continue;
          const int first = __ffsll((long long)act) - 1;
          const int s0 = __shfl(slot, first, kWave);
          const uint64_t same = wave_ballot(found && slot == s0);
          if (__popcll(same) >= kCombineMin) {
            const bool mine = found && slot == s0;
            const uint64_t tsum_p = wave_sum_u64(mine ? pv : 0);
            const uint64_t tsum_q = wave_sum_u64(mine ? qv : 0);
            if ((int)lane == first) {
              atomicAdd((unsigned long long*)&tsp[s0], (unsigned long long)tsum_p);
              atomicAdd((unsigned long long*)&tsq[s0], (unsigned long long)tsum_q);
              atomicAdd(&cnt[s0], (uint32_t)__popcll(same));
            }
            found = found && !mine;
          }
        }
        if (found) {
          atomicAdd((unsigned long long*)&tsp[slot], (unsigned long long)pv);
          atomicAdd((unsigned long long*)&tsq[slot], (unsigned long long)qv);
          atomicAdd(&cnt[slot], 1u);
        }
      }
    }
    if (tid == 0) {  // the next unit, read by everyone after the barrier
      s_u = t_ahead;
      s_desc = nd;
      s_split = ns;
    }
    __syncthreads();
    const int64_t un = s_u;
    const uint4 dn = s_desc;
    const uint2 sn = s_split;
    const uint4 pd = un < n_units ? dn : d;  // past the last unit the loads read this one again (discarded)
    // whether a dim key holds slot s of this unit
    auto owned = [&](uint32_t s) {
      const uint32_t g = kbase | s;
      return s < nslots && ((own[(g >> 5) - (kbase >> 5)] >> (g & 31)) & 1u) != 0u;
    };
    auto key_at = [&](uint32_t s) { return (int64_t)(int32_t)(sub + ((((kbase | s) * inv)) & lmask)); };
    if (sp.x == 0) {
      // Whole unit: emit its owned slots with rows, round k holding slots k * kJBlock + thread.
      uint32_t occ[kJPer];
      uint64_t bal[kJPer];
#pragma unroll
      for (int k = 0; k < kJPer; ++k) {
        const uint32_t s = k * kJBlock + tid;
        occ[k] = owned(s) ? cnt[s] : 0u;
        bal[k] = wave_ballot(occ[k] != 0);
        if (lane == 0) s_wk[k][wave] = (uint32_t)__popcll(bal[k]);
      }
      __syncthreads();
      uint32_t total = 0, base[kJPer];
#pragma unroll
      for (int k = 0; k < kJPer; ++k) {
#pragma unroll
        for (int w = 0; w < kJBlock / kWave; ++w) {
          if (w == (int)wave) base[k] = total;
          total += s_wk[k][w];
        }
      }
      int64_t resv = 0;
      if (tid == 0 && total) resv = reserve_nowait(a, total);
      prefetch(pd);
      if (tid == 0) s_excl = (uint64_t)resv;
      __syncthreads();
      const int64_t o0 = (int64_t)s_excl;
#pragma unroll
      for (int k = 0; k < kJPer; ++k) {
        const uint32_t s = k * kJBlock + tid;
        if (occ[k] != 0) put_group(a, o0 + base[k] + mask_rank(bal[k]), key_at(s), tsp[s], tsq[s], occ[k]);
        matched += occ[k];
        if (s < nslots) {
          cnt[s] = 0u;
          tsp[s] = 0;
          tsq[s] = 0;
        }
      }
    } else {
      // Sub-unit of a split unit: partial sums into the unit's accumulator
      // (one entry per slot); the last sub-unit to finish emits and clears it.
      prefetch(pd);
      SplitAcc* acc = a.split_acc + (size_t)(sp.x - 1) * kJSlots;
#pragma unroll
      for (int k = 0; k < kJPer; ++k) {
        const uint32_t s = k * kJBlock + tid;
        if (s >= nslots) continue;
        const uint32_t c = owned(s) ? cnt[s] : 0u;
        if (c != 0) {
          matched += c;
          dev_add<uint64_t>(&acc[s].sp, tsp[s]);
          dev_add<uint64_t>(&acc[s].sq, tsq[s]);
          dev_add<uint64_t>(&acc[s].cnt, (uint64_t)c);
        }
        cnt[s] = 0u;
        tsp[s] = 0;
        tsq[s] = 0;
      }
      __threadfence();
      __syncthreads();
      if (tid == 0) s_last = dev_add_ret<uint32_t>(&a.split_done[sp.x - 1], 1u) + 1 == sp.y;
      __syncthreads();
      if (s_last) {
        __threadfence();
        uint32_t vc[kJPer];
        uint32_t mine = 0;
#pragma unroll
        for (int k = 0; k < kJPer; ++k) {
          const uint32_t s = k * kJBlock + tid;
          vc[k] = s < nslots ? (uint32_t)__hip_atomic_load(&acc[s].cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
          mine += vc[k] != 0;
        }
        if (tid == 0) a.split_done[sp.x - 1] = 0;
        int64_t o = reserve_out(a, mine, scr, &s_excl);
#pragma unroll
        for (int k = 0; k < kJPer; ++k) {
          if (vc[k] == 0) continue;
          const uint32_t s = k * kJBlock + tid;
          SplitAcc* e = acc + s;
          const uint64_t vp = __hip_atomic_load(&e->sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint64_t vq = __hip_atomic_load(&e->sq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          put_group(a, o++, key_at(s), vp, vq, vc[k]);
          e->sp = 0;
          e->sq = 0;
          e->cnt = 0;
        }
      }
    }
    __syncthreads();  // the table, s_excl and s_last are reused by the next unit
    t_ahead = t_req;
    u = un;
    d = dn;
    sp = sn;
  }
  matched = block_sum_u64<kJBlock>(matched, sh.s_matched);
  if (threadIdx.x == 0 && matched) dev_add<unsigned long long>((unsigned long long*)a.matched, (unsigned long long)matched);
}

__global__ __launch_bounds__(kJBlock, 3) void k_part_groupjoin(JoinArgs a) {
  __shared__ GroupjoinLds sh;
  if (a.km->dense != 0) groupjoin_dense(a, sh);
  else groupjoin_units(a, sh);
}

// ---- partitioned join + aggregate ------------------------------------------------------------------------------------
//
// GROUP BY a dim attribute: each unit's dim keys go into an LDS join table
// with their payload (dim.grp, or dim.prio), its fact rows probe it, and the
// matches aggregate into an LDS group table that lives for the whole kernel
// (units of one workgroup share it) and is flushed into the device-memory
// table at the end. A key the LDS table cannot place within its probe budget
// goes to the device-memory table directly. Units need no merging: a fact row
// matches at most one dim key, hence one unit.

constexpr int kAggSlots = 1024;
constexpr int kABlock = 512;                              // two workgroups per CU (56 KB of LDS each)
constexpr int kADK = (kJChunk + kABlock - 1) / kABlock;  // dim keys per thread

struct AggArgs {
  const uint4* unit_desc;
  const uint2* unit_split;  // {0, partition's dim end} for whole chunks
  const int64_t* n_units;
  const int32_t* dkey;
  const int32_t* dpay;
  const int32_t* fkey;
  const int64_t* fprice;
  const int32_t* fqty;
  const int8_t* fflag;  // (prio, flag) grouping only
  int64_t* ticket;
  int64_t* matched;
  uint32_t* status;
  GroupView groups;
  int32_t lds_probe;
  uint32_t zero;  // 0 at run time; see take_ticket
};

// Units by static round robin, as in k_part_groupjoin.
__device__ __forceinline__ int64_t take_ticket(const AggArgs& a, int64_t& seq) {
  (void)a;
  seq += gridDim.x;
  return seq;
}

template <bool FL>
struct AggRows {
  int32_t key[kJR];
  int32_t qty[kJR];
  uint64_t sp[kJR];
  uint32_t fl;  // the rows' flag bytes (FL only)
};

// Fact rows i0 + k * kABlock of a unit, indices clamped into its (never
// empty) range so that the number of loads is fixed; the probe skips the
// copies past the range.
template <bool FL>
__device__ __forceinline__ void load_agg_rows(const AggArgs& a, uint32_t i0, uint32_t fhi, AggRows<FL>& r) {
  r.fl = 0;
#pragma unroll
  for (int k = 0; k < kJR; ++k) {
    uint32_t i = i0 + k * kABlock;
    i = i < fhi ? i : fhi - 1;
    r.key[k] = a.fkey[i];
    r.sp[k] = (uint64_t)a.fprice[i];
    r.qty[k] = a.fqty[i];
    if constexpr (FL) r.fl |= (uint32_t)(uint8_t)a.fflag[i] << (8 * k);
  }
}

__device__ __forceinline__ void load_agg_dim(const AggArgs& a, uint4 u, int32_t (&dk)[kADK], int32_t (&dp)[kADK]) {
#pragma unroll
  for (int k = 0; k < kADK; ++k) {
    uint32_t j = u.x + threadIdx.x + k * kABlock;
    j = j < u.y ? j : u.y - 1;
    dk[k] = a.dkey[j];
    dp[k] = a.dpay[j];
  }
}

template <int MODE>
__device__ __forceinline__ int64_t agg_group_key(int32_t pay, uint32_t fl, int k) {
  if (MODE == REL_GROUP_PRIO_FLAG) return (int64_t)pay * 256 + (int64_t)((fl >> (8 * k)) & 0xffu);
  return (int64_t)pay;
}

// Two workgroups per CU (56 KB of LDS each).
template <int MODE>
__global__ __launch_bounds__(kABlock, 4) void k_part_join_agg(AggArgs a) {
  constexpr bool FL = MODE == REL_GROUP_PRIO_FLAG;
  __shared__ uint64_t tkey[kJSlots];  // {key, 1} packed; all ones = empty
  __shared__ int32_t tpay[kJSlots];
  __shared__ LdsGroups<kAggSlots> grp;
  __shared__ uint4 s_desc;
  __shared__ uint2 s_split;
  __shared__ int64_t s_u;
  const int64_t n_units = *a.n_units;
  const uint32_t tid = threadIdx.x, lane = lane_id();
  uint64_t matched = 0;
  grp.init(tid, kABlock);
  // units in static round robin from the largest-first list, thread 0 a unit
  // ahead (as in k_part_groupjoin)
  int64_t t_ahead = 0;
  int64_t seq = blockIdx.x;
  if (tid == 0) {
    const int64_t t = blockIdx.x;  // first unit without a round trip
    t_ahead = take_ticket(a, seq);
    s_u = t;
    if (t < n_units) {
      s_desc = a.unit_desc[t];
      s_split = a.unit_split[t];
    }
  }
  __syncthreads();
  int64_t u = s_u;
  uint4 d = s_desc;
  uint2 usplit = s_split;
  int32_t dk[kADK], dp[kADK];
  AggRows<FL> cur, nxt;
  if (u < n_units) {
    load_agg_dim(a, d, dk, dp);
    load_agg_rows<FL>(a, d.z + tid, d.w, cur);
  }
  while (u < n_units) {
    const uint32_t dlo = d.x, dhi = d.y, flo = d.z, fhi = d.w;
    int64_t t_req = 0;
    uint4 nd = make_uint4(0, 0, 0, 0);
    uint2 ns = make_uint2(0, 0);
    if (tid == 0) {
      if (t_ahead < n_units) {
        nd = a.unit_desc[t_ahead];
        ns = a.unit_split[t_ahead];
      }
      t_req = take_ticket(a, seq);
    }
    for (int s = tid; s < kJSlots; s += kABlock) tkey[s] = kLdsEmpty;
    __syncthreads();
    // build: at most kJChunk unique keys into kJSlots slots, so a free slot always exists
#pragma unroll
    for (int k = 0; k < kADK; ++k) {
      if (dlo + tid + k * kABlock >= dhi) continue;
      const int32_t key = dk[k];
      const uint64_t want = (uint64_t)(uint32_t)key | (1ull << 32);
      uint32_t h = slot_hash(key);
      for (int step = 0; step < kJSlots; ++step) {
        const uint64_t old = atomicCAS((unsigned long long*)&tkey[h], (unsigned long long)kLdsEmpty, (unsigned long long)want);
        if (old == kLdsEmpty) {
          tpay[h] = dp[k];
          break;
        }
        if (old == want) {
          set_status(a.status, kDevDupKey);
          break;
        }
        h = (h + 1) & (kJSlots - 1);
      }
    }
    if (tid == 0) {
      s_u = t_ahead;
      s_desc = nd;
      s_split = ns;
    }
    __syncthreads();
    const int64_t un = s_u;
    const uint4 dn = s_desc;
    const uint2 sn = s_split;
    if (usplit.x == 0 && usplit.y > dhi) check_later_chunks<kABlock>(tkey, a.dkey, dhi, usplit.y, a.status);
    const uint4 pd = un < n_units ? dn : d;  // past the last unit: reread this one (discarded)
    int32_t ndk[kADK], ndp[kADK];
    const uint32_t nrows = fhi - flo;
    const uint32_t iters = (nrows + kJR * kABlock - 1) / (kJR * kABlock);
    const bool early = iters <= 1;
    if (early) {
      load_agg_dim(a, pd, ndk, ndp);
      load_agg_rows<FL>(a, pd.z + tid, pd.w, nxt);
    }
    for (uint32_t it = 0; it < iters; ++it) {
      const uint32_t i0 = flo + it * (kJR * kABlock) + tid;
      if (it > 0) cur = nxt;
      if (it + 1 < iters) load_agg_rows<FL>(a, i0 + kJR * kABlock, fhi, nxt);
      bool fnd[kJR];
      int32_t pay[kJR];
#pragma unroll
      for (int k = 0; k < kJR; ++k) {
        fnd[k] = false;
        pay[k] = 0;
        if (i0 + k * kABlock < fhi) {
          const uint64_t want = (uint64_t)(uint32_t)cur.key[k] | (1ull << 32);
          uint32_t h = slot_hash(cur.key[k]);
          for (int step = 0; step < kJSlots; ++step) {
            const uint64_t c = tkey[h];
            if (c == want) {
              fnd[k] = true;
              pay[k] = tpay[h];
              break;
            }
            if (c == kLdsEmpty) break;
            h = (h + 1) & (kJSlots - 1);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kJR; ++k) {
        const bool hit = fnd[k];
        matched += hit;
        const int64_t key = hit ? agg_group_key<MODE>(pay[k], cur.fl, k) : 0;
        const uint64_t sp = cur.sp[k], sq = (uint64_t)(int64_t)cur.qty[k];
        const int s = hit ? grp.find(key, a.lds_probe) : -1;
        bool add = s >= 0;
        // hot groups: many lanes of the wave on one slot are pre-summed
        const uint64_t act = wave_ballot(add);
        if (act != 0) {
          const int first = __ffsll((long long)act) - 1;
          const int s0 = __shfl(s, first, kWave);
          const bool mine = add && s == s0;
          const uint64_t same = wave_ballot(mine);
          if (__popcll(same) >= kCombineMin) {
            const uint64_t tp = wave_sum_u64(mine ? sp : 0);
            const uint64_t tq = wave_sum_u64(mine ? sq : 0);
            if ((int)lane == first) grp.add(s0, tp, tq, (uint64_t)__popcll(same));
            add = add && !mine;
          }
        }
        if (add) grp.add(s, sp, sq, 1ull);
        group_add_wave(a.groups, hit && s < 0, key, sp, sq);
      }
    }
    if (!early) {
      load_agg_dim(a, pd, ndk, ndp);
      load_agg_rows<FL>(a, pd.z + tid, pd.w, nxt);
    }
    __syncthreads();  // the join table and s_u / s_desc are reused by the next unit
    t_ahead = t_req;
    u = un;
    d = dn;
    usplit = sn;
#pragma unroll
    for (int k = 0; k < kADK; ++k) {
      dk[k] = ndk[k];
      dp[k] = ndp[k];
    }
    cur = nxt;
  }
  __syncthreads();
  grp.flush(a.groups, tid, kABlock);
  __shared__ uint64_t s_matched[kABlock / kWave];
  matched = block_sum_u64<kABlock>(matched, s_matched);
  if (threadIdx.x == 0 && matched) dev_add<unsigned long long>((unsigned long long*)a.matched, (unsigned long long)matched);
}

constexpr int kEagerCacheSlots = 256;
constexpr int kEagerCacheProbe = 4;

// GROUP BY dim.grp with more groups than an LDS group table holds: the
// matches of a unit first aggregate per dim key in the unit's LDS join table
// (count in the high half of the key word, sums beside it, as in the
// groupjoin), and at the end of the unit each matched dim key adds its partial
// sums to the device-memory group table under its grp (equal grp values of a
// wave summed first). The device table then sees one update per dim key and
// unit instead of one per fact row, which under skew is far fewer.
__global__ __launch_bounds__(kABlock, 4) void k_part_join_eager(AggArgs a) {
  __shared__ uint64_t tkc[kJSlots];  // {key, rows matched}; all ones = empty
  __shared__ int32_t tpay[kJSlots];
  __shared__ uint64_t tsp[kJSlots];
  __shared__ uint64_t tsq[kJSlots];
  __shared__ LdsGroups<kEagerCacheSlots> cache;  // the workgroup's most frequent groups, flushed at the end
  __shared__ uint4 s_desc;
  __shared__ uint2 s_split;
  __shared__ int64_t s_u;
  const int64_t n_units = *a.n_units;
  const uint32_t tid = threadIdx.x, lane = lane_id();
  uint64_t matched = 0;
  cache.init(tid, kABlock);
  // units in static round robin from the largest-first list, thread 0 a unit ahead
  int64_t t_ahead = 0;
  int64_t seq = blockIdx.x;
  if (tid == 0) {
    const int64_t t = blockIdx.x;  // first unit without a round trip
    t_ahead = take_ticket(a, seq);
    s_u = t;
    if (t < n_units) {
      s_desc = a.unit_desc[t];
      s_split = a.unit_split[t];
    }
  }
  __syncthreads();
  int64_t u = s_u;
  uint4 d = s_desc;
  uint2 usplit = s_split;
  int32_t dk[kADK], dp[kADK];
  AggRows<false> cur, nxt;
  if (u < n_units) {
    load_agg_dim(a, d, dk, dp);
    load_agg_rows<false>(a, d.z + tid, d.w, cur);
  }
  while (u < n_units) {
    const uint32_t dlo = d.x, dhi = d.y, flo = d.z, fhi = d.w;
    int64_t t_req = 0;
    uint4 nd = make_uint4(0, 0, 0, 0);
    uint2 ns = make_uint2(0, 0);
    if (tid == 0) {
      if (t_ahead < n_units) {
        nd = a.unit_desc[t_ahead];
        ns = a.unit_split[t_ahead];
      }
      t_req = take_ticket(a, seq);
    }
    for (int s = tid; s < kJSlots; s += kABlock) tkc[s] = kLdsEmpty;
    __syncthreads();
    // build: at most kJChunk unique keys into kJSlots slots, so a free slot always exists
#pragma unroll
    for (int k = 0; k < kADK; ++k) {
      if (dlo + tid + k * kABlock >= dhi) continue;
      const int32_t key = dk[k];
      uint32_t h = slot_hash(key);
      for (int step = 0; step < kJSlots; ++step) {
        const uint64_t old = atomicCAS((unsigned long long*)&tkc[h], (unsigned long long)kLdsEmpty,
                                       (unsigned long long)(uint32_t)key);
        if (old == kLdsEmpty) {
          tpay[h] = dp[k];
          tsp[h] = 0;
          tsq[h] = 0;
          break;
        }
        if ((uint32_t)old == (uint32_t)key) {
          set_status(a.status, kDevDupKey);
          break;
        }
        h = (h + 1) & (kJSlots - 1);
      }
    }
    if (tid == 0) {
      s_u = t_ahead;
      s_desc = nd;
      s_split = ns;
    }
    __syncthreads();
    const int64_t un = s_u;
    const uint4 dn = s_desc;
    const uint2 sn = s_split;
    if (usplit.x == 0 && usplit.y > dhi) check_later_chunks<kABlock>(tkc, a.dkey, dhi, usplit.y, a.status);
    const uint4 pd = un < n_units ? dn : d;  // past the last unit: reread this one (discarded)
    int32_t ndk[kADK], ndp[kADK];
    const uint32_t nrows = fhi - flo;
    const uint32_t iters = (nrows + kJR * kABlock - 1) / (kJR * kABlock);
    const bool early = iters <= 1;
    if (early) {
      load_agg_dim(a, pd, ndk, ndp);
      load_agg_rows<false>(a, pd.z + tid, pd.w, nxt);
    }
    for (uint32_t it = 0; it < iters; ++it) {
      const uint32_t i0 = flo + it * (kJR * kABlock) + tid;
      if (it > 0) cur = nxt;
      if (it + 1 < iters) load_agg_rows<false>(a, i0 + kJR * kABlock, fhi, nxt);
      bool fnd[kJR];
      int slt[kJR];
#pragma unroll
      for (int k = 0; k < kJR; ++k) {
        fnd[k] = false;
        slt[k] = 0;
        if (i0 + k * kABlock < fhi) {
          uint32_t h = slot_hash(cur.key[k]);
          for (int step = 0; step < kJSlots; ++step) {
            const uint64_t c = tkc[h];
            if (c == kLdsEmpty) break;
            if ((uint32_t)c == (uint32_t)cur.key[k]) {
              fnd[k] = true;
              slt[k] = (int)h;
              break;
            }
            h = (h + 1) & (kJSlots - 1);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kJR; ++k) {
        bool found = fnd[k];
        const int slot = slt[k];
        matched += found;
        // hot keys: many lanes of the wave on one slot are pre-summed
        const uint64_t act = wave_ballot(found);
        if (act == 0) continue;
        const int first = __ffsll((long long)act) - 1;
        const int s0 = __shfl(slot, first, kWave);
        const uint64_t same = wave_ballot(found && slot == s0);
        if (__popcll(same) >= kCombineMin) {
          const bool mine = found && slot == s0;
          const uint64_t tp = wave_sum_u64(mine ? cur.sp[k] : 0);
          const uint64_t tq = wave_sum_u64(mine ? (uint64_t)(int64_t)cur.qty[k] : 0);
          if ((int)lane == first) {
            atomicAdd((unsigned long long*)&tsp[s0], (unsigned long long)tp);
            atomicAdd((unsigned long long*)&tsq[s0], (unsigned long long)tq);
            atomicAdd((unsigned long long*)&tkc[s0], (unsigned long long)__popcll(same) << 32);
          }
          found = found && !mine;
        }
        if (found) {
          atomicAdd((unsigned long long*)&tsp[slot], (unsigned long long)cur.sp[k]);
          atomicAdd((unsigned long long*)&tsq[slot], (unsigned long long)(int64_t)cur.qty[k]);
          atomicAdd((unsigned long long*)&tkc[slot], 1ull << 32);
        }
      }
    }
    if (!early) {
      load_agg_dim(a, pd, ndk, ndp);
      load_agg_rows<false>(a, pd.z + tid, pd.w, nxt);
    }
    __syncthreads();
    // one partial per matched dim key under its grp: into the LDS cache when
    // the group is there or finds room within a short probe, else into the
    // device table
#pragma unroll
    for (int k = 0; k < kJSlots / kABlock; ++k) {
      const int s = k * kABlock + tid;
      const uint64_t c = tkc[s];
      const bool occ = c != kLdsEmpty && (c >> 32) != 0;
      const int64_t g = occ ? (int64_t)tpay[s] : 0;
      const int cs = occ ? cache.find(g, kEagerCacheProbe) : -1;
      if (cs >= 0) cache.add(cs, tsp[s], tsq[s], c >> 32);
      const bool dev = occ && cs < 0;
      group_add_wave_n(a.groups, dev, g, dev ? tsp[s] : 0, dev ? tsq[s] : 0, c >> 32);
    }
    __syncthreads();  // the join table and s_u / s_desc are reused by the next unit
    t_ahead = t_req;
    u = un;
    d = dn;
    usplit = sn;
#pragma unroll
    for (int k = 0; k < kADK; ++k) {
      dk[k] = ndk[k];
      dp[k] = ndp[k];
    }
    cur = nxt;
  }
  __syncthreads();
  cache.flush(a.groups, tid, kABlock);
  __shared__ uint64_t s_matched[kABlock / kWave];
  matched = block_sum_u64<kABlock>(matched, s_matched);
  if (threadIdx.x == 0 && matched) dev_add<unsigned long long>((unsigned long long*)a.matched, (unsigned long long)matched);
}

#define TRY(x)                   \
  do {                           \
    rel_status s_ = (x);         \
    if (s_ != REL_OK) return s_; \
  } while (0)

rel_status partition_side(rel_ctx* ctx, PartSide& s, bool fact, int64_t* passed) {
  const uint32_t nb1 = 1u << s.b1;
  const int64_t ntiles1 = (s.n + kTile1 - 1) / kTile1;
  const dim3 blk(kBlk), sblk(kSBlk);
  // persistent grids, multiples of 8 (one share per XCD)
  const unsigned gs = (unsigned)(ctx->num_cus * 2 / 8 * 8 > 8 ? ctx->num_cus * 2 / 8 * 8 : 8);
  const unsigned gh = gs * 2;
  if (s.n > 0) {
    {
      relh::KernelTimer kt(ctx, fact ? "fact_p1_hist" : "dim_p1_hist");
      if (fact) hipLaunchKernelGGL(k_p1_hist<true>, dim3((unsigned)ntiles1), blk, 0, ctx->stream, s);
      else hipLaunchKernelGGL(k_p1_hist<false>, dim3((unsigned)ntiles1), blk, 0, ctx->stream, s);
    }
    {
      relh::KernelTimer kt(ctx, fact ? "fact_p1_colscan" : "dim_p1_colscan");
      hipLaunchKernelGGL(k_p1_colscan, dim3(nb1), blk, 0, ctx->stream, s.hist1, ntiles1, nb1, s.tot1, passed,
                         s.pcount, 1u << s.b2);
    }
    {
      relh::KernelTimer kt(ctx, fact ? "fact_p1_scatter" : "dim_p1_scatter");
      if (fact) hipLaunchKernelGGL(k_p1_scatter<true>, dim3((unsigned)ntiles1), sblk, 0, ctx->stream, s);
      else hipLaunchKernelGGL(k_p1_scatter<false>, dim3((unsigned)ntiles1), sblk, 0, ctx->stream, s);
    }
  } else {
    TRY(relh::fill_u32(ctx, s.tot1, nb1, 0));
    TRY(relh::fill_u32(ctx, s.pcount, (size_t)nb1 << s.b2, 0));
  }
  REL_LAUNCH_CHECK(ctx, "partition level 1");
  {
    relh::KernelTimer kt(ctx, fact ? "fact_p2_hist" : "dim_p2_hist");
    hipLaunchKernelGGL(k_p2_hist, dim3(gh), blk, 0, ctx->stream, s);
  }
  {
    relh::KernelTimer kt(ctx, fact ? "fact_p2_scan" : "dim_p2_scan");
    hipLaunchKernelGGL(k_p2_scan, dim3(nb1), blk, 0, ctx->stream, s);
  }
  {
    relh::KernelTimer kt(ctx, fact ? "fact_p2_scatter" : "dim_p2_scatter");
    // upper bound of second-level tiles: sum over partitions of ceil(c_p / kTile)
    const dim3 g2((unsigned)(s.n / kTile + nb1));
    if (fact) hipLaunchKernelGGL(k_p2_scatter<true>, g2, sblk, 0, ctx->stream, s);
    else hipLaunchKernelGGL(k_p2_scatter<false>, g2, sblk, 0, ctx->stream, s);
  }
  REL_LAUNCH_CHECK(ctx, "partition level 2");
  return REL_OK;
}

// Carve a scratch buffer into aligned pieces.
struct Carver {
  char* p;
  size_t used = 0;
  template <class T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* r = reinterpret_cast<T*>(p + used);
    used += count * sizeof(T);
    return r;
  }
};

void split_bits(int64_t m, uint32_t* b1, uint32_t* b2) {
  // about 1000 dim keys per final partition, split over two levels of at most 8 bits
  uint32_t pb = 0;
  while (pb < 16 && (m >> pb) > 1000) ++pb;
  if (pb < 2) pb = 2;
  *b1 = (pb + 1) / 2;
  *b2 = pb - *b1;
}

}  // namespace

namespace relh {

bool partitioned_supported(int64_t n, int64_t m) { return n < (1ll << 31) && m < (1ll << 30); }

// Both sides of fact JOIN dim ON fk = pk (fact rows filtered by day < day_lt)
// radix-partitioned into 2^(b1 + b2) partitions, and the work units listed.
struct Partitioned {
  PartSide F, D;
  uint32_t b1, b2, nparts;
  uint4* unit_desc;
  uint2* unit_split;
  int64_t* n_units;
  int64_t* ticket;
  void* split_scratch;
  uint32_t* split_done;
  uint32_t* bitmap;  // dense order (GROUP BY fk): the dim keys' presence bits
};

// dense_ok: the key order may be the dense one (GROUP BY fk), decided on the
// device from the dim keys' range; otherwise the hash order.
rel_status partition_both(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, int32_t day_lt, int pkind,
                          const void* payload, bool with_flag, bool dense_ok, int64_t* counters, int64_t* out_n,
                          Partitioned* P) {
  const int64_t n = fact->n, m = dim->m;
  uint32_t b1, b2;
  split_bits(m, &b1, &b2);
  const uint32_t nb1 = 1u << b1, nb2 = 1u << b2, nparts = nb1 * nb2;
  const int64_t fnt1 = (n + kTile1 - 1) / kTile1, dnt1 = (m + kTile1 - 1) / kTile1;
  // second-level tiles: sum over partitions of ceil(c_p / kTile) <= rows / kTile + partitions
  const int64_t fnt2 = n / kTile + nb1, dnt2 = m / kTile + nb1;
  // whole chunks, plus the sub-units of split chunks (each split chunk adds at most one partial sub-unit)
  const int64_t max_units = (int64_t)nparts + m / kJChunk + 1 + n / kSubRows + kMaxSplit;

  // scratch: partitioned columns (A: fact level 1, B: fact level 2, C: dim both levels), bookkeeping (D)
  void *pa, *pb, *pc, *pd;
  const size_t fact_bytes = (size_t)(n > 0 ? n : 1) * 17 + 4 * 256;  // fk, qty, price, flag
  TRY(scratch(ctx, SCR_PART_A, fact_bytes, &pa));
  TRY(scratch(ctx, SCR_PART_B, fact_bytes, &pb));
  // dim copies, and (GROUP BY fk) the presence bitmap of the dense order: at
  // most 2^(P + 11) key positions, one bit each
  const size_t bitmap_bytes = dense_ok ? ((size_t)1 << (b1 + b2 + kJSlotBits)) / 8 + 256 : 0;
  TRY(scratch(ctx, SCR_PART_C, (size_t)(m > 0 ? m : 1) * 16 + 4 * 256 + bitmap_bytes, &pc));
  const size_t book = ((size_t)fnt1 * nb1 + (size_t)dnt1 * nb1 + (size_t)fnt2 * nb2 + (size_t)dnt2 * nb2 + 2 * nb1 +
                       5 * (size_t)nparts + ((size_t)nparts / kUBlk + 1) * kClasses) * 4 +
                      (size_t)max_units * (sizeof(uint4) + sizeof(uint2)) + (size_t)(fnt2 + dnt2) * sizeof(uint4) +
                      sizeof(KeyMap) + 8 * (size_t)kKeyMinMaxParts + ((size_t)n / 64 + 1) * 8 + ((size_t)fnt1 * kRngWaves + 1) * 16 +
                      64 * 256;
  TRY(scratch(ctx, SCR_PART_D, book, &pd));
  // split-chunk accumulators and their done counters: zero when allocated, and
  // left zero by every call (the last sub-unit of a chunk clears what it emits)
  void* pe;
  const size_t split_bytes = (size_t)kMaxSplit * kJSlots * sizeof(SplitAcc) + (kMaxSplit + 1) * sizeof(uint32_t);
  const bool fresh = ctx->scratch[SCR_PART_E].bytes < split_bytes;
  TRY(scratch(ctx, SCR_PART_E, split_bytes, &pe));
  if (fresh) TRY(fill_u32(ctx, pe, split_bytes / 4, 0));
  uint32_t* split_done = (uint32_t*)((char*)pe + (size_t)kMaxSplit * kJSlots * sizeof(SplitAcc));
  uint32_t* split_ctr = split_done + kMaxSplit;

  PartSide F{};
  F.key = fact->fk;
  F.day = fact->day;
  F.price = fact->price_cents;
  F.qty = fact->qty;
  F.flag = with_flag ? fact->flag : nullptr;
  F.day_lt = day_lt;
  F.n = n;
  F.b1 = b1;
  F.b2 = b2;
  Carver ca{(char*)pa}, cb{(char*)pb}, cc{(char*)pc}, cd{(char*)pd};
  F.key1 = ca.take<int32_t>(n);
  F.qty1 = ca.take<int32_t>(n);
  F.price1 = ca.take<int64_t>(n);
  F.flag1 = with_flag ? ca.take<int8_t>(n) : nullptr;
  F.key2 = cb.take<int32_t>(n);
  F.qty2 = cb.take<int32_t>(n);
  F.price2 = cb.take<int64_t>(n);
  F.flag2 = with_flag ? cb.take<int8_t>(n) : nullptr;
  F.hist1 = cd.take<uint32_t>((size_t)fnt1 * nb1);
  F.pass1 = cd.take<uint32_t>(((size_t)n / 64 + 1) * 2);
  // GROUP BY fk: the passing rows' price and quantity ranges, for narrow second-level rows
  F.rng_part = dense_ok ? cd.take<uint32_t>((size_t)fnt1 * kRngWaves * 4) : nullptr;
  F.rng = dense_ok ? cd.take<uint32_t>(4) : nullptr;
  F.narrow = dense_ok ? 1u : 0u;
  F.tot1 = cd.take<uint32_t>(nb1);
  F.hist2 = cd.take<uint32_t>((size_t)fnt2 * nb2);
  F.pstart = cd.take<uint32_t>(nparts);
  F.pcount = cd.take<uint32_t>(nparts);
  F.tdesc2 = cd.take<uint4>((size_t)fnt2);
  F.ntiles2 = cd.take<int64_t>(1);
  F.zero2 = counters;  // rows passed and join matches: cleared by the fact side's first kernel

  PartSide D{};
  D.key = dim->pk;
  D.pkind = pkind;
  D.payload = payload;
  D.n = m;
  D.b1 = b1;
  D.b2 = b2;
  D.key1 = cc.take<int32_t>(m);
  D.pay1 = cc.take<int32_t>(m);
  D.key2 = cc.take<int32_t>(m);
  D.pay2 = cc.take<int32_t>(m);
  uint32_t* bitmap = dense_ok ? cc.take<uint32_t>(bitmap_bytes / 4) : nullptr;
  D.dense_stop = dense_ok ? 1u : 0u;
  D.hist1 = cd.take<uint32_t>((size_t)dnt1 * nb1);
  D.tot1 = cd.take<uint32_t>(nb1);
  D.hist2 = cd.take<uint32_t>((size_t)dnt2 * nb2);
  D.pstart = cd.take<uint32_t>(nparts);
  D.pcount = cd.take<uint32_t>(nparts);
  D.tdesc2 = cd.take<uint4>((size_t)dnt2);
  D.ntiles2 = cd.take<int64_t>(1);

  uint4* unit_desc = cd.take<uint4>(max_units);
  uint2* unit_split = cd.take<uint2>(max_units);
  uint32_t* sbase = cd.take<uint32_t>(nparts);
  const uint32_t unit_wgs = (nparts + kUBlk - 1) / kUBlk;
  uint32_t* wg_cls = cd.take<uint32_t>((size_t)unit_wgs * kClasses);
  KeyMap* km = cd.take<KeyMap>(1);
  uint32_t* mm_part = cd.take<uint32_t>(2 * (size_t)kKeyMinMaxParts);
  F.km = km;
  D.km = km;

  // the key order of both sides' bins, from the dim keys' range (dense_ok)
  const int32_t n_mm = dense_ok ? key_minmax_partials(ctx, dim->pk, m, mm_part) : 0;
  {
    KernelTimer kt(ctx, "keymap");
    hipLaunchKernelGGL(k_keymap, dim3(1), dim3(kWave), 0, ctx->stream, mm_part, n_mm, b1 + b2, km);
  }
  REL_LAUNCH_CHECK(ctx, "keymap");

  // The two sides are independent until the join: the dim side (small,
  // latency-bound kernels) runs on the auxiliary stream beside the fact side.
  TRY(aux_fork(ctx));
  {
    hipStream_t main = ctx->stream;
    ctx->stream = ctx->aux;
    rel_status sd = partition_side(ctx, D, false, nullptr);
    if (sd == REL_OK && dense_ok) {
      // dense order: the presence bitmap instead of the dim side's second level
      KernelTimer kt(ctx, "dim_bitmap");
      const uint32_t pbw_max = b1 + b2 + kJSlotBits - b1;
      const size_t lds = std::max<size_t>(((size_t)1 << pbw_max) / 8, 256);
      if (lds > 32768)  // past the default dynamic LDS limit (at most 64 KB: 2^19 positions per partition)
        (void)hipFuncSetAttribute((const void*)k_dim_bitmap, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(k_dim_bitmap, dim3(1u << b1), dim3(kBmBlock), lds, ctx->stream, D, bitmap, ctx->d_status);
      if (hipGetLastError() != hipSuccess) sd = fail(ctx, REL_HIP, "dim_bitmap launch");
    }
    ctx->stream = main;
    if (sd != REL_OK) return sd;
  }
  TRY(partition_side(ctx, F, true, counters + CNT_ROWS_PASSED));
  TRY(aux_join(ctx));

  UnitArgs ua{};
  ua.dstart = D.pstart;
  ua.dcount = D.pcount;
  ua.fstart = F.pstart;
  ua.fcount = F.pcount;
  ua.nparts = nparts;
  ua.rows_passed = counters + CNT_ROWS_PASSED;
  ua.split_ctr = split_ctr;
  ua.sbase = sbase;
  ua.wg_cls = wg_cls;
  ua.desc = unit_desc;
  ua.split = unit_split;
  ua.n_units = counters + CNT_AUX0;
  ua.ticket = counters + CNT_TICKET;
  ua.out_n = out_n;
  ua.km = km;
  {
    KernelTimer kt(ctx, "unit_count");
    hipLaunchKernelGGL(k_unit_count, dim3(unit_wgs), dim3(kUBlk), 0, ctx->stream, ua);
  }
  {
    KernelTimer kt(ctx, "unit_emit");
    hipLaunchKernelGGL(k_unit_emit, dim3(unit_wgs), dim3(kUBlk), 0, ctx->stream, ua);
  }
  REL_LAUNCH_CHECK(ctx, "make_units");

  P->F = F;
  P->D = D;
  P->b1 = b1;
  P->b2 = b2;
  P->nparts = nparts;
  P->unit_desc = unit_desc;
  P->unit_split = unit_split;
  P->n_units = counters + CNT_AUX0;
  P->ticket = counters + CNT_TICKET;
  P->split_scratch = pe;
  P->split_done = split_done;
  P->bitmap = bitmap;
  return REL_OK;
}

// GROUP BY fk over fact JOIN dim ON fk = pk, WHERE day < day_lt, radix-partitioned.
rel_status partitioned_groupjoin(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, int32_t day_lt,
                                 rel_groups_out* out, int64_t* counters) {
  Partitioned P;
  // the group key is the join key: no dim payload travels
  TRY(partition_both(ctx, fact, dim, day_lt, PAY_NONE, nullptr, false, true, counters, out->d_n_groups, &P));
  KernelTimer kt(ctx, "part_groupjoin");
  JoinArgs a{};
  a.unit_desc = P.unit_desc;
  a.unit_split = P.unit_split;
  a.n_units = P.n_units;
  a.dkey = P.D.key2;
  a.fkey = P.F.key2;
  a.fprice = P.F.price2;
  a.fqty = P.F.qty2;
  a.split_acc = (SplitAcc*)P.split_scratch;
  a.split_done = P.split_done;
  a.zero = 0;
  a.ticket = P.ticket;
  a.matched = counters + CNT_JOIN_MATCHES;
  a.status = ctx->d_status;
  a.out_key = out->key;
  a.out_sp = out->sum_price;
  a.out_sq = out->sum_qty;
  a.out_cnt = out->count;
  a.out_cap = out->cap;
  a.d_n = out->d_n_groups;
  a.km = P.F.km;
  a.bitmap = P.bitmap;
  a.rng = P.F.rng;
  a.narrow = P.F.narrow;
  a.fpack = reinterpret_cast<const uint64_t*>(P.F.price2);
  const unsigned grid = (unsigned)ctx->num_cus * 3;  // 48 KB of LDS each: three per CU
  hipLaunchKernelGGL(k_part_groupjoin, dim3(grid), dim3(kJBlock), 0, ctx->stream, a);
  REL_LAUNCH_CHECK(ctx, "part_groupjoin");
  return REL_OK;
}

// GROUP BY a dim attribute (dim.grp, or (dim.prio, fact.flag)) over the
// partitioned join: the dim payload travels with the keys (and the fact flag
// with the rows when the key needs it), and k_part_join_agg aggregates into
// the device-memory group table g with an LDS table in front of it.
rel_status partitioned_join_agg(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, int32_t day_lt, int group_by,
                                void* group_slots, uint32_t group_log2cap, uint32_t max_probe, int32_t lds_probe,
                                bool eager, int64_t* counters) {
  Partitioned P;
  const bool prio_flag = group_by == REL_GROUP_PRIO_FLAG;
  TRY(partition_both(ctx, fact, dim, day_lt, prio_flag ? PAY_I8 : PAY_I32,
                     prio_flag ? (const void*)dim->prio : (const void*)dim->grp, prio_flag, false, counters, nullptr,
                     &P));
  KernelTimer kt(ctx, "part_join_agg");
  AggArgs a{};
  a.unit_desc = P.unit_desc;
  a.unit_split = P.unit_split;
  a.n_units = P.n_units;
  a.dkey = P.D.key2;
  a.dpay = P.D.pay2;
  a.fkey = P.F.key2;
  a.fprice = P.F.price2;
  a.fqty = P.F.qty2;
  a.fflag = P.F.flag2;
  a.ticket = P.ticket;
  a.matched = counters + CNT_JOIN_MATCHES;
  a.status = ctx->d_status;
  a.groups = GroupView{(GroupSlot*)group_slots, (uint32_t)((1ull << group_log2cap) - 1), 32u - group_log2cap,
                       ctx->d_status, max_probe};
  a.lds_probe = lds_probe;
  a.zero = 0;
  const unsigned grid = (unsigned)ctx->num_cus * 2;
  if (prio_flag) hipLaunchKernelGGL(k_part_join_agg<REL_GROUP_PRIO_FLAG>, dim3(grid), dim3(kABlock), 0, ctx->stream, a);
  else if (eager) hipLaunchKernelGGL(k_part_join_eager, dim3(grid), dim3(kABlock), 0, ctx->stream, a);
  else hipLaunchKernelGGL(k_part_join_agg<REL_GROUP_DIM_GRP>, dim3(grid), dim3(kABlock), 0, ctx->stream, a);
  REL_LAUNCH_CHECK(ctx, "part_join_agg");
  return REL_OK;
}

}  // namespace relh
