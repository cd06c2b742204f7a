// Learned planner: the input sketch (HyperLogLog of fact.fk and dim.grp,
// statistics of sampled rows), the MLP's forward / backward / Adam kernels,
// and the sizing rule that turns a prediction into a plan.
//
// HyperLogLog follows Flajolet, Fusy, Gandouet and Meunier (2007): m = 64
// registers indexed by the top 6 bits of a 64-bit hash; each keeps the
// largest rho = 1 + leading zeros of the remaining 58 bits (59 if all zero).
// The hash of an int32 key is the first SplitMix64 output (Steele, Lea and
// Flood 2014) with the key as the state.
#include <cmath>

#include "rel_device.h"
#include "rel_host.h"
#include "rel_ops.h"

namespace {

using namespace rel;

constexpr int kFeat = REL_SKETCH_FEATURES;
constexpr int kIn = 40, kH = 64, kOut = 2;
constexpr int kW1 = 0, kB1 = kW1 + kIn * kH, kW2 = kB1 + kH, kB2 = kW2 + kH * kH, kW3 = kB2 + kH, kB3 = kW3 + kH * kOut;
constexpr int kParams = kB3 + kOut;
static_assert(kParams == REL_MLP_PARAMS, "parameter layout");
constexpr int kMaxSample = 256;

__device__ __forceinline__ uint64_t hll_hash(int32_t v) {
  uint64_t z = (uint64_t)(uint32_t)v + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ void hll_add(uint32_t* regs, int32_t v) {
  const uint64_t h = hll_hash(v);
  const uint32_t idx = (uint32_t)(h >> 58);
  const uint64_t w = h << 6;
  const uint32_t rho = w ? (uint32_t)__clzll((long long)w) + 1u : 59u;
  if (rho > regs[idx]) atomicMax(&regs[idx], rho);  // the read skips most atomics once registers settle
}

// Registers of one column over all rows; regs (device, 64 words) must start at zero.
__global__ __launch_bounds__(256) void k_hll(const int32_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ regs) {
  __shared__ uint32_t r[64];
  if (threadIdx.x < 64) r[threadIdx.x] = 0;
  __syncthreads();
  const int64_t n4 = n / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += stride) {
    const int4 v = reinterpret_cast<const int4*>(keys)[i];
    hll_add(r, v.x);
    hll_add(r, v.y);
    hll_add(r, v.z);
    hll_add(r, v.w);
  }
  for (int64_t i = 4 * n4 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) hll_add(r, keys[i]);
  __syncthreads();
  if (threadIdx.x < 64 && r[threadIdx.x]) __hip_atomic_fetch_max(&regs[threadIdx.x], r[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ double hll_estimate(const uint32_t* regs, int* zeros_out) {
  double z = 0.0;
  int zeros = 0;
  for (int r = 0; r < 64; ++r) {
    z += ldexp(1.0, -(int)regs[r]);
    zeros += regs[r] == 0;
  }
  double e = 0.709 * 64.0 * 64.0 / z;
  if (e <= 2.5 * 64.0 && zeros > 0) e = 64.0 * log(64.0 / (double)zeros);
  *zeros_out = zeros;
  return e;
}

struct SketchArgs {
  const int32_t* fk;
  const int32_t* day;
  const int32_t* pk;
  const int32_t* grp;
  int64_t n, m;
  int32_t day_lt, group_by;
  const int64_t* fsample;
  const int64_t* dsample;
  int32_t k;
  const uint32_t* regs;  // 128: fk then grp
  float* features;
  uint8_t* hll_out;
};

// Deterministic tree sum over the 256 threads of the block.
__device__ double block_sum_d(double v, double* buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) buf[threadIdx.x] += buf[threadIdx.x + s];
    __syncthreads();
  }
  const double r = buf[0];
  __syncthreads();
  return r;
}

// Per sampled value: its count among the k samples, whether it is the first
// occurrence, then distinct / singleton / doubleton counts and the maximum.
struct FreqStats {
  double distinct, singles, doubles, maxfreq;
};

__device__ FreqStats freq_stats(const int32_t* vals, int k, double* dbuf) {
  int c = 0;
  bool first = true;
  const int t = threadIdx.x;
  if (t < k) {
    const int32_t v = vals[t];
    for (int j = 0; j < k; ++j) {
      c += vals[j] == v;
      first = first && !(j < t && vals[j] == v);
    }
  }
  const bool in = t < k;
  FreqStats f;
  f.distinct = block_sum_d(in && first ? 1.0 : 0.0, dbuf);
  f.singles = block_sum_d(in && c == 1 ? 1.0 : 0.0, dbuf);
  f.doubles = block_sum_d(in && first && c == 2 ? 1.0 : 0.0, dbuf);
  // maximum through the same tree with max
  dbuf[t] = in ? (double)c : 0.0;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) dbuf[t] = fmax(dbuf[t], dbuf[t + s]);
    __syncthreads();
  }
  f.maxfreq = dbuf[0];
  __syncthreads();
  return f;
}

__device__ void block_minmax(const int32_t* vals, int k, int32_t* mn, int32_t* mx, int32_t* buf_lo, int32_t* buf_hi) {
  const int t = threadIdx.x;
  buf_lo[t] = t < k ? vals[t] : INT32_MAX;
  buf_hi[t] = t < k ? vals[t] : INT32_MIN;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      buf_lo[t] = min(buf_lo[t], buf_lo[t + s]);
      buf_hi[t] = max(buf_hi[t], buf_hi[t + s]);
    }
    __syncthreads();
  }
  *mn = buf_lo[0];
  *mx = buf_hi[0];
  __syncthreads();
}

// The 40 features (one workgroup of 256 threads, k <= 256 samples):
//  0 log2(1+N)  1 log2(1+M)  2 log2((1+N)/(1+M))  3 sampled selectivity
//  4..6 one-hot group mode (fk, dim.grp, (prio, flag))
//  7..10 sampled fk: distinct, singletons, doubletons, max frequency (each / k)
//  11 fraction of sampled fk inside [min, max] of sampled pk
//  12 log2(1 + range of sampled fk)  13 log2(1 + range of sampled pk)
//  14..16 sampled grp: distinct / k, singletons / k, log2(1 + range)
//  17..20 HLL(fk): log2(1 + estimate), zero registers / 64, mean register / 16, max register / 64
//  21..36 histogram of the fk registers (value v in bin min(v, 15)) / 64
//  37..38 HLL(grp): log2(1 + estimate), zero registers / 64
//  39 Pearson correlation of sampled (day, fk), 0 when degenerate
__global__ __launch_bounds__(256) void k_sketch_features(SketchArgs a) {
  __shared__ int32_t s_fk[kMaxSample], s_day[kMaxSample], s_pk[kMaxSample], s_grp[kMaxSample];
  __shared__ double dbuf[256];
  __shared__ int32_t ibuf_lo[256], ibuf_hi[256];
  __shared__ double f[kFeat];
  const int t = threadIdx.x, k = a.k;
  const double kk = (double)k;
  if (t < kFeat) f[t] = 0.0;
  if (t < k) {
    const bool hn = a.n > 0, hm = a.m > 0;
    const int64_t fs = hn ? a.fsample[t] : 0, ds = hm ? a.dsample[t] : 0;
    s_fk[t] = hn ? a.fk[fs] : 0;
    s_day[t] = hn ? a.day[fs] : 0;
    s_pk[t] = hm ? a.pk[ds] : 0;
    s_grp[t] = (hm && a.grp) ? a.grp[ds] : 0;
  }
  __syncthreads();
  if (t == 0) {
    f[0] = log2(1.0 + (double)a.n);
    f[1] = log2(1.0 + (double)a.m);
    f[2] = log2((1.0 + (double)a.n) / (1.0 + (double)a.m));
    f[4] = a.group_by == REL_GROUP_FK;
    f[5] = a.group_by == REL_GROUP_DIM_GRP;
    f[6] = a.group_by == REL_GROUP_PRIO_FLAG;
  }
  __syncthreads();
  if (a.n > 0) {  // uniform branch
    const double pass = block_sum_d(t < k && s_day[t] < a.day_lt ? 1.0 : 0.0, dbuf);
    const FreqStats fs = freq_stats(s_fk, k, dbuf);
    int32_t fmin, fmax;
    block_minmax(s_fk, k, &fmin, &fmax, ibuf_lo, ibuf_hi);
    double inside = 0.0, prange = 0.0;
    if (a.m > 0) {
      int32_t pmin, pmax;
      block_minmax(s_pk, k, &pmin, &pmax, ibuf_lo, ibuf_hi);
      inside = block_sum_d(t < k && s_fk[t] >= pmin && s_fk[t] <= pmax ? 1.0 : 0.0, dbuf);
      prange = (double)pmax - (double)pmin;
    }
    const double md = block_sum_d(t < k ? (double)s_day[t] : 0.0, dbuf) / kk;
    const double mf = block_sum_d(t < k ? (double)s_fk[t] : 0.0, dbuf) / kk;
    const double a_ = t < k ? (double)s_day[t] - md : 0.0, b_ = t < k ? (double)s_fk[t] - mf : 0.0;
    const double sdd = block_sum_d(a_ * a_, dbuf), sff = block_sum_d(b_ * b_, dbuf), sdf = block_sum_d(a_ * b_, dbuf);
    if (t == 0) {
      f[3] = pass / kk;
      f[7] = fs.distinct / kk;
      f[8] = fs.singles / kk;
      f[9] = fs.doubles / kk;
      f[10] = fs.maxfreq / kk;
      f[12] = log2(1.0 + ((double)fmax - (double)fmin));
      if (a.m > 0) {
        f[11] = inside / kk;
        f[13] = log2(1.0 + prange);
      }
      f[39] = (sdd > 0 && sff > 0) ? sdf / sqrt(sdd * sff) : 0.0;
    }
  }
  if (a.grp != nullptr && a.m > 0) {
    const FreqStats gs = freq_stats(s_grp, k, dbuf);
    int32_t gmin, gmax;
    block_minmax(s_grp, k, &gmin, &gmax, ibuf_lo, ibuf_hi);
    if (t == 0) {
      f[14] = gs.distinct / kk;
      f[15] = gs.singles / kk;
      f[16] = log2(1.0 + ((double)gmax - (double)gmin));
    }
  }
  __syncthreads();
  if (t == 0) {
    int zeros;
    const double e = hll_estimate(a.regs, &zeros);
    uint32_t mx = 0;
    double sum = 0;
    for (int r = 0; r < 64; ++r) {
      mx = max(mx, a.regs[r]);
      sum += a.regs[r];
      f[21 + min(a.regs[r], 15u)] += 1.0 / 64.0;
    }
    f[17] = log2(1.0 + e);
    f[18] = zeros / 64.0;
    f[19] = sum / 64.0 / 16.0;
    f[20] = mx / 64.0;
    if (a.grp != nullptr) {
      int gz;
      const double ge = hll_estimate(a.regs + 64, &gz);
      f[37] = log2(1.0 + ge);
      f[38] = gz / 64.0;
    }
  }
  __syncthreads();
  if (t < kFeat) a.features[t] = (float)f[t];
  if (t < 128) a.hll_out[t] = (uint8_t)a.regs[t];
}

// ---- MLP ----------------------------------------------------------------------------------------------------------------

constexpr int kSPB = 16;  // samples per workgroup

// The parameters into LDS, 16 loads per thread in flight at a time (one
// after another they cost a round trip each, which dominated a single-sample
// forward pass).
__device__ __forceinline__ void load_params(float* lp, const float* __restrict__ p) {
  constexpr int kBurst = 16;
  for (int base = 0; base < kParams; base += kBurst * (int)blockDim.x) {
    float v[kBurst];
#pragma unroll
    for (int k = 0; k < kBurst; ++k) {
      const int i = base + k * (int)blockDim.x + (int)threadIdx.x;
      v[k] = i < kParams ? p[i] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kBurst; ++k) {
      const int i = base + k * (int)blockDim.x + (int)threadIdx.x;
      if (i < kParams) lp[i] = v[k];
    }
  }
}

// 64 threads: thread j computes hidden unit j; threads 0 and 1 the outputs.
__global__ __launch_bounds__(64) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ x, int32_t B,
                                                    float* __restrict__ y) {
  __shared__ float P[kParams];
  __shared__ float xs[kIn], h1[kH], h2[kH];
  load_params(P, params);
  const int j = threadIdx.x;
  for (int s = blockIdx.x * kSPB; s < B && s < (int)(blockIdx.x + 1) * kSPB; ++s) {
    __syncthreads();
    if (j < kIn) xs[j] = x[(size_t)s * kIn + j];
    __syncthreads();
    float z = P[kB1 + j];
    for (int i = 0; i < kIn; ++i) z += xs[i] * P[kW1 + i * kH + j];
    h1[j] = z > 0.f ? z : 0.f;
    __syncthreads();
    z = P[kB2 + j];
    for (int i = 0; i < kH; ++i) z += h1[i] * P[kW2 + i * kH + j];
    h2[j] = z > 0.f ? z : 0.f;
    __syncthreads();
    if (j < kOut) {
      float o = P[kB3 + j];
      for (int i = 0; i < kH; ++i) o += h2[i] * P[kW3 + i * kOut + j];
      y[(size_t)s * kOut + j] = o;
    }
  }
}

// Per-workgroup partial gradients; thread j owns column j of W1 and W2, row j
// of W3 and entry j of b1, b2 (thread 0 also b3), so no two threads write the
// same entry and nothing needs an atomic.
__global__ __launch_bounds__(64) void k_mlp_backward(const float* __restrict__ params, const float* __restrict__ x,
                                                     const float* __restrict__ tgt, int32_t B, float* __restrict__ partial,
                                                     float* __restrict__ partial_loss) {
  __shared__ float P[kParams];
  __shared__ float G[kParams];
  __shared__ float xs[kIn], z1[kH], h1[kH], z2[kH], h2[kH], dz2[kH], dy[kOut];
  __shared__ float yv[kOut];
  load_params(P, params);
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) G[i] = 0.f;
  const int j = threadIdx.x;
  const float invB = 1.0f / (float)B;
  float loss = 0.f;
  for (int s = blockIdx.x * kSPB; s < B && s < (int)(blockIdx.x + 1) * kSPB; ++s) {
    __syncthreads();
    if (j < kIn) xs[j] = x[(size_t)s * kIn + j];
    __syncthreads();
    float z = P[kB1 + j];
    for (int i = 0; i < kIn; ++i) z += xs[i] * P[kW1 + i * kH + j];
    z1[j] = z;
    h1[j] = z > 0.f ? z : 0.f;
    __syncthreads();
    z = P[kB2 + j];
    for (int i = 0; i < kH; ++i) z += h1[i] * P[kW2 + i * kH + j];
    z2[j] = z;
    h2[j] = z > 0.f ? z : 0.f;
    __syncthreads();
    if (j < kOut) {
      float o = P[kB3 + j];
      for (int i = 0; i < kH; ++i) o += h2[i] * P[kW3 + i * kOut + j];
      yv[j] = o;
      const float d = o - tgt[(size_t)s * kOut + j];
      dy[j] = d * invB;
    }
    __syncthreads();
    if (j == 0) loss += (yv[0] - tgt[(size_t)s * kOut]) * (yv[0] - tgt[(size_t)s * kOut]) +
                        (yv[1] - tgt[(size_t)s * kOut + 1]) * (yv[1] - tgt[(size_t)s * kOut + 1]);
    // output layer
    G[kW3 + j * kOut + 0] += h2[j] * dy[0];
    G[kW3 + j * kOut + 1] += h2[j] * dy[1];
    if (j == 0) {
      G[kB3 + 0] += dy[0];
      G[kB3 + 1] += dy[1];
    }
    const float dh2 = dy[0] * P[kW3 + j * kOut] + dy[1] * P[kW3 + j * kOut + 1];
    dz2[j] = z2[j] > 0.f ? dh2 : 0.f;
    __syncthreads();
    // second layer: column j of W2
    for (int i = 0; i < kH; ++i) G[kW2 + i * kH + j] += h1[i] * dz2[j];
    G[kB2 + j] += dz2[j];
    float dh1 = 0.f;
    for (int c = 0; c < kH; ++c) dh1 += dz2[c] * P[kW2 + j * kH + c];
    const float dz1 = z1[j] > 0.f ? dh1 : 0.f;
    // first layer: column j of W1
    for (int i = 0; i < kIn; ++i) G[kW1 + i * kH + j] += xs[i] * dz1;
    G[kB1 + j] += dz1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) partial[(size_t)blockIdx.x * kParams + i] = G[i];
  if (j == 0) partial_loss[blockIdx.x] = loss;
}

// Sum the per-workgroup partials in workgroup order (deterministic).
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, const float* __restrict__ partial_loss,
                                                    int32_t nparts, int32_t B, float* __restrict__ grad,
                                                    float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kParams) {
    float s = 0.f;
    for (int b = 0; b < nparts; ++b) s += partial[(size_t)b * kParams + i];
    grad[i] = s;
  }
  if (i == 0 && loss) {
    float s = 0.f;
    for (int b = 0; b < nparts; ++b) s += partial_loss[b];
    *loss = s / (2.0f * (float)B);
  }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, float lr, float b1, float b2, float eps,
                                              float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// The network's input. Features that grow with the input size enter relative
// to a reference scale r, the log2 HyperLogLog estimate of the group key
// (fk; dim.grp; for (prio, flag) the smaller of the fk estimate and
// log2(1 + M)): log2 N, log2 M, the sampled key ranges and both estimates
// become differences from r, and the register-level HLL features (their
// level moves with the size) are left out. The network's group output is
// likewise log2(1 + groups) - r and its join output log2(1 + join rows) -
// log2(1 + N). A model trained on small instances then carries over to much
// larger ones. The result is standardised with the training mean and scale.
// aux[0] = raw sampled max frequency (feature 10, the sizing rule's skew
// signal), aux[1] = r, aux[2] = log2(1 + N).
constexpr int kRelFeat[] = {0, 1, 12, 13, 16, 17, 37};

__global__ void k_prepare_input(float* __restrict__ x, const float* __restrict__ mean, const float* __restrict__ scale,
                                float* __restrict__ aux) {
  __shared__ float s_r;
  const int i = threadIdx.x;
  if (i == 0) {
    const float r = x[4] > 0.5f ? x[17] : x[5] > 0.5f ? x[37] : fminf(x[17], x[1]);
    s_r = r;
    aux[0] = x[10];
    aux[1] = r;
    aux[2] = x[0];
  }
  __syncthreads();
  if (i < kFeat) {
    float v = x[i];
    bool rel = false;
#pragma unroll
    for (int j = 0; j < 7; ++j) rel |= i == kRelFeat[j];
    if (rel) v -= s_r;
    else if (i >= 19 && i <= 36) v = 0.f;
    x[i] = (v - mean[i]) / scale[i];
  }
}

// A key seen this often among the sampled rows marks a heavy hitter (about
// 1.5% of the rows or more).
constexpr float kSkewMaxFreq = 4.0f / 256.0f;
// Under such a heavy hitter, with at most this many groups from a dim
// attribute, the plain join (device-memory table) beats the partitioned one:
// the hot keys' probes stay in cache and the groups in LDS, while
// partitioning still pays its passes (measured on 60M fact rows, Zipf(1.2):
// 1.05 vs 1.26 ms at 100 groups; the partitioned path wins from 10^4 groups,
// and for every group count when no key is hot).
constexpr int64_t kSkewPlainJoinGroups = 2048;

#define TRY(e)                   \
  do {                           \
    rel_status s_ = (e);         \
    if (s_ != REL_OK) return s_; \
  } while (0)

}  // namespace

struct rel_planner {
  rel_ctx* ctx = nullptr;
  float* mem = nullptr;  // params, mean, scale, features, prediction
  float margin = 0.f;
};

extern "C" {

rel_status rel_sketch(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, const rel_query* q,
                      const int64_t* d_fact_sample, const int64_t* d_dim_sample, int32_t k, float* d_features,
                      uint8_t* d_hll) {
  if (!ctx || !fact || !dim || !q || !d_features || !d_hll || k < 1 || k > kMaxSample || fact->n < 0 || dim->m < 0 ||
      (fact->n > 0 && (!fact->fk || !fact->day || !d_fact_sample)) || (dim->m > 0 && (!dim->pk || !d_dim_sample)))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_sketch: bad argument");
  if ((fact->fk && !relh::aligned16(fact->fk)) || (dim->grp && !relh::aligned16(dim->grp)))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_sketch: column not 16-byte aligned");
  void* regs;
  TRY(relh::scratch(ctx, SCR_SKETCH, 128 * sizeof(uint32_t), &regs));
  TRY(relh::fill_u32(ctx, regs, 128, 0));
  {
    relh::KernelTimer kt(ctx, "sketch_hll");
    if (fact->n > 0)
      hipLaunchKernelGGL(k_hll, dim3(relh::grid_for(ctx, fact->n / 4 + 1, 256 * 8, 4)), dim3(256), 0, ctx->stream,
                         fact->fk, fact->n, (uint32_t*)regs);
    if (dim->grp && dim->m > 0)
      hipLaunchKernelGGL(k_hll, dim3(relh::grid_for(ctx, dim->m / 4 + 1, 256 * 8, 4)), dim3(256), 0, ctx->stream,
                         dim->grp, dim->m, (uint32_t*)regs + 64);
  }
  SketchArgs a{};
  a.fk = fact->fk;
  a.day = fact->day;
  a.pk = dim->pk;
  a.grp = dim->grp;
  a.n = fact->n;
  a.m = dim->m;
  a.day_lt = q->day_lt;
  a.group_by = q->group_by;
  a.fsample = d_fact_sample;
  a.dsample = d_dim_sample;
  a.k = k;
  a.regs = (const uint32_t*)regs;
  a.features = d_features;
  a.hll_out = d_hll;
  relh::KernelTimer kt(ctx, "sketch_features");
  hipLaunchKernelGGL(k_sketch_features, dim3(1), dim3(256), 0, ctx->stream, a);
  REL_LAUNCH_CHECK(ctx, "sketch");
  return REL_OK;
}

rel_status rel_mlp_forward(rel_ctx* ctx, const float* d_params, const float* d_x, int32_t B, float* d_y) {
  if (!ctx || !d_params || !d_x || !d_y || B < 0) return relh::fail(ctx, REL_INVALID_ARG, "rel_mlp_forward: bad argument");
  if (B == 0) return REL_OK;
  relh::KernelTimer kt(ctx, "mlp_forward");
  hipLaunchKernelGGL(k_mlp_forward, dim3((B + kSPB - 1) / kSPB), dim3(64), 0, ctx->stream, d_params, d_x, B, d_y);
  REL_LAUNCH_CHECK(ctx, "mlp_forward");
  return REL_OK;
}

rel_status rel_mlp_backward(rel_ctx* ctx, const float* d_params, const float* d_x, const float* d_t, int32_t B,
                            float* d_grad, float* d_loss) {
  if (!ctx || !d_params || !d_x || !d_t || !d_grad || B < 1)
    return relh::fail(ctx, REL_INVALID_ARG, "rel_mlp_backward: bad argument");
  const int32_t nb = (B + kSPB - 1) / kSPB;
  void* part;
  TRY(relh::scratch(ctx, SCR_MLP, ((size_t)nb * kParams + nb) * sizeof(float), &part));
  float* pl = (float*)part + (size_t)nb * kParams;
  relh::KernelTimer kt(ctx, "mlp_backward");
  hipLaunchKernelGGL(k_mlp_backward, dim3(nb), dim3(64), 0, ctx->stream, d_params, d_x, d_t, B, (float*)part, pl);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, ctx->stream, (const float*)part,
                     (const float*)pl, nb, B, d_grad, d_loss);
  REL_LAUNCH_CHECK(ctx, "mlp_backward");
  return REL_OK;
}

rel_status rel_mlp_adam_step(rel_ctx* ctx, float* d_params, float* d_m, float* d_v, const float* d_grad, int32_t t,
                             float lr, float beta1, float beta2, float eps) {
  if (!ctx || !d_params || !d_m || !d_v || !d_grad || t < 1) return relh::fail(ctx, REL_INVALID_ARG, "rel_mlp_adam_step: bad argument");
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)t));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)t));
  relh::KernelTimer kt(ctx, "mlp_adam");
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, ctx->stream, d_params, d_m, d_v, d_grad, lr, beta1,
                     beta2, eps, bc1, bc2);
  REL_LAUNCH_CHECK(ctx, "mlp_adam");
  return REL_OK;
}

rel_status rel_planner_create(rel_ctx* ctx, const float* params, const float* mean, const float* scale,
                              float margin_log2, rel_planner** out) {
  if (!ctx || !params || !mean || !scale || !out || !(margin_log2 >= 0.f))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_planner_create: bad argument");
  for (int i = 0; i < kFeat; ++i)
    if (!(scale[i] > 0.f)) return relh::fail(ctx, REL_INVALID_ARG, "rel_planner_create: scale[%d] must be > 0", i);
  rel_planner* p = new rel_planner();
  p->ctx = ctx;
  p->margin = margin_log2;
  const size_t floats = kParams + 3 * kFeat + 8 + 64;  // params, mean, scale, features, prediction + aux, HLL bytes
  hipError_t e = hipMalloc(&p->mem, floats * sizeof(float));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return relh::fail(ctx, REL_OOM, "rel_planner_create: allocation failed");
  }
  if (hipMemcpy(p->mem, params, kParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->mem + kParams, mean, kFeat * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->mem + kParams + kFeat, scale, kFeat * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->mem);
    delete p;
    return relh::fail(ctx, REL_HIP, "rel_planner_create: copy failed");
  }
  *out = p;
  return REL_OK;
}

rel_status rel_planner_plan(rel_planner* p, const rel_fact* fact, const rel_dim* dim, const rel_query* q,
                            const int64_t* d_fact_sample, const int64_t* d_dim_sample, int32_t k, rel_plan* plan,
                            float* pred) {
  if (!p || !plan) return REL_INVALID_ARG;
  rel_ctx* ctx = p->ctx;
  float* params = p->mem;
  float* mean = params + kParams;
  float* scale = mean + kFeat;
  float* feat = scale + kFeat;
  float* y = feat + kFeat;  // y[0], y[1]: network outputs; y[2..4]: aux of k_prepare_input
  uint8_t* hll = (uint8_t*)(y + 8);
  TRY(rel_sketch(ctx, fact, dim, q, d_fact_sample, d_dim_sample, k, feat, hll));
  {
    relh::KernelTimer kt(ctx, "planner_input");
    hipLaunchKernelGGL(k_prepare_input, dim3(1), dim3(64), 0, ctx->stream, feat, (const float*)mean,
                       (const float*)scale, y + 2);
  }
  REL_LAUNCH_CHECK(ctx, "prepare_input");
  TRY(rel_mlp_forward(ctx, params, feat, 1, y));
  float hy[5];
  REL_HIP_CHECK(ctx, hipMemcpyAsync(hy, y, sizeof hy, hipMemcpyDeviceToHost, ctx->stream));
  REL_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  const double log2_join = (double)hy[0] + hy[4], log2_groups = (double)hy[1] + hy[3];
  if (pred) {
    pred[0] = (float)log2_join;
    pred[1] = (float)log2_groups;
  }
  // sizing rule: expected groups = 2^(prediction + margin), never above the plain bound
  const int64_t n = fact->n, m = dim->m;
  const int64_t ub = q->group_by == REL_GROUP_PRIO_FLAG ? std::min<int64_t>(n, 65536) : std::min(n, m);
  double e = std::exp2(log2_groups + (double)p->margin);
  if (!std::isfinite(e) || e > (double)ub) e = (double)ub;
  int64_t expected = (int64_t)std::ceil(e);
  if (expected < 1) expected = 1;
  plan->group_capacity = expected;
  // LDS holds every group when they are few; under a heavy hitter it also pays
  // as a cache in front of a larger device-memory table
  const bool skewed = hy[2] >= kSkewMaxFreq;
  plan->group_placement = (expected <= relh::kLdsGroupCap || skewed) ? REL_PLACE_LDS : REL_PLACE_GLOBAL;
  plan->join_placement = (skewed && q->group_by != REL_GROUP_FK && expected <= kSkewPlainJoinGroups)
                             ? REL_PLACE_GLOBAL
                             : REL_PLACE_AUTO;
  plan->allow_fallback = 1;
  plan->reserved = 0;
  return REL_OK;
}

rel_status rel_planner_destroy(rel_planner* p) {
  if (!p) return REL_INVALID_ARG;
  (void)hipStreamSynchronize(p->ctx->stream);
  if (p->mem) (void)hipFree(p->mem);
  delete p;
  return REL_OK;
}

}  // extern "C"
