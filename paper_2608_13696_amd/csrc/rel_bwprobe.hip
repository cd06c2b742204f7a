// Streaming bandwidth probe: what HBM delivers to the simplest access pattern
// this library's kernels use (16-byte vector loads and stores by consecutive
// lanes), measured with kernels of the library's own rather than a framework's
// copy. It is the "achievable" line drawn under the 8 TB/s vendor peak, the
// denominator choice the paper discusses for its own rooflines (Section 3.1,
// Table 2).
//
// Each thread moves kUnroll 16-byte words per step, all loads of a step issued
// before any is used, with the non-temporal hint; workgroups stride over the
// buffer so every XCD streams its share from the start.
#include "rel_device.h"
#include "rel_host.h"

namespace {

using namespace rel;

constexpr int kBlock = 256;
constexpr int kUnroll = 4;

// 16-byte words as a native vector type, so that loads and stores can carry
// the non-temporal hint (streamed data is not kept in the caches; measured
// 5-10% faster than plain accesses for a copy on this chip).
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Read: XOR every word into a per-thread accumulator. The accumulator is
// stored only when it equals a value no input here produces, so the compiler
// keeps every load but the kernel writes (almost) nothing.
__global__ __launch_bounds__(kBlock) void k_bw_read(const v4u* __restrict__ src, int64_t words, uint64_t* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * kBlock * kUnroll;
  uint32_t acc = 0;
  for (int64_t base = (int64_t)blockIdx.x * kBlock * kUnroll + threadIdx.x; base < words; base += stride) {
    v4u v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kBlock;
      v[u] = i < words ? __builtin_nontemporal_load(&src[i]) : v4u{0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

__global__ __launch_bounds__(kBlock) void k_bw_copy(const v4u* __restrict__ src, v4u* __restrict__ dst, int64_t words) {
  const int64_t stride = (int64_t)gridDim.x * kBlock * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * kBlock * kUnroll + threadIdx.x; base < words; base += stride) {
    v4u v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kBlock;
      if (i < words) v[u] = __builtin_nontemporal_load(&src[i]);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kBlock;
      if (i < words) __builtin_nontemporal_store(v[u], &dst[i]);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_bw_write(v4u* __restrict__ dst, int64_t words, uint32_t value) {
  const int64_t stride = (int64_t)gridDim.x * kBlock * kUnroll;
  const v4u v = {value, value, value, value};
  for (int64_t base = (int64_t)blockIdx.x * kBlock * kUnroll + threadIdx.x; base < words; base += stride) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kBlock;
      if (i < words) __builtin_nontemporal_store(v, &dst[i]);
    }
  }
}

}  // namespace

extern "C" rel_status rel_bw_probe(rel_ctx* ctx, int32_t mode, const void* src, void* dst, int64_t bytes,
                                   int32_t blocks_per_cu, uint64_t* d_sink) {
  if (!ctx || bytes < 0 || (bytes & 15) != 0 || mode < REL_BW_READ || mode > REL_BW_WRITE || blocks_per_cu < 1 ||
      blocks_per_cu > 64)
    return relh::fail(ctx, REL_INVALID_ARG, "rel_bw_probe: bad argument");
  if ((mode != REL_BW_WRITE && (!src || !relh::aligned16(src))) || (mode != REL_BW_READ && (!dst || !relh::aligned16(dst))) ||
      (mode == REL_BW_READ && !d_sink))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_bw_probe: missing or misaligned buffer");
  const int64_t words = bytes / 16;
  if (words == 0) return REL_OK;
  int64_t grid = (int64_t)ctx->num_cus * blocks_per_cu;
  const int64_t need = (words + kBlock * kUnroll - 1) / (kBlock * kUnroll);
  if (grid > need) grid = need;
  relh::KernelTimer kt(ctx, mode == REL_BW_READ ? "bw_read" : mode == REL_BW_COPY ? "bw_copy" : "bw_write");
  if (mode == REL_BW_READ)
    hipLaunchKernelGGL(k_bw_read, dim3((unsigned)grid), dim3(kBlock), 0, ctx->stream, (const v4u*)src, words, d_sink);
  else if (mode == REL_BW_COPY)
    hipLaunchKernelGGL(k_bw_copy, dim3((unsigned)grid), dim3(kBlock), 0, ctx->stream, (const v4u*)src, (v4u*)dst, words);
  else
    hipLaunchKernelGGL(k_bw_write, dim3((unsigned)grid), dim3(kBlock), 0, ctx->stream, (v4u*)dst, words, 0x5A5A5A5Au);
  REL_LAUNCH_CHECK(ctx, "bw_probe");
  return REL_OK;
}
