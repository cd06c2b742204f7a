// Join-output materialisation: out[i] = in[map[i]] for the columns a consumer
// of the join wants, with map = the probe's fact rows or dim rows.
//
// This is the gather the paper finds behind cuDF's most expensive kernel by
// aggregate time (Section 7, the transform kernel): an unrolled loop that
// reads and writes one element per access and so leaves bandwidth unused. Here
// each thread owns four consecutive pairs: it reads their indices with one
// 16-byte load per side, issues the four element reads of a column together,
// and writes the four results with one store of 4 x elem_bytes (16 bytes for
// int32 columns, two for int64). Row indices are checked against the source
// column's length; an index out of range sets REL_DEV_BADARG and writes zero.
#include "rel_device.h"
#include "rel_host.h"
#include "rel_ops.h"

namespace {

using namespace rel;

constexpr int kGBlock = 256;
constexpr int kGMaxCols = 8;

struct GCol {
  const void* src;
  void* dst;
  int64_t src_rows;
  int32_t eb;    // element bytes: 1, 2, 4 or 8
  int32_t side;  // 0: indexed by fact row, 1: by dim row
};

struct GatherArgs {
  const int32_t* fidx;
  const int32_t* didx;
  const int64_t* d_n;
  int64_t max_pairs;
  uint32_t* status;
  int32_t ncols;
  GCol cols[kGMaxCols];
};

template <class T>
__device__ __forceinline__ T gather_one(const GCol& c, int32_t row, uint32_t* status) {
  if ((uint64_t)(uint32_t)row >= (uint64_t)c.src_rows) {
    set_status(status, kDevBadArg);
    return T(0);
  }
  return static_cast<const T*>(c.src)[row];
}

// Four pairs starting at i0 (all in range): element reads first, then one store.
template <class T>
__device__ __forceinline__ void gather_quad(const GCol& c, const int4& idx, int64_t i0, uint32_t* status) {
  const T v0 = gather_one<T>(c, idx.x, status);
  const T v1 = gather_one<T>(c, idx.y, status);
  const T v2 = gather_one<T>(c, idx.z, status);
  const T v3 = gather_one<T>(c, idx.w, status);
  T* d = static_cast<T*>(c.dst) + i0;
  if constexpr (sizeof(T) == 1) {
    *reinterpret_cast<uint32_t*>(d) = (uint32_t)(uint8_t)v0 | (uint32_t)(uint8_t)v1 << 8 |
                                      (uint32_t)(uint8_t)v2 << 16 | (uint32_t)(uint8_t)v3 << 24;
  } else if constexpr (sizeof(T) == 2) {
    *reinterpret_cast<uint2*>(d) = make_uint2((uint32_t)(uint16_t)v0 | (uint32_t)(uint16_t)v1 << 16,
                                              (uint32_t)(uint16_t)v2 | (uint32_t)(uint16_t)v3 << 16);
  } else if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<uint4*>(d) = make_uint4((uint32_t)v0, (uint32_t)v1, (uint32_t)v2, (uint32_t)v3);
  } else {
    *reinterpret_cast<ulonglong2*>(d) = make_ulonglong2((unsigned long long)v0, (unsigned long long)v1);
    *reinterpret_cast<ulonglong2*>(d + 2) = make_ulonglong2((unsigned long long)v2, (unsigned long long)v3);
  }
}

template <class T>
__device__ __forceinline__ void gather_tail(const GCol& c, const int32_t* fidx, const int32_t* didx, int64_t i,
                                            uint32_t* status) {
  const int32_t row = c.side ? didx[i] : fidx[i];
  static_cast<T*>(c.dst)[i] = gather_one<T>(c, row, status);
}

__global__ __launch_bounds__(kGBlock) void k_join_gather(GatherArgs a) {
  int64_t n = *a.d_n;
  if (n > a.max_pairs) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_status(a.status, kDevBadArg);
    n = a.max_pairs;
  }
  if (n < 0) n = 0;
  const int64_t quads = n / 4;
  const int64_t stride = (int64_t)gridDim.x * kGBlock;
  bool need_f = false, need_d = false;
  for (int c = 0; c < a.ncols; ++c) {
    need_f |= a.cols[c].side == 0;
    need_d |= a.cols[c].side != 0;
  }
  for (int64_t q = blockIdx.x * (int64_t)kGBlock + threadIdx.x; q < quads; q += stride) {
    const int64_t i0 = 4 * q;
    const int4 f = need_f ? *reinterpret_cast<const int4*>(a.fidx + i0) : make_int4(0, 0, 0, 0);
    const int4 d = need_d ? *reinterpret_cast<const int4*>(a.didx + i0) : make_int4(0, 0, 0, 0);
    for (int c = 0; c < a.ncols; ++c) {
      const GCol& col = a.cols[c];
      const int4& idx = col.side ? d : f;
      switch (col.eb) {
        case 1: gather_quad<uint8_t>(col, idx, i0, a.status); break;
        case 2: gather_quad<uint16_t>(col, idx, i0, a.status); break;
        case 4: gather_quad<uint32_t>(col, idx, i0, a.status); break;
        default: gather_quad<uint64_t>(col, idx, i0, a.status); break;
      }
    }
  }
  // the last n mod 4 pairs, one thread each
  const int64_t t = blockIdx.x * (int64_t)kGBlock + threadIdx.x;
  if (t < n - 4 * quads) {
    const int64_t i = 4 * quads + t;
    for (int c = 0; c < a.ncols; ++c) {
      const GCol& col = a.cols[c];
      switch (col.eb) {
        case 1: gather_tail<uint8_t>(col, a.fidx, a.didx, i, a.status); break;
        case 2: gather_tail<uint16_t>(col, a.fidx, a.didx, i, a.status); break;
        case 4: gather_tail<uint32_t>(col, a.fidx, a.didx, i, a.status); break;
        default: gather_tail<uint64_t>(col, a.fidx, a.didx, i, a.status); break;
      }
    }
  }
}

}  // namespace

extern "C" {

rel_status rel_join_gather(rel_ctx* ctx, const int32_t* fact_idx, const int32_t* dim_idx, const int64_t* d_n_pairs,
                           int64_t max_pairs, const rel_gather_col* cols, int32_t n_cols) {
  if (!ctx || !cols || !d_n_pairs || n_cols < 1 || n_cols > kGMaxCols || max_pairs < 0)
    return relh::fail(ctx, REL_INVALID_ARG, "rel_join_gather: bad argument");
  if (max_pairs >= (1ll << 31)) return relh::fail(ctx, REL_UNSUPPORTED, "rel_join_gather: max_pairs >= 2^31");
  GatherArgs a{};
  bool need_f = false, need_d = false;
  for (int32_t c = 0; c < n_cols; ++c) {
    const rel_gather_col& g = cols[c];
    const int eb = g.elem_bytes;
    if ((eb != 1 && eb != 2 && eb != 4 && eb != 8) || (g.side != REL_SIDE_FACT && g.side != REL_SIDE_DIM) ||
        g.src_rows < 0 || (g.src_rows > 0 && !g.src) || (max_pairs > 0 && !g.dst))
      return relh::fail(ctx, REL_INVALID_ARG, "rel_join_gather: column %d invalid", c);
    if (((uintptr_t)g.src % (uintptr_t)eb) != 0 || !relh::aligned16(g.dst))
      return relh::fail(ctx, REL_INVALID_ARG, "rel_join_gather: column %d misaligned (src to its element, dst to 16 B)", c);
    a.cols[c] = GCol{g.src, g.dst, g.src_rows, eb, g.side};
    need_f |= g.side == REL_SIDE_FACT;
    need_d |= g.side == REL_SIDE_DIM;
  }
  if (max_pairs > 0 && ((need_f && (!fact_idx || !relh::aligned16(fact_idx))) || (need_d && (!dim_idx || !relh::aligned16(dim_idx)))))
    return relh::fail(ctx, REL_INVALID_ARG, "rel_join_gather: index arrays must be non-null and 16-byte aligned");
  if (max_pairs == 0) return REL_OK;
  a.fidx = fact_idx;
  a.didx = dim_idx;
  a.d_n = d_n_pairs;
  a.max_pairs = max_pairs;
  a.status = ctx->d_status;
  a.ncols = n_cols;
  const unsigned grid = relh::grid_for(ctx, (max_pairs + 3) / 4, kGBlock, 8);
  relh::KernelTimer kt(ctx, "join_gather");
  hipLaunchKernelGGL(k_join_gather, dim3(grid), dim3(kGBlock), 0, ctx->stream, a);
  REL_LAUNCH_CHECK(ctx, "join_gather");
  return REL_OK;
}

}  // extern "C"
