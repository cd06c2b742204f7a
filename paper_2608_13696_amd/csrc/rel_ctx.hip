// Context, scratch memory, status word and fill kernels.
#include "rel_device.h"
#include "rel_host.h"

namespace {

__global__ void k_fill_u64(uint64_t* __restrict__ p, size_t n, uint64_t v) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

}  // namespace

namespace relh {

rel_status fail(rel_ctx* ctx, rel_status s, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return s;
}

rel_status hip_fail(rel_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, e == hipErrorOutOfMemory ? REL_OOM : REL_HIP, "%s: %s", what, hipGetErrorString(e));
}

rel_status scratch(rel_ctx* ctx, int id, size_t bytes, void** out) {
  ScratchBuf& b = ctx->scratch[id];
  if (b.bytes < bytes) {
    if (b.ptr) {
      // the old buffer may still be in use by enqueued work
      REL_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
      REL_HIP_CHECK(ctx, hipFree(b.ptr));
      b.ptr = nullptr;
      b.bytes = 0;
    }
    size_t want = bytes < 4096 ? 4096 : bytes;
    hipError_t e = hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
      b.ptr = nullptr;
      (void)hipGetLastError();
      return fail(ctx, REL_OOM, "scratch allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
    }
    b.bytes = want;
    b.clean = 0;
  }
  *out = b.ptr;
  return REL_OK;
}

rel_status ensure_counters(rel_ctx* ctx) {
  void* p;
  return scratch(ctx, SCR_COUNTERS, CNT_WORDS * sizeof(int64_t), &p);
}

int64_t* counters(rel_ctx* ctx) { return (int64_t*)ctx->scratch[SCR_COUNTERS].ptr; }

rel_status fill_u64(rel_ctx* ctx, void* p, size_t n, uint64_t v) {
  if (n == 0) return REL_OK;
  const unsigned grid = grid_for(ctx, (int64_t)n, 256 * 8, 4);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, ctx->stream, (uint64_t*)p, n, v);
  REL_LAUNCH_CHECK(ctx, "fill_u64");
  return REL_OK;
}

rel_status fill_u32(rel_ctx* ctx, void* p, size_t n, uint32_t v) {
  if (n == 0) return REL_OK;
  const unsigned grid = grid_for(ctx, (int64_t)n, 256 * 8, 4);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, ctx->stream, (uint32_t*)p, n, v);
  REL_LAUNCH_CHECK(ctx, "fill_u32");
  return REL_OK;
}

static hipEvent_t take_event(rel_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

rel_status aux_fork(rel_ctx* ctx) {
  if (!ctx->aux) {
    REL_HIP_CHECK(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    REL_HIP_CHECK(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    REL_HIP_CHECK(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  }
  REL_HIP_CHECK(ctx, hipEventRecord(ctx->ev_fork, ctx->stream));
  REL_HIP_CHECK(ctx, hipStreamWaitEvent(ctx->aux, ctx->ev_fork, 0));
  return REL_OK;
}

rel_status aux_join(rel_ctx* ctx) {
  REL_HIP_CHECK(ctx, hipEventRecord(ctx->ev_join, ctx->aux));
  REL_HIP_CHECK(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
  return REL_OK;
}

KernelTimer::KernelTimer(rel_ctx* ctx, const char* name) : ctx_(ctx) {
  if (!ctx || !ctx->timing) return;
  for (size_t i = 0; i < ctx->timings.size(); ++i)
    if (ctx->timings[i].name == name) slot_ = (int)i;
  if (slot_ < 0) {
    ctx->timings.push_back(KernelTiming{});
    ctx->timings.back().name = name;
    slot_ = (int)ctx->timings.size() - 1;
  }
  start_ = take_event(ctx);
  if (start_) (void)hipEventRecord(start_, ctx->stream);
}

KernelTimer::~KernelTimer() {
  if (slot_ < 0 || !start_) return;
  hipEvent_t stop = take_event(ctx_);
  if (!stop) return;
  (void)hipEventRecord(stop, ctx_->stream);
  ctx_->timings[slot_].pending.emplace_back(start_, stop);
}

}  // namespace relh

extern "C" {

/* Enable (1) or disable (0) per-kernel event timing on this context; enabling
 * also clears the accumulated times. */
rel_status rel_ctx_enable_timing(rel_ctx* ctx, int enable) {
  if (!ctx) return REL_INVALID_ARG;
  REL_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& t : ctx->timings)
    for (auto& pr : t.pending) {
      ctx->event_pool.push_back(pr.first);
      ctx->event_pool.push_back(pr.second);
    }
  ctx->timings.clear();
  ctx->timing = enable != 0;
  return REL_OK;
}

/* Resolve recorded events (synchronises) and report up to `max` kernels:
 * names[i] (owned by the context, valid until timing is re-enabled), summed
 * milliseconds and launch counts. *count = number of kernels timed. */
rel_status rel_ctx_kernel_times(rel_ctx* ctx, const char** names, double* total_ms, int64_t* launches, int max,
                                int* count) {
  if (!ctx || !count || max < 0 || (max > 0 && (!names || !total_ms || !launches))) return REL_INVALID_ARG;
  REL_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& t : ctx->timings) {
    for (auto& pr : t.pending) {
      float ms = 0.f;
      REL_HIP_CHECK(ctx, hipEventElapsedTime(&ms, pr.first, pr.second));
      t.total_ms += ms;
      t.launches += 1;
      ctx->event_pool.push_back(pr.first);
      ctx->event_pool.push_back(pr.second);
    }
    t.pending.clear();
  }
  const int n = (int)ctx->timings.size();
  for (int i = 0; i < n && i < max; ++i) {
    names[i] = ctx->timings[i].name.c_str();
    total_ms[i] = ctx->timings[i].total_ms;
    launches[i] = ctx->timings[i].launches;
  }
  *count = n;
  return REL_OK;
}

const char* rel_status_string(rel_status s) {
  switch (s) {
    case REL_OK: return "ok";
    case REL_INVALID_ARG: return "invalid argument";
    case REL_CAPACITY: return "output capacity too small";
    case REL_DUPLICATE_KEY: return "duplicate build key";
    case REL_HIP: return "HIP runtime error";
    case REL_OOM: return "out of device memory";
    case REL_UNSUPPORTED: return "unsupported";
    case REL_OVERFLOW: return "table overflow";
  }
  return "unknown status";
}

const char* rel_last_error(const rel_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

rel_status rel_ctx_create(int device, void* hip_stream, rel_ctx** out) {
  if (!out) return REL_INVALID_ARG;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || device < 0 || device >= ndev) return e != hipSuccess ? REL_HIP : REL_INVALID_ARG;
  e = hipSetDevice(device);
  if (e != hipSuccess) return REL_HIP;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return REL_HIP;
  rel_ctx* ctx = new rel_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  ctx->lds_per_block = prop.sharedMemPerBlock;
  e = hipMalloc(&ctx->d_status_words, 256);
  if (e != hipSuccess) {
    delete ctx;
    return REL_OOM;
  }
  ctx->d_status = ctx->d_status_words;
  if (relh::fill_u32(ctx, ctx->d_status_words, 64, 0) != REL_OK || relh::ensure_counters(ctx) != REL_OK ||
      relh::noalloc_scratch_init(ctx, device) != REL_OK || hipStreamSynchronize(ctx->stream) != hipSuccess) {
    (void)hipFree(ctx->d_status_words);
    delete ctx;
    return REL_HIP;
  }
  *out = ctx;
  return REL_OK;
}

rel_status rel_ctx_destroy(rel_ctx* ctx) {
  if (!ctx) return REL_INVALID_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& b : ctx->scratch)
    if (b.ptr) (void)hipFree(b.ptr);
  for (auto& t : ctx->timings)
    for (auto& pr : t.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
    (void)hipEventDestroy(ctx->ev_fork);
    (void)hipEventDestroy(ctx->ev_join);
  }
  if (ctx->d_status_words) (void)hipFree(ctx->d_status_words);
  delete ctx;
  return REL_OK;
}

rel_status rel_ctx_set_stream(rel_ctx* ctx, void* hip_stream) {
  if (!ctx) return REL_INVALID_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return REL_OK;
}

rel_status rel_ctx_sync(rel_ctx* ctx, uint32_t* status_bits) {
  if (!ctx) return REL_INVALID_ARG;
  REL_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  REL_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  uint32_t bits = 0;
  REL_HIP_CHECK(ctx, hipMemcpy(&bits, ctx->d_status_words, sizeof bits, hipMemcpyDeviceToHost));
  if (bits) {
    rel_status s = relh::fill_u32(ctx, ctx->d_status_words, 1, 0);
    if (s != REL_OK) return s;
    REL_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  }
  if (status_bits) *status_bits = bits;
  return REL_OK;
}

}  // extern "C"
