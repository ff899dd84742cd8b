// Handle, error reporting, scratch arena and small fill kernels.
#include <cstdarg>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace {
thread_local std::string g_last_error;
}

namespace fpca {

int set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return set_error(FPCA_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int check_handle(fpca_context *ctx) {
  if (!ctx) return set_error(FPCA_ERR_INVALID_ARG, "null handle");
  return FPCA_OK;
}

int set_device(fpca_context *ctx) {
  FPCA_HIP(hipSetDevice(ctx->device));
  return FPCA_OK;
}

int check_grid(const fpca_grid *g, int64_t *P) {
  if (!g) return set_error(FPCA_ERR_INVALID_ARG, "null grid");
  if (g->d < 1 || g->d > 3) return set_error(FPCA_ERR_UNSUPPORTED, "grid dimension d=%d (1..3 supported)", g->d);
  int64_t p = 1;
  for (int k = 0; k < g->d; ++k) {
    if (g->M[k] < 2) return set_error(FPCA_ERR_INVALID_ARG, "grid M[%d]=%d < 2", k, g->M[k]);
    if (g->M[k] > (1 << 20)) return set_error(FPCA_ERR_UNSUPPORTED, "grid M[%d] too large", k);
    p *= g->M[k];
  }
  if (p > (int64_t(1) << 31)) return set_error(FPCA_ERR_UNSUPPORTED, "grid has too many nodes");
  *P = p;
  return FPCA_OK;
}

GridDims make_dims(const fpca_grid *g) {
  GridDims gd{};
  gd.d = g->d;
  for (int k = 0; k < 3; ++k) gd.M[k] = k < g->d ? g->M[k] : 1;
  int64_t s = 1;
  for (int k = g->d - 1; k >= 0; --k) {
    gd.stride[k] = s;
    s *= g->M[k];
  }
  for (int k = g->d; k < 3; ++k) gd.stride[k] = 0;
  gd.P = s;
  return gd;
}

int ws_reserve(fpca_context *ctx, size_t bytes) {
  if (bytes <= ctx->ws_size) return FPCA_OK;
  if (ctx->ws_limit && bytes > ctx->ws_limit)
    return set_error(FPCA_ERR_WORKSPACE, "scratch request %zu bytes exceeds the limit %zu", bytes,
                     ctx->ws_limit);
  if (ctx->ws) {
    // Earlier queued work may still read the old arena.
    FPCA_HIP(hipStreamSynchronize(ctx->stream));
    FPCA_HIP(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_size = 0;
  }
  size_t want = bytes + bytes / 8;
  hipError_t e = hipMalloc(&ctx->ws, want);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    (void)hipGetLastError();
    return set_error(FPCA_ERR_WORKSPACE, "hipMalloc of %zu scratch bytes failed: %s", want,
                     hipGetErrorString(e));
  }
  ctx->ws_size = want;
  return FPCA_OK;
}

static int arena_reserve(fpca_context *ctx, void **arena, size_t *size, size_t bytes) {
  if (bytes <= *size) return FPCA_OK;
  if (ctx->ws_limit && bytes > ctx->ws_limit)
    return set_error(FPCA_ERR_WORKSPACE, "scratch request %zu bytes exceeds the limit %zu", bytes, ctx->ws_limit);
  if (*arena) {
    FPCA_HIP(hipStreamSynchronize(ctx->stream));
    FPCA_HIP(hipFree(*arena));
    *arena = nullptr;
    *size = 0;
  }
  hipError_t e = hipMalloc(arena, bytes);
  if (e != hipSuccess) {
    *arena = nullptr;
    (void)hipGetLastError();
    return set_error(FPCA_ERR_WORKSPACE, "hipMalloc of %zu scratch bytes failed: %s", bytes, hipGetErrorString(e));
  }
  *size = bytes;
  return FPCA_OK;
}

int tables_stage(fpca_context *ctx, size_t bytes, char **out) {
  if (!ctx->ev_tables) FPCA_HIP(hipEventCreateWithFlags(&ctx->ev_tables, hipEventDisableTiming));
  else FPCA_HIP(hipEventSynchronize(ctx->ev_tables));
  if (bytes > ctx->h_tables_size) {
    if (ctx->h_tables) FPCA_HIP(hipHostFree(ctx->h_tables));
    ctx->h_tables = nullptr;
    ctx->h_tables_size = 0;
    const size_t want = std::max<size_t>(bytes, 64 * 1024);
    hipError_t e = hipHostMalloc(&ctx->h_tables, want);
    if (e != hipSuccess) {
      ctx->h_tables = nullptr;
      (void)hipGetLastError();
      return set_error(FPCA_ERR_WORKSPACE, "pinned staging of %zu bytes failed: %s", want, hipGetErrorString(e));
    }
    ctx->h_tables_size = want;
  }
  *out = static_cast<char *>(ctx->h_tables);
  return FPCA_OK;
}

int ws2_reserve(fpca_context *ctx, size_t bytes) { return arena_reserve(ctx, &ctx->ws2, &ctx->ws2_size, bytes); }
int ws3_reserve(fpca_context *ctx, size_t bytes) { return arena_reserve(ctx, &ctx->ws3, &ctx->ws3_size, bytes); }

template <typename T>
__global__ void k_fill(T *__restrict__ p, T v, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (; i < n; i += step) p[i] = v;
}

template <typename T>
static int fill_t(fpca_context *ctx, T *p, T v, int64_t n) {
  if (n <= 0) return FPCA_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill<T>, dim3(unsigned(blocks)), dim3(256), 0, ctx->stream, p, v, n);
  FPCA_LAUNCH_CHECK("fill");
  return FPCA_OK;
}

int fill_f32(fpca_context *ctx, float *p, float v, int64_t n) { return fill_t(ctx, p, v, n); }
int fill_f64(fpca_context *ctx, double *p, double v, int64_t n) { return fill_t(ctx, p, v, n); }
int fill_i64(fpca_context *ctx, int64_t *p, int64_t v, int64_t n) { return fill_t(ctx, p, v, n); }
int fill_bytes_zero(fpca_context *ctx, void *p, int64_t nbytes) {
  if (nbytes % 4 == 0) return fill_t(ctx, reinterpret_cast<uint32_t *>(p), 0u, nbytes / 4);
  return fill_t(ctx, reinterpret_cast<uint8_t *>(p), uint8_t(0), nbytes);
}

}  // namespace fpca

using namespace fpca;

extern "C" {

const char *fpca_last_error(void) { return g_last_error.c_str(); }

int fpca_create(fpca_handle *handle, int device) {
  if (!handle) return set_error(FPCA_ERR_INVALID_ARG, "null handle pointer");
  *handle = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return set_error(FPCA_ERR_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return set_error(FPCA_ERR_INVALID_ARG, "device %d out of range", device);
  FPCA_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  FPCA_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(FPCA_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device,
                     prop.gcnArchName);
  if (int rc = pace_scratch_init(device)) return rc;
  auto *ctx = new fpca_context();
  ctx->device = device;
  ctx->num_cus = prop.multiProcessorCount;
  if (const char *lim = std::getenv("FPCA_DEBUG_WS_LIMIT")) ctx->ws_limit = std::strtoull(lim, nullptr, 10);
  if (hipMalloc(&ctx->d_flags, 256) != hipSuccess || hipHostMalloc(&ctx->h_flags, 256) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&ctx->h_stage), fpca_context::kStageBytes) != hipSuccess) {
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
    delete ctx;
    return set_error(FPCA_ERR_DEVICE, "flag allocation failed");
  }
  FPCA_HIP(hipMemset(ctx->d_flags, 0, 256));
  *ctx->h_flags = 0;
  *handle = ctx;
  return FPCA_OK;
}

int fpca_destroy(fpca_handle ctx) {
  if (!ctx) return FPCA_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->ws2) (void)hipFree(ctx->ws2);
  if (ctx->ws3) (void)hipFree(ctx->ws3);
  if (ctx->cv_exec) (void)hipGraphExecDestroy(ctx->cv_exec);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->ev_a) (void)hipEventDestroy(ctx->ev_a);
  if (ctx->ev_b) (void)hipEventDestroy(ctx->ev_b);
  if (ctx->d_flags) (void)hipFree(ctx->d_flags);
  if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->h_tables) (void)hipHostFree(ctx->h_tables);
  if (ctx->ev_tables) (void)hipEventDestroy(ctx->ev_tables);
  delete ctx;
  return FPCA_OK;
}

int fpca_set_stream(fpca_handle ctx, void *stream) {
  if (int rc = check_handle(ctx)) return rc;
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  return FPCA_OK;
}

int fpca_stream_create_cu_range(int device, int cu_begin, int cu_end, void **stream) {
  if (!stream) return set_error(FPCA_ERR_INVALID_ARG, "null stream pointer");
  *stream = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return set_error(FPCA_ERR_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return set_error(FPCA_ERR_INVALID_ARG, "device %d out of range", device);
  hipDeviceProp_t prop;
  FPCA_HIP(hipGetDeviceProperties(&prop, device));
  const int n = prop.multiProcessorCount;
  if (cu_begin < 0 || cu_end > n || cu_begin >= cu_end)
    return set_error(FPCA_ERR_INVALID_ARG, "CU range [%d, %d) outside [0, %d)", cu_begin, cu_end, n);
  std::vector<uint32_t> mask(size_t((n + 31) / 32), 0u);
  for (int i = cu_begin; i < cu_end; ++i) mask[size_t(i / 32)] |= 1u << (i % 32);
  int cur = 0;
  FPCA_HIP(hipGetDevice(&cur));
  FPCA_HIP(hipSetDevice(device));
  hipStream_t st = nullptr;
  const hipError_t e = hipExtStreamCreateWithCUMask(&st, uint32_t(mask.size()), mask.data());
  (void)hipSetDevice(cur);
  if (e != hipSuccess)
    return set_error(FPCA_ERR_UNSUPPORTED, "the runtime refused CU range [%d, %d): %s", cu_begin, cu_end,
                     hipGetErrorString(e));
  *stream = st;
  return FPCA_OK;
}

int fpca_stream_destroy(void *stream) {
  if (!stream) return FPCA_OK;
  FPCA_HIP(hipStreamDestroy(reinterpret_cast<hipStream_t>(stream)));
  return FPCA_OK;
}

int fpca_sync(fpca_handle ctx) {
  if (int rc = check_handle(ctx)) return rc;
  if (int rc = set_device(ctx)) return rc;
  FPCA_HIP(hipMemcpyAsync(ctx->h_flags, ctx->d_flags, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  FPCA_HIP(hipStreamSynchronize(ctx->stream));
  if (*ctx->h_flags) {
    int flags = *ctx->h_flags;
    *ctx->h_flags = 0;
    FPCA_HIP(hipMemsetAsync(ctx->d_flags, 0, sizeof(int), ctx->stream));
    FPCA_HIP(hipStreamSynchronize(ctx->stream));
    if (flags & 2)
      return set_error(FPCA_ERR_DEVICE, "a task of the persistent smoother waited past its spin limit");
    if (flags & 1) return set_error(FPCA_ERR_DOMAIN, "an observation lies outside [0,1]^d or is NaN");
  }
  return FPCA_OK;
}

}  // extern "C"
