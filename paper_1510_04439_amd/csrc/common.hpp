// Internal declarations of the gfx950 FPCA library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "fpca.h"

struct fpca_context {
  int device = 0;
  hipStream_t stream = nullptr;
  // One growable scratch arena; carved into sub-buffers per call.
  void *ws = nullptr;
  size_t ws_size = 0;
  size_t ws_limit = 0;  // 0 = unlimited
  // Second arena for the split bf16 operands of the Gram product (its inputs
  // may live in the first arena).
  void *ws2 = nullptr;
  size_t ws2_size = 0;
  // Third arena for the cross-validation buffers (the smoother it calls uses
  // the first).
  void *ws3 = nullptr;
  size_t ws3_size = 0;
  // Captured batched-CV graph: valid for the shape and scratch layout in cv_key.
  std::vector<double> cv_key;
  int cv_key_seen = 0;  // eager runs with this key so far
  hipGraphExec_t cv_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  // Device-side error flags (bit 0: an observation outside [0,1]^d or NaN).
  int *d_flags = nullptr;
  int *h_flags = nullptr;  // pinned mirror
  // d_flags[16], d_flags[17]: the two flags of the PACE right-hand-side
  // kernel; zero between calls (each call's last kernel clears them), and
  // false here while a call that set them may not have cleared them yet.
  bool pace_flags_clean = true;
  // Pinned staging for small device-to-host results (eigenvalues and FVE).
  static constexpr size_t kStageBytes = 4096;
  double *h_stage = nullptr;
  int num_cus = 256;
  // Pinned staging of the task-queue tables (grows); ev_tables marks the
  // last upload from it, so it is not rewritten while a copy is pending.
  void *h_tables = nullptr;
  size_t h_tables_size = 0;
  hipEvent_t ev_tables = nullptr;
  // Pass method of the general smoother (FPCA_CONV_*), and the choices AUTO
  // has timed, per pass shape.
  int conv_mode = FPCA_CONV_DIRECT;
  std::vector<std::pair<std::vector<int64_t>, int>> conv_cache;
  // Covariance smoother engine for general pair weights (FPCA_ENGINE_*).
  int engine = FPCA_ENGINE_AUTO;
  // Tile shapes chosen by the autotuner, per batched-CV shape key.
  std::vector<std::pair<std::vector<double>, std::pair<int, int>>> tune_cache;
};

namespace fpca {

// bf16 split of an FP32 value (the BF16x3 products): hi = round-to-nearest-even
// bf16(x), lo = bf16(x - hi).
__device__ inline unsigned short bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

int set_error(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

#define FPCA_HIP(call)                              \
  do {                                              \
    hipError_t e_ = (call);                         \
    if (e_ != hipSuccess) return fpca::hip_fail(e_, #call); \
  } while (0)

#define FPCA_LAUNCH_CHECK(what)                             \
  do {                                                      \
    hipError_t e_ = hipGetLastError();                      \
    if (e_ != hipSuccess) return fpca::hip_fail(e_, what);  \
  } while (0)

// Scratch arenas: ensure at least `bytes`; returns FPCA_OK or an error.
int ws_reserve(fpca_context *ctx, size_t bytes);
int ws2_reserve(fpca_context *ctx, size_t bytes);
int ws3_reserve(fpca_context *ctx, size_t bytes);
// Pinned host staging of at least `bytes` for table uploads; waits for the
// previous upload from it first.
int tables_stage(fpca_context *ctx, size_t bytes, char **out);

// Whether the persistent task-queue engine runs a covariance smoother on this
// grid under the handle's engine setting (AUTO: when the pass engine's FP64
// moment arrays would not fit in the 256 MB Infinity Cache).
bool use_queue_engine(const fpca_context *ctx, const fpca_grid *grid);
// Covariance smoother behind fpca_smooth_cov (arguments already validated).
int smooth_cov_internal(fpca_context *ctx, const fpca_grid *grid, int dtype, const void *C, double c_uniform,
                        const void *G, const void *mu, const double *bw, void *gamma, int8_t *status);

// Bump allocator over the reserved arena (256-byte aligned carving).
struct Carver {
  char *base;
  size_t off = 0;
  size_t cap;
  template <typename T>
  T *take(size_t count) {
    size_t b = (count * sizeof(T) + 255) & ~size_t(255);
    if (off + b > cap) return nullptr;
    T *p = reinterpret_cast<T *>(base + off);
    off += b;
    return p;
  }
};
inline size_t carve_bytes(size_t count, size_t elem) { return (count * elem + 255) & ~size_t(255); }

int check_handle(fpca_context *ctx);
// Device address of the allocation-free PACE scratch (pace.hip), per device.
int pace_scratch_init(int device);
int check_grid(const fpca_grid *g, int64_t *P);
int set_device(fpca_context *ctx);

// Grid geometry passed by value to kernels.
struct GridDims {
  int d;
  int M[3];
  int64_t stride[3];
  int64_t P;
};
GridDims make_dims(const fpca_grid *g);

// Launch helpers implemented in the .hip sources.
int fill_f32(fpca_context *ctx, float *p, float v, int64_t n);
int fill_f64(fpca_context *ctx, double *p, double v, int64_t n);
int fill_i64(fpca_context *ctx, int64_t *p, int64_t v, int64_t n);
int fill_bytes_zero(fpca_context *ctx, void *p, int64_t nbytes);

// Symmetric rank-k product C = A^T A (A: K x N row-major, ld = N), written to
// both triangles of the N x N output with ldc, scaled by `alpha`; entries on
// the diagonal set to `diag_value` if zero_diag. FP32 operands on MFMA.
// prec = FPCA_PREC_BF16X3 with colsum given: the pass that splits A also
// leaves FP64 column sums of A (and of its squares, with colsq) per chunk of
// 64 rows at colsum[chunk][N] (ceil(K / 64) chunks).
int syrk_f32(fpca_context *ctx, const float *A, int64_t K, int64_t N, float *C, int64_t ldc,
             float alpha, bool zero_diag, int prec, double *colsum = nullptr, double *colsq = nullptr);
int syrk_f64(fpca_context *ctx, const double *A, int64_t K, int64_t N, double *C, int64_t ldc,
             double alpha, bool zero_diag);

}  // namespace fpca
