// Host-side runtime shared by the C ABI translation units: the context and matrix
// handle structures, device allocation through the caller's allocator, error
// reporting, per-kernel event timing and pinned read-backs.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gp2s_internal.h"

struct gp2s_ctx_s {
  hipStream_t stream = nullptr;
  gp2s_alloc_fn alloc = nullptr;
  gp2s_free_fn free_fn = nullptr;
  void* user = nullptr;
  std::string err;
  void* pinned = nullptr;  // small pinned host buffer for scalar read-backs
  // second stream (default priority) for the probe block, which runs beside the y solve
  hipStream_t aux = nullptr;
  // optional per-kernel timing with HIP events: bit k set = category k (GP2S_T_*) timed
  uint32_t timing_mask = 0;
  struct Pending {
    int cat;
    hipEvent_t e0, e1;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double ms[GP2S_NUM_TIMERS] = {};
  int64_t count[GP2S_NUM_TIMERS] = {};
  gp2s_progress_fn progress = nullptr;
  void* progress_user = nullptr;
  // block-product choices of earlier handles, by shape: a new handle of the same shape
  // takes the choice instead of timing the candidates again
  struct TunedShape {
    int64_t n, nnz;
    int prec, S;
    bool f32vec;
    int variant;
  };
  std::vector<TunedShape> tuned;
};

struct gp2s_matrix_s {
  gp2s_ctx ctx = nullptr;
  int64_t n = 0, nnz = 0;
  int prec = GP2S_FP64;
  // block product per column count: >= 0 the variant, -2 to be chosen (a remembered
  // choice for the shape allowed), -3 to be timed afresh
  int spmm_variant[gp2s::kMaxProbes + 1];
  // row tiles of the LDS-staged block product (assembled handles; built on first use)
  gp2s::RowTile* tiles = nullptr;
  int64_t ntiles = 0;
  bool tiles_tried = false;
  // row-grouped copy for the block product (built on first use; values refreshed after a refill)
  int64_t* grp_ptr = nullptr;
  int32_t* grp_col = nullptr;
  void* grp_val = nullptr;
  int32_t* grp_map = nullptr;
  int64_t grp_n = 0;
  bool grp_tried = false, grp_values = false;
  // block split of the block product (variant 5; built on first use, values refreshed
  // after a refill)
  void* bs_val = nullptr;
  int2* bs_seg = nullptr;
  bool bs_tried = false, bs_values = false;
  gp2s_matrix_s() {
    for (int& v : spmm_variant) v = -2;
  }
  bool assembled = false;
  // hyperparameters (assembled handles)
  int dim = 0, P = 0;
  double radius = 0, bump_width = 0, noise = 0;
  int kern = 0;  // Wendland member
  // general kernel (Eq. wendconv): per-axis radii (all equal to radius when isotropic)
  // and the length-scale field's weights c_q; lsq = l(x)^2 per internal point
  double radii[3] = {0.0, 0.0, 0.0};
  bool ard = false;
  std::vector<double> ls_h;
  double* ls_d = nullptr;
  double* lsq = nullptr;
  double ell_bound = 1.0;
  // far-field kernel (Eq. bump_kernel): group of every bump, U groups, G [n * U]
  std::vector<int32_t> ffgrp_h;
  int32_t* ffgrp_d = nullptr;
  int ffU = 0;
  double* ffG = nullptr;
  std::vector<double> centers_h, weights_h;
  double* centers_d = nullptr;
  double* weights_d = nullptr;
  gp2s::GridDev grid{};
  int32_t* perm = nullptr;  // internal -> user (null for imported handles)
  float4* pts32 = nullptr;
  double4* pts64 = nullptr;
  double* x64 = nullptr;
  double* g64 = nullptr;
  int32_t* binid = nullptr;
  int64_t* bin_start = nullptr;
  int64_t* row_ptr = nullptr;
  int32_t* col = nullptr;  // nnz + kQuadPad entries (the pad zeroed)
  void* val = nullptr;     // nnz + kQuadPad entries (the pad zeroed)
  int32_t* rowblk = nullptr;  // row blocks of the streaming single-RHS product [nrowblk + 1]
  int64_t nrowblk = 0;
  double* diag = nullptr;
  double* dinv = nullptr;
  bool diag_ok = true;
  // block-Jacobi factors, [0] over 64-row runs, [1] over 128-row runs (built on first use,
  // dropped when the values change)
  struct BjFactor {
    double* L = nullptr;    // [nblk * B * B] row-major L per block
    double* M = nullptr;    // [nblk * B * B] M^-1 per block, matrix-core operand order
    float* M32 = nullptr;   // the same in float32 (y and refinement solves)
    double* piv = nullptr;  // [n] L_ii^2
    bool ready = false;
  } bj[2];
  std::vector<void*> owned;
};

namespace gp2s {
namespace rt {


constexpr size_t kPinnedBytes = 1 << 16;

inline gp2s_status fail(gp2s_ctx c, gp2s_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

inline void* dalloc(gp2s_ctx c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  if (c->alloc) return c->alloc(bytes, c->user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

inline void dfree(gp2s_ctx c, void* p) {
  if (!p) return;
  if (c->free_fn) c->free_fn(p, c->user);
  else (void)hipFree(p);
}

// Temporary device buffers released when the call returns.
struct Scratch {
  gp2s_ctx c;
  std::vector<void*> ptrs;
  bool oom = false;
  explicit Scratch(gp2s_ctx cc) : c(cc) {}
  ~Scratch() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(c->stream);
    for (void* p : ptrs) dfree(c, p);
  }
  template <typename T>
  T* get(size_t count) {
    void* p = dalloc(c, count * sizeof(T));
    if (!p) {
      oom = true;
      return nullptr;
    }
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
};

template <typename T>
inline T* own(gp2s_matrix m, size_t count) {
  void* p = dalloc(m->ctx, count * sizeof(T));
  if (p) m->owned.push_back(p);
  return static_cast<T*>(p);
}

inline bool is_fin(double v) { return std::isfinite(v); }

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(ctx, GP2S_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define OOMCHK(ptr)                                                                             \
  do {                                                                                          \
    if (!(ptr)) return fail(ctx, GP2S_E_OOM, "device allocation failed (%s)", #ptr);            \
  } while (0)

inline hipEvent_t ev_get(gp2s_ctx c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Collect finished event pairs into the per-category totals; pairs still in flight
// (on another stream) stay pending.
inline void harvest(gp2s_ctx c) {
  size_t keep = 0;
  for (auto& p : c->pending) {
    if (hipEventQuery(p.e1) != hipSuccess) {
      c->pending[keep++] = p;
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      c->ms[p.cat] += ms;
      c->count[p.cat] += 1;
    }
    c->pool.push_back(p.e0);
    c->pool.push_back(p.e1);
  }
  c->pending.resize(keep);
}

// Brackets one or more launches on stream `st` with events when timing is enabled.
struct Timed {
  gp2s_ctx c;
  int cat;
  hipStream_t st;
  hipEvent_t e0 = nullptr;
  Timed(gp2s_ctx cc, int k, hipStream_t s) : c(cc), cat(k), st(s) {
    if ((c->timing_mask >> cat) & 1u) {
      e0 = ev_get(c);
      if (e0) (void)hipEventRecord(e0, st);
    }
  }
  ~Timed() {
    if (!e0) return;
    hipEvent_t e1 = ev_get(c);
    if (!e1) return;
    (void)hipEventRecord(e1, st);
    c->pending.push_back({cat, e0, e1});
  }
};

#define TIMED(cat, expr)                \
  do {                                  \
    Timed t_(ctx, cat, ctx->stream);    \
    HIPCHK(expr);                       \
  } while (0)
#define TIMED_ON(cat, stream, expr)     \
  do {                                  \
    Timed t_(ctx, cat, stream);         \
    HIPCHK(expr);                       \
  } while (0)

inline gp2s_status ensure_device(gp2s_ctx ctx) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0)
    return fail(ctx, GP2S_E_HIP, "no HIP device available (%s)", hipGetErrorString(e));
  if (!ctx->pinned) {
    HIPCHK(hipHostMalloc(&ctx->pinned, kPinnedBytes, hipHostMallocDefault));
  }
  if (!ctx->aux) {
    HIPCHK(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
  }
  return GP2S_OK;
}

// The first half of the pinned buffer serves read-backs; the second half holds the
// lagged convergence polls of the CG drivers (kPollSlot bytes per slot).
constexpr size_t kReadbackBytes = kPinnedBytes / 2;
constexpr size_t kPollSlot = 2048;

// Copy `bytes` from device to the pinned buffer and wait for the stream.
inline gp2s_status readback(gp2s_ctx ctx, const void* dev, size_t bytes, void* host) {
  if (bytes > kReadbackBytes) return fail(ctx, GP2S_E_INVALID, "internal: readback too large");
  HIPCHK(hipMemcpyAsync(ctx->pinned, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::memcpy(host, ctx->pinned, bytes);
  if (!ctx->pending.empty()) harvest(ctx);
  return GP2S_OK;
}

// Same as readback, on stream `s`.
inline gp2s_status readback_on(gp2s_ctx ctx, hipStream_t s, const void* dev, size_t bytes, void* host) {
  if (bytes > kReadbackBytes) return fail(ctx, GP2S_E_INVALID, "internal: readback too large");
  HIPCHK(hipMemcpyAsync(ctx->pinned, dev, bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::memcpy(host, ctx->pinned, bytes);
  return GP2S_OK;
}

inline gp2s_status check_opts(gp2s_ctx ctx, const gp2s_solve_opts* o, bool need_probes) {
  if (!o) return fail(ctx, GP2S_E_INVALID, "opts is NULL");
  if (o->n_probes < 0 || o->n_probes > kMaxProbes)
    return fail(ctx, GP2S_E_INVALID, "n_probes must be in [0, %d]", kMaxProbes);
  if (need_probes && o->n_probes < 1) return fail(ctx, GP2S_E_INVALID, "n_probes must be >= 1");
  if (o->max_iter < 1 || o->max_iter > 10000000) return fail(ctx, GP2S_E_INVALID, "max_iter out of range");
  if (o->max_ir < 0 || o->max_ir > 100) return fail(ctx, GP2S_E_INVALID, "max_ir out of range");
  if (o->check_every < 1) return fail(ctx, GP2S_E_INVALID, "check_every must be >= 1");
  if (!is_fin(o->tol) || o->tol <= 0 || o->tol >= 1) return fail(ctx, GP2S_E_INVALID, "tol must be in (0, 1)");
  if (!is_fin(o->probe_tol) || o->probe_tol <= 0 || o->probe_tol >= 1)
    return fail(ctx, GP2S_E_INVALID, "probe_tol must be in (0, 1)");
  if (o->precond != GP2S_PRECOND_JACOBI && o->precond != GP2S_PRECOND_BLOCK && o->precond != GP2S_PRECOND_BLOCK64)
    return fail(ctx, GP2S_E_INVALID,
                "precond must be GP2S_PRECOND_JACOBI (0), GP2S_PRECOND_BLOCK (1) or GP2S_PRECOND_BLOCK64 (2)");
  return GP2S_OK;
}

// Block preconditioners of a matrix handle: 128-row runs (GP2S_PRECOND_BLOCK) or 64-row runs
// (GP2S_PRECOND_BLOCK64).
inline bool pc_block(int precond) { return precond == GP2S_PRECOND_BLOCK || precond == GP2S_PRECOND_BLOCK64; }
inline int pc_rows(int precond) { return precond == GP2S_PRECOND_BLOCK64 ? kBJ : kBJM; }
inline int pc_idx(int precond) { return precond == GP2S_PRECOND_BLOCK64 ? 0 : 1; }

inline gp2s_status check_matrix(gp2s_ctx ctx, gp2s_matrix m) {
  if (!m) return fail(ctx, GP2S_E_INVALID, "matrix handle is NULL");
  if (m->ctx != ctx) return fail(ctx, GP2S_E_INVALID, "matrix handle belongs to another context");
  return GP2S_OK;
}

}  // namespace rt
}  // namespace gp2s
