// C ABI of the batched mode: many independent instances assembled and solved as one
// block-diagonal system. CG iterations are captured once per solve as a hipGraph
// chunk on a private stream and replayed until every instance has converged; the host
// only polls the convergence flags between chunks.
#include "runtime.h"

using namespace gp2s;
using namespace gp2s::rt;

struct gp2s_batch_s {
  gp2s_ctx ctx = nullptr;
  int M = 0, prec = GP2S_MIXED, S = 0;
  gp2s_solve_opts opts{};
  std::vector<int64_t> n, row0;
  int64_t N = 0;
  std::vector<int> dim, P, cent0, kern;
  int Ptot = 0;
  std::vector<double> radius, width, noise, centers3, weights;
  std::vector<double> bbox;  // [M * 6]
  double capacity_factor = 1.25;
  // device
  double* x3 = nullptr;
  BInst* inst_d = nullptr;
  std::vector<BInst> inst_h;
  int64_t* row_start_d = nullptr;
  int32_t* inst_of_row = nullptr;
  int32_t* blk_inst = nullptr;
  int64_t nblk = 0;
  double* centers3_d = nullptr;
  double* weights_d = nullptr;
  int32_t* goff_d = nullptr;
  std::vector<int32_t> goff_h;
  int64_t nbins = 0, nbins_cap = 0;
  int64_t* bin_start = nullptr;
  int32_t* bin_count = nullptr;
  int32_t* perm = nullptr;
  float4* pts32 = nullptr;
  double4* pts64 = nullptr;
  double* x64 = nullptr;
  double* g64 = nullptr;
  int32_t* binid = nullptr;
  int64_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  void* val = nullptr;
  double* diag = nullptr;
  double* dinv = nullptr;
  int64_t cap = 0, nnz = 0;
  // block-Jacobi preconditioner (opts.precond == GP2S_PRECOND_BLOCK): the batch's row
  // blocks (64 rows of one instance) factored once per run
  double* bj_L = nullptr;
  double* bj_M = nullptr;
  float* bj_M32 = nullptr;  // the same in float32 (y and refinement solves)
  double* bj_piv = nullptr;
  int64_t* bj_r0 = nullptr;
  int32_t* bj_m = nullptr;
  // tuned launch shapes
  int m_ref = 1, spmv_lanes = 16, spmm_lanes = 64;
  double tune_ms[8] = {};
  hipStream_t cap_stream = nullptr;  // y solves and refinement
  hipStream_t cap2 = nullptr;        // probe block, beside the y solves
  int32_t* pin = nullptr;  // pinned poll slots: 4 x (M * S + 8) int32
  std::vector<void*> owned;
};

namespace {

template <typename T>
T* bown(gp2s_batch b, size_t count) {
  void* p = dalloc(b->ctx, count * sizeof(T));
  if (p) b->owned.push_back(p);
  return static_cast<T*>(p);
}

BatchGeom geom(const gp2s_batch b) {
  BatchGeom g{};
  g.inst = b->inst_d;
  g.M = b->M;
  g.row_start = b->row_start_d;
  g.inst_of_row = b->inst_of_row;
  g.blk_inst = b->blk_inst;
  g.n = b->N;
  g.nblk = b->nblk;
  g.blk_map = nullptr;
  g.grid = b->nblk;
  return g;
}

// Grids of every instance for bin refinement m (bins of side >= r / m, at most
// max(4 n, 4096) bins per instance), and the per-instance table.
void build_grids(gp2s_batch b, int m) {
  int64_t bin0 = 0;
  b->inst_h.assign(b->M, BInst{});
  int64_t blk = 0;
  for (int i = 0; i < b->M; ++i) {
    BInst& I = b->inst_h[i];
    const int d = b->dim[i];
    double h = b->radius[i] * (1.0 + 1e-6) / m;
    const double max_bins = std::max(4.0 * (double)b->n[i], 4096.0);
    for (int it = 0; it < 64; ++it) {
      double tot = 1.0;
      for (int k = 0; k < d; ++k) tot *= std::floor((b->bbox[i * 6 + 3 + k] - b->bbox[i * 6 + k]) / h) + 1.0;
      if (tot <= max_bins) break;
      h *= std::pow(tot / max_bins, 1.0 / d) * 1.01;
    }
    I.grid.dim = 3;
    I.grid.nbins = 1;
    for (int k = 0; k < 3; ++k) {
      I.grid.origin[k] = k < d ? b->bbox[i * 6 + k] : 0.0;
      I.grid.nb[k] = k < d ? (int32_t)(std::floor((b->bbox[i * 6 + 3 + k] - b->bbox[i * 6 + k]) / h) + 1.0) : 1;
      I.grid.nbins *= I.grid.nb[k];
    }
    for (int k = 0; k < 3; ++k) I.grid.inv_h[k] = 1.0 / h;
    I.row0 = b->row0[i];
    I.rows = b->n[i];
    I.bin0 = bin0;
    bin0 += I.grid.nbins;
    I.blk0 = blk;
    I.nblk = (b->n[i] + kBRows - 1) / kBRows;
    blk += I.nblk;
    I.radius = b->radius[i];
    I.r2 = b->radius[i] * b->radius[i];
    I.inv_r2 = 1.0 / I.r2;
    I.noise = b->noise[i];
    I.bump_w2 = b->width[i] * b->width[i];
    I.dim = d;
    I.P = b->P[i];
    I.cent0 = b->cent0[i];
    I.m = m;
    I.kern = b->kern[i];
  }
  b->nbins = bin0;
  b->nblk = blk;
}

// Prologue, bin sort, gathers and the count pass; leaves row_ptr and nnz. Bins and
// the point arrays are (re)allocated when the grid needs more room.
gp2s_status assemble_pattern(gp2s_batch b, Scratch& sc, int32_t** row_cnt_out, float* count_ms) {
  gp2s_ctx ctx = b->ctx;
  hipStream_t st = ctx->stream;
  if (b->nbins > b->nbins_cap) {
    b->bin_start = bown<int64_t>(b, b->nbins + 1);
    b->bin_count = bown<int32_t>(b, b->nbins);
    OOMCHK(b->bin_start);
    OOMCHK(b->bin_count);
    b->nbins_cap = b->nbins;
  }
  HIPCHK(hipMemcpyAsync(b->inst_d, b->inst_h.data(), b->M * sizeof(BInst), hipMemcpyHostToDevice, st));
  const BatchGeom g = geom(b);
  int32_t* bin_of = sc.get<int32_t>(b->N);
  int32_t* slot = sc.get<int32_t>(b->N);
  double* g64u = sc.get<double>(b->N);
  uint8_t* gam = sc.get<uint8_t>(b->N);
  int32_t* perm_tmp = sc.get<int32_t>(b->N);
  uint32_t* fkey = sc.get<uint32_t>(b->N);
  uint32_t* key_tmp = sc.get<uint32_t>(b->N);
  int32_t* row_cnt = sc.get<int32_t>(b->N);
  void* scan_ws = sc.get<uint8_t>(std::max(scan_workspace_bytes(b->nbins), scan_workspace_bytes(b->N)));
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "batch assembly workspace allocation failed");
  HIPCHK(hipMemsetAsync(b->bin_count, 0, b->nbins * sizeof(int32_t), st));
  HIPCHK(launch_bprologue(b->x3, g, b->centers3_d, b->weights_d, bin_of, slot, b->bin_count, g64u, gam, fkey, st));
  HIPCHK(launch_exscan_i32_i64(b->bin_count, b->bin_start, b->nbins, scan_ws, st));
  HIPCHK(launch_scatter(b->N, bin_of, slot, fkey, b->bin_start, perm_tmp, key_tmp, st));
  HIPCHK(launch_binsort(b->N, perm_tmp, key_tmp, bin_of, b->bin_start, b->perm, st));
  HIPCHK(launch_bgather(b->x3, g, b->perm, bin_of, g64u, gam, b->pts32, b->pts64, b->x64, b->g64, b->binid,
                        b->inst_of_row, st));
  BAsm a{};
  a.g = g;
  a.pts32 = b->pts32;
  a.pts64 = b->pts64;
  a.g64 = b->g64;
  a.binid = b->binid;
  a.bin_start = b->bin_start;
  a.cap = b->cap;
  hipEvent_t e0 = ev_get(ctx), e1 = ev_get(ctx);
  HIPCHK(hipEventRecord(e0, st));
  HIPCHK(launch_bassemble_count(a, b->prec, row_cnt, st));
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(launch_exscan_i32_i64(row_cnt, b->row_ptr, b->N, scan_ws, st));
  gp2s_status s = readback(ctx, b->row_ptr + b->N, sizeof(int64_t), &b->nnz);
  if (count_ms) (void)hipEventElapsedTime(count_ms, e0, e1);
  ctx->pool.push_back(e0);
  ctx->pool.push_back(e1);
  if (s) return s;
  if (row_cnt_out) *row_cnt_out = row_cnt;
  return GP2S_OK;
}

gp2s_status assemble_fill(gp2s_batch b, Scratch& sc) {
  gp2s_ctx ctx = b->ctx;
  hipStream_t st = ctx->stream;
  if (b->nnz > b->cap)
    return fail(ctx, GP2S_E_CAPACITY, "batch needs %lld stored entries, capacity is %lld: plan again",
                (long long)b->nnz, (long long)b->cap);
  int32_t* flags = sc.get<int32_t>(2);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "allocation failed");
  HIPCHK(hipMemsetAsync(flags, 0, 2 * sizeof(int32_t), st));
  BAsm a{};
  a.g = geom(b);
  a.pts32 = b->pts32;
  a.pts64 = b->pts64;
  a.g64 = b->g64;
  a.binid = b->binid;
  a.bin_start = b->bin_start;
  a.cap = b->cap;
  HIPCHK(launch_bassemble_fill(a, b->prec, b->row_ptr, b->col, b->val, b->diag, flags, st));
  HIPCHK(launch_dinv(b->N, b->diag, b->dinv, flags + 1, st));
  int32_t hf[2];
  gp2s_status s = readback(ctx, flags, sizeof(hf), hf);
  if (s) return s;
  if (hf[0]) return fail(ctx, GP2S_E_CAPACITY, "batch capacity exceeded during the fill");
  if (hf[1]) return fail(ctx, GP2S_E_NOT_SPD, "a diagonal entry of K is not positive");
  return GP2S_OK;
}

// Host copy through pageable memory (any size), ordered on stream `s`.
gp2s_status bread(gp2s_ctx ctx, hipStream_t s, const void* dev, size_t bytes, void* host) {
  HIPCHK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return GP2S_OK;
}

// Makes stream `to` wait for the work queued so far on stream `from`.
gp2s_status order_after(gp2s_ctx ctx, hipStream_t from, hipStream_t to) {
  hipEvent_t e = nullptr;
  HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipError_t e1 = hipEventRecord(e, from);
  hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(to, e, 0) : e1;
  (void)hipEventDestroy(e);
  if (e2 != hipSuccess) return fail(ctx, GP2S_E_HIP, "stream ordering: %s", hipGetErrorString(e2));
  return GP2S_OK;
}

// Batched Jacobi-PCG over M instances x S columns on its own stream. Iterations run as
// replays of a captured chunk of `check_every` iterations. After each replay the host
// queues an asynchronous copy of the done flags into a pinned slot plus an event, and
// evaluates the copy queued one replay earlier, so the stream never drains while the
// host polls. When the row blocks of instances with open columns fall to half of those
// launched, the chunk is captured again over just those blocks (a block map private to
// this solve), so two solves can run side by side on two streams.
struct BCg {
  gp2s_batch b = nullptr;
  int S = 1;
  double* X = nullptr;
  const char* label = "";
  hipStream_t st = nullptr;
  int32_t* slots = nullptr;  // two pinned slots of SM + 4 int32
  // state
  CgState cs{};
  bool f32vec = false;
  int SM = 0, max_iter = 0, chunk = 1;
  double* R = nullptr;
  double* Z = nullptr;  // M^-1 r (block preconditioner)
  bool bj = false;
  bool probe = false;  // the probe block: float64 M^-1 (it enters the estimators)
  void* P = nullptr;
  void* Q = nullptr;
  int32_t* si = nullptr;
  int32_t* iter_dev = nullptr;
  int32_t* map_d = nullptr;
  BatchGeom gc{};
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int nq = 0, it = 0;
  bool open = true;
  std::vector<int32_t> map, iters, done;
  int total = 0;
  bool converged = false;

  int32_t* slot(int k) const { return slots + (size_t)k * (SM + 4); }
  ~BCg() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

gp2s_status bcg_capture(BCg& c) {
  gp2s_batch b = c.b;
  gp2s_ctx ctx = b->ctx;
  if (c.exec) {
    (void)hipGraphExecDestroy(c.exec);
    c.exec = nullptr;
  }
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(c.st, hipStreamCaptureModeThreadLocal));
  hipError_t ce = hipSuccess;
  for (int k = 0; k < c.chunk && ce == hipSuccess; ++k) {
    ce = launch_bcg_matvec(b->prec, c.gc, b->row_ptr, b->col, b->val, c.S, c.S == 1 ? b->spmv_lanes : b->spmm_lanes,
                           c.P, c.Q, c.f32vec, c.cs, c.st);
    if (c.bj) {
      if (ce == hipSuccess)
        ce = launch_bbj_update(c.gc, c.S, c.X, c.R, c.P, c.Q, c.f32vec, b->bj_M, c.Z, c.cs, c.iter_dev, c.st,
                               c.S == 1 && !c.probe ? b->bj_M32 : nullptr);
      if (ce == hipSuccess) ce = launch_bcg_pupdate(c.gc, c.S, c.P, c.Z, nullptr, c.f32vec, c.cs, c.iter_dev, c.st);
    } else {
      if (ce == hipSuccess)
        ce = launch_bcg_update(c.gc, c.S, c.X, c.R, c.P, c.Q, c.f32vec, b->dinv, c.cs, c.iter_dev, c.st);
      if (ce == hipSuccess) ce = launch_bcg_pupdate(c.gc, c.S, c.P, c.R, b->dinv, c.f32vec, c.cs, c.iter_dev, c.st);
    }
  }
  hipError_t ee = hipStreamEndCapture(c.st, &graph);
  if (ce != hipSuccess || ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(ctx, GP2S_E_HIP, "capturing the CG chunk failed: %s", hipGetErrorString(ce != hipSuccess ? ce : ee));
  }
  hipError_t ie = hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    c.exec = nullptr;
    return fail(ctx, GP2S_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
  }
  return GP2S_OK;
}

// Workspace, initial state (after the work queued on the context's stream) and the
// first chunk's graph.
gp2s_status bcg_begin(BCg& c, const double* B, const double* tol_dev, double tol, bool keep_hist, Scratch& sc) {
  gp2s_batch b = c.b;
  gp2s_ctx ctx = b->ctx;
  const int64_t n = b->N;
  const int S = c.S;
  c.SM = b->M * S;
  const int SM = c.SM;
  c.f32vec = b->prec == GP2S_MIXED && S > 1;
  const size_t vb = c.f32vec ? sizeof(float) : sizeof(double);
  c.max_iter = b->opts.max_iter;
  c.R = sc.get<double>((size_t)n * S);
  c.bj = pc_block(b->opts.precond) && b->bj_M;
  c.Z = c.bj ? sc.get<double>((size_t)n * S) : nullptr;
  c.P = sc.get<uint8_t>((size_t)n * S * vb);
  c.Q = sc.get<double>((size_t)n * S);
  double* sd = sc.get<double>(6 * (size_t)SM + (size_t)b->nblk * S * 2);
  c.si = sc.get<int32_t>(2 * (size_t)SM + 8);
  c.map_d = sc.get<int32_t>((size_t)b->nblk);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "batch CG workspace allocation failed");
  CgState& cs = c.cs;
  cs.rz = sd;
  cs.bb = sd + SM;
  cs.tol2 = sd + 2 * SM;
  cs.alpha = sd + 3 * SM;
  cs.beta = sd + 4 * SM;
  cs.rr = sd + 5 * SM;
  cs.partial = sd + 6 * SM;
  cs.done = c.si;
  cs.flags = c.si + SM;
  c.iter_dev = c.si + SM + 4;
  cs.iters = c.si + SM + 8;
  cs.hist_a = cs.hist_b = nullptr;
  cs.max_hist = 0;
  if (keep_hist) {
    cs.hist_a = sc.get<double>((size_t)c.max_iter * SM);
    cs.hist_b = sc.get<double>((size_t)c.max_iter * SM);
    if (sc.oom) return fail(ctx, GP2S_E_OOM, "batch CG history allocation failed");
    cs.max_hist = c.max_iter;
  }
  HIPCHK(hipEventCreateWithFlags(&c.ev[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c.ev[1], hipEventDisableTiming));
  gp2s_status s = order_after(ctx, ctx->stream, c.st);
  if (s) return s;
  HIPCHK(hipMemsetAsync(c.si, 0, (2 * (size_t)SM + 8) * sizeof(int32_t), c.st));
  const BatchGeom g = geom(b);
  if (c.bj)
    HIPCHK(launch_bbj_init(g, S, B, c.X, c.R, c.P, c.f32vec, b->bj_M, c.Z, cs, tol, c.st,
                           S == 1 && !c.probe ? b->bj_M32 : nullptr));
  else
    HIPCHK(launch_bcg_init(g, S, B, b->dinv, c.X, c.R, c.P, c.f32vec, cs, tol, c.st));
  if (tol_dev) {
    // per-column squared tolerances (refinement restarts)
    HIPCHK(hipMemcpyAsync(cs.tol2, tol_dev, SM * sizeof(double), hipMemcpyDeviceToDevice, c.st));
  }
  std::vector<int32_t> poll(SM + 4);
  s = bread(ctx, c.st, c.si, (SM + 4) * sizeof(int32_t), poll.data());
  if (s) return s;
  if (poll[SM + 2]) return fail(ctx, GP2S_E_NONFINITE, "non-finite right-hand side (%s)", c.label);
  int o = 0;
  for (int k = 0; k < SM; ++k) o += poll[k] == 0;
  c.open = o > 0;
  c.done.assign(poll.begin(), poll.begin() + SM);
  c.chunk = std::max(1, std::min(b->opts.check_every, c.max_iter));
  c.gc = g;
  if (c.open) return bcg_capture(c);
  return GP2S_OK;
}

// Evaluates a poll copy: errors, open columns, progress, and compaction of the grid.
gp2s_status bcg_eval(BCg& c, const int32_t* f, int at) {
  gp2s_batch b = c.b;
  gp2s_ctx ctx = b->ctx;
  const int S = c.S, SM = c.SM;
  if (f[SM + 0])
    return fail(ctx, GP2S_E_NOT_SPD, "CG breakdown in the batched %s (instance %d, column %d)", c.label,
                f[SM + 3] / S, f[SM + 3] % S);
  if (f[SM + 2]) return fail(ctx, GP2S_E_NONFINITE, "non-finite values during the batched %s", c.label);
  int o = 0;
  for (int k = 0; k < SM; ++k) o += f[k] == 0;
  c.open = o > 0;
  if (ctx->progress) ctx->progress(c.label, at, o, 0.0, ctx->progress_user);
  if (!c.open || c.it >= c.max_iter) return GP2S_OK;
  int64_t active = 0;
  for (int i = 0; i < b->M; ++i) {
    bool any = false;
    for (int k = 0; k < S; ++k) any = any || f[i * S + k] == 0;
    if (any) active += b->inst_h[i].nblk;
  }
  if (2 * active > c.gc.grid) return GP2S_OK;
  c.map.clear();
  for (int i = 0; i < b->M; ++i) {
    bool any = false;
    for (int k = 0; k < S; ++k) any = any || f[i * S + k] == 0;
    if (any)
      for (int64_t k = 0; k < b->inst_h[i].nblk; ++k) c.map.push_back((int32_t)(b->inst_h[i].blk0 + k));
  }
  // the replay in flight still reads the old map: let it finish first
  HIPCHK(hipStreamSynchronize(c.st));
  HIPCHK(hipMemcpyAsync(c.map_d, c.map.data(), c.map.size() * sizeof(int32_t), hipMemcpyHostToDevice, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  c.gc.blk_map = c.map_d;
  c.gc.grid = (int64_t)c.map.size();
  return bcg_capture(c);
}

bool bcg_active(const BCg& c) { return c.open && c.it < c.max_iter; }

// One replay of the chunk, then the lagged poll.
gp2s_status bcg_step(BCg& c) {
  gp2s_ctx ctx = c.b->ctx;
  HIPCHK(hipGraphLaunch(c.exec, c.st));
  c.it += c.chunk;
  if (c.nq > 0) {
    const int k = (c.nq - 1) & 1;
    HIPCHK(hipEventSynchronize(c.ev[k]));
    gp2s_status s = bcg_eval(c, c.slot(k), c.it - c.chunk);
    if (s) return s;
  }
  const int k = c.nq & 1;
  HIPCHK(hipMemcpyAsync(c.slot(k), c.si, (c.SM + 4) * sizeof(int32_t), hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipEventRecord(c.ev[k], c.st));
  ++c.nq;
  return GP2S_OK;
}

// Final flags and iteration counts; the context's stream then waits for this solve.
gp2s_status bcg_end(BCg& c) {
  gp2s_ctx ctx = c.b->ctx;
  const int SM = c.SM;
  std::vector<int32_t> f(SM + 4);
  gp2s_status s = bread(ctx, c.st, c.si, (SM + 4) * sizeof(int32_t), f.data());
  if (s) return s;
  if (c.it > 0) {
    gp2s_progress_fn keep = ctx->progress;
    ctx->progress = nullptr;
    s = bcg_eval(c, f.data(), c.it);
    ctx->progress = keep;
    if (s) return s;
  }
  c.iters.resize(SM);
  s = bread(ctx, c.st, c.cs.iters, SM * sizeof(int32_t), c.iters.data());
  if (s) return s;
  c.done.assign(f.begin(), f.begin() + SM);
  c.total = 0;
  for (int k = 0; k < SM; ++k) c.total = std::max(c.total, c.iters[k]);
  c.converged = !c.open;
  return order_after(ctx, c.st, ctx->stream);
}

// Runs one or two batched solves to completion, interleaving their replays.
gp2s_status bcg_drive(BCg* a, BCg* d) {
  for (;;) {
    const bool ra = a && bcg_active(*a), rd = d && bcg_active(*d);
    if (!ra && !rd) break;
    for (BCg* c : {a, d}) {
      if (!c || !bcg_active(*c)) continue;
      gp2s_status s = bcg_step(*c);
      if (s) return s;
    }
  }
  for (BCg* c : {a, d}) {
    if (!c) continue;
    gp2s_status s = bcg_end(*c);
    if (s) return s;
  }
  return GP2S_OK;
}

// A single batched solve on the y stream (refinement restarts).
gp2s_status run_bcg(gp2s_batch b, int S, const double* B, double* X, const double* tol_dev, double tol, bool keep_hist,
                    Scratch& sc, BCg& c, const char* label) {
  c.b = b;
  c.S = S;
  c.X = X;
  c.label = label;
  c.st = b->cap_stream;
  c.slots = b->pin;
  gp2s_status s = bcg_begin(c, B, tol_dev, tol, keep_hist, sc);
  if (s) return s;
  return bcg_drive(&c, nullptr);
}

// Time `reps` launches of a CG product with the given lane setting.
gp2s_status time_matvec(gp2s_batch b, int S, int lanes, Scratch& sc, float* ms) {
  gp2s_ctx ctx = b->ctx;
  const bool f32vec = b->prec == GP2S_MIXED && S > 1;
  const size_t vb = f32vec ? sizeof(float) : sizeof(double);
  void* P = sc.get<uint8_t>((size_t)b->N * S * vb);
  void* Q = sc.get<double>((size_t)b->N * S);
  double* sd = sc.get<double>(6 * (size_t)b->M * S + (size_t)b->nblk * S * 2);
  int32_t* si = sc.get<int32_t>(2 * (size_t)b->M * S + 8);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "autotune workspace allocation failed");
  hipStream_t st = ctx->stream;
  HIPCHK(hipMemsetAsync(P, 0, (size_t)b->N * S * vb, st));
  HIPCHK(hipMemsetAsync(sd, 0, (6 * (size_t)b->M * S + (size_t)b->nblk * S * 2) * sizeof(double), st));
  HIPCHK(hipMemsetAsync(si, 0, (2 * (size_t)b->M * S + 8) * sizeof(int32_t), st));
  CgState cs{};
  const int SM = b->M * S;
  cs.rz = sd;
  cs.alpha = sd + 3 * SM;
  cs.partial = sd + 6 * SM;
  cs.done = si;
  cs.flags = si + SM;
  const BatchGeom g = geom(b);
  HIPCHK(launch_bcg_matvec(b->prec, g, b->row_ptr, b->col, b->val, S, lanes, P, Q, f32vec, cs, st));
  hipEvent_t e0 = ev_get(ctx), e1 = ev_get(ctx);
  HIPCHK(hipEventRecord(e0, st));
  const int reps = 5;
  for (int r = 0; r < reps; ++r)
    HIPCHK(launch_bcg_matvec(b->prec, g, b->row_ptr, b->col, b->val, S, lanes, P, Q, f32vec, cs, st));
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float t = 0.f;
  HIPCHK(hipEventElapsedTime(&t, e0, e1));
  ctx->pool.push_back(e0);
  ctx->pool.push_back(e1);
  *ms = t / reps;
  return GP2S_OK;
}

BjBlocks bj_blocks(const gp2s_batch b) { return BjBlocks{b->bj_r0, b->bj_m, b->nblk}; }

// Factors the block-Jacobi preconditioner of the current values: the batch's row blocks
// (64 rows of one instance; the last block of an instance may be shorter). Arrays are
// allocated on first use and kept with the batch.
gp2s_status factor_blocks(gp2s_batch b) {
  gp2s_ctx ctx = b->ctx;
  hipStream_t st = ctx->stream;
  if (!b->bj_M) {
    const size_t nb = (size_t)b->nblk;
    b->bj_L = bown<double>(b, nb * kBJ * kBJ);
    b->bj_M = bown<double>(b, nb * kBJ * kBJ);
    b->bj_M32 = bown<float>(b, nb * kBJ * kBJ);
    b->bj_piv = bown<double>(b, (size_t)b->N);
    b->bj_r0 = bown<int64_t>(b, nb);
    b->bj_m = bown<int32_t>(b, nb);
    if (!b->bj_L || !b->bj_M || !b->bj_M32 || !b->bj_piv || !b->bj_r0 || !b->bj_m) {
      b->bj_M = nullptr;
      return fail(ctx, GP2S_E_OOM, "block preconditioner allocation failed (%zu blocks)", nb);
    }
    std::vector<int64_t> r0(nb);
    std::vector<int32_t> m(nb);
    for (int i = 0; i < b->M; ++i) {
      const BInst& I = b->inst_h[i];
      for (int64_t k = 0; k < I.nblk; ++k) {
        r0[I.blk0 + k] = I.row0 + k * kBRows;
        m[I.blk0 + k] = (int32_t)std::min<int64_t>(kBRows, I.rows - k * kBRows);
      }
    }
    HIPCHK(hipMemcpyAsync(b->bj_r0, r0.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->bj_m, m.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  Scratch sc(ctx);
  int32_t* bad = sc.get<int32_t>(1);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "allocation failed");
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
  HIPCHK(launch_bj_factor(b->N, b->row_ptr, b->col, b->val, b->prec, nullptr, 0, b->bj_L, b->bj_M, b->bj_M32, b->bj_piv, bad, st,
                          bj_blocks(b), kBJ));
  int32_t hb = 0;
  gp2s_status s = readback(ctx, bad, sizeof(hb), &hb);
  if (s) return s;
  if (hb) return fail(ctx, GP2S_E_NOT_SPD, "a diagonal block of K is not positive definite");
  return GP2S_OK;
}

gp2s_status check_batch_params(gp2s_ctx ctx, int M, const int64_t* n, const gp2s_params* p) {
  for (int i = 0; i < M; ++i) {
    gp2s_status s = gp2s_check_params(ctx, n[i], &p[i]);
    if (!s && (p[i].radii || p[i].ls_weights || p[i].ff_groups))
      s = fail(ctx, GP2S_E_INVALID, "instance %d: the batched path takes the stationary isotropic kernel only "
                                    "(radii, ls_weights and ff_groups must be NULL)", i);
    if (s) return fail(ctx, s, "instance %d: %s", i, ctx->err.c_str());
  }
  return GP2S_OK;
}

}  // namespace

extern "C" {

gp2s_status gp2s_batch_plan(gp2s_ctx ctx, int32_t n_inst, const int64_t* n, const double* const* x,
                            const gp2s_params* params, gp2s_precision prec, const gp2s_solve_opts* opts,
                            gp2s_batch* out) {
  if (!ctx) return GP2S_E_INVALID;
  if (!out) return fail(ctx, GP2S_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n_inst < 1 || n_inst > 65536) return fail(ctx, GP2S_E_INVALID, "n_inst must be in [1, 65536]");
  if (!n || !x || !params) return fail(ctx, GP2S_E_INVALID, "n, x and params must be non-NULL");
  if (prec != GP2S_FP64 && prec != GP2S_MIXED) return fail(ctx, GP2S_E_INVALID, "unknown precision");
  gp2s_status st = check_opts(ctx, opts, true);
  if (st) return st;
  const int S = opts->n_probes;
  if ((S & (S - 1)) != 0) return fail(ctx, GP2S_E_INVALID, "batched mode needs n_probes a power of two");
  st = check_batch_params(ctx, n_inst, n, params);
  if (st) return st;
  int64_t N = 0;
  for (int i = 0; i < n_inst; ++i) {
    if (!x[i]) return fail(ctx, GP2S_E_INVALID, "x[%d] is NULL", i);
    N += n[i];
  }
  if (N >= (int64_t)INT32_MAX || N * S >= (int64_t)INT32_MAX)
    return fail(ctx, GP2S_E_INVALID, "total points (times n_probes) must be below 2^31");
  st = ensure_device(ctx);
  if (st) return st;

  gp2s_batch b = new (std::nothrow) gp2s_batch_s();
  if (!b) return fail(ctx, GP2S_E_OOM, "host allocation failed");
  struct Guard {
    gp2s_batch b;
    bool keep = false;
    ~Guard() {
      if (!keep) gp2s_batch_free(b);
    }
  } guard{b};
  b->ctx = ctx;
  b->M = n_inst;
  b->prec = prec;
  b->S = S;
  b->opts = *opts;
  b->N = N;
  b->n.assign(n, n + n_inst);
  b->row0.resize(n_inst + 1);
  b->row0[0] = 0;
  for (int i = 0; i < n_inst; ++i) {
    b->row0[i + 1] = b->row0[i] + n[i];
    b->dim.push_back(params[i].dim);
    b->kern.push_back(params[i].kernel);
    b->P.push_back(params[i].n_bumps);
    b->cent0.push_back(b->Ptot);
    b->Ptot += params[i].n_bumps;
    b->radius.push_back(params[i].radius);
    b->width.push_back(params[i].bump_width);
    b->noise.push_back(params[i].noise_var);
    for (int k = 0; k < params[i].n_bumps; ++k) {
      for (int c = 0; c < 3; ++c) b->centers3.push_back(c < params[i].dim ? params[i].centers[k * params[i].dim + c] : 0.0);
      b->weights.push_back(params[i].weights[k]);
    }
    b->goff_h.push_back(i == 0 ? 0 : b->goff_h[i - 1] + params[i - 1].n_bumps + 2);
  }
  hipStream_t sm = ctx->stream;
  HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&b->cap2, hipStreamNonBlocking));
  HIPCHK(hipHostMalloc((void**)&b->pin, (2 * ((size_t)n_inst + 4) + 2 * ((size_t)n_inst * S + 4)) * sizeof(int32_t),
                       hipHostMallocDefault));
  b->x3 = bown<double>(b, (size_t)N * 3);
  b->inst_d = bown<BInst>(b, n_inst);
  b->row_start_d = bown<int64_t>(b, n_inst + 1);
  b->inst_of_row = bown<int32_t>(b, N);
  b->centers3_d = bown<double>(b, b->centers3.size());
  b->weights_d = bown<double>(b, b->weights.size());
  b->goff_d = bown<int32_t>(b, n_inst);
  b->perm = bown<int32_t>(b, N);
  b->x64 = bown<double>(b, (size_t)N * 3);
  b->g64 = bown<double>(b, N);
  b->binid = bown<int32_t>(b, N);
  b->row_ptr = bown<int64_t>(b, N + 1);
  b->diag = bown<double>(b, N);
  b->dinv = bown<double>(b, N);
  if (prec == GP2S_MIXED) b->pts32 = bown<float4>(b, N);
  else b->pts64 = bown<double4>(b, N);
  if (!b->x3 || !b->inst_d || !b->row_start_d || !b->inst_of_row || !b->centers3_d || !b->weights_d || !b->goff_d ||
      !b->perm || !b->x64 || !b->g64 || !b->binid || !b->row_ptr || !b->diag || !b->dinv ||
      (!b->pts32 && !b->pts64))
    return fail(ctx, GP2S_E_OOM, "batch allocation failed");
  HIPCHK(hipMemsetAsync(b->x3, 0, (size_t)N * 3 * sizeof(double), sm));
  for (int i = 0; i < n_inst; ++i)
    HIPCHK(hipMemcpy2DAsync(b->x3 + b->row0[i] * 3, 3 * sizeof(double), x[i], params[i].dim * sizeof(double),
                            params[i].dim * sizeof(double), n[i], hipMemcpyDeviceToDevice, sm));
  HIPCHK(hipMemcpyAsync(b->row_start_d, b->row0.data(), (n_inst + 1) * sizeof(int64_t), hipMemcpyHostToDevice, sm));
  HIPCHK(hipMemcpyAsync(b->centers3_d, b->centers3.data(), b->centers3.size() * sizeof(double),
                        hipMemcpyHostToDevice, sm));
  HIPCHK(hipMemcpyAsync(b->weights_d, b->weights.data(), b->weights.size() * sizeof(double), hipMemcpyHostToDevice,
                        sm));
  HIPCHK(hipMemcpyAsync(b->goff_d, b->goff_h.data(), n_inst * sizeof(int32_t), hipMemcpyHostToDevice, sm));

  // per-instance bounding boxes (fixed for the life of the plan)
  Scratch sc(ctx);
  double* part = sc.get<double>((size_t)n_inst * 6);
  int32_t* nonfinite = sc.get<int32_t>(1);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "allocation failed");
  HIPCHK(hipMemsetAsync(nonfinite, 0, sizeof(int32_t), sm));
  b->inst_h.assign(n_inst, BInst{});
  for (int i = 0; i < n_inst; ++i) {
    b->inst_h[i].row0 = b->row0[i];
    b->inst_h[i].rows = n[i];
  }
  HIPCHK(hipMemcpyAsync(b->inst_d, b->inst_h.data(), n_inst * sizeof(BInst), hipMemcpyHostToDevice, sm));
  BatchGeom g0{};
  g0.inst = b->inst_d;
  g0.M = n_inst;
  g0.row_start = b->row_start_d;
  g0.n = N;
  HIPCHK(launch_bbbox(b->x3, g0, part, nonfinite, sm));
  b->bbox.resize((size_t)n_inst * 6);
  int32_t nf = 0;
  st = readback(ctx, nonfinite, sizeof(int32_t), &nf);
  if (st) return st;
  if (nf) return fail(ctx, GP2S_E_NONFINITE, "x contains NaN or infinity");
  {
    std::vector<double> tmp((size_t)n_inst * 6);
    HIPCHK(hipMemcpy(tmp.data(), part, tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
    b->bbox = tmp;
  }

  // Autotune 1: bin refinement (bins of side r or r / 2) by the count-pass time.
  b->cap = 0;
  float best = 1e30f;
  int best_m = 1;
  for (int m = 1; m <= 2; ++m) {
    build_grids(b, m);
    if (m == 1) {
      b->blk_inst = bown<int32_t>(b, b->nblk);
      OOMCHK(b->blk_inst);
      std::vector<int32_t> bi(b->nblk);
      for (int i = 0; i < n_inst; ++i)
        for (int64_t k = 0; k < b->inst_h[i].nblk; ++k) bi[b->inst_h[i].blk0 + k] = i;
      HIPCHK(hipMemcpyAsync(b->blk_inst, bi.data(), b->nblk * sizeof(int32_t), hipMemcpyHostToDevice, sm));
    }
    float ms = 0.f;
    Scratch sc2(ctx);
    st = assemble_pattern(b, sc2, nullptr, &ms);
    if (st) return st;
    b->tune_ms[m - 1] = ms;
    if (ms < best) {
      best = ms;
      best_m = m;
    }
  }
  b->m_ref = best_m;
  build_grids(b, best_m);
  {
    Scratch sc2(ctx);
    st = assemble_pattern(b, sc2, nullptr, nullptr);
    if (st) return st;
  }
  b->cap = (int64_t)std::ceil((double)b->nnz * b->capacity_factor) + 1024;
  b->col = bown<int32_t>(b, b->cap);
  b->val = prec == GP2S_MIXED ? (void*)bown<float>(b, b->cap) : (void*)bown<double>(b, b->cap);
  OOMCHK(b->col);
  OOMCHK(b->val);
  {
    Scratch sc2(ctx);
    st = assemble_fill(b, sc2);
    if (st) return st;
  }
  // Autotune 2: lanes per row of the single-RHS product and of the probe block product.
  {
    Scratch sc2(ctx);
    float bt = 1e30f;
    for (int G = 4; G <= 32; G *= 2) {
      float ms = 0.f;
      st = time_matvec(b, 1, G, sc2, &ms);
      if (st) return st;
      if (ms < bt) {
        bt = ms;
        b->spmv_lanes = G;
      }
    }
    b->tune_ms[2] = bt;
    bt = 1e30f;
    std::vector<int> cand;
    for (int L = S; L <= 64; L *= 2) cand.push_back(L);
    if (S == 8 || S == 16 || S == 32 || S == 64) cand.push_back(1);
    for (int G = 4; G <= 16; G *= 2)
      if (entry_product_ok(S, G)) cand.push_back(-G);
    for (int L : cand) {
      float ms = 0.f;
      st = time_matvec(b, S, L, sc2, &ms);
      if (st) return st;
      if (ms < bt) {
        bt = ms;
        b->spmm_lanes = L;
      }
    }
    b->tune_ms[3] = bt;
  }
  HIPCHK(hipStreamSynchronize(sm));
  guard.keep = true;
  *out = b;
  return GP2S_OK;
}

gp2s_status gp2s_batch_info(gp2s_batch b, int64_t* n_total, int64_t* nnz, int64_t* capacity, int32_t* tuned) {
  if (!b) return GP2S_E_INVALID;
  if (n_total) *n_total = b->N;
  if (nnz) *nnz = b->nnz;
  if (capacity) *capacity = b->cap;
  if (tuned) {
    tuned[0] = b->m_ref;
    tuned[1] = b->spmv_lanes;
    tuned[2] = b->spmm_lanes;
  }
  return GP2S_OK;
}

gp2s_status gp2s_batch_run(gp2s_batch b, const double* const* y, const gp2s_params* params, double* lml,
                           double* const* grad, gp2s_report* reports) {
  if (!b) return GP2S_E_INVALID;
  gp2s_ctx ctx = b->ctx;
  if (!y || !lml) return fail(ctx, GP2S_E_INVALID, "y and lml must be non-NULL");
  const int M = b->M, S = b->S;
  for (int i = 0; i < M; ++i)
    if (!y[i]) return fail(ctx, GP2S_E_INVALID, "y[%d] is NULL", i);
  hipStream_t sm = ctx->stream;
  gp2s_status st = GP2S_OK;
  // new hyperparameters: same geometry (dimension, bump count, centres, width), new r, weights, noise
  if (params) {
    st = check_batch_params(ctx, M, b->n.data(), params);
    if (st) return st;
    for (int i = 0; i < M; ++i) {
      if (params[i].dim != b->dim[i] || params[i].n_bumps != b->P[i] || params[i].bump_width != b->width[i] ||
          params[i].kernel != b->kern[i])
        return fail(ctx, GP2S_E_INVALID, "instance %d: dimension, bump count, width and kernel are fixed by the plan",
                    i);
      for (int k = 0; k < b->P[i] * b->dim[i]; ++k)
        if (params[i].centers[k] != b->centers3[(size_t)(b->cent0[i] + k / b->dim[i]) * 3 + k % b->dim[i]])
          return fail(ctx, GP2S_E_INVALID, "instance %d: bump centres are fixed by the plan", i);
      b->radius[i] = params[i].radius;
      b->noise[i] = params[i].noise_var;
      for (int k = 0; k < b->P[i]; ++k) b->weights[b->cent0[i] + k] = params[i].weights[k];
    }
    HIPCHK(hipMemcpyAsync(b->weights_d, b->weights.data(), b->weights.size() * sizeof(double),
                          hipMemcpyHostToDevice, sm));
    build_grids(b, b->m_ref);
    Scratch sc2(ctx);
    st = assemble_pattern(b, sc2, nullptr, nullptr);
    if (st) return st;
    st = assemble_fill(b, sc2);
    if (st) return st;
  }
  if (pc_block(b->opts.precond)) {
    st = factor_blocks(b);
    if (st) return st;
  }
  const int64_t N = b->N;
  const BatchGeom g = geom(b);
  Scratch sc(ctx);
  // every exit waits for the solve streams before the workspace is released
  struct StreamsIdle {
    gp2s_batch b;
    ~StreamsIdle() {
      (void)hipStreamSynchronize(b->cap_stream);
      (void)hipStreamSynchronize(b->cap2);
    }
  } idle{b};
  double* yu = sc.get<double>(N);
  double* yi = sc.get<double>(N);
  double* ai = sc.get<double>(N);
  double* r = sc.get<double>(N);
  double* kx = sc.get<double>(N);
  double* d = sc.get<double>(N);
  double* seg = sc.get<double>(4 * (size_t)M);
  double* tolv = sc.get<double>(M);
  double* Qs = sc.get<double>((size_t)N * S);
  double* Bp = sc.get<double>((size_t)N * S);
  uint64_t* mask = sc.get<uint64_t>(N);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "batch run workspace allocation failed");
  for (int i = 0; i < M; ++i)
    HIPCHK(hipMemcpyAsync(yu + b->row0[i], y[i], b->n[i] * sizeof(double), hipMemcpyDeviceToDevice, sm));
  HIPCHK(launch_gather_rows(N, 1, b->perm, yu, yi, sm));
  // y solves, then refinement restarts for instances above the tolerance
  std::vector<double> bb(M), rr(M), resid(M, 0.0);
  HIPCHK(launch_bseg_reduce(g, 0, yi, nullptr, seg, sm));
  st = bread(ctx, sm, seg, M * sizeof(double), bb.data());
  if (st) return st;
  for (int i = 0; i < M; ++i)
    if (!is_fin(bb[i])) return fail(ctx, GP2S_E_NONFINITE, "y[%d] contains NaN or infinity", i);
  // The probe block runs on its own stream beside the y solves (both start after the
  // work queued so far on the context's stream and are joined back into it).
  const bool bj = pc_block(b->opts.precond);
  // trace vectors of the gradient: L^-T z (block preconditioner; the probe solve's first z)
  double* W = bj ? sc.get<double>((size_t)N * S) : nullptr;
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "batch run workspace allocation failed");
  HIPCHK(launch_bprobe_masks(g, b->perm, b->opts.seed, S, mask, sm));
  if (bj)
    HIPCHK(launch_bj_rhs(N, S, mask, b->bj_L, Bp, sm, bj_blocks(b), kBJ));
  else
    HIPCHK(launch_probe_rhs(N, S, mask, b->diag, Bp, sm));
  BCg cy, pr;
  cy.b = pr.b = b;
  cy.S = 1;
  cy.X = ai;
  cy.label = "y solve";
  cy.st = b->cap_stream;
  cy.slots = b->pin;
  pr.S = S;
  pr.probe = true;
  pr.X = Qs;
  pr.label = "probe block";
  pr.st = b->cap2;
  pr.slots = b->pin + 2 * ((size_t)M + 4);
  st = bcg_begin(pr, Bp, nullptr, b->opts.probe_tol, true, sc);
  if (st) return st;
  // z_0 = M^-1 L z = L^-T z, before the first iteration overwrites it
  if (bj) HIPCHK(hipMemcpyAsync(W, pr.Z, (size_t)N * S * sizeof(double), hipMemcpyDeviceToDevice, pr.st));
  st = bcg_begin(cy, yi, nullptr, b->opts.tol, false, sc);
  if (st) return st;
  st = bcg_drive(&cy, &pr);
  if (st) return st;
  std::vector<int> iters_y(M, 0), ir(M, 0);
  for (int i = 0; i < M; ++i) iters_y[i] = cy.iters[i];
  bool conv = false;
  for (int step = 0;; ++step) {
    HIPCHK(launch_spmv(b->prec, b->row_ptr, b->col, b->val, N, (double)b->nnz / N, ai, kx, sm));
    HIPCHK(launch_axpy_sub(N, yi, kx, r, sm));
    HIPCHK(launch_bseg_reduce(g, 0, r, nullptr, seg, sm));
    st = bread(ctx, sm, seg, M * sizeof(double), rr.data());
    if (st) return st;
    conv = true;
    std::vector<double> tl(M);
    for (int i = 0; i < M; ++i) {
      resid[i] = bb[i] > 0 ? std::sqrt(rr[i] / bb[i]) : 0.0;
      const bool ok = resid[i] <= b->opts.tol;
      conv = conv && ok;
      const double t = ok ? 0.999 : std::min(0.5, 0.5 * b->opts.tol / resid[i]);
      tl[i] = t * t;
    }
    if (conv || step >= b->opts.max_ir) break;
    for (int i = 0; i < M; ++i)
      if (resid[i] > b->opts.tol) ir[i] += 1;
    HIPCHK(hipMemcpyAsync(tolv, tl.data(), M * sizeof(double), hipMemcpyHostToDevice, sm));
    BCg r2;
    st = run_bcg(b, 1, r, d, tolv, b->opts.tol, false, sc, r2, "refinement solve");
    if (st) return st;
    for (int i = 0; i < M; ++i) iters_y[i] += r2.iters[i];
    HIPCHK(launch_add(N, ai, d, sm));
  }
  // the quadrature
  const int SM = M * S;
  const int64_t max_m = std::max(1, pr.total);
  double* work = sc.get<double>((size_t)2 * SM * max_m);
  double* quad = sc.get<double>(SM);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "quadrature workspace allocation failed");
  HIPCHK(launch_slq_ws(SM, pr.cs.hist_a, pr.cs.hist_b, pr.cs.iters, work, max_m, quad, sm));
  std::vector<double> qh(SM), sumlog(M), yta(M);
  st = bread(ctx, sm, quad, SM * sizeof(double), qh.data());
  if (st) return st;
  HIPCHK(launch_bseg_reduce(g, 1, bj ? b->bj_piv : b->diag, nullptr, seg, sm));  // ln|M|
  st = bread(ctx, sm, seg, M * sizeof(double), sumlog.data());
  if (st) return st;
  HIPCHK(launch_bseg_reduce(g, 0, yi, ai, seg, sm));
  st = bread(ctx, sm, seg, M * sizeof(double), yta.data());
  if (st) return st;
  for (int i = 0; i < M; ++i) {
    double mean = 0.0, var = 0.0;
    for (int s = 0; s < S; ++s) mean += (double)b->n[i] * qh[i * S + s];
    mean /= S;
    for (int s = 0; s < S; ++s) {
      const double v = (double)b->n[i] * qh[i * S + s] - mean;
      var += v * v;
    }
    const double logdet = sumlog[i] + mean;
    lml[i] = -0.5 * yta[i] - 0.5 * logdet - 0.5 * (double)b->n[i] * std::log(2.0 * M_PI);
    if (reports) {
      gp2s_report& rp = reports[i];
      std::memset(&rp, 0, sizeof(rp));
      rp.lml = lml[i];
      rp.logdet = logdet;
      rp.yTa = yta[i];
      rp.resid = resid[i];
      rp.logdet_stderr = S > 1 ? std::sqrt(var / (S - 1) / S) : 0.0;
      rp.iters = iters_y[i];
      int pm = 0;
      for (int s = 0; s < S; ++s) pm = std::max(pm, pr.iters[i * S + s]);
      rp.probe_iters = pm;
      rp.ir_steps = ir[i];
      rp.n_probes = S;
    }
  }
  if (grad) {
    double* Rr = sc.get<double>(N);
    double* Tr = sc.get<double>(N);
    double* Ur = sc.get<double>(N);
    const int total = b->goff_h[M - 1] + b->P[M - 1] + 2;
    double* gd = sc.get<double>(total);
    if (sc.oom) return fail(ctx, GP2S_E_OOM, "gradient workspace allocation failed");
    BBackward bw{};
    bw.g = g;
    bw.rp = b->row_ptr;
    bw.col = b->col;
    bw.pts32 = b->pts32;
    bw.pts64 = b->pts64;
    bw.a = ai;
    bw.Q = Qs;
    bw.mask = mask;
    bw.dinv = b->dinv;
    bw.W = W;
    bw.g64 = b->g64;
    bw.S = S;
    HIPCHK(launch_bbackward_rows(bw, b->prec, Rr, Tr, Ur, sm));
    HIPCHK(launch_bgrad_reduce(g, S, b->x64, b->g64, ai, Rr, Tr, Ur, b->centers3_d, b->goff_d, gd, sm));
    std::vector<double> gh(total);
    HIPCHK(hipMemcpyAsync(gh.data(), gd, total * sizeof(double), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipStreamSynchronize(sm));
    for (int i = 0; i < M; ++i)
      if (grad[i]) std::memcpy(grad[i], gh.data() + b->goff_h[i], (b->P[i] + 2) * sizeof(double));
  }
  HIPCHK(hipStreamSynchronize(sm));
  if (!conv || !pr.converged)
    return fail(ctx, GP2S_E_NOCONV, "batched CG did not converge within max_iter (y: %s, probes: %s)",
                conv ? "yes" : "no", pr.converged ? "yes" : "no");
  return GP2S_OK;
}

gp2s_status gp2s_batch_free(gp2s_batch b) {
  if (!b) return GP2S_E_INVALID;
  if (b->ctx) {
    (void)hipStreamSynchronize(b->ctx->stream);
    if (b->cap_stream) (void)hipStreamSynchronize(b->cap_stream);
    if (b->cap2) (void)hipStreamSynchronize(b->cap2);
    for (void* q : b->owned) dfree(b->ctx, q);
  }
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->cap2) (void)hipStreamDestroy(b->cap2);
  if (b->pin) (void)hipHostFree(b->pin);
  delete b;
  return GP2S_OK;
}

}  // extern "C"
