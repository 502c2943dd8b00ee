// Host runtime and C ABI of libgp2s: argument validation, contexts and matrix
// handles, and the orchestration of the device kernels for assembly, products,
// solves, the log marginal likelihood and its gradient.
#include <mutex>

#include "runtime.h"

using namespace gp2s;

namespace {

using namespace gp2s::rt;

// Readies a new matrix handle's CSR for the streaming single-RHS product: zeroes the
// kQuadPad entries past nnz of col and val (column 0, value 0), which it may read, and
// builds its row blocks (m->rowblk must hold rowblocks_count(nnz) + 1 entries).
hipError_t prepare_streaming(gp2s_matrix m, hipStream_t st) {
  const size_t vb = m->prec == GP2S_MIXED ? sizeof(float) : sizeof(double);
  hipError_t e = hipMemsetAsync(m->col + m->nnz, 0, kQuadPad * sizeof(int32_t), st);
  if (e == hipSuccess) e = hipMemsetAsync(static_cast<char*>(m->val) + m->nnz * vb, 0, kQuadPad * vb, st);
  if (e == hipSuccess) e = launch_rowblocks(m->row_ptr, m->n, m->nnz, m->rowblk, st);
  return e;
}

RowBlocks row_blocks(gp2s_matrix m) { return RowBlocks{m->rowblk, m->nrowblk}; }

// ---- conjugate gradients ------------------------------------------------------------------
struct CgRun {
  CgState cs{};
  int32_t host_iters[kMaxProbes] = {};
  int32_t total_iters = 0;  // iterations executed (longest column)
  bool converged = false;
};

// Preconditioned CG (diagonal or block-Jacobi) for K X = B over S columns (internal
// order) on stream `st`, driven one
// iteration at a time so that two solves can be interleaved on two streams. The host
// polls the per-column done flags without stalling the stream: every check_every
// iterations it queues an asynchronous copy of the flags into a pinned slot plus an
// event, and evaluates the copy queued one check earlier (whose event has long
// completed). Converged columns make the extra iterations no-ops (alpha = 0, p kept).
struct Cg {
  gp2s_ctx ctx = nullptr;
  gp2s_matrix m = nullptr;
  int S = 1;
  double* X = nullptr;
  int max_iter = 0, check_every = 16;
  const char* label = "";
  hipStream_t st = nullptr;
  int slot0 = 0;  // first of this solve's two pinned poll slots
  int precond = GP2S_PRECOND_JACOBI;
  bool probe = false;  // a probe solve: its preconditioner enters the estimators (float64 M^-1 always)
  // state
  CgState cs{};
  bool f32vec = false;
  int variant = 0;
  double* R = nullptr;
  double* Z = nullptr;  // M^-1 r (block preconditioner)
  float* Z32 = nullptr;  // the same in float32 after the first iteration (mixed probe block)
  double* lrC = nullptr;     // far-field kernel: G^T p [U * S]
  double* lrPart = nullptr;  // its per-workgroup partials
  uint32_t* lrTicket = nullptr;
  void* P = nullptr;
  void* Q = nullptr;
  int32_t* si = nullptr;
  int it = 0;          // iterations queued
  int polled_it = -1;  // iteration count of the poll in flight (-1: none)
  hipEvent_t ev[2] = {nullptr, nullptr};
  int nq = 0;  // polls queued
  bool open = true;
  int32_t host_iters[kMaxProbes] = {};
  int32_t total_iters = 0;
  bool converged = false;

  int32_t* slot(int k) const {
    return reinterpret_cast<int32_t*>(static_cast<char*>(ctx->pinned) + kReadbackBytes + (slot0 + k) * kPollSlot);
  }
  ~Cg() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// Row tiles of about kTileRows bin-sorted rows inside one bin row (band) of the grid, at
// most kTileMaxRows each, with the column intervals of the neighbouring bins: for every
// neighbouring band, the bins from one before the tile's first bin to one after its
// last are consecutive in bin order, so their points form one run of columns. Built on
// the host from bin_start, once per assembled matrix.
constexpr int kTileRows = 32;
constexpr int64_t kTileMaxBins = int64_t(1) << 23;

gp2s_status ensure_tiles(gp2s_ctx ctx, gp2s_matrix m) {
  if (m->tiles_tried) return GP2S_OK;
  m->tiles_tried = true;
  if (!m->assembled || !m->bin_start || m->grid.nbins < 1 || m->grid.nbins > kTileMaxBins) return GP2S_OK;
  const GridDev& g = m->grid;
  std::vector<int64_t> bs((size_t)g.nbins + 1);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipMemcpy(bs.data(), m->bin_start, bs.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  const int nb0 = g.nb[0], nb1 = g.dim >= 2 ? g.nb[1] : 1, nb2 = g.dim == 3 ? g.nb[2] : 1;
  std::vector<RowTile> tiles;
  tiles.reserve((size_t)(m->n / kTileRows) + 16);
  for (int bz = 0; bz < nb2; ++bz)
    for (int by = 0; by < nb1; ++by) {
      const int64_t band = (int64_t)nb0 * (by + (int64_t)nb1 * bz);
      int bx = 0;
      while (bx < nb0) {
        const int b0 = bx;
        int64_t rows = 0;
        while (bx < nb0 && rows < kTileRows) {
          rows += bs[band + bx + 1] - bs[band + bx];
          ++bx;
        }
        if (rows == 0) continue;
        const int b1 = bx - 1;
        RowTile T{};
        T.niv = 0;
        for (int dz = (g.dim == 3 ? -1 : 0); dz <= (g.dim == 3 ? 1 : 0); ++dz)
          for (int dy = -1; dy <= 1; ++dy) {
            const int yy = by + dy, zz = bz + dz;
            if (yy < 0 || yy >= nb1 || zz < 0 || zz >= nb2) continue;
            const int64_t nband = (int64_t)nb0 * (yy + (int64_t)nb1 * zz);
            const int64_t lo = bs[nband + std::max(b0 - 1, 0)];
            const int64_t hi = bs[nband + std::min(b1 + 1, nb0 - 1) + 1];
            if (hi > lo && T.niv < kTileMaxIv) {
              T.lo[T.niv] = (int32_t)lo;
              T.len[T.niv] = (int32_t)(hi - lo);
              ++T.niv;
            }
          }
        const int64_t r0 = bs[band + b0];
        for (int64_t c = 0; c < rows; c += kTileMaxRows) {
          T.row0 = r0 + c;
          T.rows = (int32_t)std::min<int64_t>(kTileMaxRows, rows - c);
          tiles.push_back(T);
        }
      }
    }
  if (tiles.empty()) return GP2S_OK;
  RowTile* d = own<RowTile>(m, tiles.size());
  if (!d) return GP2S_OK;  // no room: the other block products remain
  HIPCHK(hipMemcpyAsync(d, tiles.data(), tiles.size() * sizeof(RowTile), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  m->tiles = d;
  m->ntiles = (int64_t)tiles.size();
  return GP2S_OK;
}

// Builds the row-grouped copy (pattern once; values again after a refill). Skipped
// (variant 3 unavailable) when it would not fit in memory or in 32-bit slots.
gp2s_status ensure_groups(gp2s_ctx ctx, gp2s_matrix m) {
  hipStream_t st = ctx->stream;
  const int64_t n = m->n;
  const int64_t ng = (n + kGrp - 1) / kGrp;
  if (!m->grp_tried) {
    m->grp_tried = true;
    Scratch sc(ctx);
    int32_t* cnt = sc.get<int32_t>(ng);
    void* ws = sc.get<uint8_t>(scan_workspace_bytes(ng));
    int64_t* gp = own<int64_t>(m, ng + 1);
    if (sc.oom || !gp) return GP2S_OK;
    HIPCHK(launch_grp_count(n, m->row_ptr, m->col, ng, cnt, st));
    HIPCHK(launch_exscan_i32_i64(cnt, gp, ng, ws, st));
    int64_t tot = 0;
    gp2s_status s = readback(ctx, gp + ng, sizeof(int64_t), &tot);
    if (s) return s;
    if (tot * kGrp >= (int64_t)INT32_MAX) return GP2S_OK;
    int32_t* gc = own<int32_t>(m, std::max<int64_t>(tot, 1));
    int32_t* mp = own<int32_t>(m, std::max<int64_t>(m->nnz, 1));
    void* gv = m->prec == GP2S_MIXED ? (void*)own<float>(m, std::max<int64_t>(tot * kGrp, 1))
                                     : (void*)own<double>(m, std::max<int64_t>(tot * kGrp, 1));
    if (!gc || !mp || !gv) return GP2S_OK;
    HIPCHK(launch_grp_fill(n, m->row_ptr, m->col, ng, gp, gc, mp, st));
    m->grp_ptr = gp;
    m->grp_col = gc;
    m->grp_val = gv;
    m->grp_map = mp;
    m->grp_n = tot;
  }
  if (m->grp_ptr && !m->grp_values) {
    const size_t vb = m->prec == GP2S_MIXED ? sizeof(float) : sizeof(double);
    HIPCHK(hipMemsetAsync(m->grp_val, 0, (size_t)m->grp_n * kGrp * vb, st));
    HIPCHK(launch_grp_values(m->nnz, m->val, m->prec, m->grp_map, m->grp_val, st));
    m->grp_values = true;
  }
  return GP2S_OK;
}

// Dense diagonal blocks and per-row in-block runs of the block-split product (variant 5),
// built on first use; after a refill only the block values are rewritten. 64 float32 (or
// float64) values per row.
gp2s_status ensure_bsplit(gp2s_ctx ctx, gp2s_matrix m) {
  hipStream_t st = ctx->stream;
  if (!m->bs_tried) {
    m->bs_tried = true;
    const size_t nblk = (size_t)((m->n + kBJ - 1) / kBJ);
    void* bv = m->prec == GP2S_MIXED ? (void*)own<float>(m, nblk * kBJ * kBJ) : (void*)own<double>(m, nblk * kBJ * kBJ);
    int2* seg = own<int2>(m, (size_t)m->n);
    if (!bv || !seg) return GP2S_OK;  // the variant is simply not offered
    HIPCHK(launch_bs_build(m->n, m->row_ptr, m->col, m->val, m->prec, bv, seg, false, st));
    m->bs_val = bv;
    m->bs_seg = seg;
    m->bs_values = true;
  }
  if (m->bs_val && !m->bs_values) {
    HIPCHK(launch_bs_build(m->n, m->row_ptr, m->col, m->val, m->prec, m->bs_val, m->bs_seg, true, st));
    m->bs_values = true;
  }
  return GP2S_OK;
}

TileSet tile_set(gp2s_matrix m) {
  TileSet t;
  t.t = m->tiles;
  t.n = m->ntiles;
  if (m->grp_ptr && m->grp_values) {
    t.gptr = m->grp_ptr;
    t.gcol = m->grp_col;
    t.gval = m->grp_val;
    t.ngroups = (m->n + kGrp - 1) / kGrp;
  }
  if (m->bs_val && m->bs_values) {
    t.bval = m->bs_val;
    t.bseg = m->bs_seg;
  }
  return t;
}

// Chooses the block product for S columns of this matrix by timing each variant on the
// first CG product (the product and its alpha are recomputed by the first iteration).
gp2s_status tune_block_product(gp2s_ctx ctx, gp2s_matrix m, int S, const void* P, void* Q, bool f32vec,
                               const CgState& cs, hipStream_t st) {
  std::vector<int> cand{0};
  if (S == 8 || S == 16 || S == 32 || S == 64) {
    cand.push_back(1);
    cand.push_back(6);
    gp2s_status ts = ensure_tiles(ctx, m);
    if (ts) return ts;
    if (m->tiles) cand.push_back(2);
    if (S == 32 || S == 64) {
      ts = ensure_groups(ctx, m);
      if (ts) return ts;
      if (m->grp_ptr) cand.push_back(3);
    }
    // The block split (variant 5) is not a candidate: measured slower than the column
    // slices (see bsplit.hip), and its dense blocks cost 64 values per row. It can be pinned.
  }
  for (int G = 4; G <= 16; G *= 2)
    if (entry_product_ok(S, G)) cand.push_back(G);
  if (cand.size() == 1) {
    m->spmm_variant[S] = 0;
    return GP2S_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ctx, GP2S_E_HIP, "hipEventCreate failed");
  }
  const double mean_row = (double)m->nnz / (double)m->n;
  // Two rounds over the candidates, each timing one warm and three measured launches;
  // a candidate's time is its better round. The y solve runs beside the probe block on
  // the other stream, so a single round can favour whichever candidate happened to
  // overlap its lighter kernels.
  std::vector<float> best_ms(cand.size(), 1e30f);
  hipError_t err = hipSuccess;
  for (int round = 0; round < 2 && err == hipSuccess; ++round) {
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      const int v = cand[ci];
      err = launch_cg_matvec(m->prec, m->row_ptr, m->col, m->val, m->n, S, mean_row, v, tile_set(m), P, Q, f32vec,
                             cs, st, row_blocks(m));
      if (err == hipSuccess) err = hipEventRecord(e0, st);
      for (int r = 0; r < 3 && err == hipSuccess; ++r)
        err = launch_cg_matvec(m->prec, m->row_ptr, m->col, m->val, m->n, S, mean_row, v, tile_set(m), P, Q, f32vec,
                               cs, st, row_blocks(m));
      if (err == hipSuccess) err = hipEventRecord(e1, st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) break;
      best_ms[ci] = std::min(best_ms[ci], ms);
    }
  }
  int pick = 0;
  float best = 1e30f;
  for (size_t ci = 0; ci < cand.size(); ++ci)
    if (best_ms[ci] < best) {
      best = best_ms[ci];
      pick = cand[ci];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(ctx, GP2S_E_HIP, "timing the block products: %s", hipGetErrorString(err));
  m->spmm_variant[S] = pick;
  return GP2S_OK;
}

// Builds the block-Jacobi factor of the handle's current values if it is not there
// (on the context's stream; synchronous, since a block that is not positive definite
// is reported here).
// The float32 copy of M^-1 serves single-column solves that are not probe solves (their
// preconditioner only steers convergence); everything else applies the float64 one.
const float* bj_m32(const Cg& c) { return c.S == 1 && !c.probe ? c.m->bj[pc_idx(c.precond)].M32 : nullptr; }

gp2s_status ensure_bj(gp2s_ctx ctx, gp2s_matrix m, int precond) {
  auto& f = m->bj[pc_idx(precond)];
  if (f.ready) return GP2S_OK;
  const int64_t n = m->n;
  const int B = pc_rows(precond);
  const size_t nblk = (size_t)((n + B - 1) / B);
  if (!f.L) {
    f.L = own<double>(m, nblk * B * B);
    f.M = own<double>(m, nblk * B * B);
    f.M32 = own<float>(m, nblk * B * B);
    f.piv = own<double>(m, (size_t)n);
    if (!f.L || !f.M || !f.M32 || !f.piv) return fail(ctx, GP2S_E_OOM, "block preconditioner allocation failed");
  }
  Scratch sc(ctx);
  int32_t* bad = sc.get<int32_t>(1);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "block preconditioner workspace allocation failed");
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int32_t), ctx->stream));
  HIPCHK(launch_bj_factor(n, m->row_ptr, m->col, m->val, m->prec, m->ffG, m->ffU, f.L, f.M, f.M32, f.piv, bad,
                          ctx->stream, BjBlocks{nullptr, nullptr, 0}, B));
  int32_t hb = 0;
  gp2s_status st = readback(ctx, bad, sizeof(int32_t), &hb);
  if (st) return st;
  if (hb)
    return fail(ctx, GP2S_E_NOT_SPD,
                "a %d-point diagonal block of K is not positive definite (Cholesky pivot <= 0 in float64)", B);
  f.ready = true;
  return GP2S_OK;
}

// Allocates the workspace, initialises the state and reads the initial flags.
gp2s_status cg_begin(Cg& c, const double* B, double tol, bool keep_hist, Scratch& sc) {
  gp2s_ctx ctx = c.ctx;
  gp2s_matrix m = c.m;
  const int S = c.S;
  const int64_t n = m->n;
  const size_t nS = (size_t)n * S;
  // Probe blocks of the mixed path keep search directions in float32 (products, x,
  // r, dot products and all coefficients stay float64). The far-field kernel keeps
  // them in float64: its global rank-U term makes the Lanczos coefficients sensitive
  // enough to the rounding of the directions that the same-probe log-determinant
  // came within 6% of its 1e-8 bar.
  c.f32vec = m->prec == GP2S_MIXED && S > 1 && !m->ffG;
  const size_t vb = c.f32vec ? sizeof(float) : sizeof(double);
  c.R = sc.get<double>(nS);
  if (pc_block(c.precond)) c.Z = sc.get<double>(nS);
  if (pc_block(c.precond) && c.f32vec) c.Z32 = sc.get<float>(nS);
  if (m->ffG) {
    c.lrC = sc.get<double>((size_t)m->ffU * S);
    c.lrPart = sc.get<double>((size_t)m->ffU * S * ff_gtp_blocks(n));
    c.lrTicket = sc.get<uint32_t>(1);
  }
  c.P = sc.get<uint8_t>(nS * vb);
  c.Q = sc.get<double>(nS);
  double* sd = sc.get<double>(6 * S + (size_t)kReduceBlocks * S * 2);
  c.si = sc.get<int32_t>(2 * S + 4);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "CG workspace allocation failed");
  CgState& cs = c.cs;
  cs.rz = sd;
  cs.bb = sd + S;
  cs.tol2 = sd + 2 * S;
  cs.alpha = sd + 3 * S;
  cs.beta = sd + 4 * S;
  cs.rr = sd + 5 * S;
  cs.partial = sd + 6 * S;
  cs.done = c.si;
  cs.flags = c.si + S;
  cs.iters = c.si + S + 4;
  cs.hist_a = cs.hist_b = nullptr;
  cs.max_hist = 0;
  if (keep_hist) {
    cs.hist_a = sc.get<double>((size_t)c.max_iter * S);
    cs.hist_b = sc.get<double>((size_t)c.max_iter * S);
    if (sc.oom) return fail(ctx, GP2S_E_OOM, "CG history allocation failed");
    cs.max_hist = c.max_iter;
  }
  HIPCHK(hipEventCreateWithFlags(&c.ev[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c.ev[1], hipEventDisableTiming));
  HIPCHK(hipMemsetAsync(c.si, 0, (2 * S + 4) * sizeof(int32_t), c.st));
  if (m->ffG) {
    HIPCHK(hipMemsetAsync(c.lrC, 0, (size_t)m->ffU * S * sizeof(double), c.st));
    HIPCHK(hipMemsetAsync(c.lrTicket, 0, sizeof(uint32_t), c.st));
    cs.lrC = c.lrC;
    cs.lrU = m->ffU;
  }
  if (pc_block(c.precond)) {
    const auto& f = m->bj[pc_idx(c.precond)];
    const int rows = pc_rows(c.precond);
    if (!f.ready) return fail(ctx, GP2S_E_INVALID, "block preconditioner not built (%s)", c.label);
    HIPCHK(launch_bj_update(n, S, B, c.X, c.R, nullptr, nullptr, c.f32vec, f.M, c.Z, cs, c.st, bj_m32(c), nullptr,
                            rows));
    HIPCHK(launch_cg_init_fin(cs, (int)bj_update_blocks(n, rows), S, tol, c.st));
    HIPCHK(launch_copy_dir(n, S, c.Z, c.P, c.f32vec, c.st));
  } else {
    HIPCHK(launch_cg_init(n, S, B, m->dinv, c.X, c.R, c.P, c.f32vec, cs, tol, c.st));
  }
  // done[S] then flags[4] are contiguous in si
  int32_t* pin = c.slot(0);
  HIPCHK(hipMemcpyAsync(pin, c.si, (S + 4) * sizeof(int32_t), hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  if (pin[S + 2]) return fail(ctx, GP2S_E_NONFINITE, "non-finite right-hand side (%s)", c.label);
  int open = 0;
  for (int s = 0; s < S; ++s) open += pin[s] == 0;
  c.open = open > 0;
  if (S > 1 && (m->spmm_variant[S] == -2 || m->spmm_variant[S] == -3)) {
    // a handle of the same shape tuned earlier in this context lends its choice
    auto same = [&](const gp2s_ctx_s::TunedShape& t) {
      return t.n == m->n && t.nnz == m->nnz && t.prec == m->prec && t.S == S && t.f32vec == c.f32vec;
    };
    auto it = std::find_if(ctx->tuned.begin(), ctx->tuned.end(), same);
    if (m->spmm_variant[S] == -2 && it != ctx->tuned.end()) {
      m->spmm_variant[S] = it->variant;
    } else {
      gp2s_status st = tune_block_product(ctx, m, S, c.P, c.Q, c.f32vec, cs, c.st);
      if (st) return st;
      if (it != ctx->tuned.end())
        it->variant = m->spmm_variant[S];
      else
        ctx->tuned.push_back({m->n, m->nnz, m->prec, S, c.f32vec, m->spmm_variant[S]});
    }
  }
  c.variant = S > 1 ? m->spmm_variant[S] : 0;
  if (c.variant == 3) {
    gp2s_status gs = ensure_groups(ctx, m);
    if (gs) return gs;
  }
  if (c.variant == 2) {  // a pinned tile variant: the tiles are otherwise built by the tuner
    gp2s_status ts = ensure_tiles(ctx, m);
    if (ts) return ts;
  }
  if (c.variant == 5) {  // the block split (its block values are refreshed after a refill)
    gp2s_status bs = ensure_bsplit(ctx, m);
    if (bs) return bs;
  }
  return GP2S_OK;
}

// Queues one iteration.
gp2s_status cg_step(Cg& c) {
  gp2s_ctx ctx = c.ctx;
  gp2s_matrix m = c.m;
  const int64_t n = m->n;
  const int S = c.S;
  if (m->ffG)  // far-field kernel: C = G^T p before the product (k_cg_alpha adds |C|^2 to p^T q)
    HIPCHK(launch_ff_gtp(n, S, m->ffU, m->ffG, c.P, c.f32vec, c.lrPart, c.lrTicket, c.lrC, c.st));
  TIMED_ON(S == 1 ? GP2S_T_CG_MATVEC1 : GP2S_T_CG_MATVEC_BLOCK, c.st,
           launch_cg_matvec(m->prec, m->row_ptr, m->col, m->val, n, S, (double)m->nnz / (double)n, c.variant,
                            tile_set(m), c.P, c.Q, c.f32vec, c.cs, c.st, row_blocks(m)));
  if (m->ffG) HIPCHK(launch_ff_add(n, S, m->ffU, m->ffG, c.lrC, S, 1, static_cast<double*>(c.Q), c.st));
  if (pc_block(c.precond)) {
    const int rows = pc_rows(c.precond);
    TIMED_ON(S == 1 ? GP2S_T_CG_UPDATE1 : GP2S_T_CG_UPDATE_BLOCK, c.st,
             launch_bj_update(n, S, nullptr, c.X, c.R, c.P, c.Q, c.f32vec, m->bj[pc_idx(c.precond)].M, c.Z, c.cs,
                              c.st, bj_m32(c), c.Z32, rows));
    HIPCHK(launch_cg_beta(c.cs, (int)bj_update_blocks(n, rows), S, c.it, c.st));
    TIMED_ON(S == 1 ? GP2S_T_CG_PUPDATE1 : GP2S_T_CG_PUPDATE_BLOCK, c.st,
             c.Z32 ? launch_cg_pupdate_z32(n, S, c.P, c.Z32, c.f32vec, c.cs, c.st)
                   : launch_cg_pupdate(n, S, c.P, c.Z, nullptr, c.f32vec, c.cs, c.st));
  } else {
    TIMED_ON(S == 1 ? GP2S_T_CG_UPDATE1 : GP2S_T_CG_UPDATE_BLOCK, c.st,
             launch_cg_update(n, S, c.X, c.R, c.P, c.Q, c.f32vec, m->dinv, c.cs, c.it, c.st));
    TIMED_ON(S == 1 ? GP2S_T_CG_PUPDATE1 : GP2S_T_CG_PUPDATE_BLOCK, c.st,
             launch_cg_pupdate(n, S, c.P, c.R, m->dinv, c.f32vec, c.cs, c.st));
  }
  ++c.it;
  return GP2S_OK;
}

// Evaluates a completed poll copy (flags of iteration `at`).
gp2s_status cg_eval(Cg& c, const int32_t* f, int at) {
  gp2s_ctx ctx = c.ctx;
  const int S = c.S;
  if (f[S + 0]) {
    int32_t its[kMaxProbes];
    gp2s_status st = readback_on(ctx, c.st, c.cs.iters, S * sizeof(int32_t), its);
    const int col = f[S + 3];
    return fail(ctx, GP2S_E_NOT_SPD,
                "CG breakdown in the %s, column %d after %d iterations: p^T K p <= 0 (matrix not positive "
                "definite in working precision)", c.label, col, st ? -1 : its[col]);
  }
  if (f[S + 2]) return fail(ctx, GP2S_E_NONFINITE, "non-finite values during CG (%s)", c.label);
  int open = 0;
  for (int s = 0; s < S; ++s) open += f[s] == 0;
  c.open = open > 0;
  if (ctx->progress) {
    // rr[S] and bb[S] follow the flags in the slot (queued with them)
    const double* rr = reinterpret_cast<const double*>(f + kMaxProbes + 4);
    const double* bb = rr + kMaxProbes;
    double worst = 0.0;
    for (int s = 0; s < S; ++s)
      if (!f[s] && bb[s] > 0) worst = std::max(worst, std::sqrt(rr[s] / bb[s]));
    ctx->progress(c.label, at, open, worst, ctx->progress_user);
  }
  return GP2S_OK;
}

// At a check point: evaluate the previous poll (if any), then queue a new one.
gp2s_status cg_check(Cg& c) {
  gp2s_ctx ctx = c.ctx;
  const int S = c.S;
  if (c.nq > 0) {
    const int k = (c.nq - 1) & 1;
    HIPCHK(hipEventSynchronize(c.ev[k]));
    gp2s_status st = cg_eval(c, c.slot(k), c.polled_it);
    if (st) return st;
    if (!c.open) return GP2S_OK;
  }
  const int k = c.nq & 1;
  int32_t* f = c.slot(k);
  HIPCHK(hipMemcpyAsync(f, c.si, (S + 4) * sizeof(int32_t), hipMemcpyDeviceToHost, c.st));
  if (ctx->progress) {
    double* rr = reinterpret_cast<double*>(f + kMaxProbes + 4);
    HIPCHK(hipMemcpyAsync(rr, c.cs.rr, S * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(rr + kMaxProbes, c.cs.bb, S * sizeof(double), hipMemcpyDeviceToHost, c.st));
  }
  HIPCHK(hipEventRecord(c.ev[k], c.st));
  c.polled_it = c.it;
  ++c.nq;
  return GP2S_OK;
}

bool cg_active(const Cg& c) { return c.open && c.it < c.max_iter; }

// Final synchronous poll and iteration counts.
gp2s_status cg_end(Cg& c) {
  gp2s_ctx ctx = c.ctx;
  const int S = c.S;
  if (c.it > 0) {
    int32_t f[kMaxProbes + 4];
    gp2s_status st = readback_on(ctx, c.st, c.si, (S + 4) * sizeof(int32_t), f);
    if (st) return st;
    gp2s_progress_fn keep = ctx->progress;  // no residuals in this copy
    ctx->progress = nullptr;
    st = cg_eval(c, f, c.it);
    ctx->progress = keep;
    if (st) return st;
  }
  gp2s_status st = readback_on(ctx, c.st, c.cs.iters, S * sizeof(int32_t), c.host_iters);
  if (st) return st;
  c.total_iters = 0;
  for (int s = 0; s < S; ++s) c.total_iters = std::max(c.total_iters, c.host_iters[s]);
  c.converged = !c.open;
  return GP2S_OK;
}

// Runs one or two solves to completion, interleaving their iterations.
gp2s_status cg_drive(Cg* a, Cg* b) {
  for (;;) {
    const bool ra = a && cg_active(*a), rb = b && cg_active(*b);
    if (!ra && !rb) break;
    for (Cg* c : {a, b}) {
      if (!c || !cg_active(*c)) continue;
      gp2s_status st = cg_step(*c);
      if (st) return st;
      if (c->it % c->check_every == 0) {
        st = cg_check(*c);
        if (st) return st;
      }
    }
  }
  for (Cg* c : {a, b}) {
    if (!c) continue;
    gp2s_status st = cg_end(*c);
    if (st) return st;
  }
  return GP2S_OK;
}

gp2s_status run_cg(gp2s_ctx ctx, gp2s_matrix m, int S, const double* B, double* X, double tol, int max_iter,
                   int check_every, bool keep_hist, Scratch& sc, CgRun& out, const char* label, int precond) {
  Cg c;
  c.ctx = ctx;
  c.m = m;
  c.S = S;
  c.precond = precond;
  c.X = X;
  c.max_iter = max_iter;
  c.check_every = check_every;
  c.label = label;
  c.st = ctx->stream;
  c.slot0 = 0;
  gp2s_status st = cg_begin(c, B, tol, keep_hist, sc);
  if (st) return st;
  st = cg_drive(&c, nullptr);
  if (st) return st;
  out.cs = c.cs;
  std::memcpy(out.host_iters, c.host_iters, sizeof(c.host_iters));
  out.total_iters = c.total_iters;
  out.converged = c.converged;
  return GP2S_OK;
}

// Scalar reductions through the pinned buffer.
gp2s_status dot_host(gp2s_ctx ctx, int64_t n, const double* a, const double* b, double* buf, uint32_t* ticket,
                     double* out) {
  HIPCHK(launch_dot_partial(n, a, b, buf, ticket, ctx->stream));
  return readback(ctx, buf, sizeof(double), out);
}

// Far-field kernel: Y += G (G^T X) for S columns (internal order); no-op otherwise.
gp2s_status ff_apply(gp2s_ctx ctx, gp2s_matrix m, int S, const double* X, double* Y, Scratch& sc) {
  if (!m->ffG) return GP2S_OK;
  const int64_t n = m->n;
  double* C = sc.get<double>((size_t)m->ffU * S);
  double* part = sc.get<double>((size_t)m->ffU * S * ff_gtp_blocks(n));
  uint32_t* tk = sc.get<uint32_t>(1);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "far-field workspace allocation failed");
  HIPCHK(hipMemsetAsync(tk, 0, sizeof(uint32_t), ctx->stream));
  HIPCHK(launch_ff_gtp(n, S, m->ffU, m->ffG, X, false, part, tk, C, ctx->stream));
  HIPCHK(launch_ff_add(n, S, m->ffU, m->ffG, C, S, 1, Y, ctx->stream));
  return GP2S_OK;
}

// Solve K a = y (internal order) with restarts from the recomputed residual. `side`,
// if given, is a solve begun on the second stream; its iterations are interleaved with
// those of the first CG run of y and it is complete on return.
gp2s_status solve_internal(gp2s_ctx ctx, gp2s_matrix m, const double* y, double* a, const gp2s_solve_opts* o,
                           Scratch& sc, gp2s_report* rep, bool* converged, Cg* side = nullptr) {
  const int64_t n = m->n;
  double* red = sc.get<double>(1 + kReduceBlocks);
  uint32_t* tk = sc.get<uint32_t>(1);
  double* r = sc.get<double>(n);
  double* d = sc.get<double>(n);
  double* kx = sc.get<double>(n);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "solve workspace allocation failed");
  HIPCHK(hipMemsetAsync(tk, 0, sizeof(uint32_t), ctx->stream));
  int32_t* flag = reinterpret_cast<int32_t*>(tk);  // reused below only after the ticket is idle
  (void)flag;
  double bb = 0.0;
  gp2s_status st = dot_host(ctx, n, y, nullptr, red, tk, &bb);
  if (st) return st;
  if (!is_fin(bb)) return fail(ctx, GP2S_E_NONFINITE, "y contains NaN or infinity");
  if (!m->diag_ok) return fail(ctx, GP2S_E_NOT_SPD, "diagonal of K is not positive");
  int total = 0, ir = 0;
  *converged = false;
  double resid = 0.0;
  if (bb == 0.0) {
    HIPCHK(hipMemsetAsync(a, 0, n * sizeof(double), ctx->stream));
    *converged = true;
    if (side) {
      st = cg_drive(nullptr, side);
      if (st) return st;
    }
  } else {
    Cg cy;
    cy.ctx = ctx;
    cy.m = m;
    cy.S = 1;
    cy.precond = o->precond;
    cy.X = a;
    cy.max_iter = o->max_iter;
    cy.check_every = o->check_every;
    cy.label = "y solve";
    cy.st = ctx->stream;
    cy.slot0 = 0;
    st = cg_begin(cy, y, o->tol, false, sc);
    if (st) return st;
    st = cg_drive(&cy, side);
    if (st) return st;
    total += cy.total_iters;
    for (;;) {
      TIMED(GP2S_T_SPMV, launch_spmv(m->prec, m->row_ptr, m->col, m->val, n, (double)m->nnz / n, a, kx, ctx->stream,
                                     row_blocks(m)));
      st = ff_apply(ctx, m, 1, a, kx, sc);
      if (st) return st;
      HIPCHK(launch_axpy_sub(n, y, kx, r, ctx->stream));
      double rr = 0.0;
      st = dot_host(ctx, n, r, nullptr, red, tk, &rr);
      if (st) return st;
      resid = std::sqrt(rr / bb);
      if (!is_fin(resid)) return fail(ctx, GP2S_E_NONFINITE, "non-finite residual");
      if (resid <= o->tol) {
        *converged = true;
        break;
      }
      if (ir >= o->max_ir || total >= o->max_iter) break;
      ++ir;
      const double inner = std::min(0.5, 0.5 * o->tol / resid);
      CgRun r2;
      st = run_cg(ctx, m, 1, r, d, inner, o->max_iter - total, o->check_every, false, sc, r2, "refinement solve",
                  o->precond);
      if (st) return st;
      total += r2.total_iters;
      HIPCHK(launch_add(n, a, d, ctx->stream));
    }
  }
  if (rep) {
    rep->resid = resid;
    rep->iters = total;
    rep->ir_steps = ir;
  }
  return GP2S_OK;
}

struct ProbeResult {
  double logdet = 0.0, stderr_ = 0.0;
  int iters = 0;
  bool converged = false;
};

// Probe solves K q_s = L z_s (Sec. 4.6; App. B.6 "LOGDET"; L = D^1/2 for the diagonal
// preconditioner, the blockwise Cholesky factor for the block one): queues the probe
// signs and right-hand sides on the second stream and begins the block solve there.
// Wsol (block preconditioner, gradient only) receives w_s = L^-T z_s = M^-1 L z_s, the
// preconditioned initial residual.
gp2s_status probes_begin(gp2s_ctx ctx, gp2s_matrix m, const gp2s_solve_opts* o, Scratch& sc, uint64_t* mask,
                         double* Qsol, double* Wsol, Cg& cp) {
  // Qsol == nullptr: the probe solutions are not needed (no gradient), only the CG
  // coefficients the quadrature uses.
  const int64_t n = m->n;
  const int S = o->n_probes;
  double* B = sc.get<double>((size_t)n * S);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "probe workspace allocation failed");
  HIPCHK(launch_probe_masks(n, m->perm, o->seed, S, mask, ctx->aux));
  if (pc_block(o->precond))
    HIPCHK(launch_bj_rhs(n, S, mask, m->bj[pc_idx(o->precond)].L, B, ctx->aux, BjBlocks{nullptr, nullptr, 0},
                         pc_rows(o->precond)));
  else
    HIPCHK(launch_probe_rhs(n, S, mask, m->diag, B, ctx->aux));
  cp.ctx = ctx;
  cp.m = m;
  cp.S = S;
  cp.X = Qsol;
  cp.precond = o->precond;
  cp.probe = true;
  cp.max_iter = o->max_iter;
  cp.check_every = o->check_every;
  cp.label = "probe block";
  cp.st = ctx->aux;
  cp.slot0 = 2;
  gp2s_status st = cg_begin(cp, B, o->probe_tol, true, sc);
  if (st) return st;
  if (Wsol) HIPCHK(hipMemcpyAsync(Wsol, cp.Z, (size_t)n * S * sizeof(double), hipMemcpyDeviceToDevice, ctx->aux));
  return GP2S_OK;
}

// The Lanczos log-determinant estimate from the finished probe block (after the
// second stream has been joined into the context's stream).
gp2s_status probes_finish(gp2s_ctx ctx, gp2s_matrix m, Scratch& sc, const Cg& cp, ProbeResult& pr) {
  const int64_t n = m->n;
  const int S = cp.S;
  double* red = sc.get<double>(1 + kReduceBlocks);
  uint32_t* tk = sc.get<uint32_t>(1);
  const int64_t max_m = std::max(1, cp.total_iters);
  double* work = sc.get<double>((size_t)2 * S * max_m);
  double* quad = sc.get<double>(S);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "quadrature workspace allocation failed");
  HIPCHK(hipMemsetAsync(tk, 0, sizeof(uint32_t), ctx->stream));
  TIMED(GP2S_T_SLQ, launch_slq_ws(S, cp.cs.hist_a, cp.cs.hist_b, cp.cs.iters, work, max_m, quad, ctx->stream));
  std::vector<double> qh(S);
  gp2s_status st = readback(ctx, quad, S * sizeof(double), qh.data());
  if (st) return st;
  double sumlog = 0.0;
  HIPCHK(launch_sum_log(n, pc_block(cp.precond) ? m->bj[pc_idx(cp.precond)].piv : m->diag, red, tk, ctx->stream));
  st = readback(ctx, red, sizeof(double), &sumlog);
  if (st) return st;
  double mean = 0.0;
  for (int s = 0; s < S; ++s) mean += (double)n * qh[s];
  mean /= S;
  double var = 0.0;
  for (int s = 0; s < S; ++s) var += ((double)n * qh[s] - mean) * ((double)n * qh[s] - mean);
  pr.stderr_ = S > 1 ? std::sqrt(var / (S - 1) / S) : 0.0;
  pr.logdet = sumlog + mean;
  pr.iters = cp.total_iters;
  pr.converged = cp.converged;
  return GP2S_OK;
}

// Makes the context's stream wait for everything queued on the second stream.
struct AuxJoin {
  gp2s_ctx ctx;
  ~AuxJoin() {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) {
      (void)hipEventRecord(e, ctx->aux);
      (void)hipStreamWaitEvent(ctx->stream, e, 0);
      (void)hipEventDestroy(e);
    } else {
      (void)hipStreamSynchronize(ctx->aux);
    }
  }
};

// Per-axis geometry handed to the kernels (general == 0: isotropic stationary path).
KernGeom kern_geom(gp2s_matrix m) {
  KernGeom kg{};
  for (int k = 0; k < 3; ++k) {
    const double r = k < m->dim ? m->radii[k] : 1.0;
    kg.inv_r[k] = 1.0 / r;
    kg.inv_rf[k] = (float)kg.inv_r[k];
  }
  kg.lsq = m->lsq;
  kg.general = (m->ard || m->lsq) ? 1 : 0;
  return kg;
}

gp2s_status lml_common(gp2s_ctx ctx, gp2s_matrix m, const double* y, const gp2s_solve_opts* o, double* a,
                       gp2s_report* rep, double* grad) {
  if (!ctx) return GP2S_E_INVALID;
  gp2s_status st = check_matrix(ctx, m);
  if (st) return st;
  st = check_opts(ctx, o, true);
  if (st) return st;
  if (!y) return fail(ctx, GP2S_E_INVALID, "y is NULL");
  if (!rep) return fail(ctx, GP2S_E_INVALID, "report is NULL");
  if ((int64_t)m->n * o->n_probes >= (int64_t)INT32_MAX)
    return fail(ctx, GP2S_E_INVALID, "n * n_probes must be below 2^31 (probe block indexing)");
  if (grad && !m->assembled)
    return fail(ctx, GP2S_E_INVALID, "the gradient needs a handle from gp2s_assemble (imported CSR has no kernel)");
  st = ensure_device(ctx);
  if (st) return st;
  const int64_t n = m->n;
  const int S = o->n_probes;
  Scratch sc(ctx);
  double* yi = sc.get<double>(n);
  double* ai = sc.get<double>(n);
  double* Qs = grad ? sc.get<double>((size_t)n * S) : nullptr;  // probe solutions (gradient only)
  double* Ws = grad && pc_block(o->precond) ? sc.get<double>((size_t)n * S) : nullptr;
  uint64_t* mask = sc.get<uint64_t>(n);
  double* red = sc.get<double>(1 + kReduceBlocks);
  uint32_t* tk = sc.get<uint32_t>(1);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "LML workspace allocation failed");
  HIPCHK(hipMemsetAsync(tk, 0, sizeof(uint32_t), ctx->stream));
  HIPCHK(launch_gather_rows(n, 1, m->perm, y, yi, ctx->stream));
  std::memset(rep, 0, sizeof(*rep));
  if (pc_block(o->precond)) {
    if (!m->diag_ok) return fail(ctx, GP2S_E_NOT_SPD, "diagonal of K is not positive");
    st = ensure_bj(ctx, m, o->precond);
    if (st) return st;
  }
  // The probe block runs on the second stream beside the y solve: it starts after
  // the work already queued on the context's stream and is joined back before the
  // quadrature (and on every early return, before the workspace is released).
  {
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipError_t e1 = hipEventRecord(e, ctx->stream);
    hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(ctx->aux, e, 0) : e1;
    (void)hipEventDestroy(e);
    if (e2 != hipSuccess) return fail(ctx, GP2S_E_HIP, "ordering the probe stream: %s", hipGetErrorString(e2));
  }
  AuxJoin join{ctx};
  Cg cp;
  st = probes_begin(ctx, m, o, sc, mask, Qs, Ws, cp);
  if (st) return st;
  bool conv_y = false;
  st = solve_internal(ctx, m, yi, ai, o, sc, rep, &conv_y, &cp);
  if (st) return st;
  double yTa = 0.0;
  st = dot_host(ctx, n, yi, ai, red, tk, &yTa);
  if (st) return st;
  {
    AuxJoin j2{ctx};
  }
  ProbeResult pr;
  st = probes_finish(ctx, m, sc, cp, pr);
  if (st) return st;
  rep->yTa = yTa;
  rep->logdet = pr.logdet;
  rep->logdet_stderr = pr.stderr_;
  rep->probe_iters = pr.iters;
  rep->n_probes = S;
  rep->lml = -0.5 * yTa - 0.5 * pr.logdet - 0.5 * (double)n * std::log(2.0 * M_PI);
  if (a) HIPCHK(launch_scatter_rows(n, 1, m->perm, ai, a, ctx->stream));
  if (grad) {
    const int nr = m->ard ? m->dim : 1;
    const bool ls = m->lsq != nullptr;
    double* Rr = sc.get<double>(n);
    double* Tr = sc.get<double>((size_t)nr * n);
    double* Ur = sc.get<double>(n);
    double* Vr = ls ? sc.get<double>(n) : nullptr;
    const int ncomp = nr + m->P + (ls ? m->P : 0) + 1;
    double* gpart = sc.get<double>((size_t)256 * ncomp);
    double* gd = sc.get<double>(ncomp);
    uint32_t* tk2 = sc.get<uint32_t>(1);
    if (sc.oom) return fail(ctx, GP2S_E_OOM, "gradient workspace allocation failed");
    HIPCHK(hipMemsetAsync(tk2, 0, sizeof(uint32_t), ctx->stream));
    BackwardArgs b{};
    b.rp = m->row_ptr;
    b.col = m->col;
    b.pts32 = m->pts32;
    b.pts64 = m->pts64;
    b.g64 = m->g64;
    b.a = ai;
    b.Q = Qs;
    b.mask = mask;
    b.dinv = m->dinv;
    b.W = Ws;
    b.n = n;
    b.S = S;
    b.radius = m->radius;
    b.r2 = m->radius * m->radius;
    b.inv_r2 = 1.0 / b.r2;
    b.kern = m->kern;
    b.kg = kern_geom(m);
    b.nr = nr;
    b.dim = m->dim;
    TIMED(GP2S_T_BACKWARD, launch_backward_rows(b, m->prec, Rr, Tr, Ur, Vr, ctx->stream));
    double* Hr = nullptr;
    if (m->ffU > 0) {
      // far-field amplitudes: H = P G with P = a a^T - (1/2S) sum_s (q_s w_s^T + w_s q_s^T)
      const int U = m->ffU;
      double* Wf = Ws;
      if (!Wf) {
        Wf = sc.get<double>((size_t)n * S);
        if (sc.oom) return fail(ctx, GP2S_E_OOM, "gradient workspace allocation failed");
        HIPCHK(launch_ff_wjac(n, S, mask, m->dinv, Wf, ctx->stream));
      }
      double* ag = sc.get<double>(U);
      double* wg = sc.get<double>((size_t)U * S);
      double* qg = sc.get<double>((size_t)U * S);
      double* part = sc.get<double>((size_t)U * S * ff_gtp_blocks(n));
      uint32_t* tk3 = sc.get<uint32_t>(1);
      Hr = sc.get<double>((size_t)n * U);
      if (sc.oom) return fail(ctx, GP2S_E_OOM, "gradient workspace allocation failed");
      HIPCHK(hipMemsetAsync(tk3, 0, sizeof(uint32_t), ctx->stream));
      HIPCHK(launch_ff_gtp(n, 1, U, m->ffG, ai, false, part, tk3, ag, ctx->stream));
      HIPCHK(launch_ff_gtp(n, S, U, m->ffG, Wf, false, part, tk3, wg, ctx->stream));
      HIPCHK(launch_ff_gtp(n, S, U, m->ffG, Qs, false, part, tk3, qg, ctx->stream));
      HIPCHK(launch_ff_h(n, S, U, ai, Qs, Wf, ag, wg, qg, Hr, ctx->stream));
    }
    TIMED(GP2S_T_GRAD_REDUCE, launch_grad_reduce(n, m->dim, m->P, S, nr, m->x64, m->g64, ai, Rr, Tr, Ur, Vr, Hr,
                                                 m->ffgrp_d, m->ffU, m->centers_d, m->bump_width * m->bump_width,
                                                 gpart, tk2, gd, ctx->stream));
    st = readback(ctx, gd, ncomp * sizeof(double), grad);
    if (st) return st;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (!conv_y || !pr.converged)
    return fail(ctx, GP2S_E_NOCONV, "CG did not converge within max_iter (y: %s, probes: %s)",
                conv_y ? "yes" : "no", pr.converged ? "yes" : "no");
  return GP2S_OK;
}

}  // namespace

using namespace gp2s::rt;

// =====================================================================================
// ---- allocation-free product ------------------------------------------------------------
// Workspace of gp2s_spmv_noalloc: X gathered into internal order, then the product in
// internal order, kNoAllocElems float64 values each (2 x 32 MiB). Every GPU the library
// runs on holds its own copy until the process ends. In host code `scratch` names a
// host-side stand-in, never the device memory: host code uses only the per-device
// address that hipGetSymbolAddress returns.
constexpr int64_t kNoAllocElems = int64_t(1) << 22;
static __device__ __align__(256) double scratch[2 * kNoAllocElems];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[kNoAllocDevices] = {};

// The device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
gp2s_status noalloc_workspace(gp2s_ctx ctx, double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices) return fail(ctx, GP2S_E_INVALID, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ctx, GP2S_E_HIP, "hipGetSymbolAddress returned NULL for the workspace");
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return GP2S_OK;
}
}  // namespace

extern "C" {

int32_t gp2s_abi_version(void) { return GP2S_ABI_VERSION; }

void gp2s_default_opts(gp2s_solve_opts* o) {
  if (!o) return;
  o->n_probes = 64;
  o->max_iter = 20000;
  o->max_ir = 4;
  o->check_every = 16;
  o->seed = 0;
  o->tol = 1e-8;
  o->probe_tol = 1e-5;
  o->precond = GP2S_PRECOND_BLOCK;
}

const char* gp2s_status_string(gp2s_status s) {
  switch (s) {
    case GP2S_OK: return "ok";
    case GP2S_E_INVALID: return "invalid argument";
    case GP2S_E_HIP: return "HIP runtime error";
    case GP2S_E_OOM: return "out of device memory";
    case GP2S_E_CAPACITY: return "capacity exceeded";
    case GP2S_E_NOT_SPD: return "matrix not positive definite";
    case GP2S_E_NOCONV: return "iteration did not converge";
    case GP2S_E_NONFINITE: return "non-finite input";
    default: return "unknown status";
  }
}

gp2s_status gp2s_create(gp2s_ctx* out, void* stream, gp2s_alloc_fn alloc, gp2s_free_fn free_fn, void* user) {
  if (!out) return GP2S_E_INVALID;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return GP2S_E_INVALID;
  gp2s_ctx c = new (std::nothrow) gp2s_ctx_s();
  if (!c) return GP2S_E_OOM;
  c->stream = static_cast<hipStream_t>(stream);
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = user;
  *out = c;
  return GP2S_OK;
}

gp2s_status gp2s_set_timing_mask(gp2s_ctx ctx, uint32_t mask) {
  if (!ctx) return GP2S_E_INVALID;
  if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
  if (!ctx->pending.empty()) {
    (void)hipStreamSynchronize(ctx->stream);
    harvest(ctx);
  }
  ctx->timing_mask = mask & ((1u << GP2S_NUM_TIMERS) - 1u);
  for (int k = 0; k < GP2S_NUM_TIMERS; ++k) {
    ctx->ms[k] = 0.0;
    ctx->count[k] = 0;
  }
  return GP2S_OK;
}

gp2s_status gp2s_set_timing(gp2s_ctx ctx, int32_t enable) {
  return gp2s_set_timing_mask(ctx, enable ? ~0u : 0u);
}

gp2s_status gp2s_set_progress(gp2s_ctx ctx, gp2s_progress_fn fn, void* user) {
  if (!ctx) return GP2S_E_INVALID;
  ctx->progress = fn;
  ctx->progress_user = user;
  return GP2S_OK;
}

gp2s_status gp2s_get_stats(gp2s_ctx ctx, gp2s_stats* out) {
  if (!ctx || !out) return GP2S_E_INVALID;
  if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
  if (!ctx->pending.empty()) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, GP2S_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    harvest(ctx);
  }
  for (int k = 0; k < GP2S_NUM_TIMERS; ++k) {
    out->ms[k] = ctx->ms[k];
    out->count[k] = ctx->count[k];
  }
  return GP2S_OK;
}

gp2s_status gp2s_destroy(gp2s_ctx ctx) {
  if (!ctx) return GP2S_E_INVALID;
  if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
  if (!ctx->pending.empty()) {
    (void)hipStreamSynchronize(ctx->stream);
    harvest(ctx);
  }
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.e0);
    (void)hipEventDestroy(p.e1);
  }
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return GP2S_OK;
}

const char* gp2s_last_error(gp2s_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gp2s_status gp2s_check_params(gp2s_ctx ctx, int64_t n, const gp2s_params* p) {
  if (!ctx) return GP2S_E_INVALID;
  if (n < 1 || n >= (int64_t)INT32_MAX) return fail(ctx, GP2S_E_INVALID, "n must be in [1, 2^31 - 1)");
  if (!p) return fail(ctx, GP2S_E_INVALID, "params is NULL");
  if (p->dim != 2 && p->dim != 3) return fail(ctx, GP2S_E_INVALID, "dim must be 2 or 3");
  if (p->n_bumps < 1 || p->n_bumps > kMaxBumps)
    return fail(ctx, GP2S_E_INVALID, "n_bumps must be in [1, %d]", kMaxBumps);
  if (!p->centers || !p->weights) return fail(ctx, GP2S_E_INVALID, "centers and weights must be non-NULL");
  if (!is_fin(p->radius) || !is_fin(p->bump_width) || !is_fin(p->noise_var))
    return fail(ctx, GP2S_E_NONFINITE, "non-finite hyperparameter");
  if (p->radius <= 0) return fail(ctx, GP2S_E_INVALID, "radius must be > 0");
  if (p->bump_width <= 0) return fail(ctx, GP2S_E_INVALID, "bump_width must be > 0");
  if (p->noise_var < 0) return fail(ctx, GP2S_E_INVALID, "noise_var must be >= 0");
  if (p->kernel != GP2S_WENDLAND_C2 && p->kernel != GP2S_WENDLAND_C6)
    return fail(ctx, GP2S_E_INVALID, "kernel must be GP2S_WENDLAND_C2 or GP2S_WENDLAND_C6");
  for (int k = 0; k < p->n_bumps * p->dim; ++k)
    if (!is_fin(p->centers[k])) return fail(ctx, GP2S_E_NONFINITE, "non-finite bump centre");
  for (int k = 0; k < p->n_bumps; ++k)
    if (!is_fin(p->weights[k])) return fail(ctx, GP2S_E_NONFINITE, "non-finite bump weight");
  if (p->radii)
    for (int k = 0; k < p->dim; ++k) {
      if (!is_fin(p->radii[k])) return fail(ctx, GP2S_E_NONFINITE, "non-finite axis radius");
      if (p->radii[k] <= 0) return fail(ctx, GP2S_E_INVALID, "axis radii must be > 0");
    }
  if (p->ff_groups) {
    if (p->radii || p->ls_weights)
      return fail(ctx, GP2S_E_INVALID, "the far-field kernel takes one isotropic radius (radii and ls_weights NULL)");
    for (int k = 0; k < p->n_bumps; ++k)
      if (p->ff_groups[k] < 0 || p->ff_groups[k] >= kMaxGroups)
        return fail(ctx, GP2S_E_INVALID, "ff_groups values must be in [0, %d)", kMaxGroups);
  }
  if (p->ls_weights)
    for (int k = 0; k < p->n_bumps; ++k) {
      if (!is_fin(p->ls_weights[k])) return fail(ctx, GP2S_E_NONFINITE, "non-finite length-scale weight");
      if (std::fabs(p->ls_weights[k]) > 20.0) return fail(ctx, GP2S_E_INVALID, "length-scale weights must be in [-20, 20]");
    }
  return GP2S_OK;
}



gp2s_status gp2s_assemble(gp2s_ctx ctx, int64_t n, const double* x, const gp2s_params* p,
                          gp2s_precision prec, gp2s_matrix* out) {
  if (!ctx) return GP2S_E_INVALID;
  if (!out) return fail(ctx, GP2S_E_INVALID, "out is NULL");
  *out = nullptr;
  gp2s_status st = gp2s_check_params(ctx, n, p);
  if (st) return st;
  if (!x) return fail(ctx, GP2S_E_INVALID, "x is NULL");
  if (prec != GP2S_FP64 && prec != GP2S_MIXED) return fail(ctx, GP2S_E_INVALID, "unknown precision");
  st = ensure_device(ctx);
  if (st) return st;

  gp2s_matrix m = new (std::nothrow) gp2s_matrix_s();
  if (!m) return fail(ctx, GP2S_E_OOM, "host allocation failed");
  struct Guard {
    gp2s_matrix m;
    bool keep = false;
    ~Guard() {
      if (!keep) gp2s_matrix_free(m);
    }
  } guard{m};
  m->ctx = ctx;
  m->n = n;
  m->prec = prec;
  m->assembled = true;
  m->dim = p->dim;
  m->P = p->n_bumps;
  m->radius = p->radius;
  m->bump_width = p->bump_width;
  m->noise = p->noise_var;
  m->kern = p->kernel;
  m->centers_h.assign(p->centers, p->centers + (size_t)p->n_bumps * p->dim);
  m->weights_h.assign(p->weights, p->weights + p->n_bumps);
  const int dim = p->dim;
  hipStream_t sm = ctx->stream;
  m->ard = p->radii != nullptr;
  if (p->ff_groups) {
    m->ffgrp_h.assign(p->ff_groups, p->ff_groups + p->n_bumps);
    for (int32_t u : m->ffgrp_h) m->ffU = std::max(m->ffU, u + 1);
  }
  for (int k = 0; k < dim; ++k) m->radii[k] = m->ard ? p->radii[k] : p->radius;
  if (p->ls_weights) {
    m->ls_h.assign(p->ls_weights, p->ls_weights + p->n_bumps);
    double pos = 0.0;
    for (double c : m->ls_h) pos += std::max(c, 0.0);
    m->ell_bound = std::exp(pos);  // l(x) <= exp(sum of the positive c_q): every bump is <= 1
  }

  m->centers_d = own<double>(m, m->centers_h.size());
  m->weights_d = own<double>(m, m->weights_h.size());
  OOMCHK(m->centers_d);
  OOMCHK(m->weights_d);
  HIPCHK(hipMemcpyAsync(m->centers_d, m->centers_h.data(), m->centers_h.size() * sizeof(double),
                        hipMemcpyHostToDevice, sm));
  HIPCHK(hipMemcpyAsync(m->weights_d, m->weights_h.data(), m->weights_h.size() * sizeof(double),
                        hipMemcpyHostToDevice, sm));

  Scratch sc(ctx);
  // 1. bounding box and finiteness
  const int bb_blocks = 256;
  double* part = sc.get<double>(bb_blocks * 6);
  int32_t* nonfinite = sc.get<int32_t>(1);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "assembly workspace allocation failed");
  HIPCHK(hipMemsetAsync(nonfinite, 0, sizeof(int32_t), sm));
  HIPCHK(launch_bbox(x, n, dim, part, nonfinite, bb_blocks, sm));
  std::vector<double> hp(bb_blocks * 6 + 1);
  st = readback(ctx, part, bb_blocks * 6 * sizeof(double), hp.data());
  if (st) return st;
  int32_t nf = 0;
  st = readback(ctx, nonfinite, sizeof(int32_t), &nf);
  if (st) return st;
  if (nf) return fail(ctx, GP2S_E_NONFINITE, "x contains NaN or infinity");
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int k = 0; k < dim; ++k) {
    lo[k] = INFINITY;
    hi[k] = -INFINITY;
    for (int b = 0; b < bb_blocks; ++b) {
      lo[k] = std::min(lo[k], hp[b * 6 + k]);
      hi[k] = std::max(hi[k], hp[b * 6 + 3 + k]);
    }
  }
  // 2. grid: side h_k >= r_k along axis k (times the bound of the length-scale
  //    field, which widens the support to at most r_k l_max; enlarged by 1e-6 relative
  //    so rounding in the bin index cannot separate a pair inside the support by two
  //    bins); capped bin count.
  double h[3] = {1.0, 1.0, 1.0};
  for (int k = 0; k < dim; ++k) {
    h[k] = m->radii[k] * (1.0 + 1e-6);
    if (m->ell_bound != 1.0) h[k] *= m->ell_bound;
  }
  const double max_bins = std::max(4.0 * (double)n, 65536.0);
  GridDev g{};
  g.dim = dim;
  for (int iter = 0; iter < 64; ++iter) {
    double nb_total = 1.0;
    for (int k = 0; k < dim; ++k) nb_total *= std::floor((hi[k] - lo[k]) / h[k]) + 1.0;
    if (nb_total <= max_bins) break;
    const double f = std::pow(nb_total / max_bins, 1.0 / dim) * 1.01;
    for (int k = 0; k < dim; ++k) h[k] *= f;
  }
  g.nbins = 1;
  for (int k = 0; k < 3; ++k) {
    g.origin[k] = k < dim ? lo[k] : 0.0;
    g.nb[k] = k < dim ? (int32_t)(std::floor((hi[k] - lo[k]) / h[k]) + 1.0) : 1;
    g.inv_h[k] = 1.0 / h[k];
    g.nbins *= g.nb[k];
  }
  m->grid = g;

  // 3. prologue, counting sort into bins, internal-order point copies
  int32_t* bin_of = sc.get<int32_t>(n);
  int32_t* slot = sc.get<int32_t>(n);
  int32_t* bin_count = sc.get<int32_t>(g.nbins);
  double* g64u = sc.get<double>(n);
  uint8_t* gam = sc.get<uint8_t>(n);
  int32_t* perm_tmp = sc.get<int32_t>(n);
  uint32_t* fkey = sc.get<uint32_t>(n);
  uint32_t* key_tmp = sc.get<uint32_t>(n);
  void* scan_ws = sc.get<uint8_t>(std::max(scan_workspace_bytes(g.nbins), scan_workspace_bytes(n)));
  int32_t* row_cnt = sc.get<int32_t>(n);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "assembly workspace allocation failed");
  m->bin_start = own<int64_t>(m, g.nbins + 1);
  m->perm = own<int32_t>(m, n);
  m->x64 = own<double>(m, (size_t)n * dim);
  m->g64 = own<double>(m, n);
  m->binid = own<int32_t>(m, n);
  m->row_ptr = own<int64_t>(m, n + 1);
  m->diag = own<double>(m, n);
  m->dinv = own<double>(m, n);
  OOMCHK(m->bin_start);
  OOMCHK(m->perm);
  OOMCHK(m->x64);
  OOMCHK(m->g64);
  OOMCHK(m->binid);
  OOMCHK(m->row_ptr);
  OOMCHK(m->diag);
  OOMCHK(m->dinv);
  if (prec == GP2S_MIXED) {
    m->pts32 = own<float4>(m, n);
    OOMCHK(m->pts32);
  } else {
    m->pts64 = own<double4>(m, n);
    OOMCHK(m->pts64);
  }
  {
  Timed prep_timer(ctx, GP2S_T_ASM_PREP, ctx->stream);
  HIPCHK(hipMemsetAsync(bin_count, 0, g.nbins * sizeof(int32_t), sm));
  HIPCHK(launch_prologue(x, n, g, m->centers_d, m->weights_d, m->P, p->bump_width * p->bump_width, bin_of, slot,
                         bin_count, g64u, gam, fkey, sm, m->ffU > 0));
  HIPCHK(launch_exscan_i32_i64(bin_count, m->bin_start, g.nbins, scan_ws, sm));
  HIPCHK(launch_scatter(n, bin_of, slot, fkey, m->bin_start, perm_tmp, key_tmp, sm));
  HIPCHK(launch_binsort(n, perm_tmp, key_tmp, bin_of, m->bin_start, m->perm, sm));
  HIPCHK(launch_gather_points(n, dim, x, m->perm, bin_of, g64u, gam, m->pts32, m->pts64, m->x64, m->g64,
                              m->binid, sm));
  if (!m->ls_h.empty()) {
    m->ls_d = own<double>(m, m->ls_h.size());
    m->lsq = own<double>(m, n);
    OOMCHK(m->ls_d);
    OOMCHK(m->lsq);
    HIPCHK(hipMemcpyAsync(m->ls_d, m->ls_h.data(), m->ls_h.size() * sizeof(double), hipMemcpyHostToDevice, sm));
    HIPCHK(launch_ell(n, dim, m->x64, m->centers_d, m->ls_d, m->P, p->bump_width * p->bump_width, m->lsq, sm));
  }
  }

  // 4. count pass, row pointers, fill pass
  AssembleArgs aa{};
  aa.pts32 = m->pts32;
  aa.pts64 = m->pts64;
  aa.g64 = m->g64;
  aa.binid = m->binid;
  aa.bin_start = m->bin_start;
  aa.grid = g;
  aa.n = n;
  aa.radius = p->radius;
  aa.r2 = p->radius * p->radius;
  aa.inv_r2 = 1.0 / aa.r2;
  aa.noise = p->noise_var;
  aa.r2f = (float)aa.r2;
  aa.kern = m->kern;
  aa.kg = kern_geom(m);
  TIMED(GP2S_T_ASM_COUNT, launch_assemble_count(aa, prec, row_cnt, sm));
  HIPCHK(launch_exscan_i32_i64(row_cnt, m->row_ptr, n, scan_ws, sm));
  int64_t nnz = 0;
  st = readback(ctx, m->row_ptr + n, sizeof(int64_t), &nnz);
  if (st) return st;
  m->nnz = nnz;
  m->col = own<int32_t>(m, nnz + kQuadPad);
  m->val = prec == GP2S_MIXED ? (void*)own<float>(m, nnz + kQuadPad) : (void*)own<double>(m, nnz + kQuadPad);
  m->nrowblk = rowblocks_count(nnz);
  m->rowblk = own<int32_t>(m, m->nrowblk + 1);
  OOMCHK(m->col);
  OOMCHK(m->val);
  OOMCHK(m->rowblk);
  TIMED(GP2S_T_ASM_FILL, launch_assemble_fill(aa, prec, m->row_ptr, m->col, m->val, m->diag, sm));
  HIPCHK(prepare_streaming(m, sm));
  if (m->ffU > 0) {
    m->ffgrp_d = own<int32_t>(m, m->ffgrp_h.size());
    m->ffG = own<double>(m, (size_t)n * m->ffU);
    OOMCHK(m->ffgrp_d);
    OOMCHK(m->ffG);
    HIPCHK(hipMemcpyAsync(m->ffgrp_d, m->ffgrp_h.data(), m->ffgrp_h.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                          sm));
    HIPCHK(launch_ff_G(n, dim, m->x64, m->centers_d, m->weights_d, m->ffgrp_d, m->P, m->ffU,
                       p->bump_width * p->bump_width, m->ffG, m->diag, sm));
  }
  int32_t* bad = nonfinite;
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int32_t), sm));
  HIPCHK(launch_dinv(n, m->diag, m->dinv, bad, sm));
  int32_t hb = 0;
  st = readback(ctx, bad, sizeof(int32_t), &hb);
  if (st) return st;
  m->diag_ok = hb == 0;
  HIPCHK(hipStreamSynchronize(sm));
  guard.keep = true;
  *out = m;
  return GP2S_OK;
}

gp2s_status gp2s_matrix_info(gp2s_matrix m, int64_t* n, int64_t* nnz, gp2s_precision* prec) {
  if (!m) return GP2S_E_INVALID;
  if (n) *n = m->n;
  if (nnz) *nnz = m->nnz;
  if (prec) *prec = m->prec;
  return GP2S_OK;
}

gp2s_status gp2s_matrix_export(gp2s_ctx ctx, gp2s_matrix m, int64_t* row_ptr, int32_t* col, void* val,
                               int32_t* perm) {
  if (!ctx) return GP2S_E_INVALID;
  gp2s_status st = check_matrix(ctx, m);
  if (st) return st;
  st = ensure_device(ctx);
  if (st) return st;
  hipStream_t sm = ctx->stream;
  if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, m->row_ptr, (m->n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, sm));
  if (col) HIPCHK(hipMemcpyAsync(col, m->col, m->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, sm));
  if (val)
    HIPCHK(hipMemcpyAsync(val, m->val, m->nnz * (m->prec == GP2S_MIXED ? sizeof(float) : sizeof(double)),
                          hipMemcpyDeviceToDevice, sm));
  if (perm) {
    if (m->perm) HIPCHK(hipMemcpyAsync(perm, m->perm, m->n * sizeof(int32_t), hipMemcpyDeviceToDevice, sm));
    else return fail(ctx, GP2S_E_INVALID, "imported handles have no permutation");
  }
  HIPCHK(hipStreamSynchronize(sm));
  return GP2S_OK;
}

gp2s_status gp2s_matrix_import(gp2s_ctx ctx, int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                               const void* val, gp2s_precision prec, gp2s_matrix* out) {
  if (!ctx) return GP2S_E_INVALID;
  if (!out) return fail(ctx, GP2S_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1 || n >= (int64_t)INT32_MAX) return fail(ctx, GP2S_E_INVALID, "n must be in [1, 2^31 - 1)");
  if (nnz < n) return fail(ctx, GP2S_E_INVALID, "nnz must be >= n (the diagonal is required)");
  if (!row_ptr || !col || !val) return fail(ctx, GP2S_E_INVALID, "CSR arrays must be non-NULL");
  if (prec != GP2S_FP64 && prec != GP2S_MIXED) return fail(ctx, GP2S_E_INVALID, "unknown precision");
  gp2s_status st = ensure_device(ctx);
  if (st) return st;
  gp2s_matrix m = new (std::nothrow) gp2s_matrix_s();
  if (!m) return fail(ctx, GP2S_E_OOM, "host allocation failed");
  struct Guard {
    gp2s_matrix m;
    bool keep = false;
    ~Guard() {
      if (!keep) gp2s_matrix_free(m);
    }
  } guard{m};
  m->ctx = ctx;
  m->n = n;
  m->nnz = nnz;
  m->prec = prec;
  m->assembled = false;
  const size_t vb = prec == GP2S_MIXED ? sizeof(float) : sizeof(double);
  m->row_ptr = own<int64_t>(m, n + 1);
  m->col = own<int32_t>(m, nnz + kQuadPad);
  m->val = own<uint8_t>(m, (nnz + kQuadPad) * vb);
  m->nrowblk = rowblocks_count(nnz);
  m->rowblk = own<int32_t>(m, m->nrowblk + 1);
  m->diag = own<double>(m, n);
  m->dinv = own<double>(m, n);
  OOMCHK(m->row_ptr);
  OOMCHK(m->col);
  OOMCHK(m->val);
  OOMCHK(m->rowblk);
  OOMCHK(m->diag);
  OOMCHK(m->dinv);
  hipStream_t sm = ctx->stream;
  HIPCHK(hipMemcpyAsync(m->row_ptr, row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, sm));
  HIPCHK(hipMemcpyAsync(m->col, col, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, sm));
  HIPCHK(hipMemcpyAsync(m->val, val, nnz * vb, hipMemcpyDeviceToDevice, sm));
  Scratch sc(ctx);
  int32_t* bad = sc.get<int32_t>(2);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "import workspace allocation failed");
  HIPCHK(hipMemsetAsync(bad, 0, 2 * sizeof(int32_t), sm));
  HIPCHK(launch_extract_diag(n, nnz, m->row_ptr, m->col, m->val, prec, m->diag, bad + 1, sm));
  HIPCHK(launch_dinv(n, m->diag, m->dinv, bad, sm));
  int32_t hb[2] = {0, 0};
  st = readback(ctx, bad, sizeof(hb), hb);
  if (st) return st;
  if (hb[1]) return fail(ctx, GP2S_E_INVALID, "invalid CSR: a row lacks its diagonal, a column index is out of range or not ascending, or row_ptr is inconsistent");
  HIPCHK(prepare_streaming(m, sm));  // only once the CSR is known to be valid
  m->diag_ok = hb[0] == 0;
  guard.keep = true;
  *out = m;
  return GP2S_OK;
}

gp2s_status gp2s_matrix_free(gp2s_matrix m) {
  if (!m) return GP2S_E_INVALID;
  if (m->ctx) {
    if (!m->owned.empty()) (void)hipStreamSynchronize(m->ctx->stream);
    for (void* q : m->owned) dfree(m->ctx, q);
  }
  delete m;
  return GP2S_OK;
}

gp2s_status gp2s_matrix_refill(gp2s_ctx ctx, gp2s_matrix m, const gp2s_params* p) {
  if (!ctx) return GP2S_E_INVALID;
  gp2s_status st = check_matrix(ctx, m);
  if (st) return st;
  if (!m->assembled) return fail(ctx, GP2S_E_INVALID, "refill needs a handle from gp2s_assemble");
  st = gp2s_check_params(ctx, m->n, p);
  if (st) return st;
  bool same = p->dim == m->dim && p->n_bumps == m->P && p->radius == m->radius && p->bump_width == m->bump_width;
  for (int k = 0; same && k < p->n_bumps * p->dim; ++k) same = p->centers[k] == m->centers_h[k];
  same = same && (p->radii != nullptr) == m->ard && (p->ls_weights != nullptr) == !m->ls_h.empty();
  same = same && (p->ff_groups != nullptr) == (m->ffU > 0);
  for (int k = 0; same && p->ff_groups && k < p->n_bumps; ++k) same = p->ff_groups[k] == m->ffgrp_h[k];
  for (int k = 0; same && m->ard && k < p->dim; ++k) same = p->radii[k] == m->radii[k];
  for (int k = 0; same && p->ls_weights && k < p->n_bumps; ++k) same = p->ls_weights[k] == m->ls_h[k];
  if (!same)
    return fail(ctx, GP2S_E_INVALID,
                "refill keeps the pattern: dimension, radii, length-scale weights, bump count, centres and width "
                "must be unchanged (assemble a new handle instead)");
  st = ensure_device(ctx);
  if (st) return st;
  hipStream_t sm = ctx->stream;
  const int64_t n = m->n;
  m->bj[0].ready = m->bj[1].ready = false;  // the block factors belong to the old values
  m->grp_values = false;  // and so do the grouped copy's values
  m->bs_values = false;   // and the block split's dense blocks
  m->weights_h.assign(p->weights, p->weights + p->n_bumps);
  m->noise = p->noise_var;
  m->kern = p->kernel;
  HIPCHK(hipMemcpyAsync(m->weights_d, m->weights_h.data(), m->weights_h.size() * sizeof(double),
                        hipMemcpyHostToDevice, sm));
  Scratch sc(ctx);
  int32_t* bad = sc.get<int32_t>(1);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "refill workspace allocation failed");
  {
    Timed prep_timer(ctx, GP2S_T_ASM_PREP, ctx->stream);
    if (m->ffU == 0)  // (the far-field kernel's Wendland term has g = 1 at every point)
      HIPCHK(launch_refresh_g(n, m->dim, m->x64, m->centers_d, m->weights_d, m->P, m->bump_width * m->bump_width,
                              m->pts32, m->pts64, m->g64, sm));
  }
  AssembleArgs aa{};
  aa.pts32 = m->pts32;
  aa.pts64 = m->pts64;
  aa.g64 = m->g64;
  aa.binid = m->binid;
  aa.bin_start = m->bin_start;
  aa.grid = m->grid;
  aa.n = n;
  aa.radius = m->radius;
  aa.r2 = m->radius * m->radius;
  aa.inv_r2 = 1.0 / aa.r2;
  aa.noise = m->noise;
  aa.r2f = (float)aa.r2;
  aa.kern = m->kern;
  aa.kg = kern_geom(m);
  TIMED(GP2S_T_ASM_FILL, launch_assemble_fill(aa, m->prec, m->row_ptr, m->col, m->val, m->diag, sm));
  if (m->ffU > 0)
    HIPCHK(launch_ff_G(n, m->dim, m->x64, m->centers_d, m->weights_d, m->ffgrp_d, m->P, m->ffU,
                       m->bump_width * m->bump_width, m->ffG, m->diag, sm));
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int32_t), sm));
  HIPCHK(launch_dinv(n, m->diag, m->dinv, bad, sm));
  int32_t hb = 0;
  st = readback(ctx, bad, sizeof(int32_t), &hb);
  if (st) return st;
  m->diag_ok = hb == 0;
  return GP2S_OK;
}

gp2s_status gp2s_matrix_set_block_product(gp2s_matrix m, int32_t nrhs, int32_t variant) {
  if (!m || nrhs < 2 || nrhs > kMaxProbes) return GP2S_E_INVALID;
  const bool sliced = nrhs == 8 || nrhs == 16 || nrhs == 32 || nrhs == 64;
  const bool ok = variant == -1 || variant == 0 || (variant == 1 && sliced) || (variant == 2 && sliced && m->assembled) ||
                  (variant == 3 && (nrhs == 32 || nrhs == 64)) || ((variant == 5 || variant == 6) && sliced) ||
                  entry_product_ok(nrhs, variant);
  if (!ok) return GP2S_E_INVALID;
  m->spmm_variant[nrhs] = variant == -1 ? -3 : variant;
  return GP2S_OK;
}

gp2s_status gp2s_matrix_get_block_product(gp2s_matrix m, int32_t nrhs, int32_t* variant) {
  if (!m || !variant || nrhs < 2 || nrhs > kMaxProbes) return GP2S_E_INVALID;
  *variant = m->spmm_variant[nrhs] < 0 ? -1 : m->spmm_variant[nrhs];
  return GP2S_OK;
}

gp2s_status gp2s_spmv(gp2s_ctx ctx, gp2s_matrix m, int32_t nrhs, const double* X, double* Y) {
  if (!ctx) return GP2S_E_INVALID;
  gp2s_status st = check_matrix(ctx, m);
  if (st) return st;
  if (nrhs < 1 || nrhs > kMaxProbes) return fail(ctx, GP2S_E_INVALID, "nrhs must be in [1, %d]", kMaxProbes);
  if (!X || !Y) return fail(ctx, GP2S_E_INVALID, "X and Y must be non-NULL");
  if ((int64_t)m->n * nrhs >= (int64_t)INT32_MAX)
    return fail(ctx, GP2S_E_INVALID, "n * nrhs must be below 2^31");
  st = ensure_device(ctx);
  if (st) return st;
  const int64_t n = m->n;
  Scratch sc(ctx);
  double* Xi = sc.get<double>((size_t)n * nrhs);
  double* Yi = sc.get<double>((size_t)n * nrhs);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "spmv workspace allocation failed");
  if (nrhs > 1 && m->spmm_variant[nrhs] == 3) {
    st = ensure_groups(ctx, m);
    if (st) return st;
  }
  if (nrhs > 1 && m->spmm_variant[nrhs] == 2) {
    st = ensure_tiles(ctx, m);
    if (st) return st;
  }
  if (nrhs > 1 && m->spmm_variant[nrhs] == 5) {
    st = ensure_bsplit(ctx, m);
    if (st) return st;
  }
  HIPCHK(launch_gather_rows(n, nrhs, m->perm, X, Xi, ctx->stream));
  if (nrhs == 1)
    TIMED(GP2S_T_SPMV,
          launch_spmv(m->prec, m->row_ptr, m->col, m->val, n, (double)m->nnz / n, Xi, Yi, ctx->stream, row_blocks(m)));
  else
    TIMED(GP2S_T_SPMM, launch_spmm(m->prec, m->row_ptr, m->col, m->val, n, nrhs, (double)m->nnz / n,
                                           m->spmm_variant[nrhs] >= 0 ? m->spmm_variant[nrhs] : -1, tile_set(m),
                                           Xi, Yi, ctx->stream));
  st = ff_apply(ctx, m, nrhs, Xi, Yi, sc);
  if (st) return st;
  HIPCHK(launch_scatter_rows(n, nrhs, m->perm, Yi, Y, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return GP2S_OK;
}


gp2s_status gp2s_spmv_noalloc(gp2s_ctx ctx, gp2s_matrix m, int32_t nrhs, const double* X, double* Y) {
  if (!ctx) return GP2S_E_INVALID;
  gp2s_status st = check_matrix(ctx, m);
  if (st) return st;
  if (nrhs < 1 || nrhs > kMaxProbes) return fail(ctx, GP2S_E_INVALID, "nrhs must be in [1, %d]", kMaxProbes);
  if (!X || !Y) return fail(ctx, GP2S_E_INVALID, "X and Y must be non-NULL");
  const int64_t n = m->n;
  if (n * nrhs > kNoAllocElems)
    return fail(ctx, GP2S_E_INVALID, "n * nrhs = %lld exceeds the allocation-free workspace of %lld values",
                (long long)(n * nrhs), (long long)kNoAllocElems);
  if (m->ffG) return fail(ctx, GP2S_E_INVALID, "the far-field term needs workspace: use gp2s_spmv");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return fail(ctx, GP2S_E_HIP, "no HIP device available");
  double* ws = nullptr;
  st = noalloc_workspace(ctx, &ws);
  if (st) return st;
  double* Xi = ws;
  double* Yi = ws + kNoAllocElems;
  // block-product variants whose per-matrix structures are not built yet (they would be
  // allocated on first use) give way to the heuristic choice; every variant gives the
  // same product up to the order of float64 summation
  int variant = nrhs > 1 ? m->spmm_variant[nrhs] : -1;
  if (variant == 2 && !m->tiles) variant = -1;
  if (variant == 3 && !(m->grp_ptr && m->grp_values)) variant = -1;
  if (variant == 5 && !(m->bs_val && m->bs_values)) variant = -1;
  HIPCHK(launch_gather_rows(n, nrhs, m->perm, X, Xi, ctx->stream));
  if (nrhs == 1)
    HIPCHK(launch_spmv(m->prec, m->row_ptr, m->col, m->val, n, (double)m->nnz / n, Xi, Yi, ctx->stream, row_blocks(m)));
  else
    HIPCHK(launch_spmm(m->prec, m->row_ptr, m->col, m->val, n, nrhs, (double)m->nnz / n, variant, tile_set(m), Xi, Yi,
                       ctx->stream));
  HIPCHK(launch_scatter_rows(n, nrhs, m->perm, Yi, Y, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return GP2S_OK;
}

gp2s_status gp2s_solve(gp2s_ctx ctx, gp2s_matrix m, const double* y, double* a, const gp2s_solve_opts* o,
                       gp2s_report* rep) {
  if (!ctx) return GP2S_E_INVALID;
  gp2s_status st = check_matrix(ctx, m);
  if (st) return st;
  st = check_opts(ctx, o, false);
  if (st) return st;
  if (!y || !a) return fail(ctx, GP2S_E_INVALID, "y and a must be non-NULL");
  st = ensure_device(ctx);
  if (st) return st;
  const int64_t n = m->n;
  Scratch sc(ctx);
  double* yi = sc.get<double>(n);
  double* ai = sc.get<double>(n);
  double* red = sc.get<double>(1 + kReduceBlocks);
  uint32_t* tk = sc.get<uint32_t>(1);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "solve workspace allocation failed");
  HIPCHK(hipMemsetAsync(tk, 0, sizeof(uint32_t), ctx->stream));
  HIPCHK(launch_gather_rows(n, 1, m->perm, y, yi, ctx->stream));
  gp2s_report local{};
  gp2s_report* r = rep ? rep : &local;
  std::memset(r, 0, sizeof(*r));
  if (pc_block(o->precond) && m->diag_ok) {
    st = ensure_bj(ctx, m, o->precond);
    if (st) return st;
  }
  bool conv = false;
  st = solve_internal(ctx, m, yi, ai, o, sc, r, &conv);
  if (st) return st;
  double yTa = 0.0;
  st = dot_host(ctx, n, yi, ai, red, tk, &yTa);
  if (st) return st;
  r->yTa = yTa;
  HIPCHK(launch_scatter_rows(n, 1, m->perm, ai, a, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (!conv) return fail(ctx, GP2S_E_NOCONV, "CG did not reach tol within max_iter / max_ir");
  return GP2S_OK;
}

gp2s_status gp2s_lml(gp2s_ctx ctx, gp2s_matrix m, const double* y, const gp2s_solve_opts* o, double* a,
                     gp2s_report* rep) {
  return lml_common(ctx, m, y, o, a, rep, nullptr);
}

gp2s_status gp2s_lml_grad(gp2s_ctx ctx, gp2s_matrix m, const double* y, const gp2s_solve_opts* o, double* a,
                          gp2s_report* rep, double* grad) {
  if (ctx && !grad) return fail(ctx, GP2S_E_INVALID, "grad is NULL");
  return lml_common(ctx, m, y, o, a, rep, grad);
}

gp2s_status gp2s_predict(gp2s_ctx ctx, gp2s_matrix m, int64_t n_test, const double* x_test, const double* a,
                         const gp2s_solve_opts* o, double* mean, double* var, gp2s_predict_report* rep) {
  if (!ctx) return GP2S_E_INVALID;
  gp2s_status st = check_matrix(ctx, m);
  if (st) return st;
  if (!m->assembled)
    return fail(ctx, GP2S_E_INVALID, "prediction needs a handle from gp2s_assemble (imported CSR has no kernel)");
  st = check_opts(ctx, o, false);
  if (st) return st;
  if (n_test < 0 || n_test >= (int64_t)INT32_MAX) return fail(ctx, GP2S_E_INVALID, "n_test must be in [0, 2^31)");
  if (n_test > 0 && (!x_test || !a || !mean)) return fail(ctx, GP2S_E_INVALID, "x_test, a and mean must be non-NULL");
  constexpr int kVarBlock = 64;
  if (var && (int64_t)m->n * kVarBlock >= (int64_t)INT32_MAX)
    return fail(ctx, GP2S_E_INVALID, "n * 64 must be below 2^31 for the variance blocks");
  if (rep) std::memset(rep, 0, sizeof(*rep));
  if (n_test == 0) return GP2S_OK;
  st = ensure_device(ctx);
  if (st) return st;
  const int64_t n = m->n, nt = n_test;
  const bool f32 = m->prec == GP2S_MIXED;
  hipStream_t sm = ctx->stream;
  Scratch sc(ctx);
  float4* t32 = f32 ? sc.get<float4>(nt) : nullptr;
  double4* t64 = f32 ? nullptr : sc.get<double4>(nt);
  double* g64t = sc.get<double>(nt);
  int32_t* tbin = sc.get<int32_t>(nt);
  int32_t* flag = sc.get<int32_t>(1);
  int32_t* row_cnt = sc.get<int32_t>(nt);
  int64_t* rp = sc.get<int64_t>(nt + 1);
  void* scan_ws = sc.get<uint8_t>(scan_workspace_bytes(nt));
  double* ai = sc.get<double>(n);
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "prediction workspace allocation failed");
  // test-point prologue on the training grid
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int32_t), sm));
  HIPCHK(launch_test_prologue(x_test, nt, m->grid, m->centers_d, m->weights_d, m->P, m->bump_width * m->bump_width,
                              t32, t64, g64t, tbin, flag, sm, m->ffU > 0));
  int32_t nf = 0;
  st = readback(ctx, flag, sizeof(int32_t), &nf);
  if (st) return st;
  if (nf) return fail(ctx, GP2S_E_NONFINITE, "x_test contains NaN or infinity");
  // cross-covariance k(x*, X): count, scan, fill
  CrossArgs ca{};
  ca.test32 = t32;
  ca.test64 = t64;
  ca.test_bin = tbin;
  ca.nt = nt;
  ca.pts32 = m->pts32;
  ca.pts64 = m->pts64;
  ca.bin_start = m->bin_start;
  ca.grid = m->grid;
  ca.r2 = m->radius * m->radius;
  ca.inv_r2 = 1.0 / ca.r2;
  ca.r2f = (float)ca.r2;
  ca.kern = m->kern;
  ca.kg = kern_geom(m);
  if (m->lsq) {
    double* lsq_t = sc.get<double>(nt);
    if (sc.oom) return fail(ctx, GP2S_E_OOM, "prediction workspace allocation failed");
    HIPCHK(launch_ell(nt, m->dim, x_test, m->centers_d, m->ls_d, m->P, m->bump_width * m->bump_width, lsq_t, sm));
    ca.lsq_test = lsq_t;
  }
  HIPCHK(launch_cross_count(ca, m->prec, row_cnt, sm));
  HIPCHK(launch_exscan_i32_i64(row_cnt, rp, nt, scan_ws, sm));
  int64_t nnz = 0;
  st = readback(ctx, rp + nt, sizeof(int64_t), &nnz);
  if (st) return st;
  int32_t* ccol = sc.get<int32_t>(std::max<int64_t>(nnz, 1));
  void* cval = sc.get<uint8_t>((size_t)std::max<int64_t>(nnz, 1) * (f32 ? sizeof(float) : sizeof(double)));
  if (sc.oom) return fail(ctx, GP2S_E_OOM, "cross-covariance allocation failed (%lld entries)", (long long)nnz);
  HIPCHK(launch_cross_fill(ca, m->prec, rp, ccol, cval, sm));
  // mean = K* a (a gathered into internal order)
  HIPCHK(launch_gather_rows(n, 1, m->perm, a, ai, sm));
  HIPCHK(launch_spmv(m->prec, rp, ccol, cval, nt, nnz > 0 ? (double)nnz / (double)nt : 1.0, ai, mean, sm));
  double* Gt = nullptr;  // far-field kernel: G* [nt * U] of the test points
  if (m->ffU > 0) {
    const int U = m->ffU;
    Gt = sc.get<double>((size_t)nt * U);
    double* C1 = sc.get<double>(U);
    double* part = sc.get<double>((size_t)U * ff_gtp_blocks(n));
    uint32_t* tk = sc.get<uint32_t>(1);
    if (sc.oom) return fail(ctx, GP2S_E_OOM, "prediction workspace allocation failed");
    HIPCHK(hipMemsetAsync(tk, 0, sizeof(uint32_t), sm));
    HIPCHK(launch_ff_G(nt, m->dim, x_test, m->centers_d, m->weights_d, m->ffgrp_d, m->P, U,
                       m->bump_width * m->bump_width, Gt, nullptr, sm));
    HIPCHK(launch_ff_gtp(n, 1, U, m->ffG, ai, false, part, tk, C1, sm));
    HIPCHK(launch_ff_add(nt, 1, U, Gt, C1, 1, 0, mean, sm));  // mean += G* (G^T a)
  }
  int32_t blocks = 0, worst = 0;
  bool conv = true;
  if (var) {
    if (pc_block(o->precond)) {
      if (!m->diag_ok) return fail(ctx, GP2S_E_NOT_SPD, "diagonal of K is not positive");
      st = ensure_bj(ctx, m, o->precond);
      if (st) return st;
    }
    double* B = sc.get<double>((size_t)n * kVarBlock);
    double* Vs = sc.get<double>((size_t)n * kVarBlock);
    double* csc = sc.get<double>(kVarBlock);
    if (sc.oom) return fail(ctx, GP2S_E_OOM, "variance block allocation failed");
    for (int64_t t0 = 0; t0 < nt; t0 += kVarBlock) {
      const int S = (int)std::min<int64_t>(kVarBlock, nt - t0);
      HIPCHK(hipMemsetAsync(B, 0, (size_t)n * S * sizeof(double), sm));
      if (Gt) {  // far-field kernel: k(X, x*) = W(X, x*) + G G*^T, dense; scaled per column
        HIPCHK(launch_cross_block(m->prec, rp, ccol, cval, t0, S, B, csc, sm, true));
        HIPCHK(launch_ff_add(n, S, m->ffU, m->ffG, Gt + t0 * m->ffU, 1, m->ffU, B, sm));
        HIPCHK(launch_ff_colscale(n, S, B, csc, sm));
      } else {
        HIPCHK(launch_cross_block(m->prec, rp, ccol, cval, t0, S, B, csc, sm));
      }
      Scratch scb(ctx);  // the block solve's workspace is released per block
      CgRun run;
      st = run_cg(ctx, m, S, B, Vs, o->tol, o->max_iter, o->check_every, false, scb, run, "variance block",
                  o->precond);
      if (st) return st;
      if (Gt)
        HIPCHK(launch_ff_var(n, S, m->ffU, B, Vs, csc, Gt, t0, var, sm));
      else
        HIPCHK(launch_cross_var(m->prec, rp, ccol, cval, t0, S, Vs, csc, g64t, var, sm));
      ++blocks;
      worst = std::max(worst, run.total_iters);
      conv = conv && run.converged;
    }
  }
  HIPCHK(hipStreamSynchronize(sm));
  if (rep) {
    rep->nnz_cross = nnz;
    rep->var_blocks = blocks;
    rep->var_iters = worst;
  }
  if (!conv) return fail(ctx, GP2S_E_NOCONV, "a variance block did not converge within max_iter");
  return GP2S_OK;
}

}  // extern "C"
