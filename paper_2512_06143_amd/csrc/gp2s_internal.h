// Internal declarations shared by the HIP kernels and the host runtime of libgp2s.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gp2s.h"

namespace gp2s {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per workgroup for streaming kernels
constexpr int kMaxProbes = 64;     // one probe per lane in the block kernels
constexpr int kMaxBumps = 256;
constexpr int kReduceBlocks = 4096;  // max workgroups of the reduction-carrying kernels
constexpr int kDotBlocks = 1024;     // workgroups of the block-preconditioned CG update (fewer partials per finalize)
constexpr int kBJ = 64;             // rows per block-Jacobi block of a batch instance (and of the block split)
constexpr int kBJM = 128;           // rows per block-Jacobi block of a matrix handle

// Point records (float4 / double4 of x, y, z and w) carry the bump mask g in w for a
// point strictly inside some bump, and a quiet NaN for a point outside every bump.
// The flag is therefore independent of the sign and value of g: amplitudes of any
// sign, and g = 0 inside a bump, keep the point in the stored pattern. Outside
// points never enter an entry value (every use tests the flag first).
__host__ __device__ inline float pt_out_f32() { return __builtin_nanf(""); }
__host__ __device__ inline double pt_out_f64() { return __builtin_nan(""); }
__device__ inline bool pt_in(float w) { return !__builtin_isnan(w); }
__device__ inline bool pt_in(double w) { return !__builtin_isnan(w); }
// g of a point record, 0 outside every bump.
__device__ inline double pt_g(double w) { return pt_in(w) ? w : 0.0; }
constexpr int kMaxGroups = 16;      // bump groups U of the far-field kernel

// Uniform grid of cubic bins with side h >= r (slightly enlarged so that rounding
// in the bin index can never separate two points closer than r by two bins).
struct GridDev {
  double origin[3];
  double inv_h[3];  // 1 / cell side along each axis
  int32_t nb[3];
  int32_t dim;
  int64_t nbins;
};

// Order of the points inside one cell: the Morton (Z-order) code of a point's offset
// from the cell's lower corner, in units of the cell side, on a sub-grid of 2^kSubBits
// steps per axis (bits interleaved, axis 0 in the lowest bit). The bin sort orders a
// cell's points by this code (ties by user index), so that runs of consecutive points,
// the blocks of the block-Jacobi preconditioner, are compact inside crowded cells.
// u = (x - origin) * inv_h is formed exactly as the cell coordinate is, and u - c is
// exact (Sterbenz), so the code is reproducible on any IEEE float64 machine.
constexpr int kSubBits = 10;
__device__ inline uint32_t sub_cell_code(const double* xi, const GridDev& g, int dim) {
  uint32_t code = 0;
  const double steps = (double)(1 << kSubBits);
  for (int k = 0; k < dim; ++k) {
    const double u = (xi[k] - g.origin[k]) * g.inv_h[k];
    const double c = fmax(0.0, fmin(floor(u), (double)(g.nb[k] - 1)));
    const double f = fmax(0.0, fmin(floor((u - c) * steps), steps - 1.0));
    const uint32_t fi = (uint32_t)f;
    for (int b = 0; b < kSubBits; ++b) code |= ((fi >> b) & 1u) << (dim * b + k);
  }
  return code;
}

// Device-resident solver state for one block CG run over S columns.
struct CgState {
  double* rz;        // [S] r^T M^-1 r of the current iterate
  double* bb;        // [S] ||b||^2
  double* tol2;      // [S] squared relative tolerance
  double* alpha;     // [S] step of the current iteration (0 for finished columns)
  double* beta;      // [S]
  double* rr;        // [S] ||r||^2 of the current iterate
  int32_t* done;     // [S] 1 once a column has converged
  int32_t* iters;    // [S] iterations performed per column
  int32_t* flags;    // [4] 0: breakdown (p^T K p <= 0), 2: non-finite, 3: breakdown column
  double* partial;   // [kReduceBlocks * S * 2] per-workgroup partial sums
  const double* lrC;  // far-field kernel: [U * S] G^T p of the current product (adds |G^T p|^2 to p^T q)
  int32_t lrU;
  double* hist_a;    // [max_iter * S] alpha history (Lanczos coefficients), or null
  double* hist_b;    // [max_iter * S] beta history, or null
  int32_t max_hist;
};

// Sum partial[b * C + c] over b < nb for every column c < C in a fixed order, using
// every thread of the calling workgroup (all threads must call it; C <= blockDim.x).
// sh must hold blockDim.x doubles. Threads c < C receive the sums via out(c, sum).
template <typename F>
__device__ inline void reduce_partials(const double* partial, int nb, int C, double* sh, F out) {
  const int nth = blockDim.x;
  const int chunks = nth / C;
  const int t = threadIdx.x;
  const int c = t % C, j = t / C;
  double v = 0.0;
  if (j < chunks)
    for (int b = j; b < nb; b += chunks) v += partial[(int64_t)b * C + c];
  sh[t] = v;
  __syncthreads();
  if (t < C) {
    double acc = 0.0;
    for (int q = 0; q < chunks; ++q) acc += sh[q * C + t];
    out(t, acc);
  }
  __syncthreads();
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2. For
// row-parallel kernels, give XCD x (workgroups with blockIdx % 8 == x) the contiguous
// row range [x n / 8, (x + 1) n / 8) and let its units interleave over consecutive rows
// inside it, so neighbouring rows -- whose gathers touch the same vector entries --
// share one L2. `unit` is this thread's unit index inside its workgroup (a wave or a
// lane group) and `units` the units per workgroup. The grid must be a multiple of 8.
struct XcdRows {
  int64_t first, step, end;
};
__device__ inline XcdRows xcd_rows(int64_t n, int unit, int units) {
  const int64_t xcd = blockIdx.x % 8;
  const int64_t blocks_x = gridDim.x / 8;
  const int64_t lb = blockIdx.x / 8;
  XcdRows r;
  r.first = n * xcd / 8 + lb * units + unit;
  r.step = blocks_x * units;
  r.end = n * (xcd + 1) / 8;
  return r;
}
__host__ inline int64_t round_up8(int64_t b) { return (b + 7) / 8 * 8; }

// A tile of consecutive (bin-sorted) rows for the LDS-staged block product, with the
// column intervals its rows can reference: the points of the neighbouring bins, which
// form one contiguous run of columns per neighbouring bin row (3 in 2-D, 9 in 3-D).
constexpr int kTileMaxIv = 9;
struct RowTile {
  int64_t row0;
  int32_t rows, niv;
  int32_t lo[kTileMaxIv], len[kTileMaxIv];
};
constexpr int kGrp = 4;  // rows per group of the row-grouped block product (grouped.hip)
struct TileSet {
  const RowTile* t = nullptr;
  int64_t n = 0;
  // row-grouped copy (variant 3): union columns of kGrp consecutive rows, one value per row
  const int64_t* gptr = nullptr;
  const int32_t* gcol = nullptr;
  const void* gval = nullptr;
  int64_t ngroups = 0;
  // block split (variant 5): dense 64 x 64 diagonal blocks in matrix-core operand order,
  // and per row the run [lo, hi) of its in-block entries
  const void* bval = nullptr;
  const int2* bseg = nullptr;
};
hipError_t launch_bs_build(int64_t n, const int64_t* rp, const int32_t* col, const void* val, int prec, void* Bv,
                           int2* seg, bool values_only, hipStream_t st);
template <typename V, typename PT, bool DOT>
bool spmm_split(const int64_t* rp, const int32_t* col, const V* val, int64_t n, int S, const TileSet& tiles,
                const PT* X, double* Y, const CgState& cs, hipStream_t st, int64_t row_blocks, int* nblocks);
hipError_t launch_grp_count(int64_t n, const int64_t* rp, const int32_t* col, int64_t ngroups, int32_t* cnt,
                            hipStream_t st);
hipError_t launch_grp_fill(int64_t n, const int64_t* rp, const int32_t* col, int64_t ngroups, const int64_t* gptr,
                           int32_t* gcol, int32_t* map, hipStream_t st);
hipError_t launch_grp_values(int64_t nnz, const void* val, int prec, const int32_t* map, void* gval, hipStream_t st);
constexpr int kTileLdsBytes = 72 * 1024;  // staged rows of X per workgroup (2 workgroups per CU)
constexpr int kTileBlock = 1024;          // 16 waves per workgroup hide the row-pointer latency
constexpr int kTileMaxRows = 64;          // rows per tile (at most)

// The entry-parallel block products exist for S in {8, 16, 32, 64} and G in {4, 8, 16}, G <= S.
__host__ inline bool entry_product_ok(int S, int G) {
  return (S == 8 || S == 16 || S == 32 || S == 64) && (G == 4 || G == 8 || G == 16) && G <= S;
}

// ---- batched instances ---------------------------------------------------------------
// Many independent instances form one block-diagonal system. Rows (and columns) are
// instance-major, bin-major inside an instance. Points are stored with three
// coordinates (z = 0 for 2-D instances, whose grids have nb[2] = 1), so one 3-D code
// path serves both dimensions with identical arithmetic.
constexpr int kBRows = 64;  // rows per workgroup in the batched CG kernels

struct BInst {
  GridDev grid;          // bins of side >= r / m (nb[2] = 1 in 2-D)
  int64_t row0, rows;    // row range of the instance (user rows are instance-major too)
  int64_t bin0;          // first global bin of the instance
  int64_t blk0, nblk;    // its workgroups in the instance-aligned decomposition
  double radius, r2, inv_r2, noise, bump_w2;
  int32_t dim, P, cent0, m;  // bump offset into the shared centre/weight arrays; bin refinement
  int32_t kern;              // Wendland member (0: C^2, 1: C^6)
};

struct BatchGeom {
  const BInst* inst;         // [M]
  int32_t M;
  const int64_t* row_start;  // [M + 1] row0 of every instance, then the total
  const int32_t* inst_of_row;  // [N]
  const int32_t* blk_inst;     // [number of workgroups] instance of each workgroup
  int64_t n, nblk;
  // CG row kernels launch `grid` workgroups; workgroup k works on row block
  // blk_map[k] (identity when blk_map is null), so converged instances can be dropped.
  const int32_t* blk_map;
  int64_t grid;
};

// ---- kernel launchers (defined in the .hip files) ---------------------------------
// prologue.hip
hipError_t launch_bbox(const double* x, int64_t n, int dim, double* part, int32_t* nonfinite,
                       int nblocks, hipStream_t st);
hipError_t launch_prologue(const double* x, int64_t n, const GridDev& g, const double* centers,
                           const double* weights, int P, double bump_w2, int32_t* bin_of,
                           int32_t* slot, int32_t* bin_count, double* g64_user, uint8_t* gam,
                           uint32_t* fkey, hipStream_t st, bool unit = false);  // unit: g = 1 at every point
hipError_t launch_scatter(int64_t n, const int32_t* bin_of, const int32_t* slot, const uint32_t* fkey,
                          const int64_t* bin_start, int32_t* perm_tmp, uint32_t* key_tmp, hipStream_t st);
hipError_t launch_binsort(int64_t n, const int32_t* perm_tmp, const uint32_t* key_tmp, const int32_t* bin_of,
                          const int64_t* bin_start, int32_t* perm, hipStream_t st);
hipError_t launch_refresh_g(int64_t n, int dim, const double* x64, const double* centers, const double* weights,
                            int P, double bump_w2, float4* pts32, double4* pts64, double* g64, hipStream_t st);
hipError_t launch_gather_points(int64_t n, int dim, const double* x, const int32_t* perm,
                                const int32_t* bin_of, const double* g64_user, const uint8_t* gam,
                                float4* pts32, double4* pts64, double* x64, double* g64,
                                int32_t* binid, hipStream_t st);
hipError_t launch_probe_masks(int64_t n, const int32_t* perm, uint64_t seed, int S, uint64_t* mask,
                              hipStream_t st);

// scan.hip: exclusive prefix sum of int32 counts into int64 offsets (out has n+1 entries).
size_t scan_workspace_bytes(int64_t n);
hipError_t launch_exscan_i32_i64(const int32_t* in, int64_t* out, int64_t n, void* ws,
                                 hipStream_t st);
hipError_t launch_i64_to_i32(const int64_t* in, int32_t* out, int64_t n, hipStream_t st);

// assemble.hip
// Per-axis geometry of the general kernel (Eq. wendconv with axis radii and the
// length-scale field l). general == 0 keeps the isotropic stationary path; otherwise
// the support test is sum_k ((x_ik - x_jk) / r_k)^2 < m_ij, m_ij = (l_i^2 + l_j^2) / 2
// (1 without the field), and entries carry the prefactor (l_i l_j / m_ij)^{d/2}.
struct KernGeom {
  double inv_r[3];    // 1 / r_k
  float inv_rf[3];
  const double* lsq;  // [n] l(x)^2 of the training points (internal order), or nullptr
  int32_t general;
};

struct AssembleArgs {
  const float4* pts32;
  const double4* pts64;
  const double* g64;
  const int32_t* binid;
  const int64_t* bin_start;
  GridDev grid;
  int64_t n;
  double radius, r2, inv_r2, noise;
  float r2f;
  int32_t kern;  // Wendland member (0: C^2, 1: C^6)
  KernGeom kg;
};
hipError_t launch_assemble_count(const AssembleArgs& a, int prec, int32_t* row_cnt, hipStream_t st);
hipError_t launch_assemble_fill(const AssembleArgs& a, int prec, const int64_t* row_ptr,
                                int32_t* col, void* val, double* diag, hipStream_t st);

// predict.hip: cross-covariance of test points with the training points
struct CrossArgs {
  const float4* test32;   // test points (float32 path) or null
  const double4* test64;  // test points (float64 path) or null
  const int32_t* test_bin;
  int64_t nt;
  const float4* pts32;  // training points, internal order
  const double4* pts64;
  const int64_t* bin_start;
  GridDev grid;
  double r2, inv_r2;
  float r2f;
  int32_t kern;
  KernGeom kg;
  const double* lsq_test;  // [nt] l(x*)^2 of the test points, or nullptr
};
hipError_t launch_test_prologue(const double* x, int64_t nt, const GridDev& g, const double* centers,
                                const double* weights, int P, double bump_w2, float4* pts32, double4* pts64,
                                double* g64, int32_t* bin, int32_t* nonfinite, hipStream_t st, bool unit = false);
hipError_t launch_cross_count(const CrossArgs& a, int prec, int32_t* row_cnt, hipStream_t st);
hipError_t launch_cross_fill(const CrossArgs& a, int prec, const int64_t* row_ptr, int32_t* col, void* val,
                             hipStream_t st);
// raw: values unscaled (cs untouched), for right-hand sides completed and scaled later
hipError_t launch_cross_block(int prec, const int64_t* rp, const int32_t* col, const void* val, int64_t t0, int S,
                              double* B, double* cs, hipStream_t st, bool raw = false);
hipError_t launch_cross_var(int prec, const int64_t* rp, const int32_t* col, const void* val, int64_t t0, int S,
                            const double* Vs, const double* cs, const double* g64t, double* var, hipStream_t st);

// spmv.hip
// Entries allocated past nnz in a matrix handle's col and val (zeroed: column 0, value
// 0), so that the streaming single-RHS product may read whole 16-byte quads.
constexpr int64_t kQuadPad = 4;
// Row blocks of the streaming single-RHS product: blk[b] = the first row whose first
// entry is at or past b * 2048, b < n; blk[n] = the row count. {nullptr, 0}: the CSR has
// no blocks (not a matrix handle's) and the lane-group product is used.
struct RowBlocks {
  const int32_t* blk;
  int64_t n;
};
int64_t rowblocks_count(int64_t nnz);
hipError_t launch_rowblocks(const int64_t* rp, int64_t n, int64_t nnz, int32_t* rowblk, hipStream_t st);
// rb: the CSR's row blocks (its col and val then hold kQuadPad valid entries past nnz)
hipError_t launch_spmv(int prec, const int64_t* rp, const int32_t* col, const void* val,
                       int64_t n, double mean_row, const double* x, double* y, hipStream_t st,
                       const RowBlocks& rb = RowBlocks{nullptr, 0});
hipError_t launch_spmm(int prec, const int64_t* rp, const int32_t* col, const void* val,
                       int64_t n, int S, double mean_row, int variant, const TileSet& tiles, const double* X,
                       double* Y, hipStream_t st);
// CG product step: Q = K P plus p^T q per column, then alpha = rz / p^T q (rb as for
// launch_spmv, used when S == 1).
// P is float32 when f32vec (block solves of the mixed path), else float64; Q is float64.
// `variant` selects the block product for S > 1: 0 one lane per column, G > 0 the
// entry-parallel product with G lanes per row, -1 a choice from S and the mean row length.
hipError_t launch_cg_matvec(int prec, const int64_t* rp, const int32_t* col, const void* val,
                            int64_t n, int S, double mean_row, int variant, const TileSet& tiles, const void* P,
                            void* Q, bool f32vec, const CgState& cs, hipStream_t st,
                            const RowBlocks& rb = RowBlocks{nullptr, 0});

// pcg.hip
hipError_t launch_cg_alpha(const CgState& cs, int nb, int S, hipStream_t st);
hipError_t launch_cg_init(int64_t n, int S, const double* B, const double* dinv, double* X,
                          double* R, void* P, bool f32vec, const CgState& cs, double tol, hipStream_t st);
// X == nullptr: the solution is not formed (coefficients only).
hipError_t launch_cg_update(int64_t n, int S, double* X, double* R, const void* P, const void* Q,
                            bool f32vec, const double* dinv, const CgState& cs, int32_t iter,
                            hipStream_t st);
hipError_t launch_cg_pupdate(int64_t n, int S, void* P, const double* R, const double* dinv, bool f32vec,
                             const CgState& cs, hipStream_t st);
// p = z + beta p with z in float32 (see launch_bj_update).
hipError_t launch_cg_pupdate_z32(int64_t n, int S, void* P, const float* Z, bool f32vec, const CgState& cs,
                                 hipStream_t st);
hipError_t launch_axpy_sub(int64_t n, const double* b, const double* kx, double* r, hipStream_t st);
hipError_t launch_add(int64_t n, double* x, const double* d, hipStream_t st);
hipError_t launch_dot_partial(int64_t n, const double* a, const double* b, double* out,
                              uint32_t* ticket, hipStream_t st);
hipError_t launch_sum_log(int64_t n, const double* d, double* out, uint32_t* ticket, hipStream_t st);
hipError_t launch_gather_rows(int64_t n, int S, const int32_t* perm, const double* src_user,
                              double* dst_int, hipStream_t st);
hipError_t launch_scatter_rows(int64_t n, int S, const int32_t* perm, const double* src_int,
                               double* dst_user, hipStream_t st);
hipError_t launch_cg_init_fin(const CgState& cs, int nb, int S, double tol, hipStream_t st);

// farfield.hip: the rank-U bump term of Eq. bump_kernel (K = K_loc + G G^T)
hipError_t launch_ff_G(int64_t n, int dim, const double* x, const double* centers, const double* weights,
                       const int32_t* group, int P, int U, double bump_w2, double* G, double* diag, hipStream_t st);
unsigned ff_gtp_blocks(int64_t n);  // partial needs U * S * ff_gtp_blocks(n) doubles
hipError_t launch_ff_gtp(int64_t n, int S, int U, const double* G, const void* X, bool f32, double* partial,
                         uint32_t* ticket, double* C, hipStream_t st);
hipError_t launch_ff_add(int64_t n, int S, int U, const double* G, const double* C, int64_t cu, int64_t cs, double* Y,
                         hipStream_t st);
hipError_t launch_ff_wjac(int64_t n, int S, const uint64_t* mask, const double* dinv, double* W, hipStream_t st);
hipError_t launch_ff_h(int64_t n, int S, int U, const double* a, const double* Q, const double* W, const double* ag,
                       const double* wg, const double* qg, double* H, hipStream_t st);
hipError_t launch_ff_colscale(int64_t n, int S, double* B, double* cs, hipStream_t st);
hipError_t launch_ff_var(int64_t n, int S, int U, const double* B, const double* V, const double* cs,
                         const double* Gt, int64_t t0, double* var, hipStream_t st);
hipError_t launch_cg_beta(const CgState& cs, int nb, int S, int32_t iter, hipStream_t st);

// blockjac.hip: block-Jacobi factor (L, M^-1 in matrix-core operand order, pivots
// L_ii^2; bad != 0 when a block is not positive definite), the fused update
// (B != nullptr: initialisation r = B, x = 0) with z = M^-1 r, the probe right-hand
// sides L z, and the direction copy P = Z.
// Explicit block list (the batched path: 64-row runs inside each instance): block b
// covers rows r0[b] .. r0[b] + m[b] - 1. {nullptr, nullptr, 0}: consecutive 64-row runs
// from row 0.
struct BjBlocks {
  const int64_t* r0;
  const int32_t* m;
  int64_t n;
};
// M32 (optional): a float32 copy of M^-1 in the same order, for the y and refinement solves.
hipError_t launch_bj_factor(int64_t n, const int64_t* rp, const int32_t* col, const void* val, int prec,
                            const double* G, int U, double* L, double* Mfrag, float* M32, double* piv, int32_t* bad,
                            hipStream_t st, const BjBlocks& bl, int bj);
unsigned bj_update_blocks(int64_t n, int bj);
// M32 non-null: apply the float32 copy of M^-1 instead (single-column solves whose
// preconditioner enters no estimator; with S > 1 the call fails).
// Z32 non-null: store z in float32 there instead of Z (the mixed path's probe block,
// whose float32 directions are formed from it by launch_cg_pupdate_z32).
hipError_t launch_bj_update(int64_t n, int S, const double* B, double* X, double* R, const void* P, const void* Q,
                            bool f32vec, const double* Mfrag, double* Z, const CgState& cs, hipStream_t st,
                            const float* M32, float* Z32, int bj);
hipError_t launch_bj_rhs(int64_t n, int S, const uint64_t* mask, const double* L, double* B, hipStream_t st,
                         const BjBlocks& bl, int bj);
hipError_t launch_copy_dir(int64_t n, int S, const double* Z, void* P, bool f32vec, hipStream_t st);
hipError_t launch_probe_rhs(int64_t n, int S, const uint64_t* mask, const double* diag, double* B,
                            hipStream_t st);
hipError_t launch_dinv(int64_t n, const double* diag, double* dinv, int32_t* bad, hipStream_t st);
hipError_t launch_extract_diag(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col, const void* val, int prec,
                               double* diag, int32_t* bad, hipStream_t st);
hipError_t launch_check_finite(int64_t n, const double* v, int32_t* flag, hipStream_t st);

// slq.hip: per-probe e1^T ln(T) e1 from the CG coefficients.
// work: 2 * S * max_m doubles, max_m >= every iters[s].
hipError_t launch_slq_ws(int S, const double* hist_a, const double* hist_b, const int32_t* iters,
                         double* work, int64_t max_m, double* out, hipStream_t st);

// backward.hip
struct BackwardArgs {
  const int64_t* rp;
  const int32_t* col;
  const float4* pts32;
  const double4* pts64;
  const double* g64;
  const double* a;        // [n] K^-1 y (internal order)
  const double* Q;        // [n * S] probe solutions (internal order)
  const uint64_t* mask;   // [n] probe sign bits
  const double* dinv;     // [n] 1 / K_ii
  const double* W;        // [n * S] trace vectors w_s (block preconditioner), or nullptr:
                          // w_s = D^-1/2 z_s from the signs and dinv
  int64_t n;
  int S;
  double radius, r2, inv_r2;
  int32_t kern;  // Wendland member (0: C^2, 1: C^6)
  KernGeom kg;   // general kernel: radius rows T hold nr = 1 or dim components
  int32_t nr;
  int32_t dim;
};
// Rrow [n], Trow [nr * n], Urow [n], Vrow [n] (length-scale field only, else nullptr)
hipError_t launch_backward_rows(const BackwardArgs& b, int prec, double* Rrow, double* Trow,
                                double* Urow, double* Vrow, hipStream_t st);
// grad = (radius components [nr], a_1..a_P, [c_1..c_P when Vrow], sigma^2); with Hrow
// (far-field kernel) amplitude p takes sum_i bhat_p(x_i) Hrow[i * U + group[p]] in place of R
hipError_t launch_grad_reduce(int64_t n, int dim, int P, int S, int nr, const double* x64, const double* g64,
                              const double* a, const double* Rrow, const double* Trow,
                              const double* Urow, const double* Vrow, const double* Hrow, const int32_t* group,
                              int U, const double* centers, double bump_w2,
                              double* partial, uint32_t* ticket, double* grad, hipStream_t st);
// lsq[i] = l(x_i)^2 = exp(2 sum_q c_q bhat_q(x_i)) for n points x (row-major, dim)
hipError_t launch_ell(int64_t n, int dim, const double* x, const double* centers, const double* ls_w, int P,
                      double bump_w2, double* lsq, hipStream_t st);

// batch.hip
hipError_t launch_bbbox(const double* x3, const BatchGeom& g, double* part, int32_t* nonfinite, hipStream_t st);
hipError_t launch_bprologue(const double* x3, const BatchGeom& g, const double* centers3, const double* weights,
                            int32_t* bin_of, int32_t* slot, int32_t* bin_count, double* g64_user, uint8_t* gam,
                            uint32_t* fkey,
                            hipStream_t st);
hipError_t launch_bgather(const double* x3, const BatchGeom& g, const int32_t* perm, const int32_t* bin_of,
                          const double* g64_user, const uint8_t* gam, float4* pts32, double4* pts64, double* x64,
                          double* g64, int32_t* binid, int32_t* inst_of_row, hipStream_t st);
struct BAsm {
  BatchGeom g;
  const float4* pts32;
  const double4* pts64;
  const double* g64;
  const int32_t* binid;
  const int64_t* bin_start;
  int64_t cap;  // fill: writes stop at this many entries (capacity of col/val)
};
hipError_t launch_bassemble_count(const BAsm& a, int prec, int32_t* row_cnt, hipStream_t st);
hipError_t launch_bassemble_fill(const BAsm& a, int prec, const int64_t* row_ptr, int32_t* col, void* val,
                                 double* diag, int32_t* overflow, hipStream_t st);
hipError_t launch_bprobe_masks(const BatchGeom& g, const int32_t* perm, uint64_t seed, int S, uint64_t* mask,
                               hipStream_t st);
// Batched CG over instance-aligned workgroups; S columns per instance (a power of two <= 64).
hipError_t launch_bcg_matvec(int prec, const BatchGeom& g, const int64_t* rp, const int32_t* col, const void* val,
                             int S, int lanes, const void* P, void* Q, bool f32vec, const CgState& cs,
                             hipStream_t st);
hipError_t launch_bcg_init(const BatchGeom& g, int S, const double* B, const double* dinv, double* X, double* R,
                           void* P, bool f32vec, const CgState& cs, double tol, hipStream_t st);
hipError_t launch_bcg_update(const BatchGeom& g, int S, double* X, double* R, const void* P, const void* Q,
                             bool f32vec, const double* dinv, const CgState& cs, const int32_t* iter_dev,
                             hipStream_t st);
hipError_t launch_bcg_pupdate(const BatchGeom& g, int S, void* P, const double* R, const double* dinv, bool f32vec,
                              const CgState& cs, int32_t* iter_dev, hipStream_t st);
// Block-Jacobi batched CG (block list: the batch's row blocks): initialisation r = B,
// x = 0, z = M^-1 r, p = z; and the per-iteration update x, r, z = M^-1 r with beta.
// The direction update is launch_bcg_pupdate with R = Z and dinv = nullptr.
// M32 as for launch_bj_update.
hipError_t launch_bbj_init(const BatchGeom& g, int S, const double* B, double* X, double* R, void* P, bool f32vec,
                           const double* Mfrag, double* Z, const CgState& cs, double tol, hipStream_t st,
                           const float* M32 = nullptr);
hipError_t launch_bbj_update(const BatchGeom& g, int S, double* X, double* R, const void* P, const void* Q,
                             bool f32vec, const double* Mfrag, double* Z, const CgState& cs, const int32_t* iter_dev,
                             hipStream_t st, const float* M32 = nullptr);
// out[i] over instance i's rows: mode 0 = a.b, 1 = sum ln a
hipError_t launch_bseg_reduce(const BatchGeom& g, int mode, const double* a, const double* b, double* out,
                              hipStream_t st);
struct BBackward {
  BatchGeom g;
  const int64_t* rp;
  const int32_t* col;
  const float4* pts32;
  const double4* pts64;
  const double* a;
  const double* Q;
  const uint64_t* mask;
  const double* dinv;
  const double* g64;  // [n_total] bump values (float64; the mixed path's dK is evaluated in float64)
  const double* W;    // [n_total * S] trace vectors L^-T z (block preconditioner); null: from mask and dinv
  int S;
};
hipError_t launch_bbackward_rows(const BBackward& b, int prec, double* Rrow, double* Trow, double* Urow,
                                 hipStream_t st);
// grad[goff[i] + c] for c < P_i + 2 (r, a_1..a_P, sigma^2) of every instance
hipError_t launch_bgrad_reduce(const BatchGeom& g, int S, const double* x64, const double* g64, const double* a,
                               const double* Rrow, const double* Trow, const double* Urow, const double* centers3,
                               const int32_t* goff, double* grad, hipStream_t st);

}  // namespace gp2s
