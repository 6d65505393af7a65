// Compressed operator: H2 in space (Section 4) x MACA across frequencies
// (Section 5), combined as in Algorithm 3.
#pragma once
#include "internal.h"

namespace cqm {

struct Cluster {
  int begin = 0, end = 0;  // range in cluster order (positions in perm)
  int level = 0, parent = -1, nsons = 0;
  int son[2] = {-1, -1};
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // box of the supports
  int leaf_id = -1;        // index among leaves
  int size() const { return end - begin; }
};

// Block kinds: far blocks keep the Tucker core (p x p) when it is smaller
// than the block, otherwise they are stored expanded U_r C_k U_c^T like near
// blocks (same values, smaller storage and work).
constexpr int kFarCore = 0;
constexpr int kFarExpanded = 1;
constexpr int kNear = 2;

struct BlockDesc {
  int r, c, kind;
  int rows, cols;          // p x p for far blocks during MACA; #r x #c otherwise
  int64_t stage_off;       // MACA output slices (FP64) in the staging buffer
  int64_t c_off;           // apply-ready slices (rank x arows x acols)
  int64_t d_off;           // fibres (Rcap x nsys, FP64)
  int arows, acols;        // apply-ready slice shape
};

// Entries of the per-leaf product lists for expanded blocks.
struct LeafTask {
  int block;   // block index
  int rowoff;  // first row of the leaf inside the block's row cluster
};

// Block-rank products on the matrix cores: 16 output rows and their tasks.
struct RankTile {
  int out_row0, nrows, t0, t1;
};
struct RankTask {
  int64_t c_off;  // slice element of (first row of the tile, column 0), rank term 0
  int64_t d_off;  // fibre of rank term 0 (stride: systems of the operator)
  int cstride;    // elements between rank terms
  int ldc;        // row length of the slice
  int acols;      // columns
  int block;      // block index (its rank is read on the device)
  int x_row0;     // first input row
  int pad;
};

struct H2Operator {
  int m = 4, p = 64, nsys = 0, Rcap = 48;
  std::vector<int> perm, iperm;
  std::vector<Cluster> cl;
  std::vector<int> leaves;
  int nlevels = 0;
  std::vector<std::vector<int>> by_level;
  std::vector<BlockDesc> blocks;
  std::vector<int> core_blocks;               // far blocks kept as cores
  std::vector<std::vector<int>> core_by_row;  // per cluster: core blocks with that row
  std::vector<int> ranks;
  int n_far = 0, n_near = 0, n_core = 0;
  int max_rank = 0;
  double mean_rank = 0;
  int64_t bytes = 0;
  int64_t plain_bytes = 0;  // the same blocks per frequency (no MACA)
  // host FP64 data
  std::vector<double> nodes;   // per cluster 3*m Chebyshev nodes
  std::vector<double> Uleaf;   // per leaf #r x p (row-major)
  std::vector<int64_t> uleaf_off;
  std::vector<double> E;       // per cluster p x p transfer to its parent
  std::vector<double> Ufull;   // per cluster that needs it: #r x p
  std::vector<int64_t> ufull_off;
  // device copies
  int* perm_d = nullptr;
  double* nodes_d = nullptr;
  double* U_d = nullptr;
  float* U32_d = nullptr;
  int64_t* uleaf_off_d = nullptr;
  double* E_d = nullptr;
  float* E32_d = nullptr;
  double* Ufull_d = nullptr;
  int64_t* ufull_off_d = nullptr;
  int* cl_d = nullptr;           // per cluster: begin, end, parent, leaf_id
  BlockDesc* blocks_d = nullptr;
  int* ranks_d = nullptr;
  // per row cluster core-block lists (CSR)
  int* core_rowptr_d = nullptr;
  int* core_list_d = nullptr;
  // per leaf expanded/near task lists (CSR)
  int* task_rowptr_d = nullptr;
  LeafTask* tasks_d = nullptr;
  int* level_cl_d = nullptr;     // clusters grouped by level
  // block-rank product tables: couplings into cluster coefficient rows, and
  // expanded-far / near blocks into the leaves' rows (cluster order)
  RankTile* core_tiles_d = nullptr;
  RankTask* core_tasks_d = nullptr;
  RankTile* leaf_tiles_d = nullptr;
  RankTask* leaf_tasks_d = nullptr;
  int n_core_tiles = 0, n_leaf_tiles = 0;
  // time marching, fast right-hand side (eq. fastrhs): per block the rank
  // terms' fibre-convolved column histories z_{b,t} (Rcap x acols, from
  // zoff[b]), the cluster coefficients of every past step and the split-K
  // partial rows of the one-system products
  int64_t* zoff_d = nullptr;
  int64_t z_elems = 0;
  std::vector<int> level_off;
  // workspace regions (byte offsets from the problem's H2 region)
  size_t off_cstore = 0, off_dvec = 0, off_stage = 0, off_xhat = 0, off_yhat = 0, total = 0;
  size_t off_xp = 0, off_yp = 0;
  size_t off_dhat = 0;  // marching: the fibres' transforms (integration weights)
  size_t off_w0 = 0;    // marching: collapsed lag-0 slices (storage precision)
  size_t off_w0dense = 0;  // marching: What_0 = Re W0, dense M x M (FP64)
  size_t off_z = 0, off_hxh = 0, off_rpart = 0;  // marching: fast right-hand side
  int64_t cstore_elems = 0, dvec_elems = 0, stage_elems = 0;
  int64_t stage_budget = 0;       // cf64 elements per MACA batch
  std::vector<std::pair<int, int>> batches;  // [b0, b1) per MACA launch
  int store_fp64 = 0;             // apply-ready slices in FP64 (else FP32)
  // per-problem views into the workspace (set before use)
  cf64* stage_d = nullptr;
  cf64* dvec_d = nullptr;
  cf64* dhat_d = nullptr;
  void* w0_d = nullptr;   // W0_b = sum_t dhat_t[0] C_t per block, at c_off / Rcap
  double* w0dense_d = nullptr;
  bool w0_ready = false;  // both formed for the current slices
  cf64* z_d = nullptr;
  cf64* hxh_d = nullptr;
  cf64* rpart_d = nullptr;
  void* cstore_d = nullptr;
  void* xhat_d = nullptr;
  void* yhat_d = nullptr;
  void* xp_d = nullptr;  // inputs in cluster order [k][l]
  void* yp_d = nullptr;
  bool built = false;
};

// host planner (h2_tree.cpp)
void h2_build_structure(Problem& p, H2Operator& h);

// kernels (k_maca.hip, k_h2.hip)
void launch_maca(const Problem& p, H2Operator& h, int b0, int nb, hipStream_t s);
void launch_maca_finalize_batch(const Problem& p, H2Operator& h, int b0, int nb, hipStream_t s);
template <typename R>
void launch_h2_apply(const Problem& p, H2Operator& h, int l0, int nsys, const cplx<R>* x, int64_t xs,
                     cplx<R>* y, int64_t ys, const cf64* fibres, hipStream_t s);
// W0_b = sum_{t < rank_b} dhat_t[0] C_t for every block, in FP64, stored in
// the storage precision at the compact offsets
void launch_collapse_lag0(const Problem& p, H2Operator& h, hipStream_t s);
// What_0 = Re W0 written densely (M x M, triangle order, FP64): near and
// expanded far blocks copy their slice, cores add U_r Re(W0_b) U_c^T
void launch_expand_lag0(const Problem& p, H2Operator& h, hipStream_t s);
// y = What_0 q (q complex with zero imaginary part; y likewise)
void launch_lag0_dense_product(const H2Operator& h, const cf64* q, cf64* y, hipStream_t s);
// fast right-hand side of the compressed marching (eq. fastrhs), FP64:
// push: hx = step m's input x (triangle order) in cluster order, and its
// cluster coefficients into history slot m; sum: y = sum_{k=1}^{n}
// What_k x_{n-k} from the histories hx (rows m = 0 .. n-1, M each)
constexpr int kConvSplit = 8;  // split-K factor of the one-system products
void launch_h2_push_history(const Problem& p, H2Operator& h, int m, const cf64* x, cf64* hx,
                            hipStream_t s);
void launch_h2_fast_history(const Problem& p, H2Operator& h, int n, const cf64* hx, cf64* y,
                            hipStream_t s);
// scaled inverse DFT of every fibre slot (eq. fastdft): dhat[n] =
// rho^-n / F sum_l d[l] zeta^(n l mod F); full band only
void launch_fibre_dft(const Problem& p, const H2Operator& h, const cf64* d, cf64* dhat, hipStream_t s);
size_t h2_apply_scratch_bytes(const H2Operator& h, int nsys);
size_t h2_perm_scratch_bytes(const H2Operator& h, int nsys);

}  // namespace cqm
