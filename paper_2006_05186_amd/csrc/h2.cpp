// Compressed operator driver: structure and tables at problem creation,
// MACA of all blocks on the GPU when the operator is prepared, products for
// the GMRES iterations.
#include <algorithm>
#include <numeric>

#include "h2_internal.h"

namespace cqm {
bool mode_is_mixed(int mode);

namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T> T* up(const std::vector<T>& h) {
  if (h.empty()) return nullptr;
  T* d = nullptr;
  CQM_HIP(hipMalloc(&d, sizeof(T) * h.size()));
  CQM_HIP(hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return d;
}
template <typename T> void release(T*& d) {
  if (d) (void)hipFree(d);
  d = nullptr;
}

void setup_structure(Problem& p) {
  if (!p.h2) p.h2 = new H2Operator();
  H2Operator& h = *p.h2;
  if (h.built) return;
  require(p.opt.cheb_m >= 2 && p.opt.cheb_m <= 8, CQM_EINVAL, "compressed modes support cheb_m in [2, 8]");
  h2_build_structure(p, h);
  h.store_fp64 = mode_is_mixed(p.opt.mode) ? 0 : 1;
  const int ncl = (int)h.cl.size(), nleaf = (int)h.leaves.size();
  // level lists followed by the leaves in leaf order
  std::vector<int> lvl;
  h.level_off.assign(h.nlevels + 1, 0);
  for (int lv = 0; lv < h.nlevels; ++lv) {
    h.level_off[lv] = (int)lvl.size();
    lvl.insert(lvl.end(), h.by_level[lv].begin(), h.by_level[lv].end());
  }
  h.level_off[h.nlevels] = (int)lvl.size();
  lvl.insert(lvl.end(), h.leaves.begin(), h.leaves.end());
  // core blocks per row cluster (CSR over clusters)
  std::vector<int> crow(ncl + 1, 0), clist;
  for (int c = 0; c < ncl; ++c) {
    clist.insert(clist.end(), h.core_by_row[c].begin(), h.core_by_row[c].end());
    crow[c + 1] = (int)clist.size();
  }
  // expanded-far and near blocks per leaf of their row cluster
  std::vector<std::vector<LeafTask>> per_leaf(nleaf);
  std::vector<int> leaf_begin(nleaf);
  for (int k = 0; k < nleaf; ++k) leaf_begin[k] = h.cl[h.leaves[k]].begin;
  for (int b = 0; b < (int)h.blocks.size(); ++b) {
    const BlockDesc& B = h.blocks[b];
    if (B.kind == kFarCore) continue;
    const Cluster& R = h.cl[B.r];
    int k = (int)(std::lower_bound(leaf_begin.begin(), leaf_begin.end(), R.begin) - leaf_begin.begin());
    for (; k < nleaf && leaf_begin[k] < R.end; ++k) per_leaf[k].push_back(LeafTask{b, leaf_begin[k] - R.begin});
  }
  std::vector<int> trow(nleaf + 1, 0);
  std::vector<LeafTask> tasks;
  for (int k = 0; k < nleaf; ++k) {
    tasks.insert(tasks.end(), per_leaf[k].begin(), per_leaf[k].end());
    trow[k + 1] = (int)tasks.size();
  }
  // block-rank product tables (16-row tiles)
  {
    std::vector<RankTile> ct, lt;
    std::vector<RankTask> ck, lk;
    const int P = h.p;
    for (int r = 0; r < ncl; ++r)
      for (int r0 = 0; r0 < P; r0 += 16) {
        RankTile t{r * P + r0, std::min(16, P - r0), (int)ck.size(), 0};
        for (int b : h.core_by_row[r]) {
          const BlockDesc& B = h.blocks[b];
          ck.push_back(RankTask{B.c_off + (int64_t)r0 * B.acols, B.d_off, B.arows * B.acols, B.acols,
                                B.acols, b, B.c * P, 0});
        }
        t.t1 = (int)ck.size();
        ct.push_back(t);
      }
    for (int k = 0; k < nleaf; ++k) {
      const Cluster& Lc = h.cl[h.leaves[k]];
      for (int r0 = 0; r0 < Lc.size(); r0 += 16) {
        RankTile t{Lc.begin + r0, std::min(16, Lc.size() - r0), (int)lk.size(), 0};
        for (int q = trow[k]; q < trow[k + 1]; ++q) {
          const LeafTask& T = tasks[q];
          const BlockDesc& B = h.blocks[T.block];
          lk.push_back(RankTask{B.c_off + (int64_t)(T.rowoff + r0) * B.acols, B.d_off,
                                B.arows * B.acols, B.acols, B.acols, T.block, h.cl[B.c].begin, 0});
        }
        t.t1 = (int)lk.size();
        lt.push_back(t);
      }
    }
    if (ck.empty()) ck.push_back(RankTask{});
    if (lk.empty()) lk.push_back(RankTask{});
    // fast right-hand side: z_{b,t} slots, Rcap x acols per block
    std::vector<int64_t> zoff(std::max<size_t>(h.blocks.size(), 1), 0);
    int64_t zo = 0;
    for (size_t b = 0; b < h.blocks.size(); ++b) {
      zoff[b] = zo;
      zo += (int64_t)h.Rcap * h.blocks[b].acols;
    }
    h.z_elems = zo;
    h.zoff_d = up(zoff);
    h.core_tiles_d = up(ct);
    h.core_tasks_d = up(ck);
    h.leaf_tiles_d = up(lt);
    h.leaf_tasks_d = up(lk);
    h.n_core_tiles = (int)ct.size();
    h.n_leaf_tiles = (int)lt.size();
  }
  // cluster table: begin, end, parent, leaf_id; then two sons per cluster
  std::vector<int> clt(6 * ncl);
  for (int c = 0; c < ncl; ++c) {
    clt[4 * c] = h.cl[c].begin;
    clt[4 * c + 1] = h.cl[c].end;
    clt[4 * c + 2] = h.cl[c].parent;
    clt[4 * c + 3] = h.cl[c].leaf_id;
    clt[4 * ncl + 2 * c] = h.cl[c].son[0];
    clt[4 * ncl + 2 * c + 1] = h.cl[c].son[1];
  }
  std::vector<float> U32(h.Uleaf.begin(), h.Uleaf.end()), E32(h.E.begin(), h.E.end());
  h.perm_d = up(h.perm);
  h.nodes_d = up(h.nodes);
  h.U_d = up(h.Uleaf);
  h.U32_d = up(U32);
  h.uleaf_off_d = up(h.uleaf_off);
  h.E_d = up(h.E);
  h.E32_d = up(E32);
  h.Ufull_d = up(h.Ufull);
  h.ufull_off_d = up(h.ufull_off);
  h.cl_d = up(clt);
  h.blocks_d = up(h.blocks);
  h.ranks.assign(h.blocks.size(), 0);
  h.ranks_d = up(h.ranks);
  h.core_rowptr_d = up(crow);
  h.core_list_d = up(clist.empty() ? std::vector<int>{0} : clist);
  h.task_rowptr_d = up(trow);
  h.tasks_d = up(tasks.empty() ? std::vector<LeafTask>{LeafTask{0, 0}} : tasks);
  h.level_cl_d = up(lvl);
  h.built = true;
}

void set_views(Problem& p) {
  H2Operator& h = *p.h2;
  require(p.ws != nullptr, CQM_ENOMEM, "no workspace attached");
  char* base = p.ws + p.lay.partial;
  h.cstore_d = base + h.off_cstore;
  h.dvec_d = (cf64*)(base + h.off_dvec);
  h.stage_d = (cf64*)(base + h.off_stage);
  h.xhat_d = base + h.off_xhat;
  h.yhat_d = base + h.off_yhat;
  h.xp_d = base + h.off_xp;
  h.yp_d = base + h.off_yp;
  h.dhat_d = h.off_dhat ? (cf64*)(base + h.off_dhat) : nullptr;
  h.w0_d = h.off_w0 ? (void*)(base + h.off_w0) : nullptr;
  h.w0dense_d = h.off_w0dense ? (double*)(base + h.off_w0dense) : nullptr;
  h.z_d = h.off_z ? (cf64*)(base + h.off_z) : nullptr;
  h.hxh_d = h.off_hxh ? (cf64*)(base + h.off_hxh) : nullptr;
  h.rpart_d = h.off_rpart ? (cf64*)(base + h.off_rpart) : nullptr;
}
}  // namespace

size_t h2_workspace_bytes(const Problem& pc) {
  Problem& p = const_cast<Problem&>(pc);
  setup_structure(p);
  H2Operator& h = *p.h2;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += align256(b);
    return o;
  };
  h.off_cstore = take((size_t)h.cstore_elems * (h.store_fp64 ? sizeof(cf64) : sizeof(cf32)));
  h.off_dvec = take((size_t)h.dvec_elems * sizeof(cf64));
  h.off_stage = take((size_t)h.stage_elems * sizeof(cf64));
  h.off_xhat = take(h2_apply_scratch_bytes(h, p.Fsys));
  h.off_yhat = take(h2_apply_scratch_bytes(h, p.Fsys));
  h.off_xp = take(h2_perm_scratch_bytes(h, p.Fsys));
  h.off_yp = take(h2_perm_scratch_bytes(h, p.Fsys));
  // time marching: the fibres' transforms beside the fibres
  h.off_dhat = p.opt.marching ? take((size_t)h.dvec_elems * sizeof(cf64)) : 0;
  h.off_w0 = p.opt.marching
                 ? take((size_t)(h.cstore_elems / h.Rcap) * (h.store_fp64 ? sizeof(cf64) : sizeof(cf32)))
                 : 0;
  h.off_w0dense = p.opt.marching ? take(h.perm.size() * h.perm.size() * sizeof(double)) : 0;
  if (p.opt.marching) {
    const size_t coef = h.cl.size() * (size_t)h.p;
    h.off_z = take((size_t)std::max<int64_t>(h.z_elems, 1) * sizeof(cf64));
    h.off_hxh = take((size_t)p.F * coef * sizeof(cf64));
    h.off_rpart = take((size_t)kConvSplit * std::max(coef, h.perm.size()) * sizeof(cf64));
  } else {
    h.off_z = h.off_hxh = h.off_rpart = 0;
  }
  h.total = off;
  return off;
}

void h2_prepare(Problem& p, hipStream_t s) {
  setup_structure(p);
  set_views(p);
  H2Operator& h = *p.h2;
  h.w0_ready = false;  // the slices change: collapse again before use
  for (auto& bt : h.batches) {
    const int nb = bt.second - bt.first;
    if (nb <= 0) continue;
    launch_maca(p, h, bt.first, nb, s);
    launch_maca_finalize_batch(p, h, bt.first, nb, s);
  }
  CQM_HIP(hipMemcpyAsync(h.ranks.data(), h.ranks_d, sizeof(int) * h.ranks.size(), hipMemcpyDeviceToHost, s));
  CQM_HIP(hipStreamSynchronize(s));
  h.max_rank = 0;
  double sum = 0.0;
  int64_t bytes = 0, plain = 0;
  const size_t es = h.store_fp64 ? sizeof(cf64) : sizeof(cf32);
  for (size_t b = 0; b < h.blocks.size(); ++b) {
    h.max_rank = std::max(h.max_rank, h.ranks[b]);
    sum += h.ranks[b];
    const int64_t slice = (int64_t)h.blocks[b].arows * h.blocks[b].acols * es;
    bytes += (int64_t)h.ranks[b] * (slice + (int64_t)h.nsys * 16);
    plain += (int64_t)h.nsys * slice;
  }
  bytes += (int64_t)(h.Uleaf.size() + h.E.size()) * 8;
  plain += (int64_t)(h.Uleaf.size() + h.E.size()) * 8;
  h.mean_rank = h.blocks.empty() ? 0.0 : sum / h.blocks.size();
  h.bytes = bytes;
  h.plain_bytes = plain;
}

template <typename R>
void h2_apply(Problem& p, int l0, int nsys, const cplx<R>* x, int64_t xs, cplx<R>* y, int64_t ys,
              const int* /*active*/, hipStream_t s) {
  set_views(p);
  launch_h2_apply<R>(p, *p.h2, l0, nsys, x, xs, y, ys, nullptr, s);
}

// y_k = What_k x_k for k = k0 .. k0+nsys-1 (compressed time-marching
// weights: the fibres' transforms, after h2_marching_weights)
void h2_apply_weights(Problem& p, int k0, int nsys, const cf64* x, int64_t xs, cf64* y, int64_t ys,
                      hipStream_t s) {
  set_views(p);
  H2Operator& h = *p.h2;
  require(h.dhat_d != nullptr, CQM_EINVAL, "no marching weights in the workspace");
  if (k0 == 0 && nsys == 1 && h.w0_ready)
    launch_lag0_dense_product(h, x, y, s);
  else
    launch_h2_apply<double>(p, h, k0, nsys, x, xs, y, ys, h.dhat_d, s);
}

void h2_history_push(Problem& p, int m, const cf64* x, cf64* hx, hipStream_t s) {
  set_views(p);
  H2Operator& h = *p.h2;
  require(h.hxh_d != nullptr, CQM_EINVAL, "no marching history in the workspace");
  launch_h2_push_history(p, h, m, x, hx, s);
}

void h2_history_sum(Problem& p, int n, const cf64* hx, cf64* y, hipStream_t s) {
  set_views(p);
  H2Operator& h = *p.h2;
  require(h.z_d != nullptr && h.dhat_d != nullptr, CQM_EINVAL, "no marching history in the workspace");
  launch_h2_fast_history(p, h, n, hx, y, s);
}

void h2_marching_weights(Problem& p, hipStream_t s) {
  set_views(p);
  H2Operator& h = *p.h2;
  require(h.dhat_d != nullptr, CQM_EINVAL, "no marching weights in the workspace");
  launch_fibre_dft(p, h, h.dvec_d, h.dhat_d, s);
  // What_0 is applied in every conjugate-gradient iteration: collapse its
  // rank terms once and hold it densely, as the solve stage of the method
  // holds What_0 for its factorisation
  require(h.w0_d != nullptr && h.w0dense_d != nullptr, CQM_EINVAL, "no lag-0 weights in the workspace");
  launch_collapse_lag0(p, h, s);
  launch_expand_lag0(p, h, s);
  h.w0_ready = true;
}
template void h2_apply<float>(Problem&, int, int, const cf32*, int64_t, cf32*, int64_t, const int*, hipStream_t);
template void h2_apply<double>(Problem&, int, int, const cf64*, int64_t, cf64*, int64_t, const int*, hipStream_t);

void h2_stats(const Problem& p, cqm_diag* d) {
  if (!p.h2) return;
  const H2Operator& h = *p.h2;
  d->max_rank = h.max_rank;
  d->mean_rank = h.mean_rank;
  d->n_far_blocks = h.n_far;
  d->n_near_blocks = h.n_near;
  d->operator_bytes = h.bytes;
  d->h2_plain_bytes = h.plain_bytes;
}

void h2_release(Problem& p) {
  if (!p.h2) return;
  H2Operator& h = *p.h2;
  release(h.perm_d);
  release(h.nodes_d);
  release(h.U_d);
  release(h.U32_d);
  release(h.uleaf_off_d);
  release(h.E_d);
  release(h.E32_d);
  release(h.Ufull_d);
  release(h.ufull_off_d);
  release(h.cl_d);
  release(h.blocks_d);
  release(h.ranks_d);
  release(h.core_rowptr_d);
  release(h.core_list_d);
  release(h.task_rowptr_d);
  release(h.tasks_d);
  release(h.level_cl_d);
  release(h.core_tiles_d);
  release(h.core_tasks_d);
  release(h.leaf_tiles_d);
  release(h.leaf_tasks_d);
  release(h.zoff_d);
  delete p.h2;
  p.h2 = nullptr;
}

}  // namespace cqm
