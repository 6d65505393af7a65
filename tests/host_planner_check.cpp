// Host planner under the address and undefined-behaviour sanitizers: builds
// the near-field adjacency (planner.cpp) and the cluster and block trees of
// the compressed operator (h2_tree.cpp) for a mesh read from a file, checks
// their invariants and prints a summary.  Built with a plain C++ compiler by
// tests/test_host_sanitizers.py; no GPU call is made.
//
// Mesh file: int64 nv, int64 M, nv*3 doubles, M*3 int32.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "../paper_2006_05186_amd/csrc/h2_internal.h"

namespace cqm {
void build_near(Problem& p);
void h2_build_structure(Problem& p, H2Operator& h);
}  // namespace cqm

using namespace cqm;

static int fails = 0;
#define CHECK(c, ...)                                  \
  do {                                                 \
    if (!(c)) {                                        \
      std::fprintf(stderr, "check failed: " __VA_ARGS__); \
      std::fprintf(stderr, "\n");                      \
      ++fails;                                         \
    }                                                  \
  } while (0)

static int shared(const int32_t* a, const int32_t* b) {
  int n = 0;
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3; ++y) n += a[x] == b[y];
  return n;
}

int main(int argc, char** argv) {
  if (argc < 6) {
    std::fprintf(stderr, "usage: %s mesh n_min eta cheb_m nsys\n", argv[0]);
    return 2;
  }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t nv = 0, M = 0;
  if (std::fread(&nv, 8, 1, f) != 1 || std::fread(&M, 8, 1, f) != 1) return 2;
  Problem p;
  p.nv = nv;
  p.M = M;
  p.verts.resize(3 * nv);
  p.tris.resize(3 * M);
  if (std::fread(p.verts.data(), 8, 3 * nv, f) != (size_t)(3 * nv)) return 2;
  if (std::fread(p.tris.data(), 4, 3 * M, f) != (size_t)(3 * M)) return 2;
  std::fclose(f);
  p.opt.n_min = std::atoi(argv[2]);
  p.opt.eta = std::atof(argv[3]);
  p.opt.cheb_m = std::atoi(argv[4]);
  p.Fsys = std::atoi(argv[5]);

  // near field: every pair shares a vertex, rows hold their own triangle,
  // the pattern is symmetric and each kind carries the vertex order its
  // rule expects
  build_near(p);
  CHECK((int64_t)p.rowptr.size() == M + 1 && p.rowptr[0] == 0, "row pointer size");
  const int64_t nnz = (int64_t)p.col.size();
  CHECK(p.rowptr[M] == nnz && (int64_t)p.kind.size() == nnz && (int64_t)p.nvtx.size() == 6 * nnz,
        "CSR sizes");
  std::set<std::pair<int, int>> pairs;
  for (int64_t i = 0; i < M; ++i) {
    bool self = false;
    CHECK(p.rowptr[i] <= p.rowptr[i + 1], "row pointers decrease at %lld", (long long)i);
    for (int k = p.rowptr[i]; k < p.rowptr[i + 1]; ++k) {
      const int j = p.col[k];
      CHECK(j >= 0 && j < M, "column out of range");
      if (j < 0 || j >= M) continue;
      const int ns = shared(&p.tris[3 * i], &p.tris[3 * (int64_t)j]);
      self |= j == i;
      CHECK(ns >= 1, "pair (%lld, %d) shares no vertex", (long long)i, j);
      CHECK(p.kind[k] == (j == i ? 0 : ns == 2 ? 1 : 2), "kind of pair (%lld, %d)", (long long)i, j);
      for (int v = 0; v < 6; ++v) CHECK(p.nvtx[6 * k + v] >= 0 && p.nvtx[6 * k + v] < nv, "vertex id");
      if (p.kind[k] == 1) CHECK(p.nvtx[6 * k] < p.nvtx[6 * k + 1], "shared edge orientation");
      pairs.insert({(int)i, j});
    }
    CHECK(self, "row %lld lacks its own triangle", (long long)i);
  }
  for (const auto& pr : pairs) CHECK(pairs.count({pr.second, pr.first}), "pattern not symmetric");

  // cluster and block trees: the permutation is one, leaves partition the
  // triangles, and the blocks cover every (row, column) pair exactly once
  H2Operator h;
  h2_build_structure(p, h);
  std::vector<int> seen(M, 0);
  CHECK((int64_t)h.perm.size() == M, "permutation size");
  for (int v : h.perm) {
    CHECK(v >= 0 && v < M, "permutation entry");
    if (v >= 0 && v < M) ++seen[v];
  }
  for (int64_t i = 0; i < M; ++i) CHECK(seen[i] == 1, "triangle %lld permuted %d times", (long long)i, seen[i]);
  int64_t leaf_cover = 0;
  for (int c : h.leaves) leaf_cover += h.cl[c].size();
  CHECK(leaf_cover == M, "leaves cover %lld of %lld", (long long)leaf_cover, (long long)M);
  std::vector<unsigned char> cover((size_t)M * M, 0);
  int far = 0, near = 0;
  for (const BlockDesc& b : h.blocks) {
    const Cluster &R = h.cl[b.r], &Cc = h.cl[b.c];
    (b.kind == kNear ? near : far)++;
    for (int a = R.begin; a < R.end; ++a)
      for (int c = Cc.begin; c < Cc.end; ++c) {
        unsigned char& e = cover[(size_t)a * M + c];
        if (e < 255) ++e;
      }
  }
  int64_t bad = 0;
  for (unsigned char e : cover) bad += e != 1;
  CHECK(bad == 0, "%lld (row, column) pairs not covered exactly once", (long long)bad);
  std::printf("planner ok: M=%lld nnz=%lld clusters=%zu leaves=%zu far=%d near=%d fails=%d\n",
              (long long)M, (long long)nnz, h.cl.size(), h.leaves.size(), far, near, fails);
  return fails ? 1 : 0;
}
