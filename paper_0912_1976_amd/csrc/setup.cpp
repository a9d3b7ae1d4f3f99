// Host setup (see setup.hpp).  Built with -ffp-contract=off: edge values,
// row sums, the locality key and the barycentric weights are computed in a
// fixed operation order, so the integer structure derived from them (node
// order, colours, extrapolation pattern, aggregates) is reproducible.
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>
#include <sstream>
#include <thread>
#include <memory>
#include <tuple>

namespace vemg {

namespace {

constexpr int kPairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
constexpr double kTolInside = 1e-12;
constexpr double kTieRtol = 1e-10;
constexpr double kGsDrop = 1e-10;

struct V3 {
  double x, y, z;
};
inline V3 sub(const V3 &a, const V3 &b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 cross(const V3 &a, const V3 &b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double dot(const V3 &a, const V3 &b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

[[noreturn]] void fail(int code, const std::string &msg) { throw SetupError(code, msg); }

// Scaled gradients of the P1 basis on one tetrahedron: grad N_a = c_a / det.
void tet_gradients(const double *xyz, const int64_t *t, V3 c[4], double &det) {
  V3 X[4];
  for (int a = 0; a < 4; ++a) X[a] = {xyz[3 * t[a]], xyz[3 * t[a] + 1], xyz[3 * t[a] + 2]};
  V3 e1 = sub(X[1], X[0]), e2 = sub(X[2], X[0]), e3 = sub(X[3], X[0]);
  c[1] = cross(e2, e3);
  c[2] = cross(e3, e1);
  c[3] = cross(e1, e2);
  c[0] = {-((c[1].x + c[2].x) + c[3].x), -((c[1].y + c[2].y) + c[3].y), -((c[1].z + c[2].z) + c[3].z)};
  det = dot(e1, c[1]);
}

// ---------------------------------------------------------------- assembly
// Off-diagonal stiffness on the edge graph, natural numbering.  Each edge
// value is a left-to-right sum over its elements in ascending element order.
Csr assemble_offdiag(int64_t n, const double *xyz, int64_t T, const int64_t *tets) {
  // orientation check, element-parallel; the first bad element is reported
  std::vector<double> dets(T);
  parallel_threads(64 * T, [&](int t, int nt) {
    for (int64_t e = T * t / nt, e1 = T * (t + 1) / nt; e < e1; ++e) {
      V3 c[4];
      tet_gradients(xyz, tets + 4 * e, c, dets[e]);
    }
  });
  for (int64_t e = 0; e < T; ++e)
    if (!(dets[e] > 0.0)) {
      std::ostringstream os;
      os << "tetrahedron " << e << " is not positively oriented (6 vol = " << dets[e] << ")";
      fail(-2, os.str());
    }
  dets = std::vector<double>();
  // elements of every node, ascending (a stable counting sort)
  std::vector<int64_t> eptr(n + 1, 0);
  for (int64_t k = 0; k < 4 * T; ++k) ++eptr[tets[k] + 1];
  for (int64_t i = 0; i < n; ++i) eptr[i + 1] += eptr[i];
  std::vector<int64_t> elem(4 * T);
  {
    std::vector<int64_t> fill(eptr.begin(), eptr.end() - 1);
    for (int64_t k = 0; k < 4 * T; ++k) elem[fill[tets[k]]++] = k / 4;
  }
  // pattern: the neighbours of node i in its elements, by node ranges
  Csr A;
  A.nrows = A.ncols = n;
  A.ptr.assign(n + 1, 0);
  std::vector<std::vector<int32_t>> nb(n);
  parallel_threads(64 * T, [&](int t, int nt) {
    for (int64_t i = n * t / nt, i1 = n * (t + 1) / nt; i < i1; ++i) {
      auto &v = nb[i];
      for (int64_t q = eptr[i]; q < eptr[i + 1]; ++q) {
        const int64_t *te = tets + 4 * elem[q];
        for (int a = 0; a < 4; ++a)
          if (te[a] != i) v.push_back((int32_t)te[a]);
      }
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      A.ptr[i + 1] = (int64_t)v.size();
    }
  });
  for (int64_t i = 0; i < n; ++i) A.ptr[i + 1] += A.ptr[i];
  A.idx.resize(A.ptr[n]);
  parallel_threads(64 * T, [&](int t, int nt) {
    for (int64_t i = n * t / nt, i1 = n * (t + 1) / nt; i < i1; ++i) {
      std::copy(nb[i].begin(), nb[i].end(), A.idx.begin() + A.ptr[i]);
      nb[i] = std::vector<int32_t>();
    }
  });
  A.val.assign(A.idx.size(), 0.0);
  auto find = [&](int64_t i, int32_t j) {
    auto b = A.idx.begin() + A.ptr[i], e = A.idx.begin() + A.ptr[i + 1];
    return (int64_t)(std::lower_bound(b, e, j) - A.idx.begin());
  };
  // values: the thread owning row lo visits lo's elements in ascending order
  // and adds every edge (lo, hi), lo < hi, of each, so each edge value is the
  // left-to-right sum over its elements in ascending element order
  parallel_threads(64 * T, [&](int t, int nt) {
    for (int64_t lo = n * t / nt, l1 = n * (t + 1) / nt; lo < l1; ++lo)
      for (int64_t q = eptr[lo]; q < eptr[lo + 1]; ++q) {
        const int64_t *te = tets + 4 * elem[q];
        V3 c[4];
        double det;
        tet_gradients(xyz, te, c, det);
        for (auto &p : kPairs) {
          const int64_t i = te[p[0]], j = te[p[1]];
          if (std::min(i, j) != lo) continue;
          const V3 &ca = c[p[0]], &cb = c[p[1]];
          const double k = ((ca.x * cb.x + ca.y * cb.y) + ca.z * cb.z) / (6.0 * det);
          A.val[find(lo, (int32_t)std::max(i, j))] += k;
        }
      }
  });
  // mirror the upper triangle (lo < hi) to the lower one
  parallel_threads(64 * T, [&](int t, int nt) {
    for (int64_t i = n * t / nt, i1 = n * (t + 1) / nt; i < i1; ++i)
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        int64_t j = A.idx[k];
        if (j < i) A.val[k] = A.val[find(j, (int32_t)i)];
      }
  });
  return A;
}

// ---------------------------------------------------------------- colouring
std::vector<int32_t> greedy_colouring(const Csr &A, const std::vector<int64_t> &order) {
  std::vector<int32_t> col(A.nrows, -1);
  std::vector<int64_t> seen;  // seen[c] == i marks colour c as used around node i
  for (int64_t i : order) {
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      int64_t j = A.idx[k];
      if (j != i && col[j] >= 0) {
        if ((int64_t)seen.size() <= col[j]) seen.resize(col[j] + 1, -1);
        seen[col[j]] = i;
      }
    }
    int32_t c = 0;
    while (c < (int32_t)seen.size() && seen[c] == i) ++c;
    col[i] = c;
  }
  return col;
}

// Smallest-last vertex order of the off-diagonal pattern: repeatedly remove a
// vertex of smallest remaining degree (ties to the smallest index), then
// reverse.  One lazy min-heap of indices per degree: a vertex whose degree
// drops is pushed again into its new degree's heap, and entries whose degree
// has since changed, or whose vertex is gone, are skipped when they reach a
// top.  Every heap below the current minimum degree is empty, so the first
// valid top from there up is the smallest (degree, index) pair.  Row indices
// are below 2^31 (int32 columns).
std::vector<int64_t> smallest_last_order(const Csr &A) {
  const int64_t n = A.nrows;
  std::vector<int64_t> deg(n, 0);
  int64_t maxd = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) deg[i] += (A.idx[k] != i);
    maxd = std::max(maxd, deg[i]);
  }
  using Heap = std::priority_queue<uint32_t, std::vector<uint32_t>, std::greater<uint32_t>>;
  std::vector<Heap> bucket(maxd + 1);
  for (int64_t i = 0; i < n; ++i) bucket[deg[i]].push((uint32_t)i);
  std::vector<char> removed(n, 0);
  std::vector<int64_t> seq;
  seq.reserve(n);
  int64_t dmin = 0;
  for (int64_t step = 0; step < n; ++step) {
    int64_t i;
    while (true) {
      while (bucket[dmin].empty()) ++dmin;
      i = bucket[dmin].top();
      bucket[dmin].pop();
      if (!removed[i] && deg[i] == dmin) break;
    }
    removed[i] = 1;
    seq.push_back(i);
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int64_t j = A.idx[k];
      if (j != i && !removed[j]) {
        const int64_t d = --deg[j];
        bucket[d].push((uint32_t)j);
        dmin = std::min(dmin, d);
      }
    }
  }
  std::reverse(seq.begin(), seq.end());
  return seq;
}

// the colouring of every SOR sweep: greedy in smallest-last order
std::vector<int32_t> sweep_colouring(const Csr &A) { return greedy_colouring(A, smallest_last_order(A)); }

std::vector<int64_t> colour_ranges(const std::vector<int32_t> &col, int64_t a, int64_t b) {
  int32_t nc = 0;
  for (int64_t i = a; i < b; ++i) nc = std::max(nc, col[i] + 1);
  std::vector<int64_t> st(nc + 1, b);
  st[0] = a;
  for (int32_t c = 0; c < nc; ++c) {
    int64_t i = st[c];
    while (i < b && col[i] == c) ++i;
    st[c + 1] = i;
  }
  return st;
}

// ---------------------------------------------------------------- patch order
// Block multicolour order of the coarse levels.  The unknowns, in their
// spatial order (rank), are cut into consecutive patches of at most
// kPatchRows unknowns holding at most kPatchEntries off-diagonal entries
// together (at least one unknown each); the patch graph (patches coupled by
// an entry) is coloured greedily in smallest-last order, and so is every
// patch's own coupling graph, its unknowns indexed in rank order.  The
// storage order sorts by (patch colour, patch, local colour, rank).  Unknowns
// of equal (patch colour, local colour) are never coupled, so a sweep that
// takes the patch colours in turn, and inside every patch its local colours
// in turn, is the sequential SOR sweep in the stored order.
struct PatchOrder {
  std::vector<int64_t> perm;                // new -> old
  std::vector<int32_t> patch, pcol, lcol;  // per unknown, in the new order
};

PatchOrder patch_order(const Csr &A, const std::vector<int64_t> &rank) {
  const int64_t n = A.nrows;
  PatchOrder out;
  std::vector<int64_t> ro(n);  // unknowns in rank order
  for (int64_t i = 0; i < n; ++i) ro[rank[i]] = i;
  std::vector<int32_t> patch(n);
  std::vector<int64_t> pstart;  // first position (in ro) of every patch
  {
    int64_t rows = 0, ents = 0;
    for (int64_t t = 0; t < n; ++t) {
      const int64_t i = ro[t];
      int64_t len = 0;
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) len += (A.idx[k] != i);
      if (pstart.empty() || rows == kPatchRows || ents + len > kPatchEntries) {
        pstart.push_back(t);
        rows = 0;
        ents = 0;
      }
      patch[i] = (int32_t)pstart.size() - 1;
      ++rows;
      ents += len;
    }
  }
  const int64_t np = (int64_t)pstart.size();
  pstart.push_back(n);
  // patch graph
  Csr G;
  G.nrows = G.ncols = np;
  G.ptr.assign(np + 1, 0);
  std::vector<int32_t> nb;
  for (int64_t p = 0; p < np; ++p) {
    nb.clear();
    for (int64_t t = pstart[p]; t < pstart[p + 1]; ++t) {
      const int64_t i = ro[t];
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const int32_t q = patch[A.idx[k]];
        if (q != p) nb.push_back(q);
      }
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    G.idx.insert(G.idx.end(), nb.begin(), nb.end());
    G.ptr[p + 1] = (int64_t)G.idx.size();
  }
  G.val.assign(G.idx.size(), 1.0);
  std::vector<int32_t> pcol = sweep_colouring(G);
  // local colourings, unknowns of a patch indexed in rank order
  std::vector<int32_t> lcol(n);
  std::vector<int64_t> local(n, -1);
  for (int64_t p = 0; p < np; ++p) {
    const int64_t a = pstart[p], m = pstart[p + 1] - a;
    for (int64_t t = 0; t < m; ++t) local[ro[a + t]] = t;
    Csr L;
    L.nrows = L.ncols = m;
    L.ptr.assign(m + 1, 0);
    for (int64_t t = 0; t < m; ++t) {
      const int64_t i = ro[a + t];
      const size_t k0 = L.idx.size();
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const int64_t j = A.idx[k];
        if (j != i && patch[j] == p) L.idx.push_back((int32_t)local[j]);
      }
      std::sort(L.idx.begin() + k0, L.idx.end());
      L.ptr[t + 1] = (int64_t)L.idx.size();
    }
    L.val.assign(L.idx.size(), 1.0);
    std::vector<int32_t> c = sweep_colouring(L);
    for (int64_t t = 0; t < m; ++t) lcol[ro[a + t]] = c[t];
  }
  out.perm.resize(n);
  std::iota(out.perm.begin(), out.perm.end(), 0);
  std::sort(out.perm.begin(), out.perm.end(), [&](int64_t a, int64_t b) {
    return std::make_tuple(pcol[patch[a]], patch[a], lcol[a], rank[a]) <
           std::make_tuple(pcol[patch[b]], patch[b], lcol[b], rank[b]);
  });
  out.patch.resize(n);
  out.pcol.resize(n);
  out.lcol.resize(n);
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = out.perm[t];
    out.patch[t] = patch[i];
    out.pcol[t] = pcol[patch[i]];
    out.lcol[t] = lcol[i];
  }
  return out;
}

// Stores a level's patch arrays (new order), its composite sweep colour and
// spatial rank, and the ranges its sweeps launch over.
void set_patches(Level &L, const PatchOrder &po, const std::vector<int64_t> &rank_old) {
  const int64_t n = (int64_t)po.perm.size();
  L.patch = po.patch;
  L.pcolour = po.pcol;
  L.lcolour = po.lcol;
  L.colour.resize(n);
  L.rank.resize(n);
  for (int64_t t = 0; t < n; ++t) {
    L.colour[t] = po.pcol[t] * (int32_t)kPatchRows + po.lcol[t];
    L.rank[t] = rank_old[po.perm[t]];
  }
  // patches are contiguous in the new order, numbered in rank order: list
  // them in storage order, with their row ranges and local colour segments
  L.patch_list.clear();
  L.patch_row.clear();
  L.seg_ptr.clear();
  L.seg_row.clear();
  L.pc_start.clear();
  for (int64_t t = 0; t < n; ++t) {
    const bool new_patch = t == 0 || po.patch[t] != po.patch[t - 1];
    if (new_patch) {
      if (L.pc_start.empty() || po.pcol[t] != po.pcol[L.patch_row.back()])
        for (int32_t c = (int32_t)L.pc_start.size(); c <= po.pcol[t]; ++c)
          L.pc_start.push_back((int64_t)L.patch_list.size());
      L.patch_list.push_back(po.patch[t]);
      L.patch_row.push_back(t);
      L.seg_ptr.push_back((int64_t)L.seg_row.size());
    }
    if (new_patch || po.lcol[t] != po.lcol[t - 1]) L.seg_row.push_back(t);
  }
  L.pc_start.push_back((int64_t)L.patch_list.size());
  L.patch_row.push_back(n);
  L.seg_ptr.push_back((int64_t)L.seg_row.size());
  L.seg_row.push_back(n);
}

// Spatial rank of the coarse unknowns (creation order): aggregates ranked by
// their member of smallest rank in the finer level, the unknowns of one
// aggregate in creation order.
std::vector<int64_t> coarse_rank(const Level &L, const std::vector<int32_t> &agg,
                                 const std::vector<int32_t> &cnode) {
  int32_t na = 0;
  for (auto a : agg) na = std::max(na, a + 1);
  std::vector<int64_t> first(na, INT64_MAX);
  for (int64_t i = 0; i < L.n(); ++i) {
    const int32_t a = agg[L.node[i]];
    first[a] = std::min(first[a], L.rank[i]);
  }
  const int64_t nc = (int64_t)cnode.size();
  std::vector<int64_t> ord(nc);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return first[cnode[a]] < first[cnode[b]]; });
  std::vector<int64_t> rank(nc);
  for (int64_t t = 0; t < nc; ++t) rank[ord[t]] = t;
  return rank;
}

// ---------------------------------------------------------------- SA pieces
// Strong node graph: ||A_IJ||_F > theta sqrt(||A_II||_F ||A_JJ||_F), I != J.
Csr node_strength(const Csr &A, const std::vector<int32_t> &node, int64_t nnodes, double theta) {
  // rows of every node, ascending
  std::vector<int64_t> nptr(nnodes + 1, 0), nrow(A.nrows);
  for (int64_t r = 0; r < A.nrows; ++r) ++nptr[node[r] + 1];
  for (int64_t I = 0; I < nnodes; ++I) nptr[I + 1] += nptr[I];
  {
    std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1);
    for (int64_t r = 0; r < A.nrows; ++r) nrow[fill[node[r]]++] = r;
  }
  // ||A_IJ||_F of every node pair: the squares of node I's entries (its rows
  // ascending, each row's entries in order) summed per J in that order.
  // Nodes are shared among threads in contiguous ranges.
  std::vector<double> fd(nnodes, 0.0);
  std::vector<std::vector<std::pair<int32_t, double>>> rows(nnodes);
  auto range = [&](int t, int nt, int64_t &I0, int64_t &I1) {
    I0 = nnodes * t / nt;
    I1 = nnodes * (t + 1) / nt;
  };
  parallel_threads(A.nnz(), [&](int t, int nt) {
    int64_t I0, I1;
    range(t, nt, I0, I1);
    std::vector<std::pair<int32_t, double>> v;
    for (int64_t I = I0; I < I1; ++I) {
      v.clear();
      for (int64_t q = nptr[I]; q < nptr[I + 1]; ++q) {
        const int64_t r = nrow[q];
        for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) v.emplace_back(node[A.idx[k]], A.val[k] * A.val[k]);
      }
      std::stable_sort(v.begin(), v.end(), [](auto &x, auto &y) { return x.first < y.first; });
      for (size_t k = 0; k < v.size();) {
        size_t l = k;
        double s = 0.0;
        while (l < v.size() && v[l].first == v[k].first) s += v[l++].second;
        double f = std::sqrt(s);
        if (v[k].first == I) fd[I] = f;
        else rows[I].emplace_back(v[k].first, f);
        k = l;
      }
    }
  });
  // strong couplings: ||A_IJ||_F > theta sqrt(||A_II||_F ||A_JJ||_F), I != J
  Csr F;
  F.nrows = F.ncols = nnodes;
  F.ptr.assign(nnodes + 1, 0);
  std::vector<std::vector<char>> keep(nnodes);
  parallel_threads(A.nnz(), [&](int t, int nt) {
    int64_t I0, I1;
    range(t, nt, I0, I1);
    for (int64_t I = I0; I < I1; ++I) {
      keep[I].resize(rows[I].size());
      int64_t cnt = 0;
      for (size_t q = 0; q < rows[I].size(); ++q) {
        const auto &e = rows[I][q];
        keep[I][q] = e.second > theta * std::sqrt(fd[I] * fd[e.first]);
        cnt += keep[I][q];
      }
      F.ptr[I + 1] = cnt;
    }
  });
  for (int64_t I = 0; I < nnodes; ++I) F.ptr[I + 1] += F.ptr[I];
  F.idx.resize(F.ptr[nnodes]);
  F.val.resize(F.ptr[nnodes]);
  parallel_threads(A.nnz(), [&](int t, int nt) {
    int64_t I0, I1;
    range(t, nt, I0, I1);
    for (int64_t I = I0; I < I1; ++I) {
      int64_t p = F.ptr[I];
      for (size_t q = 0; q < rows[I].size(); ++q)
        if (keep[I][q]) {
          F.idx[p] = rows[I][q].first;
          F.val[p] = rows[I][q].second;
          ++p;
        }
    }
  });
  return F;
}

// Three aggregation passes over the node order (see the oracle's reading).
std::vector<int32_t> aggregate_graph(const Csr &G) {
  int64_t n = G.nrows;
  std::vector<int32_t> agg(n, -1);
  int32_t na = 0;
  for (int64_t i = 0; i < n; ++i) {  // P1
    if (agg[i] >= 0) continue;
    bool free = true;
    for (int64_t k = G.ptr[i]; k < G.ptr[i + 1]; ++k)
      if (agg[G.idx[k]] >= 0) {
        free = false;
        break;
      }
    if (!free) continue;
    agg[i] = na;
    for (int64_t k = G.ptr[i]; k < G.ptr[i + 1]; ++k) agg[G.idx[k]] = na;
    ++na;
  }
  std::vector<int32_t> p1 = agg;
  for (int64_t i = 0; i < n; ++i) {  // P2
    if (agg[i] >= 0) continue;
    double wmax = -1.0;
    for (int64_t k = G.ptr[i]; k < G.ptr[i + 1]; ++k)
      if (p1[G.idx[k]] >= 0) wmax = std::max(wmax, G.val[k]);
    if (wmax < 0.0) continue;
    int32_t best = -1;
    for (int64_t k = G.ptr[i]; k < G.ptr[i + 1]; ++k) {
      int32_t j = G.idx[k];
      if (p1[j] >= 0 && G.val[k] >= wmax * (1.0 - kTieRtol) && (best < 0 || j < best)) best = j;
    }
    agg[i] = p1[best];
  }
  for (int64_t i = 0; i < n; ++i) {  // P3
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int64_t k = G.ptr[i]; k < G.ptr[i + 1]; ++k)
      if (agg[G.idx[k]] < 0) agg[G.idx[k]] = na;
    ++na;
  }
  return agg;
}

// Tentative prolongator from the near-kernel vectors: modified Gram-Schmidt
// on each aggregate.  Fills P0 (CSR n x nc), Bc (nc x k), cnode.
void tentative(const Level &L, const std::vector<int32_t> &agg, Csr &P0, std::vector<double> &Bc,
               std::vector<int32_t> &cnode) {
  int64_t n = L.n(), k = L.k;
  int32_t na = 0;
  for (auto a : agg) na = std::max(na, a + 1);
  std::vector<std::vector<int64_t>> dofs(na);
  for (int64_t r = 0; r < n; ++r) dofs[agg[L.node[r]]].push_back(r);
  std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
  int32_t nc = 0;
  Bc.clear();
  cnode.clear();
  std::vector<std::vector<double>> Q;
  for (int32_t a = 0; a < na; ++a) {
    auto &idx = dofs[a];
    size_t m = idx.size();
    Q.clear();
    for (int64_t c = 0; c < k; ++c) {
      std::vector<double> v(m);
      for (size_t t = 0; t < m; ++t) v[t] = L.B[idx[t] * k + c];
      double n0 = 0.0;
      for (double x : v) n0 += x * x;
      n0 = std::sqrt(n0);
      for (auto &q : Q) {
        double s = 0.0;
        for (size_t t = 0; t < m; ++t) s += q[t] * v[t];
        for (size_t t = 0; t < m; ++t) v[t] = v[t] - s * q[t];
      }
      double nv = 0.0;
      for (double x : v) nv += x * x;
      nv = std::sqrt(nv);
      if (n0 > 0.0 && nv > kGsDrop * n0) {
        for (auto &x : v) x /= nv;
        Q.push_back(std::move(v));
      }
    }
    for (auto &q : Q) {
      for (size_t t = 0; t < m; ++t) rows[idx[t]].emplace_back(nc, q[t]);
      for (int64_t c = 0; c < k; ++c) {
        double s = 0.0;
        for (size_t t = 0; t < m; ++t) s += q[t] * L.B[idx[t] * k + c];
        Bc.push_back(s);
      }
      cnode.push_back(a);
      ++nc;
    }
  }
  P0.nrows = n;
  P0.ncols = nc;
  P0.ptr.assign(n + 1, 0);
  P0.idx.clear();
  P0.val.clear();
  for (int64_t r = 0; r < n; ++r) {
    for (auto &e : rows[r]) {
      P0.idx.push_back(e.first);
      P0.val.push_back(e.second);
    }
    P0.ptr[r + 1] = (int64_t)P0.idx.size();
  }
}

// S = I - omega D^{-1} A on the pattern of A plus the diagonal.
Csr jacobi_smoother(const Csr &A, double omega) {
  auto dg = diagonal(A);
  Csr S;
  S.nrows = S.ncols = A.nrows;
  S.ptr.assign(A.nrows + 1, 0);
  for (int64_t i = 0; i < A.nrows; ++i) {
    bool has_diag = false;
    double inv = 1.0 / dg[i];
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      int32_t j = A.idx[k];
      if (!has_diag && j > i) {
        S.idx.push_back((int32_t)i);
        S.val.push_back(1.0);
        has_diag = true;
      }
      double v = omega * (inv * A.val[k]);
      if (j == i) {
        S.idx.push_back(j);
        S.val.push_back(1.0 - v);
        has_diag = true;
      } else {
        S.idx.push_back(j);
        S.val.push_back(-v);
      }
    }
    if (!has_diag) {
      S.idx.push_back((int32_t)i);
      S.val.push_back(1.0);
    }
    S.ptr[i + 1] = (int64_t)S.idx.size();
  }
  return S;
}

// Dense inverse of a small SPD matrix (row-major, in place): Cholesky
// A = L L^T, then L^{-1} row by row, then A^{-1} = L^{-T} L^{-1}; every inner
// loop runs over contiguous memory.
void spd_inverse(std::vector<double> &M, int64_t n) {
  // Cholesky by rows: L_ij = (M_ij - sum_{k<j} L_ik L_jk) / L_jj for j < i,
  // then L_ii = sqrt(M_ii - sum_{k<i} L_ik^2), sums in ascending k.  Threads
  // take every nt-th row; entry (i, j) waits until row j is complete.
  std::vector<double> L(n * n, 0.0);
  std::unique_ptr<std::atomic<int>[]> ready(new std::atomic<int>[n]);
  for (int64_t i = 0; i < n; ++i) ready[i].store(0, std::memory_order_relaxed);
  std::atomic<bool> indefinite(false);
  parallel_threads(n * n * n / 6, [&](int t, int nt) {
    for (int64_t i = t; i < n; i += nt) {
      double *li = &L[i * n];
      for (int64_t j = 0; j < i; ++j) {
        while (!ready[j].load(std::memory_order_acquire)) std::this_thread::yield();
        const double *lj = &L[j * n];
        double v = M[i * n + j];
        for (int64_t k = 0; k < j; ++k) v -= li[k] * lj[k];
        li[j] = v / lj[j];
      }
      double s = M[i * n + i];
      for (int64_t k = 0; k < i; ++k) s -= li[k] * li[k];
      if (!(s > 0.0)) indefinite.store(true);
      li[i] = std::sqrt(s);
      ready[i].store(1, std::memory_order_release);
    }
  });
  if (indefinite.load()) fail(-2, "coarsest multigrid level is not positive definite");
  // W = L^{-1} (lower triangular): row i = (e_i - sum_{k<i} L_ik W_k) / L_ii.
  // Column blocks of W are independent; each thread takes every nt-th block
  // of 32 columns and updates them in the serial order (k ascending).
  std::vector<double> W(n * n, 0.0);
  constexpr int64_t kCols = 32;
  const int64_t nblk = (n + kCols - 1) / kCols;
  parallel_threads(n * n * n / 6, [&](int t, int nt) {
    for (int64_t b = t; b < nblk; b += nt) {
      const int64_t j0 = b * kCols, j1 = std::min(n, j0 + kCols);
      for (int64_t i = j0; i < n; ++i) {
        double *wi = &W[i * n];
        if (i < j1) wi[i] = 1.0;
        for (int64_t k = j0; k < i; ++k) {
          double l = L[i * n + k];
          const double *wk = &W[k * n];
          const int64_t je = std::min(j1, k + 1);
          for (int64_t j = j0; j < je; ++j) wi[j] -= l * wk[j];
        }
        double inv = 1.0 / L[i * n + i];
        const int64_t je = std::min(j1, i + 1);
        for (int64_t j = j0; j < je; ++j) wi[j] *= inv;
      }
    }
  });
  // A^{-1} = W^T W: M_ij = sum over k >= max(i, j), ascending, of W_ki W_kj.
  // Rows of M are independent; each thread takes every nt-th row.
  std::fill(M.begin(), M.end(), 0.0);
  parallel_threads(n * n * n / 6, [&](int t, int nt) {
    for (int64_t i = t; i < n; i += nt) {
      double *mi = &M[i * n];
      for (int64_t k = i; k < n; ++k) {
        const double *wk = &W[k * n];
        double a = wk[i];
        for (int64_t j = 0; j <= k; ++j) mi[j] += a * wk[j];
      }
    }
  });
}

// The sparse approximate inverse alternative to the projection (Section 5.4,
// second approach).  The exact extrapolation is E = [I; -A_bar^{-1} C^T]
// (Section 5.3); E~ keeps the projection's pattern, and column i of its
// non-top block F is refitted on its own: with J the non-top rows of the
// column's pattern, v = F[J, i] solves A_bar[J, J] v = -C^T[J, i] (entries
// outside J stay zero).  A_bar[J, J] is a principal submatrix of a symmetric
// positive definite matrix: one dense Cholesky factorisation per column.
// Columns are independent and are shared among host threads.
void sspai_refit(Csr &E, const Csr &A, int64_t m) {
  const int64_t n = E.nrows, nc = E.ncols;
  // non-top entries of every column, rows ascending, with their position in E
  std::vector<int64_t> cptr(nc + 1, 0);
  for (int64_t r = m; r < n; ++r)
    for (int64_t k = E.ptr[r]; k < E.ptr[r + 1]; ++k) ++cptr[E.idx[k] + 1];
  for (int64_t i = 0; i < nc; ++i) cptr[i + 1] += cptr[i];
  std::vector<int64_t> crow(cptr[nc]), cpos(cptr[nc]), next(cptr.begin(), cptr.end() - 1);
  for (int64_t r = m; r < n; ++r)
    for (int64_t k = E.ptr[r]; k < E.ptr[r + 1]; ++k) {
      int64_t c = E.idx[k];
      crow[next[c]] = r;
      cpos[next[c]] = k;
      ++next[c];
    }
  std::atomic<int64_t> next_col{0}, bad{-1};
  auto work = [&]() {
    std::vector<double> L, v;
    for (;;) {
      int64_t c = next_col.fetch_add(1);
      if (c >= nc) return;
      const int64_t b = cptr[c], q = cptr[c + 1] - b;
      if (q == 0) continue;
      const int64_t *J = &crow[b];
      L.assign(q * q, 0.0);
      v.assign(q, 0.0);
      for (int64_t a = 0; a < q; ++a) {
        const int64_t r = J[a];
        for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
          const int64_t j = A.idx[k];
          if (j == c) {
            v[a] = -A.val[k];
          } else if (j >= m) {
            const int64_t *p = std::lower_bound(J, J + q, j);
            if (p != J + q && *p == j) L[a * q + (p - J)] = A.val[k];
          }
        }
      }
      // lower Cholesky factor in place (row-major, lower triangle)
      bool ok = true;
      for (int64_t j = 0; j < q && ok; ++j) {
        double s = L[j * q + j];
        for (int64_t k = 0; k < j; ++k) s -= L[j * q + k] * L[j * q + k];
        if (!(s > 0.0)) {
          ok = false;
          break;
        }
        const double ljj = std::sqrt(s);
        L[j * q + j] = ljj;
        for (int64_t i = j + 1; i < q; ++i) {
          double t = L[i * q + j];
          for (int64_t k = 0; k < j; ++k) t -= L[i * q + k] * L[j * q + k];
          L[i * q + j] = t / ljj;
        }
      }
      if (!ok) {
        int64_t none = -1;
        bad.compare_exchange_strong(none, c);
        return;
      }
      for (int64_t i = 0; i < q; ++i) {  // L y = rhs
        double t = v[i];
        for (int64_t k = 0; k < i; ++k) t -= L[i * q + k] * v[k];
        v[i] = t / L[i * q + i];
      }
      for (int64_t i = q - 1; i >= 0; --i) {  // L^T x = y
        double t = v[i];
        for (int64_t k = i + 1; k < q; ++k) t -= L[k * q + i] * v[k];
        v[i] = t / L[i * q + i];
      }
      for (int64_t a = 0; a < q; ++a) E.val[cpos[b + a]] = v[a];
    }
  };
  parallel_threads((int64_t)1 << 20, [&](int, int) { work(); });
  if (bad.load() >= 0) {
    std::ostringstream os;
    os << "extrapolation refit: the system of surface column " << bad.load() << " is not positive definite";
    fail(-3, os.str());
  }
}

void build_hierarchy(std::vector<Level> &levels, const SetupOptions &opt) {
  int64_t nnodes = levels[0].n();
  while (true) {
    Level &L = levels.back();
    if (L.patch.empty()) L.colour_start = colour_ranges(L.colour, 0, L.n());
    if (L.n() <= opt.coarse_max || (int)levels.size() >= opt.max_levels) break;
    Csr G = node_strength(L.A, L.node, nnodes, opt.theta);
    std::vector<int32_t> agg = aggregate_graph(G);
    Csr P0;
    std::vector<double> Bc;
    std::vector<int32_t> cnode;
    tentative(L, agg, P0, Bc, cnode);
    int64_t nc = P0.ncols;
    if ((double)nc > 0.8 * (double)L.n()) {
      // too few couplings pass the threshold (vertical columns at small eps
      // leave none once the columns are aggregated): aggregate this level
      // again with every coupling strong before giving up, which keeps the
      // coarsest level small enough for its dense solve
      G = node_strength(L.A, L.node, nnodes, 0.0);
      agg = aggregate_graph(G);
      P0 = Csr();
      Bc.clear();
      cnode.clear();
      tentative(L, agg, P0, Bc, cnode);
      nc = P0.ncols;
      if ((double)nc > 0.8 * (double)L.n()) break;
    }
    Csr P = spgemm(jacobi_smoother(L.A, opt.prolong_omega), P0);
    Csr Pt = transpose(P);
    Csr Ac = spgemm(Pt, spgemm(L.A, P));
    const std::vector<int64_t> crank = coarse_rank(L, agg, cnode);
    const PatchOrder po = patch_order(Ac, crank);
    const std::vector<int64_t> &cperm = po.perm;
    std::vector<int64_t> cinv(nc);
    for (int64_t i = 0; i < nc; ++i) cinv[cperm[i]] = i;
    L.P = permute_cols(P, cinv);
    L.agg = agg;
    nnodes = 0;
    for (auto a : agg) nnodes = std::max<int64_t>(nnodes, a + 1);
    Level C;
    C.A = permute_sym(Ac, cperm);
    set_patches(C, po, crank);
    C.node.resize(nc);
    C.k = L.k;
    C.B.resize(nc * L.k);
    for (int64_t i = 0; i < nc; ++i) {
      C.node[i] = cnode[cperm[i]];
      for (int c = 0; c < L.k; ++c) C.B[i * L.k + c] = Bc[cperm[i] * L.k + c];
    }
    levels.push_back(std::move(C));
  }
  Level &last = levels.back();
  int64_t m = last.n();
  last.Cinv.assign(m * m, 0.0);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t k = last.A.ptr[i]; k < last.A.ptr[i + 1]; ++k) last.Cinv[i * m + last.A.idx[k]] = last.A.val[k];
  spd_inverse(last.Cinv, m);
}

// ---------------------------------------------------------------- E~
struct Locator {
  const double *xyz;
  const std::vector<std::array<int64_t, 3>> &tri;
  int64_t ng;
  double gx0, gy0, sx, sy;
  std::vector<int64_t> cstart;
  std::vector<int32_t> ctri;

  Locator(const double *xyz_, const std::vector<std::array<int64_t, 3>> &tri_, double px0, double py0,
          double px1, double py1)
      : xyz(xyz_), tri(tri_) {
    int64_t nt = (int64_t)tri.size();
    ng = std::max<int64_t>(1, (int64_t)std::sqrt((double)nt / 2.0));
    double x0 = px0, y0 = py0, x1 = px1, y1 = py1;
    for (auto &t : tri)
      for (int a = 0; a < 3; ++a) {
        x0 = std::min(x0, xyz[3 * t[a]]);
        x1 = std::max(x1, xyz[3 * t[a]]);
        y0 = std::min(y0, xyz[3 * t[a] + 1]);
        y1 = std::max(y1, xyz[3 * t[a] + 1]);
      }
    gx0 = x0;
    gy0 = y0;
    sx = std::max(x1 - x0, 1e-300);
    sy = std::max(y1 - y0, 1e-300);
    std::vector<std::vector<int32_t>> cells(ng * ng);
    for (int64_t ti = 0; ti < nt; ++ti) {
      double lx = 1e300, hx = -1e300, ly = 1e300, hy = -1e300;
      for (int a = 0; a < 3; ++a) {
        lx = std::min(lx, xyz[3 * tri[ti][a]]);
        hx = std::max(hx, xyz[3 * tri[ti][a]]);
        ly = std::min(ly, xyz[3 * tri[ti][a] + 1]);
        hy = std::max(hy, xyz[3 * tri[ti][a] + 1]);
      }
      int64_t cx0 = cell(lx - 1e-9 * sx, gx0, sx), cx1 = cell(hx + 1e-9 * sx, gx0, sx);
      int64_t cy0 = cell(ly - 1e-9 * sy, gy0, sy), cy1 = cell(hy + 1e-9 * sy, gy0, sy);
      for (int64_t cy = cy0; cy <= cy1; ++cy)
        for (int64_t cx = cx0; cx <= cx1; ++cx) cells[cy * ng + cx].push_back((int32_t)ti);
    }
    cstart.assign(ng * ng + 1, 0);
    for (int64_t c = 0; c < ng * ng; ++c) cstart[c + 1] = cstart[c] + (int64_t)cells[c].size();
    ctri.reserve(cstart.back());
    for (auto &c : cells) ctri.insert(ctri.end(), c.begin(), c.end());
  }
  int64_t cell(double v, double g0, double s) const {
    int64_t c = (int64_t)std::floor((v - g0) / s * (double)ng);
    return std::min<int64_t>(ng - 1, std::max<int64_t>(0, c));
  }
  // smallest triangle containing (x, y); lam gets the barycentric coordinates
  int64_t locate(double x, double y, double lam[3]) const {
    int64_t c = cell(y, gy0, sy) * ng + cell(x, gx0, sx);
    int64_t best = -1;
    for (int64_t k = cstart[c]; k < cstart[c + 1]; ++k) {
      int64_t t = ctri[k];
      if (best >= 0 && t >= best) continue;
      double x1 = xyz[3 * tri[t][0]], y1 = xyz[3 * tri[t][0] + 1];
      double x2 = xyz[3 * tri[t][1]], y2 = xyz[3 * tri[t][1] + 1];
      double x3 = xyz[3 * tri[t][2]], y3 = xyz[3 * tri[t][2] + 1];
      double det = (y2 - y3) * (x1 - x3) + (x3 - x2) * (y1 - y3);
      double l1 = ((y2 - y3) * (x - x3) + (x3 - x2) * (y - y3)) / det;
      double l2 = ((y3 - y1) * (x - x3) + (x1 - x3) * (y - y3)) / det;
      double l3 = (1.0 - l1) - l2;
      if (l1 >= -kTolInside && l2 >= -kTolInside && l3 >= -kTolInside) {
        best = t;
        lam[0] = l1;
        lam[1] = l2;
        lam[2] = l3;
      }
    }
    return best;
  }
};

}  // namespace

// ---------------------------------------------------------------- driver
// Top-surface triangles: tetrahedron faces with three top nodes, each as its
// sorted vertex triple, in ascending lexicographic order without repeats.
std::vector<std::array<int64_t, 3>> top_triangles(int64_t n_tets, const int64_t *tets, const std::vector<uint8_t> &top) {
  std::vector<std::array<int64_t, 3>> tri;
  static const int faces[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
  for (int64_t e = 0; e < n_tets; ++e)
    for (auto &f : faces) {
      std::array<int64_t, 3> t = {tets[4 * e + f[0]], tets[4 * e + f[1]], tets[4 * e + f[2]]};
      if (top[t[0]] && top[t[1]] && top[t[2]]) {
        std::sort(t.begin(), t.end());
        tri.push_back(t);
      }
    }
  std::sort(tri.begin(), tri.end());
  tri.erase(std::unique(tri.begin(), tri.end()), tri.end());
  return tri;
}

// Robin term of the free-surface condition: alpha times the P1 mass matrix
// of the top triangles projected onto (x, y).  Its off-diagonal values
// (left-to-right sums of area/12 over the triangles holding an edge, in
// ascending triangle order) are scaled by alpha and added to the entries of
// A (every top edge is a mesh edge); L_i (the sum of area/3 over the
// triangles holding node i) times alpha is the deficit the term adds.
void add_robin(Csr &A, const double *xyz, const std::vector<std::array<int64_t, 3>> &tri, double alpha,
               std::vector<double> &dR) {
  const int64_t n = A.nrows;
  std::vector<double> m(A.idx.size(), 0.0), L(n, 0.0);
  auto find = [&](int64_t i, int64_t j) {
    auto b = A.idx.begin() + A.ptr[i], e = A.idx.begin() + A.ptr[i + 1];
    auto it = std::lower_bound(b, e, (int32_t)j);
    if (it == e || *it != (int32_t)j) fail(-2, "a top-surface edge is not an edge of the mesh");
    return (int64_t)(it - A.idx.begin());
  };
  static const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (auto &t : tri) {
    const double x1 = xyz[3 * t[0]], y1 = xyz[3 * t[0] + 1];
    const double x2 = xyz[3 * t[1]], y2 = xyz[3 * t[1] + 1];
    const double x3 = xyz[3 * t[2]], y3 = xyz[3 * t[2] + 1];
    const double area = 0.5 * std::fabs((x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1));
    for (auto &p : pairs) {
      const int64_t i = std::min(t[p[0]], t[p[1]]), j = std::max(t[p[0]], t[p[1]]);
      m[find(i, j)] += area / 12.0;
    }
    for (int a = 0; a < 3; ++a) L[t[a]] += area / 3.0;
  }
  // mirror the upper triangle (i < j) to the lower one, then add alpha m
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (A.idx[k] < i) m[k] = m[find(A.idx[k], i)];
  for (size_t k = 0; k < m.size(); ++k) A.val[k] = A.val[k] + alpha * m[k];
  dR.assign(n, 0.0);
  for (int64_t i = 0; i < n; ++i) dR[i] = alpha * L[i];
}

void build_problem(Problem &P, const SetupOptions &opt, int64_t n_nodes, const double *xyz,
                   int64_t n_tets, const int64_t *tets, const uint8_t *top) {
  if (n_nodes < 4 || n_tets < 1 || !xyz || !tets || !top) fail(-1, "empty mesh or null pointer");
  for (int64_t k = 0; k < 4 * n_tets; ++k)
    if (tets[k] < 0 || tets[k] >= n_nodes) {
      std::ostringstream os;
      os << "tetrahedron " << k / 4 << " refers to node " << tets[k] << " outside [0, " << n_nodes << ")";
      fail(-2, os.str());
    }
  P.opt = opt;
  P.n_nodes = n_nodes;
  P.xyz.assign(xyz, xyz + 3 * n_nodes);
  P.tets.assign(tets, tets + 4 * n_tets);
  P.top.resize(n_nodes);
  int64_t m_top = 0;
  for (int64_t i = 0; i < n_nodes; ++i) {
    P.top[i] = top[i] ? 1 : 0;
    m_top += P.top[i];
  }
  if (m_top < 3) fail(-2, "the top surface needs at least 3 nodes");

  // Dirichlet set (empty for the Robin top)
  std::vector<uint8_t> fixed(n_nodes, 0);
  if (opt.robin) {
    if (!(opt.robin_alpha > 0.0)) fail(-1, "the Robin coefficient must be positive");
  } else if (opt.top_dirichlet) {
    for (int64_t i = 0; i < n_nodes; ++i) fixed[i] = P.top[i];
  } else {
    int64_t pin = opt.pin_node;
    if (pin < 0) {
      double best = 0.0;
      for (int64_t i = 0; i < n_nodes; ++i)
        if (P.top[i]) {
          double d2 = (xyz[3 * i] * xyz[3 * i] + xyz[3 * i + 1] * xyz[3 * i + 1]) + xyz[3 * i + 2] * xyz[3 * i + 2];
          if (pin < 0 || d2 < best) {
            best = d2;
            pin = i;
          }
        }
    } else if (pin >= n_nodes || !P.top[pin]) {
      fail(-1, "pin_node must be a top-surface node");
    }
    P.pin = pin;
    fixed[pin] = 1;
  }

  // assembly (natural numbering)
  Csr Afull = assemble_offdiag(n_nodes, xyz, n_tets, tets);
  std::vector<double> dR;
  if (opt.robin) add_robin(Afull, xyz, top_triangles(n_tets, tets, P.top), opt.robin_alpha, dR);

  // free nodes U (ascending natural index), A_UU and the deficit
  std::vector<int64_t> U;
  std::vector<int64_t> posU(n_nodes, -1);
  for (int64_t i = 0; i < n_nodes; ++i)
    if (!fixed[i]) {
      posU[i] = (int64_t)U.size();
      U.push_back(i);
    }
  int64_t n = (int64_t)U.size();
  Csr Auu;
  Auu.nrows = Auu.ncols = n;
  Auu.ptr.assign(n + 1, 0);
  std::vector<double> dnat(n, 0.0);
  for (int64_t u = 0; u < n; ++u) {
    int64_t i = U[u];
    double s = 0.0;
    for (int64_t k = Afull.ptr[i]; k < Afull.ptr[i + 1]; ++k) {
      int64_t j = Afull.idx[k];
      if (fixed[j]) {
        s += Afull.val[k];
      } else {
        Auu.idx.push_back((int32_t)posU[j]);
        Auu.val.push_back(Afull.val[k]);
      }
    }
    dnat[u] = -s + 0.0;
    if (opt.robin) dnat[u] = dnat[u] + dR[i];
    Auu.ptr[u + 1] = (int64_t)Auu.idx.size();
  }
  Afull = Csr();

  // locality order (top block first)
  double xmin = xyz[0], xmax = xyz[0], ymin = xyz[1], ymax = xyz[1];
  for (int64_t i = 0; i < n_nodes; ++i) {
    xmin = std::min(xmin, xyz[3 * i]);
    xmax = std::max(xmax, xyz[3 * i]);
    ymin = std::min(ymin, xyz[3 * i + 1]);
    ymax = std::max(ymax, xyz[3 * i + 1]);
  }
  int64_t T = std::max<int64_t>(1, (int64_t)std::nearbyint(std::sqrt((double)m_top / 64.0)));
  int64_t F = 8 * T;
  struct Key {
    int64_t block, tile, fine;
    double negz;
    int64_t node;
  };
  std::vector<Key> keys(n);
  for (int64_t u = 0; u < n; ++u) {
    int64_t i = U[u];
    int64_t fx = std::min<int64_t>(F - 1, (int64_t)std::floor((xyz[3 * i] - xmin) / (xmax - xmin) * (double)F));
    int64_t fy = std::min<int64_t>(F - 1, (int64_t)std::floor((xyz[3 * i + 1] - ymin) / (ymax - ymin) * (double)F));
    keys[u] = {P.top[i] ? 0 : 1, (fy / 8) * T + fx / 8, (fy % 8) * 8 + fx % 8, -xyz[3 * i + 2], i};
  }
  std::vector<int64_t> loc(n);
  std::iota(loc.begin(), loc.end(), 0);
  std::sort(loc.begin(), loc.end(), [&](int64_t a, int64_t b) {
    const Key &p = keys[a], &q = keys[b];
    return std::tie(p.block, p.tile, p.fine, p.negz, p.node) < std::tie(q.block, q.tile, q.fine, q.negz, q.node);
  });
  std::vector<int32_t> colu = sweep_colouring(Auu);
  std::vector<int64_t> order = loc;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return std::make_pair(keys[a].block, colu[a]) < std::make_pair(keys[b].block, colu[b]);
  });
  P.n = n;
  P.perm.resize(n);
  P.pos.assign(n_nodes, -1);
  for (int64_t s = 0; s < n; ++s) {
    P.perm[s] = U[order[s]];
    P.pos[P.perm[s]] = s;
  }
  {
    std::vector<int64_t> rank_u(n);
    for (int64_t k = 0; k < n; ++k) rank_u[loc[k]] = k;
    P.loc_rank.resize(n);
    for (int64_t s = 0; s < n; ++s) P.loc_rank[s] = rank_u[order[s]];
  }
  P.n_top = 0;
  for (int64_t s = 0; s < n; ++s) P.n_top += P.top[P.perm[s]];
  P.Aoff = permute_sym(Auu, order);
  Auu = Csr();
  P.d.resize(n);
  P.colour.resize(n);
  for (int64_t s = 0; s < n; ++s) {
    P.d[s] = dnat[order[s]] + 0.0;
    P.colour[s] = colu[order[s]];
  }
  P.diag.resize(n);
  for (int64_t s = 0; s < n; ++s) {
    double rs = 0.0;
    for (int64_t k = P.Aoff.ptr[s]; k < P.Aoff.ptr[s + 1]; ++k) rs += P.Aoff.val[k];
    P.diag[s] = P.d[s] - rs;
  }
  P.top_colour_start = colour_ranges(P.colour, 0, P.n_top);
  P.bar_colour_start = colour_ranges(P.colour, P.n_top, n);

  // standard form A_UU (diagonal inserted in sorted position)
  Csr A;
  A.nrows = A.ncols = n;
  A.ptr.assign(n + 1, 0);
  A.idx.reserve(P.Aoff.nnz() + n);
  A.val.reserve(P.Aoff.nnz() + n);
  for (int64_t s = 0; s < n; ++s) {
    bool put = false;
    for (int64_t k = P.Aoff.ptr[s]; k < P.Aoff.ptr[s + 1]; ++k) {
      if (!put && P.Aoff.idx[k] > s) {
        A.idx.push_back((int32_t)s);
        A.val.push_back(P.diag[s]);
        put = true;
      }
      A.idx.push_back(P.Aoff.idx[k]);
      A.val.push_back(P.Aoff.val[k]);
    }
    if (!put) {
      A.idx.push_back((int32_t)s);
      A.val.push_back(P.diag[s]);
    }
    A.ptr[s + 1] = (int64_t)A.idx.size();
  }

  // vertical extrapolation E~ and the surface hierarchy
  int64_t m = P.n_top;
  if (m > 0) {
    std::vector<std::array<int64_t, 3>> tri = top_triangles(n_tets, tets, P.top);
    if (tri.empty()) fail(-2, "no top-surface triangles (faces with three top nodes)");
    Locator loc2(xyz, tri, xmin, ymin, xmax, ymax);
    // at most three entries a row, located row-parallel; the first node in
    // storage order that projects onto no triangle is reported
    std::vector<int32_t> eidx(3 * n);
    std::vector<double> eval(3 * n);
    std::vector<int8_t> ecnt(n, 0);
    parallel_threads(64 * n, [&](int t, int nt) {
      for (int64_t s = n * t / nt, s1 = n * (t + 1) / nt; s < s1; ++s) {
        int64_t i = P.perm[s];
        if (P.top[i]) {
          eidx[3 * s] = (int32_t)s;
          eval[3 * s] = 1.0;
          ecnt[s] = 1;
          continue;
        }
        double lam[3];
        int64_t tr = loc2.locate(xyz[3 * i], xyz[3 * i + 1], lam);
        if (tr < 0) {
          ecnt[s] = -1;
          continue;
        }
        for (double &l : lam)
          if (std::fabs(l) <= kTolInside) l = 0.0;
        double sum = (lam[0] + lam[1]) + lam[2];
        std::pair<int32_t, double> ent[3];
        int ne = 0;
        for (int a = 0; a < 3; ++a) {
          double w = lam[a] / sum;
          int64_t v = tri[tr][a];
          if (w != 0.0 && !fixed[v]) ent[ne++] = {(int32_t)P.pos[v], w};
        }
        std::sort(ent, ent + ne);
        for (int a = 0; a < ne; ++a) {
          eidx[3 * s + a] = ent[a].first;
          eval[3 * s + a] = ent[a].second;
        }
        ecnt[s] = (int8_t)ne;
      }
    });
    Csr E0;
    E0.nrows = n;
    E0.ncols = m;
    E0.ptr.assign(n + 1, 0);
    for (int64_t s = 0; s < n; ++s) {
      if (ecnt[s] < 0) {
        std::ostringstream os;
        os << "node " << P.perm[s] << " does not project onto the top surface";
        fail(-3, os.str());
      }
      E0.ptr[s + 1] = E0.ptr[s] + ecnt[s];
    }
    E0.idx.resize(E0.ptr[n]);
    E0.val.resize(E0.ptr[n]);
    for (int64_t s = 0; s < n; ++s)
      for (int a = 0; a < ecnt[s]; ++a) {
        E0.idx[E0.ptr[s] + a] = eidx[3 * s + a];
        E0.val[E0.ptr[s] + a] = eval[3 * s + a];
      }
    if (opt.extrapolation == 1) sspai_refit(E0, A, m);
    Csr E0t = transpose(E0);
    Csr S0 = spgemm(E0t, spgemm(A, E0));
    const std::vector<int64_t> srank(P.loc_rank.begin(), P.loc_rank.begin() + m);  // the top block ranks first
    const PatchOrder spo = patch_order(S0, srank);
    P.S_perm = spo.perm;
    std::vector<int64_t> sinv(m);
    for (int64_t i = 0; i < m; ++i) sinv[P.S_perm[i]] = i;
    P.E = permute_cols(E0, sinv);
    P.Et = transpose(P.E);
    Level L0;
    L0.A = permute_sym(S0, P.S_perm);
    set_patches(L0, spo, srank);
    L0.node.resize(m);
    L0.k = 3;
    L0.B.resize(3 * m);
    for (int64_t i = 0; i < m; ++i) {
      L0.node[i] = (int32_t)i;
      int64_t nd = P.perm[P.S_perm[i]];
      L0.B[3 * i] = 1.0;
      L0.B[3 * i + 1] = xyz[3 * nd];
      L0.B[3 * i + 2] = xyz[3 * nd + 1];
    }
    P.S.clear();
    P.S.push_back(std::move(L0));
    build_hierarchy(P.S, opt);
  }

  // interior hierarchy on A_bar (non-top block)
  Level B0;
  int64_t nb = n - m;
  if (nb <= 0) fail(-2, "no interior nodes below the top surface");
  B0.A.nrows = B0.A.ncols = nb;
  B0.A.ptr.assign(nb + 1, 0);
  for (int64_t s = m; s < n; ++s) {
    for (int64_t k = A.ptr[s]; k < A.ptr[s + 1]; ++k)
      if (A.idx[k] >= m) {
        B0.A.idx.push_back(A.idx[k] - (int32_t)m);
        B0.A.val.push_back(A.val[k]);
      }
    B0.A.ptr[s - m + 1] = (int64_t)B0.A.idx.size();
  }
  B0.colour.assign(P.colour.begin() + m, P.colour.end());
  B0.rank.resize(nb);
  for (int64_t i = 0; i < nb; ++i) B0.rank[i] = P.loc_rank[m + i] - m;
  B0.node.resize(nb);
  std::iota(B0.node.begin(), B0.node.end(), 0);
  B0.k = 1;
  B0.B.assign(nb, 1.0);
  P.Abar.clear();
  P.Abar.push_back(std::move(B0));
  build_hierarchy(P.Abar, opt);

  // the paper's baseline: smoothed aggregation on the whole A_UU, in the
  // storage order (colour c of the fine level = its top and non-top ranges)
  P.SA.clear();
  if (opt.build_sa) {
    Level F;
    F.A = A;
    F.colour = P.colour;
    F.rank = P.loc_rank;
    F.node.resize(n);
    std::iota(F.node.begin(), F.node.end(), 0);
    F.k = 1;
    F.B.assign(n, 1.0);
    P.SA.push_back(std::move(F));
    build_hierarchy(P.SA, opt);
  }
}

void mass_rhs(const Problem &P, const double *f, double *b) {
  int64_t N = P.n_nodes, T = (int64_t)P.tets.size() / 4;
  std::vector<double> bf(N, 0.0), w(N, 0.0);
  for (int64_t e = 0; e < T; ++e) {
    V3 c[4];
    double det;
    tet_gradients(P.xyz.data(), P.tets.data() + 4 * e, c, det);
    double vol = det / 6.0;
    const int64_t *t = P.tets.data() + 4 * e;
    for (int a = 0; a < 4; ++a) {
      double s = 0.0;
      for (int bb = 0; bb < 4; ++bb) s += (a == bb ? 2.0 : 1.0) * f[t[bb]];
      bf[t[a]] += vol / 20.0 * s;
      w[t[a]] += vol / 20.0 * 5.0;
    }
  }
  if (!P.opt.top_dirichlet && !P.opt.robin) {  // the pure Neumann problem needs int f = 0
    double sb = 0.0, sw = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      sb += bf[i];
      sw += w[i];
    }
    double c = sb / sw;
    for (int64_t i = 0; i < N; ++i) bf[i] -= c * w[i];
  }
  for (int64_t i = 0; i < N; ++i) b[i] = P.pos[i] >= 0 ? bf[i] : 0.0;
}

}  // namespace vemg
