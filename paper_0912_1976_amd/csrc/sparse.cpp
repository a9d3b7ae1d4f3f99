#include "sparse.hpp"

#include <algorithm>
#include <numeric>

namespace vemg {

Csr transpose(const Csr &A) {
  Csr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.ptr.assign(T.nrows + 1, 0);
  for (int64_t k = 0; k < A.nnz(); ++k) T.ptr[A.idx[k] + 1]++;
  for (int64_t i = 0; i < T.nrows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.idx.resize(A.nnz());
  T.val.resize(A.nnz());
  std::vector<int64_t> next(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      int64_t p = next[A.idx[k]]++;
      T.idx[p] = (int32_t)i;
      T.val[p] = A.val[k];
    }
  return T;  // rows visited in ascending order, so columns are sorted
}

// columns ascending in every row (a row's columns are distinct, so the
// result does not depend on the sort); rows are shared among threads
static void sort_rows(Csr &A) {
  parallel_threads(A.nnz(), [&](int t, int nt) {
    std::vector<std::pair<int32_t, double>> tmp;
    for (int64_t i = A.nrows * t / nt, i1 = A.nrows * (t + 1) / nt; i < i1; ++i) {
      int64_t a = A.ptr[i], b = A.ptr[i + 1];
      tmp.clear();
      for (int64_t k = a; k < b; ++k) tmp.emplace_back(A.idx[k], A.val[k]);
      std::sort(tmp.begin(), tmp.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
      for (int64_t k = a; k < b; ++k) {
        A.idx[k] = tmp[k - a].first;
        A.val[k] = tmp[k - a].second;
      }
    }
  });
}

Csr permute_sym(const Csr &A, const std::vector<int64_t> &perm) {
  std::vector<int64_t> inv(perm.size());
  for (size_t i = 0; i < perm.size(); ++i) inv[perm[i]] = (int64_t)i;
  Csr B;
  B.nrows = A.nrows;
  B.ncols = A.ncols;
  B.ptr.assign(B.nrows + 1, 0);
  for (int64_t i = 0; i < B.nrows; ++i) B.ptr[i + 1] = B.ptr[i] + (A.ptr[perm[i] + 1] - A.ptr[perm[i]]);
  B.idx.resize(A.nnz());
  B.val.resize(A.nnz());
  parallel_threads(A.nnz(), [&](int t, int nt) {
    for (int64_t i = B.nrows * t / nt, i1 = B.nrows * (t + 1) / nt; i < i1; ++i) {
      int64_t o = perm[i], p = B.ptr[i];
      for (int64_t k = A.ptr[o]; k < A.ptr[o + 1]; ++k, ++p) {
        B.idx[p] = (int32_t)inv[A.idx[k]];
        B.val[p] = A.val[k];
      }
    }
  });
  sort_rows(B);
  return B;
}

Csr permute_cols(const Csr &A, const std::vector<int64_t> &colmap) {
  Csr B = A;
  for (auto &c : B.idx) c = (int32_t)colmap[c];
  sort_rows(B);
  return B;
}

Csr spgemm(const Csr &A, const Csr &B) {
  Csr C;
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  C.ptr.assign(C.nrows + 1, 0);
  // rows are shared among threads in contiguous blocks; each row is formed
  // by one thread exactly as in a serial pass
  auto block = [&](int t, int nt, int64_t &i0, int64_t &i1) {
    i0 = A.nrows * t / nt;
    i1 = A.nrows * (t + 1) / nt;
  };
  const int64_t work = A.nnz() + B.nnz();
  // pass 1: pattern size of every row
  parallel_threads(work, [&](int t, int nt) {
    int64_t i0, i1;
    block(t, nt, i0, i1);
    std::vector<int64_t> mark(B.ncols, -1);
    for (int64_t i = i0; i < i1; ++i) {
      int64_t cnt = 0;
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        int64_t r = A.idx[k];
        for (int64_t l = B.ptr[r]; l < B.ptr[r + 1]; ++l)
          if (mark[B.idx[l]] != i) {
            mark[B.idx[l]] = i;
            ++cnt;
          }
      }
      C.ptr[i + 1] = cnt;
    }
  });
  for (int64_t i = 0; i < C.nrows; ++i) C.ptr[i + 1] += C.ptr[i];
  C.idx.resize(C.ptr.back());
  C.val.resize(C.ptr.back());
  // pass 2: values, accumulated in the order of A's row and then B's rows
  parallel_threads(work, [&](int t, int nt) {
    int64_t i0, i1;
    block(t, nt, i0, i1);
    std::vector<int64_t> mark(B.ncols, -1);
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int32_t> cols;
    for (int64_t i = i0; i < i1; ++i) {
      cols.clear();
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        int64_t r = A.idx[k];
        double a = A.val[k];
        for (int64_t l = B.ptr[r]; l < B.ptr[r + 1]; ++l) {
          int32_t c = B.idx[l];
          if (mark[c] != i) {
            mark[c] = i;
            acc[c] = 0.0;
            cols.push_back(c);
          }
          acc[c] += a * B.val[l];
        }
      }
      std::sort(cols.begin(), cols.end());
      int64_t p = C.ptr[i];
      for (int32_t c : cols) {
        C.idx[p] = c;
        C.val[p] = acc[c];
        ++p;
      }
    }
  });
  return C;
}

std::vector<double> diagonal(const Csr &A) {
  std::vector<double> d(A.nrows, 0.0);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (A.idx[k] == i) d[i] = A.val[k];
  return d;
}

}  // namespace vemg
