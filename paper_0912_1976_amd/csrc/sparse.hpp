// Host-side compressed sparse row matrices used by the setup phase.
// Column indices are kept sorted in every row; products keep their full
// structural pattern (entries that cancel to zero are stored).
#pragma once

#include <cstdint>
#include <vector>

namespace vemg {

struct Csr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> ptr;   // nrows + 1
  std::vector<int32_t> idx;   // column of each entry, ascending within a row
  std::vector<double> val;
  int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

Csr transpose(const Csr &A);
// B = A[perm][:, perm] with perm mapping new index -> old index
Csr permute_sym(const Csr &A, const std::vector<int64_t> &perm);
// columns of A renumbered: new column = colmap[old column]; rows unchanged
Csr permute_cols(const Csr &A, const std::vector<int64_t> &colmap);
// C = A * B on the structural pattern of pattern(A) * pattern(B)
Csr spgemm(const Csr &A, const Csr &B);
// diagonal entry of every row (0 if absent)
std::vector<double> diagonal(const Csr &A);

}  // namespace vemg
