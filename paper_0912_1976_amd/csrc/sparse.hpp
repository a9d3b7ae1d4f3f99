// Host-side compressed sparse row matrices used by the setup phase.
// Column indices are kept sorted in every row; products keep their full
// structural pattern (entries that cancel to zero are stored).
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <thread>
#include <vector>

namespace vemg {

// Runs fn(t, nt) on nt host threads (t = 0 on the caller): nt is the
// environment's VEMG_SETUP_THREADS (1..64) when set, else the hardware
// concurrency capped at 16, and 1 when the work is small.  Every caller splits
// its work so that each output element is computed by one thread with the
// serial code's operation order, so the results do not depend on nt.
template <class F>
void parallel_threads(int64_t work, F fn) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (work < (int64_t)1 << 16) nt = 1;
  if (const char *e = std::getenv("VEMG_SETUP_THREADS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1 && v <= 64) nt = (unsigned)v;
  }
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < nt; ++t) pool.emplace_back(fn, (int)t, (int)nt);
  fn(0, (int)nt);
  for (auto &th : pool) th.join();
}

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
