// Host-side compressed sparse row matrices used by the setup phase.
// Column indices are kept sorted in every row; products keep their full
// structural pattern (entries that cancel to zero are stored).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <exception>
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
  // The threads start together once all exist (some callers' threads wait
  // on each other's rows); if one cannot be created, those created return at
  // once and the caller does all the work alone.  An exception in any thread
  // (an allocation failure, say) is rethrown on the caller's thread once
  // every thread has finished.
  std::vector<std::exception_ptr> err(nt);
  std::atomic<int> gate(0);  // 0: wait, 1: run, 2: abandon
  auto run = [&](int t) {
    while (gate.load(std::memory_order_acquire) == 0) std::this_thread::yield();
    if (gate.load(std::memory_order_acquire) == 2) return;
    try {
      fn(t, (int)nt);
    } catch (...) {
      err[t] = std::current_exception();
    }
  };
  std::vector<std::thread> pool;
  try {
    for (unsigned t = 1; t < nt; ++t) pool.emplace_back(run, (int)t);
  } catch (...) {
    gate.store(2, std::memory_order_release);
    for (auto &th : pool) th.join();
    fn(0, 1);
    return;
  }
  gate.store(1, std::memory_order_release);
  run(0);
  for (auto &th : pool) th.join();
  for (auto &e : err)
    if (e) std::rethrow_exception(e);
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
