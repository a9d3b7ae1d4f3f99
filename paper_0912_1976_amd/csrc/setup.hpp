// Host setup of the vertical-extrapolation multigrid: P1 assembly, node
// ordering and colouring, the vertical extrapolation operator E~ and the two
// smoothed aggregation hierarchies.  Everything here runs once per mesh on
// the host; the GPU only ever sees the packed results.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "sparse.hpp"

namespace vemg {

struct SetupError : std::runtime_error {
  int code;
  SetupError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// Patches of the block multicolour order of the coarse levels: at most
// kPatchRows unknowns and kPatchEntries off-diagonal entries each (the sweep
// kernel takes one patch per block, an unknown per group of lanes).
constexpr int64_t kPatchRows = 128;
constexpr int64_t kPatchEntries = 4096;

struct Level {
  Csr A;                              // standard form, storage order
  std::vector<int32_t> colour;        // sweep colour per row (composite on patch-ordered levels)
  std::vector<int64_t> colour_start;  // fine levels: ncolours + 1 (rows sorted by colour)
  std::vector<int64_t> rank;          // position of each row in the level's spatial order
  // patch-ordered levels (every coarse level and the surface level):
  std::vector<int32_t> patch, pcolour, lcolour;  // per row
  std::vector<int64_t> pc_start;    // patch colour c: entries [pc_start[c], pc_start[c+1]) of patch_list
  std::vector<int32_t> patch_list;  // patches in storage order
  std::vector<int64_t> patch_row;   // row range of the i-th stored patch: [patch_row[i], patch_row[i+1])
  std::vector<int64_t> seg_ptr;     // its local colour segments: seg_row[seg_ptr[i] .. seg_ptr[i+1]]
  std::vector<int64_t> seg_row;     // segment starts (+ n at the end)
  std::vector<int32_t> node;          // aggregation node of each row
  std::vector<double> B;              // near-kernel vectors, row-major [n][k]
  int k = 1;
  Csr P;                              // prolongator from the next level (empty on the coarsest)
  std::vector<int32_t> agg;           // aggregate of each node
  std::vector<double> Cinv;           // coarsest level: explicit inverse, row-major
  int64_t n() const { return A.nrows; }
};

struct SetupOptions {
  int top_dirichlet = 0;     // 0: point condition at pin_node, 1: Dirichlet on the whole top
  int robin = 0;             // 1: Robin top d phi/dn + robin_alpha phi = 0, nothing fixed
  double robin_alpha = 0.0;
  int build_sa = 0;          // 1: also the smoothed aggregation hierarchy of the whole A_UU
  int extrapolation = 0;     // 0: vertical projection, 1: F refitted on its pattern (SSPAI)
  int64_t pin_node = -1;     // -1: top node closest to the origin corner
  double theta = 0.01;
  double prolong_omega = 2.0 / 3.0;
  int max_levels = 10;
  int64_t coarse_max = 2048;
};

struct Problem {
  SetupOptions opt;
  int64_t n_nodes = 0, n = 0, n_top = 0, pin = -1;
  std::vector<double> xyz;            // mesh copy (natural order)
  std::vector<int64_t> tets;
  std::vector<uint8_t> top;
  std::vector<int64_t> perm;          // storage position -> natural node
  std::vector<int64_t> pos;           // natural node -> storage position (-1: fixed)
  std::vector<int64_t> loc_rank;      // storage position -> rank in the spatial (colour-blind) order
  Csr Aoff;                           // off-diagonals of A_UU, storage order
  std::vector<double> d;              // deficit d_i = -sum_{j fixed} a_ij
  std::vector<double> diag;           // a_ii = d_i - sum_j a_ij
  std::vector<int32_t> colour;        // fine colouring (sorted within each block)
  std::vector<int64_t> top_colour_start, bar_colour_start;  // ranges in storage order
  Csr E, Et;                          // E~ (n x m') and its transpose
  std::vector<int64_t> S_perm;        // S storage position -> top-block position
  std::vector<Level> S, Abar;         // hierarchies (S empty when m' = 0)
  std::vector<Level> SA;              // SA on the whole A_UU (baseline; only with opt.build_sa)
};

// Builds the whole problem.  Throws SetupError with a status code on
// invalid meshes (-2), projection failure (-3) or invalid arguments (-1).
void build_problem(Problem &P, const SetupOptions &opt, int64_t n_nodes, const double *xyz,
                   int64_t n_tets, const int64_t *tets, const uint8_t *top);

// b = M f (consistent P1 mass matrix) in natural order; in the pinned
// (Neumann) case b is made orthogonal to constants first.  Fixed nodes get 0.
void mass_rhs(const Problem &P, const double *f, double *b);

}  // namespace vemg
