// Upward solve sweep on the FP64 matrix cores (sweep.hip): one launch per
// level, one workgroup per (cell, 64 right-hand-side columns).
#pragma once

#include <algorithm>

#include "common.hpp"

namespace fds {

struct SweepCell {        // one cell of a compressed level
  int64_t a_off;          // LU(A_i), column-major, ld b
  int64_t dinv_off;       // inverted 16 x 16 diagonal blocks: per block L^{-1} then U^{-1} (256 each)
  int64_t v_off;          // W_i = A~_i V_i, r x b, ld r
  int64_t at_off;         // A~_i, r x r, ld r
  int64_t x_off;          // X_i = A_i^{-1} U_i, b x r, ld b
  int64_t f_off;          // first row in the level vector
  int64_t t_off;          // first row in the skeleton vector (and in up_dst)
  int64_t perm_off;       // composed row permutation of the LU (b ints)
  int64_t piv_off;        // the LU's row interchanges (b ints)
  int b, r;
};

struct SweepLaunch {
  const SweepCell* cells = nullptr;
  int n_cells = 0, n_slab = 0, ncol = 0;
  int nb_class = 0, nr_class = 0;   // tile classes (8, 12, 16 blocks of 16) of the level's largest b and r
  const c64* A = nullptr;           // level's LU blocks
  const c64* Dinv = nullptr;
  const int* perm = nullptr;
  const c64* W = nullptr;           // A~_i V_i of the level's cells
  const c64* At = nullptr;          // A~_i
  const c64* X = nullptr;           // X_i
  const int64_t* up_dst = nullptr;  // per skeleton row (indexed by t_off + j): its row in the parent's vector
  c64* F = nullptr;                 // level vector (ld ldF)
  int64_t ldF = 0;
  c64* T = nullptr;                 // skeleton vector (ld ldT)
  int64_t ldT = 0;
  c64* Fp = nullptr;                // parent's level vector (ld ldFp)
  int64_t ldFp = 0;
};

// 8, 12 or 16 blocks of 16 for an order n (0: too large for the matrix-core sweeps)
int sweep_tile_class(int n);
// true when a level with these largest b and r has a matrix-core variant
inline bool sweep_supported(int bmax, int rmax) {
  const int cb = sweep_tile_class(bmax), cr = sweep_tile_class(std::max(rmax, 1));
  return cb != 0 && cr != 0 && cr <= cb && !(cb == 16 && cr == 16);
}
// composed permutations and inverted diagonal blocks of a level's LUs
// (blk_cell / blk_k: the (cell, block) pairs, one wavefront each)
void launch_sweep_prepare(const SweepCell* cells, int n_cells, const int* blk_cell, const int* blk_k, int n_blk,
                          const int* piv, const c64* A, int* perm, c64* Dinv, hipStream_t s);
void launch_sweep_up(const SweepLaunch& L, hipStream_t s);
// fewest right-hand sides for which the matrix-core sweep is used
constexpr int kSweepMinCols = 16;
// up to this many right-hand sides, one workgroup per cell on the vector
// units, one launch per level and direction (between the two: the LU-solve
// kernel and a GEMM with W)
constexpr int kSweepFewCols = 4;
void launch_sweep_few(const SweepLaunch& L, bool up, hipStream_t s);

}  // namespace fds
