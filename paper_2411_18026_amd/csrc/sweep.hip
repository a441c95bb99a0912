// Solve sweeps on the FP64 matrix cores (Sections 6.2, 6.3, 7.3 step 5).
//
// One wavefront owns one cell and 16 right-hand-side columns (a "slab")
// and keeps them in matrix-core accumulators from the first load to the
// last store, so a level of the upward sweep is one launch:
//   g = A_i^{-1} f_i      (LU solve: the LU's row interchanges as one
//                          permutation, then 16-row blocks: the diagonal
//                          block applied through its explicit 16 x 16
//                          inverse, the rows below / above updated by
//                          16 x 16 x 16 complex products),
//   f~ = W_i g            (W_i = A~_i V_i formed once per factor: one
//                          product with the accumulators as operand),
// and g, f~ are written to the level vector, the skeleton vector and the
// parent's rows.  (The downward sweep, f~ <- A~_i y - f~ and x = g + X_i f~,
// is two plain products per cell and stays with the batched GEMM kernel.)
//
// Matrix-core layout (v_mfma_f64_16x16x4f64, lane l, step v = 0..3): the
// A operand is A(l % 16, k), the B operand B(k, l % 16), the result
// element v of lane l is D(l / 16 + 4 v, l % 16).  The reduction index of
// lane l at step v is taken as k = l / 16 + 4 v, so that a result tile,
// left where it is, is the B operand of the next product: no data moves
// between the steps of a wavefront.  A complex product takes four real
// ones (re re, -im im, re im, im re).
//
// Blocks of a cell's matrices beyond its order b (the last block of 16
// rows is partial when 16 does not divide b) read as zero, and the
// inverted diagonal blocks carry the identity there, so padded rows stay
// zero throughout.
#include <algorithm>

#include "sweep.hpp"

namespace fds {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

struct MTile {
  d4 re, im;
};

__device__ inline void tile_zero(MTile& t) {
  t.re = d4{0.0, 0.0, 0.0, 0.0};
  t.im = d4{0.0, 0.0, 0.0, 0.0};
}

// Rows [r0, r0 + 16) of a column: lane value v sits at row r0 + l / 16 + 4 v.
__device__ inline int trow(int r0, int lane, int v) { return r0 + (lane >> 4) + 4 * v; }

// acc += op(M) * B for the 16 x 16 block of M (column-major, ld) at rows
// [r0, r0 + 16), columns [c0, c0 + 16); entries outside rows < rmax,
// columns < cmax read as zero.  NEG: acc -= M B.  B is a tile in result
// layout (see the top of the file).
template <bool NEG>
__device__ inline void mma(MTile& acc, const c64* __restrict__ M, int64_t ld, int r0, int c0, int rmax, int cmax,
                           const MTile& B, int lane) {
  const int i = r0 + (lane & 15);
  const int kb = c0 + (lane >> 4);
  double ar[4], ai[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int k = kb + 4 * v;
    c64 a = cmk(0.0, 0.0);
    if (i < rmax && k < cmax) a = M[i + (int64_t)k * ld];
    ar[v] = NEG ? -a.re : a.re;
    ai[v] = NEG ? -a.im : a.im;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    acc.re = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[v], B.re[v], acc.re, 0, 0, 0);
    acc.re = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[v], B.im[v], acc.re, 0, 0, 0);
    acc.im = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[v], B.im[v], acc.im, 0, 0, 0);
    acc.im = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[v], B.re[v], acc.im, 0, 0, 0);
  }
}

}  // namespace

// ---------------------------------------------------------------- preparation
// Composed row permutation of each cell's LU (row j swapped with piv[j],
// j ascending): (P f)(i) = f(perm(i)).  One wavefront per cell: the
// pivots into LDS, the swaps there by one lane, the result out by all.
constexpr int kPermMax = 256;   // largest order of a matrix-core sweep cell

__global__ void __launch_bounds__(64) k_compose_perm(const SweepCell* __restrict__ cells, int n_cells,
                                                     const int* __restrict__ piv, int* __restrict__ perm) {
  __shared__ int sp[kPermMax], sv[kPermMax];
  const int q = blockIdx.x;
  if (q >= n_cells) return;
  const SweepCell c = cells[q];
  const int b = min(c.b, kPermMax);
  for (int i = threadIdx.x; i < b; i += 64) {
    sp[i] = i;
    sv[i] = piv[c.piv_off + i];
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < b; ++j) {
      const int k = sv[j];
      if (k != j) {
        const int t = sp[j];
        sp[j] = sp[k];
        sp[k] = t;
      }
    }
  __syncthreads();
  for (int i = threadIdx.x; i < b; i += 64) perm[c.perm_off + i] = sp[i];
}

// Inverses of the 16 x 16 diagonal blocks of L (unit lower) and U (upper)
// of each cell's LU: one wavefront per (cell, block), lane j < 16 column j
// of L_kk^{-1} by forward substitution, lane 16 + j column j of U_kk^{-1} by
// backward substitution; identity beyond the cell's order.
__global__ void __launch_bounds__(64) k_diag_inverse(const SweepCell* __restrict__ cells,
                                                     const int* __restrict__ blk_cell, const int* __restrict__ blk_k,
                                                     const c64* __restrict__ A, c64* __restrict__ Dinv) {
  const int w = blockIdx.x;
  const SweepCell c = cells[blk_cell[w]];
  const int k = blk_k[w];
  const int lane = threadIdx.x;
  if (lane >= 32) return;
  const int j = lane & 15;
  const bool upper = lane >= 16;
  const int b = c.b, r0 = 16 * k;
  const c64* M = A + c.a_off;
  c64 x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = cmk(i == j ? 1.0 : 0.0, 0.0);
  if (!upper) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (r0 + i >= b) continue;   // identity beyond the order
      c64 s = x[i];
#pragma unroll
      for (int m = 0; m < i; ++m) s = s - M[(r0 + i) + (int64_t)(r0 + m) * b] * x[m];
      x[i] = s;
    }
  } else {
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      if (r0 + i >= b) continue;
      c64 s = x[i];
#pragma unroll
      for (int m = i + 1; m < 16; ++m)
        if (r0 + m < b) s = s - M[(r0 + i) + (int64_t)(r0 + m) * b] * x[m];
      x[i] = cdiv(s, M[(r0 + i) + (int64_t)(r0 + i) * b]);
    }
  }
  c64* out = Dinv + c.dinv_off + (int64_t)k * 512 + (upper ? 256 : 0) + 16 * j;
#pragma unroll
  for (int i = 0; i < 16; ++i) out[i] = x[i];
}

// ---------------------------------------------------------------- sweeps
// Work order: workgroup w runs on XCD w % 8; the groups of four slabs of
// one cell are given to workgroups of one XCD, so the cell's factors come
// from HBM once and then from that XCD's L2.
__device__ inline void sweep_unit(int n_groups, int& cell, int& grp) {
  const int w = blockIdx.x;
  const int xcd = w & 7, slot = w >> 3;
  cell = xcd + 8 * (slot / n_groups);
  grp = slot % n_groups;
}

// LDS pitch of a staged 16-column panel of a cell of at most 16 NB rows
// (odd: no bank aliasing across columns); the smaller cells' panels leave
// room for a second workgroup on the CU
template <int NB>
constexpr int pan_ld() { return 16 * NB + 1; }

// One 16-column panel of a cell's LU, rows [r0, r1), columns [c0, c0 + 16),
// staged in LDS with the 16 x 16 inverted diagonal block: the workgroup
// loads it into registers while the previous panel is in use, then stores
// it (P: pan_ld x 16 complex, D: 256 complex).  Rows at or beyond the
// order b (the padding of a partial last block) are stored as zeros: a
// padded entry meets the zero part of an inverted diagonal block, and
// 0 times stale LDS contents (possibly NaN) is not 0.
struct PanelRegs {
  c64 v[16];
  c64 d;
};

// Thread t takes row r0 + t of the panel (a panel has at most 240 rows,
// the workgroup 256 threads) and its 16 columns: consecutive threads read
// consecutive rows of a column.
__device__ inline void panel_fetch(PanelRegs& pr, const c64* __restrict__ L, int b, int r0, int r1, int c0,
                                   const c64* __restrict__ Di, int tid) {
  const int rr = r0 + tid;
  const bool in = rr < r1 && rr < b;
#pragma unroll
  for (int c = 0; c < 16; ++c) pr.v[c] = in ? L[rr + (int64_t)(c0 + c) * b] : cmk(0.0, 0.0);
  pr.d = Di[tid];
}

template <int LD>
__device__ inline void panel_store(const PanelRegs& pr, c64* __restrict__ P, c64* __restrict__ D, int r0, int r1,
                                   int tid) {
  if (r0 + tid < r1)
#pragma unroll
    for (int c = 0; c < 16; ++c) P[c * LD + r0 + tid] = pr.v[c];
  D[tid] = pr.d;
}

// acc -= P(rows [r0, r0 + 16), 16 panel columns) * B, P staged in LDS
template <int LD>
__device__ inline void mma_panel(MTile& acc, const c64* __restrict__ P, int r0, const MTile& B, int lane) {
  const int i = r0 + (lane & 15);
  double ar[4], ai[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const c64 a = P[((lane >> 4) + 4 * v) * LD + i];
    ar[v] = -a.re;
    ai[v] = -a.im;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    acc.re = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[v], B.re[v], acc.re, 0, 0, 0);
    acc.re = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[v], B.im[v], acc.re, 0, 0, 0);
    acc.im = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[v], B.im[v], acc.im, 0, 0, 0);
    acc.im = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[v], B.re[v], acc.im, 0, 0, 0);
  }
}

// Upward sweep of one level: a workgroup = one cell and four 16-column
// slabs (one per wavefront).  The LU solve walks the 16-column panels of
// the factor (forward: L's panel k below the diagonal block, backward: U's
// panel k above it), each staged once in LDS for the four wavefronts and
// prefetched during the previous step; then f~ = W g.
template <int NB, int NR>
__global__ void __launch_bounds__(256) k_sweep_up(const SweepCell* __restrict__ cells, int n_cells, int n_groups,
                                                  int ncol, const c64* __restrict__ A, const c64* __restrict__ Dinv,
                                                  const int* __restrict__ perm, const c64* __restrict__ W,
                                                  const int64_t* __restrict__ up_dst,
                                                  c64* __restrict__ Fv, int64_t ldF, c64* __restrict__ Tv,
                                                  int64_t ldT, c64* __restrict__ Fp, int64_t ldFp) {
  constexpr int LD = pan_ld<NB>();
  __shared__ c64 Pan[2][16 * LD];
  __shared__ c64 Dg[2][256];
  int q, grp;
  sweep_unit(n_groups, q, grp);
  if (q >= n_cells) return;   // the whole workgroup
  const int tid = threadIdx.x, lane = tid & 63;
  const SweepCell c = cells[q];
  const int b = c.b, r = c.r, nb = (b + 15) / 16, nr = (r + 15) / 16;
  const int col = (grp * 4 + (tid >> 6)) * 16 + (lane & 15);
  const bool cok = col < ncol;
  const c64* L = A + c.a_off;
  const c64* Di = Dinv + c.dinv_off;
  const int* P = perm + c.perm_off;
  // f in pivoted order
  MTile X[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = trow(16 * i, lane, v);
      c64 f = cmk(0.0, 0.0);
      if (i < nb && row < b && cok) f = Fv[c.f_off + P[row] + (int64_t)col * ldF];
      X[i].re[v] = f.re;
      X[i].im[v] = f.im;
    }
  }
  // steps s = 0 .. 2 nb - 1: forward k = s (L rows [16 k + 16, b)), then
  // backward k = 2 nb - 1 - s (U rows [0, 16 k))
  PanelRegs pr;
  const int bp = 16 * nb;   // rows of the forward panels, padding included
  panel_fetch(pr, L, b, 16, bp, 0, Di, tid);
  panel_store<LD>(pr, Pan[0], Dg[0], 16, bp, tid);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < 2 * NB; ++s) {
    if (s < 2 * nb) {
      const int buf = s & 1;
      const bool fwd = s < nb;
      const int k = fwd ? s : 2 * nb - 1 - s;
      // prefetch the next step's panel
      const int sn = s + 1;
      const bool more = sn < 2 * nb;
      if (more) {
        const bool fn = sn < nb;
        const int kn = fn ? sn : 2 * nb - 1 - sn;
        panel_fetch(pr, L, b, fn ? 16 * kn + 16 : 0, fn ? bp : 16 * kn, 16 * kn,
                    Di + (int64_t)kn * 512 + (fn ? 0 : 256), tid);
      }
      // this step: the diagonal block through its inverse, then the other rows
#pragma unroll
      for (int kk = 0; kk < NB; ++kk)
        if (kk == k) {
          MTile out;
          tile_zero(out);
          {
            double ar[4], ai[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const c64 a = Dg[buf][(lane & 15) + 16 * ((lane >> 4) + 4 * v)];
              ar[v] = a.re;
              ai[v] = a.im;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              out.re = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[v], X[kk].re[v], out.re, 0, 0, 0);
              out.re = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[v], X[kk].im[v], out.re, 0, 0, 0);
              out.im = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[v], X[kk].im[v], out.im, 0, 0, 0);
              out.im = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[v], X[kk].re[v], out.im, 0, 0, 0);
            }
          }
          X[kk] = out;
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            const bool upd = fwd ? (i > kk && i < nb) : (i < kk);
            if (upd) mma_panel<LD>(X[i], Pan[buf], 16 * i, X[kk], lane);
          }
        }
      if (more) panel_store<LD>(pr, Pan[buf ^ 1], Dg[buf ^ 1], (sn < nb) ? 16 * sn + 16 : 0,
                            (sn < nb) ? bp : 16 * (2 * nb - 1 - sn), tid);
      __syncthreads();
    }
  }
  // g = A_i^{-1} f in place
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = trow(16 * i, lane, v);
      if (i < nb && row < b && cok) Fv[c.f_off + row + (int64_t)col * ldF] = cmk(X[i].re[v], X[i].im[v]);
    }
  if (r == 0) return;
  // f~ = W g with W = A~_i V_i (formed once per factor), one tile at a time,
  // to the skeleton vector and to the parent's rows
  const int64_t* dst = up_dst + c.t_off;
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    if (j >= nr) continue;
    MTile Z;
    tile_zero(Z);
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < nb) mma<false>(Z, W + c.v_off, r, 16 * j, 16 * k, r, b, X[k], lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = trow(16 * j, lane, v);
      if (row < r && cok) {
        const c64 z = cmk(Z.re[v], Z.im[v]);
        Tv[c.t_off + row + (int64_t)col * ldT] = z;
        Fp[dst[row] + (int64_t)col * ldFp] = z;
      }
    }
  }
}

// Upward sweep of a level with few cells: a workgroup = one cell and one
// 16-column slab, its four wavefronts splitting the 16-row tiles (tile i
// belongs to wavefront i mod 4).  At step s the owner of tile k applies the
// inverted diagonal block and publishes the result in LDS; every
// wavefront then updates its own tiles below (forward) or above (backward)
// with the staged panel.  f~ = W g afterwards from all tiles in LDS, the
// rows j of W split the same way.  The same products in the same order as
// k_sweep_up (bitwise the same results), four times the workgroups and a
// quarter of the sequential tile products per step.
template <int NB, int NR>
__global__ void __launch_bounds__(256) k_sweep_up_rows(const SweepCell* __restrict__ cells, int n_cells, int n_slab,
                                                       int ncol, const c64* __restrict__ A,
                                                       const c64* __restrict__ Dinv, const int* __restrict__ perm,
                                                       const c64* __restrict__ W, const int64_t* __restrict__ up_dst,
                                                       c64* __restrict__ Fv, int64_t ldF, c64* __restrict__ Tv,
                                                       int64_t ldT, c64* __restrict__ Fp, int64_t ldFp) {
  static_assert(NB % 4 == 0 && NR % 4 == 0, "tiles are dealt to four wavefronts");
  constexpr int LD = pan_ld<NB>();
  constexpr int NT = NB / 4;
  __shared__ c64 Pan[2][16 * LD];
  __shared__ c64 Dg[2][256];
  __shared__ double Xs[2][2][4][64];   // published tile: [buffer][re, im][v][lane]
  static_assert(sizeof(Pan) >= (size_t)NB * 512 * sizeof(double), "all tiles fit in the panel buffers");
  int q, slab;
  sweep_unit(n_slab, q, slab);
  if (q >= n_cells) return;   // the whole workgroup
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const SweepCell c = cells[q];
  const int b = c.b, r = c.r, nb = (b + 15) / 16, nr = (r + 15) / 16;
  const int col = slab * 16 + (lane & 15);
  const bool cok = col < ncol;
  const c64* L = A + c.a_off;
  const c64* Di = Dinv + c.dinv_off;
  const int* P = perm + c.perm_off;
  // the wavefront's tiles i = 4 t + wv of f, in pivoted order
  MTile X[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int i = 4 * t + wv;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = trow(16 * i, lane, v);
      c64 f = cmk(0.0, 0.0);
      if (i < nb && row < b && cok) f = Fv[c.f_off + P[row] + (int64_t)col * ldF];
      X[t].re[v] = f.re;
      X[t].im[v] = f.im;
    }
  }
  PanelRegs pr;
  const int bp = 16 * nb;
  panel_fetch(pr, L, b, 16, bp, 0, Di, tid);
  panel_store<LD>(pr, Pan[0], Dg[0], 16, bp, tid);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < 2 * NB; ++s) {
    if (s < 2 * nb) {
      const int buf = s & 1;
      const bool fwd = s < nb;
      const int k = fwd ? s : 2 * nb - 1 - s;
      const int sn = s + 1;
      const bool more = sn < 2 * nb;
      if (more) {
        const bool fn = sn < nb;
        const int kn = fn ? sn : 2 * nb - 1 - sn;
        panel_fetch(pr, L, b, fn ? 16 * kn + 16 : 0, fn ? bp : 16 * kn, 16 * kn,
                    Di + (int64_t)kn * 512 + (fn ? 0 : 256), tid);
      }
      // the owner of tile k: the diagonal block through its inverse, published
      if ((k & 3) == wv) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (4 * t + wv == k) {
            MTile out;
            tile_zero(out);
            double ar[4], ai[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const c64 a = Dg[buf][(lane & 15) + 16 * ((lane >> 4) + 4 * v)];
              ar[v] = a.re;
              ai[v] = a.im;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              out.re = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[v], X[t].re[v], out.re, 0, 0, 0);
              out.re = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[v], X[t].im[v], out.re, 0, 0, 0);
              out.im = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[v], X[t].im[v], out.im, 0, 0, 0);
              out.im = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[v], X[t].re[v], out.im, 0, 0, 0);
            }
            X[t] = out;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              Xs[buf][0][v][lane] = out.re[v];
              Xs[buf][1][v][lane] = out.im[v];
            }
          }
      }
      __syncthreads();
      MTile B;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        B.re[v] = Xs[buf][0][v][lane];
        B.im[v] = Xs[buf][1][v][lane];
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int i = 4 * t + wv;
        const bool upd = fwd ? (i > k && i < nb) : (i < k);
        if (upd) mma_panel<LD>(X[t], Pan[buf], 16 * i, B, lane);
      }
      if (more) panel_store<LD>(pr, Pan[buf ^ 1], Dg[buf ^ 1], (sn < nb) ? 16 * sn + 16 : 0,
                                (sn < nb) ? bp : 16 * (2 * nb - 1 - sn), tid);
      __syncthreads();
    }
  }
  // g = A_i^{-1} f in place, each wavefront its tiles
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int i = 4 * t + wv;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = trow(16 * i, lane, v);
      if (i < nb && row < b && cok) Fv[c.f_off + row + (int64_t)col * ldF] = cmk(X[t].re[v], X[t].im[v]);
    }
  }
  if (r == 0) return;   // the whole workgroup
  // every tile of g to LDS (the panel buffers are free), then f~ = W g with
  // the rows j of W dealt to the wavefronts
  double* Xa = reinterpret_cast<double*>(&Pan[0][0]);   // [tile][re, im][v][lane]
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int i = 4 * t + wv;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Xa[((i * 2 + 0) * 4 + v) * 64 + lane] = X[t].re[v];
      Xa[((i * 2 + 1) * 4 + v) * 64 + lane] = X[t].im[v];
    }
  }
  __syncthreads();
  const int64_t* dst = up_dst + c.t_off;
#pragma unroll
  for (int jt = 0; jt < NR / 4; ++jt) {
    const int j = 4 * jt + wv;
    if (j >= nr) continue;
    MTile Z;
    tile_zero(Z);
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < nb) {
        MTile G;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          G.re[v] = Xa[((k * 2 + 0) * 4 + v) * 64 + lane];
          G.im[v] = Xa[((k * 2 + 1) * 4 + v) * 64 + lane];
        }
        mma<false>(Z, W + c.v_off, r, 16 * j, 16 * k, r, b, G, lane);
      }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = trow(16 * j, lane, v);
      if (row < r && cok) {
        const c64 z = cmk(Z.re[v], Z.im[v]);
        Tv[c.t_off + row + (int64_t)col * ldT] = z;
        Fp[dst[row] + (int64_t)col * ldFp] = z;
      }
    }
  }
}

// ---------------------------------------------------------------- few right-hand sides
// One to four right-hand sides (the first solve, sequential use): the
// matrix-core tiles would be mostly empty, so one workgroup per cell runs
// the same steps on the vector units with a thread per row.  Upward: LU
// solve by 16-row blocks (the block's 16 rows solve their diagonal block
// with lane-to-lane broadcasts, then every row below / above subtracts the
// block's contribution; the next panel row is fetched while the current one
// is used), then f~ = W g with a thread per row of W.  Downward: y from the
// parent's rows, z = A~ y - f~, x = g + X z, a thread per row.  Cells of at
// most 256 unknowns (one row per thread).

// value of lane Q of each row of 16 lanes, to the whole row (DPP row_newbcast)
template <int Q>
__device__ inline double bcast16_lane(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x150 + Q, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x150 + Q, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline c64 bcast16(c64 v, int q) {   // q is a constant once the caller's loop is unrolled
  switch (q) {
#define FDS_BC(Q) \
  case Q: return cmk(bcast16_lane<Q>(v.re), bcast16_lane<Q>(v.im));
    FDS_BC(0) FDS_BC(1) FDS_BC(2) FDS_BC(3) FDS_BC(4) FDS_BC(5) FDS_BC(6) FDS_BC(7)
    FDS_BC(8) FDS_BC(9) FDS_BC(10) FDS_BC(11) FDS_BC(12) FDS_BC(13) FDS_BC(14) FDS_BC(15)
#undef FDS_BC
    default: return v;
  }
}

// acc -= a * x with fused multiply-adds
__device__ inline void cfms64(c64& acc, c64 a, c64 x) {
  acc.re = fma(-a.re, x.re, acc.re);
  acc.re = fma(a.im, x.im, acc.re);
  acc.im = fma(-a.re, x.im, acc.im);
  acc.im = fma(-a.im, x.re, acc.im);
}

template <int NC>
__global__ void __launch_bounds__(256) k_sweep_up_few(const SweepCell* __restrict__ cells, int ncol,
                                                      const c64* __restrict__ A, const int* __restrict__ perm,
                                                      const c64* __restrict__ W, const int64_t* __restrict__ up_dst,
                                                      c64* __restrict__ Fv, int64_t ldF, c64* __restrict__ Tv,
                                                      int64_t ldT, c64* __restrict__ Fp, int64_t ldFp) {
  __shared__ c64 xs[2][16 * NC];   // the block just solved, by block parity
  __shared__ c64 gs[256 * NC];     // g, for the product with W
  const SweepCell c = cells[blockIdx.x];
  const int b = c.b, r = c.r, nb = (b + 15) / 16;
  const int tid = threadIdx.x, q16 = tid & 15, kown = tid >> 4;
  const bool own = tid < b;
  const c64* L = A + c.a_off;
  c64 x[NC];
#pragma unroll
  for (int cc = 0; cc < NC; ++cc)
    x[cc] = (own && cc < ncol) ? Fv[c.f_off + perm[c.perm_off + tid] + (int64_t)cc * ldF] : cmk(0.0, 0.0);
  c64 lr[16], ln[16];
  auto fetch = [&](c64 (&dst)[16], int k) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int col = 16 * k + q;
      dst[q] = (own && col < b) ? L[tid + (int64_t)col * b] : cmk(0.0, 0.0);
    }
  };
  // forward substitution with unit L
  fetch(lr, 0);
  for (int k = 0; k < nb; ++k) {
    if (k + 1 < nb) fetch(ln, k + 1);
    if (kown == k) {   // the 16 rows of block k (one DPP row of lanes)
#pragma unroll
      for (int q = 0; q < 15; ++q)
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          const c64 xq = bcast16(x[cc], q);
          if (q16 > q) cfms64(x[cc], lr[q], xq);
        }
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) xs[k & 1][q16 * NC + cc] = x[cc];
    }
    __syncthreads();
    if (own && kown > k)
#pragma unroll
      for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) cfms64(x[cc], lr[q], xs[k & 1][q * NC + cc]);
#pragma unroll
    for (int q = 0; q < 16; ++q) lr[q] = ln[q];
  }
  // backward substitution with U
  fetch(lr, nb - 1);
  for (int k = nb - 1; k >= 0; --k) {
    if (k > 0) fetch(ln, k - 1);
    if (kown == k) {
#pragma unroll
      for (int q = 15; q >= 0; --q)
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          if (q16 == q && own) x[cc] = cdiv(x[cc], lr[q]);
          const c64 xq = bcast16(x[cc], q);
          if (q16 < q) cfms64(x[cc], lr[q], xq);
        }
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) xs[k & 1][q16 * NC + cc] = x[cc];
    }
    __syncthreads();
    if (own && kown < k)
#pragma unroll
      for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) cfms64(x[cc], lr[q], xs[k & 1][q * NC + cc]);
#pragma unroll
    for (int q = 0; q < 16; ++q) lr[q] = ln[q];
  }
  // g = A_i^{-1} f in place, and to LDS for f~ = W g
#pragma unroll
  for (int cc = 0; cc < NC; ++cc) {
    if (own && cc < ncol) Fv[c.f_off + tid + (int64_t)cc * ldF] = x[cc];
    gs[tid * NC + cc] = x[cc];
  }
  __syncthreads();
  if (tid < r) {
    const c64* Wr = W + c.v_off + tid;
    c64 z[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) z[cc] = cmk(0.0, 0.0);
    for (int i = 0; i < b; ++i) {
      const c64 w = Wr[(int64_t)i * r];
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) cfms64(z[cc], cmk(-w.re, -w.im), gs[i * NC + cc]);
    }
    const int64_t dst = up_dst[c.t_off + tid];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc)
      if (cc < ncol) {
        Tv[c.t_off + tid + (int64_t)cc * ldT] = z[cc];
        Fp[dst + (int64_t)cc * ldFp] = z[cc];
      }
  }
}

template <int NC>
__global__ void __launch_bounds__(256) k_sweep_down_few(const SweepCell* __restrict__ cells, int ncol,
                                                        const c64* __restrict__ At, const c64* __restrict__ Xm,
                                                        const int64_t* __restrict__ up_dst, c64* __restrict__ Fv,
                                                        int64_t ldF, const c64* __restrict__ Tv, int64_t ldT,
                                                        const c64* __restrict__ Fp, int64_t ldFp) {
  __shared__ c64 ys[256 * NC];
  __shared__ c64 zs[256 * NC];
  const SweepCell c = cells[blockIdx.x];
  const int b = c.b, r = c.r;
  if (r == 0) return;   // the whole workgroup: x = g already
  const int tid = threadIdx.x;
  if (tid < r) {
    const int64_t src = up_dst[c.t_off + tid];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) ys[tid * NC + cc] = cc < ncol ? Fp[src + (int64_t)cc * ldFp] : cmk(0.0, 0.0);
  }
  __syncthreads();
  if (tid < r) {   // z = A~ y - f~
    const c64* Ar = At + c.at_off + tid;
    c64 z[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const c64 t = cc < ncol ? Tv[c.t_off + tid + (int64_t)cc * ldT] : cmk(0.0, 0.0);
      z[cc] = cmk(-t.re, -t.im);
    }
    for (int k = 0; k < r; ++k) {
      const c64 a = Ar[(int64_t)k * r];
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) cfms64(z[cc], cmk(-a.re, -a.im), ys[k * NC + cc]);
    }
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) zs[tid * NC + cc] = z[cc];
  }
  __syncthreads();
  if (tid < b) {   // x = g + X z
    const c64* Xr = Xm + c.x_off + tid;
    c64 x[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) x[cc] = cc < ncol ? Fv[c.f_off + tid + (int64_t)cc * ldF] : cmk(0.0, 0.0);
    for (int j = 0; j < r; ++j) {
      const c64 a = Xr[(int64_t)j * b];
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) cfms64(x[cc], cmk(-a.re, -a.im), zs[j * NC + cc]);
    }
#pragma unroll
    for (int cc = 0; cc < NC; ++cc)
      if (cc < ncol) Fv[c.f_off + tid + (int64_t)cc * ldF] = x[cc];
  }
}

// ---------------------------------------------------------------- launchers
void launch_sweep_prepare(const SweepCell* cells, int n_cells, const int* blk_cell, const int* blk_k, int n_blk,
                          const int* piv, const c64* A, int* perm, c64* Dinv, hipStream_t s) {
  if (n_cells == 0) return;
  k_compose_perm<<<n_cells, 64, 0, s>>>(cells, n_cells, piv, perm);
  FDS_HIP(hipGetLastError());
  if (n_blk == 0) return;
  k_diag_inverse<<<n_blk, 64, 0, s>>>(cells, blk_cell, blk_k, A, Dinv);
  FDS_HIP(hipGetLastError());
}

int sweep_tile_class(int n) { return n <= 128 ? 8 : n <= 192 ? 12 : n <= 256 ? 16 : 0; }

// The row-split kernel (one slab per workgroup, four times the
// workgroups) for levels of fewer than kRowsBelow workgroups of four slabs,
// and for the 16-tile class, whose sixteen tiles per wavefront do not fit
// the four-slab kernel's registers.
constexpr int kRowsBelow = 128;

template <int NB, int NR>
static void up_t(const SweepLaunch& L, hipStream_t s) {
  const int n_groups = (L.n_slab + 3) / 4;
  if (NB == 16 || (int64_t)L.n_cells * n_groups < kRowsBelow) {
    const int grid = 8 * ((L.n_cells + 7) / 8) * L.n_slab;
    k_sweep_up_rows<NB, NR><<<grid, 256, 0, s>>>(L.cells, L.n_cells, L.n_slab, L.ncol, L.A, L.Dinv, L.perm, L.W,
                                                 L.up_dst, L.F, L.ldF, L.T, L.ldT, L.Fp, L.ldFp);
    return;
  }
  const int grid = 8 * ((L.n_cells + 7) / 8) * n_groups;
  k_sweep_up<NB, NR><<<grid, 256, 0, s>>>(L.cells, L.n_cells, n_groups, L.ncol, L.A, L.Dinv, L.perm, L.W, L.up_dst,
                                          L.F, L.ldF, L.T, L.ldT, L.Fp, L.ldFp);
}

#define FDS_SWEEP_DISPATCH(fn)                                         \
  switch (L.nb_class * 100 + L.nr_class) {                             \
    case 808: fn<8, 8>(L, s); break;                                   \
    case 1208: fn<12, 8>(L, s); break;                                 \
    case 1212: fn<12, 12>(L, s); break;                                \
    case 1608: fn<16, 8>(L, s); break;                                 \
    case 1612: fn<16, 12>(L, s); break;                                \
    default: throw Error(1, "sweep: no matrix-core variant for this level"); \
  }

template <int NC>
static void few_t(const SweepLaunch& L, bool up, hipStream_t s) {
  if (up)
    k_sweep_up_few<NC><<<L.n_cells, 256, 0, s>>>(L.cells, L.ncol, L.A, L.perm, L.W, L.up_dst, L.F, L.ldF, L.T, L.ldT,
                                                  L.Fp, L.ldFp);
  else
    k_sweep_down_few<NC><<<L.n_cells, 256, 0, s>>>(L.cells, L.ncol, L.At, L.X, L.up_dst, L.F, L.ldF, L.T, L.ldT,
                                                    L.Fp, L.ldFp);
}

void launch_sweep_few(const SweepLaunch& L, bool up, hipStream_t s) {
  if (L.n_cells == 0 || L.ncol == 0) return;
  if (L.ncol > kSweepFewCols) throw Error(1, "sweep: too many columns for the few-column kernels");
  if (L.ncol == 1)
    few_t<1>(L, up, s);
  else if (L.ncol == 2)
    few_t<2>(L, up, s);
  else
    few_t<4>(L, up, s);
  FDS_HIP(hipGetLastError());
}

void launch_sweep_up(const SweepLaunch& L, hipStream_t s) {
  if (L.n_cells == 0 || L.ncol == 0) return;
  FDS_SWEEP_DISPATCH(up_t)
  FDS_HIP(hipGetLastError());
}

}  // namespace fds
