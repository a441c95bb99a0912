// Batched variable-size complex linear algebra kernels (gfx950).
//
// One workgroup per problem (LU, pivoted QR, interpolation matrices) or per
// (problem, tile) (solves, GEMM, scatters); every launch covers a whole
// batch of unevenly sized problems described by descriptor arrays.  The LU,
// LU-solve, GEMM and copy kernels are templated on the complex scalar type:
// complex FP64 for the plain form, complex FP32 (FP32 accumulation) for the
// merges and sweeps of the mixed-precision form.
#include <algorithm>
#include <map>
#include <mutex>

#include "devmem.hpp"
#include "linalg.hpp"

namespace fds {

constexpr int kBlk = 256;

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename T>
__device__ inline T zero() {
  return Cx<T>::make(0.0, 0.0);
}

// acc += a b with explicitly fused multiply-adds, so that every tile shape
// performs the same floating-point operations
__device__ inline void cfma(c64& acc, c64 a, c64 b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
__device__ inline void cfma(c32& acc, c32 a, c32 b) {
  acc.re = fmaf(a.re, b.re, acc.re);
  acc.re = fmaf(-a.im, b.im, acc.re);
  acc.im = fmaf(a.re, b.im, acc.im);
  acc.im = fmaf(a.im, b.re, acc.im);
}

// Value of lane q of each row of 16 lanes, broadcast to the row (DPP
// row_newbcast: a register move, no LDS round trip).  All lanes active.
template <int Q>
__device__ inline double row_bcast_lane(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x150 + Q, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x150 + Q, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int Q>
__device__ inline float row_bcast_lane(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + Q, 0xF, 0xF, false));
}
template <typename T>
__device__ inline T row_bcast(T v, int q) {   // q is a constant once the caller's loop is unrolled
  switch (q) {
#define FDS_RB(Q) \
  case Q: v.re = row_bcast_lane<Q>(v.re); v.im = row_bcast_lane<Q>(v.im); return v;
    FDS_RB(0) FDS_RB(1) FDS_RB(2) FDS_RB(3) FDS_RB(4) FDS_RB(5) FDS_RB(6) FDS_RB(7)
    FDS_RB(8) FDS_RB(9) FDS_RB(10) FDS_RB(11) FDS_RB(12) FDS_RB(13) FDS_RB(14) FDS_RB(15)
#undef FDS_RB
    default: return v;
  }
}

// acc -= a b with explicit fused multiply-adds (same rounding in every kernel)
template <typename T>
__device__ inline void cfms(T& acc, T a, T b) {
  cfma(acc, Cx<T>::make(-(double)a.re, -(double)a.im), b);
}

template <typename TD, typename TS>
__device__ inline TD cvt(TS a) {
  return Cx<TD>::make((double)a.re, (double)a.im);
}

// ------------------------------------------------------------------ LU
// Right-looking LU with partial pivoting (largest modulus, lowest row on
// ties).  L is unit lower triangular, stored below the diagonal; piv[j] is
// the row swapped with row j at step j (LAPACK convention, 0-based).
// Unblocked form: the fallback for matrices too large for the panel in LDS.
template <typename T>
__global__ void __launch_bounds__(kBlk) k_lu(const LUDesc* __restrict__ descs, T* __restrict__ base,
                                             int* __restrict__ piv, int* __restrict__ info) {
  const LUDesc d = descs[blockIdx.x];
  T* A = base + d.a_off;
  int* P = piv + d.piv_off;
  const int n = d.n, lda = d.lda;
  const int tid = threadIdx.x;
  __shared__ double sv[kBlk];
  __shared__ int si[kBlk];
  int bad = 0;
  for (int j = 0; j < n; ++j) {
    double best = -1.0;
    int bi = n;
    for (int i = j + tid; i < n; i += kBlk) {
      const double v = abs2(A[i + (int64_t)j * lda]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int o = kBlk / 2; o > 0; o >>= 1) {
      if (tid < o) {
        const double a = sv[tid], b = sv[tid + o];
        const int ia = si[tid], ib = si[tid + o];
        if (b > a || (b == a && ib < ia)) {
          sv[tid] = b;
          si[tid] = ib;
        }
      }
      __syncthreads();
    }
    const int p = si[0] < n ? si[0] : j;   // no finite candidate: keep the row (reported below)
    const double pv = sv[0];
    __syncthreads();
    if (tid == 0) P[j] = p;
    if (!(pv > 0.0) || !isfinite(pv)) bad = bad ? bad : j + 1;
    if (p != j) {
      for (int c = tid; c < n; c += kBlk) {
        const T t = A[j + (int64_t)c * lda];
        A[j + (int64_t)c * lda] = A[p + (int64_t)c * lda];
        A[p + (int64_t)c * lda] = t;
      }
    }
    __syncthreads();
    const T piv_v = A[j + (int64_t)j * lda];
    const T inv = (pv > 0.0) ? cdiv(Cx<T>::make(1.0, 0.0), piv_v) : zero<T>();
    for (int i = j + 1 + tid; i < n; i += kBlk) A[i + (int64_t)j * lda] = A[i + (int64_t)j * lda] * inv;
    __syncthreads();
    const int m = n - j - 1;
    const int64_t mm = (int64_t)m * m;
    for (int64_t t = tid; t < mm; t += kBlk) {
      const int i = j + 1 + (int)(t % m);
      const int c = j + 1 + (int)(t / m);
      A[i + (int64_t)c * lda] -= A[i + (int64_t)j * lda] * A[j + (int64_t)c * lda];
    }
    __syncthreads();
  }
  if (tid == 0 && info) info[blockIdx.x] = bad;
}

// Blocked right-looking LU with partial pivoting, panel width NB.  Same
// pivot rule and output layout as k_lu.  The panel (rows k0.., NB columns)
// is factored in LDS by one wavefront; its row interchanges are then
// applied to the other columns, U12 = L11^{-1} A12 is formed column by
// column, and the trailing matrix gets one rank-NB update per panel in
// register tiles.  TB threads per workgroup: 256
// when a launch has a matrix per CU or more, 1024 for the few large
// matrices of the upper levels (more wavefronts to hide the trailing
// update's memory latency).
template <int NB, typename T, int TB>
__global__ void __launch_bounds__(TB) k_lu_blk(const LUDesc* __restrict__ descs, T* __restrict__ base,
                                                 int* __restrict__ piv, int* __restrict__ info) {
  extern __shared__ unsigned char smem_lu[];
  T* Pn = reinterpret_cast<T*>(smem_lu);   // panel, column-major with leading dimension ldp
  __shared__ int sp[NB];                   // the panel's pivot rows (relative to k0)
  const LUDesc d = descs[blockIdx.x];
  T* A = base + d.a_off;
  int* P = piv + d.piv_off;
  const int n = d.n, lda = d.lda;
  const int ldp = n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int bad = 0;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nb = min(NB, n - k0), mp = n - k0;
    for (int t = tid; t < mp * nb; t += TB) {
      const int i = t % mp, c = t / mp;
      Pn[i + c * ldp] = A[(k0 + i) + (int64_t)(k0 + c) * lda];
    }
    __syncthreads();
    // the panel is factored by wavefront 0 alone: pivot search by lane
    // reductions, no workgroup barrier per column (the LDS accesses of one
    // wavefront take effect in program order; the fences keep the compiler
    // from reordering them)
    if (wid == 0) {
      for (int j = 0; j < nb; ++j) {
        // pivot: largest modulus in panel column j at rows >= j, lowest row on ties
        double best = -1.0;
        int bi = INT32_MAX;
        for (int i = j + lane; i < mp; i += 64) {
          const double v = abs2(Pn[i + j * ldp]);
          if (v > best) {
            best = v;
            bi = i;
          }
        }
        const double top = wmax_full(best);
        int p = wmin_int_full(best == top ? bi : INT32_MAX);
        if (p >= mp) p = j;   // no finite candidate: keep the row (reported below)
        if (lane == 0) {
          sp[j] = p;
          P[k0 + j] = k0 + p;
          if (!(top > 0.0) || !isfinite(top)) bad = bad ? bad : k0 + j + 1;
        }
        if (p != j && lane < nb) {
          const T t = Pn[j + lane * ldp];
          Pn[j + lane * ldp] = Pn[p + lane * ldp];
          Pn[p + lane * ldp] = t;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const T pj = Pn[j + j * ldp];
        const T inv = abs2(pj) > 0 ? cdiv(Cx<T>::make(1.0, 0.0), pj) : zero<T>();
        for (int i = j + 1 + lane; i < mp; i += 64) {
          const T l = Pn[i + j * ldp] * inv;
          Pn[i + j * ldp] = l;
          for (int c = j + 1; c < nb; ++c) Pn[i + c * ldp] -= l * Pn[j + c * ldp];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    }
    __syncthreads();
    for (int t = tid; t < mp * nb; t += TB) {
      const int i = t % mp, c = t / mp;
      A[(k0 + i) + (int64_t)(k0 + c) * lda] = Pn[i + c * ldp];
    }
    // row interchanges of this panel on the columns outside it, one thread per column
    for (int c = tid; c < n; c += TB) {
      if (c >= k0 && c < k0 + nb) continue;
      T* col = A + (int64_t)c * lda;
      for (int j = 0; j < nb; ++j) {
        const int p = k0 + sp[j];
        if (p != k0 + j) {
          const T t = col[k0 + j];
          col[k0 + j] = col[p];
          col[p] = t;
        }
      }
    }
    __syncthreads();
    // U12 = L11^{-1} A12, one thread per column
    for (int c = k0 + nb + tid; c < n; c += TB) {
      T* col = A + (int64_t)c * lda + k0;
      T x[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        if (r < nb) {
          T s = col[r];
#pragma unroll
          for (int q = 0; q < NB; ++q)
            if (q < r) s -= Pn[r + q * ldp] * x[q];
          x[r] = s;
          col[r] = s;
        }
      }
    }
    __syncthreads();
    // A22 -= L21 U12 in register tiles of TR x TC entries: rows ti + t2r a
    // and columns tj + t2c b, so that a wavefront's lanes take consecutive
    // rows (coalesced, conflict-free LDS reads of L21) and share the U12
    // entries of a column; padded rows and columns read a valid entry and
    // are not stored
    {
      constexpr int TR = TB >= 1024 ? 4 : 2, TC = 2;
      const int m2 = n - k0 - nb, t2r = (m2 + TR - 1) / TR, t2c = (m2 + TC - 1) / TC;
      T* A22 = A + (k0 + nb) + (int64_t)(k0 + nb) * lda;
      const T* U12 = A + k0 + (int64_t)(k0 + nb) * lda;
      for (int tt = tid; tt < t2r * t2c; tt += TB) {
        const int ti = tt % t2r, tj = tt / t2r;
        T acc[TR][TC];
#pragma unroll
        for (int b = 0; b < TC; ++b)
#pragma unroll
          for (int a = 0; a < TR; ++a)
            acc[a][b] = A22[min(ti + t2r * a, m2 - 1) + (int64_t)min(tj + t2c * b, m2 - 1) * lda];
#pragma unroll 1
        for (int q = 0; q < nb; ++q) {
          T l[TR], u[TC];
#pragma unroll
          for (int a = 0; a < TR; ++a) l[a] = Pn[(nb + min(ti + t2r * a, m2 - 1)) + q * ldp];
#pragma unroll
          for (int b = 0; b < TC; ++b) u[b] = U12[q + (int64_t)min(tj + t2c * b, m2 - 1) * lda];
#pragma unroll
          for (int a = 0; a < TR; ++a)
#pragma unroll
            for (int b = 0; b < TC; ++b) cfms(acc[a][b], l[a], u[b]);
        }
#pragma unroll
        for (int b = 0; b < TC; ++b)
#pragma unroll
          for (int a = 0; a < TR; ++a)
            if (ti + t2r * a < m2 && tj + t2c * b < m2)
              A22[(ti + t2r * a) + (int64_t)(tj + t2c * b) * lda] = acc[a][b];
      }
    }
    __syncthreads();
  }
  if (tid == 0 && info) info[blockIdx.x] = bad;
}

// Blocked LU for matrices too large for the LDS panel of k_lu_blk, spread
// over many workgroups: per panel of kPanel columns, k_panel_lu factors the
// panel (one workgroup per matrix), k_swap_outside applies its row
// interchanges to the other columns, k_trsm_u12 forms U12 = L11^{-1} A12 and
// the batched GEMM updates the trailing matrix.  Same pivot rule and output
// layout as k_lu.
constexpr int kPanel = 32;

template <typename T>
__global__ void __launch_bounds__(kBlk) k_panel_lu(const LUDesc* __restrict__ descs, int k0, T* __restrict__ base,
                                                   int* __restrict__ piv, int* __restrict__ info) {
  __shared__ double sv[kBlk / 64];
  __shared__ int si[kBlk / 64];
  __shared__ int s_p;
  const LUDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  T* A = base + d.a_off;
  int* P = piv + d.piv_off;
  const int n = d.n, lda = d.lda, nb = min(kPanel, n - k0);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int j = 0; j < nb; ++j) {
    const int col = k0 + j;
    T* cj = A + (int64_t)col * lda;
    double best = -1.0;
    int bi = n;
    for (int i = col + tid; i < n; i += kBlk) {
      const double v = abs2(cj[i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      sv[wid] = best;
      si[wid] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = sv[0];
      int ib = si[0];
      for (int w = 1; w < kBlk / 64; ++w)
        if (sv[w] > b || (sv[w] == b && si[w] < ib)) {
          b = sv[w];
          ib = si[w];
        }
      if (ib >= n) ib = col;   // no finite candidate: keep the row (reported below)
      s_p = ib;
      P[col] = ib;
      if ((!(b > 0.0) || !isfinite(b)) && info && info[blockIdx.x] == 0) info[blockIdx.x] = col + 1;
    }
    __syncthreads();
    const int p = s_p;
    if (p != col && tid < nb) {
      T* cc = A + (int64_t)(k0 + tid) * lda;
      const T t = cc[col];
      cc[col] = cc[p];
      cc[p] = t;
    }
    __syncthreads();
    const T pj = cj[col];
    const T inv = abs2(pj) > 0 ? cdiv(Cx<T>::make(1.0, 0.0), pj) : zero<T>();
    for (int i = col + 1 + tid; i < n; i += kBlk) {
      const T l = cj[i] * inv;
      cj[i] = l;
      for (int c = j + 1; c < nb; ++c) {
        T* cc = A + (int64_t)(k0 + c) * lda;
        cc[i] -= l * cc[col];
      }
    }
    __syncthreads();
  }
}

// The same panel step with the panel (rows k0.., KP columns) staged in LDS:
// per column a pivot search by lane reductions and one exchange of partial
// results between the wavefronts, the row swap and the rank-1 update in
// LDS, then one write-back.  Dynamic LDS: (n - k0) KP entries.
template <typename T, int KP>
__global__ void __launch_bounds__(kBlk) k_panel_lu_lds(const LUDesc* __restrict__ descs, int k0,
                                                       T* __restrict__ base, int* __restrict__ piv,
                                                       int* __restrict__ info) {
  extern __shared__ unsigned char smem_pl[];
  T* Pn = reinterpret_cast<T*>(smem_pl);   // column-major, leading dimension mp
  constexpr int NW = kBlk / 64;
  __shared__ double s_v[NW];
  __shared__ int s_i[NW];
  const LUDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  T* A = base + d.a_off;
  int* P = piv + d.piv_off;
  const int n = d.n, lda = d.lda, nb = min(KP, n - k0), mp = n - k0;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int t = tid; t < mp * nb; t += kBlk) {
    const int i = t % mp, c = t / mp;
    Pn[i + c * mp] = A[(k0 + i) + (int64_t)(k0 + c) * lda];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    // pivot: largest modulus in column j at rows >= j, lowest row on ties
    double best = -1.0;
    int bi = INT32_MAX;
    for (int i = j + tid; i < mp; i += kBlk) {
      const double v = abs2(Pn[i + j * mp]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    const double top = wmax_full(best);
    const int wi = wmin_int_full(best == top ? bi : INT32_MAX);
    if (lane == 0) {
      s_v[wid] = top;
      s_i[wid] = wi;
    }
    __syncthreads();
    double b = s_v[0];
    int p = s_i[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
      if (s_v[w] > b || (s_v[w] == b && s_i[w] < p)) {
        b = s_v[w];
        p = s_i[w];
      }
    if (p >= mp) p = j;   // no finite candidate: keep the row (reported)
    if (tid == 0) {
      P[k0 + j] = k0 + p;
      if ((!(b > 0.0) || !isfinite(b)) && info && info[blockIdx.x] == 0) info[blockIdx.x] = k0 + j + 1;
    }
    if (p != j && tid < nb) {
      const T t = Pn[j + tid * mp];
      Pn[j + tid * mp] = Pn[p + tid * mp];
      Pn[p + tid * mp] = t;
    }
    __syncthreads();
    const T pj = Pn[j + j * mp];
    const T inv = abs2(pj) > 0 ? cdiv(Cx<T>::make(1.0, 0.0), pj) : zero<T>();
    for (int i = j + 1 + tid; i < mp; i += kBlk) {
      const T l = Pn[i + j * mp] * inv;
      Pn[i + j * mp] = l;
      for (int c = j + 1; c < nb; ++c) Pn[i + c * mp] -= l * Pn[j + c * mp];
    }
    __syncthreads();
  }
  for (int t = tid; t < mp * nb; t += kBlk) {
    const int i = t % mp, c = t / mp;
    A[(k0 + i) + (int64_t)(k0 + c) * lda] = Pn[i + c * mp];
  }
}

// row interchanges of panel k0 (KP columns) on every column outside it:
// the panel's interchanges composed into one permutation (simulated on the
// rows k0.. in LDS by one thread), whose cnt <= 2 KP moved rows are then
// applied with one thread per (column, moved row): every load of the
// workgroup before its barrier, every store after it.  A workgroup takes
// 256 / cnt of the columns outside the panel; the grid covers cnt = 64.
// Dynamic LDS: n - k0 ints.
template <typename T, int KP>
__global__ void __launch_bounds__(256) k_swap_outside(const LUDesc* __restrict__ descs, int k0, T* __restrict__ base,
                                                      const int* __restrict__ piv) {
  static_assert(2 * KP <= 64, "at least four columns per workgroup");
  extern __shared__ int perm[];   // perm[x]: the row (relative to k0) whose entry ends at row x
  __shared__ int s_row[2 * KP], s_src[2 * KP];
  __shared__ int s_cnt;
  const LUDesc d = descs[blockIdx.y];
  if (k0 >= d.n) return;
  const int nb = min(KP, d.n - k0), mp = d.n - k0;
  const int* P = piv + d.piv_off;
  for (int i = threadIdx.x; i < mp; i += blockDim.x) perm[i] = i;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < nb; ++j) {
      const int p = P[k0 + j] - k0;
      if (p != j) {
        const int t = perm[j];
        perm[j] = perm[p];
        perm[p] = t;
      }
    }
  __syncthreads();
  for (int i = threadIdx.x; i < mp; i += blockDim.x)
    if (perm[i] != i) {
      const int q = atomicAdd(&s_cnt, 1);
      s_row[q] = i;
      s_src[q] = perm[i];
    }
  __syncthreads();
  const int cnt = s_cnt;
  if (cnt == 0) return;
  const int per = 256 / cnt, cl = threadIdx.x / cnt, q = threadIdx.x % cnt;
  const int oc = blockIdx.x * per + cl;          // index among the columns outside the panel
  const int c = oc < k0 ? oc : oc + nb;
  const bool act = cl < per && c < d.n;
  T* A = base + d.a_off + k0;
  T v{};
  if (act) v = A[s_src[q] + (int64_t)c * d.lda];
  __syncthreads();
  if (act) A[s_row[q] + (int64_t)c * d.lda] = v;
}

// The same interchanges one column per thread, in sequence (rows too many
// for the composed permutation in LDS)
template <typename T, int KP>
__global__ void k_swap_outside_seq(const LUDesc* __restrict__ descs, int k0, T* __restrict__ base,
                                   const int* __restrict__ piv) {
  const LUDesc d = descs[blockIdx.y];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (k0 >= d.n || c >= d.n) return;
  const int nb = min(KP, d.n - k0);
  if (c >= k0 && c < k0 + nb) return;
  T* col = base + d.a_off + (int64_t)c * d.lda;
  const int* P = piv + d.piv_off;
  for (int j = 0; j < nb; ++j) {
    const int p = P[k0 + j];
    if (p != k0 + j) {
      const T t = col[k0 + j];
      col[k0 + j] = col[p];
      col[p] = t;
    }
  }
}

// U12 = L11^{-1} A12 for the columns right of panel k0 (KP columns; one
// thread per column)
template <typename T, int KP>
__global__ void __launch_bounds__(kBlk) k_trsm_u12(const LUDesc* __restrict__ descs, int k0, T* __restrict__ base) {
  __shared__ T L11[KP][KP + 1];
  const LUDesc d = descs[blockIdx.y];
  if (k0 >= d.n) return;
  const int nb = min(KP, d.n - k0);
  T* A = base + d.a_off;
  for (int t = threadIdx.x; t < nb * nb; t += kBlk) {
    const int r = t % nb, c = t / nb;
    L11[r][c] = A[(k0 + r) + (int64_t)(k0 + c) * d.lda];
  }
  __syncthreads();
  const int c = k0 + nb + blockIdx.x * kBlk + threadIdx.x;
  if (c >= d.n) return;
  T* col = A + (int64_t)c * d.lda + k0;
  T x[KP];
#pragma unroll
  for (int r = 0; r < KP; ++r) {
    if (r < nb) {
      T s = col[r];
#pragma unroll
      for (int q = 0; q < KP; ++q)
        if (q < r) s -= L11[r][q] * x[q];
      x[r] = s;
      col[r] = s;
    }
  }
}

__global__ void k_scatter_int(int64_t n, const int64_t* __restrict__ sidx, const int64_t* __restrict__ didx,
                              const int* __restrict__ src, int* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[didx[i]] = src[sidx[i]];
}

// ------------------------------------------------------------------ LU solve
// block (blockIdx.x = problem, blockIdx.y = chunk of ``chunk`` columns);
// ncol_override > 0 replaces every problem's column count.  The chunk of B
// is staged in LDS; substitution proceeds by blocks of 16 rows: the
// diagonal block is solved by 16 lanes per column with shuffles, the rest
// of the chunk is updated with one barrier pair per block.
// WIDE: more than 8 columns per workgroup (diagonal blocks in groups of 8).
// Rows of the right-hand sides in pivoted order: the row interchanges of
// the LU (row j with row P[j], j ascending) composed into one permutation in
// LDS by one thread (pivots staged first, so no step waits on memory), then
// X(i, c) = B(perm(i), c) gathered by all threads; columns c >= nc are
// zero.  perm and pv: 2 n ints of LDS.  Without room for them (staged =
// 0: very large single matrices) the interchanges are applied to X in place,
// one thread per column, with the same result.
template <typename T>
__device__ inline void load_permuted(const T* __restrict__ B, int64_t ldb, const int* __restrict__ P, int n, int nc,
                                     int ncols, T* __restrict__ X, int* perm, int* pv, int staged) {
  const int tid = threadIdx.x;
  if (!staged) {
    for (int t = tid; t < n * ncols; t += kBlk) {
      const int i = t % n, c = t / n;
      X[i + c * n] = c < nc ? B[i + (int64_t)c * ldb] : zero<T>();
    }
    __syncthreads();
    if (tid < nc)
      for (int j = 0; j < n; ++j) {
        const int p = P[j];
        if (p != j) {
          const T t = X[j + tid * n];
          X[j + tid * n] = X[p + tid * n];
          X[p + tid * n] = t;
        }
      }
    __syncthreads();
    return;
  }
  for (int t = tid; t < n; t += kBlk) {
    perm[t] = t;
    pv[t] = P[t];
  }
  __syncthreads();
  if (tid == 0)
    for (int j = 0; j < n; ++j) {
      const int p = pv[j];
      if (p != j) {
        const int a = perm[j];
        perm[j] = perm[p];
        perm[p] = a;
      }
    }
  __syncthreads();
  for (int t = tid; t < n * ncols; t += kBlk) {
    const int i = t % n, c = t / n;
    X[i + c * n] = c < nc ? B[perm[i] + (int64_t)c * ldb] : zero<T>();
  }
  __syncthreads();
}

template <typename T, bool WIDE, bool GX = false>
__global__ void __launch_bounds__(kBlk) k_lu_solve(const SolveDesc* __restrict__ descs, int chunk, int ncol_override,
                                                   const T* __restrict__ abase, const int* __restrict__ piv,
                                                   T* __restrict__ bbase, int staged) {
  extern __shared__ unsigned char smem_sv[];
  const SolveDesc d = descs[blockIdx.x];
  const int ncol = ncol_override > 0 ? ncol_override : d.ncol;
  const int c0 = blockIdx.y * chunk;
  if (c0 >= ncol || d.n == 0) return;
  const T* A = abase + d.a_off;
  const int* P = piv + d.piv_off;
  T* B = bbase + d.b_off + (int64_t)c0 * d.ldb;
  const int n = d.n, lda = d.lda, nc = min(chunk, ncol - c0);
  const int tid = threadIdx.x;
  // GX: the columns are solved in place in memory (a block too large for
  // LDS); else staged in LDS
  T* X = GX ? B : reinterpret_cast<T*>(smem_sv);
  const int64_t ldx = GX ? d.ldb : n;
  if (GX) {
    if (tid < nc)
      for (int j = 0; j < n; ++j) {
        const int p = P[j];
        if (p != j) {
          const T t = X[j + tid * ldx];
          X[j + tid * ldx] = X[p + tid * ldx];
          X[p + tid * ldx] = t;
        }
      }
    __syncthreads();
  } else {
    int* perm = reinterpret_cast<int*>(X + (size_t)n * chunk);
    load_permuted(B, d.ldb, P, n, nc, nc, X, perm, perm + n, staged);
  }
  const int cc = tid % nc;
  const int r0 = tid / nc;
  const int rs = kBlk / nc;
  constexpr int SB = 16;   // rows per substitution block
  const int br = tid & 15;            // row within the block
  const int bc = tid >> 4;            // column handled by this lane group
  // forward substitution with unit L
  for (int k0 = 0; k0 < n; k0 += SB) {
    const int nb = min(SB, n - k0);
    for (int cg = 0; cg < (WIDE ? nc : 1) && tid < 8 * 16; cg += 8) {   // two wavefronts, 8 columns at a time
      const int col = cg + bc;
      const bool act = col < nc && br < nb;
      T x = act ? X[k0 + br + col * ldx] : zero<T>();
      T l[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) l[q] = (act && q < br) ? A[(k0 + br) + (int64_t)(k0 + q) * lda] : zero<T>();
#pragma unroll
      for (int q = 0; q < SB - 1; ++q) {
        const T xq = row_bcast(x, q);
        if (br > q) cfms(x, l[q], xq);
      }
      if (act) X[k0 + br + col * ldx] = x;
    }
    __syncthreads();
    if (r0 < rs)
      for (int i = k0 + nb + r0; i < n; i += rs) {
        T s = X[i + cc * ldx];
        if (nb == SB) {   // full block: all loads of the factor in flight at once
          T a[SB];
#pragma unroll
          for (int q = 0; q < SB; ++q) a[q] = A[i + (int64_t)(k0 + q) * lda];
#pragma unroll
          for (int q = 0; q < SB; ++q) cfms(s, a[q], X[k0 + q + cc * ldx]);
        } else {
          for (int q = 0; q < nb; ++q) cfms(s, A[i + (int64_t)(k0 + q) * lda], X[k0 + q + cc * ldx]);
        }
        X[i + cc * ldx] = s;
      }
    __syncthreads();
  }
  // backward substitution with U, from the bottom
  for (int k1 = n; k1 > 0; k1 -= SB) {
    const int k0 = max(0, k1 - SB), nb = k1 - k0;
    for (int cg = 0; cg < (WIDE ? nc : 1) && tid < 8 * 16; cg += 8) {
      const int col = cg + bc;
      const bool act = col < nc && br < nb;
      T x = act ? X[k0 + br + col * ldx] : zero<T>();
      T u[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q)
        u[q] = (act && q >= br && q < nb) ? A[(k0 + br) + (int64_t)(k0 + q) * lda] : zero<T>();
      // u[q] holds U(row, k0 + q) for q >= row; the diagonal sits at u[row]
#pragma unroll
      for (int q = SB - 1; q >= 0; --q) {
        if (act && q < nb && br == q) x = cdiv(x, u[q]);
        const T xq = row_bcast(x, q);
        if (q < nb && br < q) cfms(x, u[q], xq);
      }
      if (act) X[k0 + br + col * ldx] = x;
    }
    __syncthreads();
    if (r0 < rs)
      for (int i = r0; i < k0; i += rs) {
        T s = X[i + cc * ldx];
        if (nb == SB) {
          T a[SB];
#pragma unroll
          for (int q = 0; q < SB; ++q) a[q] = A[i + (int64_t)(k0 + q) * lda];
#pragma unroll
          for (int q = 0; q < SB; ++q) cfms(s, a[q], X[k0 + q + cc * ldx]);
        } else {
          for (int q = 0; q < nb; ++q) cfms(s, A[i + (int64_t)(k0 + q) * lda], X[k0 + q + cc * ldx]);
        }
        X[i + cc * ldx] = s;
      }
    __syncthreads();
  }
  if (!GX)
    for (int t = tid; t < n * nc; t += kBlk) {
      const int i = t % n, c = t / n;
      B[i + (int64_t)c * d.ldb] = X[i + c * n];
    }
}

// Triangular solves with many right-hand sides, NC (16 or 32) columns per
// workgroup.  The diagonal 16 x 16 blocks are solved one column per thread
// with the block staged in LDS; the updates of the other rows are small
// GEMMs, two threads per row each owning NC/2 columns: the row of the factor
// is read once from memory (consecutive threads, consecutive rows) and the
// solved rows are broadcast from LDS.  Every entry sees the same operations
// in the same order as in k_lu_solve (explicit fused multiply-adds), so the
// two kernels give identical results and the chunk width is a pure launch
// choice.
template <typename T, int NC>
__global__ void __launch_bounds__(kBlk) k_lu_solve_wide(const SolveDesc* __restrict__ descs, int ncol_override,
                                                        const T* __restrict__ abase, const int* __restrict__ piv,
                                                        T* __restrict__ bbase, int staged) {
  constexpr int SB = 16, CPT = NC / 2, RPP = kBlk / 2;
  extern __shared__ unsigned char smem_sw[];
  T* X = reinterpret_cast<T*>(smem_sw);   // n x NC, column-major (ld n)
  const SolveDesc d = descs[blockIdx.x];
  const int ncol = ncol_override > 0 ? ncol_override : d.ncol;
  const int c0 = blockIdx.y * NC;
  if (c0 >= ncol || d.n == 0) return;
  const T* A = abase + d.a_off;
  const int* P = piv + d.piv_off;
  T* B = bbase + d.b_off + (int64_t)c0 * d.ldb;
  const int n = d.n, lda = d.lda, nc = min(NC, ncol - c0);
  const int tid = threadIdx.x;
  int* perm = reinterpret_cast<int*>(X + (size_t)n * NC);
  load_permuted(B, d.ldb, P, n, nc, NC, X, perm, perm + n, staged);
  const int tr = tid % RPP, cg = (tid / RPP) * CPT;   // update: row slot, first column
  const int br = tid & 15, bc = tid >> 4;             // diagonal: row in block, column
  // forward substitution with unit L
  for (int k0 = 0; k0 < n; k0 += SB) {
    const int nb = min(SB, n - k0);
    __syncthreads();
    // diagonal block: 16 lanes per column (one row each), 16 columns at a time
    for (int cgd = 0; cgd < nc; cgd += 16) {
      const int col = cgd + bc;
      const bool act = col < nc && br < nb;
      T x = act ? X[k0 + br + col * n] : zero<T>();
      T l[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) l[q] = (act && q < br) ? A[(k0 + br) + (int64_t)(k0 + q) * lda] : zero<T>();
#pragma unroll
      for (int q = 0; q < SB - 1; ++q) {
        const T xq = row_bcast(x, q);
        if (br > q) cfms(x, l[q], xq);
      }
      if (act) X[k0 + br + col * n] = x;
    }
    __syncthreads();
    for (int i = k0 + nb + tr; i < n; i += RPP) {
      T l[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) l[q] = q < nb ? A[i + (int64_t)(k0 + q) * lda] : zero<T>();
      T acc[CPT];
#pragma unroll
      for (int c = 0; c < CPT; ++c) acc[c] = X[i + (cg + c) * n];
#pragma unroll
      for (int q = 0; q < SB; ++q)
        if (q < nb)
#pragma unroll
          for (int c = 0; c < CPT; ++c) cfms(acc[c], l[q], X[k0 + q + (cg + c) * n]);
#pragma unroll
      for (int c = 0; c < CPT; ++c) X[i + (cg + c) * n] = acc[c];
    }
  }
  // backward substitution with U, from the bottom
  for (int k1 = n; k1 > 0; k1 -= SB) {
    const int k0 = max(0, k1 - SB), nb = k1 - k0;
    __syncthreads();
    for (int cgd = 0; cgd < nc; cgd += 16) {
      const int col = cgd + bc;
      const bool act = col < nc && br < nb;
      T x = act ? X[k0 + br + col * n] : zero<T>();
      T u[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q)
        u[q] = (act && q >= br && q < nb) ? A[(k0 + br) + (int64_t)(k0 + q) * lda] : zero<T>();
#pragma unroll
      for (int q = SB - 1; q >= 0; --q) {
        if (act && q < nb && br == q) x = cdiv(x, u[q]);
        const T xq = row_bcast(x, q);
        if (q < nb && br < q) cfms(x, u[q], xq);
      }
      if (act) X[k0 + br + col * n] = x;
    }
    __syncthreads();
    for (int i = tr; i < k0; i += RPP) {
      T u[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) u[q] = q < nb ? A[i + (int64_t)(k0 + q) * lda] : zero<T>();
      T acc[CPT];
#pragma unroll
      for (int c = 0; c < CPT; ++c) acc[c] = X[i + (cg + c) * n];
#pragma unroll
      for (int q = 0; q < SB; ++q)
        if (q < nb)
#pragma unroll
          for (int c = 0; c < CPT; ++c) cfms(acc[c], u[q], X[k0 + q + (cg + c) * n]);
#pragma unroll
      for (int c = 0; c < CPT; ++c) X[i + (cg + c) * n] = acc[c];
    }
  }
  __syncthreads();
  for (int t = tid; t < n * nc; t += kBlk) {
    const int i = t % n, c = t / n;
    B[i + (int64_t)c * d.ldb] = X[i + c * n];
  }
}

// ------------------------------------------------------------------ GEMM
// C = alpha op(A) B + beta C, 64 x 64 output tiles, k-slices of 16 staged in
// LDS, each thread owning a 4 x 4 block of outputs.
// block (blockIdx.x = row tile (problem, tm) from ``tiles``, blockIdx.y = tn);
// n_override > 0 replaces every problem's column count.
// BN: output columns per workgroup (64, or 16 for few right-hand sides);
// the accumulation order over k is the same for both, so the two tile
// shapes give bitwise identical results.
template <int TA, typename T, int BN>
__global__ void __launch_bounds__(kBlk) k_gemm(const GemmDesc* __restrict__ descs, const GemmTile* __restrict__ tiles,
                                               int n_override, const T* __restrict__ abase,
                                               const T* __restrict__ bbase, T* __restrict__ cbase) {
  constexpr int NB = BN / 16;
  __shared__ T As[16][65];
  __shared__ T Bs[16][BN + 1];
  const GemmTile tl = tiles[blockIdx.x];
  GemmDesc d = descs[tl.desc];
  if (n_override > 0) d.n = n_override;
  if ((int)blockIdx.y * BN >= d.n) return;
  const T* A = abase + d.a_off;
  const T* B = bbase + d.b_off;
  T* C = cbase + d.c_off;
  const int m0 = tl.tm * 64, n0 = blockIdx.y * BN;
  const int tid = threadIdx.x;
  const int tr = tid % 16, tc = tid / 16;   // thread owns rows tr + 16 a, cols tc + 16 b
  T acc[4][NB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = zero<T>();
  for (int k0 = 0; k0 < d.k; k0 += 16) {
    // stage op(A)[m0:m0+64, k0:k0+16] and B[k0:k0+16, n0:n0+BN] in one loop
    for (int t = tid; t < 64 * 16; t += kBlk) {
      const int ii = t % 64, kk = t / 64;
      const int gi = m0 + ii, gk = k0 + kk;
      T va = zero<T>();
      if (gi < d.m && gk < d.k) va = TA ? A[gk + (int64_t)gi * d.lda] : A[gi + (int64_t)gk * d.lda];
      As[kk][ii] = va;
      if (t < BN * 16) {
        const int kb = t % 16, jj = t / 16;
        const int gkb = k0 + kb, gj = n0 + jj;
        T vb = zero<T>();
        if (gkb < d.k && gj < d.n) vb = B[gkb + (int64_t)gj * d.ldb];
        Bs[kb][jj] = vb;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      T av[4], bv[NB];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][tr + 16 * a];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = Bs[kk][tc + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) cfma(acc[a][b], av[a], bv[b]);
    }
    __syncthreads();
  }
  const T al = Cx<T>::make(d.alpha_re, d.alpha_im), be = Cx<T>::make(d.beta_re, d.beta_im);
  const bool zero_beta = (d.beta_re == 0.0 && d.beta_im == 0.0);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int gi = m0 + tr + 16 * a, gj = n0 + tc + 16 * b;
      if (gi < d.m && gj < d.n) {
        T* cp = C + gi + (int64_t)gj * d.ldc;
        T v = zero<T>();
        cfma(v, al, acc[a][b]);
        if (!zero_beta) cfma(v, be, *cp);
        *cp = v;
      }
    }
}

// ------------------------------------------------------------------ pivoted QR
constexpr int kQrMaxM = 2048;    // rows with the Householder vector in LDS
constexpr int kQrMaxN = 1024;
constexpr int kQrMaxNTall = 4096;
constexpr int64_t kQrwMinElems = 1 << 16;   // problems this large use the multi-workgroup QR
constexpr int kQrFewProblems = 128;          // launches of at most this many problems: 1024 threads each

// Reflector update of columns cols[0..G) (g < ng valid) of one problem by
// one wavefront: w = tau v^H a, a <- a - v w, and the exact norm of the part
// below row j.  CH > 0: the trailing rows j.. of each column (at most 64 CH
// of them) stay in registers between the two passes; CH = 0: two passes over
// memory.  Per lane the rows are visited in the same order
// either way, and the lane sums are taken together (wsum_rows) in both, so
// the results do not depend on the variant.
template <int G, int CH>
__device__ inline void qr_update_cols(c64* __restrict__ A, int lda, int m, int j, const int (&cols)[G], int ng,
                                      const c64* v, c64 vtop, double tau, int lane, double* __restrict__ nrm) {
  static_assert(G % 4 == 0, "lane sums four rows at a time");
  double dw[2 * G];   // v^H a of column g: real part dw[g], imaginary dw[G + g]
  double sq[G];
#pragma unroll
  for (int g = 0; g < G; ++g) dw[g] = dw[G + g] = sq[g] = 0.0;
  c64 w[G];
  if constexpr (CH > 0) {
    c64 a[G][CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int i = j + lane + 64 * t;
      const bool in = i < m;
      const c64 vv = i == j ? vtop : (in ? v[i] : cmk(0, 0));
#pragma unroll
      for (int g = 0; g < G; ++g) {
        a[g][t] = (in && g < ng) ? A[i + (int64_t)cols[g] * lda] : cmk(0, 0);
        dw[g] += vv.re * a[g][t].re + vv.im * a[g][t].im;   // conj(v) a
        dw[G + g] += vv.re * a[g][t].im - vv.im * a[g][t].re;
      }
    }
    wsum_rows<2 * G>(dw);
#pragma unroll
    for (int g = 0; g < G; ++g) w[g] = cmk(tau * wsum_rows_get(dw, g), tau * wsum_rows_get(dw, G + g));
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int i = j + lane + 64 * t;
      if (i >= m) continue;
      const c64 vv = i == j ? vtop : v[i];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g >= ng) continue;
        const c64 x = a[g][t] - vv * w[g];
        A[i + (int64_t)cols[g] * lda] = x;
        if (i > j) sq[g] += abs2(x);
      }
    }
  } else {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (g >= ng) continue;
      const c64* col = A + (int64_t)cols[g] * lda;
      for (int i = j + lane; i < m; i += 64) {
        const c64 x = col[i], vv = i == j ? vtop : v[i];
        dw[g] += vv.re * x.re + vv.im * x.im;
        dw[G + g] += vv.re * x.im - vv.im * x.re;
      }
    }
    wsum_rows<2 * G>(dw);
#pragma unroll
    for (int g = 0; g < G; ++g) w[g] = cmk(tau * wsum_rows_get(dw, g), tau * wsum_rows_get(dw, G + g));
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (g >= ng) continue;
      c64* col = A + (int64_t)cols[g] * lda;
      for (int i = j + lane; i < m; i += 64) {
        const c64 x = col[i] - (i == j ? vtop : v[i]) * w[g];
        col[i] = x;
        if (i > j) sq[g] += abs2(x);
      }
    }
  }
  // lane 16 r writes the norms of columns r G/4 ..
  wsum_rows<G>(sq);
  if ((lane & 15) == 0) {
#pragma unroll
    for (int k = 0; k < G / 4; ++k) {
      const int g = k + (lane >> 4) * (G / 4);
      if (g < ng) nrm[cols[g]] = sq[k];
    }
  }
}


// TALL = false: the Householder vector is staged in LDS (m <= kQrMaxM,
// n <= kQrMaxN).  TALL = true: any m, n <= kQrMaxNTall; the vector is read
// in place from column j (its entries below the diagonal are the column's
// own), its top entry kept in LDS, and the column cleared after the update.
// Per step: pivot search by wavefront reductions (two barriers), column
// swap, reflector (one wavefront), and the update of the trailing columns,
// four at a time per wavefront.
template <bool TALL, int TB>
__global__ void __launch_bounds__(TB) k_cpqr(const CpqrDesc* __restrict__ descs, c64* __restrict__ base,
                                               int* __restrict__ piv, double tol, int* __restrict__ rank) {
  constexpr int NMAX = TALL ? kQrMaxNTall : kQrMaxN;
  constexpr int NW = TB / 64;
  constexpr int G = 4;
  __shared__ double nrm[NMAX];
  __shared__ int pv[NMAX];
  __shared__ c64 v_lds[TALL ? 1 : kQrMaxM];
  __shared__ c64 s_vtop;
  __shared__ double s_max[NW], s_tau;
  __shared__ int s_org[NW], s_col[NW];
  const CpqrDesc d = descs[blockIdx.x];
  c64* A = base + d.a_off;
  int* P = piv + d.piv_off;
  const int m = d.m, n = d.n, lda = d.lda;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int kmax = min(d.k_end, min(m, n));
  for (int c = tid; c < n; c += TB) pv[c] = d.k_start == 0 ? c : P[c];
  // exactly computed norms of the remaining part of each column
  for (int c = d.k_start + wid; c < n; c += NW) {
    double s = 0.0;
    for (int i = d.k_start + lane; i < m; i += 64) s += abs2(A[i + (int64_t)c * lda]);
    s = wsum_full(s);
    if (lane == 0) nrm[c] = s;
  }
  double r00 = d.k_start > 0 ? sqrt(abs2(A[0])) : 0.0;
  __syncthreads();
  int j = d.k_start;
  for (; j < kmax; ++j) {
    // pivot: largest norm; ties within a relative 1e-12 -> lowest original column
    double best = -1.0;
    for (int c = j + tid; c < n; c += TB) best = fmax(best, nrm[c]);
    best = wmax_full(best);
    if (lane == 0) s_max[wid] = best;
    __syncthreads();
    double top = s_max[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) top = fmax(top, s_max[w]);
    int bo = 0x7fffffff, bc = -1;
    for (int c = j + tid; c < n; c += TB)
      if (nrm[c] >= top * (1.0 - 1e-12) && pv[c] < bo) {
        bo = pv[c];
        bc = c;
      }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int ob = __shfl_xor(bo, o), oc = __shfl_xor(bc, o);
      if (ob < bo) {
        bo = ob;
        bc = oc;
      }
    }
    if (lane == 0) {
      s_org[wid] = bo;
      s_col[wid] = bc;
    }
    __syncthreads();
    int p = s_col[0], po = s_org[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
      if (s_org[w] < po) {
        po = s_org[w];
        p = s_col[w];
      }
    // every thread takes the same stopping decision from the same values
    const double rjj = sqrt(nrm[p]);
    if (j == 0) r00 = rjj;
    if (rjj == 0.0 || (d.stop_at_tol && j > 0 && rjj <= tol * r00)) break;
    if (p != j) {
      for (int i = tid; i < m; i += TB) {
        const c64 t = A[i + (int64_t)j * lda];
        A[i + (int64_t)j * lda] = A[i + (int64_t)p * lda];
        A[i + (int64_t)p * lda] = t;
      }
    }
    __syncthreads();
    if (p != j && tid == 0) {
      const double t = nrm[j];
      nrm[j] = nrm[p];
      nrm[p] = t;
      const int q = pv[j];
      pv[j] = pv[p];
      pv[p] = q;
    }
    // Householder reflector H = I - tau v v^H with H x = alpha e1 (one wavefront)
    c64* colj = A + (int64_t)j * lda;
    const c64* v = TALL ? colj : v_lds;   // v[i] for i > j; v[j] is s_vtop
    if (wid == 0) {
      double s = 0.0;
      for (int i = j + lane; i < m; i += 64) {
        const c64 x = colj[i];
        if (!TALL) v_lds[i] = x;
        s += abs2(x);
      }
      s = wsum_full(s);
      if (lane == 0) {
        const double xn = sqrt(s);
        const c64 x0 = colj[j];
        const double ax0 = sqrt(abs2(x0));
        const c64 ph = ax0 > 0.0 ? cmk(x0.re / ax0, x0.im / ax0) : cmk(1.0, 0.0);
        const c64 alpha = (-xn) * ph;
        s_vtop = x0 - alpha;
        const double vn2 = 2.0 * s + 2.0 * ax0 * xn;
        s_tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
        colj[j] = alpha;
      }
    }
    __syncthreads();
    if (!TALL)
      for (int i = j + 1 + tid; i < m; i += TB) colj[i] = cmk(0, 0);
    const double tau = s_tau;
    const c64 vtop = s_vtop;
    const int rows = m - j;
    for (int c0 = j + 1 + wid * G; c0 < n; c0 += NW * G) {
      int cols[G];
#pragma unroll
      for (int g = 0; g < G; ++g) cols[g] = c0 + g;
      const int ng = min(G, n - c0);
      if (rows <= 64)
        qr_update_cols<G, 1>(A, lda, m, j, cols, ng, v, vtop, tau, lane, nrm);
      else if (rows <= 128)
        qr_update_cols<G, 2>(A, lda, m, j, cols, ng, v, vtop, tau, lane, nrm);
      else if (rows <= 256)
        qr_update_cols<G, 4>(A, lda, m, j, cols, ng, v, vtop, tau, lane, nrm);
      else
        qr_update_cols<G, 0>(A, lda, m, j, cols, ng, v, vtop, tau, lane, nrm);
    }
    __syncthreads();
    if (TALL) {
      for (int i = j + 1 + tid; i < m; i += TB) colj[i] = cmk(0, 0);
      __syncthreads();
    }
  }
  __syncthreads();
  for (int c = tid; c < n; c += TB) P[c] = pv[c];
  if (tid == 0) rank[blockIdx.x] = j;
}


// Register-resident pivoted QR for small problems (m <= 64 CH rows, n <= 8 NS
// columns), same pivot and stopping rules as k_cpqr.  Eight wavefronts;
// column c lives in wavefront c % 8, register slot c / 8, lane l holding
// rows l + 64 t.  The matrix is read once and written back once; a step
// touches only registers and LDS: every wavefront picks the pivot from the
// norms in LDS, the two owners swap columns through LDS, the owner of
// column j forms the reflector into LDS, and every wavefront updates its
// columns.
constexpr int kQrRegWaves = 8;
constexpr int kQrRegRows = 256;
constexpr int kQrRegCols = 64;

template <int NS, int CH>
__global__ void __launch_bounds__(64 * kQrRegWaves) k_cpqr_reg(const CpqrDesc* __restrict__ descs,
                                                              c64* __restrict__ base, int* __restrict__ piv, double tol,
                                                              int* __restrict__ rank) {
  constexpr int NW = kQrRegWaves;
  constexpr int NC = NW * NS;
  constexpr int MR = 64 * CH;
  static_assert(NC <= 64, "pivot keys hold the column in 6 bits");
  __shared__ double nrm[NC];
  __shared__ int pv[NC];
  __shared__ c64 vbuf[MR];
  __shared__ c64 xbuf[2][MR];
  __shared__ double s_tau;
  const CpqrDesc d = descs[blockIdx.x];
  c64* A = base + d.a_off;
  int* P = piv + d.piv_off;
  const int m = d.m, n = d.n, lda = d.lda;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int kmax = min(d.k_end, min(m, n));
  c64 a[NS][CH];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = sl * NW + wid;
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int i = lane + 64 * t;
      a[sl][t] = (c < n && i < m) ? A[i + (int64_t)c * lda] : cmk(0, 0);
    }
  }
  for (int c = tid; c < n; c += 64 * NW) pv[c] = d.k_start == 0 ? c : P[c];
  {
    double sq[NS];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      sq[sl] = 0.0;
#pragma unroll
      for (int t = 0; t < CH; ++t)
        if (lane + 64 * t >= d.k_start) sq[sl] += abs2(a[sl][t]);
      sq[sl] = wsum_full(sq[sl]);
    }
    if (lane == 0) {
#pragma unroll
      for (int sl = 0; sl < NS; ++sl)
        if (sl * NW + wid < n) nrm[sl * NW + wid] = sq[sl];
    }
  }
  double r00 = d.k_start > 0 ? sqrt(abs2(A[0])) : 0.0;
  __syncthreads();
  int j = d.k_start;
  for (; j < kmax; ++j) {
    // pivot, found by every wavefront from the same LDS values: largest
    // norm; ties within a relative 1e-12 -> lowest original column
    const int cc = j + lane;
    const double nv = cc < n ? nrm[cc] : -1.0;
    const double top = wmax_full(nv);
    const int key = (cc < n && nv >= top * (1.0 - 1e-12)) ? pv[cc] * 64 + cc : 0x7fffffff;
    const int p = wmin_int_full(key) & 63;
    const double rjj = sqrt(nrm[p]);
    if (j == 0) r00 = rjj;
    if (rjj == 0.0 || (d.stop_at_tol && j > 0 && rjj <= tol * r00)) break;
    const int wj = j % NW, sj = j / NW;
    if (p != j) {
      const int wp = p % NW, sp = p / NW;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        if (wid == wj && sl == sj)
#pragma unroll
          for (int t = 0; t < CH; ++t) xbuf[0][lane + 64 * t] = a[sl][t];
        if (wid == wp && sl == sp)
#pragma unroll
          for (int t = 0; t < CH; ++t) xbuf[1][lane + 64 * t] = a[sl][t];
      }
      __syncthreads();
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        if (wid == wj && sl == sj)
#pragma unroll
          for (int t = 0; t < CH; ++t) a[sl][t] = xbuf[1][lane + 64 * t];
        if (wid == wp && sl == sp)
#pragma unroll
          for (int t = 0; t < CH; ++t) a[sl][t] = xbuf[0][lane + 64 * t];
      }
      if (tid == 0) {
        const double tn = nrm[j];
        nrm[j] = nrm[p];
        nrm[p] = tn;
        const int q = pv[j];
        pv[j] = pv[p];
        pv[p] = q;
      }
    }
    // Householder reflector H = I - tau v v^H with H x = alpha e1, formed by
    // the owner of column j: v (rows < j zero, row j its top entry) to LDS
    if (wid == wj) {
      c64 x[CH];
#pragma unroll
      for (int t = 0; t < CH; ++t) x[t] = cmk(0, 0);
#pragma unroll
      for (int sl = 0; sl < NS; ++sl)
        if (sl == sj)
#pragma unroll
          for (int t = 0; t < CH; ++t) x[t] = a[sl][t];
      double ss = 0.0;
      c64 xt = cmk(0, 0);
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int i = lane + 64 * t;
        if (i >= j) ss += abs2(x[t]);
        if (t == j / 64) xt = x[t];
      }
      ss = wsum_full(ss);
      const int jl = j % 64;
      const c64 x0 = cmk(lane_value(xt.re, jl), lane_value(xt.im, jl));
      const double xn = sqrt(ss);
      const double ax0 = sqrt(abs2(x0));
      const c64 ph = ax0 > 0.0 ? cmk(x0.re / ax0, x0.im / ax0) : cmk(1.0, 0.0);
      const c64 alpha = (-xn) * ph;
      const c64 vtop = x0 - alpha;
      const double vn2 = 2.0 * ss + 2.0 * ax0 * xn;
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int i = lane + 64 * t;
        vbuf[i] = (i < j || i >= m) ? cmk(0, 0) : (i == j ? vtop : x[t]);
      }
#pragma unroll
      for (int sl = 0; sl < NS; ++sl)
        if (sl == sj)
#pragma unroll
          for (int t = 0; t < CH; ++t) {
            const int i = lane + 64 * t;
            if (i == j) a[sl][t] = alpha;
            else if (i > j) a[sl][t] = cmk(0, 0);
          }
      if (lane == 0) s_tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    }
    __syncthreads();
    const double tau = s_tau;
    c64 vv[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) vv[t] = vbuf[lane + 64 * t];
    // w = v^H a of every slot (real parts in dw[sl], imaginary in dw[NS + sl]),
    // summed over the lanes together
    double dw[2 * NS];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      dw[sl] = dw[NS + sl] = 0.0;
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        dw[sl] += vv[t].re * a[sl][t].re + vv[t].im * a[sl][t].im;   // conj(v) a
        dw[NS + sl] += vv[t].re * a[sl][t].im - vv[t].im * a[sl][t].re;
      }
    }
    wsum_rows<2 * NS>(dw);
    c64 w[NS];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) w[sl] = cmk(tau * wsum_rows_get(dw, sl), tau * wsum_rows_get(dw, NS + sl));
    double sq[NS];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      sq[sl] = 0.0;
      const int c = sl * NW + wid;
      if (c > j && c < n) {
#pragma unroll
        for (int t = 0; t < CH; ++t) {
          a[sl][t] = a[sl][t] - vv[t] * w[sl];
          if (lane + 64 * t > j) sq[sl] += abs2(a[sl][t]);
        }
      }
    }
    // the slots' remaining norms: lane 16 r writes those of slots r NS/4 ..
    wsum_rows<NS>(sq);
    if ((lane & 15) == 0) {
#pragma unroll
      for (int k = 0; k < NS / 4; ++k) {
        const int c = (k + (lane >> 4) * (NS / 4)) * NW + wid;
        if (c > j && c < n) nrm[c] = sq[k];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = sl * NW + wid;
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int i = lane + 64 * t;
      if (c < n && i < m) A[i + (int64_t)c * lda] = a[sl][t];
    }
  }
  __syncthreads();
  for (int c = tid; c < n; c += 64 * NW) P[c] = pv[c];
  if (tid == 0) rank[blockIdx.x] = j;
}

// Multi-workgroup pivoted QR for large problems (same pivot and stopping
// rules as k_cpqr): a host loop over steps j launches k_qrw_pivot (one
// workgroup per problem: clear the previous reflector's column, choose the
// pivot, swap, form the reflector in place) and k_qrw_update (problem x
// column chunks: apply the reflector, recompute the exact remaining norms).
struct QrwState {
  double r00, tau;
  c64 vtop;
  int stop, rank;
};

constexpr int kQrwCols = 16;   // columns per workgroup of k_qrw_update (4 per wavefront)

__global__ void k_qrw_init(const CpqrDesc* __restrict__ descs, c64* __restrict__ base, int* __restrict__ piv,
                           double* __restrict__ nrm, QrwState* __restrict__ st) {
  const CpqrDesc d = descs[blockIdx.y];
  const c64* A = base + d.a_off;
  int* P = piv + d.piv_off;
  double* N = nrm + d.piv_off;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = blockIdx.x * kQrwCols + wid; c < min(d.n, (int)(blockIdx.x + 1) * kQrwCols); c += blockDim.x / 64) {
    if (lane == 0 && d.k_start == 0) P[c] = c;
    if (c < d.k_start) continue;
    double s = 0.0;
    for (int i = d.k_start + lane; i < d.m; i += 64) s += abs2(A[i + (int64_t)c * d.lda]);
    s = wsum(s);
    if (lane == 0) N[c] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    QrwState q{};
    q.r00 = d.k_start > 0 ? sqrt(abs2(A[0])) : 0.0;
    q.stop = 0;
    q.rank = d.k_start;
    st[blockIdx.y] = q;
  }
}

__global__ void __launch_bounds__(kBlk) k_qrw_pivot(const CpqrDesc* __restrict__ descs, int j, c64* __restrict__ base,
                                                    int* __restrict__ piv, double* __restrict__ nrm,
                                                    QrwState* __restrict__ st, double tol) {
  __shared__ double sv[kBlk];
  __shared__ int si[kBlk];
  __shared__ int s_p, s_stop;
  const CpqrDesc d = descs[blockIdx.x];
  if (j < d.k_start || st[blockIdx.x].stop) return;
  c64* A = base + d.a_off;
  int* P = piv + d.piv_off;
  double* N = nrm + d.piv_off;
  const int m = d.m, n = d.n, lda = d.lda;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int kmax = min(d.k_end, min(m, n));
  // the previous step's reflector is no longer needed: clear it
  if (j > d.k_start)
    for (int i = j + tid; i < m; i += kBlk) A[i + (int64_t)(j - 1) * lda] = cmk(0.0, 0.0);
  if (j >= kmax) {
    if (tid == 0) {
      st[blockIdx.x].stop = 1;
      st[blockIdx.x].rank = j;
    }
    return;
  }
  double best = -1.0;
  for (int c = j + tid; c < n; c += kBlk) best = fmax(best, N[c]);
  sv[tid] = best;
  __syncthreads();
  for (int o = kBlk / 2; o > 0; o >>= 1) {
    if (tid < o) sv[tid] = fmax(sv[tid], sv[tid + o]);
    __syncthreads();
  }
  const double top = sv[0];
  __syncthreads();
  int bo = 0x7fffffff, bc = -1;
  for (int c = j + tid; c < n; c += kBlk)
    if (N[c] >= top * (1.0 - 1e-12) && P[c] < bo) {
      bo = P[c];
      bc = c;
    }
  si[tid] = bo;
  sv[tid] = (double)bc;
  __syncthreads();
  for (int o = kBlk / 2; o > 0; o >>= 1) {
    if (tid < o && si[tid + o] < si[tid]) {
      si[tid] = si[tid + o];
      sv[tid] = sv[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int p = (int)sv[0];
    const double rjj = sqrt(N[p]);
    QrwState q = st[blockIdx.x];
    if (j == 0) q.r00 = rjj;
    s_stop = (rjj == 0.0 || (d.stop_at_tol && j > 0 && rjj <= tol * q.r00)) ? 1 : 0;
    if (s_stop) {
      q.stop = 1;
      q.rank = j;
    }
    st[blockIdx.x] = q;
    s_p = p;
  }
  __syncthreads();
  if (s_stop) return;
  const int p = s_p;
  if (p != j) {
    for (int i = tid; i < m; i += kBlk) {
      const c64 t = A[i + (int64_t)j * lda];
      A[i + (int64_t)j * lda] = A[i + (int64_t)p * lda];
      A[i + (int64_t)p * lda] = t;
    }
    if (tid == 0) {
      const double t = N[j];
      N[j] = N[p];
      N[p] = t;
      const int q = P[j];
      P[j] = P[p];
      P[p] = q;
    }
  }
  __syncthreads();
  c64* colj = A + (int64_t)j * lda;
  double s = 0.0;
  for (int i = j + tid; i < m; i += kBlk) s += abs2(colj[i]);
  s = wsum(s);
  if (lane == 0) sv[wid] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlk / 64; ++w) t += sv[w];
    const double xn = sqrt(t);
    const c64 x0 = colj[j];
    const double ax0 = sqrt(abs2(x0));
    const c64 ph = ax0 > 0.0 ? cmk(x0.re / ax0, x0.im / ax0) : cmk(1.0, 0.0);
    const c64 alpha = (-xn) * ph;
    const double vn2 = 2.0 * t + 2.0 * ax0 * xn;
    st[blockIdx.x].vtop = x0 - alpha;
    st[blockIdx.x].tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    colj[j] = alpha;
  }
}

// NR > 0: the workgroup takes the chunk's columns one at a time, rows
// j..m-1 held in NR registers per thread (m - j <= 256 NR), so each column is
// read once; NR = 0: one wavefront per column, two passes over memory.
template <int NR>
__global__ void __launch_bounds__(kBlk) k_qrw_update(const CpqrDesc* __restrict__ descs, int j,
                                                     c64* __restrict__ base, double* __restrict__ nrm,
                                                     const QrwState* __restrict__ st) {
  __shared__ double red[3][kBlk / 64];
  const CpqrDesc d = descs[blockIdx.y];
  const QrwState q = st[blockIdx.y];
  if (j < d.k_start || q.stop) return;
  c64* A = base + d.a_off;
  double* N = nrm + d.piv_off;
  const int m = d.m, lda = d.lda;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const c64* v = A + (int64_t)j * lda;
  const int c_lo = j + 1 + (int)blockIdx.x * kQrwCols, c_hi = min(d.n, c_lo + kQrwCols);
  if (NR > 0 && m - j <= kBlk * NR) {
    c64 vr[NR > 0 ? NR : 1];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = j + tid + kBlk * r;
      vr[r] = i < m ? (i == j ? q.vtop : v[i]) : cmk(0.0, 0.0);
    }
    for (int c = c_lo; c < c_hi; ++c) {
      c64* col = A + (int64_t)c * lda;
      c64 a[NR > 0 ? NR : 1];
      double wr = 0.0, wi = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int i = j + tid + kBlk * r;
        a[r] = i < m ? col[i] : cmk(0.0, 0.0);
        wr += vr[r].re * a[r].re + vr[r].im * a[r].im;
        wi += vr[r].re * a[r].im - vr[r].im * a[r].re;
      }
      wr = wsum(wr);
      wi = wsum(wi);
      if (lane == 0) {
        red[0][wid] = wr;
        red[1][wid] = wi;
      }
      __syncthreads();
      wr = red[0][0] + red[0][1] + red[0][2] + red[0][3];
      wi = red[1][0] + red[1][1] + red[1][2] + red[1][3];
      const c64 w = cmk(q.tau * wr, q.tau * wi);
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int i = j + tid + kBlk * r;
        if (i < m) {
          const c64 b = a[r] - vr[r] * w;
          col[i] = b;
          if (i > j) s += abs2(b);
        }
      }
      s = wsum(s);
      if (lane == 0) red[2][wid] = s;
      __syncthreads();
      if (tid == 0) N[c] = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    }
    return;
  }
  for (int c = c_lo + wid; c < c_hi; c += kBlk / 64) {
    c64* col = A + (int64_t)c * lda;
    double wr = 0.0, wi = 0.0;
    for (int i = j + lane; i < m; i += 64) {
      const c64 a = col[i], vv = i == j ? q.vtop : v[i];
      wr += vv.re * a.re + vv.im * a.im;
      wi += vv.re * a.im - vv.im * a.re;
    }
    wr = wsum(wr);
    wi = wsum(wi);
    const c64 w = cmk(q.tau * wr, q.tau * wi);
    double s = 0.0;
    for (int i = j + lane; i < m; i += 64) {
      const c64 a = col[i] - (i == j ? q.vtop : v[i]) * w;
      col[i] = a;
      if (i > j) s += abs2(a);
    }
    s = wsum(s);
    if (lane == 0) N[c] = s;
  }
}

__global__ void k_qrw_rank(int n, const QrwState* __restrict__ st, const int* __restrict__ idx, int* __restrict__ rank) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rank[idx[i]] = st[i].rank;
}

// W = [I, R1^{-1} R2] P^T: solve R1 T = R2 in place (unless already solved),
// then write W or W^T.
// Grid: (problem, chunk of kInterpCols columns of W).
constexpr int kInterpCols = 64;
constexpr int kInterpSmallK = 64;   // k_interp_small: ranks up to this

// Back substitution one column per thread (any rank), R1 read from memory.
__device__ inline void interp_solve_columns(c64* __restrict__ A, int lda, int k, int c_lo, int c_hi, int tid,
                                            int nthreads) {
  for (int c = max(k, c_lo) + tid; c < c_hi; c += nthreads) {
    c64* col = A + (int64_t)c * lda;
    for (int i = k - 1; i >= 0; --i) {
      c64 s = col[i];
      for (int l = i + 1; l < k; ++l) s -= A[i + (int64_t)l * lda] * col[l];
      col[i] = cdiv(s, A[i + (int64_t)i * lda]);
    }
  }
}

__device__ inline void interp_write(const InterpDesc& d, const c64* __restrict__ A, const int* __restrict__ P,
                                    c64* __restrict__ D, int c_lo, int c_hi, int tid, int nthreads) {
  const int k = d.k;
  for (int t = tid; t < k * (c_hi - c_lo); t += nthreads) {
    const int r = t % k, c = c_lo + t / k;     // W(r, P[c])
    c64 val;
    if (c < k)
      val = (r == c) ? cmk(1.0, 0.0) : cmk(0.0, 0.0);
    else
      val = A[r + (int64_t)c * d.lda];
    const int cc = P[c];
    if (d.transpose)
      D[cc + (int64_t)r * d.d_ld] = val;
    else
      D[r + (int64_t)cc * d.d_ld] = val;
  }
}

__global__ void __launch_bounds__(kBlk) k_interp(const InterpDesc* __restrict__ descs, c64* __restrict__ abase,
                                                 const int* __restrict__ piv, c64* __restrict__ dbase) {
  const InterpDesc d = descs[blockIdx.x];
  const int c_lo = blockIdx.y * kInterpCols;
  if (c_lo >= d.n) return;
  const int c_hi = min(d.n, c_lo + kInterpCols);
  c64* A = abase + d.a_off;
  if (!d.solved) interp_solve_columns(A, d.lda, d.k, c_lo, c_hi, threadIdx.x, kBlk);
  __syncthreads();
  interp_write(d, A, piv + d.piv_off, dbase + d.d_off, c_lo, c_hi, threadIdx.x, kBlk);
}

// Ranks up to kInterpSmallK: R1 staged in LDS, the chunk's columns of R2 in
// registers (lane = column, wavefront w holding rows w, w + 4, ...), and the
// back substitution taken four rows at a time: the group's current rows go
// through LDS, every thread finishes them for its column with the group's
// 4 x 4 triangle, the wavefront owning each row stores it, and the rows
// above are updated in registers.  A rank above the limit takes the
// column-per-thread loop.
__global__ void __launch_bounds__(256) k_interp_small(const InterpDesc* __restrict__ descs,
                                                      c64* __restrict__ abase, const int* __restrict__ piv,
                                                      c64* __restrict__ dbase) {
  constexpr int KS = kInterpSmallK, NS = KS / 4;
  static_assert(kInterpCols == 64, "one column per lane");
  __shared__ c64 r1[KS * KS];   // R1, column-major with leading dimension KS
  __shared__ c64 grp[4][kInterpCols];
  const InterpDesc d = descs[blockIdx.x];
  const int c_lo = blockIdx.y * kInterpCols;
  if (c_lo >= d.n) return;
  const int c_hi = min(d.n, c_lo + kInterpCols);
  c64* A = abase + d.a_off;
  const int lda = d.lda, k = d.k;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c0 = max(k, c_lo);
  if (!d.solved && k > KS) {
    interp_solve_columns(A, lda, k, c_lo, c_hi, tid, 256);
  } else if (!d.solved && c0 < c_hi) {
    for (int t = tid; t < k * k; t += 256) {
      const int i = t % k, l = t / k;
      r1[i + KS * l] = A[i + (int64_t)l * lda];
    }
    const int c = c0 + lane;
    const bool act = c < c_hi;
    c64 x[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = w + 4 * s;
      x[s] = (act && i < k) ? A[i + (int64_t)c * lda] : cmk(0, 0);
    }
    __syncthreads();
    for (int g = (k + 3) / 4 - 1; g >= 0; --g) {
      // rows 4 g .. 4 g + 3 as they stand (row 4 g + w from wavefront w)
      c64 xg = x[0];
#pragma unroll
      for (int s = 1; s < NS; ++s)
        if (s == g) xg = x[s];
      grp[w][lane] = xg;
      __syncthreads();
      c64 t[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) t[q] = grp[q][lane];
#pragma unroll
      for (int q = 3; q >= 0; --q) {
        const int l = 4 * g + q;
        if (l < k) {
          c64 sv = t[q];
#pragma unroll
          for (int p = q + 1; p < 4; ++p)
            if (4 * g + p < k) sv -= r1[l + KS * (4 * g + p)] * t[p];
          t[q] = cdiv(sv, r1[l + KS * l]);
        } else {
          t[q] = cmk(0, 0);
        }
      }
      c64 tw = t[0];
#pragma unroll
      for (int q = 1; q < 4; ++q)
        if (q == w) tw = t[q];
      if (act && 4 * g + w < k) A[(4 * g + w) + (int64_t)c * lda] = tw;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s < g) {
          const int i = w + 4 * s;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (4 * g + q < k) x[s] -= r1[i + KS * (4 * g + q)] * t[q];
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  interp_write(d, A, piv + d.piv_off, dbase + d.d_off, c_lo, c_hi, tid, 256);
}

// ------------------------------------------------------------------ scatter / copies
// Block scatter with an optional type conversion (FP32 A~ into FP64 blocks and back).
template <typename TS, typename TD>
__global__ void k_scatter(const ScatterDesc* __restrict__ descs, const ScatterTile* __restrict__ tiles,
                          const int* __restrict__ pos, const TS* __restrict__ src, TD* __restrict__ dst) {
  const ScatterTile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count) return;
  const ScatterDesc d = descs[t.desc];
  const int64_t e = t.start + threadIdx.x;
  const int r = (int)(e % d.nr), c = (int)(e / d.nr);
  const int64_t rp = d.rpos_off >= 0 ? pos[d.rpos_off + r] : r;
  const int64_t cp = d.cpos_off >= 0 ? pos[d.cpos_off + c] : c;
  dst[d.dst_off + rp + cp * d.dst_ld] = cvt<TD>(src[d.src_off + r + (int64_t)c * d.src_ld]);
}

template <typename T>
__global__ void k_copy_rows(int64_t n, const int64_t* __restrict__ sidx, const int64_t* __restrict__ didx, int ncol,
                            const T* __restrict__ src, int64_t lds, T* __restrict__ dst, int64_t ldd) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || c >= ncol) return;
  dst[didx[i] + (int64_t)c * ldd] = src[sidx[i] + (int64_t)c * lds];
}

__global__ void k_axpby(int64_t n, double alpha, const c64* __restrict__ src, double beta, c64* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  dst[i] = alpha * src[i] + beta * dst[i];
}

// dst = convert(src) (contiguous)
template <typename TS, typename TD>
__global__ void k_convert(int64_t n, const TS* __restrict__ src, TD* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  dst[i] = cvt<TD>(src[i]);
}

// dst += (double) src
__global__ void k_add_c32(int64_t n, const c32* __restrict__ src, c64* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  dst[i] += cvt<c64>(src[i]);
}

// out[c] = sum_i |src[i + c ld]|^2 in FP64, one block per column
template <typename T>
__global__ void __launch_bounds__(kBlk) k_colnorm2(int64_t n, const T* __restrict__ src, int64_t ld,
                                                   double* __restrict__ out) {
  __shared__ double part[kBlk / 64];
  const T* p = src + (int64_t)blockIdx.x * ld;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBlk) {
    const double re = (double)p[i].re, im = (double)p[i].im;
    s += re * re + im * im;
  }
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlk / 64; ++w) t += part[w];
    out[blockIdx.x] = t;
  }
}

template <typename T>
__global__ void k_fill_identity(const int64_t* __restrict__ offs, const int* __restrict__ ns, const int* __restrict__ lds,
                                T* __restrict__ base) {
  const int p = blockIdx.x;
  const int n = ns[p], ld = lds[p];
  T* A = base + offs[p];
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t % n, c = t / n;
    A[i + (int64_t)c * ld] = Cx<T>::make(i == c ? 1.0 : 0.0, 0.0);
  }
}

// flag[0] = 1 when any of info[0..n) is nonzero (every writer stores the same value)
__global__ void k_flag_nonzero(int64_t n, const int* __restrict__ info, int* __restrict__ flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (info[i] != 0) flag[0] = 1;
}

// ------------------------------------------------------------------ launchers
// All launchers are asynchronous on ``s``: descriptor arrays are device
// pointers owned by the caller (workspace or factor storage).
// LDS a workgroup may take on the current device (queried once per device)
static size_t max_lds_bytes() {
  static std::mutex mu;
  static std::map<int, size_t> cache;
  int dev = 0;
  FDS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  FDS_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // the kernels' static LDS (a few hundred bytes) comes on top
  const size_t b = v > 4096 ? (size_t)v - 4096 : 0;
  cache[dev] = b;
  return b;
}

template <typename T>
void launch_lu(const LUDesc* d, int n, int nmax, T* base, int* piv, int* info, hipStream_t s) {
  if (n == 0) return;
  // panel of NB columns staged in LDS: nmax * NB * sizeof(T) <= 48 KiB
  const size_t row = (size_t)std::max(1, nmax) * sizeof(T);
  const bool wide = n >= 16 && n < 256 && nmax > 96;
  if (row * 16 <= 49152) {
    if (wide)
      k_lu_blk<16, T, 1024><<<n, 1024, row * 16, s>>>(d, base, piv, info);
    else
      k_lu_blk<16, T, kBlk><<<n, kBlk, row * 16, s>>>(d, base, piv, info);
  } else if (row * 8 <= 49152) {
    if (wide)
      k_lu_blk<8, T, 1024><<<n, 1024, row * 8, s>>>(d, base, piv, info);
    else
      k_lu_blk<8, T, kBlk><<<n, kBlk, row * 8, s>>>(d, base, piv, info);
  } else if (row * 4 <= 49152)
    k_lu_blk<4, T, kBlk><<<n, kBlk, row * 4, s>>>(d, base, piv, info);
  else
    k_lu<T><<<n, kBlk, 0, s>>>(d, base, piv, info);
  FDS_HIP(hipGetLastError());
}

template <typename T>
void lu_factor(const std::vector<LUDesc>& d, T* base, int* piv, int* info, Workspace& ws, const std::string& tag,
               hipStream_t s) {
  if (d.empty()) return;
  // matrices whose 8-column LDS panel fits go to the one-workgroup kernels;
  // larger ones are few per level and get the multi-workgroup form, and so
  // do the matrices above 128 of a batch of at most 8 (the root, the top
  // levels), where one workgroup per matrix would leave the chip idle
  std::vector<LUDesc> small, big;
  std::vector<int> small_i, big_i;
  int nsmall = 0, nbig = 0;
  const bool few = d.size() <= 8;
  for (int i = 0; i < (int)d.size(); ++i) {
    if ((size_t)d[i].n * sizeof(T) * 8 <= 49152 && !(few && d[i].n > 128)) {
      small.push_back(d[i]);
      small_i.push_back(i);
      nsmall = std::max(nsmall, d[i].n);
    } else {
      big.push_back(d[i]);
      big_i.push_back(i);
      nbig = std::max(nbig, d[i].n);
    }
  }
  if (big.empty()) {
    launch_lu(ws.upload(tag + "_d", d), (int)d.size(), nsmall, base, piv, info, s);
    return;
  }
  // info slots follow the caller's order: small matrices first report into
  // a scratch array, then everything is scattered back by index
  int* inf_s = ws.get<int>(tag + "_is", std::max<size_t>(small.size(), 1));
  int* inf_b = ws.get<int>(tag + "_ib", big.size());
  FDS_HIP(hipMemsetAsync(inf_b, 0, big.size() * sizeof(int), s));
  if (!small.empty()) launch_lu(ws.upload(tag + "_ds", small), (int)small.size(), nsmall, base, piv, inf_s, s);
  const LUDesc* db = ws.upload(tag + "_db", big);
  // panel width: 32 columns with the panel in LDS when it fits, else 16
  // columns in LDS, else 32 columns worked in memory
  const size_t lds_max = max_lds_bytes();
  const size_t need32 = (size_t)nbig * kPanel * sizeof(T), need16 = (size_t)nbig * 16 * sizeof(T);
  const int kp = need32 <= lds_max ? kPanel : (need16 <= lds_max ? 16 : kPanel);
  const bool lds = need32 <= lds_max || need16 <= lds_max;
  // every panel's trailing update, uploaded once
  std::vector<GemmDesc> gd;
  std::vector<GemmTile> gt_all;
  std::vector<int64_t> g_off, t_off;
  for (int k0 = 0; k0 < nbig; k0 += kp) {
    g_off.push_back((int64_t)gd.size());
    t_off.push_back((int64_t)gt_all.size());
    const int g0 = (int)gd.size();
    for (const LUDesc& x : big) {
      const int r = x.n - k0 - kp;
      if (r <= 0) continue;
      GemmDesc g{};
      g.a_off = x.a_off + (k0 + kp) + (int64_t)k0 * x.lda;
      g.b_off = x.a_off + k0 + (int64_t)(k0 + kp) * x.lda;
      g.c_off = x.a_off + (k0 + kp) + (int64_t)(k0 + kp) * x.lda;
      g.m = g.n = r;
      g.k = kp;
      g.lda = g.ldb = g.ldc = x.lda;
      g.alpha_re = -1.0;
      g.beta_re = 1.0;
      gd.push_back(g);
      for (int tm = 0; tm * 64 < r; ++tm) gt_all.push_back(GemmTile{(int)gd.size() - 1 - g0, tm});
    }
  }
  g_off.push_back((int64_t)gd.size());
  t_off.push_back((int64_t)gt_all.size());
  const GemmDesc* dgd = ws.upload(tag + "_g", gd);
  const GemmTile* dgt = ws.upload(tag + "_gt", gt_all);
  for (int k0 = 0, pi = 0; k0 < nbig; k0 += kp, ++pi) {
    const size_t shm = (size_t)(nbig - k0) * kp * sizeof(T);
    if (!lds)
      k_panel_lu<T><<<(unsigned)big.size(), kBlk, 0, s>>>(db, k0, base, piv, inf_b);
    else if (kp == kPanel)
      k_panel_lu_lds<T, kPanel><<<(unsigned)big.size(), kBlk, shm, s>>>(db, k0, base, piv, inf_b);
    else
      k_panel_lu_lds<T, 16><<<(unsigned)big.size(), kBlk, shm, s>>>(db, k0, base, piv, inf_b);
    FDS_HIP(hipGetLastError());
    dim3 gs((unsigned)((nbig + 3) / 4), (unsigned)big.size());
    const size_t shs = (size_t)(nbig - k0) * sizeof(int);
    if (shs > lds_max)
      k_swap_outside_seq<T, kPanel><<<dim3((unsigned)((nbig + 255) / 256), (unsigned)big.size()), 256, 0, s>>>(
          db, k0, base, piv);
    else if (kp == kPanel)
      k_swap_outside<T, kPanel><<<gs, 256, shs, s>>>(db, k0, base, piv);
    else
      k_swap_outside<T, 16><<<gs, 256, shs, s>>>(db, k0, base, piv);
    FDS_HIP(hipGetLastError());
    const int rest = nbig - k0 - kp;
    if (rest <= 0) continue;
    dim3 gt((unsigned)((rest + kBlk - 1) / kBlk), (unsigned)big.size());
    if (kp == kPanel)
      k_trsm_u12<T, kPanel><<<gt, kBlk, 0, s>>>(db, k0, base);
    else
      k_trsm_u12<T, 16><<<gt, kBlk, 0, s>>>(db, k0, base);
    FDS_HIP(hipGetLastError());
    const int nt = (int)(t_off[pi + 1] - t_off[pi]);
    launch_gemm(dgd + g_off[pi], dgt + t_off[pi], nt, rest, 0, base, base, base, 0, s);
  }
  if (info) {
    // info slots back in the caller's order
    std::vector<int64_t> src, dst;
    for (size_t i = 0; i < small_i.size(); ++i) {
      src.push_back((int64_t)i);
      dst.push_back(small_i[i]);
    }
    const size_t ns = src.size();
    for (size_t i = 0; i < big_i.size(); ++i) {
      src.push_back((int64_t)(ns + i));
      dst.push_back(big_i[i]);
    }
    int* both = ws.get<int>(tag + "_ia", src.size());
    if (ns) FDS_HIP(hipMemcpyAsync(both, inf_s, ns * sizeof(int), hipMemcpyDeviceToDevice, s));
    FDS_HIP(hipMemcpyAsync(both + ns, inf_b, big_i.size() * sizeof(int), hipMemcpyDeviceToDevice, s));
    const int64_t* ds = ws.upload(tag + "_is_src", src);
    const int64_t* dd = ws.upload(tag + "_is_dst", dst);
    k_scatter_int<<<(unsigned)((src.size() + 255) / 256), 256, 0, s>>>((int64_t)src.size(), ds, dd, both, info);
    FDS_HIP(hipGetLastError());
  }
}

int solve_chunk(int nmax) { return std::max(1, std::min(8, 32768 / (16 * std::max(1, nmax)))); }
// LDS of an LU solve launch: the n x chunk block plus the pivots and the
// composed permutation (2 n ints)
size_t lu_solve_smem(int nmax, int chunk, size_t elem) {
  const size_t n = (size_t)std::max(1, nmax);
  return n * (size_t)chunk * elem + 2 * n * sizeof(int);
}

template <typename T>
void launch_lu_solve(const SolveDesc* d, int n, int nmax, int ncol_max, int ncol_override, const T* abase,
                     const int* piv, T* bbase, hipStream_t s, int chunk) {
  if (n == 0 || ncol_max == 0) return;
  int nc = solve_chunk(nmax);
  if (chunk > 0 && lu_solve_smem(nmax, chunk, sizeof(T)) <= 65536) nc = chunk;
  // the pivots staged in LDS when they fit next to the block (else in
  // place); large single matrices (a compressed root of several thousand
  // unknowns) use up to the whole LDS of a CU
  constexpr size_t kLdsMax = 160 * 1024;
  const int staged = lu_solve_smem(nmax, nc, sizeof(T)) <= kLdsMax ? 1 : 0;
  const size_t smem = staged ? lu_solve_smem(nmax, nc, sizeof(T)) : (size_t)std::max(1, nmax) * nc * sizeof(T);
  if (smem > kLdsMax) {
    // solved in place in memory, 8 columns per workgroup
    const int ng = 8;
    dim3 grid(n, (ncol_max + ng - 1) / ng);
    k_lu_solve<T, true, true><<<grid, kBlk, 0, s>>>(d, ng, ncol_override, abase, piv, bbase, 0);
    FDS_HIP(hipGetLastError());
    return;
  }
  if (smem > 65536) {
    FDS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lu_solve<T, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    FDS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lu_solve<T, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  }
  dim3 grid(n, (ncol_max + nc - 1) / nc);
  if (nc == 16 || nc == 32) {
    // many right-hand sides: diagonal blocks per column, updates as small GEMMs
    if (nc == 16)
      k_lu_solve_wide<T, 16><<<grid, kBlk, smem, s>>>(d, ncol_override, abase, piv, bbase, staged);
    else
      k_lu_solve_wide<T, 32><<<grid, kBlk, smem, s>>>(d, ncol_override, abase, piv, bbase, staged);
  } else if (nc > 8) {
    k_lu_solve<T, true><<<grid, kBlk, smem, s>>>(d, nc, ncol_override, abase, piv, bbase, staged);
  } else {
    k_lu_solve<T, false><<<grid, kBlk, smem, s>>>(d, nc, ncol_override, abase, piv, bbase, staged);
  }
  FDS_HIP(hipGetLastError());
}

std::vector<GemmTile> gemm_tiles(const std::vector<GemmDesc>& d) {
  std::vector<GemmTile> t;
  for (int i = 0; i < (int)d.size(); ++i)
    for (int tm = 0; tm * 64 < d[i].m; ++tm) t.push_back(GemmTile{i, tm});
  return t;
}

template <typename T>
void launch_gemm(const GemmDesc* d, const GemmTile* tiles, int n_tiles, int n_max, int n_override, const T* abase,
                 const T* bbase, T* cbase, int transA, hipStream_t s, int bn) {
  if (n_tiles == 0 || n_max == 0) return;
  if (bn == 16) {
    dim3 grid(n_tiles, (n_max + 15) / 16);
    if (transA)
      k_gemm<1, T, 16><<<grid, kBlk, 0, s>>>(d, tiles, n_override, abase, bbase, cbase);
    else
      k_gemm<0, T, 16><<<grid, kBlk, 0, s>>>(d, tiles, n_override, abase, bbase, cbase);
  } else {
    dim3 grid(n_tiles, (n_max + 63) / 64);
    if (transA)
      k_gemm<1, T, 64><<<grid, kBlk, 0, s>>>(d, tiles, n_override, abase, bbase, cbase);
    else
      k_gemm<0, T, 64><<<grid, kBlk, 0, s>>>(d, tiles, n_override, abase, bbase, cbase);
  }
  FDS_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ MFMA GEMM, C = alpha A^T B + beta C
// A workgroup of four wavefronts computes a 64 x 64 tile of C; each
// wavefront a 32 x 32 block as 2 x 2 tiles of the FP64 16x16x4 MFMA, four
// real products per complex one.  MFMA lanes: the A operand of lane l is row
// l % 16, the B operand column l % 16, both at k group l / 16; result slot
// v of lane l is row l / 16 + 4 v, column l % 16.  Per chunk of 16 k the
// workgroup stages the 64 rows of A^T and the 64 columns of B in LDS (each
// thread one run of four consecutive complex numbers of one column of A and
// of B), double-buffered, one barrier per chunk; within a chunk lane group
// g takes k = 4 g + v at step v (any assignment A and B share).  Rows,
// columns and k beyond the matrix read as zero.  K is cut into slabs of
// kZSlab (the last one shorter): each workgroup does one (row tile, column
// tile, slab) and, with more than one slab, writes its partial tile to P;
// k_zgemm_reduce then adds the slabs in order.  The cut depends on k only,
// so every entry of C is the same sum whatever m and n.  Workgroups are
// dealt to the 8 XCDs in turn; work units are renumbered so that each XCD
// runs a contiguous range: one slab of B at a time (it stays in that XCD's
// L2), the column tiles of a row tile together (they read the same rows
// of A).
typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kZLd = 17;      // LDS row pitch in complex numbers (16 k + 1)
constexpr int kZSlab = 1024;  // k per slab

__device__ inline void zg_fetch(c64 (&ra)[4], c64 (&rb)[4], const c64* ap, const c64* bp, bool aok, bool bok,
                                int kk, int k) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const bool ok = kk + v < k;
    ra[v] = (aok && ok) ? ap[kk + v] : cmk(0.0, 0.0);
    rb[v] = (bok && ok) ? bp[kk + v] : cmk(0.0, 0.0);
  }
}

__global__ void __launch_bounds__(256) k_zgemm_tn(int m, int n, int k, c64 alpha, const c64* __restrict__ A,
                                                  int64_t lda, const c64* __restrict__ B, int64_t ldb, c64 beta,
                                                  c64* __restrict__ C, int64_t ldc, int tiles_n, int n_tiles,
                                                  int n_slabs, c64* __restrict__ P) {
  __shared__ c64 As[2][64 * kZLd];
  __shared__ c64 Bs[2][64 * kZLd];
  const int per = (int)(gridDim.x / 8);
  const int L = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (L >= n_tiles * n_slabs) return;   // the whole workgroup
  const int ks = L / n_tiles, tl = L % n_tiles;
  const int tm = tl / tiles_n, tn = tl % tiles_n;
  const int kb = ks * kZSlab, ke = min(k, kb + kZSlab);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int r16 = lane & 15, g = lane >> 4;
  // staging: thread tid loads row / column tid / 4 at k offset 4 (tid % 4)
  const int srow = tid >> 2, sk = 4 * (tid & 3);
  const int gi = tm * 64 + srow, gj = tn * 64 + srow;
  const bool aok = gi < m, bok = gj < n;
  const c64* ap = A + (int64_t)(aok ? gi : 0) * lda;
  const c64* bp = B + (int64_t)(bok ? gj : 0) * ldb;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  d4v cr[2][2], ci[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) cr[t][u] = ci[t][u] = d4v{0.0, 0.0, 0.0, 0.0};
  c64 ra[4], rb[4];
  zg_fetch(ra, rb, ap, bp, aok, bok, kb + sk, ke);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    As[0][srow * kZLd + sk + v] = ra[v];
    Bs[0][srow * kZLd + sk + v] = rb[v];
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    const bool more = k0 + 16 < ke;
    if (more) zg_fetch(ra, rb, ap, bp, aok, bok, k0 + 16 + sk, ke);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double xr[2], xi[2], yr[2], yi[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const c64 a = As[buf][(wr + 16 * t + r16) * kZLd + 4 * g + v];
        const c64 b = Bs[buf][(wc + 16 * t + r16) * kZLd + 4 * g + v];
        xr[t] = a.re, xi[t] = a.im, yr[t] = b.re, yi[t] = b.im;
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          cr[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[t], yr[u], cr[t][u], 0, 0, 0);
          cr[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xi[t], yi[u], cr[t][u], 0, 0, 0);
          ci[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[t], yi[u], ci[t][u], 0, 0, 0);
          ci[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi[t], yr[u], ci[t][u], 0, 0, 0);
        }
    }
    if (more) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        As[buf ^ 1][srow * kZLd + sk + v] = ra[v];
        Bs[buf ^ 1][srow * kZLd + sk + v] = rb[v];
      }
    }
    __syncthreads();
    buf ^= 1;
  }
  const bool zero_beta = beta.re == 0.0 && beta.im == 0.0;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = tm * 64 + wr + 16 * t + g + 4 * v, col = tn * 64 + wc + 16 * u + r16;
        if (row < m && col < n) {
          if (n_slabs > 1) {
            P[(int64_t)ks * m * n + row + (int64_t)col * m] = cmk(cr[t][u][v], ci[t][u][v]);
          } else {
            c64* p = C + row + (int64_t)col * ldc;
            c64 val = alpha * cmk(cr[t][u][v], ci[t][u][v]);
            if (!zero_beta) val += beta * *p;
            *p = val;
          }
        }
      }
}

__global__ void k_zgemm_reduce(int m, int n, int n_slabs, const c64* __restrict__ P, c64 alpha, c64 beta,
                               c64* __restrict__ C, int64_t ldc) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)m * n) return;
  const int row = (int)(t % m), col = (int)(t / m);
  c64 acc = P[t];
  for (int s = 1; s < n_slabs; ++s) acc += P[(int64_t)s * m * n + t];
  c64* p = C + row + (int64_t)col * ldc;
  c64 val = alpha * acc;
  if (!(beta.re == 0.0 && beta.im == 0.0)) val += beta * *p;
  *p = val;
}

int zgemm_tn_slabs(int k) { return (k + kZSlab - 1) / kZSlab; }

void launch_zgemm_tn(int m, int n, int k, c64 alpha, const c64* A, int64_t lda, const c64* B, int64_t ldb, c64 beta,
                     c64* C, int64_t ldc, c64* P, hipStream_t s) {
  if (m < 1 || n < 1 || k < 1) return;
  const int tiles_m = (m + 63) / 64, tiles_n = (n + 63) / 64;
  const int n_tiles = tiles_m * tiles_n;
  const int n_slabs = zgemm_tn_slabs(k);
  if (n_slabs > 1 && !P) throw Error(1, "zgemm: slab buffer missing");
  const int64_t units = (int64_t)n_tiles * n_slabs;
  if (units > ((int64_t)1 << 30)) throw Error(1, "zgemm: problem too large");
  const int grid = (int)((units + 7) / 8 * 8);
  k_zgemm_tn<<<grid, 256, 0, s>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, tiles_n, n_tiles, n_slabs, P);
  FDS_HIP(hipGetLastError());
  if (n_slabs > 1) {
    const int64_t cnt = (int64_t)m * n;
    k_zgemm_reduce<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(m, n, n_slabs, P, alpha, beta, C, ldc);
    FDS_HIP(hipGetLastError());
  }
}

int check_cpqr_sizes(const std::vector<CpqrDesc>& d) {
  int tall = 0;
  for (auto& x : d) {
    if (x.n > kQrMaxNTall) throw Error(1, "cpqr: more than 4096 columns");
    if (x.m > kQrMaxM || x.n > kQrMaxN) tall = 1;
  }
  return tall;
}

// small problems: register-resident kernel, sized by the group's largest problem
static void launch_cpqr_reg(const CpqrDesc* d, int n, int mmax, int nmax, c64* base, int* piv, double tol, int* rank,
                            hipStream_t s) {
  const dim3 blk(64 * kQrRegWaves);
  const int ch = (mmax + 63) / 64;
  if (nmax <= 32) {
    if (ch <= 2) k_cpqr_reg<4, 2><<<n, blk, 0, s>>>(d, base, piv, tol, rank);
    else if (ch <= 3) k_cpqr_reg<4, 3><<<n, blk, 0, s>>>(d, base, piv, tol, rank);
    else k_cpqr_reg<4, 4><<<n, blk, 0, s>>>(d, base, piv, tol, rank);
  } else {
    if (ch <= 2) k_cpqr_reg<8, 2><<<n, blk, 0, s>>>(d, base, piv, tol, rank);
    else if (ch <= 3) k_cpqr_reg<8, 3><<<n, blk, 0, s>>>(d, base, piv, tol, rank);
    else k_cpqr_reg<8, 4><<<n, blk, 0, s>>>(d, base, piv, tol, rank);
  }
  FDS_HIP(hipGetLastError());
}

void cpqr_factor(const std::vector<CpqrDesc>& d, c64* base, int* piv, double tol, int* rank, Workspace& ws,
                 const std::string& tag, hipStream_t s) {
  if (d.empty()) return;
  // three groups: register-resident (m <= 256, n <= 64), one workgroup per
  // problem, many workgroups per problem (large problems)
  std::vector<CpqrDesc> grp[3];
  std::vector<int> gidx[3];
  int rm = 0, rn = 0;
  for (int i = 0; i < (int)d.size(); ++i) {
    int g = 1;
    if ((int64_t)d[i].m * d[i].n >= kQrwMinElems || d[i].n > kQrMaxN) g = 2;
    else if (d[i].m <= kQrRegRows && d[i].n <= kQrRegCols) g = 0;
    if (g == 0) {
      rm = std::max(rm, d[i].m);
      rn = std::max(rn, d[i].n);
    }
    grp[g].push_back(d[i]);
    gidx[g].push_back(i);
  }
  for (int g = 0; g < 2; ++g) {
    if (grp[g].empty()) continue;
    const std::string k = tag + (g == 0 ? "_r" : "_o");
    const bool all = grp[g].size() == d.size();
    int* r = all ? rank : ws.get<int>(k + "_rk", grp[g].size());
    const CpqrDesc* dd = ws.upload(k + "_d", grp[g]);
    if (g == 0)
      launch_cpqr_reg(dd, (int)grp[g].size(), rm, rn, base, piv, tol, r, s);
    else
      launch_cpqr(dd, (int)grp[g].size(), base, piv, tol, r, s, check_cpqr_sizes(grp[g]));
    if (!all) {
      std::vector<int64_t> src(grp[g].size()), dst(grp[g].size());
      for (size_t i = 0; i < grp[g].size(); ++i) {
        src[i] = (int64_t)i;
        dst[i] = gidx[g][i];
      }
      k_scatter_int<<<(unsigned)((src.size() + 255) / 256), 256, 0, s>>>(
          (int64_t)src.size(), ws.upload(k + "_s", src), ws.upload(k + "_t", dst), r, rank);
      FDS_HIP(hipGetLastError());
    }
  }
  if (grp[2].empty()) return;
  const std::vector<CpqrDesc>& wide = grp[2];
  const std::vector<int>& wide_i = gidx[2];
  int nmax = 0, mmax = 0, j0 = INT32_MAX, j1 = 0;
  int64_t ntot = 0;
  for (const CpqrDesc& x : wide) {
    if (x.n > kQrMaxNTall) throw Error(1, "cpqr: more than 4096 columns");
    nmax = std::max(nmax, x.n);
    mmax = std::max(mmax, x.m);
    j0 = std::min(j0, x.k_start);
    j1 = std::max(j1, std::min(x.k_end, std::min(x.m, x.n)));
    ntot = std::max<int64_t>(ntot, x.piv_off + x.n);
  }
  const CpqrDesc* dw = ws.upload(tag + "_dw", wide);
  double* nrm = ws.get<double>(tag + "_nrm", (size_t)ntot);
  QrwState* stt = ws.get<QrwState>(tag + "_st", wide.size());
  const unsigned chunks = (unsigned)((nmax + kQrwCols - 1) / kQrwCols);
  k_qrw_init<<<dim3(chunks, (unsigned)wide.size()), kBlk, 0, s>>>(dw, base, piv, nrm, stt);
  FDS_HIP(hipGetLastError());
  std::vector<QrwState> hs(wide.size());
  for (int j = j0; j <= j1; ++j) {
    k_qrw_pivot<<<(unsigned)wide.size(), kBlk, 0, s>>>(dw, j, base, piv, nrm, stt, tol);
    FDS_HIP(hipGetLastError());
    if (j < j1) {
      const unsigned ch = (unsigned)((nmax - j - 1 + kQrwCols - 1) / kQrwCols);
      if (ch > 0) {
        if (mmax - j <= kBlk * 12)
          k_qrw_update<12><<<dim3(ch, (unsigned)wide.size()), kBlk, 0, s>>>(dw, j, base, nrm, stt);
        else
          k_qrw_update<0><<<dim3(ch, (unsigned)wide.size()), kBlk, 0, s>>>(dw, j, base, nrm, stt);
        FDS_HIP(hipGetLastError());
      }
    }
    // every 32 steps: stop early once every problem has reached its rank
    if ((j - j0) % 32 == 31 && j < j1) {
      FDS_HIP(hipMemcpyAsync(hs.data(), stt, hs.size() * sizeof(QrwState), hipMemcpyDeviceToHost, s));
      FDS_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (auto& q : hs) all = all && q.stop;
      if (all) break;
    }
  }
  k_qrw_rank<<<(unsigned)((wide.size() + 255) / 256), 256, 0, s>>>((int)wide.size(), stt,
                                                                    ws.upload(tag + "_wi", wide_i), rank);
  FDS_HIP(hipGetLastError());
}

void launch_cpqr(const CpqrDesc* d, int n, c64* base, int* piv, double tol, int* rank, hipStream_t s, int tall) {
  if (n == 0) return;
  // fewer problems than compute units: sixteen wavefronts per problem
  // update its columns (the same arithmetic per column, so the same results)
  const bool few = n <= kQrFewProblems;
  if (tall) {
    if (few) k_cpqr<true, 1024><<<n, 1024, 0, s>>>(d, base, piv, tol, rank);
    else k_cpqr<true, kBlk><<<n, kBlk, 0, s>>>(d, base, piv, tol, rank);
  } else {
    if (few) k_cpqr<false, 1024><<<n, 1024, 0, s>>>(d, base, piv, tol, rank);
    else k_cpqr<false, kBlk><<<n, kBlk, 0, s>>>(d, base, piv, tol, rank);
  }
  FDS_HIP(hipGetLastError());
}

void launch_interp(const InterpDesc* d, int n, c64* abase, const int* piv, c64* dbase, hipStream_t s,
                   InterpSize sz) {
  if (n == 0) return;
  const dim3 grid((unsigned)n, (unsigned)((std::max(sz.nmax, 1) + kInterpCols - 1) / kInterpCols));
  if (sz.kmax <= kInterpSmallK)
    k_interp_small<<<grid, 256, 0, s>>>(d, abase, piv, dbase);
  else
    k_interp<<<grid, kBlk, 0, s>>>(d, abase, piv, dbase);
  FDS_HIP(hipGetLastError());
}

InterpSize interp_size(const std::vector<InterpDesc>& d) {
  InterpSize z;
  for (auto& x : d) {
    z.nmax = std::max(z.nmax, x.n);
    z.kmax = std::max(z.kmax, x.k);
  }
  return z;
}

std::vector<ScatterTile> scatter_tiles(const std::vector<ScatterDesc>& d) {
  std::vector<ScatterTile> tiles;
  for (int i = 0; i < (int)d.size(); ++i) {
    const int64_t ne = (int64_t)d[i].nr * d[i].nc;
    for (int64_t a = 0; a < ne; a += 256) tiles.push_back(ScatterTile{i, (int)std::min<int64_t>(256, ne - a), a});
  }
  return tiles;
}

template <typename TS, typename TD>
void launch_scatter(const ScatterDesc* d, const ScatterTile* tiles, int n_tiles, const int* pos, const TS* src,
                    TD* dst, hipStream_t s) {
  if (n_tiles == 0) return;
  k_scatter<TS, TD><<<n_tiles, 256, 0, s>>>(d, tiles, pos, src, dst);
  FDS_HIP(hipGetLastError());
}

template <typename T>
void launch_copy_rows(int64_t n, const int64_t* sidx, const int64_t* didx, int ncol, const T* src, int64_t lds,
                      T* dst, int64_t ldd, hipStream_t s) {
  if (n == 0 || ncol == 0) return;
  dim3 grid((unsigned)((n + 255) / 256), ncol);
  k_copy_rows<T><<<grid, 256, 0, s>>>(n, sidx, didx, ncol, src, lds, dst, ldd);
  FDS_HIP(hipGetLastError());
}

void launch_axpby(int64_t n, double alpha, const c64* src, double beta, c64* dst, hipStream_t s) {
  if (n == 0) return;
  k_axpby<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, alpha, src, beta, dst);
  FDS_HIP(hipGetLastError());
}

template <typename TS, typename TD>
void launch_convert(int64_t n, const TS* src, TD* dst, hipStream_t s) {
  if (n == 0) return;
  k_convert<TS, TD><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, src, dst);
  FDS_HIP(hipGetLastError());
}

void launch_add_c32(int64_t n, const c32* src, c64* dst, hipStream_t s) {
  if (n == 0) return;
  k_add_c32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, src, dst);
  FDS_HIP(hipGetLastError());
}

template <typename T>
void launch_colnorm2(int64_t n, int ncol, const T* src, int64_t ld, double* out, hipStream_t s) {
  if (ncol == 0) return;
  k_colnorm2<T><<<ncol, kBlk, 0, s>>>(n, src, ld, out);
  FDS_HIP(hipGetLastError());
}

void launch_flag_nonzero(int64_t n, const int* info, int* flag, hipStream_t s) {
  if (n <= 0) return;
  k_flag_nonzero<<<(unsigned)std::min<int64_t>((n + 255) / 256, 1024), 256, 0, s>>>(n, info, flag);
  FDS_HIP(hipGetLastError());
}

template <typename T>
void launch_fill_identity(int64_t n_mats, const int64_t* offs, const int* ns, const int* lds, T* base, hipStream_t s) {
  if (n_mats == 0) return;
  k_fill_identity<T><<<(unsigned)n_mats, 256, 0, s>>>(offs, ns, lds, base);
  FDS_HIP(hipGetLastError());
}

#define FDS_INST(T)                                                                                                 \
  template void launch_lu<T>(const LUDesc*, int, int, T*, int*, int*, hipStream_t);                                \
  template void lu_factor<T>(const std::vector<LUDesc>&, T*, int*, int*, Workspace&, const std::string&,           \
                             hipStream_t);                                                                          \
  template void launch_lu_solve<T>(const SolveDesc*, int, int, int, int, const T*, const int*, T*, hipStream_t,     \
                                   int);                                                                            \
  template void launch_gemm<T>(const GemmDesc*, const GemmTile*, int, int, int, const T*, const T*, T*, int,       \
                               hipStream_t, int);                                                                   \
  template void launch_copy_rows<T>(int64_t, const int64_t*, const int64_t*, int, const T*, int64_t, T*, int64_t,  \
                                    hipStream_t);                                                                   \
  template void launch_colnorm2<T>(int64_t, int, const T*, int64_t, double*, hipStream_t);                         \
  template void launch_fill_identity<T>(int64_t, const int64_t*, const int*, const int*, T*, hipStream_t);
FDS_INST(c64)
FDS_INST(c32)
#undef FDS_INST
template void launch_scatter<c64, c64>(const ScatterDesc*, const ScatterTile*, int, const int*, const c64*, c64*,
                                       hipStream_t);
template void launch_scatter<c32, c32>(const ScatterDesc*, const ScatterTile*, int, const int*, const c32*, c32*,
                                       hipStream_t);
template void launch_scatter<c32, c64>(const ScatterDesc*, const ScatterTile*, int, const int*, const c32*, c64*,
                                       hipStream_t);
template void launch_convert<c64, c32>(int64_t, const c64*, c32*, hipStream_t);
template void launch_convert<c32, c64>(int64_t, const c32*, c64*, hipStream_t);

}  // namespace fds
