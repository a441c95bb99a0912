// Batched variable-size complex linear algebra used by the elimination
// (Section 6.2), the ID (Sections 7.1-7.2) and the sweeps (Section 6.3).
// Every problem of a batch has its own sizes and offsets into one base
// array; one launch covers the whole batch.
#pragma once

#include <vector>

#include "common.hpp"
#include "devmem.hpp"

namespace fds {

struct LUDesc {         // in-place LU with partial pivoting of an n x n matrix
  int64_t a_off;
  int64_t piv_off;
  int n, lda;
};

struct SolveDesc {      // B <- A^{-1} B using the LU of LUDesc (B is n x ncol)
  int64_t a_off, piv_off, b_off;
  int n, lda, ldb, ncol;
};

struct GemmDesc {       // C = alpha op(A) B + beta C; op(A) is m x k
  int64_t a_off, b_off, c_off;
  int m, n, k, lda, ldb, ldc;
  double alpha_re, alpha_im, beta_re, beta_im;
};

struct CpqrDesc {       // column-pivoted QR of an m x n matrix (ld = lda)
  int64_t a_off, piv_off;
  int m, n, lda;
  int k_start, k_end;   // steps [k_start, k_end)
  int stop_at_tol;
};

struct InterpDesc {     // W = [I, R1^{-1} R2] P^T (k x n) from a finished CPQR
  int64_t a_off, piv_off;
  int n, lda, k;
  int64_t d_off;        // destination (col-major, ld = d_ld)
  int d_ld;
  int transpose;        // 0: write W at (r, c); 1: write W^T at (c, r)
  int solved;           // 1: R12 already holds T = R11^{-1} R12 (an earlier launch solved in place)
};

struct ScatterDesc {    // dst[dst_off + rpos[r] + cpos[c] * dst_ld] = src[src_off + r + c * src_ld]
  int64_t src_off, dst_off;
  int nr, nc, src_ld, dst_ld;
  int rpos_off, cpos_off;   // -1: identity
};

struct GemmTile {         // one 64-row tile of a GEMM problem
  int desc, tm;
};

struct ScatterTile {
  int desc;
  int count;
  int64_t start;
};

// Asynchronous launchers; descriptor arrays are device pointers.  The
// templated ones exist for T = c64 (plain form) and T = c32 (the FP32 merges
// and sweeps of the mixed-precision form).
template <typename T>
void launch_lu(const LUDesc* d, int n, int nmax, T* base, int* piv, int* info, hipStream_t s);
// LU of a batch given on the host: one workgroup per matrix where its panel
// fits in LDS, the multi-workgroup blocked LU (panels of 32 columns, GEMM
// trailing updates) for larger ones.  Descriptors go through ``ws`` under
// keys starting with ``tag``; info[i] for d[i] as in launch_lu.
template <typename T>
void lu_factor(const std::vector<LUDesc>& d, T* base, int* piv, int* info, Workspace& ws, const std::string& tag,
               hipStream_t s);
int solve_chunk(int nmax);
// chunk > 0: right-hand-side columns per workgroup (if its LDS staging fits),
// else solve_chunk(nmax)
// LDS bytes of an LU-solve launch for blocks up to nmax rows, chunk columns
size_t lu_solve_smem(int nmax, int chunk, size_t elem);
template <typename T>
void launch_lu_solve(const SolveDesc* d, int n, int nmax, int ncol_max, int ncol_override, const T* abase,
                     const int* piv, T* bbase, hipStream_t s, int chunk = 0);
std::vector<GemmTile> gemm_tiles(const std::vector<GemmDesc>& d);
// bn: output columns per workgroup, 64 (default) or 16; same results
template <typename T>
void launch_gemm(const GemmDesc* d, const GemmTile* tiles, int n_tiles, int n_max, int n_override, const T* abase,
                 const T* bbase, T* cbase, int transA, hipStream_t s, int bn = 64);
// C = alpha A^T B + beta C (complex FP64, column-major: A k x m, B k x n,
// C m x n) on the FP64 matrix cores; one GEMM, no descriptors.  K is cut
// into zgemm_tn_slabs(k) slabs whose partial products go to P
// (zgemm_tn_slabs(k) * m * n complex numbers; unused, may be null, for one
// slab) and are added in slab order, so results do not depend on m or n.
int zgemm_tn_slabs(int k);
void launch_zgemm_tn(int m, int n, int k, c64 alpha, const c64* A, int64_t lda, const c64* B, int64_t ldb, c64 beta,
                     c64* C, int64_t ldc, c64* P, hipStream_t s);
// 1 if some problem needs the tall variant (m > 2048 or n > 1024); throws
// beyond 4096 columns
int check_cpqr_sizes(const std::vector<CpqrDesc>& d);
void launch_cpqr(const CpqrDesc* d, int n, c64* base, int* piv, double tol, int* rank, hipStream_t s, int tall);
// Pivoted QR of a batch given on the host: one workgroup per problem for the
// usual sizes, the multi-workgroup step loop for problems of 2^18 elements
// or more (results identical in rule; rank[i] for d[i]).  Synchronises the
// stream every 32 steps of the multi-workgroup loop.
void cpqr_factor(const std::vector<CpqrDesc>& d, c64* base, int* piv, double tol, int* rank, Workspace& ws,
                 const std::string& tag, hipStream_t s);
// nmax: the largest n of the batch (the grid covers it in column chunks)
struct InterpSize {      // largest n and k of a batch of InterpDesc
  int nmax = 0, kmax = 0;
};
void launch_interp(const InterpDesc* d, int n, c64* abase, const int* piv, c64* dbase, hipStream_t s,
                   InterpSize sz);
InterpSize interp_size(const std::vector<InterpDesc>& d);
std::vector<ScatterTile> scatter_tiles(const std::vector<ScatterDesc>& d);
// (TS, TD) in {(c64, c64), (c32, c32), (c32, c64)}
template <typename TS, typename TD>
void launch_scatter(const ScatterDesc* d, const ScatterTile* tiles, int n_tiles, const int* pos, const TS* src,
                    TD* dst, hipStream_t s);
// dst[didx[i] + c * ldd] = src[sidx[i] + c * lds], i < n, c < ncol
template <typename T>
void launch_copy_rows(int64_t n, const int64_t* sidx, const int64_t* didx, int ncol, const T* src, int64_t lds,
                      T* dst, int64_t ldd, hipStream_t s);
// dst[i] = alpha * src[i] + beta * dst[i]
void launch_axpby(int64_t n, double alpha, const c64* src, double beta, c64* dst, hipStream_t s);
// dst[i] = src[i] converted, (TS, TD) in {(c64, c32), (c32, c64)}
template <typename TS, typename TD>
void launch_convert(int64_t n, const TS* src, TD* dst, hipStream_t s);
// dst[i] += src[i] (FP32 correction added to an FP64 vector)
void launch_add_c32(int64_t n, const c32* src, c64* dst, hipStream_t s);
// out[c] = sum_{i<n} |src[i + c ld]|^2 (FP64), c < ncol
template <typename T>
void launch_colnorm2(int64_t n, int ncol, const T* src, int64_t ld, double* out, hipStream_t s);
// flag[0] = 1 if any of the n ints at info is nonzero (flag is never cleared here)
void launch_flag_nonzero(int64_t n, const int* info, int* flag, hipStream_t s);
template <typename T>
void launch_fill_identity(int64_t n_mats, const int64_t* offs, const int* ns, const int* lds, T* base, hipStream_t s);

}  // namespace fds
