// Shared device/host declarations of the solver library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "special.hpp"

namespace fds {

// A straight element of a polygon: from (x0, y0) to (x1, y1).  ``nx, ny`` is
// its unit normal (into the cavity for a boundary curve, outward for a proxy
// circle) and dN0, dN1 the constant tangential derivatives (along t = J n)
// of the two hat functions restricted to it.
struct Elem {
  double x0, y0, x1, y1;
  double h, nx, ny, dN0, dN1;
  int poly;     // polygon id (boundary curve or proxy)
  int idx;      // index of the element within its polygon
  int npoly;    // number of elements of the polygon
  int pad;
};

// Material constants needed by the kernels.
struct MatConst {
  double kT, kL, beta, mu, rw2;   // rw2 = rho omega^2
  double ikT;                     // 1 / kT
  double alpha_re, alpha_im;
  SeriesCoef sc;                  // small-argument expansions for this beta
};

// One dense block A(rows, cols) to assemble.  Each side is a list of
// elements (global ids into the element table) and a list of DOFs; a DOF
// refers to the two elements of its hat (as indices into the side's element
// list: ``eL`` the element the node ends, ``eR`` the element it starts) and
// a displacement component.  The output entry for DOFs (r, c) goes to
// out[out_off + rpos(r) * rs + cpos(c) * cs], rpos = identity when
// rpos_off < 0.  Element-pair results for the job live at pair_off +
// je * nre + ie when the output's rows are its fast direction (rs == 1, or
// cs != 1), else at pair_off + ie * nce + je: the gather then walks the
// output in its fast direction and reads the pair results in order.
struct Job {
  int64_t pair_off;
  int64_t out_off;
  int64_t rs, cs;
  int re_off, nre;
  int ce_off, nce;
  int rd_off, nrd;
  int cd_off, ncd;
  int rpos_off, cpos_off;
};

__host__ __device__ inline bool job_rows_fast(const Job& j) { return j.rs == 1 || j.cs != 1; }
__host__ __device__ inline int64_t pair_slot(const Job& j, int ie, int je) {
  return j.pair_off + (job_rows_fast(j) ? (int64_t)je * j.nre + ie : (int64_t)ie * j.nce + je);
}
// the element pair of a job's pair number p (its slot is pair_off + p)
__host__ __device__ inline void pair_elems(const Job& j, int64_t p, int& ie, int& je) {
  if (job_rows_fast(j)) {
    ie = (int)(p % j.nre);
    je = (int)(p / j.nre);
  } else {
    ie = (int)(p / j.nce);
    je = (int)(p % j.nce);
  }
}

struct Dof {
  int eL, eR, comp, pad;
};

// Work tiles: a contiguous range [start, start+count) of a job's items
// (element pairs or output entries).
struct Tile {
  int job;
  int count;
  int64_t start;
};

// Element-pair classes.  A regular pair (no shared vertex) is integrated
// by a tensor Gauss rule with kOrders[oe] points along the test element and
// kOrders[of] along the trial element, each order chosen from the gap and
// that element's own length (elem_order_index); a pair is "series-only"
// (ser = 1) when its kernels stay on their small-argument series at every
// point (k_T times the largest distance between the two elements below
// kSeriesOnly): the same arithmetic in a kernel without the Bessel-function
// code.  Pairs that need 10 points on an element take 10 on both.
constexpr int kNumOrd = 4;
__host__ __device__ constexpr int order_of(int o) { return o == 0 ? 2 : (o == 1 ? 3 : (o == 2 ? 4 : 6)); }
enum PairClass : int { kQ10 = 0, kCoinc = 1, kAdjNext = 2, kAdjPrev = 3, kRegBase = 4 };
constexpr int kNumClass = kRegBase + 2 * kNumOrd * kNumOrd;
__host__ __device__ constexpr int reg_class(int oe, int of, int ser) { return kRegBase + (oe * kNumOrd + of) * 2 + ser; }
// Reported classes (fds_stats): 0 regular pairs with at most 4 points on the
// test element, 1 regular pairs with 6, 2 the 10-point pairs, 3 coincident,
// 4 and 5 adjacent (shared vertex at the end / the start of the test element).
constexpr int kNumPublicClass = 6;
// a pair is series-only when k_T d_max < kSeriesOnly (d_max the largest
// endpoint distance, which bounds every point distance); the margin below
// the series switch (1) keeps rounding from deciding the class
constexpr double kSeriesOnly = 0.999;
static_assert(kSeriesOnly < kSeriesSwitch, "series-only pairs must stay below the series switch");

// quadrature constants (filled at library initialisation)
constexpr int kQCoinc = 20;
constexpr int kPCoinc = 6;
constexpr int kQAdj = 12;
constexpr int kPAdj = 4;
constexpr int kNCoincPts = 4 * kQCoinc;
constexpr int kNAdjPts = 2 * kQAdj * kQAdj;
// Gauss points along one element of a regular pair, by the gap d over the
// element's length h: 2 from kRatioQ2, 3 from kRatioQ3, 4 from kFarRatio, 6
// from kNearRatio, else 10.  Orders grow with the oscillation of the kernels
// over the element: at least 3 points when k_T h > kKhQ2, 4 when
// k_T h > kKhQ3, 6 when k_T h > kKhQ4 and 10 when k_T h > kKhQ6.  A singular
// pair takes the longer rules below when k_T h > kKhQ4 (h the longer
// element).  Boundary elements need k_T h <= kKhMax.
constexpr double kRatioQ2 = 512.0;
constexpr double kRatioQ3 = 32.0;
constexpr double kFarRatio = 8.0;
constexpr double kNearRatio = 2.0;
constexpr double kKhQ2 = 0.004;
constexpr double kKhQ3 = 0.02;
constexpr double kKhQ4 = 0.5;
constexpr double kKhQ6 = 2.5;
constexpr double kKhMax = 5.0;
constexpr int kQCoincHi = 30;
constexpr int kQAdjHi = 24;
constexpr int kNCoincHiPts = 4 * kQCoincHi;
constexpr int kNAdjHiPts = 2 * kQAdjHi * kQAdjHi;
// smallest proxy polygon for a proxy radius rho at wavenumber k: outgoing
// fields on the circle carry Fourier modes up to about k rho
inline int proxy_count(double k, double rho, int m_min) {
  const double m = std::ceil(2.0 * k * rho) + 40.0;
  return m > (double)m_min ? (int)m : m_min;
}

// Sum over the 64 lanes of a wavefront with DPP moves inside each row of 16
// lanes (swap neighbours, swap pairs, half-row mirror, row mirror: after
// these every lane holds its row's sum) and the four row sums read out of
// lanes 0, 16, 32, 48.  Every lane of the wavefront must be active.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline double lane_value(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ inline double wsum_full(double v) {
  v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);   // row_half_mirror
  v += dpp_move<0x140>(v);   // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// maximum over the 64 lanes (same DPP pattern as wsum_full; every lane active)
__device__ inline double wmax_full(double v) {
  v = fmax(v, dpp_move<0xB1>(v));
  v = fmax(v, dpp_move<0x4E>(v));
  v = fmax(v, dpp_move<0x141>(v));
  v = fmax(v, dpp_move<0x140>(v));
  return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

// Integer minimum over the 64 lanes (same DPP pattern; every lane active).
template <int CTRL>
__device__ inline int dpp_move_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ inline int wmin_int_full(int v) {
  v = min(v, dpp_move_int<0xB1>(v));
  v = min(v, dpp_move_int<0x4E>(v));
  v = min(v, dpp_move_int<0x141>(v));
  v = min(v, dpp_move_int<0x140>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Row exchanges of two doubles between lane groups (v_permlane32_swap and
// v_permlane16_swap of gfx950, on both 32-bit halves):
//   swap_rows32: a <- [a 0..31, b 0..31],  b <- [a 32..63, b 32..63]
//   swap_rows16: a <- [a 0..15, b 0..15, a 32..47, b 32..47],
//                b <- [a 16..31, b 16..31, a 48..63, b 48..63]
__device__ inline void swap_rows32(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ inline void swap_rows16(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}

// Sums over the 64 lanes of N values at once (N a multiple of 4), for a
// fraction of the moves of N separate wsum_full: halve the values twice by
// row exchanges (lanes 32 apart, then 16 apart; each exchange leaves half of
// the lanes with one value and half with the other), then finish each of the
// N/4 left in its rows of 16 lanes.  On return v[k] (k < N/4) holds, in
// every lane of row r (lanes 16 r .. 16 r + 15), the 64-lane sum of input
// v[k + r N/4]; wsum_rows_get reads a sum by its input index.  Every lane
// of the wavefront must be active.
template <int N>
__device__ inline void wsum_rows(double (&v)[N]) {
  static_assert(N % 4 == 0, "four rows of sums");
  constexpr int H = N / 2, Q = N / 4;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    double a = v[k], b = v[k + H];
    swap_rows32(a, b);
    v[k] = a + b;
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double a = v[k], b = v[k + Q];
    swap_rows16(a, b);
    v[k] = a + b;
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    v[k] += dpp_move<0xB1>(v[k]);
    v[k] += dpp_move<0x4E>(v[k]);
    v[k] += dpp_move<0x141>(v[k]);
    v[k] += dpp_move<0x140>(v[k]);
  }
}
template <int N>
__device__ inline double wsum_rows_get(const double (&v)[N], int i) {
  return lane_value(v[i % (N / 4)], 16 * (i / (N / 4)));
}

struct QuadTables {
  double g2[2], w2[2], g3[3], w3[3], g4[4], w4[4], g6[6], w6[6], g10[10], w10[10];
  double cu[kNCoincPts], cv[kNCoincPts], cw[kNCoincPts], coff[kNCoincPts];
  double au[kNAdjPts], av[kNAdjPts], aw[kNAdjPts];
  double rg[6], rw[6];   // load-vector rule
  // the longer singular rules (k_T h > kKhQ4)
  double chu[kNCoincHiPts], chv[kNCoincHiPts], chw[kNCoincHiPts], choff[kNCoincHiPts];
  double ahu[kNAdjHiPts], ahv[kNAdjHiPts], ahw[kNAdjHiPts];
};

class Error : public std::runtime_error {
 public:
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define FDS_HIP(call)                                                                \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw ::fds::Error(4, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

}  // namespace fds
