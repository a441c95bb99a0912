// Galerkin entry assembly on gfx950.
//
// Entries of A = D + I0/2 + alpha N (Section 5.2) between P1 hats are sums
// of element-pair integrals.  The hypersingular operator is used in a
// weakly singular form obtained by integrating by parts along the closed
// polygons (the identity T^n u = 2 mu d_s(J u) + (lambda + 2 mu) n div u +
// mu (curl u) t, t = J n, with div/curl of the fundamental solution reducing
// to scalar Helmholtz kernels).  With Phi_k = (i/4) H0(k r),
// Q = mu G - Phi_T I and dPhi = Phi_L - Phi_T, the entry between a test hat
// psi on element e and a trial hat phi on element f is
//
//   int int psi phi' (Phi_T J - 2 Q J^T) + psi phi ((d_ny Phi_T) I + grad_y dPhi n_y^T)
//   + alpha [ 4 mu psi' phi' J Q J^T
//             - 2 mu psi' phi ((d_ny Phi_T) J + (J grad_y dPhi) n_y^T)
//             + 2 mu psi phi' ((d_nx Phi_T) J - n_x (J grad_x dPhi)^T)
//             + rho omega^2 psi phi (n_x n_y^T Phi_L + t_x t_y^T Phi_T) ],
//
// plus (1/2) int psi phi on coincident elements.  All kernels are at most
// logarithmically singular on coincident elements and O(1/r) only at the
// common vertex of adjacent elements.
//
// Pipeline for a batch of dense blocks ("jobs"):
//   k_classify   every (row element, column element) pair of every job is
//                put into a list by its quadrature class: regular pairs by
//                the tensor orders (2, 3, 4 or 6 points along each element,
//                chosen by the gap over that element's length and by k_T h)
//                and whether they stay on the small-argument series; the
//                10-point pairs; coincident; adjacent (two orientations);
//   k_regular<OE,SER> one thread per regular pair with the test order OE;
//   k_regular_wave10 one wavefront per 10-point pair;
//   k_special<C>, k_special2<C>
//                one wavefront per singular pair (the 80 or 288 points of
//                its rule spread over the 64 lanes, then reduced); the
//                adjacent classes run at two wavefronts per SIMD;
//   k_gather     one thread per output entry: sum of the four element pairs
//                of its two hats, written at its (row, column) position.
// Pair results are 16 complex numbers [a][b][i][j] stored
// structure-of-arrays; the gather order is fixed, so results are
// bit-reproducible.
#include <algorithm>

#include "assembly.hpp"

namespace fds {

__constant__ QuadTables c_quad;

// two doubles as one 16-byte vector (one load or store instruction)
typedef double d2v __attribute__((ext_vector_type(2)));

// The four 2 x 2 blocks of one quadrature point (d = x - y, normals n_x,
// n_y of the test and trial elements) whose hat-weighted sums make up a
// pair's 16 entries:
//   entry[a][b][ij] += N_a dN_b M1 + w dN_a dN_b M2 + N_a N_b M3 + w dN_a N_b M4
// (N the hat values, dN their constant tangential derivatives, w the
// quadrature weight; N_a carries w).  The blocks are formed entry by entry
// (ij) and added at once, so only one entry's four values are live.  SER:
// the point is known to lie on the small-argument series (k_T r < 1): the
// same values without the Bessel-function branch.

// A pair's 16 entries accumulated point by point (64 registers, which lets
// two wavefronts share a SIMD; the special pairs sum them over the lanes of
// their wavefront afterwards).  During the accumulation slot [a][b][ij]
// (index 8 a + 4 b + ij) holds, instead of entry [a][b], the combination
//   [0][0]: sum over a and b,  [0][1]: sum over a at b = 1,
//   [1][0]: sum over b at a = 1,  [1][1]: the entry [1][1] itself,
// which the hat structure (N_0 + N_1 = 1 for the values, dN_1 = -dN_0 for
// the derivatives) makes cheaper to accumulate: 18 real multiply-adds per
// point and ij instead of 32.  pair_entries turns the sums into entries.
struct PairRes {
  c64 R[16];
};

__device__ inline void pair_entries(PairRes& A) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const c64 ss = A.R[k], s1 = A.R[4 + k], t1 = A.R[8 + k], b11 = A.R[12 + k];
    const c64 e01 = s1 - b11, e10 = t1 - b11;
    A.R[k] = ss - e01 - e10 - b11;
    A.R[4 + k] = e01;
    A.R[8 + k] = e10;
  }
}

// 1/sqrt(x) for a positive normal x: the hardware estimate refined by two
// Newton steps y <- y + y (1 - x y^2)/2 (each squares the relative error;
// within about 1 ulp).
__device__ inline double rsqrt_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

template <bool SER = false>
__device__ inline void acc_point_direct(const MatConst& m, double dx, double dy, double w, double u, double v,
                                        double nx0, double nx1, double ny0, double ny1, double dA0, double dA1,
                                        double dB0, double dB1, PairRes& A) {
  const double r2 = dx * dx + dy * dy;
  const double ir = rsqrt_newton(r2);
  const double r = r2 * ir;
  const double e0 = dx * ir, e1 = dy * ir;
  const double je0 = -e1, je1 = e0;
  const double a = m.kT * r, ia = ir * m.ikT;
  c64 h0a, h1a, h0b, E, chi;
  if (SER)
    kernel_values_series(a, ia, m.sc, h0a, h1a, h0b, E, chi);
  else
    kernel_values(a, ia, m.sc, h0a, h1a, h0b, E, chi);
  const c64 phiT = cmk(-0.25 * h0a.im, 0.25 * h0a.re);
  const c64 phiL = cmk(-0.25 * h0b.im, 0.25 * h0b.re);
  const c64 q = cmk(-0.25 * m.kT * h1a.im, 0.25 * m.kT * h1a.re);   // (i/4) k_T H1(a)
  const double eny = e0 * ny0 + e1 * ny1;
  const double enx = e0 * nx0 + e1 * nx1;
  const c64 dny = q * eny;          // d_{n_y} Phi_T
  const c64 dnx = q * (-enx);       // d_{n_x} Phi_T
  // grad_y dPhi = cg e,  cg = -(i/4) k_T a E
  const double ka = 0.25 * m.kT * a;
  const c64 cg = cmk(ka * E.im, -ka * E.re);
  const c64 al = cmk(m.alpha_re, m.alpha_im);
  const c64 K = (2.0 * m.mu) * al;             // 2 alpha mu
  const c64 Z = mul_i(m.mu * al);              // i alpha mu
  const c64 P = phiT - cmk(-0.5 * E.im, 0.5 * E.re);   // Phi_T - (i/2) E
  const c64 hc = cmk(-0.5 * chi.im, 0.5 * chi.re);     // (i/2) chi
  const c64 PK = P + K * dnx;                  // the J parts of M1
  const c64 Kcg = K * cg;
  const c64 ZE = Z * E, Zchi = Z * chi;
  const c64 Kdny = K * dny;
  const double ex[2] = {e0, e1};
  const double jex[2] = {je0, je1};
  const double nx[2] = {nx0, nx1};
  const double ny[2] = {ny0, ny1};
  const double tx[2] = {-nx1, nx0};
  const double ty[2] = {-ny1, ny0};
  const c64 arw = (m.rw2) * al;
  const c64 arwL = arw * phiL;
  const c64 arwT = arw * phiT;
  // weights of the four accumulated combinations (dA1 = -dA0, dB1 = -dB0)
  (void)dA0;
  (void)dB0;
  const double wu = w * u, wv = w * v, wuv = wu * v;
  const double s1_m1 = w * dB1;                  // [0][1]: w dB1 M1 + w v M3
  const double t1_m4 = w * dA1;                  // [1][0]: w u M3 + w dA1 M4
  const double b_m1 = wu * dB1, b_m2 = (w * dA1) * dB1, b_m4 = (w * dA1) * v;   // [1][1]
  // entry ij: J = [[0, -1], [1, 0]], delta the identity; terms with a zero
  // factor J_ij or delta_ij are left out
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = 2 * i + j;
      c64 M1 = (nx[i] * jex[j]) * Kcg - (ex[i] * jex[j]) * hc;
      c64 M2 = (jex[i] * jex[j]) * Zchi;
      c64 M3 = (ex[i] * ny[j]) * cg + (nx[i] * ny[j]) * arwL + (tx[i] * ty[j]) * arwT;
      c64 M4 = -((jex[i] * ny[j]) * Kcg);
      if (i == j) {
        M2 -= ZE;
        M3 += dny;
      } else if (i == 0) {   // J_01 = -1
        M1 -= PK;
        M4 += Kdny;
      } else {               // J_10 = 1
        M1 += PK;
        M4 -= Kdny;
      }
      A.R[k] += w * M3;
      A.R[4 + k] += s1_m1 * M1 + wv * M3;
      A.R[8 + k] += wu * M3 + t1_m4 * M4;
      A.R[12 + k] += b_m1 * M1 + wuv * M3 + b_m2 * M2 + b_m4 * M4;
    }
}

__device__ inline double seg_point_dist(double px, double py, double ax, double ay, double bx, double by) {
  const double dx = bx - ax, dy = by - ay;
  double t = ((px - ax) * dx + (py - ay) * dy) / (dx * dx + dy * dy);
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  const double qx = ax + t * dx - px, qy = ay + t * dy - py;
  return sqrt(qx * qx + qy * qy);
}

__device__ inline double seg_seg_dist(const Elem& e, const Elem& f) {
  double d = seg_point_dist(e.x0, e.y0, f.x0, f.y0, f.x1, f.y1);
  d = fmin(d, seg_point_dist(e.x1, e.y1, f.x0, f.y0, f.x1, f.y1));
  d = fmin(d, seg_point_dist(f.x0, f.y0, e.x0, e.y0, e.x1, e.y1));
  d = fmin(d, seg_point_dist(f.x1, f.y1, e.x0, e.y0, e.x1, e.y1));
  return d;
}

// Index into the regular orders (0..kNumOrd-1 for 2, 3, 4, 6 points) of one
// element of a regular pair with gap d, or kNumOrd for 10 points.
__device__ inline int elem_order_index(double d, double h, double kT) {
  int o = kNumOrd;
  if (d >= kNearRatio * h) o = 3;
  if (d >= kFarRatio * h) o = 2;
  if (d >= kRatioQ3 * h) o = 1;
  if (d >= kRatioQ2 * h) o = 0;
  const double kh = kT * h;
  if (kh > kKhQ2 && o < 1) o = 1;
  if (kh > kKhQ3 && o < 2) o = 2;
  if (kh > kKhQ4 && o < 3) o = 3;
  if (kh > kKhQ6) o = kNumOrd;
  return o;
}

__device__ inline int classify_pair(const Elem& e, const Elem& f, int ge, int gf, double kT) {
  if (e.poly == f.poly) {
    if (ge == gf) return kCoinc;
    const int n = e.npoly;
    if (f.idx == (e.idx + 1) % n) return kAdjNext;
    if (f.idx == (e.idx + n - 1) % n) return kAdjPrev;
  }
  const double d = seg_seg_dist(e, f);
  const int oe = elem_order_index(d, e.h, kT), of = elem_order_index(d, f.h, kT);
  if (oe == kNumOrd || of == kNumOrd) return kQ10;
  // the largest distance between two points of the elements is an endpoint distance
  double dm2 = 0.0;
  {
    const double p[4][2] = {{e.x0 - f.x0, e.y0 - f.y0}, {e.x0 - f.x1, e.y0 - f.y1},
                            {e.x1 - f.x0, e.y1 - f.y0}, {e.x1 - f.x1, e.y1 - f.y1}};
#pragma unroll
    for (int k = 0; k < 4; ++k) dm2 = fmax(dm2, p[k][0] * p[k][0] + p[k][1] * p[k][1]);
  }
  return reg_class(oe, of, kT * sqrt(dm2) < kSeriesOnly ? 1 : 0);
}

// ------------------------------------------------------------------ geometry
__global__ void k_elem_geometry(const double* __restrict__ xy, const int* __restrict__ curve_of,
                                const int* __restrict__ curve_off, const int* __restrict__ curve_n,
                                int n_elem, Elem* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_elem) return;
  const int c = curve_of[g];
  const int o = curve_off[c], n = curve_n[c];
  const int l = g - o;
  const int g1 = o + (l + 1) % n;
  Elem e;
  e.x0 = xy[2 * g];
  e.y0 = xy[2 * g + 1];
  e.x1 = xy[2 * g1];
  e.y1 = xy[2 * g1 + 1];
  const double dx = e.x1 - e.x0, dy = e.y1 - e.y0;
  e.h = sqrt(dx * dx + dy * dy);
  const double tx = dx / e.h, ty = dy / e.h;
  // n = J tau (into the cavity); t = J n = -tau;  d_s N0 = 1/h, d_s N1 = -1/h
  e.nx = -ty;
  e.ny = tx;
  e.dN0 = 1.0 / e.h;
  e.dN1 = -1.0 / e.h;
  e.poly = c;
  e.idx = l;
  e.npoly = n;
  e.pad = 0;
  out[g] = e;
}

// proxy polygons: n_proxy vertices c + rho (cos 2 pi s/n, sin 2 pi s/n),
// outward normal n = -J tau, t = J n = tau: d_s N0 = -1/h, d_s N1 = 1/h.
__global__ void k_proxy_elems(const double* __restrict__ crd, const int* __restrict__ poff, int n_cells, int total,
                              int poly_base, Elem* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  // cell of element g: the last c with poff[c] <= g (poff ascending, poff[n_cells] = total)
  int lo = 0, hi = n_cells - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (poff[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  const int c = lo, n_proxy = poff[c + 1] - poff[c], s = g - poff[c];
  const double cx = crd[3 * c], cy = crd[3 * c + 1], rho = crd[3 * c + 2];
  const double t0 = 2.0 * kPi * s / n_proxy;
  const double t1 = 2.0 * kPi * ((s + 1) % n_proxy) / n_proxy;
  double s0, c0, s1, c1;
  sincos(t0, &s0, &c0);
  sincos(t1, &s1, &c1);
  Elem e;
  e.x0 = cx + rho * c0;
  e.y0 = cy + rho * s0;
  e.x1 = cx + rho * c1;
  e.y1 = cy + rho * s1;
  const double dx = e.x1 - e.x0, dy = e.y1 - e.y0;
  e.h = sqrt(dx * dx + dy * dy);
  const double tx = dx / e.h, ty = dy / e.h;
  e.nx = ty;
  e.ny = -tx;
  e.dN0 = -1.0 / e.h;
  e.dN1 = 1.0 / e.h;
  e.poly = poly_base + c;
  e.idx = s;
  e.npoly = n_proxy;
  e.pad = 0;
  out[g] = e;
}

// ------------------------------------------------------------------ classify
// Each block takes a tile of up to kClsTile pairs (4 per thread).  Slots are
// counted per class with LDS atomics and reserved with one global atomic per
// class per block; the order of a list does not matter (each pair's result
// goes to its own slot).
constexpr int kClsTile = 1024;

__global__ void __launch_bounds__(256) k_classify(const Tile* __restrict__ tiles, const Job* __restrict__ jobs,
                                                  const int* __restrict__ elist, const Elem* __restrict__ elems,
                                                  unsigned long long* __restrict__ lists, int64_t list_cap,
                                                  unsigned int* __restrict__ counters, double kT) {
  __shared__ unsigned int s_cnt[kNumClass];
  __shared__ unsigned int s_base[kNumClass];
  const Tile t = tiles[blockIdx.x];
  const Job jb = jobs[t.job];
  for (int c = threadIdx.x; c < kNumClass; c += blockDim.x) s_cnt[c] = 0;
  __syncthreads();
  int cls[4];
  unsigned int off[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int li = j * 256 + threadIdx.x;
    cls[j] = -1;
    off[j] = 0;
    if (li < t.count) {
      const int64_t p = t.start + li;
      int ie, je;
      pair_elems(jb, p, ie, je);
      const int ge = elist[jb.re_off + ie], gf = elist[jb.ce_off + je];
      cls[j] = classify_pair(elems[ge], elems[gf], ge, gf, kT);
      off[j] = atomicAdd(&s_cnt[cls[j]], 1u);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kNumClass; c += blockDim.x) s_base[c] = s_cnt[c] ? atomicAdd(&counters[c], s_cnt[c]) : 0u;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (cls[j] < 0) continue;
    const int64_t p = t.start + j * 256 + threadIdx.x;
    const unsigned long long key = ((unsigned long long)(unsigned)t.job << 32) | (unsigned long long)p;
    const int64_t slot = (int64_t)s_base[cls[j]] + off[j];
    if (slot < list_cap) lists[cls[j] * list_cap + slot] = key;
  }
}

__device__ inline void decode(unsigned long long key, const Job* jobs, const int* elist, Job& jb, int& ie, int& je,
                              int& ge, int& gf) {
  const int job = (int)(key >> 32);
  const int64_t p = (int64_t)(key & 0xffffffffull);
  jb = jobs[job];
  pair_elems(jb, p, ie, je);
  ge = elist[jb.re_off + ie];
  gf = elist[jb.ce_off + je];
}

// ------------------------------------------------------------------ regular pairs
__device__ inline const double* gauss_points(int q) {
  return q == 2 ? c_quad.g2 : (q == 3 ? c_quad.g3 : (q == 4 ? c_quad.g4 : c_quad.g6));
}
__device__ inline const double* gauss_weights(int q) {
  return q == 2 ? c_quad.w2 : (q == 3 ? c_quad.w3 : (q == 4 ? c_quad.w4 : c_quad.w6));
}

// QE points along the test element (compile time), qf along the trial element
template <int QE, bool SER>
__device__ inline void regular_pair(unsigned long long key, int qf, const Job* __restrict__ jobs,
                                    const int* __restrict__ elist, const Elem* __restrict__ elems, const MatConst& m,
                                    c64* __restrict__ res, int64_t np) {
  Job jb;
  int ie, je, ge, gf;
  decode(key, jobs, elist, jb, ie, je, ge, gf);
  const Elem e = elems[ge];
  const Elem f = elems[gf];
  const double* ge_ = gauss_points(QE);
  const double* we_ = gauss_weights(QE);
  const double* gf_ = gauss_points(qf);
  const double* wf_ = gauss_weights(qf);
  PairRes A;
#pragma unroll
  for (int k = 0; k < 16; ++k) A.R[k] = cmk(0.0, 0.0);
  const double ox = e.x0 - f.x0, oy = e.y0 - f.y0;
  const double ax = e.x1 - e.x0, ay = e.y1 - e.y0;
  const double bx = f.x1 - f.x0, by = f.y1 - f.y0;
  const double hh = e.h * f.h;
  for (int i = 0; i < QE; ++i) {
    const double u = ge_[i];
    const double wu = we_[i] * hh;
    for (int j = 0; j < qf; ++j) {
      const double v = gf_[j];
      const double dx = ox + u * ax - v * bx;
      const double dy = oy + u * ay - v * by;
      acc_point_direct<SER>(m, dx, dy, wu * wf_[j], u, v, e.nx, e.ny, f.nx, f.ny, e.dN0, e.dN1, f.dN0, f.dN1, A);
    }
  }
  pair_entries(A);
  const int64_t slot = pair_slot(jb, ie, je);
#pragma unroll
  for (int k = 0; k < 16; ++k)   // read once, by the gather: streaming stores
    __builtin_nontemporal_store(d2v{A.R[k].re, A.R[k].im}, reinterpret_cast<d2v*>(res + k * np + slot));
}

// The regular pairs with order index OE on the test element, one thread per
// pair: the kNumOrd lists of that test order (one per trial order) taken in
// sequence by a grid-stride loop, so neighbouring lanes mostly share their
// trial order.  List lengths are read on the device.  Two wavefronts per
// SIMD: the register budget is 256 per lane.  SER: the series-only lists
// (no Bessel-function code, no call).
template <int OE, bool SER>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_regular(const unsigned long long* __restrict__ lists, int64_t cap, const unsigned int* __restrict__ counts,
          const Job* __restrict__ jobs, const int* __restrict__ elist, const Elem* __restrict__ elems, MatConst m,
          c64* __restrict__ res, int64_t np) {
  int64_t cnt[kNumOrd], total = 0;
#pragma unroll
  for (int of = 0; of < kNumOrd; ++of) {
    cnt[of] = min((int64_t)counts[reg_class(OE, of, SER ? 1 : 0)], cap);
    total += cnt[of];
  }
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int of = 0;
    int64_t i = t;
    while (of < kNumOrd - 1 && i >= cnt[of]) {
      i -= cnt[of];
      ++of;
    }
    const unsigned long long key = lists[(int64_t)reg_class(OE, of, SER ? 1 : 0) * cap + i];
    regular_pair<order_of(OE), SER>(key, order_of(of), jobs, elist, elems, m, res, np);
  }
}

// 10-point pairs: one wavefront per pair (the 100 points of the tensor rule
// over the 64 lanes, the 16 sums reduced by DPP).  A level has few of them
// (about 20 000 per batch on the large ellipse), which at one thread per
// pair filled a third of the SIMDs.
__device__ inline void regular_pair_wave10(unsigned long long key, int lane, const Job* __restrict__ jobs,
                                           const int* __restrict__ elist, const Elem* __restrict__ elems,
                                           const MatConst& m, c64* __restrict__ res, int64_t np) {
  Job jb;
  int ie, je, ge, gf;
  decode(key, jobs, elist, jb, ie, je, ge, gf);
  const Elem e = elems[ge];
  const Elem f = elems[gf];
  PairRes A;
#pragma unroll
  for (int k = 0; k < 16; ++k) A.R[k] = cmk(0.0, 0.0);
  const double ox = e.x0 - f.x0, oy = e.y0 - f.y0;
  const double ax = e.x1 - e.x0, ay = e.y1 - e.y0;
  const double bx = f.x1 - f.x0, by = f.y1 - f.y0;
  const double hh = e.h * f.h;
  for (int p = lane; p < 100; p += 64) {
    const int i = p / 10, j = p - 10 * i;
    const double u = c_quad.g10[i], v = c_quad.g10[j];
    acc_point_direct(m, ox + u * ax - v * bx, oy + u * ay - v * by, (c_quad.w10[i] * hh) * c_quad.w10[j], u, v,
                     e.nx, e.ny, f.nx, f.ny, e.dN0, e.dN1, f.dN0, f.dN1, A);
  }
  const int64_t slot = pair_slot(jb, ie, je);
  pair_entries(A);   // linear: each lane's partial sums, then the lane sums
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    c64 val = A.R[k];
    val.re = wsum_full(val.re);
    val.im = wsum_full(val.im);
    if (lane == 0) res[k * np + slot] = val;
  }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_regular_wave10(const unsigned long long* __restrict__ list, const unsigned int* __restrict__ count_ptr,
                 const Job* __restrict__ jobs, const int* __restrict__ elist, const Elem* __restrict__ elems,
                 MatConst m, c64* __restrict__ res, int64_t np) {
  const int64_t count = min((int64_t)*count_ptr, np);
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; w < count; w += nw)
    regular_pair_wave10(list[w], lane, jobs, elist, elems, m, res, np);
}

// ------------------------------------------------------------------ singular pairs
template <int C>
__device__ inline void special_pair(unsigned long long key, int lane, const Job* __restrict__ jobs,
                                    const int* __restrict__ elist, const Elem* __restrict__ elems, const MatConst& m,
                                    c64* __restrict__ res, int64_t np);

// one wavefront per pair, grid-stride over the class list
template <int C>
__device__ inline void special_loop(const unsigned long long* __restrict__ list, const unsigned int* __restrict__ count_ptr,
                                    const Job* __restrict__ jobs, const int* __restrict__ elist,
                                    const Elem* __restrict__ elems, const MatConst& m, c64* __restrict__ res,
                                    int64_t np) {
  const int64_t count = min((int64_t)*count_ptr, np);
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; w < count; w += nw)
    special_pair<C>(list[w], lane, jobs, elist, elems, m, res, np);
}

// coincident pairs: one wavefront per SIMD (all registers)
template <int C>
__global__ void __launch_bounds__(256) k_special(const unsigned long long* __restrict__ list,
                                                 const unsigned int* __restrict__ count_ptr,
                                                 const Job* __restrict__ jobs, const int* __restrict__ elist,
                                                 const Elem* __restrict__ elems, MatConst m,
                                                 c64* __restrict__ res, int64_t np) {
  special_loop<C>(list, count_ptr, jobs, elist, elems, m, res, np);
}

// adjacent pairs (288 points): two wavefronts per SIMD measured faster
template <int C>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_special2(const unsigned long long* __restrict__ list, const unsigned int* __restrict__ count_ptr,
           const Job* __restrict__ jobs, const int* __restrict__ elist, const Elem* __restrict__ elems, MatConst m,
           c64* __restrict__ res, int64_t np) {
  special_loop<C>(list, count_ptr, jobs, elist, elems, m, res, np);
}

template <int C>
__device__ inline void special_pair(unsigned long long key, int lane, const Job* __restrict__ jobs,
                                    const int* __restrict__ elist, const Elem* __restrict__ elems, const MatConst& m,
                                    c64* __restrict__ res, int64_t np) {
  Job jb;
  int ie, je, ge, gf;
  decode(key, jobs, elist, jb, ie, je, ge, gf);
  const Elem e = elems[ge];
  const Elem f = elems[gf];
  PairRes A;
#pragma unroll
  for (int k = 0; k < 16; ++k) A.R[k] = cmk(0.0, 0.0);
  const double hh = e.h * f.h;
  // the longer rule when the kernels oscillate over the pair (uniform over
  // the wavefront: one pair per wavefront)
  const bool hi = m.kT * fmax(e.h, f.h) > kKhQ4;
  if (C == kCoinc) {
    const double ax = e.x1 - e.x0, ay = e.y1 - e.y0;
    const int npts = hi ? kNCoincHiPts : kNCoincPts;
    const double* cu = hi ? c_quad.chu : c_quad.cu;
    const double* cv = hi ? c_quad.chv : c_quad.cv;
    const double* cw = hi ? c_quad.chw : c_quad.cw;
    const double* co = hi ? c_quad.choff : c_quad.coff;
    for (int p = lane; p < npts; p += 64) {
      const double off = co[p];
      acc_point_direct(m, off * ax, off * ay, cw[p] * hh, cu[p], cv[p], e.nx, e.ny, f.nx, f.ny, e.dN0, e.dN1, f.dN0,
                       f.dN1, A);
    }
  } else {
    // vectors from the shared vertex to the far ends of e and f
    double Ax, Ay, Bx, By;
    if (C == kAdjNext) {   // shared vertex = end of e = start of f
      Ax = e.x0 - e.x1;
      Ay = e.y0 - e.y1;
      Bx = f.x1 - f.x0;
      By = f.y1 - f.y0;
    } else {               // shared vertex = start of e = end of f
      Ax = e.x1 - e.x0;
      Ay = e.y1 - e.y0;
      Bx = f.x0 - f.x1;
      By = f.y0 - f.y1;
    }
    const int npts = hi ? kNAdjHiPts : kNAdjPts;
    const double* au = hi ? c_quad.ahu : c_quad.au;
    const double* av = hi ? c_quad.ahv : c_quad.av;
    const double* aw = hi ? c_quad.ahw : c_quad.aw;
    for (int p = lane; p < npts; p += 64) {
      const double up = au[p], vp = av[p];
      const double u = (C == kAdjNext) ? 1.0 - up : up;
      const double v = (C == kAdjNext) ? vp : 1.0 - vp;
      acc_point_direct(m, up * Ax - vp * Bx, up * Ay - vp * By, aw[p] * hh, u, v, e.nx, e.ny, f.nx, f.ny, e.dN0,
                       e.dN1, f.dN0, f.dN1, A);
    }
  }
  const int64_t slot = pair_slot(jb, ie, je);
  pair_entries(A);   // linear: each lane's partial sums, then the lane sums
#pragma unroll
  for (int aa = 0; aa < 2; ++aa)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        c64 val = A.R[aa * 8 + bb * 4 + k];
        val.re = wsum_full(val.re);
        val.im = wsum_full(val.im);
        if (C == kCoinc && (k == 0 || k == 3)) {
          // (1/2) int psi phi on the coincident element: h/3 on the diagonal, h/6 off it
          val.re += 0.5 * e.h * (aa == bb ? (1.0 / 3.0) : (1.0 / 6.0));
        }
        if (lane == 0) res[(aa * 8 + bb * 4 + k) * np + slot] = val;
      }
}

// ------------------------------------------------------------------ gather

__global__ void k_gather(const Tile* __restrict__ tiles, const Job* __restrict__ jobs,
                         const Dof* __restrict__ dofs, const int* __restrict__ pos,
                         const c64* __restrict__ res, int64_t np, c64* __restrict__ out) {
  const Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count) return;
  const Job jb = jobs[t.job];
  const int64_t item = t.start + threadIdx.x;
  // consecutive threads: consecutive output entries and pair results
  const bool rf = job_rows_fast(jb);
  const int r = (int)(rf ? item % jb.nrd : item / jb.ncd), c = (int)(rf ? item / jb.nrd : item % jb.ncd);
  const Dof dr = dofs[jb.rd_off + r];
  const Dof dc = dofs[jb.cd_off + c];
  const int k = dr.comp * 2 + dc.comp;
  c64 s = cmk(0, 0);
  // node is local node 1 of eL and local node 0 of eR
  const int ier[2] = {dr.eL, dr.eR}, ia[2] = {1, 0};
  const int jec[2] = {dc.eL, dc.eR}, jb2[2] = {1, 0};
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int64_t slot = pair_slot(jb, ier[x], jec[y]);
      // each pair result is read once: a streaming (non-temporal) load
      const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(res + (ia[x] * 8 + jb2[y] * 4 + k) * np + slot));
      s.re += v.x;
      s.im += v.y;
    }
  const int64_t rp = jb.rpos_off >= 0 ? pos[jb.rpos_off + r] : r;
  const int64_t cp = jb.cpos_off >= 0 ? pos[jb.cpos_off + c] : c;
  out[jb.out_off + rp * jb.rs + cp * jb.cs] = s;
}

// ------------------------------------------------------------------ load vectors
// f[2 t + i] for node t: both elements of its hat, 6-point Gauss each.
__global__ void k_rhs_plane(const Elem* __restrict__ elems, const int* __restrict__ prev_elem, int n_nodes,
                            MatConst m, double lam, int nrhs, const int* __restrict__ kind,
                            const double* __restrict__ ang, c64* __restrict__ out, int64_t ld) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (t >= n_nodes || k >= nrhs) return;
  double sd, cd;
  sincos(ang[k], &sd, &cd);
  const int kd = kind[k];
  const double wn = kd == 0 ? m.kL : m.kT;
  const c64 al = cmk(m.alpha_re, m.alpha_im);
  c64 f0 = cmk(0, 0), f1 = cmk(0, 0);
  const int els[2] = {prev_elem[t], t};
  for (int s = 0; s < 2; ++s) {
    const Elem e = elems[els[s]];
    for (int q = 0; q < 6; ++q) {
      const double u = c_quad.rg[q];
      const double N = s == 0 ? u : 1.0 - u;     // node is local 1 of the previous element
      const double w = c_quad.rw[q] * e.h * N;
      const double x = e.x0 + u * (e.x1 - e.x0), y = e.y0 + u * (e.y1 - e.y0);
      double sp, cp;
      sincos(wn * (x * cd + y * sd), &sp, &cp);
      const c64 E = cmk(cp, sp);
      const double nd = e.nx * cd + e.ny * sd;
      c64 u0, u1, t0, t1;
      if (kd == 0) {
        // u = d E;  T u = i k_L E (lambda n + 2 mu (n.d) d)
        u0 = cd * E;
        u1 = sd * E;
        const c64 ikE = mul_i(m.kL * E);
        t0 = (lam * e.nx + 2.0 * m.mu * nd * cd) * ikE;
        t1 = (lam * e.ny + 2.0 * m.mu * nd * sd) * ikE;
      } else {
        // u = (J d) E;  T u = i k_T mu E ((n.d) J d + (n.J d) d)
        const double dpx = -sd, dpy = cd;
        const double ndp = e.nx * dpx + e.ny * dpy;
        u0 = dpx * E;
        u1 = dpy * E;
        const c64 ikE = mul_i((m.kT * m.mu) * E);
        t0 = (nd * dpx + ndp * cd) * ikE;
        t1 = (nd * dpy + ndp * sd) * ikE;
      }
      f0 += w * (u0 + al * t0);
      f1 += w * (u1 + al * t1);
    }
  }
  out[(int64_t)k * ld + 2 * t] = f0;
  out[(int64_t)k * ld + 2 * t + 1] = f1;
}

// ------------------------------------------------------------------ special-function probe
__global__ void k_special_eval(const double* __restrict__ x, int64_t n, double beta, double* __restrict__ out,
                               c64* __restrict__ outc) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  double j0, j1, y0, y1;
  bessel_jy01(x[k], j0, j1, y0, y1);
  out[4 * k] = j0;
  out[4 * k + 1] = j1;
  out[4 * k + 2] = y0;
  out[4 * k + 3] = y1;
  const Hankel2 h = hankel_pair(x[k], beta * x[k]);
  c64 E, chi;
  e_chi(x[k], beta, h, E, chi);
  outc[2 * k] = E;
  outc[2 * k + 1] = chi;
}

// ------------------------------------------------------------------ host launchers
void upload_quad_tables(const QuadTables& q) { FDS_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_quad), &q, sizeof(q))); }

void launch_elem_geometry(const double* xy, const int* curve_of, const int* curve_off, const int* curve_n,
                          int n_elem, Elem* out, hipStream_t s) {
  k_elem_geometry<<<(n_elem + 255) / 256, 256, 0, s>>>(xy, curve_of, curve_off, curve_n, n_elem, out);
  FDS_HIP(hipGetLastError());
}

void launch_proxy_elems(const double* crd, const int* poff, int n_cells, int total, int poly_base, Elem* out,
                        hipStream_t s) {
  if (total == 0 || n_cells == 0) return;
  k_proxy_elems<<<(total + 255) / 256, 256, 0, s>>>(crd, poff, n_cells, total, poly_base, out);
  FDS_HIP(hipGetLastError());
}

void launch_classify(const Tile* tiles, int n_tiles, const Job* jobs, const int* elist, const Elem* elems,
                     unsigned long long* lists, int64_t cap, unsigned int* counters, double kT, hipStream_t s) {
  if (n_tiles == 0) return;
  k_classify<<<n_tiles, 256, 0, s>>>(tiles, jobs, elist, elems, lists, cap, counters, kT);
  FDS_HIP(hipGetLastError());
}

int classify_tile_size() { return kClsTile; }

// Class list lengths stay on the device (``counts``); grids are sized from
// the batch's pair count and the kernels stride over their list.
void launch_pairs(const unsigned long long* lists, int64_t cap, const unsigned int* counts, const Job* jobs,
                  const int* elist, const Elem* elems, const MatConst& m, c64* res, int64_t np, hipStream_t s,
                  hipEvent_t* ev) {
  // ev (optional): kNumPairLaunches + 1 events bracketing the launches in order
  auto mark = [&](int i) {
    if (ev) FDS_HIP(hipEventRecord(ev[i], s));
  };
  const unsigned greg = (unsigned)std::min<int64_t>((np + 127) / 128, 4096);
  const unsigned gspc = (unsigned)std::min<int64_t>((np + 3) / 4, 2048);
  mark(0);
  k_regular<0, false><<<greg, 128, 0, s>>>(lists, cap, counts, jobs, elist, elems, m, res, np);
  mark(1);
  k_regular<0, true><<<greg, 128, 0, s>>>(lists, cap, counts, jobs, elist, elems, m, res, np);
  mark(2);
  k_regular<1, false><<<greg, 128, 0, s>>>(lists, cap, counts, jobs, elist, elems, m, res, np);
  mark(3);
  k_regular<1, true><<<greg, 128, 0, s>>>(lists, cap, counts, jobs, elist, elems, m, res, np);
  mark(4);
  k_regular<2, false><<<greg, 128, 0, s>>>(lists, cap, counts, jobs, elist, elems, m, res, np);
  mark(5);
  k_regular<2, true><<<greg, 128, 0, s>>>(lists, cap, counts, jobs, elist, elems, m, res, np);
  mark(6);
  k_regular<3, false><<<greg, 128, 0, s>>>(lists, cap, counts, jobs, elist, elems, m, res, np);
  mark(7);
  k_regular<3, true><<<greg, 128, 0, s>>>(lists, cap, counts, jobs, elist, elems, m, res, np);
  mark(8);
  k_regular_wave10<<<gspc, 256, 0, s>>>(lists + kQ10 * cap, counts + kQ10, jobs, elist, elems, m, res, np);
  mark(9);
  k_special<kCoinc><<<gspc, 256, 0, s>>>(lists + kCoinc * cap, counts + kCoinc, jobs, elist, elems, m, res, np);
  mark(10);
  k_special2<kAdjNext><<<gspc, 256, 0, s>>>(lists + kAdjNext * cap, counts + kAdjNext, jobs, elist, elems, m, res, np);
  mark(11);
  k_special2<kAdjPrev><<<gspc, 256, 0, s>>>(lists + kAdjPrev * cap, counts + kAdjPrev, jobs, elist, elems, m, res, np);
  mark(12);
  FDS_HIP(hipGetLastError());
}

void launch_gather(const Tile* tiles, int n_tiles, const Job* jobs, const Dof* dofs, const int* pos,
                   const c64* res, int64_t np, c64* out, hipStream_t s) {
  if (n_tiles == 0) return;
  k_gather<<<n_tiles, 256, 0, s>>>(tiles, jobs, dofs, pos, res, np, out);
  FDS_HIP(hipGetLastError());
}

void launch_rhs_plane(const Elem* elems, const int* prev_elem, int n_nodes, const MatConst& m, double lam, int nrhs,
                      const int* kind, const double* ang, c64* out, int64_t ld, hipStream_t s) {
  dim3 grid((n_nodes + 255) / 256, nrhs);
  k_rhs_plane<<<grid, 256, 0, s>>>(elems, prev_elem, n_nodes, m, lam, nrhs, kind, ang, out, ld);
  FDS_HIP(hipGetLastError());
}

void launch_special_eval(const double* x, int64_t n, double beta, double* out, c64* outc, hipStream_t s) {
  k_special_eval<<<(int)((n + 255) / 256), 256, 0, s>>>(x, n, beta, out, outc);
  FDS_HIP(hipGetLastError());
}

}  // namespace fds
