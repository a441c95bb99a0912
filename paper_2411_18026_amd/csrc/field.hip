// Field off the boundary by the integral representation (Section 3): for a
// point x of the solid and a boundary solution u (the P1 interpolant of its
// nodal values, Section 4),
//
//   u(x) = u^I(x) - int_Gamma K(x, y) u(y) ds(y),   K_ij = T^{n_y}_{jk} G_ik(x - y).
//
// K is used in the form the Galerkin assembly uses for the double-layer
// operator: the tangential-derivative part of the traction is moved onto
// the trial hat by integration by parts along the closed polygon (no end
// terms; x is off the polygon, so every integrand is smooth).  With
// Phi_k = (i/4) H0(k r), e = (x - y)/r, E and chi the scaled Hankel
// differences of special.hpp, per point y of an element with hat phi:
//
//   K phi  ->  phi' [(Phi_T - (i/2) E) J - (i/2) chi e (J e)^T]
//            + phi  [(d_{n_y} Phi_T) I + grad_y(Phi_L - Phi_T) n_y^T].
//
// Quadrature per (target, element), by the distance d from the target to
// the element and the element length h: Gauss-Legendre with 4 points for
// d >= 8 h, 6 for d >= 2 h, 10 for d >= h, and for d < h the element split
// into min(64, ceil(h / d)) panels of 10 points each.
//
// Work split: one wavefront per (target, run of 63 nodes of one curve).
// Lane 0 integrates the element that ends at the run's first node, lane
// l >= 1 the element that starts at node first + l - 1.  Each element's
// integral against its end hat moves one lane up, so node t gets
// (start-hat integral of element t) + (end-hat integral of the element
// before t), each element integrated once (one extra element per run).
// The entries go to E^T: row 2 t + j, column 2 m + i, so that a wavefront
// writes 63 consecutive 32-byte pairs per column.  The matrix-core GEMM
// (launch_zgemm_tn) then forms out = u^I - E X for all solutions at once.
#include <cmath>

#include "assembly.hpp"
#include "field.hpp"

namespace fds {

struct FieldQuad {
  double g4[4], w4[4], g6[6], w6[6], g10[10], w10[10];
};

__constant__ FieldQuad c_fq;

static bool g_field_quad_ready = false;

void ensure_field_quad() {
  if (g_field_quad_ready) return;
  const QuadTables q = make_quad_tables();
  FieldQuad f;
  for (int i = 0; i < 4; ++i) f.g4[i] = q.g4[i], f.w4[i] = q.w4[i];
  for (int i = 0; i < 6; ++i) f.g6[i] = q.g6[i], f.w6[i] = q.w6[i];
  for (int i = 0; i < 10; ++i) f.g10[i] = q.g10[i], f.w10[i] = q.w10[i];
  FDS_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_fq), &f, sizeof(f)));
  g_field_quad_ready = true;
}

std::vector<FieldRun> field_runs(const std::vector<int>& curve_off, const std::vector<int>& curve_n,
                                 const std::vector<int>& prev_node) {
  std::vector<FieldRun> runs;
  for (size_t c = 0; c < curve_off.size(); ++c)
    for (int l = 0; l < curve_n[c]; l += kFieldRunNodes) {
      const int first = curve_off[c] + l;
      runs.push_back(FieldRun{first, std::min(kFieldRunNodes, curve_n[c] - l), prev_node[first], 0});
    }
  return runs;
}

// The two 2 x 2 blocks multiplying phi' and phi at one point (d = x - y).
__device__ inline void field_point(const MatConst& m, double dx, double dy, double ny0, double ny1, c64 (&Md)[4],
                                   c64 (&Mv)[4]) {
  const double r = sqrt(dx * dx + dy * dy);
  const double ir = 1.0 / r;
  const double e0 = dx * ir, e1 = dy * ir;
  const double je[2] = {-e1, e0};
  const double ex[2] = {e0, e1};
  const double ny[2] = {ny0, ny1};
  const double a = m.kT * r;
  c64 h0a, h1a, h0b, E, chi;
  kernel_values(a, m.sc, h0a, h1a, h0b, E, chi);
  const c64 P = cmk(-0.25 * h0a.im + 0.5 * E.im, 0.25 * h0a.re - 0.5 * E.re);    // Phi_T - (i/2) E
  const c64 hc = cmk(-0.5 * chi.im, 0.5 * chi.re);                               // (i/2) chi
  const c64 dny = cmk(-0.25 * m.kT * h1a.im, 0.25 * m.kT * h1a.re) * (e0 * ny0 + e1 * ny1);
  const double ka = 0.25 * m.kT * a;
  const c64 cg = cmk(ka * E.im, -ka * E.re);                                     // grad_y dPhi = cg e
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double Jij = (i == j) ? 0.0 : (i == 0 ? -1.0 : 1.0);
      Md[2 * i + j] = Jij * P - (ex[i] * je[j]) * hc;
      Mv[2 * i + j] = ((i == j) ? 1.0 : 0.0) * dny + (ex[i] * ny[j]) * cg;
    }
}

// One quadrature point at parameter u with weight wt (element length
// included) added to the start-hat (As) and end-hat (Ae) integrals.
__device__ inline void field_accumulate(const MatConst& m, const Elem& e, double tx, double ty, double u, double wt,
                                        c64 (&As)[4], c64 (&Ae)[4]) {
  c64 Md[4], Mv[4];
  field_point(m, tx - (e.x0 + u * (e.x1 - e.x0)), ty - (e.y0 + u * (e.y1 - e.y0)), e.nx, e.ny, Md, Mv);
  const double c0 = wt * (1.0 - u), c1 = wt * u;
  const double d0 = wt * e.dN0, d1 = wt * e.dN1;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    As[q] += d0 * Md[q] + c0 * Mv[q];
    Ae[q] += d1 * Md[q] + c1 * Mv[q];
  }
}

// Integrals of K against the start hat (As) and the end hat (Ae) of
// element e for the target (tx, ty); returns whether the target is closer
// than h / 64.  When every lane of the wavefront takes the 4-point rule
// (the far field: nearly all pairs) the loop is unrolled with the rule
// read as wavefront-uniform constants; the arithmetic is the same.
__device__ inline bool field_element(const MatConst& m, const Elem& e, double tx, double ty, bool live,
                                     c64 (&As)[4], c64 (&Ae)[4]) {
  const double qx = e.x1 - e.x0, qy = e.y1 - e.y0;
  double s = ((tx - e.x0) * qx + (ty - e.y0) * qy) / (qx * qx + qy * qy);
  s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  const double px = e.x0 + s * qx - tx, py = e.y0 + s * qy - ty;
  const double d = sqrt(px * px + py * py);
  const double h = e.h;
  if (__ballot(live && !(d >= 8.0 * h)) == 0ull) {
    if (live) {
#pragma unroll
      for (int k = 0; k < 4; ++k) field_accumulate(m, e, tx, ty, c_fq.g4[k], c_fq.w4[k] * h, As, Ae);
    }
    return false;
  }
  if (!live) return false;
  const double* g;
  const double* w;
  int nq, np = 1;
  if (d >= 8.0 * h) {
    nq = 4, g = c_fq.g4, w = c_fq.w4;
  } else if (d >= 2.0 * h) {
    nq = 6, g = c_fq.g6, w = c_fq.w6;
  } else {
    nq = 10, g = c_fq.g10, w = c_fq.w10;
    if (d < h) np = d * kFieldMaxPanels > h ? (int)ceil(h / d) : kFieldMaxPanels;
  }
  const double inv = 1.0 / np;
  for (int p = 0; p < np; ++p)
    for (int k = 0; k < nq; ++k) field_accumulate(m, e, tx, ty, (p + g[k]) * inv, w[k] * h * inv, As, Ae);
  return d * kFieldMaxPanels < h;
}

// Two wavefronts per SIMD (214 registers, none spilled when the series and
// Bessel constants stay at their uses): the kernel values' long dependent chains
// need the second wavefront to hide their latency (8.6 ms against 9.8 ms
// for the whole field call of 4096 targets x 6400 nodes x 180 solutions at
// one wavefront per SIMD; the uniform 4-point path then took it from 7.7
// to 7.3 ms).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_field_matrix(const Elem* __restrict__ elems, const FieldRun* __restrict__ runs, const double* __restrict__ targets,
               int64_t m0, int mc, MatConst m, c64* __restrict__ Et, int64_t ld, unsigned int* __restrict__ near) {
  const int lane = threadIdx.x & 63;
  const int ml = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (ml >= mc) return;   // the whole wavefront
  const FieldRun run = runs[blockIdx.x];
  const int64_t mg = m0 + ml;
  const double tx = targets[2 * mg], ty = targets[2 * mg + 1];
  const int el = lane == 0 ? run.prev_elem : (lane <= run.count ? run.first + lane - 1 : -1);
  c64 As[4], Ae[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) As[q] = Ae[q] = cmk(0.0, 0.0);
  // every lane takes part (the rule choice is voted over the wavefront);
  // lanes past the run integrate nothing
  const bool close = field_element(m, elems[el >= 0 ? el : run.first], tx, ty, el >= 0, As, Ae);
  c64 Pe[4];   // end-hat integral of the element before this lane's node
#pragma unroll
  for (int q = 0; q < 4; ++q) Pe[q] = cmk(__shfl_up(Ae[q].re, 1), __shfl_up(Ae[q].im, 1));
  if (__ballot(close) != 0ull && lane == 0) near[mg] = 1u;
  if (lane >= 1 && lane <= run.count) {
    const int t = run.first + lane - 1;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      c64* col = Et + (int64_t)(2 * ml + i) * ld + 2 * (int64_t)t;
      col[0] = As[2 * i] + Pe[2 * i];
      col[1] = As[2 * i + 1] + Pe[2 * i + 1];
    }
  }
}

void launch_field_matrix(const Elem* elems, const FieldRun* runs, int n_runs, const double* targets, int64_t m0,
                         int mc, const MatConst& m, c64* Et, int64_t ld, unsigned int* near, hipStream_t s) {
  if (n_runs < 1 || mc < 1) return;
  const dim3 grid(n_runs, (mc + 3) / 4);
  k_field_matrix<<<grid, 256, 0, s>>>(elems, runs, targets, m0, mc, m, Et, ld, near);
  FDS_HIP(hipGetLastError());
}

__global__ void k_field_incident(const double* __restrict__ targets, int64_t n_target, MatConst m, int nrhs,
                                 const int* __restrict__ kind, const double* __restrict__ ang, c64* __restrict__ out,
                                 int64_t ld) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (t >= n_target || r >= nrhs) return;
  c64 u0 = cmk(0.0, 0.0), u1 = cmk(0.0, 0.0);
  if (kind) {
    double sd, cd;
    sincos(ang[r], &sd, &cd);
    const bool p = kind[r] == 0;
    double sp, cp;
    sincos((p ? m.kL : m.kT) * (targets[2 * t] * cd + targets[2 * t + 1] * sd), &sp, &cp);
    const c64 E = cmk(cp, sp);
    u0 = (p ? cd : -sd) * E;   // P: d E;  S: (J d) E
    u1 = (p ? sd : cd) * E;
  }
  out[r * ld + 2 * t] = u0;
  out[r * ld + 2 * t + 1] = u1;
}

void launch_field_incident(const double* targets, int64_t n_target, const MatConst& m, int nrhs, const int* kind,
                           const double* ang, c64* out, int64_t ld, hipStream_t s) {
  if (n_target < 1 || nrhs < 1) return;
  const dim3 grid((unsigned)((n_target + 255) / 256), nrhs);
  k_field_incident<<<grid, 256, 0, s>>>(targets, n_target, m, nrhs, kind, ang, out, ld);
  FDS_HIP(hipGetLastError());
}

}  // namespace fds
