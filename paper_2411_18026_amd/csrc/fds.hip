// Host driver and C ABI of the proxy-surface fast direct solver.
//
// Algorithm summary (Section 7.3):
//   1-2. binary tree of contiguous node ranges and leaf index sets (Section 5.1);
//   3.   for l = L ... l0+1: proxy-surface interaction matrices, IDs by
//        column-pivoted QR giving U_i, V_i and the skeletons (Sections 7.1,
//        7.2); A_i^{-1} U_i through the LU of A_i, A~_i = (V_i A_i^{-1} U_i)^{-1}
//        (Section 6.2); parent diagonal blocks from [[A~_a, R_ab], [R_ba, A~_b]]
//        in component-major order (rearrangement of Section 6.2);
//   4.   LU of the compressed system at level l0;
//   5.   the solve: upward sweep g_i = A_i^{-1} f_i, f~_i = A~_i V_i g_i,
//        root solve, downward sweep x_i = g_i + A_i^{-1} U_i (A~_i y_i - f~_i)
//        (equation of the downward conversion, Section 6.3).
//
// Readings where the paper leaves a choice:
//   * four skeleton sets per cell (rows / columns x component); rows and
//     columns of a component share the rank k_c = max(k_row, k_col) and take
//     the first k_c pivots of their pivoted QRs, so that A~_i is square;
//   * ID rank: first j with |R_jj| <= tol |R_11|;
//   * proxy: m-gon of radius rho = 1.5 R about the centre of the
//     bounding box of the supports of the cell's active hats, outward normal,
//     m = max(n_proxy, ceil(2 k_T rho) + 40) (an outgoing field on the circle
//     carries Fourier modes up to about k_T rho);
//   * near field: active DOFs of the other cells of the level whose hat
//     support meets the proxy disk.
// The host keeps only index bookkeeping (tree, DOF lists, near sets);
// every arithmetic step runs in the device kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <unordered_map>
#include <vector>
#include <cstdio>
#include <cstdlib>

#include "../../include/fds.h"
#include "assembly.hpp"
#include "devmem.hpp"
#include "field.hpp"
#include "learned.hpp"
#include "linalg.hpp"
#include "parallel.hpp"
#include "sweep.hpp"

namespace fds {

static bool g_quad_ready = false;
static void ensure_quad() {
  if (!g_quad_ready) {
    upload_quad_tables(make_quad_tables());
    g_quad_ready = true;
  }
}

struct Geometry {
  int n_nodes = 0, n_curves = 0;
  std::vector<int> curve_off, curve_n, curve_of;
  std::vector<double> xy;
  std::vector<int> prev_node, next_node;   // neighbours along the curve
  double hmax = 0.0;
};

static int make_geometry(const fds_geometry* g, Geometry& G) {
  if (!g || g->n_curves < 1 || !g->n_nodes || !g->xy) return FDS_EINVAL;
  G.n_curves = g->n_curves;
  G.curve_off.resize(g->n_curves);
  G.curve_n.resize(g->n_curves);
  int64_t tot = 0;
  for (int c = 0; c < g->n_curves; ++c) {
    if (g->n_nodes[c] < 8) return FDS_EGEOM;
    G.curve_off[c] = (int)tot;
    G.curve_n[c] = g->n_nodes[c];
    tot += g->n_nodes[c];
  }
  if (tot > (1 << 29)) return FDS_EINVAL;
  G.n_nodes = (int)tot;
  G.xy.assign(g->xy, g->xy + 2 * tot);
  G.curve_of.resize(tot);
  G.prev_node.resize(tot);
  G.next_node.resize(tot);
  for (int c = 0; c < g->n_curves; ++c) {
    const int o = G.curve_off[c], n = G.curve_n[c];
    double area = 0.0;
    for (int l = 0; l < n; ++l) {
      const int t = o + l, t1 = o + (l + 1) % n;
      G.curve_of[t] = c;
      G.prev_node[t] = o + (l + n - 1) % n;
      G.next_node[t] = t1;
      const double dx = G.xy[2 * t1] - G.xy[2 * t], dy = G.xy[2 * t1 + 1] - G.xy[2 * t + 1];
      const double h = std::sqrt(dx * dx + dy * dy);
      if (!(h > 0.0) || !std::isfinite(h)) return FDS_EGEOM;
      G.hmax = std::max(G.hmax, h);
      area += G.xy[2 * t] * G.xy[2 * t1 + 1] - G.xy[2 * t1] * G.xy[2 * t + 1];
    }
    if (area <= 0.0) return FDS_EGEOM;
  }
  return FDS_OK;
}

static MatConst make_mat(double omega, double lam, double mu, double rho, const fds_options& o, double* alpha_re,
                         double* alpha_im) {
  MatConst m{};
  const double cL = std::sqrt((lam + 2.0 * mu) / rho), cT = std::sqrt(mu / rho);
  m.kL = omega / cL;
  m.kT = omega / cT;
  m.ikT = 1.0 / m.kT;
  m.beta = m.kL / m.kT;
  m.mu = mu;
  m.rw2 = rho * omega * omega;
  m.sc = make_series_coef(m.beta);
  if (o.use_alpha) {
    m.alpha_re = o.alpha.re;
    m.alpha_im = o.alpha.im;
  } else {
    m.alpha_re = 0.0;
    m.alpha_im = 1.0 / (mu * m.kT);
  }
  if (alpha_re) *alpha_re = m.alpha_re;
  if (alpha_im) *alpha_im = m.alpha_im;
  return m;
}

// device copy of the boundary elements (+ room for proxies)
struct DevGeom {
  DevBuf<double> xy;
  DevBuf<int> curve_of, curve_off, curve_n, prev_elem;
  DevBuf<Elem> elems;
  int n_gamma = 0;
  int64_t cap = 0;
  void init(const Geometry& G, int64_t proxy_cap, hipStream_t s) {
    n_gamma = G.n_nodes;
    xy = DevBuf<double>(G.xy);
    curve_of = DevBuf<int>(G.curve_of);
    curve_off = DevBuf<int>(G.curve_off);
    curve_n = DevBuf<int>(G.curve_n);
    std::vector<int> pe(G.n_nodes);
    for (int t = 0; t < G.n_nodes; ++t) pe[t] = G.prev_node[t];   // element ending at t starts at prev(t)
    prev_elem = DevBuf<int>(pe);
    cap = G.n_nodes + proxy_cap;
    elems = DevBuf<Elem>((size_t)cap);
    launch_elem_geometry(xy.p, curve_of.p, curve_off.p, curve_n.p, G.n_nodes, elems.p, s);
  }
  // room for at least ``need`` elements (boundary elements kept)
  void reserve(int64_t need, hipStream_t s) {
    if (need <= cap) return;
    DevBuf<Elem> grown((size_t)need);
    FDS_HIP(hipMemcpyAsync(grown.p, elems.p, (size_t)n_gamma * sizeof(Elem), hipMemcpyDeviceToDevice, s));
    FDS_HIP(hipStreamSynchronize(s));
    elems = std::move(grown);
    cap = need;
  }
};

// Side of a block from a list of boundary DOFs (2 t + i).  A per-thread slot
// array over the boundary elements deduplicates the elements of the hats.
static Side side_from_dofs(const Geometry& G, const std::vector<int64_t>& dofs) {
  static thread_local std::vector<int> slot;
  if ((int)slot.size() < G.n_nodes) slot.assign(G.n_nodes, -1);
  Side sd;
  sd.elems.reserve(dofs.size() + 2);
  auto get = [&](int e) {
    int& s = slot[e];
    if (s < 0) {
      s = (int)sd.elems.size();
      sd.elems.push_back(e);
    }
    return s;
  };
  sd.dofs.reserve(dofs.size());
  for (int64_t d : dofs) {
    const int t = (int)(d >> 1);
    const int eL = get(G.prev_node[t]);   // element (prev(t), t)
    const int eR = get(t);                // element (t, next(t))
    sd.dofs.push_back(Dof{eL, eR, (int)(d & 1), 0});
  }
  for (int e : sd.elems) slot[e] = -1;
  return sd;
}

// Append the DOFs of a proxy polygon (all n_proxy nodes, component-major) to a side.
static void side_add_proxy(Side& sd, int elem_base, int n_proxy) {
  const int b = (int)sd.elems.size();
  for (int s = 0; s < n_proxy; ++s) sd.elems.push_back(elem_base + s);
  for (int c = 0; c < 2; ++c)
    for (int s = 0; s < n_proxy; ++s) sd.dofs.push_back(Dof{b + (s + n_proxy - 1) % n_proxy, b + s, c, 0});
}

static void side_append(const Geometry& G, Side& sd, const std::vector<int64_t>& dofs) {
  Side add = side_from_dofs(G, dofs);
  const int b = (int)sd.elems.size();
  sd.elems.insert(sd.elems.end(), add.elems.begin(), add.elems.end());
  for (auto d : add.dofs) sd.dofs.push_back(Dof{d.eL + b, d.eR + b, d.comp, 0});
}


// ------------------------------------------------------------------ factor data
// Device-resident solve plan of one compressed level (built once per factor).
struct SolveLevel {
  // arrays in the factor's plan arena
  DevView<SolveDesc> lu;                       // g_i = A_i^{-1} f_i (ncol given at solve time)
  DevView<GemmDesc> g_v, g_at, g_dn1, g_dn2;   // V g, A~ (V g), A~ y - f~, g + X f~
  DevView<GemmTile> t_v, t_at, t_dn1, t_dn2;
  int n_lu = 0, n_tv = 0, n_tat = 0, n_tdn1 = 0, n_tdn2 = 0, bmax = 0;
  DevView<GemmDesc> g_w;                       // matrix-core levels: f~ = W g (W = A~ V), for few columns
  DevView<GemmTile> t_w;
  int n_tw = 0;
  DevView<int64_t> up_src, up_dst;             // rows of f~ -> rows of the parent's F
  int64_t n_up = 0;
};

struct CellLevel {
  int lev = 0, n = 0;                            // cells 2^lev - 1 + q, q < n
  std::vector<std::vector<int64_t>> rows, cols;  // active DOFs (component-major)
  std::vector<int> b, n0;                        // sizes, # component-0 DOFs
  std::vector<int64_t> a_off;                    // A_i / LU(A_i) (ld = b)
  std::vector<int64_t> piv_off;
  int64_t a_tot = 0, piv_tot = 0;
  int bmax = 0;
  int max_proxy = 0;                             // largest proxy polygon of the level
  // compression results (levels > l0)
  std::vector<int> k0, k1, r;
  std::vector<int> kr0, kc0, kr1, kc1;           // ranks at tolerance
  std::vector<std::vector<int64_t>> rskel, cskel;
  std::vector<int64_t> x_off, at_off, v_off, s_piv_off;
  int64_t x_tot = 0, at_tot = 0, v_tot = 0, s_piv_tot = 0;
  // plain form: A = LU(A_i), X = A_i^{-1} U_i, At = A~_i, V = V_i.
  // mixed form: A = the FP64 diagonal block without the children's A~
  // (the full A_i at the leaves), X = U_i, V = V_i (all FP64, for the
  // compressed-operator product); A32 = LU(A_i), X32 = A_i^{-1} U_i,
  // At32 = A~_i, V32 = V_i in FP32.
  DevBuf<c64> A, X, At, V;
  DevBuf<c32> A32, X32, At32, V32;
  DevBuf<int> piv, s_piv;
  // solve layout: level vector of height B = sum b, skeleton height R = sum r
  std::vector<int64_t> f_off, t_off;
  int64_t B = 0, R = 0;
  // parent position of each skeleton entry (set when the parent is built)
  std::vector<std::vector<int>> ppos;
  SolveLevel plan;
  // matrix-core sweeps (plain FP64 form, levels whose blocks have a
  // variant): per-cell descriptors, composed LU permutations, inverted 16 x 16
  // diagonal blocks; V then holds W = A~ V (the upward sweep's product)
  bool mfma = false;
  int nb_class = 0, nr_class = 0;
  DevView<SweepCell> sweep;   // in the factor's plan arena
  DevBuf<int> perm;
  DevBuf<c64> Dinv;
  // compressed-operator product (mixed form): y = B z per cell
  DevView<GemmDesc> g_diag;   // in the factor's plan arena
  DevView<GemmTile> t_diag;
  int n_tdiag = 0;
};

// Compressed system at l0: diagonal blocks are the cells' A_i, the rest are
// original entries; one LU.
struct Root {
  int n = 0;
  DevBuf<c64> A;
  DevBuf<c64> B;            // mixed form: the root system without the children's A~
  DevBuf<GemmDesc> g_b;
  DevBuf<GemmTile> t_b;
  int n_tb = 0;
  DevBuf<int> piv;
  DevBuf<SolveDesc> desc;
};

struct TimedSpan {
  hipEvent_t a, b;
  int what;   // 0 id, 1 merge, 2 root
};

}  // namespace fds

struct fds_factor_s {
  fds::Geometry G;
  fds::DevGeom DG;
  fds::MatConst m{};
  fds_options opt{};
  double tol = 0, lam = 0, mu = 0, rho = 0, omega = 0;
  int L = 0, l0 = 0;
  std::vector<fds::CellLevel> levels;   // index = level
  fds::Root root;
  fds::AssemblyStats ast;
  std::vector<fds::TimedSpan> spans;
  fds_stats st{};
  hipStream_t stream = nullptr;
  fds::Workspace ws;
  fds::ArenaBuilder plan_ab;                // host side of plan_arena while the factorisation runs
  fds::DevBuf<unsigned char> plan_arena;    // the solve's descriptors and row maps (one allocation)
  fds::DevBuf<unsigned char> plan_arena_sweep;   // the same, added before the matrix-core sweep preparation
  fds::DevView<int64_t> leaf_dofs_rows, leaf_dofs_cols, leaf_iota;
  fds::DevBuf<float> pred;                  // learned form: predictor blob
  fds::DevBuf<int> sing;                    // per level: a block LU met a zero pivot
  int tune_chunk[4] = {0, 0, 0, 0};         // autotuned LU-solve columns per workgroup per nrhs class
  int tune_bn[4] = {64, 64, 64, 64};        // autotuned GEMM tile width per nrhs class
  float* pred_host = nullptr;               // learned form: pinned copy of a level's predictions
  size_t pred_host_n = 0, pred_host_bytes = 0;
  hipEvent_t pred_ev = nullptr;
  std::vector<fds_rank_record> rank_log;    // per compressed cell: features, ranks, prediction
  // the next level to compress, prepared ahead (disks, interaction matrices)
  struct LevelPrep {
    int lev = -1;
    std::vector<double> crd;                 // per cell: centre x, y and proxy radius
    std::vector<int> mv_m, mu_m;             // rows of M^V, M^U^T per cell
    std::vector<int64_t> mv_off, mu_off;
    fds::c64* MV = nullptr;
    fds::c64* MU = nullptr;
  } prep;
  std::map<int64_t, hipGraphExec_t> graphs; // captured solve sweeps per (nrhs, kind)
  hipStream_t gstream = nullptr;            // library stream for graph capture and replay
  ~fds_factor_s() {
    if (pred_host) {
      if (pred_ev) (void)hipEventSynchronize(pred_ev);
      fds::pinned_free(pred_host, pred_host_bytes);
    }
    if (pred_ev) (void)hipEventDestroy(pred_ev);
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (gstream) {
      (void)hipStreamSynchronize(gstream);
      (void)hipStreamDestroy(gstream);
    }
    for (auto& sp : spans) {
      (void)hipEventDestroy(sp.a);
      (void)hipEventDestroy(sp.b);
    }
  }
};

namespace fds {

using Factor = fds_factor_s;

static void span_begin(Factor& F, int what) {
  TimedSpan sp{};
  FDS_HIP(hipEventCreate(&sp.a));
  FDS_HIP(hipEventCreate(&sp.b));
  sp.what = what;
  FDS_HIP(hipEventRecord(sp.a, F.stream));
  F.spans.push_back(sp);
}

static void span_end(Factor& F) { FDS_HIP(hipEventRecord(F.spans.back().b, F.stream)); }

// Curves in Morton (Z-order) order of their bounding-box centres: each
// coordinate scaled to the bounding box of the centres, quantised to 16 bits,
// bits interleaved with x in the even positions; equal codes keep input order.
static std::vector<int> morton_order(const Geometry& G) {
  const int nc = G.n_curves;
  std::vector<double> cx(nc), cy(nc);
  for (int c = 0; c < nc; ++c) {
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int t = G.curve_off[c]; t < G.curve_off[c] + G.curve_n[c]; ++t) {
      x0 = std::min(x0, G.xy[2 * t]);
      x1 = std::max(x1, G.xy[2 * t]);
      y0 = std::min(y0, G.xy[2 * t + 1]);
      y1 = std::max(y1, G.xy[2 * t + 1]);
    }
    cx[c] = 0.5 * (x0 + x1);
    cy[c] = 0.5 * (y0 + y1);
  }
  std::vector<int> order(nc);
  std::iota(order.begin(), order.end(), 0);
  if (nc <= 1) return order;
  const double lx = *std::min_element(cx.begin(), cx.end()), hx = *std::max_element(cx.begin(), cx.end());
  const double ly = *std::min_element(cy.begin(), cy.end()), hy = *std::max_element(cy.begin(), cy.end());
  const double sx = hx > lx ? hx - lx : 1.0, sy = hy > ly ? hy - ly : 1.0;
  std::vector<uint64_t> code(nc, 0);
  for (int c = 0; c < nc; ++c) {
    const int64_t qx = std::min<int64_t>(65535, std::max<int64_t>(0, (int64_t)std::floor((cx[c] - lx) / sx * 65535.0)));
    const int64_t qy = std::min<int64_t>(65535, std::max<int64_t>(0, (int64_t)std::floor((cy[c] - ly) / sy * 65535.0)));
    for (int b = 0; b < 16; ++b) {
      code[c] |= (uint64_t)((qx >> b) & 1) << (2 * b);
      code[c] |= (uint64_t)((qy >> b) & 1) << (2 * b + 1);
    }
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return code[a] < code[b]; });
  return order;
}

// Complete binary tree of depth L = ceil(log2(N / leaf)) (Section 5.1) over
// a node numbering that takes the curves in Morton order: a cell holding two
// or more whole curves splits its curve list into two groups of node counts
// as equal as possible (curves kept whole, ties to the first split); a cell
// within one curve splits its node range at the midpoint.
static void build_tree(Factor& F) {
  const Geometry& G = F.G;
  const int N = G.n_nodes, leaf = F.opt.leaf_nodes;
  int L = 0;
  while (((int64_t)leaf << L) < N) ++L;
  F.L = L;
  F.l0 = std::min(F.opt.root_level, L);
  F.levels.resize(L + 1);
  const std::vector<int> order = morton_order(G);
  const int nc = G.n_curves;
  std::vector<int> perm;
  std::vector<int64_t> pstart(nc + 1, 0);
  perm.reserve(N);
  for (int k = 0; k < nc; ++k) {
    const int c = order[k];
    for (int t = 0; t < G.curve_n[c]; ++t) perm.push_back(G.curve_off[c] + t);
    pstart[k + 1] = pstart[k] + G.curve_n[c];
  }
  struct Range {
    int lo, hi, ca, cb;   // node range; whole curves [ca, cb) or ca = -1 within one curve
  };
  std::vector<Range> cur{{0, N, 0, nc}};
  for (int lev = 0; lev < L; ++lev) {
    std::vector<Range> nxt;
    for (const Range& r : cur) {
      int mid;
      Range a{}, b{};
      if (r.ca >= 0 && r.cb - r.ca >= 2) {
        int sp = r.ca + 1;
        int64_t best = INT64_MAX;
        for (int k = r.ca + 1; k < r.cb; ++k) {
          const int64_t d = std::llabs(2 * (pstart[k] - r.lo) - (int64_t)(r.hi - r.lo));
          if (d < best) {
            best = d;
            sp = k;
          }
        }
        mid = (int)pstart[sp];
        a = Range{r.lo, mid, r.ca, sp};
        b = Range{mid, r.hi, sp, r.cb};
      } else {
        mid = r.lo + (r.hi - r.lo) / 2;
        a = Range{r.lo, mid, -1, -1};
        b = Range{mid, r.hi, -1, -1};
      }
      if (mid == r.lo || mid == r.hi) throw Error(FDS_EGEOM, "a tree cell would have no nodes: use a larger leaf size");
      nxt.push_back(a);
      nxt.push_back(b);
    }
    cur.swap(nxt);
  }
  CellLevel& lv = F.levels[L];
  lv.lev = L;
  lv.n = (int)cur.size();
  lv.rows.resize(lv.n);
  for (int q = 0; q < lv.n; ++q) {
    auto& rw = lv.rows[q];
    for (int c = 0; c < 2; ++c)
      for (int p = cur[q].lo; p < cur[q].hi; ++p) rw.push_back(2 * (int64_t)perm[p] + c);
  }
  lv.cols = lv.rows;
}

static void layout_blocks(CellLevel& lv) {
  lv.b.resize(lv.n);
  lv.n0.resize(lv.n);
  lv.a_off.resize(lv.n);
  lv.piv_off.resize(lv.n);
  lv.f_off.resize(lv.n);
  lv.a_tot = lv.piv_tot = lv.B = 0;
  lv.bmax = 0;
  for (int q = 0; q < lv.n; ++q) {
    lv.b[q] = (int)lv.rows[q].size();
    lv.bmax = std::max(lv.bmax, lv.b[q]);
    int c0 = 0;
    for (auto d : lv.cols[q]) c0 += (d & 1) == 0;
    lv.n0[q] = c0;
    lv.a_off[q] = lv.a_tot;
    lv.a_tot += (int64_t)lv.b[q] * lv.b[q];
    lv.piv_off[q] = lv.piv_tot;
    lv.piv_tot += lv.b[q];
    lv.f_off[q] = lv.B;
    lv.B += lv.b[q];
  }
  lv.A = DevBuf<c64>((size_t)std::max<int64_t>(lv.a_tot, 1));
  lv.piv = DevBuf<int>((size_t)std::max<int64_t>(lv.piv_tot, 1));
}

// Host wall-time of the factorisation's phases (printed when FDS_TIMING is set).
static double g_host_t[9];
static const char* g_host_name[9] = {"disks+near", "interaction requests", "device waits", "parent merge",
                                     "leaf blocks", "root", "solve plan", "other", "  of which packing+launch"};
struct HostTimer {
  int k;
  std::chrono::steady_clock::time_point t0;
  explicit HostTimer(int kk) : k(kk), t0(std::chrono::steady_clock::now()) {}
  ~HostTimer() { g_host_t[k] += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

// support nodes of a DOF list (prev, node, next)
static void cell_disk(const Geometry& G, const std::vector<int64_t>& rows, const std::vector<int64_t>& cols,
                      double& cx, double& cy, double& R) {
  double lox = 1e300, loy = 1e300, hix = -1e300, hiy = -1e300;
  std::vector<int> pts;
  pts.reserve(3 * (rows.size() + cols.size()));
  auto add = [&](int64_t d) {
    const int t = (int)(d >> 1);
    pts.push_back(G.prev_node[t]);
    pts.push_back(t);
    pts.push_back(G.next_node[t]);
  };
  for (auto d : rows) add(d);
  for (auto d : cols) add(d);
  for (int t : pts) {
    lox = std::min(lox, G.xy[2 * t]);
    hix = std::max(hix, G.xy[2 * t]);
    loy = std::min(loy, G.xy[2 * t + 1]);
    hiy = std::max(hiy, G.xy[2 * t + 1]);
  }
  cx = 0.5 * (lox + hix);
  cy = 0.5 * (loy + hiy);
  R = 0.0;
  for (int t : pts) R = std::max(R, std::hypot(G.xy[2 * t] - cx, G.xy[2 * t + 1] - cy));
}

static double seg_dist(double px, double py, double ax, double ay, double bx, double by) {
  const double dx = bx - ax, dy = by - ay;
  double t = ((px - ax) * dx + (py - ay) * dy) / (dx * dx + dy * dy);
  t = std::min(1.0, std::max(0.0, t));
  return std::hypot(ax + t * dx - px, ay + t * dy - py);
}

// does the hat support of node t meet the disk (c, rho)?
static bool support_meets(const Geometry& G, int t, double cx, double cy, double rho) {
  const int p = G.prev_node[t], n = G.next_node[t];
  const double* X = G.xy.data();
  return seg_dist(cx, cy, X[2 * p], X[2 * p + 1], X[2 * t], X[2 * t + 1]) < rho ||
         seg_dist(cx, cy, X[2 * t], X[2 * t + 1], X[2 * n], X[2 * n + 1]) < rho;
}

// uniform grid over the nodes for near-field queries
struct NodeGrid {
  double x0 = 0, y0 = 0, hx = 1;
  int nx = 1, ny = 1;
  std::vector<int> start, items;
  // bins the listed nodes only (a level's near sets can only hold nodes that
  // still carry an active DOF)
  void build(const Geometry& G, const std::vector<int>& nodes, double cell) {
    double lox = 1e300, loy = 1e300, hix = -1e300, hiy = -1e300;
    for (int t : nodes) {
      lox = std::min(lox, G.xy[2 * t]);
      hix = std::max(hix, G.xy[2 * t]);
      loy = std::min(loy, G.xy[2 * t + 1]);
      hiy = std::max(hiy, G.xy[2 * t + 1]);
    }
    if (nodes.empty()) lox = loy = hix = hiy = 0.0;
    hx = std::max(cell, 1e-12);
    nx = std::max(1, std::min(4096, (int)std::ceil((hix - lox) / hx) + 1));
    ny = std::max(1, std::min(4096, (int)std::ceil((hiy - loy) / hx) + 1));
    hx = std::max(hx, std::max((hix - lox) / (nx - 0.5), (hiy - loy) / (ny - 0.5)));
    x0 = lox;
    y0 = loy;
    std::vector<int> cnt((size_t)nx * ny + 1, 0);
    std::vector<int> bin(nodes.size());
    for (size_t i = 0; i < nodes.size(); ++i) {
      const int t = nodes[i];
      const int ix = std::min(nx - 1, (int)((G.xy[2 * t] - x0) / hx));
      const int iy = std::min(ny - 1, (int)((G.xy[2 * t + 1] - y0) / hx));
      bin[i] = iy * nx + ix;
      cnt[bin[i] + 1]++;
    }
    for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
    start = cnt;
    items.resize(nodes.size());
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (size_t i = 0; i < nodes.size(); ++i) items[fill[bin[i]]++] = nodes[i];
  }
  template <typename F>
  void query(double cx, double cy, double rad, F&& f) const {
    const int ix0 = std::max(0, (int)std::floor((cx - rad - x0) / hx));
    const int ix1 = std::min(nx - 1, (int)std::floor((cx + rad - x0) / hx));
    const int iy0 = std::max(0, (int)std::floor((cy - rad - y0) / hx));
    const int iy1 = std::min(ny - 1, (int)std::floor((cy + rad - y0) / hx));
    for (int iy = iy0; iy <= iy1; ++iy)
      for (int ix = ix0; ix <= ix1; ++ix) {
        const int b = iy * nx + ix;
        for (int k = start[b]; k < start[b + 1]; ++k) f(items[k]);
      }
  }
};

template <typename T>
static std::vector<T> download(Workspace& ws, const T* d, size_t n) {
  HostTimer ht(2);
  std::vector<T> h(n);
  if (n) {
    FDS_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, ws.stream()));
    FDS_HIP(hipStreamSynchronize(ws.stream()));
  }
  return h;
}

// Children's A~ (level lev + 1) into the diagonal blocks of level lev at
// their parent positions: block p starts at dst_off(p), leading dimension
// dst_ld(p).  TS -> TD converts on the fly.
template <typename TS, typename TD, typename Off, typename Ld>
static void place_child_at_t(Factor& F, int lev, Off dst_off, Ld dst_ld, const TS* src, TD* dst, const char* tag) {
  CellLevel& ch = F.levels[lev + 1];
  const int np = F.levels[lev].n;
  std::vector<int> pos;
  std::vector<ScatterDesc> sc;
  for (int p = 0; p < np; ++p)
    for (int side = 0; side < 2; ++side) {
      const int c = 2 * p + side;
      if (ch.r[c] == 0) continue;
      ScatterDesc d{};
      d.src_off = ch.at_off[c];
      d.src_ld = ch.r[c];
      d.nr = ch.r[c];
      d.nc = ch.r[c];
      d.dst_off = dst_off(p);
      d.dst_ld = dst_ld(p);
      d.rpos_off = (int)pos.size();
      pos.insert(pos.end(), ch.ppos[c].begin(), ch.ppos[c].end());
      d.cpos_off = d.rpos_off;
      sc.push_back(d);
    }
  if (pos.empty()) pos.push_back(0);
  const std::string t(tag);
  auto st = scatter_tiles(sc);
  launch_scatter(F.ws.upload("pca_desc" + t, sc), F.ws.upload("pca_tiles" + t, st), (int)st.size(),
                 F.ws.upload("pca_pos" + t, pos), src, dst, F.stream);
}

template <typename Off, typename Ld>
static void place_child_at(Factor& F, int lev, Off dst_off, Ld dst_ld, c32* dst, const char* tag) {
  place_child_at_t(F, lev, dst_off, dst_ld, F.levels[lev + 1].At32.p, dst, tag);
}

// Inverse-free elimination of one level (Section 6.2) in the scalar type of
// right-hand-side columns per workgroup of the elimination's triangular
// solves (many columns: the updates run as small GEMMs): 32 where the
// staged block fits in LDS, else 16, else the default
static int elim_chunk(int nmax, size_t elem) {
  for (int c : {32, 16})
    if (lu_solve_smem(nmax, c, elem) <= 65536) return c;
  return 0;
}

// the buffers: LU(A_i) in place; X_i <- A_i^{-1} X_i; S_i = V_i X_i; LU(S_i);
// At_i = S_i^{-1} (the LU of S_i applied to the identity).
template <typename T>
static void eliminate(Factor& F, CellLevel& lv, int rmax, T* A, T* X, T* V, T* At, const std::string& tag) {
  Workspace& ws = F.ws;
  hipStream_t s = F.stream;
  const int n = lv.n;
  std::vector<LUDesc> ld(n);
  std::vector<SolveDesc> sd;
  for (int q = 0; q < n; ++q) {
    ld[q] = LUDesc{lv.a_off[q], lv.piv_off[q], lv.b[q], lv.b[q]};
    if (lv.r[q] > 0)
      sd.push_back(SolveDesc{lv.a_off[q], lv.piv_off[q], lv.x_off[q], lv.b[q], lv.b[q], lv.b[q], lv.r[q]});
  }
  int* info = ws.get<int>("lu_info", (size_t)n);
  lu_factor(ld, A, lv.piv.p, info, ws, "lu_desc", s);
  launch_lu_solve(ws.upload("x_desc", sd), (int)sd.size(), lv.bmax, rmax, 0, A, lv.piv.p, X, s,
                  elim_chunk(lv.bmax, sizeof(T)));
  T* S = ws.get<T>("S" + tag, (size_t)std::max<int64_t>(lv.at_tot, 1));
  std::vector<GemmDesc> gd;
  std::vector<LUDesc> lds;
  std::vector<SolveDesc> sds;
  std::vector<int64_t> id_off;
  std::vector<int> id_n;
  for (int q = 0; q < n; ++q) {
    if (lv.r[q] == 0) continue;
    GemmDesc g{};
    g.a_off = lv.v_off[q];
    g.b_off = lv.x_off[q];
    g.c_off = lv.at_off[q];
    g.m = lv.r[q];
    g.n = lv.r[q];
    g.k = lv.b[q];
    g.lda = lv.r[q];
    g.ldb = lv.b[q];
    g.ldc = lv.r[q];
    g.alpha_re = 1.0;
    gd.push_back(g);
    lds.push_back(LUDesc{lv.at_off[q], lv.s_piv_off[q], lv.r[q], lv.r[q]});
    sds.push_back(SolveDesc{lv.at_off[q], lv.s_piv_off[q], lv.at_off[q], lv.r[q], lv.r[q], lv.r[q], lv.r[q]});
    id_off.push_back(lv.at_off[q]);
    id_n.push_back(lv.r[q]);
  }
  auto gt = gemm_tiles(gd);
  launch_gemm(ws.upload("s_desc", gd), ws.upload("s_tiles", gt), (int)gt.size(), rmax, 0, V, X, S, 0, s);
  int* info2 = ws.get<int>("lu_info2", std::max<size_t>(lds.size(), 1));
  lu_factor(lds, S, lv.s_piv.p, info2, ws, "slu_desc", s);
  {
    int* dn = ws.upload("id_n", id_n);
    launch_fill_identity((int64_t)id_off.size(), ws.upload("id_off", id_off), dn, dn, At, s);
  }
  launch_lu_solve(ws.upload("at_desc", sds), (int)sds.size(), rmax, rmax, 0, S, lv.s_piv.p, At, s,
                  elim_chunk(rmax, sizeof(T)));
  // zero pivots are reported once the build has finished (no wait here)
  launch_flag_nonzero(n, info, F.sing.p + lv.lev, s);
  launch_flag_nonzero((int64_t)lds.size(), info2, F.sing.p + lv.lev, s);
}

// Pair the ranks of each component (k_c = max(k_row, k_col)) and extend
// the shorter pivoted QR to k_c steps (Section 7.3 reading: nested pivots).
// dv / du: the V / U problems of ``cells`` (2 per cell, comp 0 then 1),
// already factored to tolerance with ranks rv / ru; their matrices live
// in baseV / baseU.  Fills the cells' ranks in lv.
static void pair_and_extend(Factor& F, CellLevel& lv, const std::vector<int>& cells, const std::vector<CpqrDesc>& dv,
                            const std::vector<CpqrDesc>& du, std::vector<int>& rv, std::vector<int>& ru, c64* baseV,
                            c64* baseU, int* dpiv, double tol) {
  Workspace& ws = F.ws;
  std::vector<CpqrDesc> ev, eu;
  std::vector<int> ev_i, eu_i;
  for (size_t ci = 0; ci < cells.size(); ++ci) {
    const int q = cells[ci];
    lv.kc0[q] = rv[2 * ci];
    lv.kc1[q] = rv[2 * ci + 1];
    lv.kr0[q] = ru[2 * ci];
    lv.kr1[q] = ru[2 * ci + 1];
    const int kk[2] = {std::max(lv.kc0[q], lv.kr0[q]), std::max(lv.kc1[q], lv.kr1[q])};
    for (int comp = 0; comp < 2; ++comp) {
      const size_t i = 2 * ci + comp;
      if (rv[i] < kk[comp]) {
        CpqrDesc d = dv[i];
        d.k_start = rv[i];
        d.k_end = kk[comp];
        d.stop_at_tol = 0;
        ev.push_back(d);
        ev_i.push_back((int)i);
      }
      if (ru[i] < kk[comp]) {
        CpqrDesc d = du[i];
        d.k_start = ru[i];
        d.k_end = kk[comp];
        d.stop_at_tol = 0;
        eu.push_back(d);
        eu_i.push_back((int)i);
      }
    }
    lv.k0[q] = kk[0];
    lv.k1[q] = kk[1];
  }
  if (!ev.empty() || !eu.empty()) {
    int* drank2 = ws.get<int>("id_rank2", ev.size() + eu.size());
    // one launch when the U matrices lie in the V matrices' allocation
    if (baseU >= baseV) {
      std::vector<CpqrDesc> both = ev;
      for (CpqrDesc x : eu) {
        x.a_off += baseU - baseV;
        both.push_back(x);
      }
      cpqr_factor(both, baseV, dpiv, tol, drank2, ws, "cpqr_vu2", F.stream);
    } else {
      cpqr_factor(ev, baseV, dpiv, tol, drank2, ws, "cpqr_v2", F.stream);
      cpqr_factor(eu, baseU, dpiv, tol, drank2 + ev.size(), ws, "cpqr_u2", F.stream);
    }
    auto h = download(ws, drank2, ev.size() + eu.size());
    for (size_t i = 0; i < ev.size(); ++i) rv[ev_i[i]] = h[i];
    for (size_t i = 0; i < eu.size(); ++i) ru[eu_i[i]] = h[ev.size() + i];
  }
  for (size_t ci = 0; ci < cells.size(); ++ci) {
    const int q = cells[ci];
    // a zero pivot can end a QR early: never use more pivots than both reached
    lv.k0[q] = std::min(lv.k0[q], std::min(rv[2 * ci], ru[2 * ci]));
    lv.k1[q] = std::min(lv.k1[q], std::min(rv[2 * ci + 1], ru[2 * ci + 1]));
  }
}

// IDs of ``cells`` by the pivoted QR of their interaction matrices
// (Sections 7.1, 7.2).
static void adaptive_ids(Factor& F, CellLevel& lv, const std::vector<int>& cells, const std::vector<CpqrDesc>& qv,
                         const std::vector<CpqrDesc>& qu, c64* MV, c64* MU, int* dpiv) {
  if (cells.empty()) return;
  Workspace& ws = F.ws;
  const size_t nc = cells.size();
  std::vector<CpqrDesc> dv(2 * nc), du(2 * nc);
  for (size_t ci = 0; ci < nc; ++ci)
    for (int comp = 0; comp < 2; ++comp) {
      dv[2 * ci + comp] = qv[2 * cells[ci] + comp];
      du[2 * ci + comp] = qu[2 * cells[ci] + comp];
    }
  int* drank = ws.get<int>("id_rank", 4 * nc);
  // V and U problems in one launch (MU lies in the same allocation after MV)
  std::vector<CpqrDesc> both = dv;
  for (CpqrDesc x : du) {
    x.a_off += MU - MV;
    both.push_back(x);
  }
  cpqr_factor(both, MV, dpiv, F.tol, drank, ws, "cpqr_vu", F.stream);
  auto rk = download(ws, drank, 4 * nc);
  std::vector<int> rv(rk.begin(), rk.begin() + 2 * nc), ru(rk.begin() + 2 * nc, rk.end());
  pair_and_extend(F, lv, cells, dv, du, rv, ru, MV, MU, dpiv, F.tol);
}

// Predictor inputs of the cells of a level: log(k_T d), log(k_L d) (d = 2 R),
// level (root 0), log(active DOFs per component), log(rows of the
// proxy-plus-near matrix), -log10 tol.
static std::vector<float> cell_features(const Factor& F, int lev, const std::vector<double>& crd,
                                        const std::vector<int>& mv_m) {
  const CellLevel& lv = F.levels[lev];
  std::vector<float> x((size_t)lv.n * kMlpIn);
  for (int q = 0; q < lv.n; ++q) {
    const double d = 2.0 * crd[3 * q + 2] / F.opt.proxy_ratio;
    float* f = x.data() + (size_t)q * kMlpIn;
    f[0] = (float)std::log(F.m.kT * d);
    f[1] = (float)std::log(F.m.kL * d);
    f[2] = (float)lev;
    f[3] = (float)std::log(0.5 * lv.b[q]);
    f[4] = (float)std::log((double)mv_m[q]);
    f[5] = (float)(-std::log10(F.tol));
  }
  return x;
}

// Learned form: the predictions of a level, launched before the level's
// interaction matrices are assembled and copied to pinned host memory, so
// that waiting for them does not wait for the assembly.
static void launch_predictions(Factor& F, int lev, const std::vector<double>& crd, const std::vector<int>& mv_m) {
  const int n = F.levels[lev].n;
  if (F.pred_host_n < (size_t)n) {
    if (F.pred_host) {
      FDS_HIP(hipEventSynchronize(F.pred_ev));
      pinned_free(F.pred_host, F.pred_host_bytes);
    }
    F.pred_host = nullptr;
    F.pred_host_n = F.pred_host_bytes = 0;
    F.pred_host = static_cast<float*>(pinned_alloc((size_t)n * sizeof(float), &F.pred_host_bytes));
    F.pred_host_n = (size_t)n;
  }
  if (!F.pred_ev) FDS_HIP(hipEventCreateWithFlags(&F.pred_ev, hipEventDisableTiming));
  const std::vector<float> feat = cell_features(F, lev, crd, mv_m);
  float* dpred = F.ws.get<float>("pred", (size_t)n);
  launch_mlp_forward(n, F.ws.upload("feat", feat), F.pred.p, dpred, 1, F.stream, kAbstainSigma);
  FDS_HIP(hipMemcpyAsync(F.pred_host, dpred, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, F.stream));
  FDS_HIP(hipEventRecord(F.pred_ev, F.stream));
}

// Learned form: per cell, the predictor's rank pre-sizes a sketch of
// s = ceil(k_pred) + oversample rows; the IDs of the sketch are accepted
// when the sketch reveals their rank and the residual judge passes on the
// interaction matrices themselves.  Sketches of at most 64 rows and 128
// columns use the LDS kernels; larger ones draw Omega into a buffer and use
// the batched GEMM for Y = Omega M and for the judge's residual.  Returns the
// cells left to the pivoted QR of their matrices (sketch no smaller than the
// matrix, rank not revealed, judge failed); srcv / srcu point the accepted
// cells' interpolation at the sketches.
static std::vector<int> learned_ids(Factor& F, int lev, const std::vector<double>& crd, const std::vector<int>& mv_m,
                                    const std::vector<CpqrDesc>& qv, const std::vector<CpqrDesc>& qu, c64* MV,
                                    c64* MU, int* dpiv, std::vector<CpqrDesc>& srcv, std::vector<CpqrDesc>& srcu,
                                    std::vector<int>& kpred, std::vector<int>& fallback) {
  CellLevel& lv = F.levels[lev];
  Workspace& ws = F.ws;
  hipStream_t s = F.stream;
  const int n = lv.n;
  auto th = std::chrono::steady_clock::now();
  FDS_HIP(hipEventSynchronize(F.pred_ev));
  const std::vector<float> pred(F.pred_host, F.pred_host + n);
  F.st.predict_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - th).count();
  std::vector<int> plain, sk;
  std::vector<int> sz(n, 0);
  for (int q = 0; q < n; ++q) {
    const float p = pred[q];
    // NaN: the predictor abstained (inputs outside its training range)
    kpred[q] = std::isfinite(p) ? (int)std::min(1e6f, std::max(0.0f, std::ceil(p))) : -1;
    const int ss = kpred[q] + F.opt.oversample;
    // a sketch pays only when it has fewer rows than every matrix it replaces
    bool ok = kpred[q] >= 0 && ss >= 1;
    for (int c = 0; c < 2; ++c) ok = ok && ss < qv[2 * q + c].m && ss < qu[2 * q + c].m;
    if (ok) {
      sz[q] = ss;
      sk.push_back(q);
    } else {
      fallback[q] = 3;
      plain.push_back(q);
    }
  }
  if (sk.empty()) return plain;
  // the 4 problems of every sketched cell: V comp 0/1 (MV), U comp 0/1 (MU)
  const size_t ns = sk.size();
  struct Prob {
    int q, comp;
    bool isV, big;
    CpqrDesc m;
    int s;
    int64_t y_off;
  };
  std::vector<Prob> pr(4 * ns);   // index: V problems 2 ci + comp, then U problems 2 ns + 2 ci + comp
  std::vector<CpqrDesc> yd(4 * ns);
  std::vector<SketchDesc> sv, su;
  std::vector<OmegaDesc> om;
  std::vector<GemmDesc> gv, gu;
  int64_t ytot = 0, otot = 0, omax = 0;
  for (size_t ci = 0; ci < ns; ++ci) {
    const int q = sk[ci];
    const int64_t cell = ((int64_t)1 << lev) - 1 + q;
    for (int k = 0; k < 4; ++k) {
      const bool isV = k < 2;
      const int comp = k & 1;
      const size_t pi = (isV ? 0 : 2 * ns) + 2 * ci + comp;
      const CpqrDesc& m = isV ? qv[2 * q + comp] : qu[2 * q + comp];
      Prob P{q, comp, isV, sz[q] > kSketchMaxS || m.n > kSketchMaxN, m, sz[q], ytot};
      pr[pi] = P;
      if (!P.big) {
        (isV ? sv : su).push_back(SketchDesc{m.a_off, ytot, 4 * cell + k, m.m, m.n, m.lda, sz[q]});
      } else {
        om.push_back(OmegaDesc{otot, 4 * cell + k, sz[q], m.m});
        GemmDesc g{};
        g.a_off = otot;
        g.b_off = m.a_off;
        g.c_off = ytot;
        g.m = sz[q];
        g.n = m.n;
        g.k = m.m;
        g.lda = sz[q];
        g.ldb = m.lda;
        g.ldc = sz[q];
        g.alpha_re = 1.0;
        (isV ? gv : gu).push_back(g);
        omax = std::max<int64_t>(omax, (int64_t)sz[q] * m.m);
        otot += (int64_t)sz[q] * m.m;
      }
      CpqrDesc y{};
      y.a_off = ytot;
      y.piv_off = m.piv_off;
      y.m = sz[q];
      y.n = m.n;
      y.lda = sz[q];
      y.k_start = 0;
      y.k_end = std::min(y.m, y.n);
      y.stop_at_tol = 1;
      yd[pi] = y;
      ytot += (int64_t)sz[q] * m.n;
    }
  }
  c64* Y = ws.get<c64>("sketch_Y", (size_t)std::max<int64_t>(ytot, 1));
  launch_sketch(ws.upload("sk_v", sv), (int)sv.size(), MV, Y, F.opt.seed, s);
  launch_sketch(ws.upload("sk_u", su), (int)su.size(), MU, Y, F.opt.seed, s);
  if (!om.empty()) {
    c64* O = ws.get<c64>("sketch_O", (size_t)otot);
    launch_omega(ws.upload("sk_om", om), (int)om.size(), omax, O, F.opt.seed, s);
    int nmax = 0;
    for (auto& g : gv) nmax = std::max(nmax, g.n);
    for (auto& g : gu) nmax = std::max(nmax, g.n);
    const auto tv = gemm_tiles(gv), tu = gemm_tiles(gu);
    launch_gemm(ws.upload("sk_gv", gv), ws.upload("sk_tv", tv), (int)tv.size(), nmax, 0, (const c64*)O,
                (const c64*)MV, Y, 0, s);
    launch_gemm(ws.upload("sk_gu", gu), ws.upload("sk_tu", tu), (int)tu.size(), nmax, 0, (const c64*)O,
                (const c64*)MU, Y, 0, s);
  }
  int* drank = ws.get<int>("sk_rank", 4 * ns);
  cpqr_factor(yd, Y, dpiv, kSketchTolFactor * F.tol, drank, ws, "sk_cpqr", s);
  const auto rk = download(ws, drank, 4 * ns);
  // the sketch must reveal every rank: a crossing inside it, or s >= n
  std::vector<int> acc;
  std::vector<size_t> acc_ci;
  std::vector<CpqrDesc> av, au;
  std::vector<int> rv, ru;
  for (size_t ci = 0; ci < ns; ++ci) {
    bool revealed = true;
    for (int k = 0; k < 4; ++k) {
      const size_t pi = (k < 2 ? 0 : 2 * ns) + 2 * ci + (k & 1);
      revealed = revealed && (rk[pi] + kRevealMargin <= yd[pi].m || yd[pi].m >= yd[pi].n);
    }
    const int q = sk[ci];
    if (!revealed) {
      fallback[q] = 1;
      continue;
    }
    acc.push_back(q);
    acc_ci.push_back(ci);
    for (int comp = 0; comp < 2; ++comp) {
      av.push_back(yd[2 * ci + comp]);
      au.push_back(yd[2 * ns + 2 * ci + comp]);
      rv.push_back(rk[2 * ci + comp]);
      ru.push_back(rk[2 * ns + 2 * ci + comp]);
    }
  }
  if (!acc.empty()) {
    pair_and_extend(F, lv, acc, av, au, rv, ru, Y, Y, dpiv, kSketchTolFactor * F.tol);
    // residual judge on the interaction matrices themselves; W (k x n) of
    // every problem first, then the small problems by the LDS kernel and
    // the large ones by gather + GEMM + column norms
    std::vector<InterpDesc> iw;
    std::vector<JudgeDesc> jv, ju;
    std::vector<ColGatherDesc> ecv, ecu, gcv, gcu;
    std::vector<GemmDesc> rgv, rgu;
    std::vector<RatioDesc> rdv, rdu;
    std::vector<size_t> jv_i, ju_i, rdv_i, rdu_i;   // accepted-problem slots (4 per accepted cell)
    int64_t wtot = 0, etot = 0, gtot = 0;
    int ecmax = 0, gcmax = 0, rnmax = 0;
    for (size_t ai = 0; ai < acc.size(); ++ai) {
      const int q = acc[ai];
      const size_t ci = acc_ci[ai];
      for (int k = 0; k < 4; ++k) {
        const bool isV = k < 2;
        const int comp = k & 1;
        const size_t slot = 4 * ai + k;
        const Prob& P = pr[(isV ? 0 : 2 * ns) + 2 * ci + comp];
        const int kk = comp ? lv.k1[q] : lv.k0[q];
        const CpqrDesc& y = isV ? av[2 * ai + comp] : au[2 * ai + comp];
        const CpqrDesc& m = P.m;
        if (kk > 0) iw.push_back(InterpDesc{y.a_off, y.piv_off, y.n, y.lda, kk, wtot, kk, 0, 0});
        if (!P.big) {
          (isV ? jv : ju).push_back(JudgeDesc{m.a_off, wtot, m.piv_off, m.m, m.n, m.lda, kk});
          (isV ? jv_i : ju_i).push_back(slot);
        } else {
          (isV ? ecv : ecu).push_back(ColGatherDesc{m.a_off, etot, -1, m.m, m.n, m.lda, m.m});
          ecmax = std::max(ecmax, m.n);
          if (kk > 0) {
            (isV ? gcv : gcu).push_back(ColGatherDesc{m.a_off, gtot, m.piv_off, m.m, kk, m.lda, m.m});
            gcmax = std::max(gcmax, kk);
            GemmDesc g{};
            g.a_off = gtot;
            g.b_off = wtot;
            g.c_off = etot;
            g.m = m.m;
            g.n = m.n;
            g.k = kk;
            g.lda = m.m;
            g.ldb = kk;
            g.ldc = m.m;
            g.alpha_re = -1.0;
            g.beta_re = 1.0;
            (isV ? rgv : rgu).push_back(g);
            rnmax = std::max(rnmax, m.n);
          }
          (isV ? rdv : rdu).push_back(RatioDesc{etot, m.a_off, m.m, m.n, m.m, m.lda});
          (isV ? rdv_i : rdu_i).push_back(slot);
          etot += (int64_t)m.m * m.n;
          gtot += (int64_t)m.m * kk;
        }
        wtot += (int64_t)kk * y.n;
      }
    }
    c64* Wj = ws.get<c64>("judge_W", (size_t)std::max<int64_t>(wtot, 1));
    const size_t nj = jv.size() + ju.size() + rdv.size() + rdu.size();
    double* ratio = ws.get<double>("judge_ratio", nj);
    launch_interp(ws.upload("judge_interp", iw), (int)iw.size(), Y, dpiv, Wj, s, interp_size(iw));
    launch_judge(ws.upload("judge_v", jv), (int)jv.size(), MV, Wj, dpiv, ratio, s);
    launch_judge(ws.upload("judge_u", ju), (int)ju.size(), MU, Wj, dpiv, ratio + jv.size(), s);
    if (!rdv.empty() || !rdu.empty()) {
      c64* E = ws.get<c64>("judge_E", (size_t)std::max<int64_t>(etot, 1));
      c64* G = ws.get<c64>("judge_G", (size_t)std::max<int64_t>(gtot, 1));
      launch_gather_cols(ws.upload("jg_ecv", ecv), (int)ecv.size(), ecmax, MV, dpiv, E, s);
      launch_gather_cols(ws.upload("jg_ecu", ecu), (int)ecu.size(), ecmax, MU, dpiv, E, s);
      launch_gather_cols(ws.upload("jg_gcv", gcv), (int)gcv.size(), gcmax, MV, dpiv, G, s);
      launch_gather_cols(ws.upload("jg_gcu", gcu), (int)gcu.size(), gcmax, MU, dpiv, G, s);
      std::vector<GemmDesc> rg(rgv);
      rg.insert(rg.end(), rgu.begin(), rgu.end());
      const auto rt = gemm_tiles(rg);
      launch_gemm(ws.upload("jg_g", rg), ws.upload("jg_t", rt), (int)rt.size(), rnmax, 0, (const c64*)G,
                  (const c64*)Wj, E, 0, s);
      const size_t o = jv.size() + ju.size();
      launch_ratio(ws.upload("jg_rv", rdv), (int)rdv.size(), E, MV, ratio + o, s);
      launch_ratio(ws.upload("jg_ru", rdu), (int)rdu.size(), E, MU, ratio + o + rdv.size(), s);
    }
    const auto rt = download(ws, ratio, nj);
    std::vector<double> slot_ratio(4 * acc.size(), 0.0);
    size_t o = 0;
    for (size_t i = 0; i < jv_i.size(); ++i) slot_ratio[jv_i[i]] = rt[o++];
    for (size_t i = 0; i < ju_i.size(); ++i) slot_ratio[ju_i[i]] = rt[o++];
    for (size_t i = 0; i < rdv_i.size(); ++i) slot_ratio[rdv_i[i]] = rt[o++];
    for (size_t i = 0; i < rdu_i.size(); ++i) slot_ratio[rdu_i[i]] = rt[o++];
    for (size_t ai = 0; ai < acc.size(); ++ai) {
      const int q = acc[ai];
      bool pass = true;
      for (int k = 0; k < 4; ++k) pass = pass && slot_ratio[4 * ai + k] <= F.tol;
      if (!pass) {
        fallback[q] = 2;
        continue;
      }
      for (int comp = 0; comp < 2; ++comp) {
        srcv[2 * q + comp] = av[2 * ai + comp];
        srcu[2 * q + comp] = au[2 * ai + comp];
      }
    }
  }
  for (int q : sk)
    if (fallback[q] != 0) plain.push_back(q);
  std::sort(plain.begin(), plain.end());
  for (int q : sk) {
    F.st.cells_sketched += fallback[q] == 0;
    F.st.cells_fallback_rank += fallback[q] == 1;
    F.st.cells_fallback_judge += fallback[q] == 2;
  }
  return plain;
}

// Rank log entry of every cell of a compressed level (the predictor's
// training data).
static void record_ranks(Factor& F, int lev, const std::vector<double>& crd, const std::vector<int>& mv_m,
                         const std::vector<int>& kpred, const std::vector<int>& fallback) {
  const CellLevel& lv = F.levels[lev];
  const std::vector<float> feat = cell_features(F, lev, crd, mv_m);
  for (int q = 0; q < lv.n; ++q) {
    fds_rank_record r{};
    r.cell = (int32_t)(((int64_t)1 << lev) - 1 + q);
    r.level = lev;
    r.rank[0] = lv.kr0[q];
    r.rank[1] = lv.kc0[q];
    r.rank[2] = lv.kr1[q];
    r.rank[3] = lv.kc1[q];
    r.k_pred = kpred[q];
    r.fallback = fallback[q];
    for (int c = 0; c < kMlpIn; ++c) r.feat[c] = feat[(size_t)q * kMlpIn + c];
    F.rank_log.push_back(r);
  }
  F.st.cells_compressed += lv.n;
}

// Proxy disks, near sets and the interaction matrices M^V, M^U^T of level
// lev (Sections 7.1, 7.2), enqueued; the IDs follow in compress_level.
static void prepare_level(Factor& F, int lev) {
  const Geometry& G = F.G;
  CellLevel& lv = F.levels[lev];
  Workspace& ws = F.ws;
  hipStream_t s = F.stream;
  const int n = lv.n;
  auto ht0 = std::make_unique<HostTimer>(0);
  // proxy disks
  std::vector<double> crd(3 * n);
  double maxrho = 0.0;
  parallel_for(n, [&](int q) {
    double cx, cy, R;
    cell_disk(G, lv.rows[q], lv.cols[q], cx, cy, R);
    crd[3 * q] = cx;
    crd[3 * q + 1] = cy;
    crd[3 * q + 2] = F.opt.proxy_ratio * R;
  });
  for (int q = 0; q < n; ++q) maxrho = std::max(maxrho, crd[3 * q + 2]);
  // near sets via a node grid
  // (the cells' row DOFs are disjoint, and so are their column DOFs)
  std::vector<int> row_owner(2 * (size_t)G.n_nodes, -1), col_owner(2 * (size_t)G.n_nodes, -1);
  std::vector<char> has(G.n_nodes, 0);
  parallel_for(n, [&](int q) {
    for (auto d : lv.rows[q]) {
      row_owner[d] = q;
      __atomic_store_n(&has[d >> 1], (char)1, __ATOMIC_RELAXED);
    }
    for (auto d : lv.cols[q]) {
      col_owner[d] = q;
      __atomic_store_n(&has[d >> 1], (char)1, __ATOMIC_RELAXED);
    }
  });
  std::vector<int> active;
  for (int t = 0; t < G.n_nodes; ++t)
    if (has[t]) active.push_back(t);
  NodeGrid grid;
  grid.build(G, active, std::max(maxrho, 4.0 * G.hmax));
  std::vector<std::vector<int64_t>> near_r(n), near_c(n);
  parallel_for(n, [&](int q) {
    const double cx = crd[3 * q], cy = crd[3 * q + 1], rho = crd[3 * q + 2];
    // every node sits in exactly one grid bucket: no duplicates
    std::vector<int> cand;
    grid.query(cx, cy, rho + G.hmax, [&](int t) { cand.push_back(t); });
    std::sort(cand.begin(), cand.end());
    const double rin = rho, rout = rho + G.hmax;
    for (int t : cand) {
      const double dx = G.xy[2 * t] - cx, dy = G.xy[2 * t + 1] - cy;
      const double d2 = dx * dx + dy * dy;
      // the support lies within hmax of the node: decide cheaply away from the circle
      if (d2 >= rout * rout) continue;
      if (d2 >= rin * rin && !support_meets(G, t, cx, cy, rho)) continue;
      for (int c = 0; c < 2; ++c) {
        const int64_t d = 2 * (int64_t)t + c;
        if (row_owner[d] >= 0 && row_owner[d] != q) near_r[q].push_back(d);
        if (col_owner[d] >= 0 && col_owner[d] != q) near_c[q].push_back(d);
      }
    }
  });
  ht0.reset();
  // proxy elements: per cell a polygon of npx[q] vertices (at least
  // n_proxy, more when the wave oscillates faster than it resolves)
  std::vector<int> npx(n), poff(n + 1, 0);
  for (int q = 0; q < n; ++q) {
    npx[q] = F.opt.proxy_fixed ? F.opt.n_proxy : proxy_count(F.m.kT, crd[3 * q + 2], F.opt.n_proxy);
    poff[q + 1] = poff[q] + npx[q];
    lv.max_proxy = std::max(lv.max_proxy, npx[q]);
  }
  F.st.max_proxy = std::max(F.st.max_proxy, lv.max_proxy);
  const int64_t pbase = F.DG.n_gamma;
  F.DG.reserve(pbase + poff[n], s);
  launch_proxy_elems(ws.upload("crd", crd), ws.upload("poff", poff), n, poff[n], G.n_curves, F.DG.elems.p + pbase,
                     s);
  // interaction matrices: MV = A(proxy + near rows, cols) and MUt = A(rows, proxy + near cols)^T
  std::vector<int64_t> mv_off(n), mu_off(n);
  std::vector<int> mv_m(n), mu_m(n);
  int64_t mv_tot = 0, mu_tot = 0;
  for (int q = 0; q < n; ++q) {
    mv_m[q] = 2 * npx[q] + (int)near_r[q].size();
    mu_m[q] = 2 * npx[q] + (int)near_c[q].size();
    mv_off[q] = mv_tot;
    mv_tot += (int64_t)mv_m[q] * lv.b[q];
    mu_off[q] = mu_tot;
    mu_tot += (int64_t)mu_m[q] * lv.b[q];
  }
  if (F.opt.rank_mode == FDS_RANK_LEARNED) launch_predictions(F, lev, crd, mv_m);
  auto ht1 = std::make_unique<HostTimer>(1);
  // one allocation: the V and U problems of a level then share each QR launch
  c64* MV = ws.get<c64>("MVU", (size_t)(mv_tot + mu_tot));
  c64* MU = MV + mv_tot;
  {
    std::vector<BlockReq> reqs(n);
    parallel_for(n, [&](int q) {
      BlockReq& a = reqs[q];
      side_add_proxy(a.rows, (int)(pbase + poff[q]), npx[q]);
      side_append(G, a.rows, near_r[q]);
      a.cols = side_from_dofs(G, lv.cols[q]);
      a.out_off = mv_off[q];
      a.rs = 1;
      a.cs = mv_m[q];
    });
    HostTimer hp(8);
    assemble_blocks(reqs, F.DG.elems.p, F.m, MV, ws, &F.ast);
  }
  {
    std::vector<BlockReq> reqs(n);
    parallel_for(n, [&](int q) {
      BlockReq& a = reqs[q];
      a.rows = side_from_dofs(G, lv.rows[q]);
      side_add_proxy(a.cols, (int)(pbase + poff[q]), npx[q]);
      side_append(G, a.cols, near_c[q]);
      a.out_off = mu_off[q];
      a.rs = mu_m[q];   // transposed storage
      a.cs = 1;
    });
    HostTimer hp(8);
    assemble_blocks(reqs, F.DG.elems.p, F.m, MU, ws, &F.ast);
  }
  ht1.reset();
  Factor::LevelPrep& pr = F.prep;
  pr.lev = lev;
  pr.crd = std::move(crd);
  pr.mv_m = std::move(mv_m);
  pr.mu_m = std::move(mu_m);
  pr.mv_off = std::move(mv_off);
  pr.mu_off = std::move(mu_off);
  pr.MV = MV;
  pr.MU = MU;
}

static void compress_level(Factor& F, int lev) {
  CellLevel& lv = F.levels[lev];
  Workspace& ws = F.ws;
  hipStream_t s = F.stream;
  const int n = lv.n;
  if (F.prep.lev != lev) throw Error(1, "internal: level " + std::to_string(lev) + " was not prepared");
  const std::vector<double>& crd = F.prep.crd;
  const std::vector<int>& mv_m = F.prep.mv_m;
  const std::vector<int>& mu_m = F.prep.mu_m;
  const std::vector<int64_t>& mv_off = F.prep.mv_off;
  const std::vector<int64_t>& mu_off = F.prep.mu_off;
  c64* MV = F.prep.MV;
  c64* MU = F.prep.MU;
  // IDs: per cell V comp0, V comp1 (in MV) and U comp0, U comp1 (in MU^T)
  span_begin(F, 0);
  std::vector<CpqrDesc> qv(2 * n), qu(2 * n);
  int64_t pv_tot = 0;
  for (int q = 0; q < n; ++q) {
    const int b = lv.b[q], c0 = lv.n0[q], c1 = b - c0;
    const int ncs[2] = {c0, c1};
    for (int k = 0; k < 4; ++k) {
      const bool isV = k < 2;
      const int comp = k & 1;
      CpqrDesc d{};
      const int mrows = isV ? mv_m[q] : mu_m[q];
      d.a_off = (isV ? mv_off[q] : mu_off[q]) + (int64_t)(comp ? c0 : 0) * mrows;
      d.m = mrows;
      d.n = ncs[comp];
      d.lda = mrows;
      d.piv_off = pv_tot;
      pv_tot += d.n;
      d.k_start = 0;
      d.k_end = std::min(d.m, d.n);
      d.stop_at_tol = 1;
      (isV ? qv : qu)[2 * q + comp] = d;
    }
  }
  check_cpqr_sizes(qv);
  check_cpqr_sizes(qu);
  int* dpiv = ws.get<int>("id_piv", (size_t)pv_tot);
  lv.kc0.assign(n, 0);
  lv.kc1.assign(n, 0);
  lv.kr0.assign(n, 0);
  lv.kr1.assign(n, 0);
  lv.k0.assign(n, 0);
  lv.k1.assign(n, 0);
  lv.r.assign(n, 0);
  // where each ID's triangular factor lives (M itself, or its sketch)
  std::vector<CpqrDesc> srcv = qv, srcu = qu;
  std::vector<int> kpred(n, -1), fallback(n, 0);
  std::vector<int> plain;
  if (F.opt.rank_mode == FDS_RANK_LEARNED) {
    plain = learned_ids(F, lev, crd, mv_m, qv, qu, MV, MU, dpiv, srcv, srcu, kpred, fallback);
  } else {
    plain.resize(n);
    std::iota(plain.begin(), plain.end(), 0);
  }
  adaptive_ids(F, lv, plain, qv, qu, MV, MU, dpiv);
  for (int q = 0; q < n; ++q) lv.r[q] = lv.k0[q] + lv.k1[q];
  record_ranks(F, lev, crd, mv_m, kpred, fallback);
  auto hpiv = download(ws, dpiv, (size_t)pv_tot);
  // skeletons, layouts
  lv.rskel.assign(n, {});
  lv.cskel.assign(n, {});
  lv.x_off.resize(n);
  lv.at_off.resize(n);
  lv.v_off.resize(n);
  lv.s_piv_off.resize(n);
  lv.t_off.resize(n);
  lv.x_tot = lv.at_tot = lv.v_tot = lv.s_piv_tot = lv.R = 0;
  parallel_for(n, [&](int q) {   // each cell's skeleton DOFs, on the host pool
    const int c0 = lv.n0[q];
    const int kk[2] = {lv.k0[q], lv.k1[q]};
    lv.cskel[q].reserve(kk[0] + kk[1]);
    lv.rskel[q].reserve(kk[0] + kk[1]);
    for (int comp = 0; comp < 2; ++comp) {
      const int base = comp ? c0 : 0;
      const int* pc = hpiv.data() + qv[2 * q + comp].piv_off;
      const int* pr = hpiv.data() + qu[2 * q + comp].piv_off;
      for (int j = 0; j < kk[comp]; ++j) {
        lv.cskel[q].push_back(lv.cols[q][base + pc[j]]);
        lv.rskel[q].push_back(lv.rows[q][base + pr[j]]);
      }
    }
  });
  int rmax = 0;
  for (int q = 0; q < n; ++q) {
    const int b = lv.b[q], r = lv.r[q];
    rmax = std::max(rmax, r);
    lv.x_off[q] = lv.x_tot;
    lv.x_tot += (int64_t)b * r;
    lv.at_off[q] = lv.at_tot;
    lv.at_tot += (int64_t)r * r;
    lv.v_off[q] = lv.v_tot;
    lv.v_tot += (int64_t)r * b;
    lv.s_piv_off[q] = lv.s_piv_tot;
    lv.s_piv_tot += r;
    lv.t_off[q] = lv.R;
    lv.R += r;
  }
  lv.X = DevBuf<c64>((size_t)std::max<int64_t>(lv.x_tot, 1));
  lv.At = DevBuf<c64>(F.opt.precision == FDS_PREC_MIXED ? 1 : (size_t)std::max<int64_t>(lv.at_tot, 1));
  lv.V = DevBuf<c64>((size_t)std::max<int64_t>(lv.v_tot, 1));
  lv.s_piv = DevBuf<int>((size_t)std::max<int64_t>(lv.s_piv_tot, 1));
  FDS_HIP(hipMemsetAsync(lv.X.p, 0, lv.X.n * sizeof(c64), s));
  FDS_HIP(hipMemsetAsync(lv.V.p, 0, lv.V.n * sizeof(c64), s));
  // V_i (r x b) from the column IDs; U_i = X_i (b x r) from the row IDs (W^T)
  std::vector<InterpDesc> ivm, ium, ivy, iuy;
  for (int q = 0; q < n; ++q) {
    const int b = lv.b[q], r = lv.r[q], c0 = lv.n0[q];
    const int kk[2] = {lv.k0[q], lv.k1[q]};
    const bool sk = F.opt.rank_mode == FDS_RANK_LEARNED && fallback[q] == 0;
    for (int comp = 0; comp < 2; ++comp) {
      if (kk[comp] == 0) continue;
      const int roff = comp ? kk[0] : 0;   // skeleton offset
      const int coff = comp ? c0 : 0;      // DOF offset
      // the sketches' triangular systems were solved in place for the judge
      const int solved = sk ? 1 : 0;
      const CpqrDesc& dv = srcv[2 * q + comp];
      (sk ? ivy : ivm).push_back(InterpDesc{dv.a_off, dv.piv_off, dv.n, dv.lda, kk[comp],
                                            lv.v_off[q] + roff + (int64_t)coff * r, r, 0, solved});
      const CpqrDesc& du = srcu[2 * q + comp];
      (sk ? iuy : ium).push_back(InterpDesc{du.a_off, du.piv_off, du.n, du.lda, kk[comp],
                                            lv.x_off[q] + coff + (int64_t)roff * b, b, 1, solved});
    }
  }
  launch_interp(ws.upload("interp_v", ivm), (int)ivm.size(), MV, dpiv, lv.V.p, s, interp_size(ivm));
  launch_interp(ws.upload("interp_u", ium), (int)ium.size(), MU, dpiv, lv.X.p, s, interp_size(ium));
  if (!ivy.empty() || !iuy.empty()) {
    c64* Y = ws.get<c64>("sketch_Y", 1);
    launch_interp(ws.upload("interp_vy", ivy), (int)ivy.size(), Y, dpiv, lv.V.p, s, interp_size(ivy));
    launch_interp(ws.upload("interp_uy", iuy), (int)iuy.size(), Y, dpiv, lv.X.p, s, interp_size(iuy));
  }
  span_end(F);

  // elimination: LU(A_i); X_i = A_i^{-1} U_i; S_i = V_i X_i; A~_i = S_i^{-1}
  span_begin(F, 1);
  if (F.opt.precision == FDS_PREC_MIXED) {
    // FP32 copies: A_i (the FP64 block plus the children's FP32 A~), U_i, V_i
    lv.A32 = DevBuf<c32>((size_t)std::max<int64_t>(lv.a_tot, 1));
    lv.X32 = DevBuf<c32>((size_t)std::max<int64_t>(lv.x_tot, 1));
    lv.V32 = DevBuf<c32>((size_t)std::max<int64_t>(lv.v_tot, 1));
    lv.At32 = DevBuf<c32>((size_t)std::max<int64_t>(lv.at_tot, 1));
    launch_convert(lv.a_tot, lv.A.p, lv.A32.p, s);
    if (lev < F.L) place_child_at(F, lev, [&](int p) { return lv.a_off[p]; }, [&](int p) { return lv.b[p]; },
                                  lv.A32.p, "c32");
    launch_convert(lv.x_tot, lv.X.p, lv.X32.p, s);
    launch_convert(lv.v_tot, lv.V.p, lv.V32.p, s);
    eliminate(F, lv, rmax, lv.A32.p, lv.X32.p, lv.V32.p, lv.At32.p, "32");
  } else {
    eliminate(F, lv, rmax, lv.A.p, lv.X.p, lv.V.p, lv.At.p, "64");
  }
  span_end(F);
  int mr = 0;
  for (int q = 0; q < n; ++q) mr = std::max(mr, std::max(lv.k0[q], lv.k1[q]));
  F.st.max_rank = std::max(F.st.max_rank, mr);
}

// Parent DOF lists of level lev-1 from level lev (rearrangement, Section 6.2)
// and the layout of the parent blocks.
static void merge_lists(Factor& F, int lev) {
  HostTimer ht(3);
  CellLevel& ch = F.levels[lev];
  CellLevel& pa = F.levels[lev - 1];
  pa.lev = lev - 1;
  pa.n = ch.n / 2;
  pa.rows.assign(pa.n, {});
  pa.cols.assign(pa.n, {});
  ch.ppos.assign(ch.n, {});
  parallel_for(pa.n, [&](int p) {   // parents on the host thread pool
    const int a = 2 * p, b = 2 * p + 1;
    const int ka0 = ch.k0[a], kb0 = ch.k0[b], ka1 = ch.k1[a], kb1 = ch.k1[b];
    auto& R = pa.rows[p];
    auto& C = pa.cols[p];
    R.reserve(ka0 + kb0 + ka1 + kb1);
    C.reserve(ka0 + kb0 + ka1 + kb1);
    auto app = [](std::vector<int64_t>& dst, const std::vector<int64_t>& src, int o, int k) {
      dst.insert(dst.end(), src.begin() + o, src.begin() + o + k);
    };
    app(R, ch.rskel[a], 0, ka0);
    app(R, ch.rskel[b], 0, kb0);
    app(R, ch.rskel[a], ka0, ka1);
    app(R, ch.rskel[b], kb0, kb1);
    app(C, ch.cskel[a], 0, ka0);
    app(C, ch.cskel[b], 0, kb0);
    app(C, ch.cskel[a], ka0, ka1);
    app(C, ch.cskel[b], kb0, kb1);
    // parent position of each child skeleton entry (same pattern for rows and cols)
    auto& pa_ = ch.ppos[a];
    auto& pb_ = ch.ppos[b];
    pa_.reserve(ka0 + ka1);
    pb_.reserve(kb0 + kb1);
    for (int j = 0; j < ka0; ++j) pa_.push_back(j);
    for (int j = 0; j < ka1; ++j) pa_.push_back(ka0 + kb0 + j);
    for (int j = 0; j < kb0; ++j) pb_.push_back(ka0 + j);
    for (int j = 0; j < kb1; ++j) pb_.push_back(ka0 + kb0 + ka1 + j);
  });
  layout_blocks(pa);
}

// The parent blocks' entries: the children's A~ and the off-diagonal
// interactions at skeleton pairs (enqueued after the parent level's
// interaction matrices, which need only the parent DOF lists).
static void merge_blocks(Factor& F, int lev) {
  HostTimer ht(3);
  const Geometry& G = F.G;
  CellLevel& ch = F.levels[lev];
  CellLevel& pa = F.levels[lev - 1];
  Workspace& ws = F.ws;
  hipStream_t s = F.stream;
  // diagonal sub-blocks: A~ of the children (plain form); the mixed form
  // keeps them out of the FP64 block and adds its FP32 A~ when the parent
  // level is eliminated
  if (F.opt.precision == FDS_PREC_MIXED)
    FDS_HIP(hipMemsetAsync(pa.A.p, 0, pa.A.n * sizeof(c64), s));
  else
    place_child_at_t(F, lev - 1, [&](int p) { return pa.a_off[p]; }, [&](int p) { return pa.b[p]; }, ch.At.p,
                     pa.A.p, "c64");
  // off-diagonal: R_ab = A(rskel_a, cskel_b), R_ba = A(rskel_b, cskel_a)
  std::vector<int> pick;   // child a of each request (b = a ^ 1)
  for (int a = 0; a < 2 * pa.n; ++a)
    if (ch.r[a] != 0 && ch.r[a ^ 1] != 0) pick.push_back(a);
  std::vector<BlockReq> reqs(pick.size());
  parallel_for((int)pick.size(), [&](int k) {
    const int a = pick[k], b = a ^ 1, p = a >> 1;
    BlockReq& q = reqs[k];
    q.rows = side_from_dofs(G, ch.rskel[a]);
    q.cols = side_from_dofs(G, ch.cskel[b]);
    q.out_off = pa.a_off[p];
    q.rs = 1;
    q.cs = pa.b[p];
    q.rpos = ch.ppos[a];
    q.cpos = ch.ppos[b];
  });
  assemble_blocks(reqs, F.DG.elems.p, F.m, pa.A.p, ws, &F.ast);
}

// Leaf diagonal blocks.
static void assemble_leaves(Factor& F) {
  HostTimer ht(4);
  CellLevel& lv = F.levels[F.L];
  layout_blocks(lv);
  std::vector<BlockReq> reqs(lv.n);
  parallel_for(lv.n, [&](int q) {
    BlockReq& a = reqs[q];
    a.rows = side_from_dofs(F.G, lv.rows[q]);
    a.cols = a.rows;
    a.out_off = lv.a_off[q];
    a.rs = 1;
    a.cs = lv.b[q];
  });
  assemble_blocks(reqs, F.DG.elems.p, F.m, lv.A.p, F.ws, &F.ast);
}

static void factor_root(Factor& F) {
  HostTimer ht(5);
  CellLevel& lv = F.levels[F.l0];
  Root& rt = F.root;
  Workspace& ws = F.ws;
  hipStream_t s = F.stream;
  rt.n = (int)lv.B;
  rt.A = DevBuf<c64>((size_t)rt.n * rt.n);
  rt.piv = DevBuf<int>((size_t)rt.n);
  std::vector<ScatterDesc> sc;
  std::vector<BlockReq> reqs;
  for (int q = 0; q < lv.n; ++q) {
    ScatterDesc d{};
    d.src_off = lv.a_off[q];
    d.src_ld = lv.b[q];
    d.nr = lv.b[q];
    d.nc = lv.b[q];
    d.dst_off = lv.f_off[q] + lv.f_off[q] * (int64_t)rt.n;
    d.dst_ld = rt.n;
    d.rpos_off = -1;
    d.cpos_off = -1;
    sc.push_back(d);
    for (int q2 = 0; q2 < lv.n; ++q2) {
      if (q2 == q) continue;
      BlockReq a;
      a.rows = side_from_dofs(F.G, lv.rows[q]);
      a.cols = side_from_dofs(F.G, lv.cols[q2]);
      a.out_off = lv.f_off[q] + lv.f_off[q2] * (int64_t)rt.n;
      a.rs = 1;
      a.cs = rt.n;
      reqs.push_back(std::move(a));
    }
  }
  auto st = scatter_tiles(sc);
  launch_scatter(ws.upload("rsc_desc", sc), ws.upload("rsc_tiles", st), (int)st.size(),
                 ws.upload("rsc_pos", std::vector<int>{0}), lv.A.p, rt.A.p, s);
  assemble_blocks(reqs, F.DG.elems.p, F.m, rt.A.p, ws, &F.ast);
  if (F.opt.precision == FDS_PREC_MIXED) {
    // keep the system without the children's A~ for the compressed-operator
    // product, then add their FP32 A~ (widened) for the FP64 LU
    rt.B = DevBuf<c64>((size_t)rt.n * rt.n);
    FDS_HIP(hipMemcpyAsync(rt.B.p, rt.A.p, rt.B.n * sizeof(c64), hipMemcpyDeviceToDevice, s));
    if (F.L > F.l0)
      place_child_at_t(F, F.l0, [&](int q) { return lv.f_off[q] + lv.f_off[q] * (int64_t)rt.n; },
                       [&](int) { return rt.n; }, F.levels[F.l0 + 1].At32.p, rt.A.p, "root");
    GemmDesc g{};
    g.m = g.n = g.k = rt.n;
    g.lda = g.ldb = g.ldc = rt.n;
    g.alpha_re = 1.0;
    std::vector<GemmDesc> gd{g};
    auto gt = gemm_tiles(gd);
    rt.g_b = DevBuf<GemmDesc>(gd);
    rt.t_b = DevBuf<GemmTile>(gt);
    rt.n_tb = (int)gt.size();
  }
  span_begin(F, 2);
  int* info = ws.get<int>("root_info", 1);
  lu_factor(std::vector<LUDesc>{LUDesc{0, 0, rt.n, rt.n}}, rt.A.p, rt.piv.p, info, ws, "root_lu", s);
  span_end(F);
  launch_flag_nonzero(1, info, F.sing.p + F.l0, s);
  rt.desc = DevBuf<SolveDesc>(std::vector<SolveDesc>{SolveDesc{0, 0, 0, rt.n, rt.n, rt.n, 0}});
}

// Device descriptors of the solve (ncol = number of right-hand sides is
// supplied at solve time).
// Matrix-core sweeps of the plain form: for every compressed level whose
// block orders have a variant, W_i = A~_i V_i (replacing V_i: the upward
// sweep needs only the product), the LU's composed permutation and the
// inverted diagonal blocks.
static void prepare_mfma_sweeps(Factor& F, ArenaBuilder& ab) {
  hipStream_t s = F.stream;
  // host arrays of every level first (one upload for all of them), then
  // the per-level launches
  struct Prep {
    int lev = 0, rmax = 0, n_blk = 0, nmax = 0, n_gt = 0;
    int64_t dtot = 0;
    DevView<int> blk_cell, blk_k;
    DevView<GemmDesc> gd;
    DevView<GemmTile> gt;
  };
  std::vector<Prep> preps;
  preps.reserve(F.L - F.l0);
  ArenaBuilder pre;
  for (int lev = F.L; lev > F.l0; --lev) {
    CellLevel& lv = F.levels[lev];
    int rmax = 0;
    for (int q = 0; q < lv.n; ++q) rmax = std::max(rmax, lv.r[q]);
    if (!sweep_supported(lv.bmax, rmax)) continue;
    preps.emplace_back();
    Prep& P = preps.back();
    P.lev = lev;
    P.rmax = rmax;
    std::vector<SweepCell> cells(lv.n);
    std::vector<int> blk_cell, blk_k;
    std::vector<GemmDesc> gd;
    int64_t dtot = 0;
    for (int q = 0; q < lv.n; ++q) {
      SweepCell& c = cells[q];
      const int b = lv.b[q], r = lv.r[q], nb = (b + 15) / 16;
      c.a_off = lv.a_off[q];
      c.dinv_off = dtot;
      dtot += (int64_t)nb * 512;
      c.v_off = lv.v_off[q];
      c.at_off = lv.at_off[q];
      c.x_off = lv.x_off[q];
      c.f_off = lv.f_off[q];
      c.t_off = lv.t_off[q];
      c.perm_off = lv.piv_off[q];
      c.piv_off = lv.piv_off[q];
      c.b = b;
      c.r = r;
      for (int k = 0; k < nb; ++k) {
        blk_cell.push_back(q);
        blk_k.push_back(k);
      }
      if (r == 0) continue;
      GemmDesc g{};   // W = A~ V
      g.a_off = lv.at_off[q];
      g.b_off = lv.v_off[q];
      g.c_off = lv.v_off[q];
      g.m = r;
      g.n = b;
      g.k = r;
      g.lda = r;
      g.ldb = r;
      g.ldc = r;
      g.alpha_re = 1.0;
      gd.push_back(g);
      P.nmax = std::max(P.nmax, g.n);
    }
    P.dtot = dtot;
    P.n_blk = (int)blk_cell.size();
    const auto gt = gemm_tiles(gd);
    P.n_gt = (int)gt.size();
    ab.add(lv.sweep, cells);   // kept with the solve plan
    pre.add(P.blk_cell, blk_cell);
    pre.add(P.blk_k, blk_k);
    pre.add(P.gd, gd);
    pre.add(P.gt, gt);
    // fewer columns than a slab: the LU-solve kernel, then f~ = W g by GEMM
    std::vector<GemmDesc> gw;
    for (int q = 0; q < lv.n; ++q) {
      if (lv.r[q] == 0) continue;
      GemmDesc g{};
      g.a_off = lv.v_off[q];
      g.b_off = lv.f_off[q];
      g.c_off = lv.t_off[q];
      g.m = lv.r[q];
      g.k = lv.b[q];
      g.lda = lv.r[q];
      g.ldb = (int)lv.B;
      g.ldc = (int)lv.R;
      g.alpha_re = 1.0;
      gw.push_back(g);
    }
    auto tw = gemm_tiles(gw);
    ab.add(lv.plan.g_w, gw);
    ab.add(lv.plan.t_w, tw);
    lv.plan.n_tw = (int)tw.size();
  }
  if (preps.empty()) return;
  // the sweep cells go up now (the preparation kernels read them), with the
  // rest of the solve plan added so far
  ab.finish(F.plan_arena_sweep);
  DevBuf<unsigned char> pre_arena;
  pre.finish(pre_arena);
  for (const Prep& P : preps) {
    CellLevel& lv = F.levels[P.lev];
    lv.perm = DevBuf<int>((size_t)std::max<int64_t>(lv.piv_tot, 1));
    lv.Dinv = DevBuf<c64>((size_t)std::max<int64_t>(P.dtot, 1));
    launch_sweep_prepare(lv.sweep.p, lv.n, P.blk_cell.p, P.blk_k.p, P.n_blk, lv.piv.p, lv.A.p, lv.perm.p, lv.Dinv.p,
                         s);
    if (P.n_gt > 0) {
      DevBuf<c64> W((size_t)lv.V.n);
      launch_gemm(P.gd.p, P.gt.p, P.n_gt, P.nmax, 0, lv.At.p, lv.V.p, W.p, 0, s);
      FDS_HIP(hipStreamSynchronize(s));   // the old V goes back to the cache now
      lv.V = std::move(W);
    }
    lv.mfma = true;
    lv.nb_class = sweep_tile_class(lv.bmax);
    lv.nr_class = sweep_tile_class(std::max(P.rmax, 1));
  }
  FDS_HIP(hipStreamSynchronize(s));   // the host arrays of pre_arena go back to the cache
}

// Host part of level lev's solve plan (descriptors, tiles, row maps), into
// the factor's plan arena.  Everything it reads is final once the parent
// level's lists are laid out, so the factorisation calls it right after
// enqueueing the level's merge, while the GPU works.
static void plan_level(Factor& F, int lev) {
  HostTimer ht(6);
  ArenaBuilder& ab = F.plan_ab;
  {
    CellLevel& lv = F.levels[lev];
    CellLevel& pa = F.levels[lev - 1];
    SolveLevel& P = lv.plan;
    std::vector<SolveDesc> sd;
    std::vector<GemmDesc> gv, gat, gd1, gd2;
    for (int q = 0; q < lv.n; ++q) {
      sd.push_back(SolveDesc{lv.a_off[q], lv.piv_off[q], lv.f_off[q], lv.b[q], lv.b[q], (int)lv.B, 0});
      if (lv.r[q] == 0) continue;
      GemmDesc a{};   // T = V g
      a.a_off = lv.v_off[q];
      a.b_off = lv.f_off[q];
      a.c_off = lv.t_off[q];
      a.m = lv.r[q];
      a.k = lv.b[q];
      a.lda = lv.r[q];
      a.ldb = (int)lv.B;
      a.ldc = (int)lv.R;
      a.alpha_re = 1.0;
      gv.push_back(a);
      GemmDesc b{};   // f~ = A~ T
      b.a_off = lv.at_off[q];
      b.b_off = lv.t_off[q];
      b.c_off = lv.t_off[q];
      b.m = lv.r[q];
      b.k = lv.r[q];
      b.lda = lv.r[q];
      b.ldb = (int)lv.R;
      b.ldc = (int)lv.R;
      b.alpha_re = 1.0;
      gat.push_back(b);
      GemmDesc c = b;  // f~ <- A~ y - f~
      c.beta_re = -1.0;
      gd1.push_back(c);
      GemmDesc d{};    // x <- g + X f~
      d.a_off = lv.x_off[q];
      d.b_off = lv.t_off[q];
      d.c_off = lv.f_off[q];
      d.m = lv.b[q];
      d.k = lv.r[q];
      d.lda = lv.b[q];
      d.ldb = (int)lv.R;
      d.ldc = (int)lv.B;
      d.alpha_re = 1.0;
      d.beta_re = 1.0;
      gd2.push_back(d);
    }
    ab.add(P.lu, sd);
    P.n_lu = (int)sd.size();
    P.bmax = lv.bmax;
    auto tv = gemm_tiles(gv), tat = gemm_tiles(gat), td1 = gemm_tiles(gd1), td2 = gemm_tiles(gd2);
    ab.add(P.g_v, gv);
    ab.add(P.g_at, gat);
    ab.add(P.g_dn1, gd1);
    ab.add(P.g_dn2, gd2);
    ab.add(P.t_v, tv);
    ab.add(P.t_at, tat);
    ab.add(P.t_dn1, td1);
    ab.add(P.t_dn2, td2);
    P.n_tv = (int)tv.size();
    P.n_tat = (int)tat.size();
    P.n_tdn1 = (int)td1.size();
    P.n_tdn2 = (int)td2.size();
    std::vector<int64_t> si, di;
    for (int q = 0; q < lv.n; ++q)
      for (int j = 0; j < lv.r[q]; ++j) {
        si.push_back(lv.t_off[q] + j);
        di.push_back(pa.f_off[q / 2] + lv.ppos[q][j]);
      }
    ab.add(P.up_src, si);
    ab.add(P.up_dst, di);
    P.n_up = (int64_t)si.size();
  }
}

// The rest of the solve plan (every level's plan_level has run): the
// matrix-core sweep data, the mixed form's diagonal-block products and the
// leaf DOF maps; then the arena goes up in one copy.
static void build_solve_plan(Factor& F) {
  HostTimer ht(6);
  const int L = F.L, l0 = F.l0;
  ArenaBuilder& ab = F.plan_ab;
  if (F.opt.precision == FDS_PREC_FP64 && F.opt.mfma_sweeps) prepare_mfma_sweeps(F, ab);
  if (F.opt.precision == FDS_PREC_MIXED) {
    // products with the FP64 diagonal blocks (without the children's A~) of
    // every compressed level: y_i = B_i z_i on the level vectors
    for (int lev = L; lev > l0; --lev) {
      CellLevel& lv = F.levels[lev];
      std::vector<GemmDesc> gd;
      for (int q = 0; q < lv.n; ++q) {
        GemmDesc g{};
        g.a_off = lv.a_off[q];
        g.b_off = lv.f_off[q];
        g.c_off = lv.f_off[q];
        g.m = lv.b[q];
        g.k = lv.b[q];
        g.lda = lv.b[q];
        g.ldb = (int)lv.B;
        g.ldc = (int)lv.B;
        g.alpha_re = 1.0;
        gd.push_back(g);
      }
      auto t = gemm_tiles(gd);
      ab.add(lv.g_diag, gd);
      ab.add(lv.t_diag, t);
      lv.n_tdiag = (int)t.size();
    }
  }
  CellLevel& lf = F.levels[L];
  std::vector<int64_t> rows, cols, iota;
  for (int q = 0; q < lf.n; ++q) {
    rows.insert(rows.end(), lf.rows[q].begin(), lf.rows[q].end());
    cols.insert(cols.end(), lf.cols[q].begin(), lf.cols[q].end());
  }
  iota.resize(rows.size());
  std::iota(iota.begin(), iota.end(), 0);
  ab.add(F.leaf_dofs_rows, rows);
  ab.add(F.leaf_dofs_cols, cols);
  ab.add(F.leaf_iota, iota);
  ab.finish(F.plan_arena);
}

// nrhs classes of the autotuner: 1 | 2-8 | 9-32 | 33+
static int nrhs_class(int nrhs) { return nrhs <= 1 ? 0 : nrhs <= 8 ? 1 : nrhs <= 32 ? 2 : 3; }

// Autotuner of the solve sweeps: on the leaf level of the factor itself,
// time each candidate LU-solve chunk and GEMM tile width for a
// representative nrhs of every class and keep the fastest.  Candidates
// only repartition the outputs, so the choice never changes the results.
// Tuning results per (device, leaf block order, leaf skeleton order class):
// later factorisations of the same shape in the process reuse them.
struct TuneKey {
  int device, bmax, rclass;
  bool operator<(const TuneKey& o) const {
    return std::tie(device, bmax, rclass) < std::tie(o.device, o.bmax, o.rclass);
  }
};
struct TuneVal {
  int chunk[4], bn[4];
};
static std::map<TuneKey, TuneVal> g_tune_cache;
static std::mutex g_tune_mutex;

static void autotune_sweeps(Factor& F) {
  if (!F.opt.autotune || F.L == F.l0) return;
  const auto t0 = std::chrono::steady_clock::now();
  CellLevel& lv = F.levels[F.L];
  SolveLevel& P = lv.plan;
  hipStream_t s = F.stream;
  int dev = 0;
  FDS_HIP(hipGetDevice(&dev));
  int rmax = 0;
  for (int q = 0; q < lv.n; ++q) rmax = std::max(rmax, lv.r[q]);
  const TuneKey key{dev, P.bmax, (rmax + 15) / 16};
  {
    std::lock_guard<std::mutex> g(g_tune_mutex);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      for (int c = 0; c < 4; ++c) {
        F.tune_chunk[c] = F.st.tune_chunk[c] = it->second.chunk[c];
        F.tune_bn[c] = F.st.tune_gemm_cols[c] = it->second.bn[c];
      }
      F.st.tune_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      return;
    }
  }
  // the whole leaf level: a subset would not fill the GPU the way the sweeps do
  const int n_lu = P.n_lu, n_tv = P.n_tv;
  const int reps[4] = {1, 8, 32, 128};
  c64* Fb = F.ws.get<c64>("tune_F", (size_t)lv.B * 128);
  c64* Yb = F.ws.get<c64>("tune_Y", (size_t)std::max<int64_t>(lv.R, 1) * 128);
  FDS_HIP(hipMemsetAsync(Fb, 0, (size_t)lv.B * 128 * sizeof(c64), s));
  hipEvent_t e0, e1;
  FDS_HIP(hipEventCreate(&e0));
  FDS_HIP(hipEventCreate(&e1));
  auto timed = [&](auto&& launch) {
    launch();   // warm
    FDS_HIP(hipEventRecord(e0, s));
    launch();
    FDS_HIP(hipEventRecord(e1, s));
    FDS_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    FDS_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms;
  };
  for (int c = 0; c < 4; ++c) {
    const int nrhs = reps[c];
    float best = 1e30f;
    for (int chunk = std::max(1, nrhs / 16); chunk <= 32 && chunk <= std::max(nrhs, 1); chunk *= 2) {
      if (lu_solve_smem(P.bmax, chunk, sizeof(c64)) > 65536) break;
      const float ms = timed([&] {
        launch_lu_solve(P.lu.p, n_lu, P.bmax, nrhs, nrhs, lv.A.p, lv.piv.p, Fb, s, chunk);
      });
      if (ms < best) {
        best = ms;
        F.tune_chunk[c] = chunk;
      }
    }
    best = 1e30f;
    for (int bn : {16, 64}) {
      const float ms = timed([&] {
        launch_gemm(P.g_v.p, P.t_v.p, n_tv, nrhs, nrhs, lv.V.p, Fb, Yb, 0, s, bn);
      });
      if (ms < best) {
        best = ms;
        F.tune_bn[c] = bn;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  TuneVal tv{};
  for (int c = 0; c < 4; ++c) {
    F.st.tune_chunk[c] = tv.chunk[c] = F.tune_chunk[c];
    F.st.tune_gemm_cols[c] = tv.bn[c] = F.tune_bn[c];
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mutex);
    g_tune_cache[key] = tv;
  }
  F.st.tune_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct SweepBufs {
  std::vector<c64*> F, T, Y;
};

// Level vectors of a solve with nrhs columns.  Graph replays use buffers of
// their own per nrhs so that the captured pointers stay valid.
static SweepBufs sweep_buffers(Factor& F, int nrhs, const std::string& prefix) {
  SweepBufs b;
  b.F.assign(F.L + 1, nullptr);
  b.T.assign(F.L + 1, nullptr);
  b.Y.assign(F.L + 1, nullptr);
  for (int lev = F.l0; lev <= F.L; ++lev) {
    const std::string l = std::to_string(lev);
    b.F[lev] = F.ws.get<c64>(prefix + "F" + l, (size_t)F.levels[lev].B * nrhs);
    if (lev > F.l0) {
      b.T[lev] = F.ws.get<c64>(prefix + "T" + l, (size_t)F.levels[lev].R * nrhs);
      b.Y[lev] = F.ws.get<c64>(prefix + "Y" + l, (size_t)F.levels[lev].R * nrhs);
    }
  }
  return b;
}

// Upward sweep, root solve, downward sweep on the level vectors (pure
// launch sequence: no allocation, no host work, no synchronisation).
static void run_sweeps(Factor& F, int nrhs, const SweepBufs& b, hipStream_t s) {
  const int L = F.L, l0 = F.l0;
  auto& levels = F.levels;
  const int ck = F.tune_chunk[nrhs_class(nrhs)], bn = F.tune_bn[nrhs_class(nrhs)];
  auto sweep_launch = [&](int lev) {
    CellLevel& lv = levels[lev];
    SweepLaunch SL;
    SL.cells = lv.sweep.p;
    SL.n_cells = lv.n;
    SL.n_slab = (nrhs + 15) / 16;
    SL.ncol = nrhs;
    SL.nb_class = lv.nb_class;
    SL.nr_class = lv.nr_class;
    SL.A = lv.A.p;
    SL.Dinv = lv.Dinv.p;
    SL.perm = lv.perm.p;
    SL.W = lv.V.p;
    SL.At = lv.At.p;
    SL.X = lv.X.p;
    SL.up_dst = lv.plan.up_dst.p;
    SL.F = b.F[lev];
    SL.ldF = lv.B;
    SL.T = b.T[lev];
    SL.ldT = lv.R;
    SL.Fp = b.F[lev - 1];
    SL.ldFp = levels[lev - 1].B;
    return SL;
  };
  // upward: g = A^{-1} f (in F), f~ = A~ (V g) (V g in Y, f~ in T)
  for (int lev = L; lev > l0; --lev) {
    CellLevel& lv = levels[lev];
    SolveLevel& P = lv.plan;
    if (lv.mfma && nrhs >= kSweepMinCols) {   // one launch: g, f~ and the parent's rows
      launch_sweep_up(sweep_launch(lev), s);
      continue;
    }
    if (lv.mfma && nrhs <= kSweepFewCols) {
      launch_sweep_few(sweep_launch(lev), true, s);
      continue;
    }
    launch_lu_solve(P.lu.p, P.n_lu, P.bmax, nrhs, nrhs, lv.A.p, lv.piv.p, b.F[lev], s, ck);
    if (lv.mfma) {   // V holds W = A~ V
      launch_gemm(P.g_w.p, P.t_w.p, P.n_tw, nrhs, nrhs, lv.V.p, b.F[lev], b.T[lev], 0, s, bn);
      launch_copy_rows(P.n_up, P.up_src.p, P.up_dst.p, nrhs, b.T[lev], lv.R, b.F[lev - 1], levels[lev - 1].B, s);
      continue;
    }
    launch_gemm(P.g_v.p, P.t_v.p, P.n_tv, nrhs, nrhs, lv.V.p, b.F[lev], b.Y[lev], 0, s, bn);
    launch_gemm(P.g_at.p, P.t_at.p, P.n_tat, nrhs, nrhs, lv.At.p, b.Y[lev], b.T[lev], 0, s, bn);
    launch_copy_rows(P.n_up, P.up_src.p, P.up_dst.p, nrhs, b.T[lev], lv.R, b.F[lev - 1], levels[lev - 1].B, s);
  }
  launch_lu_solve(F.root.desc.p, 1, F.root.n, nrhs, nrhs, F.root.A.p, F.root.piv.p, b.F[l0], s, ck);
  // downward: y from the parent (in Y), f~ <- A~ y - f~, x = g + X f~
  for (int lev = l0 + 1; lev <= L; ++lev) {
    CellLevel& lv = levels[lev];
    SolveLevel& P = lv.plan;
    if (lv.mfma && nrhs <= kSweepFewCols) {
      launch_sweep_few(sweep_launch(lev), false, s);
      continue;
    }
    launch_copy_rows(P.n_up, P.up_dst.p, P.up_src.p, nrhs, b.F[lev - 1], levels[lev - 1].B, b.Y[lev], lv.R, s);
    launch_gemm(P.g_dn1.p, P.t_dn1.p, P.n_tdn1, nrhs, nrhs, lv.At.p, b.Y[lev], b.T[lev], 0, s, bn);
    launch_gemm(P.g_dn2.p, P.t_dn2.p, P.n_tdn2, nrhs, nrhs, lv.X.p, b.T[lev], b.F[lev], 0, s, bn);
  }
}

// Run ``launches`` (a pure launch sequence) directly, or as a hipGraph
// captured on first use under ``key`` and replayed afterwards.
template <typename Fn>
static void run_maybe_captured(Factor& F, bool graph, int64_t key, hipStream_t s, Fn&& launches) {
  if (!graph) {
    launches();
    return;
  }
  auto it = F.graphs.find(key);
  if (it == F.graphs.end()) {
    hipGraph_t g;
    FDS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      launches();
    } catch (...) {
      hipGraph_t dummy;
      (void)hipStreamEndCapture(s, &dummy);
      throw;
    }
    FDS_HIP(hipStreamEndCapture(s, &g));
    hipGraphExec_t ex;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    FDS_HIP(e);
    it = F.graphs.emplace(key, ex).first;
  }
  FDS_HIP(hipGraphLaunch(it->second, s));
}

static void run_solve(Factor& F, int nrhs, const c64* rhs, int64_t ld_rhs, c64* x, int64_t ld_x, hipStream_t s,
                      bool graph) {
  CellLevel& lf = F.levels[F.L];
  const SweepBufs b = sweep_buffers(F, nrhs, graph ? "g" + std::to_string(nrhs) + "_" : "sv_");
  launch_copy_rows(lf.B, F.leaf_dofs_rows.p, F.leaf_iota.p, nrhs, rhs, ld_rhs, b.F[F.L], lf.B, s);
  run_maybe_captured(F, graph, 4 * (int64_t)nrhs, s, [&] { run_sweeps(F, nrhs, b, s); });
  launch_copy_rows(lf.B, F.leaf_iota.p, F.leaf_dofs_cols.p, nrhs, b.F[F.L], lf.B, x, ld_x, s);
}

// ------------------------------------------------------------------ solve without allocation
// Device scratch of fds_solve_noalloc: the sweep level vectors of one call,
// carved from one file-scope array.  Each device holds its own copy at its
// own address; host code uses only the addresses returned by
// hipGetSymbolAddress (the array's name in host code is not a device address).
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, unsigned char*> g_scratch_addr;   // device -> address of ``scratch`` there

static unsigned char* scratch_address() {
  int dev = 0;
  FDS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  void* p = nullptr;
  FDS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error(FDS_EHIP, "no device address for the solve scratch");
  g_scratch_addr[dev] = static_cast<unsigned char*>(p);
  return static_cast<unsigned char*>(p);
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// bytes of the level vectors of a solve with nrhs columns (as sweep_buffers)
static size_t sweep_scratch_bytes(const Factor& F, int nrhs) {
  size_t tot = 0;
  for (int lev = F.l0; lev <= F.L; ++lev) {
    tot += align256((size_t)F.levels[lev].B * nrhs * sizeof(c64));
    if (lev > F.l0) tot += 2 * align256((size_t)F.levels[lev].R * nrhs * sizeof(c64));
  }
  return tot;
}

static SweepBufs sweep_buffers_at(const Factor& F, int nrhs, unsigned char* base) {
  SweepBufs b;
  b.F.assign(F.L + 1, nullptr);
  b.T.assign(F.L + 1, nullptr);
  b.Y.assign(F.L + 1, nullptr);
  size_t off = 0;
  for (int lev = F.l0; lev <= F.L; ++lev) {
    b.F[lev] = reinterpret_cast<c64*>(base + off);
    off += align256((size_t)F.levels[lev].B * nrhs * sizeof(c64));
    if (lev > F.l0) {
      b.T[lev] = reinterpret_cast<c64*>(base + off);
      off += align256((size_t)F.levels[lev].R * nrhs * sizeof(c64));
      b.Y[lev] = reinterpret_cast<c64*>(base + off);
      off += align256((size_t)F.levels[lev].R * nrhs * sizeof(c64));
    }
  }
  return b;
}

// ------------------------------------------------------------------ mixed form
struct MixedBufs {
  std::vector<c32*> F, T, Y;   // FP32 sweep level vectors
  c64* root = nullptr;         // FP64 root vector (order of the root system x nrhs)
  std::vector<c64*> Z, W, M;   // compressed-operator product: input, output and skeleton level vectors
  c64* f = nullptr;            // right-hand sides in leaf row order
  double* norms = nullptr;     // |f|^2, |r|^2, |x|^2, |delta|^2 per column
};

static MixedBufs mixed_buffers(Factor& F, int nrhs, const std::string& prefix) {
  MixedBufs b;
  b.F.assign(F.L + 1, nullptr);
  b.T.assign(F.L + 1, nullptr);
  b.Y.assign(F.L + 1, nullptr);
  b.Z.assign(F.L + 1, nullptr);
  b.W.assign(F.L + 1, nullptr);
  b.M.assign(F.L + 1, nullptr);
  for (int lev = F.l0; lev <= F.L; ++lev) {
    const std::string l = std::to_string(lev);
    const size_t nb = (size_t)F.levels[lev].B * nrhs;
    b.F[lev] = F.ws.get<c32>(prefix + "F32_" + l, nb);
    b.Z[lev] = F.ws.get<c64>(prefix + "Z" + l, nb);
    b.W[lev] = F.ws.get<c64>(prefix + "W" + l, nb);
    if (lev > F.l0) {
      const size_t nr = (size_t)F.levels[lev].R * nrhs;
      b.T[lev] = F.ws.get<c32>(prefix + "T32_" + l, nr);
      b.Y[lev] = F.ws.get<c32>(prefix + "Y32_" + l, nr);
      b.M[lev] = F.ws.get<c64>(prefix + "M" + l, nr);
    }
  }
  b.root = F.ws.get<c64>(prefix + "root", (size_t)F.root.n * nrhs);
  b.f = F.ws.get<c64>(prefix + "f", (size_t)F.levels[F.L].B * nrhs);
  b.norms = F.ws.get<double>(prefix + "norms", (size_t)4 * nrhs);
  return b;
}

// FP32 upward sweep, FP64 root solve, FP32 downward sweep: F[L] <- A_c^{-1} F[L]
// (the same plan as the plain form on the FP32 factors).
static void run_sweeps32(Factor& F, int nrhs, const MixedBufs& b, hipStream_t s) {
  const int L = F.L, l0 = F.l0;
  auto& levels = F.levels;
  const int ck = F.tune_chunk[nrhs_class(nrhs)], bn = F.tune_bn[nrhs_class(nrhs)];
  for (int lev = L; lev > l0; --lev) {
    CellLevel& lv = levels[lev];
    SolveLevel& P = lv.plan;
    launch_lu_solve(P.lu.p, P.n_lu, P.bmax, nrhs, nrhs, lv.A32.p, lv.piv.p, b.F[lev], s, ck);
    launch_gemm(P.g_v.p, P.t_v.p, P.n_tv, nrhs, nrhs, lv.V32.p, b.F[lev], b.Y[lev], 0, s, bn);
    launch_gemm(P.g_at.p, P.t_at.p, P.n_tat, nrhs, nrhs, lv.At32.p, b.Y[lev], b.T[lev], 0, s, bn);
    launch_copy_rows(P.n_up, P.up_src.p, P.up_dst.p, nrhs, b.T[lev], lv.R, b.F[lev - 1], levels[lev - 1].B, s);
  }
  const int64_t nroot = (int64_t)F.root.n * nrhs;
  launch_convert(nroot, b.F[l0], b.root, s);
  launch_lu_solve(F.root.desc.p, 1, F.root.n, nrhs, nrhs, F.root.A.p, F.root.piv.p, b.root, s, ck);
  launch_convert(nroot, b.root, b.F[l0], s);
  for (int lev = l0 + 1; lev <= L; ++lev) {
    CellLevel& lv = levels[lev];
    SolveLevel& P = lv.plan;
    launch_copy_rows(P.n_up, P.up_dst.p, P.up_src.p, nrhs, b.F[lev - 1], levels[lev - 1].B, b.Y[lev], lv.R, s);
    launch_gemm(P.g_dn1.p, P.t_dn1.p, P.n_tdn1, nrhs, nrhs, lv.At32.p, b.Y[lev], b.T[lev], 0, s, bn);
    launch_gemm(P.g_dn2.p, P.t_dn2.p, P.n_tdn2, nrhs, nrhs, lv.X32.p, b.T[lev], b.F[lev], 0, s, bn);
  }
}

// W[L] = A_c Z[L] in FP64 through the nested form of the compressed operator:
// A_c = B_L + U_L (B_{L-1} + U_{L-1} ( ... B_l0 ... ) V_{L-1}) V_L, where B_l
// holds the FP64 diagonal blocks of level l without the children's A~
// (the plain leaf blocks at L) and B_l0 the root system likewise.
static void run_apply(Factor& F, int nrhs, const MixedBufs& b, hipStream_t s) {
  const int L = F.L, l0 = F.l0;
  auto& levels = F.levels;
  const int bn = F.tune_bn[nrhs_class(nrhs)];
  for (int lev = L; lev > l0; --lev) {   // skeleton values z_{l-1} = V_l z_l
    CellLevel& lv = levels[lev];
    SolveLevel& P = lv.plan;
    launch_gemm(P.g_v.p, P.t_v.p, P.n_tv, nrhs, nrhs, lv.V.p, b.Z[lev], b.M[lev], 0, s, bn);
    launch_copy_rows(P.n_up, P.up_src.p, P.up_dst.p, nrhs, b.M[lev], lv.R, b.Z[lev - 1], levels[lev - 1].B, s);
  }
  launch_gemm(F.root.g_b.p, F.root.t_b.p, F.root.n_tb, nrhs, nrhs, F.root.B.p, b.Z[l0], b.W[l0], 0, s, bn);
  for (int lev = l0 + 1; lev <= L; ++lev) {   // w_l = B_l z_l + U_l w_{l-1}
    CellLevel& lv = levels[lev];
    SolveLevel& P = lv.plan;
    launch_copy_rows(P.n_up, P.up_dst.p, P.up_src.p, nrhs, b.W[lev - 1], levels[lev - 1].B, b.M[lev], lv.R, s);
    launch_gemm(lv.g_diag.p, lv.t_diag.p, lv.n_tdiag, nrhs, nrhs, lv.A.p, b.Z[lev], b.W[lev], 0, s, bn);
    launch_gemm(P.g_dn2.p, P.t_dn2.p, P.n_tdn2, nrhs, nrhs, lv.X.p, b.M[lev], b.W[lev], 0, s, bn);
  }
}

// Iterative refinement against the FP64 compressed operator (mixed form).
// Returns FDS_OK or FDS_ENOCONV; x is written in both cases.
static int run_solve_mixed(Factor& F, int nrhs, const c64* rhs, int64_t ld_rhs, c64* x, int64_t ld_x, hipStream_t s,
                           bool graph) {
  CellLevel& lf = F.levels[F.L];
  const int L = F.L;
  const int64_t nl = lf.B * (int64_t)nrhs;
  const MixedBufs b = mixed_buffers(F, nrhs, graph ? "mg" + std::to_string(nrhs) + "_" : "mx_");
  launch_copy_rows(lf.B, F.leaf_dofs_rows.p, F.leaf_iota.p, nrhs, rhs, ld_rhs, b.f, lf.B, s);
  launch_colnorm2(lf.B, nrhs, b.f, lf.B, b.norms, s);
  launch_convert(nl, b.f, b.F[L], s);
  run_maybe_captured(F, graph, 4 * (int64_t)nrhs + 1, s, [&] { run_sweeps32(F, nrhs, b, s); });
  launch_convert(nl, b.F[L], b.Z[L], s);   // x_0 in leaf column order
  std::vector<double> h(4 * (size_t)nrhs);
  int it = 0, status = FDS_OK;
  double res = 0.0, cor = 1.0;
  for (;;) {
    run_maybe_captured(F, graph, 4 * (int64_t)nrhs + 2, s, [&] { run_apply(F, nrhs, b, s); });
    launch_axpby(nl, 1.0, b.f, -1.0, b.W[L], s);   // r = f - A_c x
    launch_colnorm2(lf.B, nrhs, b.W[L], lf.B, b.norms + nrhs, s);
    launch_colnorm2(lf.B, nrhs, b.Z[L], lf.B, b.norms + 2 * nrhs, s);
    FDS_HIP(hipMemcpyAsync(h.data(), b.norms, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    FDS_HIP(hipStreamSynchronize(s));
    res = 0.0;
    cor = it == 0 ? 1.0 : 0.0;
    for (int k = 0; k < nrhs; ++k) {
      const double f2 = h[k], r2 = h[nrhs + k], x2 = h[2 * nrhs + k], d2 = h[3 * nrhs + k];
      res = std::max(res, f2 > 0 ? std::sqrt(r2 / f2) : (r2 > 0 ? INFINITY : 0.0));
      if (it > 0) cor = std::max(cor, x2 > 0 ? std::sqrt(d2 / x2) : (d2 > 0 ? INFINITY : 0.0));
    }
    if (!std::isfinite(res)) throw Error(FDS_ESINGULAR, "mixed solve: non-finite residual");
    if (res <= F.opt.ir_rtol && cor <= F.opt.ir_dtol) break;
    if (it >= F.opt.ir_max_iter) {
      status = FDS_ENOCONV;
      break;
    }
    launch_convert(nl, b.W[L], b.F[L], s);
    run_maybe_captured(F, graph, 4 * (int64_t)nrhs + 1, s, [&] { run_sweeps32(F, nrhs, b, s); });
    launch_colnorm2(lf.B, nrhs, b.F[L], lf.B, b.norms + 3 * nrhs, s);
    launch_add_c32(nl, b.F[L], b.Z[L], s);
    ++it;
  }
  launch_copy_rows(lf.B, F.leaf_iota.p, F.leaf_dofs_cols.p, nrhs, b.Z[L], lf.B, x, ld_x, s);
  F.st.ir_iterations = it;
  F.st.ir_residual = res;
  F.st.ir_correction = cor;
  return status;
}

static void resolve_stats(Factor& F) {
  F.ast.resolve(F.stream);
  FDS_HIP(hipStreamSynchronize(F.stream));
  for (auto& sp : F.spans) {
    float ms = 0.f;
    FDS_HIP(hipEventElapsedTime(&ms, sp.a, sp.b));
    double* dst = sp.what == 0 ? &F.st.id_seconds : (sp.what == 1 ? &F.st.merge_seconds : &F.st.root_seconds);
    *dst += 1e-3 * ms;
    (void)hipEventDestroy(sp.a);
    (void)hipEventDestroy(sp.b);
  }
  F.spans.clear();
}

}  // namespace fds

using namespace fds;

static int translate(const std::exception& e) {
  if (auto* x = dynamic_cast<const Error*>(&e)) return x->code;
  return FDS_EHIP;
}

static thread_local std::string g_last_error;

extern "C" {

int fds_options_default(fds_options* o) {
  if (!o) return FDS_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->leaf_nodes = 64;
  o->n_proxy = 64;
  o->root_level = 1;
  o->proxy_ratio = 1.5;
  o->use_alpha = 0;
  o->precision = FDS_PREC_FP64;
  o->ir_max_iter = 10;
  o->ir_rtol = 1e-8;
  o->ir_dtol = 1e-6;
  o->rank_mode = FDS_RANK_ADAPTIVE;
  o->oversample = 10;
  o->seed = 0x5EED;
  o->predictor = nullptr;
  o->autotune = 1;
  o->mfma_sweeps = 1;
  return FDS_OK;
}

static int check_material(double omega, double lam, double mu, double rho) {
  if (!(omega > 0) || !(mu > 0) || !(lam + mu > 0) || !(rho > 0)) return FDS_EINVAL;
  return FDS_OK;
}

int fds_build(const fds_geometry* geom, double omega, double lambda, double mu, double rho, double tol,
              const fds_options* opt, void* stream, fds_factor* out) {
  AllocScope scope((hipStream_t)stream);
  if (!out) return FDS_EINVAL;
  if (int e = check_material(omega, lambda, mu, rho)) return e;
  if (!(tol > 0.0 && tol < 1.0)) return FDS_EINVAL;
  fds_options o;
  fds_options_default(&o);
  if (opt) o = *opt;
  if (o.leaf_nodes < 4 || o.n_proxy < 8 || o.root_level < 0 || !(o.proxy_ratio > 1.0)) return FDS_EINVAL;
  if (o.precision != FDS_PREC_FP64 && o.precision != FDS_PREC_MIXED) return FDS_EINVAL;
  if (o.precision == FDS_PREC_MIXED && (o.ir_max_iter < 0 || !(o.ir_rtol > 0) || !(o.ir_dtol > 0)))
    return FDS_EINVAL;
  if (o.rank_mode != FDS_RANK_ADAPTIVE && o.rank_mode != FDS_RANK_LEARNED) return FDS_EINVAL;
  if (o.rank_mode == FDS_RANK_LEARNED && (!o.predictor || o.oversample < 0 || o.oversample > kSketchMaxS))
    return FDS_EINVAL;
  auto* F = new Factor();
  try {
    if (int e = make_geometry(geom, F->G)) {
      delete F;
      return e;
    }
    const auto t0 = std::chrono::steady_clock::now();
    ensure_quad();
    F->opt = o;
    F->tol = tol;
    F->lam = lambda;
    F->mu = mu;
    F->rho = rho;
    F->omega = omega;
    F->stream = (hipStream_t)stream;
    F->ws.set_stream(F->stream);
    F->m = make_mat(omega, lambda, mu, rho, o, nullptr, nullptr);
    if (F->m.kT * F->G.hmax > kKhMax) {   // the quadrature rules hold up to k_T h = kKhMax
      delete F;
      return FDS_EGEOM;
    }
    if (o.rank_mode == FDS_RANK_LEARNED) {
      F->pred = DevBuf<float>(std::vector<float>(o.predictor, o.predictor + kMlpBlob));
      F->opt.predictor = nullptr;   // the caller's array is not kept
    }
    F->st.rank_mode = o.rank_mode;
    build_tree(*F);
    F->sing = DevBuf<int>((size_t)F->L + 1);
    FDS_HIP(hipMemsetAsync(F->sing.p, 0, F->sing.n * sizeof(int), F->stream));
    const int64_t proxy_cap = (int64_t)F->levels[F->L].n * o.n_proxy;
    F->DG.init(F->G, proxy_cap, F->stream);
    assemble_leaves(*F);
    // level lev - 1's interaction matrices are enqueued behind level lev's
    // elimination (their host work overlaps it), before the parent blocks
    if (F->L > F->l0) prepare_level(*F, F->L);
    for (int lev = F->L; lev > F->l0; --lev) {
      compress_level(*F, lev);
      merge_lists(*F, lev);
      if (lev - 1 > F->l0) prepare_level(*F, lev - 1);
      merge_blocks(*F, lev);
      plan_level(*F, lev);
    }
    factor_root(*F);
    build_solve_plan(*F);
    autotune_sweeps(*F);
    FDS_HIP(hipStreamSynchronize(F->stream));
    const auto t1 = std::chrono::steady_clock::now();
    {
      const auto sing = download(F->ws, F->sing.p, F->sing.n);
      for (int lev = 0; lev <= F->L; ++lev)
        if (sing[lev])
          throw Error(FDS_ESINGULAR, lev == F->l0 ? std::string("singular root LU")
                                                  : "singular block LU at level " + std::to_string(lev));
    }
    resolve_stats(*F);
    if (std::getenv("FDS_TIMING")) {
      for (int k = 0; k < 9; ++k) std::fprintf(stderr, "[fds host] %-22s %8.2f ms\n", g_host_name[k], 1e3 * g_host_t[k]);
      std::fprintf(stderr, "[fds host] factor wall %8.2f ms\n", 1e3 * std::chrono::duration<double>(t1 - t0).count());
    }
    for (double& v : g_host_t) v = 0.0;
    F->st.factor_seconds = std::chrono::duration<double>(t1 - t0).count();
    F->st.levels = F->L;
    F->st.root_level = F->l0;
    F->st.n_unknowns = 2 * (int64_t)F->G.n_nodes;
    F->st.root_size = F->root.n;
    int64_t bytes = 0;
    for (auto& lv : F->levels)
      bytes += (int64_t)(lv.A.n + lv.X.n + lv.At.n + lv.V.n + lv.Dinv.n) * sizeof(c64) +
               (int64_t)(lv.A32.n + lv.X32.n + lv.At32.n + lv.V32.n) * sizeof(c32) +
               (lv.piv.n + lv.s_piv.n + lv.perm.n) * sizeof(int) + lv.sweep.n * sizeof(SweepCell);
    bytes += (int64_t)(F->root.A.n + F->root.B.n) * sizeof(c64);
    F->st.precision = o.precision;
    F->st.factor_bytes = bytes;
    F->st.assembly_seconds = F->ast.seconds;
    F->st.kernel_evals = F->ast.evals;
    for (int c = 0; c < kNumPublicClass; ++c) {
      F->st.class_seconds[c] = F->ast.class_seconds[c];
      F->st.class_evals[c] = F->ast.class_evals[c];
      F->st.class_launches[c] = F->ast.class_launches[c];
    }
    for (int li = 0; li < kNumPairLaunches; ++li) {
      F->st.pair_kernel_seconds[li] = F->ast.kernel_seconds[li];
      F->st.pair_kernel_evals[li] = F->ast.kernel_evals[li];
      F->st.pair_kernel_launches[li] = F->ast.kernel_launches[li];
    }
    *out = F;
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    int c = translate(e);
    if (F->stream) (void)hipStreamSynchronize(F->stream);
    delete F;
    return c;
  }
}

int fds_size(fds_factor f, int64_t* n) {
  if (!f || !n) return FDS_EINVAL;
  *n = 2 * (int64_t)f->G.n_nodes;
  return FDS_OK;
}

int fds_rhs_plane(fds_factor f, int32_t nrhs, const int32_t* kind, const double* angle, fds_c64* rhs, int64_t ld,
                  void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (!f || nrhs < 1 || !kind || !angle || !rhs || ld < 2 * (int64_t)f->G.n_nodes) return FDS_EINVAL;
  try {
    for (int k = 0; k < nrhs; ++k)
      if (kind[k] != 0 && kind[k] != 1) return FDS_EINVAL;
    ensure_quad();
    hipStream_t s = (hipStream_t)stream;
    DevBuf<int> dk(std::vector<int>(kind, kind + nrhs));
    DevBuf<double> da(std::vector<double>(angle, angle + nrhs));
    launch_rhs_plane(f->DG.elems.p, f->DG.prev_elem.p, f->G.n_nodes, f->m, f->lam, nrhs, dk.p, da.p, (c64*)rhs, ld, s);
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_solve(fds_factor f, int32_t nrhs, const fds_c64* rhs, int64_t ld_rhs, fds_c64* x, int64_t ld_x, void* stream) {
  const int64_t N = f ? 2 * (int64_t)f->G.n_nodes : 0;
  if (!f || nrhs < 1 || !rhs || !x || ld_rhs < N || ld_x < N) return FDS_EINVAL;
  try {
    hipStream_t s = (hipStream_t)stream;
    const bool graph = f->opt.solve_graph != 0;
    if (graph) {
      // capture needs a stream of our own; the caller's stream is drained first
      FDS_HIP(hipStreamSynchronize(s));
      if (!f->gstream) FDS_HIP(hipStreamCreateWithFlags(&f->gstream, hipStreamNonBlocking));
      s = f->gstream;
    }
    if (s != f->ws.stream()) {
      // workspace buffers are reused in stream order: keep them on one stream
      FDS_HIP(hipStreamSynchronize(f->ws.stream()));
      f->ws.set_stream(s);
    }
    AllocScope scope(s);
    int status = FDS_OK;
    if (f->opt.precision == FDS_PREC_MIXED)
      status = run_solve_mixed(*f, nrhs, (const c64*)rhs, ld_rhs, (c64*)x, ld_x, s, graph);
    else
      run_solve(*f, nrhs, (const c64*)rhs, ld_rhs, (c64*)x, ld_x, s, graph);
    FDS_HIP(hipStreamSynchronize(s));
    if (status == FDS_ENOCONV) g_last_error = "iterative refinement did not reach its tolerance";
    return status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_solve_noalloc(fds_factor f, int32_t nrhs, const fds_c64* rhs, int64_t ld_rhs, fds_c64* x, int64_t ld_x,
                      void* stream) {
  const int64_t N = f ? 2 * (int64_t)f->G.n_nodes : 0;
  if (!f || nrhs < 1 || nrhs > 65535 || !rhs || !x || ld_rhs < N || ld_x < N) return FDS_EINVAL;
  if (f->opt.precision != FDS_PREC_FP64) {
    g_last_error = "fds_solve_noalloc: the mixed-precision form needs refinement buffers; use fds_solve";
    return FDS_EINVAL;
  }
  const size_t need = sweep_scratch_bytes(*f, nrhs);
  if (need > kNoAllocScratchBytes) {
    g_last_error = "fds_solve_noalloc: " + std::to_string(nrhs) + " right-hand sides need " +
                   std::to_string(need >> 20) + " MiB of scratch, more than its " +
                   std::to_string(kNoAllocScratchBytes >> 20) + " MiB: solve fewer at a time";
    return FDS_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    unsigned char* base = scratch_address();
    const SweepBufs b = sweep_buffers_at(*f, nrhs, base);
    CellLevel& lf = f->levels[f->L];
    // every level vector is written before it is read: nothing to clear
    launch_copy_rows(lf.B, f->leaf_dofs_rows.p, f->leaf_iota.p, nrhs, (const c64*)rhs, ld_rhs, b.F[f->L], lf.B, s);
    run_sweeps(*f, nrhs, b, s);
    launch_copy_rows(lf.B, f->leaf_iota.p, f->leaf_dofs_cols.p, nrhs, b.F[f->L], lf.B, (c64*)x, ld_x, s);
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_apply(fds_factor f, int32_t nrhs, const fds_c64* x, int64_t ld_x, fds_c64* y, int64_t ld_y, void* stream) {
  AllocScope scope((hipStream_t)stream);
  const int64_t N = f ? 2 * (int64_t)f->G.n_nodes : 0;
  if (!f || nrhs < 1 || !x || !y || ld_x < N || ld_y < N) return FDS_EINVAL;
  if (f->opt.precision != FDS_PREC_MIXED) {
    g_last_error = "fds_apply needs a factor built with FDS_PREC_MIXED";
    return FDS_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    if (s != f->ws.stream()) {
      FDS_HIP(hipStreamSynchronize(f->ws.stream()));
      f->ws.set_stream(s);
    }
    Factor& F = *f;
    CellLevel& lf = F.levels[F.L];
    const MixedBufs b = mixed_buffers(F, nrhs, "ap_");
    launch_copy_rows(lf.B, F.leaf_dofs_cols.p, F.leaf_iota.p, nrhs, (const c64*)x, ld_x, b.Z[F.L], lf.B, s);
    run_apply(F, nrhs, b, s);
    launch_copy_rows(lf.B, F.leaf_iota.p, F.leaf_dofs_rows.p, nrhs, b.W[F.L], lf.B, (c64*)y, ld_y, s);
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_get_stats(fds_factor f, fds_stats* s) {
  if (!f || !s) return FDS_EINVAL;
  *s = f->st;
  return FDS_OK;
}

int fds_get_ranks(fds_factor f, int32_t* out, int64_t n_out) {
  if (!f || !out) return FDS_EINVAL;
  const int64_t ncell = (2LL << f->L) - 1;
  if (n_out < 4 * ncell) return FDS_EINVAL;
  for (int64_t i = 0; i < 4 * ncell; ++i) out[i] = -1;
  for (int lev = f->l0 + 1; lev <= f->L; ++lev) {
    const CellLevel& lv = f->levels[lev];
    for (int q = 0; q < lv.n; ++q) {
      const int64_t c = (1LL << lev) - 1 + q;
      out[4 * c] = lv.kr0[q];
      out[4 * c + 1] = lv.kc0[q];
      out[4 * c + 2] = lv.kr1[q];
      out[4 * c + 3] = lv.kc1[q];
    }
  }
  return FDS_OK;
}

int fds_get_skeleton(fds_factor f, int32_t cell, int64_t* rows, int64_t* cols, int64_t cap, int64_t* n_out) {
  if (!f || !rows || !cols || !n_out || cell < 0) return FDS_EINVAL;
  int lev = 0;
  while (((2LL << lev) - 1) <= cell) ++lev;
  if (lev > f->L || lev <= f->l0) return FDS_EINVAL;
  const CellLevel& lv = f->levels[lev];
  const int q = cell - ((1 << lev) - 1);
  const int64_t k = (int64_t)lv.rskel[q].size();
  if (cap < k) return FDS_EINVAL;
  std::copy(lv.rskel[q].begin(), lv.rskel[q].end(), rows);
  std::copy(lv.cskel[q].begin(), lv.cskel[q].end(), cols);
  *n_out = k;
  return FDS_OK;
}

void fds_release_cache(void) { cache_release(); }

int64_t fds_cached_bytes(void) { return (int64_t)cache_bytes(); }

int fds_set_allocator(fds_alloc_fn alloc, fds_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) return FDS_EINVAL;
  UserAllocator u;
  u.alloc = alloc;
  u.free = free_fn;
  u.ctx = alloc ? ctx : nullptr;
  if (!set_user_allocator(u)) {
    g_last_error = "device blocks are still held (destroy every factor first)";
    return FDS_EINVAL;
  }
  return FDS_OK;
}

void fds_destroy(fds_factor f) {
  if (!f) return;
  if (f->ws.stream()) (void)hipStreamSynchronize(f->ws.stream());
  delete f;
}

const char* fds_strerror(int code) {
  switch (code) {
    case FDS_OK: return "ok";
    case FDS_EINVAL: return "invalid argument";
    case FDS_EGEOM: return "invalid geometry";
    case FDS_ENOMEM: return "out of memory";
    case FDS_EHIP: return "HIP runtime error";
    case FDS_ESINGULAR: return "singular pivot";
    case FDS_ENOCONV: return "iterative refinement did not converge";
    default: return "unknown error";
  }
}

const char* fds_last_error(void) { return g_last_error.c_str(); }

int fds_entries(const fds_geometry* geom, double omega, double lambda, double mu, double rho, const fds_options* opt,
                int64_t nr, const int64_t* rows, int64_t nc, const int64_t* cols, fds_c64* out, int64_t ld,
                void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (int e = check_material(omega, lambda, mu, rho)) return e;
  if (nr < 1 || nc < 1 || !rows || !cols || !out || ld < nr) return FDS_EINVAL;
  fds_options o;
  fds_options_default(&o);
  if (opt) o = *opt;
  try {
    Geometry G;
    if (int e = make_geometry(geom, G)) return e;
    for (int64_t i = 0; i < nr; ++i)
      if (rows[i] < 0 || rows[i] >= 2 * (int64_t)G.n_nodes) return FDS_EINVAL;
    for (int64_t i = 0; i < nc; ++i)
      if (cols[i] < 0 || cols[i] >= 2 * (int64_t)G.n_nodes) return FDS_EINVAL;
    ensure_quad();
    hipStream_t s = (hipStream_t)stream;
    DevGeom DG;
    DG.init(G, 0, s);
    MatConst m = make_mat(omega, lambda, mu, rho, o, nullptr, nullptr);
    BlockReq q;
    q.rows = side_from_dofs(G, std::vector<int64_t>(rows, rows + nr));
    q.cols = side_from_dofs(G, std::vector<int64_t>(cols, cols + nc));
    q.out_off = 0;
    q.rs = 1;
    q.cs = ld;
    Workspace ws(s);
    assemble_blocks(std::vector<BlockReq>{q}, DG.elems.p, m, (c64*)out, ws, nullptr);
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    if (stream) (void)hipStreamSynchronize((hipStream_t)stream);
    return translate(e);
  }
}

int fds_field(const fds_geometry* geom, double omega, double lambda, double mu, double rho, int32_t nrhs,
              const fds_c64* x, int64_t ld_x, int64_t n_target, const double* targets, const int32_t* kind,
              const double* angle, fds_c64* out, int64_t ld_out, int64_t* n_near, void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (int e = check_material(omega, lambda, mu, rho)) return e;
  if (nrhs < 0 || nrhs > 65535 || n_target < 0 || (kind == nullptr) != (angle == nullptr)) return FDS_EINVAL;
  if (kind)
    for (int32_t r = 0; r < nrhs; ++r)
      if (kind[r] != 0 && kind[r] != 1) return FDS_EINVAL;
  try {
    Geometry G;
    if (int e = make_geometry(geom, G)) return e;
    const int64_t nu = 2 * (int64_t)G.n_nodes;
    if (nrhs == 0 || n_target == 0) {
      if (n_near) *n_near = 0;
      return FDS_OK;
    }
    if (!x || !targets || !out || ld_x < nu || ld_out < 2 * n_target || ld_x > INT32_MAX || ld_out > INT32_MAX)
      return FDS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    ensure_quad();
    ensure_field_quad();
    DevGeom DG;
    DG.init(G, 0, s);
    fds_options o;
    fds_options_default(&o);
    const MatConst m = make_mat(omega, lambda, mu, rho, o, nullptr, nullptr);
    Workspace ws(s);
    const auto runs = field_runs(G.curve_off, G.curve_n, G.prev_node);
    const FieldRun* d_runs = ws.upload("field_runs", runs);
    unsigned int* d_near = ws.get<unsigned int>("field_near", (size_t)n_target);
    FDS_HIP(hipMemsetAsync(d_near, 0, (size_t)n_target * sizeof(unsigned int), s));
    int* d_kind = nullptr;
    double* d_ang = nullptr;
    if (kind) {
      d_kind = ws.upload("field_kind", std::vector<int>(kind, kind + nrhs));
      d_ang = ws.upload("field_ang", std::vector<double>(angle, angle + nrhs));
    }
    launch_field_incident(targets, n_target, m, nrhs, d_kind, d_ang, (c64*)out, ld_out, s);
    // targets per chunk: E^T (2 nu x 2 mc complex) and the product's slab
    // partials (slabs x 2 mc x nrhs) within FDS_FIELD_CHUNK_MB (default 2048)
    // MiB, a multiple of 32 targets (one 64-row GEMM tile), at least 32
    const char* env_chunk = std::getenv("FDS_FIELD_CHUNK_MB");
    const int64_t chunk_mb = env_chunk ? std::max<int64_t>(1, std::atoll(env_chunk)) : (int64_t)2048;
    const int slabs = zgemm_tn_slabs((int)nu);
    const int64_t per_target = (2 * nu + (slabs > 1 ? (int64_t)slabs * 2 * nrhs : 0)) * (int64_t)sizeof(c64);
    int64_t mc = std::max<int64_t>(32, ((chunk_mb << 20) / per_target) / 32 * 32);
    mc = std::min<int64_t>({mc, n_target, (int64_t)4 * 65535});
    c64* Et = ws.get<c64>("field_E", (size_t)(nu * 2 * mc));
    c64* Pz = slabs > 1 ? ws.get<c64>("field_P", (size_t)slabs * 2 * mc * nrhs) : nullptr;
    for (int64_t m0 = 0; m0 < n_target; m0 += mc) {
      const int cur = (int)std::min(mc, n_target - m0);
      launch_field_matrix(DG.elems.p, d_runs, (int)runs.size(), targets, m0, cur, m, Et, nu, d_near, s);
      // out = u^I - E X on the matrix cores (E^T is nu x 2 cur)
      launch_zgemm_tn(2 * cur, nrhs, (int)nu, cmk(-1.0, 0.0), Et, nu, (const c64*)x, ld_x, cmk(1.0, 0.0),
                      (c64*)out + 2 * m0, ld_out, Pz, s);
    }
    if (n_near) {
      std::vector<unsigned int> fl((size_t)n_target);
      FDS_HIP(hipMemcpyAsync(fl.data(), d_near, fl.size() * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
      FDS_HIP(hipStreamSynchronize(s));
      int64_t c = 0;
      for (unsigned int v : fl) c += v != 0;
      *n_near = c;
    }
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    if (stream) (void)hipStreamSynchronize((hipStream_t)stream);
    return translate(e);
  }
}

int fds_special_eval(int64_t n, const double* x, double beta, double* out, fds_c64* outc, void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (n < 1 || !x || !out || !outc || !(beta > 0)) return FDS_EINVAL;
  try {
    launch_special_eval(x, n, beta, out, (c64*)outc, (hipStream_t)stream);
    FDS_HIP(hipStreamSynchronize((hipStream_t)stream));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_get_rank_log(fds_factor f, fds_rank_record* out, int64_t cap, int64_t* n_out) {
  if (!f || !n_out || cap < 0 || (cap > 0 && !out)) return FDS_EINVAL;
  const int64_t n = (int64_t)f->rank_log.size();
  for (int64_t i = 0; i < std::min(n, cap); ++i) out[i] = f->rank_log[i];
  *n_out = n;
  return FDS_OK;
}

int fds_lu_batched(int32_t np, fds_c64* a, const int64_t* off, const int64_t* n, int32_t* piv,
                   const int64_t* pivoff, int32_t* info, void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (np < 1 || !a || !off || !n || !piv || !pivoff || !info) return FDS_EINVAL;
  try {
    std::vector<LUDesc> d(np);
    for (int i = 0; i < np; ++i) {
      if (n[i] < 1 || n[i] > INT32_MAX / 2) return FDS_EINVAL;
      d[i] = LUDesc{off[i], pivoff[i], (int)n[i], (int)n[i]};
    }
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    int* dinfo = ws.get<int>("info", (size_t)np);
    lu_factor(d, (c64*)a, piv, dinfo, ws, "lu", s);
    FDS_HIP(hipMemcpyAsync(info, dinfo, np * sizeof(int), hipMemcpyDeviceToHost, s));
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_rid_batched(int32_t np, const fds_c64* a, const int64_t* off, const int64_t* m, const int64_t* n,
                    const int64_t* sz, const int64_t* gid, uint64_t seed, double tol, int32_t* piv,
                    const int64_t* pivoff, int32_t* rank, int32_t* revealed, double* ratio, void* stream) {
  AllocScope scope((hipStream_t)stream);
  // ``tol`` is the sketch's stopping tolerance (sketch_tol in the header)
  if (np < 1 || !a || !off || !m || !n || !sz || !gid || !piv || !pivoff || !rank || !revealed || !ratio ||
      !(tol > 0.0 && tol < 1.0))
    return FDS_EINVAL;
  try {
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    const c64* M = (const c64*)a;
    // sketches: the LDS kernel for s <= 64 and n <= 128, Omega + GEMM beyond
    std::vector<SketchDesc> sd;
    std::vector<OmegaDesc> od;
    std::vector<GemmDesc> gd;
    std::vector<CpqrDesc> yd(np);
    std::vector<char> big(np);
    int64_t ytot = 0, otot = 0, omax = 0, ptot = 0;
    int gnmax = 0;
    for (int i = 0; i < np; ++i) {
      if (m[i] < 1 || n[i] < 1 || n[i] > 4096 || sz[i] < 1 || sz[i] > m[i]) return FDS_EINVAL;
      big[i] = sz[i] > kSketchMaxS || n[i] > kSketchMaxN;
      if (!big[i]) {
        sd.push_back(SketchDesc{off[i], ytot, gid[i], (int)m[i], (int)n[i], (int)m[i], (int)sz[i]});
      } else {
        od.push_back(OmegaDesc{otot, gid[i], (int)sz[i], (int)m[i]});
        GemmDesc g{};
        g.a_off = otot;
        g.b_off = off[i];
        g.c_off = ytot;
        g.m = (int)sz[i];
        g.n = (int)n[i];
        g.k = (int)m[i];
        g.lda = (int)sz[i];
        g.ldb = (int)m[i];
        g.ldc = (int)sz[i];
        g.alpha_re = 1.0;
        gd.push_back(g);
        gnmax = std::max(gnmax, (int)n[i]);
        omax = std::max<int64_t>(omax, sz[i] * m[i]);
        otot += sz[i] * m[i];
      }
      yd[i] = CpqrDesc{ytot, pivoff[i], (int)sz[i], (int)n[i], (int)sz[i], 0, (int)std::min(sz[i], n[i]), 1};
      ytot += sz[i] * n[i];
      ptot = std::max(ptot, pivoff[i] + n[i]);
    }
    c64* Y = ws.get<c64>("Y", (size_t)ytot);
    int* dpiv = ws.get<int>("piv", (size_t)ptot);
    int* drank = ws.get<int>("rank", (size_t)np);
    launch_sketch(ws.upload("sd", sd), (int)sd.size(), M, Y, seed, s);
    if (!od.empty()) {
      c64* O = ws.get<c64>("O", (size_t)otot);
      launch_omega(ws.upload("od", od), (int)od.size(), omax, O, seed, s);
      const auto t = gemm_tiles(gd);
      launch_gemm(ws.upload("gd", gd), ws.upload("gt", t), (int)t.size(), gnmax, 0, (const c64*)O, M, Y, 0, s);
    }
    cpqr_factor(yd, Y, dpiv, tol, drank, ws, "qr", s);
    const std::vector<int> hr = download(ws, drank, (size_t)np);
    // judge: W from the sketch, then the LDS kernel or gather + GEMM + norms
    std::vector<InterpDesc> iw;
    std::vector<JudgeDesc> jd;
    std::vector<int> jd_i, rd_i;
    std::vector<ColGatherDesc> ec, gc;
    std::vector<GemmDesc> rg;
    std::vector<RatioDesc> rd;
    int64_t wtot = 0, etot = 0, gtot = 0;
    int ecmax = 0, gcmax = 0, rnmax = 0;
    for (int i = 0; i < np; ++i) {
      const int k = hr[i];
      if (k > 0) iw.push_back(InterpDesc{yd[i].a_off, pivoff[i], (int)n[i], (int)sz[i], k, wtot, k, 0, 0});
      if (!big[i]) {
        jd.push_back(JudgeDesc{off[i], wtot, pivoff[i], (int)m[i], (int)n[i], (int)m[i], k});
        jd_i.push_back(i);
      } else {
        ec.push_back(ColGatherDesc{off[i], etot, -1, (int)m[i], (int)n[i], (int)m[i], (int)m[i]});
        ecmax = std::max(ecmax, (int)n[i]);
        if (k > 0) {
          gc.push_back(ColGatherDesc{off[i], gtot, pivoff[i], (int)m[i], k, (int)m[i], (int)m[i]});
          gcmax = std::max(gcmax, k);
          GemmDesc g{};
          g.a_off = gtot;
          g.b_off = wtot;
          g.c_off = etot;
          g.m = (int)m[i];
          g.n = (int)n[i];
          g.k = k;
          g.lda = (int)m[i];
          g.ldb = k;
          g.ldc = (int)m[i];
          g.alpha_re = -1.0;
          g.beta_re = 1.0;
          rg.push_back(g);
          rnmax = std::max(rnmax, (int)n[i]);
        }
        rd.push_back(RatioDesc{etot, off[i], (int)m[i], (int)n[i], (int)m[i], (int)m[i]});
        rd_i.push_back(i);
        etot += m[i] * n[i];
        gtot += m[i] * k;
      }
      wtot += (int64_t)k * n[i];
    }
    c64* W = ws.get<c64>("W", (size_t)std::max<int64_t>(wtot, 1));
    double* dratio = ws.get<double>("ratio", (size_t)np);
    launch_interp(ws.upload("iw", iw), (int)iw.size(), Y, dpiv, W, s, interp_size(iw));
    launch_judge(ws.upload("jd", jd), (int)jd.size(), M, W, dpiv, dratio, s);
    if (!rd.empty()) {
      c64* E = ws.get<c64>("E", (size_t)etot);
      c64* G = ws.get<c64>("G", (size_t)std::max<int64_t>(gtot, 1));
      launch_gather_cols(ws.upload("ec", ec), (int)ec.size(), ecmax, M, dpiv, E, s);
      launch_gather_cols(ws.upload("gc", gc), (int)gc.size(), gcmax, M, dpiv, G, s);
      const auto t = gemm_tiles(rg);
      launch_gemm(ws.upload("rg", rg), ws.upload("rt", t), (int)t.size(), rnmax, 0, (const c64*)G, (const c64*)W,
                  E, 0, s);
      launch_ratio(ws.upload("rd", rd), (int)rd.size(), E, M, dratio + jd.size(), s);
    }
    const std::vector<double> hratio = download(ws, dratio, (size_t)np);
    FDS_HIP(hipMemcpyAsync(piv, dpiv, ptot * sizeof(int), hipMemcpyDeviceToHost, s));
    FDS_HIP(hipStreamSynchronize(s));
    for (size_t t = 0; t < jd_i.size(); ++t) ratio[jd_i[t]] = hratio[t];
    for (size_t t = 0; t < rd_i.size(); ++t) ratio[rd_i[t]] = hratio[jd_i.size() + t];
    for (int i = 0; i < np; ++i) {
      rank[i] = hr[i];
      revealed[i] = (hr[i] + kRevealMargin <= sz[i] || sz[i] >= n[i]) ? 1 : 0;
    }
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_mlp_init(float* blob, int64_t n, const float* x, const float* y, uint64_t seed, void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (!blob || n < 1 || !x || !y) return FDS_EINVAL;
  try {
    hipStream_t s = (hipStream_t)stream;
    std::vector<float> hx((size_t)n * kMlpIn), hy((size_t)n);
    FDS_HIP(hipMemcpyAsync(hx.data(), x, hx.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    FDS_HIP(hipMemcpyAsync(hy.data(), y, hy.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    FDS_HIP(hipStreamSynchronize(s));
    double mu[kMlpIn] = {}, sd[kMlpIn] = {}, ymax = 1.0;
    for (int64_t k = 0; k < n; ++k)
      for (int c = 0; c < kMlpIn; ++c) mu[c] += hx[k * kMlpIn + c];
    for (int c = 0; c < kMlpIn; ++c) mu[c] /= (double)n;
    for (int64_t k = 0; k < n; ++k) {
      for (int c = 0; c < kMlpIn; ++c) {
        const double d = hx[k * kMlpIn + c] - mu[c];
        sd[c] += d * d;
      }
      ymax = std::max(ymax, (double)hy[k]);
    }
    for (int c = 0; c < kMlpIn; ++c) {
      sd[c] = std::sqrt(sd[c] / (double)n);
      if (sd[c] == 0.0) sd[c] = 1.0;
    }
    // He-uniform weights lim (2 u - 1), u from SplitMix64 output p; zero biases
    const int layout[8][3] = {{0, kMlpH * kMlpIn, kMlpIn}, {kMlpH * kMlpIn, kMlpH, 0},
                              {kMlpH * kMlpIn + kMlpH, kMlpH * kMlpH, kMlpH},
                              {kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH, kMlpH, 0},
                              {kMlpH * kMlpIn + 2 * kMlpH + kMlpH * kMlpH, kMlpH * kMlpH, kMlpH},
                              {kMlpH * kMlpIn + 2 * kMlpH + 2 * kMlpH * kMlpH, kMlpH, 0},
                              {kMlpH * kMlpIn + 3 * kMlpH + 2 * kMlpH * kMlpH, kMlpH, kMlpH},
                              {kMlpH * kMlpIn + 4 * kMlpH + 2 * kMlpH * kMlpH, 1, 0}};
    for (auto& L : layout) {
      const double lim = L[2] ? std::sqrt(6.0 / L[2]) : 0.0;
      for (int p = L[0]; p < L[0] + L[1]; ++p) {
        const double u = (double)(splitmix64(seed, (uint64_t)p) >> 11) * 0x1.0p-53;
        blob[p] = L[2] ? (float)(lim * (2.0 * u - 1.0)) : 0.0f;
      }
    }
    for (int c = 0; c < kMlpIn; ++c) {
      blob[kMlpParams + c] = (float)mu[c];
      blob[kMlpParams + kMlpIn + c] = (float)sd[c];
    }
    blob[kMlpParams + 2 * kMlpIn] = (float)ymax;
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_mlp_forward(const float* blob, int64_t n, const float* x, float* y, int32_t bf16, void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (!blob || n < 1 || !x || !y) return FDS_EINVAL;
  try {
    hipStream_t s = (hipStream_t)stream;
    DevBuf<float> b(std::vector<float>(blob, blob + kMlpBlob));
    launch_mlp_forward(n, x, b.p, y, bf16 ? 1 : 0, s);
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_mlp_loss_grad(const float* blob, int64_t n, const float* x, const float* y, float* grad, float* loss,
                      void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (!blob || n < 1 || !x || !y || !grad || !loss) return FDS_EINVAL;
  try {
    hipStream_t s = (hipStream_t)stream;
    DevBuf<float> b(std::vector<float>(blob, blob + kMlpBlob));
    MlpWork w;
    w.n_waves = mlp_grad_waves();
    DevBuf<float> part((size_t)w.n_waves * (kMlpParams + 1)), g(kMlpParams), l(1);
    w.partial = part.p;
    launch_mlp_grad(n, n, x, y, b.p, 0, -1, w, g.p, l.p, s);
    FDS_HIP(hipMemcpyAsync(grad, g.p, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, s));
    FDS_HIP(hipMemcpyAsync(loss, l.p, sizeof(float), hipMemcpyDeviceToHost, s));
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_mlp_train(float* blob, int64_t n, const float* x, const float* y, int32_t steps, int64_t batch, float lr,
                  uint64_t seed, float* loss_hist, void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (!blob || n < 1 || !x || !y || steps < 0 || batch < 0 || !(lr > 0.0f)) return FDS_EINVAL;
  try {
    hipStream_t s = (hipStream_t)stream;
    DevBuf<float> b(std::vector<float>(blob, blob + kMlpBlob));
    MlpWork w;
    w.n_waves = mlp_grad_waves();
    DevBuf<float> part((size_t)w.n_waves * (kMlpParams + 1)), g(kMlpParams), l((size_t)std::max(steps, 1));
    DevBuf<float> m(std::vector<float>(kMlpParams, 0.0f)), v(std::vector<float>(kMlpParams, 0.0f));
    w.partial = part.p;
    for (int t = 1; t <= steps; ++t) {
      if (batch == 0)
        launch_mlp_grad(n, n, x, y, b.p, seed, -1, w, g.p, l.p + (t - 1), s);
      else
        launch_mlp_grad(n, batch, x, y, b.p, seed, t, w, g.p, l.p + (t - 1), s);
      launch_adam(g.p, b.p, m.p, v.p, t, lr, s);
    }
    FDS_HIP(hipMemcpyAsync(blob, b.p, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, s));
    if (loss_hist && steps > 0)
      FDS_HIP(hipMemcpyAsync(loss_hist, l.p, steps * sizeof(float), hipMemcpyDeviceToHost, s));
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_cpqr_batched(int32_t np, fds_c64* a, const int64_t* off, const int64_t* m, const int64_t* n, int32_t* piv,
                     const int64_t* pivoff, const int64_t* kmax, double tol, int32_t stop_at_tol, int32_t* rank,
                     void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (np < 1 || !a || !off || !m || !n || !piv || !pivoff || !kmax || !rank) return FDS_EINVAL;
  try {
    std::vector<CpqrDesc> d(np);
    for (int i = 0; i < np; ++i) {
      if (m[i] < 1 || n[i] < 1) return FDS_EINVAL;
      d[i] = CpqrDesc{off[i], pivoff[i], (int)m[i], (int)n[i], (int)m[i], 0, (int)kmax[i], stop_at_tol};
    }
    check_cpqr_sizes(d);
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    cpqr_factor(d, (c64*)a, piv, tol, rank, ws, "cpqr", s);
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

int fds_interp_batched(int32_t np, fds_c64* a, const int64_t* off, const int64_t* m, const int64_t* n,
                       const int32_t* piv, const int64_t* pivoff, const int32_t* rank, fds_c64* w,
                       const int64_t* woff, void* stream) {
  AllocScope scope((hipStream_t)stream);
  if (np < 1 || !a || !off || !m || !n || !piv || !pivoff || !rank || !w || !woff) return FDS_EINVAL;
  try {
    std::vector<InterpDesc> d;
    for (int i = 0; i < np; ++i) {
      if (m[i] < 1 || n[i] < 1 || rank[i] < 0 || rank[i] > std::min(m[i], n[i])) return FDS_EINVAL;
      if (rank[i] > 0)
        d.push_back(InterpDesc{off[i], pivoff[i], (int)n[i], (int)m[i], rank[i], woff[i], rank[i], 0, 0});
    }
    if (d.empty()) return FDS_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace ws(s);
    launch_interp(ws.upload("interp", d), (int)d.size(), (c64*)a, piv, (c64*)w, s, interp_size(d));
    FDS_HIP(hipStreamSynchronize(s));
    return FDS_OK;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return translate(e);
  }
}

}  // extern "C"
