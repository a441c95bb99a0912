// Host side of the Galerkin assembly: quadrature tables and batching of
// dense block requests into classify / pair / gather launches.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "assembly.hpp"
#include "devmem.hpp"
#include "parallel.hpp"

namespace fds {

// n-point Gauss-Legendre rule on [0, 1] (Newton iteration on P_n).
static void gauss_legendre01(int n, double* x01, double* w01) {
  std::vector<double> xs(n), ws(n);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
    }
    xs[i] = x;
    ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  // ascending order on [0, 1]
  for (int i = 0; i < n; ++i) {
    x01[i] = 0.5 * (1.0 + xs[n - 1 - i]);
    w01[i] = 0.5 * ws[n - 1 - i];
  }
}

// coincident rule: d = s^P on each triangle of the square, 2-point Gauss
// along the diagonal; Q offsets, 4 Q points
static void coincident_rule(int Q, int P, double* cu, double* cv, double* cw, double* coff) {
  std::vector<double> s(Q), ws(Q);
  double g2[2], w2[2];
  gauss_legendre01(Q, s.data(), ws.data());
  gauss_legendre01(2, g2, w2);
  int p = 0;
  for (int i = 0; i < Q; ++i) {
    const double d = std::pow(s[i], P);
    const double wd = ws[i] * P * std::pow(s[i], P - 1);
    const double ell = 1.0 - d;
    for (int k = 0; k < 2; ++k) {
      const double t = ell * g2[k];
      const double w = wd * ell * w2[k];
      cu[p] = t + d;
      cv[p] = t;
      cw[p] = w;
      coff[p] = d;
      ++p;
      cu[p] = t;
      cv[p] = t + d;
      cw[p] = w;
      coff[p] = -d;
      ++p;
    }
  }
}

// adjacent rule: Duffy map of both triangles about the shared vertex,
// xi = s^P, Q x Q points per triangle
static void adjacent_rule(int Q, int P, double* au, double* av, double* aw) {
  std::vector<double> s(Q), ws(Q), eta(Q), we(Q);
  gauss_legendre01(Q, s.data(), ws.data());
  gauss_legendre01(Q, eta.data(), we.data());
  const int half = Q * Q;
  for (int i = 0; i < Q; ++i) {
    const double xi = std::pow(s[i], P);
    const double wxi = ws[i] * P * std::pow(s[i], P - 1);
    for (int j = 0; j < Q; ++j) {
      const int p = i * Q + j;
      const double w = wxi * we[j] * xi;
      au[p] = xi;
      av[p] = xi * eta[j];
      aw[p] = w;
      au[half + p] = xi * eta[j];
      av[half + p] = xi;
      aw[half + p] = w;
    }
  }
}

QuadTables make_quad_tables() {
  QuadTables q{};
  gauss_legendre01(2, q.g2, q.w2);
  gauss_legendre01(3, q.g3, q.w3);
  gauss_legendre01(4, q.g4, q.w4);
  gauss_legendre01(6, q.g6, q.w6);
  gauss_legendre01(10, q.g10, q.w10);
  gauss_legendre01(6, q.rg, q.rw);
  coincident_rule(kQCoinc, kPCoinc, q.cu, q.cv, q.cw, q.coff);
  adjacent_rule(kQAdj, kPAdj, q.au, q.av, q.aw);
  coincident_rule(kQCoincHi, kPCoinc, q.chu, q.chv, q.chw, q.choff);
  adjacent_rule(kQAdjHi, kPAdj, q.ahu, q.ahv, q.ahw);
  return q;
}

// quadrature points per pair and reported class of each list
static int points_of_class(int c) {
  if (c == kQ10) return 100;
  if (c == kCoinc) return kNCoincPts;
  if (c == kAdjNext || c == kAdjPrev) return kNAdjPts;
  const int r = (c - kRegBase) / 2;
  return order_of(r / kNumOrd) * order_of(r % kNumOrd);
}
static int public_class_of(int c) {
  if (c < kRegBase) return 2 + c;
  return ((c - kRegBase) / 2) / kNumOrd == kNumOrd - 1 ? 1 : 0;
}
// the launch (in launch_pairs' order) that integrates a list
static int launch_of_class(int c) {
  if (c < kRegBase) return 8 + c;
  const int r = c - kRegBase;
  return 2 * ((r / 2) / kNumOrd) + (r % 2);
}
constexpr int kBatchEvents = kNumPairLaunches + 3;   // start, kNumPairLaunches + 1 marks, end

// resolved events of the current device, kept for later batches
static std::mutex g_ev_mu;
static std::map<int, std::vector<hipEvent_t>> g_ev_spare;
static void give_back(const std::vector<hipEvent_t>& ev) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    for (auto e : ev) (void)hipEventDestroy(e);
    return;
  }
  std::lock_guard<std::mutex> lk(g_ev_mu);
  auto& v = g_ev_spare[dev];
  v.insert(v.end(), ev.begin(), ev.end());
}

void AssemblyStats::resolve(hipStream_t s) {
  if (pending.empty()) return;
  FDS_HIP(hipStreamSynchronize(s));
  std::vector<unsigned int> cnt(pending.size() * kNumClass);
  FDS_HIP(hipMemcpy(cnt.data(), d_counts, cnt.size() * sizeof(unsigned), hipMemcpyDeviceToHost));
  for (size_t b = 0; b < pending.size(); ++b) {
    auto& ev = pending[b];
    float ms = 0.f;
    FDS_HIP(hipEventElapsedTime(&ms, ev[0], ev[kBatchEvents - 1]));
    seconds += 1e-3 * ms;
    bool busy[kNumPublicClass] = {}, lbusy[kNumPairLaunches] = {};
    for (int c = 0; c < kNumClass; ++c) {
      const unsigned n = cnt[b * kNumClass + c];
      const int pc = public_class_of(c), li = launch_of_class(c);
      const int64_t e = (int64_t)n * points_of_class(c);
      evals += e;
      class_evals[pc] += e;
      kernel_evals[li] += e;
      busy[pc] = busy[pc] || n;
      lbusy[li] = lbusy[li] || n;
    }
    for (int li = 0; li < kNumPairLaunches; ++li) {
      float cm = 0.f;
      FDS_HIP(hipEventElapsedTime(&cm, ev[1 + li], ev[2 + li]));
      class_seconds[launch_public_class(li)] += 1e-3 * cm;
      kernel_seconds[li] += 1e-3 * cm;
      if (lbusy[li]) kernel_launches[li] += 1;
    }
    for (int pc = 0; pc < kNumPublicClass; ++pc)
      if (busy[pc]) class_launches[pc] += 1;
    give_back(ev);
  }
  pending.clear();
}

AssemblyStats::~AssemblyStats() {
  for (auto& ev : pending)
    for (auto e : ev) (void)hipEventDestroy(e);
}

hipEvent_t AssemblyStats::event() {
  int dev = 0;
  FDS_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    auto& v = g_ev_spare[dev];
    if (!v.empty()) {
      const hipEvent_t e = v.back();
      v.pop_back();
      return e;
    }
  }
  hipEvent_t e;
  FDS_HIP(hipEventCreate(&e));
  return e;
}

void assemble_blocks(const std::vector<BlockReq>& reqs, const Elem* d_elems, const MatConst& m, c64* d_out,
                     Workspace& ws, AssemblyStats* st, int64_t max_pairs) {
  hipStream_t s = ws.stream();
  size_t i0 = 0;
  while (i0 < reqs.size()) {
    // batch [i0, i1)
    size_t i1 = i0;
    int64_t np = 0;
    while (i1 < reqs.size()) {
      const int64_t p = (int64_t)reqs[i1].rows.elems.size() * (int64_t)reqs[i1].cols.elems.size();
      if (i1 > i0 && np + p > max_pairs) break;
      np += p;
      ++i1;
    }
    // pack the batch's tables: sizes and offsets first, then every request
    // filled in parallel (the layout is the one a serial append would give)
    const size_t nb = i1 - i0;
    const int ct = classify_tile_size();
    std::vector<Job> jobs(nb);
    std::vector<int64_t> e_off(nb + 1, 0), d_off(nb + 1, 0), p_off(nb + 1, 0), pt_off(nb + 1, 0),
        ot_off(nb + 1, 0);
    int64_t pair_off = 0;
    for (size_t k = 0; k < nb; ++k) {
      const BlockReq& q = reqs[i0 + k];
      Job& j = jobs[k];
      j.pair_off = pair_off;
      j.out_off = q.out_off;
      j.rs = q.rs;
      j.cs = q.cs;
      j.nre = (int)q.rows.elems.size();
      j.nce = (int)q.cols.elems.size();
      j.nrd = (int)q.rows.dofs.size();
      j.ncd = (int)q.cols.dofs.size();
      j.re_off = (int)e_off[k];
      j.ce_off = (int)(e_off[k] + j.nre);
      e_off[k + 1] = e_off[k] + j.nre + j.nce;
      j.rd_off = (int)d_off[k];
      j.cd_off = (int)(d_off[k] + j.nrd);
      d_off[k + 1] = d_off[k] + j.nrd + j.ncd;
      j.rpos_off = q.rpos.empty() ? -1 : (int)p_off[k];
      j.cpos_off = q.cpos.empty() ? -1 : (int)(p_off[k] + q.rpos.size());
      p_off[k + 1] = p_off[k] + (int64_t)q.rpos.size() + (int64_t)q.cpos.size();
      const int64_t npj = (int64_t)j.nre * j.nce, noj = (int64_t)j.nrd * j.ncd;
      pt_off[k + 1] = pt_off[k] + (npj + ct - 1) / ct;
      ot_off[k + 1] = ot_off[k] + (noj + 255) / 256;
      pair_off += npj;
    }
    // the batch's tables, packed straight into pinned host memory and sent
    // in one copy: jobs, element lists, positions, DOFs, pair tiles, entry tiles
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o_jobs = 0, o_elist = al(nb * sizeof(Job)), o_pos = o_elist + al((size_t)e_off[nb] * sizeof(int)),
                 o_dofs = o_pos + al((size_t)std::max<int64_t>(p_off[nb], 1) * sizeof(int)),
                 o_pt = o_dofs + al((size_t)d_off[nb] * sizeof(Dof)),
                 o_ot = o_pt + al((size_t)pt_off[nb] * sizeof(Tile)),
                 tot = o_ot + al((size_t)ot_off[nb] * sizeof(Tile));
    char* hb = static_cast<char*>(ws.pinned(tot));
    int* elist = reinterpret_cast<int*>(hb + o_elist);
    int* pos = reinterpret_cast<int*>(hb + o_pos);
    Dof* dofs = reinterpret_cast<Dof*>(hb + o_dofs);
    Tile* ptiles = reinterpret_cast<Tile*>(hb + o_pt);
    Tile* otiles = reinterpret_cast<Tile*>(hb + o_ot);
    std::copy(jobs.begin(), jobs.end(), reinterpret_cast<Job*>(hb + o_jobs));
    pos[0] = 0;
    parallel_for((int)nb, [&](int k) {
      const BlockReq& q = reqs[i0 + k];
      const Job& j = jobs[k];
      std::copy(q.rows.elems.begin(), q.rows.elems.end(), elist + j.re_off);
      std::copy(q.cols.elems.begin(), q.cols.elems.end(), elist + j.ce_off);
      std::copy(q.rows.dofs.begin(), q.rows.dofs.end(), dofs + j.rd_off);
      std::copy(q.cols.dofs.begin(), q.cols.dofs.end(), dofs + j.cd_off);
      std::copy(q.rpos.begin(), q.rpos.end(), pos + p_off[k]);
      std::copy(q.cpos.begin(), q.cpos.end(), pos + p_off[k] + q.rpos.size());
      const int64_t npj = (int64_t)j.nre * j.nce, noj = (int64_t)j.nrd * j.ncd;
      int64_t t = pt_off[k];
      for (int64_t a = 0; a < npj; a += ct) ptiles[t++] = Tile{(int)k, (int)std::min<int64_t>(ct, npj - a), a};
      t = ot_off[k];
      for (int64_t a = 0; a < noj; a += 256) otiles[t++] = Tile{(int)k, (int)std::min<int64_t>(256, noj - a), a};
    });
    char* db = ws.get<char>("asm_tables", tot);
    ws.pinned_upload(db, tot);
    Job* d_jobs = reinterpret_cast<Job*>(db + o_jobs);
    int* d_elist = reinterpret_cast<int*>(db + o_elist);
    int* d_pos = reinterpret_cast<int*>(db + o_pos);
    Dof* d_dofs = reinterpret_cast<Dof*>(db + o_dofs);
    Tile* d_pt = reinterpret_cast<Tile*>(db + o_pt);
    Tile* d_ot = reinterpret_cast<Tile*>(db + o_ot);
    const size_t n_ptiles = (size_t)pt_off[nb], n_otiles = (size_t)ot_off[nb];
    unsigned long long* d_lists = ws.get<unsigned long long>("asm_lists", (size_t)kNumClass * np);
    c64* d_res = ws.get<c64>("asm_res", (size_t)16 * np);
    unsigned int* d_cnt;
    std::vector<hipEvent_t> ev;
    if (st && (int)st->pending.size() < AssemblyStats::kMaxBatches) {
      if (!st->d_counts)
        st->d_counts = ws.get<unsigned int>("asm_counts", (size_t)AssemblyStats::kMaxBatches * kNumClass);
      d_cnt = st->d_counts + st->pending.size() * kNumClass;
      ev.resize(kBatchEvents);
      for (auto& e : ev) e = st->event();
    } else {
      d_cnt = ws.get<unsigned int>("asm_cnt_tmp", kNumClass);
    }
    FDS_HIP(hipMemsetAsync(d_cnt, 0, kNumClass * sizeof(unsigned), s));
    if (!ev.empty()) FDS_HIP(hipEventRecord(ev[0], s));
    launch_classify(d_pt, (int)n_ptiles, d_jobs, d_elist, d_elems, d_lists, np, d_cnt, m.kT, s);
    launch_pairs(d_lists, np, d_cnt, d_jobs, d_elist, d_elems, m, d_res, np, s, ev.empty() ? nullptr : ev.data() + 1);
    launch_gather(d_ot, (int)n_otiles, d_jobs, d_dofs, d_pos, d_res, np, d_out, s);
    if (!ev.empty()) {
      FDS_HIP(hipEventRecord(ev[kBatchEvents - 1], s));
      st->pending.push_back(ev);
    }
    i0 = i1;
  }
}

}  // namespace fds
