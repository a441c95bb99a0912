// Launchers of the Galerkin assembly kernels (assembly.hip) and the host
// side that batches dense blocks into jobs.
#pragma once

#include <vector>

#include "common.hpp"

namespace fds {

void upload_quad_tables(const QuadTables& q);
void launch_elem_geometry(const double* xy, const int* curve_of, const int* curve_off, const int* curve_n,
                          int n_elem, Elem* out, hipStream_t s);
// proxy polygons: cell c gets poff[c+1] - poff[c] vertices on the circle
// (crd[3c], crd[3c+1]) of radius crd[3c+2]; poff device, [n_cells + 1]
void launch_proxy_elems(const double* crd, const int* poff, int n_cells, int total, int poly_base, Elem* out,
                        hipStream_t s);
void launch_classify(const Tile* tiles, int n_tiles, const Job* jobs, const int* elist, const Elem* elems,
                     unsigned long long* lists, int64_t cap, unsigned int* counters, double kT, hipStream_t s);
void launch_pairs(const unsigned long long* lists, int64_t cap, const unsigned int* counts, const Job* jobs,
                  const int* elist, const Elem* elems, const MatConst& m, c64* res, int64_t np, hipStream_t s,
                  hipEvent_t* ev = nullptr);
int classify_tile_size();
void launch_gather(const Tile* tiles, int n_tiles, const Job* jobs, const Dof* dofs, const int* pos,
                   const c64* res, int64_t np, c64* out, hipStream_t s);
void launch_rhs_plane(const Elem* elems, const int* prev_elem, int n_nodes, const MatConst& m, double lam, int nrhs,
                      const int* kind, const double* ang, c64* out, int64_t ld, hipStream_t s);
void launch_special_eval(const double* x, int64_t n, double beta, double* out, c64* outc, hipStream_t s);

QuadTables make_quad_tables();

// One side of a block: an element list and the DOFs on it.
struct Side {
  std::vector<int> elems;   // global element ids
  std::vector<Dof> dofs;    // eL, eR index into ``elems``
};

// A dense block request: out[out_off + rpos[r] * rs + cpos[c] * cs] = A(r, c).
struct BlockReq {
  Side rows, cols;
  int64_t out_off = 0;
  int64_t rs = 1, cs = 0;
  std::vector<int> rpos, cpos;   // empty = identity
};

class Workspace;

// Pair-integration launches of a batch, in order: k_regular for test
// orders 2, 3, 4, 6 (each general, then series-only), the 10-point pairs,
// coincident, adjacent next, adjacent previous; and the reported class of
// each (fds_stats).
constexpr int kNumPairLaunches = 12;
constexpr int launch_public_class(int li) { return li < 6 ? 0 : (li < 8 ? 1 : li - 6); }

// Timing and work counts of the assembly launches.  Events and the device
// class counters of every batch are recorded without synchronising;
// ``resolve`` (after the stream has been synchronised) turns them into
// seconds and evaluation counts.
struct AssemblyStats {
  static constexpr int kMaxBatches = 8192;
  double seconds = 0.0;
  int64_t evals = 0;
  // per reported class (the series-only lists count with their order)
  double class_seconds[kNumPublicClass] = {0, 0, 0, 0, 0, 0};
  int64_t class_evals[kNumPublicClass] = {0, 0, 0, 0, 0, 0};
  int64_t class_launches[kNumPublicClass] = {0, 0, 0, 0, 0, 0};
  // per pair-integration kernel (launch order)
  double kernel_seconds[kNumPairLaunches] = {};
  int64_t kernel_evals[kNumPairLaunches] = {};
  int64_t kernel_launches[kNumPairLaunches] = {};
  unsigned int* d_counts = nullptr;       // kMaxBatches x kNumClass device counters
  std::vector<std::vector<hipEvent_t>> pending;   // per batch: start, kNumPairLaunches + 1 marks, end
  hipEvent_t event();   // from a per-device pool of resolved events (creating one is slow)
  void resolve(hipStream_t s);
  ~AssemblyStats();
};

// Batches block requests, runs classify / pair / gather kernels, writes the
// blocks into ``out`` (a device array).  Splits the work so that the pair
// scratch stays below ``max_pairs`` element pairs.  Asynchronous on the
// workspace stream.
void assemble_blocks(const std::vector<BlockReq>& reqs, const Elem* d_elems, const MatConst& m, c64* d_out,
                     Workspace& ws, AssemblyStats* st, int64_t max_pairs = 24000000);

}  // namespace fds
