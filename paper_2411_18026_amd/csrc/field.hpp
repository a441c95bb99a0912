// Field off the boundary by the integral representation (field.hip).
#pragma once

#include <vector>

#include "common.hpp"

namespace fds {

// A run of at most 63 consecutive nodes of one curve: nodes first ..
// first + count - 1, and the element that ends at ``first`` (elements are
// numbered by their first node).
struct FieldRun {
  int first, count, prev_elem, pad;
};

constexpr int kFieldRunNodes = 63;
constexpr int kFieldMaxPanels = 64;   // panels of an element near a target

std::vector<FieldRun> field_runs(const std::vector<int>& curve_off, const std::vector<int>& curve_n,
                                 const std::vector<int>& prev_node);

// Gauss tables of the field kernel (uploaded once per process from the
// assembly's host tables).
void ensure_field_quad();

// Et (2 N x 2 mc, leading dimension ld >= 2 N): column 2 m + i, row 2 t + j
// holds the integral over the two elements of node t of K_ij(x, y) times the
// hat of node t, for targets x = targets[m0 + m], m < mc.  near[m0 + m] is
// set to 1 when some element is closer to the target than 1/64 of its
// length (left untouched otherwise).
void launch_field_matrix(const Elem* elems, const FieldRun* runs, int n_runs, const double* targets, int64_t m0,
                         int mc, const MatConst& m, c64* Et, int64_t ld, unsigned int* near, hipStream_t s);

// out[r * ld + 2 m + i] = u^I_i(targets[m]) of plane wave r (kind 0: P,
// 1: S; direction angle ang[r]), or 0 for every r when kind == nullptr.
void launch_field_incident(const double* targets, int64_t n_target, const MatConst& m, int nrhs, const int* kind,
                           const double* ang, c64* out, int64_t ld, hipStream_t s);

}  // namespace fds
