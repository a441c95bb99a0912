// Learned rank pre-sizing (randomized ID with a residual judge) and the
// rank-predictor MLP (6-64-64-64-1, ReLU): device kernels and launchers.
#pragma once

#include <vector>

#include "common.hpp"

namespace fds {

constexpr int kMlpIn = 6, kMlpH = 64;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + 2 * (kMlpH * kMlpH + kMlpH) + kMlpH + 1;   // 8833
constexpr int kMlpBlob = kMlpParams + 2 * kMlpIn + 1;                                          // + mu, sigma, y_scale
constexpr int kSketchMaxS = 64;    // sketch rows
constexpr int kSketchMaxN = 128;   // columns of a sketched problem
// The sketch's rank is taken at this fraction of the ID tolerance: its column
// norms are a random projection of the matrix's (distorted by up to ~2x at
// these sizes), and the judge then checks the tolerance on the matrix itself.
constexpr double kSketchTolFactor = 0.1;
// A sketch reveals a rank only with this many rows to spare (randomized
// range estimates need a few rows beyond the rank to be reliable).
constexpr int kRevealMargin = 4;
// The predictor abstains (the cell goes to the pivoted QR) when a
// standardised input lies further than this from the training mean.
constexpr float kAbstainSigma = 4.0f;

// SplitMix64 output number c for seed ``seed`` (Steele, Lea and Flood:
// golden-ratio increment, 64-bit finaliser).
__host__ __device__ inline uint64_t splitmix64(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct SketchDesc {     // Y (s x n, ld s) = Omega_gid (s x m) M (m x n, ld lda)
  int64_t m_off, y_off, gid;
  int m, n, lda, s;
};

struct JudgeDesc {      // ratio = max_j |M(:,j) - M(:,J) W(:,j)| / max_j |M(:,j)|, W k x n (ld k)
  int64_t m_off, w_off, piv_off;
  int m, n, lda, k;
};

void launch_sketch(const SketchDesc* d, int n, const c64* mbase, c64* ybase, uint64_t seed, hipStream_t s);

// Large problems (s > 64 rows or n > 128 columns): Omega drawn into a buffer
// (s x m, ld s, same entries as the sketch kernel), Y = Omega M by GEMM;
// the judge from E = M - M(:, J) W formed by GEMM.
struct OmegaDesc {
  int64_t o_off, gid;
  int s, m;
};
struct ColGatherDesc {   // dst(:, c) = src(:, idx[c]) (idx_off < 0: c), c < ncol, m rows
  int64_t src_off, dst_off, idx_off;
  int m, ncol, lds, ldd;
};
struct RatioDesc {       // max_j |E(:,j)| / max_j |M(:,j)| over n columns
  int64_t e_off, m_off;
  int m, n, lde, ldm;
};
void launch_omega(const OmegaDesc* d, int n, int64_t max_elems, c64* obase, uint64_t seed, hipStream_t s);
void launch_gather_cols(const ColGatherDesc* d, int n, int max_cols, const c64* src, const int* idx, c64* dst,
                        hipStream_t s);
void launch_ratio(const RatioDesc* d, int n, const c64* ebase, const c64* mbase, double* ratio, hipStream_t s);
void launch_judge(const JudgeDesc* d, int n, const c64* mbase, const c64* wbase, const int* piv, double* ratio,
                  hipStream_t s);

// MLP.  blob: device floats in the layout W1 (64 x 6), b1, W2 (64 x 64), b2,
// W3 (64 x 64), b3, w4 (64), b4, mu (6), sigma (6), y_scale.  x: n x 6
// row-major features.
// abstain > 0: NaN for samples with a standardised input beyond +-abstain
void launch_mlp_forward(int64_t n, const float* x, const float* blob, float* out, int bf16, hipStream_t s,
                        float abstain = 0.0f);
// Gradient of the mean squared error over a batch: samples are x rows
// 0..batch-1 when seed_step < 0, else rows drawn by SplitMix64(seed) at
// counters (step << 32) | slot reduced mod n.  Writes grad[kMlpParams] and
// loss[0] (deterministic: fixed reduction order).
struct MlpWork {
  float* partial = nullptr;   // n_waves x (kMlpParams + 1)
  int n_waves = 0;
};
int mlp_grad_waves();
void launch_mlp_grad(int64_t n, int64_t batch, const float* x, const float* y, const float* blob, uint64_t seed,
                     int64_t step, const MlpWork& w, float* grad, float* loss, hipStream_t s);
void launch_adam(const float* grad, float* blob, float* m, float* v, int t, float lr, hipStream_t s);

}  // namespace fds
