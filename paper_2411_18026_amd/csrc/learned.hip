// Learned rank pre-sizing: sketches for the randomized ID, the residual
// judge, and the rank-predictor MLP (forward, backward, Adam) on gfx950.
//
// The MLP maps one sample to one wavefront: lane j is neuron j of every
// 64-wide hidden layer, activations move between lanes by shuffles, and
// the weights sit in LDS with rows padded to 65 floats so that both the
// row reads of the forward pass and the column reads of the backward pass
// are free of bank conflicts.
#include "learned.hpp"

namespace fds {

constexpr int kLB = 256;

__device__ inline double wsum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline float wsum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ------------------------------------------------------------------ sketch
// Y = Omega M, Omega(i, l) = (+-1) + i (+-1) from SplitMix64 output
// (gid << 44) | (i << 24) | l: bit 0 the sign of the real part, bit 1 that of
// the imaginary part.  One workgroup per problem; M is streamed in chunks of
// 16 rows through LDS; wave w owns sketch rows w, w + 4, ..., lane l the
// columns l and l + 64.
__global__ void __launch_bounds__(kLB) k_sketch(const SketchDesc* __restrict__ descs, const c64* __restrict__ mbase,
                                                c64* __restrict__ ybase, uint64_t seed) {
  constexpr int LC = 16;
  __shared__ unsigned char om[kSketchMaxS][LC];
  __shared__ c64 mc[LC][kSketchMaxN];
  const SketchDesc d = descs[blockIdx.x];
  const c64* M = mbase + d.m_off;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  c64 acc[kSketchMaxS / 4][2];
#pragma unroll
  for (int a = 0; a < kSketchMaxS / 4; ++a) acc[a][0] = acc[a][1] = cmk(0.0, 0.0);
  for (int l0 = 0; l0 < d.m; l0 += LC) {
    for (int e = t; e < d.s * LC; e += kLB) {
      const int i = e / LC, ll = e % LC, l = l0 + ll;
      unsigned char code = 0;
      if (l < d.m) code = (unsigned char)(splitmix64(seed, ((uint64_t)d.gid << 44) | ((uint64_t)i << 24) | (uint64_t)l) & 3u);
      om[i][ll] = code;
    }
    for (int e = t; e < LC * d.n; e += kLB) {
      const int ll = e % LC, j = e / LC, l = l0 + ll;
      mc[ll][j] = l < d.m ? M[l + (int64_t)j * d.lda] : cmk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < kSketchMaxS / 4; ++a) {
      const int i = w + 4 * a;
      if (i < d.s) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int j = lane + 64 * b;
          if (j < d.n) {
            c64 s = acc[a][b];
            for (int ll = 0; ll < LC; ++ll) {
              const unsigned c = om[i][ll];
              const c64 v = mc[ll][j];
              const double sr = (c & 1u) ? -1.0 : 1.0, si = (c & 2u) ? -1.0 : 1.0;
              s.re += sr * v.re - si * v.im;
              s.im += sr * v.im + si * v.re;
            }
            acc[a][b] = s;
          }
        }
      }
    }
    __syncthreads();
  }
  c64* Y = ybase + d.y_off;
#pragma unroll
  for (int a = 0; a < kSketchMaxS / 4; ++a) {
    const int i = w + 4 * a;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = lane + 64 * b;
      if (i < d.s && j < d.n) Y[i + (int64_t)j * d.s] = acc[a][b];
    }
  }
}

// ------------------------------------------------------------------ judge
// ratio = max_j |M(:,j) - M(:,J) W(:,j)| / max_j |M(:,j)| (0 for M = 0).
// One workgroup per problem; rows in tiles of 64 (lane = row), wave w owns
// columns w, w + 4, ...; the pivot columns and W are staged in chunks of 16.
__global__ void __launch_bounds__(kLB) k_judge(const JudgeDesc* __restrict__ descs, const c64* __restrict__ mbase,
                                               const c64* __restrict__ wbase, const int* __restrict__ piv,
                                               double* __restrict__ ratio) {
  constexpr int KC = 16;
  constexpr int NQ = kSketchMaxN / 4;
  __shared__ c64 mj[64][KC + 1];
  __shared__ c64 wc[KC][kSketchMaxN];
  __shared__ double cn_e[kSketchMaxN], cn_m[kSketchMaxN];
  __shared__ int J[kSketchMaxN];
  const JudgeDesc d = descs[blockIdx.x];
  const c64* M = mbase + d.m_off;
  const c64* W = wbase + d.w_off;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int l = t; l < d.k; l += kLB) J[l] = piv[d.piv_off + l];
  for (int j = t; j < kSketchMaxN; j += kLB) cn_e[j] = cn_m[j] = 0.0;
  __syncthreads();
  for (int rt = 0; rt < d.m; rt += 64) {
    const int i = rt + lane;
    const bool valid = i < d.m;
    c64 e[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = w + 4 * q;
      e[q] = (valid && j < d.n) ? M[i + (int64_t)j * d.lda] : cmk(0.0, 0.0);
      const double s = wsum_d(abs2(e[q]));
      if (lane == 0 && j < d.n) cn_m[j] += s;
    }
    for (int l0 = 0; l0 < d.k; l0 += KC) {
      const int kc = min(KC, d.k - l0);
      for (int x = t; x < 64 * KC; x += kLB) {
        const int r = x % 64, ll = x / 64;
        mj[r][ll] = (rt + r < d.m && ll < kc) ? M[(rt + r) + (int64_t)J[l0 + ll] * d.lda] : cmk(0.0, 0.0);
      }
      for (int x = t; x < KC * d.n; x += kLB) {
        const int ll = x % KC, j = x / KC;
        wc[ll][j] = ll < kc ? W[(l0 + ll) + (int64_t)j * d.k] : cmk(0.0, 0.0);
      }
      __syncthreads();
      for (int ll = 0; ll < KC; ++ll) {
        const c64 a = mj[lane][ll];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int j = w + 4 * q;
          if (j < d.n) e[q] -= a * wc[ll][j];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = w + 4 * q;
      const double s = wsum_d(valid ? abs2(e[q]) : 0.0);
      if (lane == 0 && j < d.n) cn_e[j] += s;
    }
  }
  __syncthreads();
  if (t == 0) {
    double me = 0.0, mm = 0.0;
    for (int j = 0; j < d.n; ++j) {
      me = fmax(me, cn_e[j]);
      mm = fmax(mm, cn_m[j]);
    }
    ratio[blockIdx.x] = mm > 0.0 ? sqrt(me / mm) : 0.0;
  }
}

// ------------------------------------------------------------------ large sketches
__global__ void k_omega(const OmegaDesc* __restrict__ descs, c64* __restrict__ obase, uint64_t seed) {
  const OmegaDesc d = descs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)d.s * d.m) return;
  const int i = (int)(e % d.s), l = (int)(e / d.s);
  const uint64_t z = splitmix64(seed, ((uint64_t)d.gid << 44) | ((uint64_t)i << 24) | (uint64_t)l);
  obase[d.o_off + e] = cmk((z & 1u) ? -1.0 : 1.0, (z & 2u) ? -1.0 : 1.0);
}

__global__ void k_gather_cols(const ColGatherDesc* __restrict__ descs, const c64* __restrict__ src,
                              const int* __restrict__ idx, c64* __restrict__ dst) {
  const ColGatherDesc d = descs[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= d.ncol) return;
  const int sc = d.idx_off >= 0 ? idx[d.idx_off + c] : c;
  const c64* from = src + d.src_off + (int64_t)sc * d.lds;
  c64* to = dst + d.dst_off + (int64_t)c * d.ldd;
  for (int i = threadIdx.x; i < d.m; i += blockDim.x) to[i] = from[i];
}

__global__ void __launch_bounds__(kLB) k_ratio(const RatioDesc* __restrict__ descs, const c64* __restrict__ ebase,
                                               const c64* __restrict__ mbase, double* __restrict__ ratio) {
  __shared__ double se[kLB / 64], sm[kLB / 64];
  const RatioDesc d = descs[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double me = 0.0, mm = 0.0;
  for (int c = w; c < d.n; c += kLB / 64) {
    const c64* e = ebase + d.e_off + (int64_t)c * d.lde;
    const c64* m = mbase + d.m_off + (int64_t)c * d.ldm;
    double a = 0.0, b = 0.0;
    for (int i = lane; i < d.m; i += 64) {
      a += abs2(e[i]);
      b += abs2(m[i]);
    }
    a = wsum_d(a);
    b = wsum_d(b);
    me = fmax(me, a);
    mm = fmax(mm, b);
  }
  if (lane == 0) {
    se[w] = me;
    sm[w] = mm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kLB / 64; ++k) {
      me = fmax(se[0], se[k]);
      se[0] = me;
      mm = fmax(sm[0], sm[k]);
      sm[0] = mm;
    }
    ratio[blockIdx.x] = sm[0] > 0.0 ? sqrt(se[0] / sm[0]) : 0.0;
  }
}

// ------------------------------------------------------------------ MLP
constexpr int oW1 = 0, ob1 = oW1 + kMlpH * kMlpIn, oW2 = ob1 + kMlpH, ob2 = oW2 + kMlpH * kMlpH,
              oW3 = ob2 + kMlpH, ob3 = oW3 + kMlpH * kMlpH, ow4 = ob3 + kMlpH, ob4 = ow4 + kMlpH,
              omu = ob4 + 1, osig = omu + kMlpIn, oys = osig + kMlpIn;
static_assert(omu == kMlpParams, "parameter layout");
static_assert(oys + 1 == kMlpBlob, "blob layout");
constexpr int kPad = kMlpH + 1;

struct MlpLds {
  float W1[kMlpH][kMlpIn], b1[kMlpH];
  float W2[kMlpH][kPad], b2[kMlpH];
  float W3[kMlpH][kPad], b3[kMlpH];
  float w4[kMlpH], b4, mu[kMlpIn], sig[kMlpIn], ys;
};

// round to the nearest bfloat16 (ties to even), kept in a float
__device__ inline float bf16r(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ void mlp_load(MlpLds& L, const float* __restrict__ blob, bool bf16) {
  for (int p = threadIdx.x; p < kMlpBlob; p += blockDim.x) {
    float v = blob[p];
    const bool weight = p < omu;
    if (bf16 && weight) v = bf16r(v);
    if (p < ob1) L.W1[(p - oW1) / kMlpIn][(p - oW1) % kMlpIn] = v;
    else if (p < oW2) L.b1[p - ob1] = v;
    else if (p < ob2) L.W2[(p - oW2) / kMlpH][(p - oW2) % kMlpH] = v;
    else if (p < oW3) L.b2[p - ob2] = v;
    else if (p < ob3) L.W3[(p - oW3) / kMlpH][(p - oW3) % kMlpH] = v;
    else if (p < ow4) L.b3[p - ob3] = v;
    else if (p < ob4) L.w4[p - ow4] = v;
    else if (p == ob4) L.b4 = v;
    else if (p < osig) L.mu[p - omu] = v;
    else if (p < oys) L.sig[p - osig] = v;
    else L.ys = v;
  }
  __syncthreads();
}

struct MlpAct {
  float xn[kMlpIn];
  float z1, h1, z2, h2, z3, h3, out;
};

// forward pass of one sample on one wavefront (lane j = neuron j)
__device__ inline MlpAct mlp_fwd(const MlpLds& L, const float* __restrict__ x, bool bf16) {
  const int j = threadIdx.x & 63;
  MlpAct a;
#pragma unroll
  for (int c = 0; c < kMlpIn; ++c) {
    const float v = (x[c] - L.mu[c]) / L.sig[c];
    a.xn[c] = bf16 ? bf16r(v) : v;
  }
  float z = L.b1[j];
#pragma unroll
  for (int c = 0; c < kMlpIn; ++c) z += L.W1[j][c] * a.xn[c];
  a.z1 = z;
  a.h1 = fmaxf(z, 0.0f);
  if (bf16) a.h1 = bf16r(a.h1);
  z = L.b2[j];
  for (int i = 0; i < kMlpH; ++i) z += L.W2[j][i] * __shfl(a.h1, i);
  a.z2 = z;
  a.h2 = fmaxf(z, 0.0f);
  if (bf16) a.h2 = bf16r(a.h2);
  z = L.b3[j];
  for (int i = 0; i < kMlpH; ++i) z += L.W3[j][i] * __shfl(a.h2, i);
  a.z3 = z;
  a.h3 = fmaxf(z, 0.0f);
  if (bf16) a.h3 = bf16r(a.h3);
  a.out = wsum_f(L.w4[j] * a.h3) + L.b4;
  return a;
}

// predictions y_scale * out, one wavefront per sample; with abstain > 0 a
// sample with a standardised input beyond +-abstain gets NaN (no prediction)
__global__ void __launch_bounds__(kLB) k_mlp_forward(int64_t n, const float* __restrict__ x,
                                                     const float* __restrict__ blob, float* __restrict__ out,
                                                     int bf16, float abstain) {
  __shared__ MlpLds L;
  mlp_load(L, blob, bf16 != 0);
  const int64_t nw = (int64_t)gridDim.x * (kLB / 64);
  for (int64_t smp = (int64_t)blockIdx.x * (kLB / 64) + (threadIdx.x >> 6); smp < n; smp += nw) {
    const MlpAct a = mlp_fwd(L, x + smp * kMlpIn, bf16 != 0);
    bool far = false;
    if (abstain > 0.0f)
      for (int c = 0; c < kMlpIn; ++c) far = far || fabsf((x[smp * kMlpIn + c] - L.mu[c]) / L.sig[c]) > abstain;
    if ((threadIdx.x & 63) == 0) out[smp] = far ? __int_as_float(0x7fc00000) : L.ys * a.out;
  }
}

// Per-wave partial gradients of sum_b (out_b - y_b / y_scale)^2 / batch.
__global__ void __launch_bounds__(kLB) k_mlp_grad(int64_t n, int64_t batch, const float* __restrict__ x,
                                                  const float* __restrict__ y, const float* __restrict__ blob,
                                                  uint64_t seed, int64_t step, float* __restrict__ partial) {
  __shared__ MlpLds L;
  mlp_load(L, blob, false);
  const int j = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (kLB / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (kLB / 64);
  float g1[kMlpIn], g2[kMlpH], g3[kMlpH];
#pragma unroll
  for (int c = 0; c < kMlpIn; ++c) g1[c] = 0.0f;
#pragma unroll
  for (int i = 0; i < kMlpH; ++i) g2[i] = g3[i] = 0.0f;
  float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f, gw4 = 0.0f, gb4 = 0.0f, lsum = 0.0f;
  const float inv_b = 1.0f / (float)batch;
  for (int64_t b = gw; b < batch; b += nw) {
    const int64_t idx = step < 0 ? b : (int64_t)(splitmix64(seed, ((uint64_t)step << 32) | (uint64_t)b) % (uint64_t)n);
    const MlpAct a = mlp_fwd(L, x + idx * kMlpIn, false);
    const float r = a.out - y[idx] / L.ys;
    lsum += r * r;
    const float go = 2.0f * r * inv_b;
    gw4 += go * a.h3;
    gb4 += go;
    const float d3 = a.z3 > 0.0f ? go * L.w4[j] : 0.0f;
    gb3 += d3;
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) g3[i] += d3 * __shfl(a.h2, i);
    float s = 0.0f;
    for (int k = 0; k < kMlpH; ++k) s += L.W3[k][j] * __shfl(d3, k);
    const float d2 = a.z2 > 0.0f ? s : 0.0f;
    gb2 += d2;
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) g2[i] += d2 * __shfl(a.h1, i);
    s = 0.0f;
    for (int k = 0; k < kMlpH; ++k) s += L.W2[k][j] * __shfl(d2, k);
    const float d1 = a.z1 > 0.0f ? s : 0.0f;
    gb1 += d1;
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) g1[c] += d1 * a.xn[c];
  }
  float* P = partial + gw * (kMlpParams + 1);
#pragma unroll
  for (int c = 0; c < kMlpIn; ++c) P[oW1 + j * kMlpIn + c] = g1[c];
  P[ob1 + j] = gb1;
#pragma unroll
  for (int i = 0; i < kMlpH; ++i) {
    P[oW2 + j * kMlpH + i] = g2[i];
    P[oW3 + j * kMlpH + i] = g3[i];
  }
  P[ob2 + j] = gb2;
  P[ob3 + j] = gb3;
  P[ow4 + j] = gw4;
  if (j == 0) {
    P[ob4] = gb4;
    P[kMlpParams] = lsum;
  }
}

// grad[p] = sum over waves in wave order; loss = sum r^2 / batch
__global__ void k_mlp_reduce(const float* __restrict__ partial, int n_waves, int64_t batch, float* __restrict__ grad,
                             float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  float s = 0.0f;
  for (int w = 0; w < n_waves; ++w) s += partial[(int64_t)w * (kMlpParams + 1) + p];
  if (p < kMlpParams)
    grad[p] = s;
  else
    loss[0] = s / (float)batch;
}

// Adam (Kingma and Ba) on the trainable parameters; t is the 1-based step
__global__ void k_adam(const float* __restrict__ grad, float* __restrict__ blob, float* __restrict__ m,
                       float* __restrict__ v, int t, float lr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.0f - b1) * g;
  const float vv = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / (1.0f - powf(b1, (float)t));
  const float vh = vv / (1.0f - powf(b2, (float)t));
  blob[p] -= lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------------------ launchers
void launch_sketch(const SketchDesc* d, int n, const c64* mbase, c64* ybase, uint64_t seed, hipStream_t s) {
  if (n == 0) return;
  k_sketch<<<n, kLB, 0, s>>>(d, mbase, ybase, seed);
  FDS_HIP(hipGetLastError());
}

void launch_judge(const JudgeDesc* d, int n, const c64* mbase, const c64* wbase, const int* piv, double* ratio,
                  hipStream_t s) {
  if (n == 0) return;
  k_judge<<<n, kLB, 0, s>>>(d, mbase, wbase, piv, ratio);
  FDS_HIP(hipGetLastError());
}

void launch_omega(const OmegaDesc* d, int n, int64_t max_elems, c64* obase, uint64_t seed, hipStream_t s) {
  if (n == 0 || max_elems == 0) return;
  k_omega<<<dim3((unsigned)((max_elems + 255) / 256), (unsigned)n), 256, 0, s>>>(d, obase, seed);
  FDS_HIP(hipGetLastError());
}

void launch_gather_cols(const ColGatherDesc* d, int n, int max_cols, const c64* src, const int* idx, c64* dst,
                        hipStream_t s) {
  if (n == 0 || max_cols == 0) return;
  k_gather_cols<<<dim3((unsigned)max_cols, (unsigned)n), 256, 0, s>>>(d, src, idx, dst);
  FDS_HIP(hipGetLastError());
}

void launch_ratio(const RatioDesc* d, int n, const c64* ebase, const c64* mbase, double* ratio, hipStream_t s) {
  if (n == 0) return;
  k_ratio<<<n, kLB, 0, s>>>(d, ebase, mbase, ratio);
  FDS_HIP(hipGetLastError());
}

void launch_mlp_forward(int64_t n, const float* x, const float* blob, float* out, int bf16, hipStream_t s,
                        float abstain) {
  if (n == 0) return;
  const int64_t blocks = std::min<int64_t>((n + 3) / 4, 1024);
  k_mlp_forward<<<(unsigned)blocks, kLB, 0, s>>>(n, x, blob, out, bf16, abstain);
  FDS_HIP(hipGetLastError());
}

int mlp_grad_waves() { return 256; }

void launch_mlp_grad(int64_t n, int64_t batch, const float* x, const float* y, const float* blob, uint64_t seed,
                     int64_t step, const MlpWork& w, float* grad, float* loss, hipStream_t s) {
  if (batch <= 0) throw Error(1, "mlp: empty batch");
  k_mlp_grad<<<w.n_waves / 4, kLB, 0, s>>>(n, batch, x, y, blob, seed, step, w.partial);
  FDS_HIP(hipGetLastError());
  k_mlp_reduce<<<(kMlpParams + 1 + 255) / 256, 256, 0, s>>>(w.partial, w.n_waves, batch, grad, loss);
  FDS_HIP(hipGetLastError());
}

void launch_adam(const float* grad, float* blob, float* m, float* v, int t, float lr, hipStream_t s) {
  k_adam<<<(kMlpParams + 255) / 256, 256, 0, s>>>(grad, blob, m, v, t, lr);
  FDS_HIP(hipGetLastError());
}

}  // namespace fds
