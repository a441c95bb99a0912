// Device special functions for the elastodynamic Galerkin kernels.
//
// The fundamental solution of 2D elastodynamics (equation of the
// fundamental solution, Section 3) needs the Hankel functions H0, H1 of
// the first kind at the transverse and longitudinal wavenumbers, i.e. the
// Bessel functions J0, J1, Y0, Y1 of real positive argument, and the two
// combinations
//     E   = (a H1(a) - b H1(b)) / a^2,      chi = H2(a) - beta^2 H2(b),
// with a = k_T r, b = k_L r = beta a, which carry exactly cancelling 1/a^2
// singular parts.
//
// Algorithms (all from the classical expansions of Bessel functions):
//   x < 2       ascending power series of J0, J1, Y0, Y1;
//   2 <= x < 17 Miller's backward recurrence J_{n-1} = (2n/x) J_n - J_{n+1}
//               from n = N >= 2x + 20, normalised by J0 + 2 sum J_{2k} = 1,
//               with Neumann series for the second kind:
//                 Y0 = (2/pi)(log(x/2) + gamma) J0 - (4/pi) sum_k (-1)^k J_{2k}/k,
//                 Y1 = -(2/(pi x)) J0 + (2/pi)(log(x/2) + gamma) J1
//                      + (2/pi) sum_k (-1)^k (J_{2k-1} - J_{2k+1})/k;
//   x >= 17     Hankel's asymptotic expansion H_nu = sqrt(2/(pi x)) (P + iQ)
//               exp(i(x - nu pi/2 - pi/4)).
//   E, chi for a < 1 from the ascending series of H1, H2 with the singular
//   parts cancelled analytically; otherwise from the Hankel values.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace fds {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kEulerGamma = 0.57721566490153286060651209008240243;
constexpr double kSeriesSwitch = 1.0;   // a below which E, chi use the series

struct c64 {
  double re, im;
};

__host__ __device__ inline c64 cmk(double r, double i) { return c64{r, i}; }
__host__ __device__ inline c64 operator+(c64 a, c64 b) { return c64{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline c64 operator-(c64 a, c64 b) { return c64{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline c64 operator-(c64 a) { return c64{-a.re, -a.im}; }
__host__ __device__ inline c64 operator*(c64 a, c64 b) {
  return c64{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline c64 operator*(double s, c64 a) { return c64{s * a.re, s * a.im}; }
__host__ __device__ inline c64 operator*(c64 a, double s) { return c64{s * a.re, s * a.im}; }
__host__ __device__ inline c64& operator+=(c64& a, c64 b) {
  a.re += b.re;
  a.im += b.im;
  return a;
}
__host__ __device__ inline c64& operator-=(c64& a, c64 b) {
  a.re -= b.re;
  a.im -= b.im;
  return a;
}
__host__ __device__ inline c64 conj(c64 a) { return c64{a.re, -a.im}; }
__host__ __device__ inline double abs2(c64 a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ inline c64 mul_i(c64 a) { return c64{-a.im, a.re}; }   // i a
// a * b / c computed as complex division
__host__ __device__ inline c64 cdiv(c64 a, c64 b) {
  double d = b.re * b.re + b.im * b.im;
  return c64{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// complex FP32 (mixed-precision merges and sweeps)
struct c32 {
  float re, im;
};
__host__ __device__ inline c32 operator+(c32 a, c32 b) { return c32{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline c32 operator-(c32 a, c32 b) { return c32{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline c32 operator*(c32 a, c32 b) {
  return c32{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline c32& operator+=(c32& a, c32 b) {
  a.re += b.re;
  a.im += b.im;
  return a;
}
__host__ __device__ inline c32& operator-=(c32& a, c32 b) {
  a.re -= b.re;
  a.im -= b.im;
  return a;
}
__host__ __device__ inline float abs2(c32 a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ inline c32 cdiv(c32 a, c32 b) {
  const float d = b.re * b.re + b.im * b.im;
  return c32{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// scalar-type helpers for kernels templated on c64 / c32
template <typename T>
struct Cx;
template <>
struct Cx<c64> {
  using real = double;
  __host__ __device__ static c64 make(double r, double i) { return c64{r, i}; }
};
template <>
struct Cx<c32> {
  using real = float;
  __host__ __device__ static c32 make(double r, double i) { return c32{(float)r, (float)i}; }
};

// Natural logarithm of a positive, finite, normal double from the series
// log((1 + s)/(1 - s)) = 2 (s + s^3/3 + s^5/5 + ...): x = 2^e m with m in
// [sqrt(1/2), sqrt(2)), s = (m - 1)/(m + 1), |s| < 0.172, twelve odd terms
// (the first neglected one is below 1e-18 of the sum), then log x =
// e log 2 + log m in one fused multiply-add.  Within about 2 ulp; about a
// third of the instructions of the library logarithm, which also handles
// zero, negative, subnormal and non-finite arguments (none occur here).
__host__ __device__ inline double log_pos(double x) {
  int e;
  double m = frexp(x, &e);   // m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = 2.0 / 23.0;
  p = p * s2 + 2.0 / 21.0;
  p = p * s2 + 2.0 / 19.0;
  p = p * s2 + 2.0 / 17.0;
  p = p * s2 + 2.0 / 15.0;
  p = p * s2 + 2.0 / 13.0;
  p = p * s2 + 2.0 / 11.0;
  p = p * s2 + 2.0 / 9.0;
  p = p * s2 + 2.0 / 7.0;
  p = p * s2 + 2.0 / 5.0;
  p = p * s2 + 2.0 / 3.0;
  p = p * s2 + 2.0;
  return fma((double)e, 0.69314718055994530942, s * p);
}

// Miller's backward recurrence for J_n(x) started at an even index N
// (N >= 2x + 20), normalised by 1 = J_0 + 2 sum_k J_2k, with the Neumann
// series of Y0 and Y1 accumulated on the way down.  N is a compile-time
// constant: the loop unrolls, every coefficient folds to a constant and all
// lanes of a wavefront run the same instructions.
template <int N>
__host__ __device__ inline void bessel_miller(double x, double& J0, double& J1, double& Y0, double& Y1) {
  const double tx = 2.0 / x;
  double cur = 1e-30, nxt = 0.0;   // J_m (unnormalised), J_{m+1}
  double s = 0.0, y0s = 0.0, y1s = 0.0, v0 = 0.0, v1 = 0.0;
#pragma unroll
  for (int m = N; m >= 0; --m) {
    const double v = cur;
    if (m & 1) {
      // odd m contributes to sum_k (-1)^k (J_{2k-1} - J_{2k+1}) / k
      const int kp = (m + 1) >> 1;   // m = 2 kp - 1
      double c = ((kp & 1) ? -1.0 : 1.0) / kp;
      if (m >= 3) {
        const int km = (m - 1) >> 1;   // m = 2 km + 1
        c -= ((km & 1) ? -1.0 : 1.0) / km;
      }
      y1s += c * v;
      if (m == 1) v1 = v;
    } else if (m > 0) {
      const int k = m >> 1;
      s += 2.0 * v;
      y0s += (((k & 1) ? -1.0 : 1.0) / k) * v;
    } else {
      s += v;
      v0 = v;
    }
    const double prev = (m * tx) * cur - nxt;
    nxt = cur;
    cur = prev;
  }
  const double inv = 1.0 / s;
  const double L = log_pos(0.5 * x) + kEulerGamma;
  J0 = v0 * inv;
  J1 = v1 * inv;
  Y0 = (2.0 / kPi) * L * J0 - (4.0 / kPi) * y0s * inv;
  Y1 = -(2.0 / (kPi * x)) * J0 + (2.0 / kPi) * L * J1 + (2.0 / kPi) * y1s * inv;
}

// J0, J1, Y0, Y1 of x > 0.
__host__ __device__ inline void bessel_jy01(double x, double& J0, double& J1, double& Y0, double& Y1) {
  if (x < 2.0) {
    const double w = 0.25 * x * x;
    double t0 = 1.0, t1 = 0.5 * x, h = 0.0;
    double j0 = 0.0, j1 = 0.0, y0s = 0.0, y1s = 0.0;
#pragma unroll
    for (int k = 0; k < 14; ++k) {
      j0 += t0;
      j1 += t1;
      y0s -= t0 * h;                                  // (-1)^{k+1} h_k w^k/(k!)^2
      y1s += (2.0 * h + 1.0 / (k + 1)) * t1;          // (psi(k+1)+psi(k+2)+2 gamma) t1_k
      t0 *= -w * (1.0 / ((k + 1.0) * (k + 1.0)));
      t1 *= -w * (1.0 / ((k + 1.0) * (k + 2.0)));
      h += 1.0 / (k + 1);
    }
    const double L = log_pos(0.5 * x);
    J0 = j0;
    J1 = j1;
    Y0 = (2.0 / kPi) * ((L + kEulerGamma) * j0 + y0s);
    Y1 = -2.0 / (kPi * x) + (2.0 / kPi) * L * j1 - (y1s - 2.0 * kEulerGamma * j1) / kPi;
    return;
  }
  if (x < 8.0) {
    bessel_miller<36>(x, J0, J1, Y0, Y1);
    return;
  }
  if (x < 17.0) {
    bessel_miller<54>(x, J0, J1, Y0, Y1);
    return;
  }
  // Hankel asymptotic expansion
  double P0 = 0.0, Q0 = 0.0, P1 = 0.0, Q1 = 0.0;
  {
    double a0 = 1.0, a1 = 1.0;
    const double inv8x = 1.0 / (8.0 * x);
    for (int k = 0; k < 40; ++k) {
      if (k > 0) {
        const double o = (2.0 * k - 1.0) * (2.0 * k - 1.0);
        a0 *= (0.0 - o) * inv8x / k;
        a1 *= (4.0 - o) * inv8x / k;
      }
      const double sg = ((k >> 1) & 1) ? -1.0 : 1.0;
      if ((k & 1) == 0) {
        P0 += sg * a0;
        P1 += sg * a1;
      } else {
        Q0 += sg * a0;
        Q1 += sg * a1;
      }
      if (fabs(a0) < 1e-17 && fabs(a1) < 1e-17) break;
    }
  }
  double sx, cx;
  sincos(x, &sx, &cx);
  const double r2 = 0.70710678118654752440084436210484903;
  const double c0 = (cx + sx) * r2, s0 = (sx - cx) * r2;     // cos, sin of x - pi/4
  const double c1 = (sx - cx) * r2, s1 = -(sx + cx) * r2;    // cos, sin of x - 3 pi/4
  const double f = sqrt(2.0 / (kPi * x));
  J0 = f * (P0 * c0 - Q0 * s0);
  Y0 = f * (P0 * s0 + Q0 * c0);
  J1 = f * (P1 * c1 - Q1 * s1);
  Y1 = f * (P1 * s1 + Q1 * c1);
}

// psi(m) - (-gamma) = harmonic number h_{m-1}
__host__ __device__ inline double harmonic(int m) {
  double h = 0.0;
  for (int j = 1; j <= m; ++j) h += 1.0 / j;
  return h;
}

// E = (a H1(a) - b H1(b))/a^2 and chi = H2(a) - beta^2 H2(b), b = beta a, by the
// ascending series (valid for all a, used for a < kSeriesSwitch).
__host__ __device__ inline void e_chi_series(double a, double beta, c64& E, c64& chi) {
  const double w = 0.25 * a * a;
  const double la = log(0.5 * a);
  const double lb = log(beta);
  const double b2 = beta * beta;
  const double twoipi = 2.0 / kPi;
  E = cmk(0.0, 0.0);
  chi = cmk(0.0, -(1.0 - b2) / kPi);
  double wk = 1.0;          // w^k
  double fk = 1.0;          // k!
  double fk1 = 1.0;         // (k+1)!
  double fk2 = 2.0;         // (k+2)!
  double bp2 = b2;          // beta^(2k+2)
  double bp4 = b2 * b2;     // beta^(2k+4)
  double hk = 0.0;          // h_k
  for (int k = 0; k < 14; ++k) {
    const double hk1 = hk + 1.0 / (k + 1);    // h_{k+1}
    const double hk2 = hk1 + 1.0 / (k + 2);   // h_{k+2}
    // psi(k+1) + psi(k+2) = -2 gamma + h_k + h_{k+1}
    const double sE = -2.0 * kEulerGamma + hk + hk1;
    const double sC = -2.0 * kEulerGamma + hk + hk2;   // psi(k+1) + psi(k+3)
    // c_k(a) = 1 + i (2/pi) log(a/2) - i (1/pi) sE
    const double ck_im = twoipi * la - sE / kPi;
    const double dk_im = twoipi * la - sC / kPi;
    const double sgn = (k & 1) ? -1.0 : 1.0;
    {
      // ((1 - beta^(2k+2)) c_k - beta^(2k+2) (2i/pi) log beta) / (2 k! (k+1)!)
      const double re = (1.0 - bp2);
      const double im = (1.0 - bp2) * ck_im - bp2 * twoipi * lb;
      const double sc = sgn * wk / (2.0 * fk * fk1);
      E.re += sc * re;
      E.im += sc * im;
    }
    {
      const double re = (1.0 - bp4);
      const double im = (1.0 - bp4) * dk_im - bp4 * twoipi * lb;
      const double sc = sgn * wk * w / (fk * fk2);
      chi.re += sc * re;
      chi.im += sc * im;
    }
    wk *= w;
    fk *= (k + 1);
    fk1 *= (k + 2);
    fk2 *= (k + 3);
    bp2 *= b2;
    bp4 *= b2;
    hk = hk1;
  }
}

// Small-argument expansions as polynomials in w = a^2/4 (a = k_T r < 1,
// b = beta a, w_b = beta^2 w).  The coefficient rows do not depend on the
// material and are compile-time constants (they fold into the code, so no
// table occupies registers):
//   S0 (-1)^k/(k!)^2                 S1 (-1)^(k+1) h_k/(k!)^2
//   S2 (-1)^k/(k!(k+1)!)             S3 (-1)^k (psi(k+1)+psi(k+2))/(k!(k+1)!)
//   S6 (-1)^k/(k!(k+2)!)             S7 (-1)^k (psi(k+1)+psi(k+3))/(k!(k+2)!)
// With L = log(a/2), Pi = Si(w), Qi = Si(w_b):
//   J0 = P0, Y0 = (2/pi)((L + gamma) J0 + P1),
//   J1 = (a/2) P2, Y1 = -2/(pi a) + (2/pi) L J1 - (1/pi)(a/2) P3,
//   H0(b) from Q0, Q1 with log(b/2) = L + log beta,
//   E   = e + i ((2/pi) L e + e'),     e  = (P2 - beta^2 Q2)/2,
//         e' = -(P3 - beta^2 Q3)/(2 pi) - (log beta/pi) beta^2 Q2,
//   chi = -(i/pi)(1 - beta^2) + w (c + i ((2/pi) L c + c')),
//         c  = P6 - beta^4 Q6,   c' = -(P7 - beta^4 Q7)/pi - (2 log beta/pi) beta^4 Q6
// (the 1/a^2 parts of E and chi cancel term by term in these forms).
constexpr int kSerTerms = 10;
struct SerTab {
  double c[6][kSerTerms];
};

constexpr SerTab make_ser_tab() {
  SerTab t{};
  double fk = 1.0, fk1 = 1.0, fk2 = 2.0, hk = 0.0;   // k!, (k+1)!, (k+2)!, h_k
  for (int k = 0; k < kSerTerms; ++k) {
    const double sg = (k & 1) ? -1.0 : 1.0;
    const double hk1 = hk + 1.0 / (k + 1), hk2 = hk1 + 1.0 / (k + 2);
    const double psiE = -2.0 * kEulerGamma + hk + hk1;   // psi(k+1) + psi(k+2)
    const double psiC = -2.0 * kEulerGamma + hk + hk2;   // psi(k+1) + psi(k+3)
    t.c[0][k] = sg / (fk * fk);
    t.c[1][k] = -sg * hk / (fk * fk);
    t.c[2][k] = sg / (fk * fk1);
    t.c[3][k] = sg * psiE / (fk * fk1);
    t.c[4][k] = sg / (fk * fk2);
    t.c[5][k] = sg * psiC / (fk * fk2);
    fk *= (k + 1);
    fk1 *= (k + 2);
    fk2 *= (k + 3);
    hk = hk1;
  }
  return t;
}

constexpr SerTab kSerTab = make_ser_tab();

// material constants of the series (host-built once per material)
struct SeriesCoef {
  double beta, logbeta, b2, b4;   // b2 = beta^2, b4 = beta^4
  double chi0;                    // -(1 - beta^2)/pi (imaginary part of chi's constant)
};

inline SeriesCoef make_series_coef(double beta) {
  SeriesCoef s{};
  s.beta = beta;
  s.logbeta = log(beta);
  s.b2 = beta * beta;
  s.b4 = s.b2 * s.b2;
  s.chi0 = -(1.0 - s.b2) / kPi;
  return s;
}

// row R of the table summed to K terms (K <= kSerTerms)
template <int K, int R>
__host__ __device__ inline double ser(double w) {
  double p = kSerTab.c[R][K - 1];
#pragma unroll
  for (int k = K - 2; k >= 0; --k) p = p * w + kSerTab.c[R][k];
  return p;
}

// Hankel values needed at one point: H0(a), H1(a), H0(b), H1(b).
struct Hankel2 {
  c64 h0a, h1a, h0b, h1b;
};

__host__ __device__ inline Hankel2 hankel_pair(double a, double b) {
  Hankel2 h;
  double j0, j1, y0, y1;
  bessel_jy01(a, j0, j1, y0, y1);
  h.h0a = cmk(j0, y0);
  h.h1a = cmk(j1, y1);
  bessel_jy01(b, j0, j1, y0, y1);
  h.h0b = cmk(j0, y0);
  h.h1b = cmk(j1, y1);
  return h;
}

__host__ __device__ inline void e_chi(double a, double beta, const Hankel2& h, c64& E, c64& chi) {
  if (a < kSeriesSwitch) {
    e_chi_series(a, beta, E, chi);
    return;
  }
  const double b = beta * a;
  const double ia2 = 1.0 / (a * a);
  E = ia2 * (a * h.h1a - b * h.h1b);
  const c64 h2a = (2.0 / a) * h.h1a - h.h0a;
  const c64 h2b = (2.0 / b) * h.h1b - h.h0b;
  chi = h2a - (beta * beta) * h2b;
}

// Small-argument form of the kernel ingredients with K terms of each series
// (ia = 1/a, which the caller has from its own reciprocal square root).
template <int K>
__host__ __device__ inline void series_values(double a, double ia, double w, const SeriesCoef& sc, c64& h0a,
                                              c64& h1a, c64& h0b, c64& E, c64& chi) {
  const double wb = sc.b2 * w;
  const double L = log_pos(0.5 * a);
  const double tp = 2.0 / kPi;
  const double P0 = ser<K, 0>(w), P1 = ser<K, 1>(w), P2 = ser<K, 2>(w), P3 = ser<K, 3>(w), P6 = ser<K, 4>(w), P7 = ser<K, 5>(w);
  const double Q0 = ser<K, 0>(wb), Q1 = ser<K, 1>(wb), Q2 = ser<K, 2>(wb), Q3 = ser<K, 3>(wb), Q6 = ser<K, 4>(wb),
               Q7 = ser<K, 5>(wb);
  const double j1 = 0.5 * a * P2;
  h0a = cmk(P0, tp * ((L + kEulerGamma) * P0 + P1));
  h1a = cmk(j1, -tp * ia + tp * L * j1 - (a * (0.5 / kPi)) * P3);
  h0b = cmk(Q0, tp * ((L + sc.logbeta + kEulerGamma) * Q0 + Q1));
  const double e = 0.5 * (P2 - sc.b2 * Q2);
  const double e1 = -(0.5 / kPi) * (P3 - sc.b2 * Q3) - (sc.logbeta / kPi) * sc.b2 * Q2;
  E = cmk(e, tp * L * e + e1);
  const double c = P6 - sc.b4 * Q6;
  const double c1 = -(1.0 / kPi) * (P7 - sc.b4 * Q7) - (2.0 * sc.logbeta / kPi) * sc.b4 * Q6;
  chi = cmk(w * c, sc.chi0 + w * (tp * L * c + c1));
}

// All kernel ingredients at one point: H0(a), H1(a), H0(b), E, chi.  Below
// kSeriesSwitch the series are summed to as many terms as the point's
// w = a^2/4 needs (the neglected tail stays below 4e-19 for every row: 4
// terms for w < 1e-4, 6 for w < 5e-3, 8 for w < 5e-2, else 10).  The choice
// depends on the point alone, so a result does not depend on which other
// points share its wavefront.
__host__ __device__ inline void kernel_values_series(double a, double ia, const SeriesCoef& sc, c64& h0a, c64& h1a,
                                                     c64& h0b, c64& E, c64& chi) {
  const double w = 0.25 * a * a;
  if (w >= 5e-2)
    series_values<10>(a, ia, w, sc, h0a, h1a, h0b, E, chi);
  else if (w >= 5e-3)
    series_values<8>(a, ia, w, sc, h0a, h1a, h0b, E, chi);
  else if (w >= 1e-4)
    series_values<6>(a, ia, w, sc, h0a, h1a, h0b, E, chi);
  else
    series_values<4>(a, ia, w, sc, h0a, h1a, h0b, E, chi);
}

__host__ __device__ inline void kernel_values(double a, double ia, const SeriesCoef& sc, c64& h0a, c64& h1a, c64& h0b,
                                              c64& E, c64& chi) {
  if (a < kSeriesSwitch) {
    kernel_values_series(a, ia, sc, h0a, h1a, h0b, E, chi);
    return;
  }
  const Hankel2 h = hankel_pair(a, sc.beta * a);
  h0a = h.h0a;
  h1a = h.h1a;
  h0b = h.h0b;
  e_chi(a, sc.beta, h, E, chi);
}
__host__ __device__ inline void kernel_values(double a, const SeriesCoef& sc, c64& h0a, c64& h1a, c64& h0b, c64& E,
                                              c64& chi) {
  kernel_values(a, 1.0 / a, sc, h0a, h1a, h0b, E, chi);
}

}  // namespace fds
