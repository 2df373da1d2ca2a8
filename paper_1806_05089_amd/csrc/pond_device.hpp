// Device-side building blocks of the PonD step for gfx950: speed sets,
// third-order Lagrange interpolation weights and the per-axis transfer rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pond {

// A double constant split into the nearest FP32 value and the FP32 rounding
// of the remainder (hi + lo equals it to about 2^-48 relative).
__host__ __device__ constexpr float split_hi(double a) { return float(a); }
__host__ __device__ constexpr float split_lo(double a) { return float(a - double(float(a))); }

// ------------------------------------------------------------ speed sets
// D2Q16: per-axis speeds are the roots of the probabilists' Hermite
// polynomial He_4, +-sqrt(3 -+ sqrt 6), with Gauss-Hermite weights
// (3 +- sqrt 6)/12 (the larger weight on the inner speed); T_L = 1.
// D2Q9 (App. A): speeds -1, 0, 1 with weights 1/6, 2/3, 1/6; T_L = 1/3.
template <int Q1> struct Lat;

template <> struct Lat<4> {
  static constexpr double TL = 1.0;
  static constexpr double inv_TL = 1.0;
  __host__ __device__ static constexpr double c(int i) {
    return i == 0 ? -2.334414218338977239317512
         : i == 1 ? -0.7419637843027258576485136
         : i == 2 ? 0.7419637843027258576485136
                  : 2.334414218338977239317512;
  }
  __host__ __device__ static constexpr double w(int i) {
    return (i == 0 || i == 3) ? 0.04587585476806849181689299 : 0.454124145231931508183107;
  }
};

template <> struct Lat<3> {
  static constexpr double TL = 1.0 / 3.0;
  static constexpr double inv_TL = 3.0;
  __host__ __device__ static constexpr double c(int i) { return double(i - 1); }
  __host__ __device__ static constexpr double w(int i) { return i == 1 ? 2.0 / 3.0 : 1.0 / 6.0; }
};

// 1 / prod_{m != k} (c_k - c_m): normalisation of the Lagrange basis
// polynomial attached to speed k.
template <int Q1>
__host__ __device__ constexpr double lag_inv_den(int k) {
  double d = 1.0;
  for (int m = 0; m < Q1; ++m)
    if (m != k) d *= (Lat<Q1>::c(k) - Lat<Q1>::c(m));
  return 1.0 / d;
}

// prod_{m != k} (z - c_m): unnormalised Lagrange basis polynomial of speed k.
template <int Q1, class R>
__device__ __forceinline__ R lag_num(int k, R z) {
  R p = R(1);
#pragma unroll
  for (int m = 0; m < Q1; ++m)
    if (m != k) p *= (z - R(Lat<Q1>::c(m)));
  return p;
}

// Monomial coefficients of the normalised Lagrange basis polynomial of speed
// k: l_k(z) = sum_e coef[e] z^e (for Horner evaluation with a run-time k).
template <int Q1>
struct LagCoef {
  double v[4][4];
  constexpr LagCoef() : v{} {
    for (int k = 0; k < Q1; ++k) {
      double p[4] = {1.0, 0.0, 0.0, 0.0};  // running product, degree <= 3
      int deg = 0;
      for (int m = 0; m < Q1; ++m) {
        if (m == k) continue;
        // p(z) *= (z - c_m)
        for (int e = deg + 1; e >= 1; --e) p[e] = p[e - 1] - Lat<Q1>::c(m) * p[e];
        p[0] = -Lat<Q1>::c(m) * p[0];
        ++deg;
      }
      const double s = lag_inv_den<Q1>(k);
      for (int e = 0; e < 4; ++e) v[k][e] = p[e] * s;
    }
  }
};

// Per-speed tables in constant memory for wave-uniform run-time indices:
// the speed c_k and the Horner coefficients of l_k.
template <int Q1>
struct SpeedTable {
  double c[4];
  double lag[4][4];
  constexpr SpeedTable() : c{}, lag{} {
    constexpr LagCoef<Q1> C{};
    for (int k = 0; k < Q1; ++k) {
      c[k] = Lat<Q1>::c(k);
      for (int e = 0; e < 4; ++e) lag[k][e] = C.v[k][e];
    }
  }
};

__constant__ const SpeedTable<4> kSpeeds4 = SpeedTable<4>();
__constant__ const SpeedTable<3> kSpeeds3 = SpeedTable<3>();

template <int Q1>
__device__ __forceinline__ const SpeedTable<Q1>& speeds();
template <>
__device__ __forceinline__ const SpeedTable<4>& speeds<4>() { return kSpeeds4; }
template <>
__device__ __forceinline__ const SpeedTable<3>& speeds<3>() { return kSpeeds3; }

// Horner coefficients of the Lagrange basis polynomial of a speed.
struct LagRow {
  double l0, l1, l2, l3;
};

template <int Q1>
__device__ __forceinline__ LagRow lag_row(int k) {
  const SpeedTable<Q1>& t = speeds<Q1>();
  return LagRow{t.lag[k][0], t.lag[k][1], t.lag[k][2], t.lag[k][3]};
}

// ------------------------------------------------ transfer rows (eq. 4)
// Matching the q per-axis moments of eq. (2) between a source gauge
// {u_s, theta_s} and a target gauge {u_t, theta_t} is Lagrange interpolation
// on the target speeds: the transfer factor is
//     G[k][i] = l_k(z_i),   z_i = r c_i + d,
//     r = sqrt(theta_s / theta_t),  d = (u_s - u_t) / sqrt(theta_t),
// with l_k the Lagrange basis polynomial of speed c_k (App. B gives the same
// matrix for D2Q9 in closed form).  Row k for all source speeds i:
template <int Q1>
__device__ __forceinline__ void transfer_row(int k, double r, double d, double* row) {
#pragma unroll
  for (int i = 0; i < Q1; ++i) row[i] = lag_num<Q1>(k, r * Lat<Q1>::c(i) + d) * lag_inv_den<Q1>(k);
}

// Full per-axis transfer factor G[k*Q1 + i] = l_k(r c_i + d) (target speed k,
// source speed i), from the differences e_m = z - c_m shared by all k.
template <int Q1, class R>
__device__ __forceinline__ void transfer_factor(R r, R d, R* G) {
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    const R z = r * R(Lat<Q1>::c(i)) + d;
    R e[Q1];
#pragma unroll
    for (int m = 0; m < Q1; ++m) e[m] = z - R(Lat<Q1>::c(m));
    if constexpr (Q1 == 4) {
      const R p01 = e[0] * e[1], p23 = e[2] * e[3];
      G[0 * 4 + i] = (e[1] * p23) * R(lag_inv_den<4>(0));
      G[1 * 4 + i] = (e[0] * p23) * R(lag_inv_den<4>(1));
      G[2 * 4 + i] = (p01 * e[3]) * R(lag_inv_den<4>(2));
      G[3 * 4 + i] = (p01 * e[2]) * R(lag_inv_den<4>(3));
    } else {
      G[0 * 3 + i] = (e[1] * e[2]) * R(lag_inv_den<3>(0));
      G[1 * 3 + i] = (e[0] * e[2]) * R(lag_inv_den<3>(1));
      G[2 * 3 + i] = (e[0] * e[1]) * R(lag_inv_den<3>(2));
    }
  }
}

// Row of the transfer factor for the basis polynomial with coefficients P.
template <int Q1>
__device__ __forceinline__ void transfer_row_coef(const LagRow& P, double r, double d, double* row) {
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    const double z = fma(r, Lat<Q1>::c(i), d);
    row[i] = fma(fma(fma(P.l3, z, P.l2), z, P.l1), z, P.l0);
  }
}

// Speed c_i for a run-time (wave-uniform) i.
template <int Q1>
__device__ __forceinline__ double speed_rt(int i) {
  return speeds<Q1>().c[i];
}

// ----------------------------------------------- reconstruction (App. C)
// Third-order Lagrange weights on the four collocation points x0 + n,
// x0 = floor(x) - 1, at local coordinate t = x - x0 in [1, 2).
// Cubic Lagrange weight of a stencil node at signed distance u from the
// departure point (node minus point), as one function of |u| (App. C): the
// four-node stencil around the point is symmetric, so the weight is
// (|u|+1)(|u|-1)(|u|-2)/2 for |u| <= 1, -(|u|-1)(|u|-2)(|u|-3)/6 for
// 1 < |u| < 2, and the node is outside the stencil (in = false, weight 0)
// beyond.  Evaluated in FT from |u| (FP32: |u| rounded once).  In FP32 the
// monomial coefficients -1/6 and -11/6 of the outer weight both round away
// from zero, which made every outer weight about 8e-8 too small: the
// weights of a departure point then summed to about 1 - 1.5e-7, a mass loss
// of that size at every step.  FP32 therefore takes the product form, whose
// factors |u| - 1, |u| - 2, 3 - |u| are exact for |u| in [1, 2] and whose 1/6
// enters as a float pair.
template <class FT>
__device__ __forceinline__ FT lagrange_weight(double u, bool& in) {
  const FT a = FT(fabs(u));
  FT near, far;
  if constexpr (sizeof(FT) == 4) {
    const FT t = (a - 1.0f) * (a - 2.0f);
    near = t * fmaf(0.5f, a, 0.5f);
    const FT p = t * (3.0f - a);
    far = fmaf(p, split_lo(1.0 / 6.0), p * split_hi(1.0 / 6.0));
  } else {
    near = fma(fma(fma(FT(0.5), a, FT(-1.0)), a, FT(-0.5)), a, FT(1.0));
    far = fma(fma(fma(FT(-1.0 / 6.0), a, FT(1.0)), a, FT(-11.0 / 6.0)), a, FT(1.0));
  }
  in = a < FT(2.0);
  const FT w = a <= FT(1.0) ? near : far;
  return in ? w : FT(0);
}

__device__ __forceinline__ void interp_weights(double t, double* a) {
  const double t0 = t, t1 = t - 1.0, t2 = t - 2.0, t3 = t - 3.0;
  a[0] = t1 * t2 * t3 * (-1.0 / 6.0);
  a[1] = t0 * t2 * t3 * 0.5;
  a[2] = t0 * t1 * t3 * (-0.5);
  a[3] = t0 * t1 * t2 * (1.0 / 6.0);
}

// Wave-wide maximum of a non-negative int.  In a branch that only part of
// the wave executes, a cross-lane read (ds_bpermute) from an inactive lane
// returns 0, which is neutral for this maximum.
__device__ __forceinline__ int wave_max_nonneg(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

// Wave-wide range [wlo, whi] of the stencil columns of the active lanes that
// have one (has = false: the lane adds nothing).  Both bounds are reduced as
// maxima of positive codes, so inactive lanes add nothing either.  Column
// offsets come from saturated floors (|x| <= 1e9), so the codes stay below
// 2^31.  Returns false if no active lane has a range.
__device__ __forceinline__ bool wave_column_range(int lo, int hi, bool has, int& wlo, int& whi) {
  constexpr int kBias = 1 << 30;
  const int a = wave_max_nonneg(has ? kBias - lo : 0);
  const int b = wave_max_nonneg(has ? hi + kBias : 0);
  wlo = kBias - a;
  whi = b - kBias;
  return a > 0;
}

// A wave walks the union of its lanes' stencil columns; a lane whose stencil
// lies further than this from its node is handled on its own instead.
constexpr int kFarColumns = 256;

// Weight of stencil node n (0..3) alone: the same products as interp_weights.
__device__ __forceinline__ double interp_weight_at(int n, double t) {
  const double e1 = t - (n == 0 ? 1.0 : 0.0);
  const double e2 = t - (n <= 1 ? 2.0 : 1.0);
  const double e3 = t - (n <= 2 ? 3.0 : 2.0);
  const double cn = n == 0 ? -1.0 / 6.0 : n == 1 ? 0.5 : n == 2 ? -0.5 : 1.0 / 6.0;
  return e1 * e2 * e3 * cn;
}

// Stencil index -> node index: periodic wrap or zero-gradient clamp.
__device__ __forceinline__ int wrap_index(int i, int n, int bc) {
  if (bc == 0) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Derivatives of the interpolation weights with respect to t.
__device__ __forceinline__ void interp_weights_d(double t, double* a, double* da) {
  const double t0 = t, t1 = t - 1.0, t2 = t - 2.0, t3 = t - 3.0;
  a[0] = t1 * t2 * t3 * (-1.0 / 6.0);
  a[1] = t0 * t2 * t3 * 0.5;
  a[2] = t0 * t1 * t3 * (-0.5);
  a[3] = t0 * t1 * t2 * (1.0 / 6.0);
  da[0] = (t2 * t3 + t1 * t3 + t1 * t2) * (-1.0 / 6.0);
  da[1] = (t2 * t3 + t0 * t3 + t0 * t2) * 0.5;
  da[2] = (t1 * t3 + t0 * t3 + t0 * t1) * (-0.5);
  da[3] = (t1 * t2 + t0 * t2 + t0 * t1) * (1.0 / 6.0);
}

// Derivative of the Lagrange basis polynomial with Horner coefficients P.
__device__ __forceinline__ double lag_deriv(const LagRow& P, double z) {
  return fma(fma(3.0 * P.l3, z, 2.0 * P.l2), z, P.l1);
}

// dG[k*Q1 + i] = l_k'(r c_i + d) for the full per-axis factor.
template <int Q1>
__device__ __forceinline__ void transfer_factor_deriv(double r, double d, double* dG) {
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    const double z = r * Lat<Q1>::c(i) + d;
    double e[Q1];
#pragma unroll
    for (int m = 0; m < Q1; ++m) e[m] = z - Lat<Q1>::c(m);
#pragma unroll
    for (int k = 0; k < Q1; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < Q1; ++m) {
        if (m == k) continue;
        double p = 1.0;
#pragma unroll
        for (int mm = 0; mm < Q1; ++mm)
          if (mm != k && mm != m) p *= e[mm];
        acc += p;
      }
      dG[k * Q1 + i] = acc * lag_inv_den<Q1>(k);
    }
  }
}


// Error-free sum (Knuth TwoSum) for compensated accumulation.  Contraction
// is off here: the error term is exact only if t is the rounded sum of s and
// x as written.
template <class R>
__device__ __forceinline__ void two_sum_acc(R& s, R& c, R x) {
#pragma clang fp contract(off)
  const R t = s + x;
  const R bp = t - s;
  c += (s - (t - bp)) + (x - bp);
  s = t;
}

// One term of a compensated dot product (Ogita, Rump & Oishi 2005, Dot2)
// with a constant factor a = a_hi + a_lo held as two values of type R: the
// product a_hi x is split exactly by one FMA (TwoProduct), its sum with s by
// TwoSum, and both rounding errors plus a_lo x go into the compensation c.
// The result carries the accuracy of a sum in twice the working precision.
template <class R>
__device__ __forceinline__ void dot2_acc(R& s, R& c, R a_hi, R a_lo, R x) {
#pragma clang fp contract(off)
  const R p = a_hi * x;
  const R pe = fma(a_hi, x, -p);
  const R t = s + p;
  const R bp = t - s;
  c += ((s - (t - bp)) + (p - bp)) + fma(a_lo, x, pe);
  s = t;
}

// LDS layout of the staged window: the Q values of a window node are kept in
// groups of G = 16 / sizeof(FT) populations whose values are adjacent, so
// that a group is one 16-byte LDS read.  Group g of node k starts at element
// g * G * WN + k * G.
template <int Q1, class FT, int WN>
struct Win {
  static constexpr int Q = Q1 * Q1;
  static constexpr int G = 16 / (int)sizeof(FT);
  static constexpr int NG = (Q + G - 1) / G;
  static constexpr int NGH = NG / 2;  // groups read from the first base
  static constexpr int GS = G * WN;   // group stride in elements
  static constexpr int size = NG * GS;
  using V = FT __attribute__((ext_vector_type(16 / sizeof(FT))));
  __device__ static int at(int p, int k) { return (p / G) * GS + k * G + p % G; }
  // The Q values of a node, element offset e = k * G; groups from NGH on are
  // read from eh = e + NGH * GS (a second base keeps every offset within the
  // 16-bit offset field of the read).
  __device__ static void load(const FT* s, int e, int eh, FT* f) {
    V v[NG];
#pragma unroll
    for (int g = 0; g < NGH; ++g) v[g] = *reinterpret_cast<const V*>(s + e + g * GS);
#pragma unroll
    for (int g = NGH; g < NG; ++g) v[g] = *reinterpret_cast<const V*>(s + eh + (g - NGH) * GS);
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int c = 0; c < G; ++c)
        if (g * G + c < Q) f[g * G + c] = v[g][c];
  }
};

}  // namespace pond
