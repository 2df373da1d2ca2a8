// Adjoint (vector-Jacobian product) of one PonD step on gfx950.
//
// The forward step is differentiated as computed: the predictor-corrector
// loop is unrolled with the pass count the forward step recorded per node, the
// stencil origins floor(x) - 1 are held fixed, and the App. E test is not
// differentiated.  Per node (one lane) the kernel
//   1. reads the pass history that the forward step recorded (the gauge
//      lambda_k and density of every pass, the last pass's populations);
//   2. runs the chain backwards: BGK (eq. 18), regauge (eq. 4), then for each
//      pass the corrector moments (eqs. 10-12) and the advection (eqs. 5-6);
//   3. adds the seed's cotangent (eqs. 7-8) to its own node.
// Cotangents of the collocation points are scattered in the block's reference
// gauge lambda_B into FP64 accumulators in LDS (ds_add_f64); after a barrier
// every window node's accumulator is mapped back through G_{s->B}^T and the
// derivative of G_{s->B} with respect to the node's own gauge, and added to
// the output with global FP64 atomics (windows of neighbouring blocks
// overlap).  Points outside the window scatter straight to HBM.  lambda_B is a
// constant of the computation: G_{B->n} G_{s->B} = G_{s->n} does not depend on
// it.  All adjoint arithmetic is FP64; the FP32-mixed state is read and
// widened.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdlib.h>

#include "pond_device.hpp"
#include "pond_internal.hpp"

namespace pond {
namespace {

constexpr int kMaxPasses = 64;

struct AdjArgs {
  int nx, ny, bc_x, bc_y, seed_mode, isothermal;
  double tau;
  const void* f_in;
  const double* g_in;
  const uint8_t* iters;
  const double* tape;    // pass history of the step (layout of StepArgs::tape)
  const double* tape_f;  // last pass's populations of the step
  int tape_slots;        // gauge slots per node in the tape
  const double* af_out;  // [Q][N]
  const double* ag_out;  // [3][N]
  double* af_in;         // [Q][N], zeroed before the launch
  double* ag_in;         // [3][N], zeroed before the launch
  double* adj_tau;       // nullable
  TileQueue* queue;      // tiles are taken from it until it is empty
};

__device__ __forceinline__ int sat_floor_a(double x) {
  x = fmin(fmax(x, -1.0e9), 1.0e9);
  return isfinite(x) ? int(floor(x)) : 0;
}

template <int NW>
__device__ __forceinline__ void block_reduce_a(int v[4], double a[4], int* s_i, double* s_d) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int o = __shfl_xor(v[k], off);
      v[k] = o < v[k] ? o : v[k];
      a[k] += __shfl_xor(a[k], off);
    }
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s_i[k * NW + wave] = v[k];
      s_d[k * NW + wave] = a[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int m = s_i[k * NW];
    double t = s_d[k * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      m = s_i[k * NW + w] < m ? s_i[k * NW + w] : m;
      t += s_d[k * NW + w];
    }
    v[k] = m;
    a[k] = t;
  }
}

// Gauge of one pass: u_x, u_y, sqrt(theta) and T.
struct Gauge {
  double ux, uy, s, T;
};

// Tile of TX x TY nodes with YS lanes per node (YS = 2 or 4: the lanes of a
// node take an equal share of the y speeds each).
template <int Q1, class FT, int TX, int TY, int H, int YS>
struct AdjShape {
  static constexpr int WX = TX + 2 * H;
  static constexpr int WY = TY + 2 * H;
  static constexpr int WN = WX * WY;
  static constexpr int NT = TX * TY * YS;  // threads
  static constexpr int NW = NT / 64;
  static_assert(YS == 1 || (Q1 % YS == 0 && (YS & (YS - 1)) == 0),
                "the y speeds split evenly over a node's lanes, a power of two");
  static_assert(((size_t)Win<Q1, double, WN>::size + (size_t)Q1 * Q1 * WN) * sizeof(double) + 1024 <=
                    160 * 1024,
                "LDS");
};

// Context of one lane: everything the per-pass routines need.
template <int Q1, class FT, int WX, int WY, int WN>
struct Lane {
  const AdjArgs* A;
  const double* s_fB;  // staged window, reference gauge
  double* s_acc;       // cotangent accumulators, reference gauge
  int X, Y, wx0, wy0;
  size_t plane;
  double uxB, uyB, sB;
};

// x axis of a pass at gauge G, for every x speed i: column offsets
// o_i = x0_i - X, the coordinate t_i of the departure point in its stencil
// (weights are evaluated per column), rows of G_{B->n} along x, and the
// wave's column walk: first the union of the stencils of its lanes (columns
// wlo .. wlo + njoint - 1), then, if a lane's stencil lies more than
// kFarColumns nodes away, 4 q columns that such lanes walk on their own
// (stencil node c % 4 of x speed c / 4).
template <int Q1>
struct XAxis {
  int o[Q1];
  double t[Q1];
  double gbx[Q1][Q1];
  bool far;
  int wlo, njoint, ncol;
};

// Cubic Lagrange weight of stencil node n (0..3) at t and its derivative:
// the same products as interp_weights / interp_weights_d.
__device__ __forceinline__ void interp_weight_n(int n, double t, double& a, double& da) {
  const double e1 = t - (n == 0 ? 1.0 : 0.0);
  const double e2 = t - (n <= 1 ? 2.0 : 1.0);
  const double e3 = t - (n <= 2 ? 3.0 : 2.0);
  // the constant factor as a sign and a magnitude (two-way selects; a
  // four-way chain on n is compiled into branches)
  const double mag = ((n + 1) & 2) == 0 ? 1.0 / 6.0 : 0.5;  // nodes 0, 3 : 1, 2
  const double cn = (n & 1) ? mag : -mag;
  a = e1 * e2 * e3 * cn;
  da = (e2 * e3 + e1 * e3 + e1 * e2) * cn;
}

template <int Q1>
__device__ __forceinline__ void x_axis(int X, const Gauge& G, double rB, double dBx, XAxis<Q1>& x) {
  using L = Lat<Q1>;
  int lo = INT_MAX, hi = INT_MIN;
  bool has = false;
  x.far = false;
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    const double xd = double(X) - (G.s * L::c(i) + G.ux);
    const double fl = floor(xd);
    x.t[i] = xd - (fl - 1.0);
    x.o[i] = sat_floor_a(fl) - 1 - X;
    transfer_row<Q1>(i, rB, dBx, x.gbx[i]);
    if (isfinite(xd)) {
      lo = x.o[i] < lo ? x.o[i] : lo;
      hi = x.o[i] + 3 > hi ? x.o[i] + 3 : hi;
      has = true;
      x.far = x.far || x.o[i] < -kFarColumns || x.o[i] > kFarColumns;
    }
  }
  int whi;
  x.njoint = wave_column_range(lo, hi, has && !x.far, x.wlo, whi) ? whi - x.wlo + 1 : 0;
  x.ncol = x.njoint + (__any(x.far) ? 4 * Q1 : 0);
}

// Column cc of the walk: offset from X and, per x speed, the weight of the
// column (zero outside the speed's stencil) and its derivative.
template <int Q1, bool kDeriv>
__device__ __forceinline__ bool x_column(const XAxis<Q1>& x, int cc, int& rel, double* wx,
                                         double* dwx) {
  const bool joint = cc < x.njoint;
  // speed and node of a far lane's own column; opaque to the optimiser so
  // that the selections below stay selections (no indexed private arrays)
  int isel = (cc - x.njoint) >> 2;
  asm volatile("" : "+v"(isel));
  const int nsel = (cc - x.njoint) & 3;
  rel = x.wlo + cc;
  if (!joint) {
    rel = x.o[0] + nsel;
#pragma unroll
    for (int i = 1; i < Q1; ++i) rel = isel == i ? x.o[i] + nsel : rel;
  }
  bool need = false;
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    const int n = rel - x.o[i];
    const bool in = (unsigned)n < 4u && (joint ? !x.far : x.far && isel == i);
    double a, d;
    interp_weight_n(n, x.t[i], a, d);
    wx[i] = in ? a : 0.0;
    if (kDeriv) dwx[i] = in ? d : 0.0;
    need = need || in;
  }
  return need;
}

__device__ __forceinline__ double pick4(const double* a, int m) {
  return m == 0 ? a[0] : m == 1 ? a[1] : m == 2 ? a[2] : a[3];
}

// Adjoint of a window collocation point for one row (staged values at
// element offsets e, eh of the grouped window layout; cotangent planes below
// Q/2 from index k, the others from kh = k + Q/2 WN): val[i] = x speed i's
// transformed value (before weights), cotangents of the G_{B->n} rows
// accumulated in gbx_bar / gby_bar, and the cotangent of the staged
// populations scattered into the LDS accumulators.  cw[i] is the cotangent
// of the point's contribution to x speed i.
template <int Q1, int WN>
__device__ __forceinline__ void adj_window_point(const double* s_fB, double* s_acc, int e, int eh,
                                                 int k, int kh, const double* gby,
                                                 const double (*gbx)[Q1], const double* cw,
                                                 double* val, double (*gbx_bar)[Q1],
                                                 double* gby_bar) {
  constexpr int Q = Q1 * Q1, QH = Q / 2;
  double fs[Q];
  Win<Q1, double, WN>::load(s_fB, e, eh, fs);
  double h[Q1], U[Q1];
#pragma unroll
  for (int ip = 0; ip < Q1; ++ip) {
    double v = 0.0;
#pragma unroll
    for (int jp = 0; jp < Q1; ++jp) v = fma(gby[jp], fs[ip * Q1 + jp], v);
    h[ip] = v;
    double u = 0.0;
#pragma unroll
    for (int i = 0; i < Q1; ++i) u = fma(cw[i], gbx[i][ip], u);
    U[ip] = u;
  }
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    double v = 0.0;
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) {
      v = fma(gbx[i][ip], h[ip], v);
      gbx_bar[i][ip] = fma(cw[i], h[ip], gbx_bar[i][ip]);
    }
    val[i] = v;
  }
#pragma unroll
  for (int jp = 0; jp < Q1; ++jp) {
    double v = 0.0;
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) v = fma(U[ip], fs[ip * Q1 + jp], v);
    gby_bar[jp] += v;
  }
  // cotangent of the staged populations of this point
#pragma unroll
  for (int ip = 0; ip < Q1; ++ip)
#pragma unroll
    for (int jp = 0; jp < Q1; ++jp) {
      const int p = ip * Q1 + jp;
      const int idx = p < QH ? k + p * WN : kh + (p - QH) * WN;
      atomicAdd(&s_acc[idx], U[ip] * gby[jp]);
    }
}

// Adjoint of the four window rows of a column in one run (the lane's whole
// column inside the window; staged values at element offsets e, eh, the
// cotangent planes at indices k, kh, of the first row).  The cotangent of a
// row's transformed point is its y weight times the vector Uc, fixed per
// column, and the x rows of G_{B->n} act on sums over the rows (hc, hd with
// the weights and their derivatives), so a row costs its y contraction, the
// cotangent of the y row and its scatter.  colv / dcol get the column's
// values of the x speeds weighted with ay / day.
template <int Q1, int WX, int WN>
__device__ __forceinline__ void adj_window_column(const double* s_fB, double* s_acc, int e, int eh,
                                                  int k, int kh, const double* ay,
                                                  const double* day, const double* fb,
                                                  const double* wx, const double* gby,
                                                  const double (*gbx)[Q1], double* colv,
                                                  double* dcol, double (*gbx_bar)[Q1],
                                                  double* gby_bar) {
  using W = Win<Q1, double, WN>;
  constexpr int Q = Q1 * Q1, QH = Q / 2;
  double fw[Q1], Uc[Q1], hc[Q1], hd[Q1];
#pragma unroll
  for (int i = 0; i < Q1; ++i) fw[i] = fb[i] * wx[i];
#pragma unroll
  for (int ip = 0; ip < Q1; ++ip) {
    double u = 0.0;
#pragma unroll
    for (int i = 0; i < Q1; ++i) u = fma(fw[i], gbx[i][ip], u);
    Uc[ip] = u;
    hc[ip] = 0.0;
    hd[ip] = 0.0;
  }
  double fnext[Q];
  W::load(s_fB, e, eh, fnext);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const double aym = pick4(ay, m), daym = pick4(day, m);  // constant index once unrolled
    double fs[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) fs[p] = fnext[p];
    // the next row's reads go out before this row's LDS atomics, which
    // the compiler does not move reads across
    if (m < 3) W::load(s_fB, e + (m + 1) * WX * W::G, eh + (m + 1) * WX * W::G, fnext);
    double U[Q1];
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) {
      double v = 0.0;
#pragma unroll
      for (int jp = 0; jp < Q1; ++jp) v = fma(gby[jp], fs[ip * Q1 + jp], v);
      hc[ip] = fma(aym, v, hc[ip]);
      hd[ip] = fma(daym, v, hd[ip]);
      U[ip] = aym * Uc[ip];
    }
#pragma unroll
    for (int jp = 0; jp < Q1; ++jp) {
      double v = 0.0;
#pragma unroll
      for (int ip = 0; ip < Q1; ++ip) v = fma(U[ip], fs[ip * Q1 + jp], v);
      gby_bar[jp] += v;
    }
    // cotangent of the staged populations of this point
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip)
#pragma unroll
      for (int jp = 0; jp < Q1; ++jp) {
        const int p = ip * Q1 + jp;
        const int idx = (p < QH ? k + p * WN : kh + (p - QH) * WN) + m * WX;
        atomicAdd(&s_acc[idx], U[ip] * gby[jp]);
      }
  }
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    double v = 0.0, d = 0.0;
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) {
      v = fma(gbx[i][ip], hc[ip], v);
      d = fma(gbx[i][ip], hd[ip], d);
      gbx_bar[i][ip] = fma(fw[i], hc[ip], gbx_bar[i][ip]);
    }
    colv[i] = v;
    dcol[i] = d;
  }
}

// Adjoint of a collocation point outside the window (HBM state at (gx, gy),
// direct transform G_{s->n}): val[i] as above, the cotangent of the pass
// gauge added to (gux, guy, gs), and the cotangents of the point's own
// populations and gauge scattered to HBM.
template <int Q1, class FT, int WX, int WY, int WN>
__device__ __forceinline__ void adj_hbm_point(const Lane<Q1, FT, WX, WY, WN>& c, const Gauge& G,
                                              int gx, int gy, const LagRow& Pj, double inv_s,
                                              const double* cw, double* val, double& gux,
                                              double& guy, double& gs) {
  using L = Lat<Q1>;
  const AdjArgs& A = *c.A;
  const FT* __restrict__ fin = static_cast<const FT*>(A.f_in);
  const size_t src = (size_t)wrap_index(gy, A.ny, A.bc_y) * A.nx + wrap_index(gx, A.nx, A.bc_x);
  double fs[Q1 * Q1];
#pragma unroll
  for (int p = 0; p < Q1 * Q1; ++p) fs[p] = double(fin[(size_t)p * c.plane + src]);
  const double ss = sqrt(A.g_in[2 * c.plane + src] * L::inv_TL);
  const double r = ss * inv_s;
  const double dx = (A.g_in[src] - G.ux) * inv_s, dy = (A.g_in[c.plane + src] - G.uy) * inv_s;
  double zx[Q1], zy[Q1], gyr[Q1];
#pragma unroll
  for (int q = 0; q < Q1; ++q) {
    zx[q] = fma(r, L::c(q), dx);
    zy[q] = fma(r, L::c(q), dy);
    gyr[q] = fma(fma(fma(Pj.l3, zy[q], Pj.l2), zy[q], Pj.l1), zy[q], Pj.l0);
  }
  double h[Q1], Ux[Q1], dsum[Q1];  // dsum[ip] = sum_i cw_i l_i'(zx[ip])
#pragma unroll
  for (int ip = 0; ip < Q1; ++ip) {
    double v = 0.0;
#pragma unroll
    for (int jp = 0; jp < Q1; ++jp) v = fma(gyr[jp], fs[ip * Q1 + jp], v);
    h[ip] = v;
    Ux[ip] = 0.0;
    dsum[ip] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    const LagRow Pi = lag_row<Q1>(i);
    double v = 0.0;
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) {
      const double gx_r = fma(fma(fma(Pi.l3, zx[ip], Pi.l2), zx[ip], Pi.l1), zx[ip], Pi.l0);
      v = fma(gx_r, h[ip], v);
      Ux[ip] = fma(cw[i], gx_r, Ux[ip]);
      dsum[ip] = fma(cw[i], lag_deriv(Pi, zx[ip]), dsum[ip]);
    }
    val[i] = v;
  }
  double zs_x = 0.0, zs_y = 0.0, zsc = 0.0, zz = 0.0;
#pragma unroll
  for (int ip = 0; ip < Q1; ++ip) {
    const double zb = h[ip] * dsum[ip];
    zs_x += zb;
    zsc = fma(zb, L::c(ip), zsc);
    zz = fma(zb, zx[ip], zz);
  }
#pragma unroll
  for (int jp = 0; jp < Q1; ++jp) {
    double v = 0.0;
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) v = fma(Ux[ip], fs[ip * Q1 + jp], v);
    const double zb = v * lag_deriv(Pj, zy[jp]);
    zs_y += zb;
    zsc = fma(zb, L::c(jp), zsc);
    zz = fma(zb, zy[jp], zz);
  }
  // z = (s_s c + u_s - u) / s
  gux -= zs_x * inv_s;
  guy -= zs_y * inv_s;
  gs -= zz * inv_s;
  atomicAdd(&A.ag_in[src], zs_x * inv_s);
  atomicAdd(&A.ag_in[c.plane + src], zs_y * inv_s);
  // d s_s / d T_s = inv_TL / (2 s_s)
  atomicAdd(&A.ag_in[2 * c.plane + src], zsc * inv_s * L::inv_TL / (2.0 * ss));
#pragma unroll
  for (int ip = 0; ip < Q1; ++ip)
#pragma unroll
    for (int jp = 0; jp < Q1; ++jp)
      atomicAdd(&A.af_in[(size_t)(ip * Q1 + jp) * c.plane + src], Ux[ip] * gyr[jp]);
}

// Adjoint of one forward pass at gauge G with cotangent Fb of its output, for
// the y speeds jlo .. jhi - 1 (all of them, or the lane's share when several
// lanes share a node).  Scatters the collocation points' cotangents and adds the
// cotangent of the gauge (u_x, u_y, s) to (gux, guy, gs).  Column by column like the forward
// pass: at each collocation point the cotangents of the four x speeds are
// summed before they are scattered (one LDS atomic per population).
template <int Q1, class FT, int WX, int WY, int WN>
__device__ void adjoint_pass(const Lane<Q1, FT, WX, WY, WN>& c, const Gauge& G, const double* Fb,
                             int jlo, int jhi, double& gux, double& guy, double& gs) {
  using L = Lat<Q1>;
  using W = Win<Q1, double, WN>;
  constexpr int QH = Q1 * Q1 / 2;
  const double inv_s = 1.0 / G.s;
  const double rB = c.sB * inv_s, dBx = (c.uxB - G.ux) * inv_s, dBy = (c.uyB - G.uy) * inv_s;
  XAxis<Q1> x;
  x_axis<Q1>(c.X, G, rB, dBx, x);
  double gbx_bar[Q1][Q1], tx_bar[Q1];
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    tx_bar[i] = 0.0;
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) gbx_bar[i][ip] = 0.0;
  }
#pragma unroll 1
  for (int j = jlo; j < jhi; ++j) {
    const double cj = speed_rt<Q1>(j);
    const double yd = double(c.Y) - (G.s * cj + G.uy);
    const double fly = floor(yd);
    double ay[4], day[4];
    interp_weights_d(yd - (fly - 1.0), ay, day);
    const int y0 = sat_floor_a(fly) - 1;
    const int ly0 = y0 - c.wy0;
    const bool rows_in = (unsigned)ly0 <= (unsigned)(WY - 4);
    const LagRow Pj = lag_row<Q1>(j);
    double gby[Q1], gby_bar[Q1];
    transfer_row_coef<Q1>(Pj, rB, dBy, gby);
#pragma unroll
    for (int jp = 0; jp < Q1; ++jp) gby_bar[jp] = 0.0;
    double fb[Q1];
#pragma unroll
    for (int i = 0; i < Q1; ++i) {
      fb[i] = 0.0;
#pragma unroll
      for (int jj = 0; jj < Q1; ++jj)
        if (jj == j) fb[i] = Fb[i * Q1 + jj];
    }
    double ty_bar = 0.0;
#pragma unroll 1
    for (int cc = 0; cc < x.ncol; ++cc) {
      int rel;
      double wx[Q1], dwx[Q1];
      const bool need = x_column<Q1, true>(x, cc, rel, wx, dwx);
      if (!__any(need)) continue;
      const int gx = c.X + rel, lx = gx - c.wx0;
      double colv[Q1], dcol[Q1];  // sum over rows of ay[m] val, day[m] val
#pragma unroll
      for (int i = 0; i < Q1; ++i) {
        colv[i] = 0.0;
        dcol[i] = 0.0;
      }
      if (need && rows_in && (unsigned)lx < (unsigned)WX) {
        const int k = ly0 * WX + lx;
        int kh = k + QH * WN;
        asm volatile("" : "+v"(kh));
        const int e = k * W::G;
        int eh = e + W::NGH * W::GS;
        asm volatile("" : "+v"(eh));
        adj_window_column<Q1, WX, WN>(c.s_fB, c.s_acc, e, eh, k, kh, ay, day, fb, wx, gby, x.gbx,
                                      colv, dcol, gbx_bar, gby_bar);
      } else if (need) {
#pragma unroll 1
        for (int m = 0; m < 4; ++m) {
          const int gy = y0 + m, ly = gy - c.wy0;
          const double aym = pick4(ay, m), daym = pick4(day, m);
          double cw[Q1], val[Q1];
#pragma unroll
          for (int i = 0; i < Q1; ++i) cw[i] = fb[i] * wx[i] * aym;
          if ((unsigned)lx < (unsigned)WX && (unsigned)ly < (unsigned)WY) {
            const int kk = ly * WX + lx;
            adj_window_point<Q1, WN>(c.s_fB, c.s_acc, kk * W::G, kk * W::G + W::NGH * W::GS, kk,
                                     kk + QH * WN, gby, x.gbx, cw, val, gbx_bar, gby_bar);
          } else {
            adj_hbm_point<Q1, FT, WX, WY, WN>(c, G, gx, gy, Pj, inv_s, cw, val, gux, guy, gs);
          }
#pragma unroll
          for (int i = 0; i < Q1; ++i) {
            colv[i] = fma(aym, val[i], colv[i]);
            dcol[i] = fma(daym, val[i], dcol[i]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < Q1; ++i) {
        tx_bar[i] = fma(fb[i] * dwx[i], colv[i], tx_bar[i]);
        ty_bar = fma(fb[i] * wx[i], dcol[i], ty_bar);
      }
    }
    // y departure: t = y - s c_j - u_y - y0
    guy -= ty_bar;
    gs -= cj * ty_bar;
    // G_{B->n} y rows: z = rB c + dBy = (sB c + uyB - u_y) / s
    double zs = 0.0, zz = 0.0;
#pragma unroll
    for (int jp = 0; jp < Q1; ++jp) {
      const double z = fma(rB, L::c(jp), dBy);
      const double zb = gby_bar[jp] * lag_deriv(Pj, z);
      zs += zb;
      zz = fma(zb, z, zz);
    }
    guy -= zs * inv_s;
    gs -= zz * inv_s;
  }
  // x departures and the G_{B->n} x rows, summed over the y speeds
  double zs = 0.0, zz = 0.0;
#pragma unroll
  for (int i = 0; i < Q1; ++i) {
    gux -= tx_bar[i];
    gs -= L::c(i) * tx_bar[i];
    const LagRow Pi = lag_row<Q1>(i);
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) {
      const double z = fma(rB, L::c(ip), dBx);
      const double zb = gbx_bar[i][ip] * lag_deriv(Pi, z);
      zs += zb;
      zz = fma(zb, z, zz);
    }
  }
  gux -= zs * inv_s;
  gs -= zz * inv_s;
}

template <int Q1, class FT, int TX, int TY, int H, int YS>
__global__ void __launch_bounds__(TX * TY * YS)
k_step_adjoint(AdjArgs A) {
  constexpr int Q = Q1 * Q1;
  using L = Lat<Q1>;
  using S = AdjShape<Q1, FT, TX, TY, H, YS>;
  constexpr int WX = S::WX, WY = S::WY, WN = S::WN, NT = S::NT;
  __shared__ __align__(16) double s_fB[Win<Q1, double, WN>::size];
  __shared__ double s_acc[Q * WN];
  __shared__ int s_ri[4 * S::NW];
  __shared__ double s_rd[4 * S::NW];
  __shared__ unsigned s_tile;

  const int tid = threadIdx.x;
  const int ntx = (A.nx + TX - 1) / TX;
  const unsigned ntiles = (unsigned)ntx * (unsigned)((A.ny + TY - 1) / TY);
  double tau_bar = 0.0;

  // Persistent blocks: tiles come from the queue (their cost follows the
  // forward pass counts, which vary by an order of magnitude).
  for (;;) {
    if (tid == 0) s_tile = atomicAdd(&A.queue->next, 1u);
    __syncthreads();
    const unsigned tile = s_tile;
    if (tile >= ntiles) break;
    const int ty = (int)(tile / (unsigned)ntx), tx = (int)tile - ty * ntx;
    const int bx0 = tx * TX, by0 = ty * TY;
    int tl = tid;
    asm volatile("" : "+v"(tl));  // keep per-lane values from being hoisted out of the loop
    const int wave = tl >> 6, lane = tl & 63;
    // YS = 1: 8 x 8 nodes per wave; YS > 1: lanes YS n .. YS n + YS - 1
    // share a node (part = which share of the y speeds), rows of 16 nodes
    const int part = YS > 1 ? (tl & (YS - 1)) : 0;
    const int X = YS > 1 ? bx0 + (tl / YS) % TX : bx0 + (wave % (TX / 8)) * 8 + (lane & 7);
    const int Y = YS > 1 ? by0 + (tl / YS) / TX : by0 + (wave / (TX / 8)) * 8 + (lane >> 3);
    const size_t plane = (size_t)A.nx * A.ny;
    const size_t node = (size_t)Y * A.nx + X;
    const FT* __restrict__ fin = static_cast<const FT*>(A.f_in);
    const double* __restrict__ gin = A.g_in;

    int K = 0;
    bool active = (X < A.nx) && (Y < A.ny);
    if (active) {
      const unsigned it = A.iters[node];
      K = it & POND_ITERS_MASK;
      // nodes the forward step flagged bad carry no derivative
      if ((it & POND_ITERS_BAD) || K < 1 || K >= kMaxPasses || K >= A.tape_slots) active = false;
    }

    // seed (eqs. 7-8) and the modes of the seed-independence experiment
    double ux0 = 0.0, uy0 = 0.0, T0 = L::TL;
    if (active) {
      ux0 = gin[node];
      uy0 = gin[plane + node];
      T0 = gin[2 * plane + node];
      if (A.seed_mode == 1) {
        ux0 = 0.0;
        uy0 = 0.0;
        if (!A.isothermal) T0 = L::TL;
      } else if (A.seed_mode == 2) {
        ux0 = -ux0;
        uy0 = -uy0;
      }
    }

    // window placement and reference gauge, as in the forward step
    int wx0, wy0;
    double uxB, uyB, sB;
    {
      int v[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
      double a[4] = {0.0, 0.0, 0.0, 0.0};
      const double s0 = sqrt(T0 * L::inv_TL);
      const double sp = s0 * L::c(Q1 - 1);
      if (active && isfinite(sp) && s0 > 0.0 && isfinite(ux0) && isfinite(uy0) &&
          fabs(ux0) < 1e9 && fabs(uy0) < 1e9) {
        v[0] = sat_floor_a(double(X) - ux0 - sp) - 2;
        v[1] = -(sat_floor_a(double(X) - ux0 + sp) + 3);
        v[2] = sat_floor_a(double(Y) - uy0 - sp) - 2;
        v[3] = -(sat_floor_a(double(Y) - uy0 + sp) + 3);
        a[0] = ux0;
        a[1] = uy0;
        a[2] = s0;
        a[3] = 1.0;
      }
      block_reduce_a<S::NW>(v, a, s_ri, s_rd);
      if (a[3] > 0.0) {
        uxB = a[0] / a[3];
        uyB = a[1] / a[3];
        sB = a[2] / a[3];
      } else {
        uxB = 0.0;
        uyB = 0.0;
        sB = 1.0;
        v[0] = bx0 - H;
        v[1] = -(bx0 + TX + H - 1);
        v[2] = by0 - H;
        v[3] = -(by0 + TY + H - 1);
      }
      const int xlo = v[0], xhi = -v[1], ylo = v[2], yhi = -v[3];
      const int nxn = xhi - xlo + 1, nyn = yhi - ylo + 1;
      wx0 = nxn <= WX ? xlo - (WX - nxn) / 2 : (int)(((long long)xlo + xhi) / 2) - WX / 2;
      wy0 = nyn <= WY ? ylo - (WY - nyn) / 2 : (int)(((long long)ylo + yhi) / 2) - WY / 2;
    }
    const double inv_sB = 1.0 / sB;

#ifdef POND_LDS_POISON
    // checking build: every staged value that the loop below does not write
    // reads as NaN, so a read of an unstaged value shows in the output
    for (int k = tid; k < Win<Q1, double, WN>::size; k += NT) s_fB[k] = __builtin_nan("");
    __syncthreads();
#endif
    // stage f^B = G_{s->B} f_s and clear the accumulators
    for (int k = tid; k < WN; k += NT) {
      const int wy = k / WX, wx = k - wy * WX;
      const size_t src = (size_t)wrap_index(wy0 + wy, A.ny, A.bc_y) * A.nx +
                         wrap_index(wx0 + wx, A.nx, A.bc_x);
      double f[Q];
#pragma unroll
      for (int p = 0; p < Q; ++p) f[p] = double(fin[(size_t)p * plane + src]);
      const double r = sqrt(gin[2 * plane + src] * L::inv_TL) * inv_sB;
      double Gx[Q], Gy[Q];
      transfer_factor<Q1, double>(r, (gin[src] - uxB) * inv_sB, Gx);
      transfer_factor<Q1, double>(r, (gin[plane + src] - uyB) * inv_sB, Gy);
#pragma unroll
      for (int kk = 0; kk < Q1; ++kk)
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          double t = 0.0;
#pragma unroll
          for (int i = 0; i < Q1; ++i) {
            double h = 0.0;
#pragma unroll
            for (int j = 0; j < Q1; ++j) h = fma(Gy[l * Q1 + j], f[i * Q1 + j], h);
            t = fma(Gx[kk * Q1 + i], h, t);
          }
          s_fB[Win<Q1, double, WN>::at(kk * Q1 + l, k)] = t;
          s_acc[(kk * Q1 + l) * WN + k] = 0.0;
        }
    }
    __syncthreads();

    if (active) {
      Lane<Q1, FT, WX, WY, WN> c;
      c.A = &A;
      c.s_fB = s_fB;
      c.s_acc = s_acc;
      c.X = X;
      c.Y = Y;
      c.wx0 = wx0;
      c.wy0 = wy0;
      c.plane = plane;
      c.uxB = uxB;
      c.uyB = uyB;
      c.sB = sB;

      // 1. pass history that the forward step recorded: the gauge lambda_k
      // and density of every pass, and the last pass's populations
      const double* __restrict__ tp = A.tape + node;
      auto hist = [&](int k, int comp) { return tp[((size_t)k * 4 + comp) * plane]; };
      const double rhoK = hist(K, 3);
      double F[Q];
#pragma unroll
      for (int p = 0; p < Q; ++p) F[p] = A.tape_f[(size_t)p * plane + node];
      // F holds the populations of the last pass, in gauge lambda_{K-1}.

      // 2a. BGK (eq. 18): f_out = f_reg + omega (rho W - f_reg)
      const double omega = 1.0 / A.tau;
      const Gauge Gk{hist(K - 1, 0), hist(K - 1, 1), sqrt(hist(K - 1, 2) * L::inv_TL),
                     hist(K - 1, 2)};
      const Gauge G1{hist(K, 0), hist(K, 1), sqrt(hist(K, 2) * L::inv_TL), hist(K, 2)};
      const double inv_s1 = 1.0 / G1.s;
      const double r = Gk.s * inv_s1;
      const double dx = (Gk.ux - G1.ux) * inv_s1, dy = (Gk.uy - G1.uy) * inv_s1;
      double Rx[Q], Ry[Q], dRx[Q], dRy[Q];
      transfer_factor<Q1, double>(r, dx, Rx);
      transfer_factor<Q1, double>(r, dy, Ry);
      transfer_factor_deriv<Q1>(r, dx, dRx);
      transfer_factor_deriv<Q1>(r, dy, dRy);
      double HY[Q];  // HY[i][l] = sum_j Ry[l][j] F[i][j]
#pragma unroll
      for (int i = 0; i < Q1; ++i)
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          double h = 0.0;
#pragma unroll
          for (int j = 0; j < Q1; ++j) h = fma(Ry[l * Q1 + j], F[i * Q1 + j], h);
          HY[i * Q1 + l] = h;
        }
      double fb_reg[Q];
      double rho_bar = 0.0;
#pragma unroll
      for (int k = 0; k < Q1; ++k)
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          double freg = 0.0;
#pragma unroll
          for (int i = 0; i < Q1; ++i) freg = fma(Rx[k * Q1 + i], HY[i * Q1 + l], freg);
          const double fb = A.af_out[(size_t)(k * Q1 + l) * plane + node];
          const double W = L::w(k) * L::w(l);
          fb_reg[k * Q1 + l] = (1.0 - omega) * fb;
          rho_bar = fma(omega * W, fb, rho_bar);
          // d omega / d tau = -omega^2
          tau_bar -= omega * omega * fb * (rhoK * W - freg);
        }

      // 2b. regauge (eq. 4) lambda_{K-1} -> lambda_K
      double Fb[Q];
      double HYb[Q];
#pragma unroll
      for (int i = 0; i < Q1; ++i)
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          double h = 0.0;
#pragma unroll
          for (int k = 0; k < Q1; ++k) h = fma(Rx[k * Q1 + i], fb_reg[k * Q1 + l], h);
          HYb[i * Q1 + l] = h;
        }
#pragma unroll
      for (int i = 0; i < Q1; ++i)
#pragma unroll
        for (int j = 0; j < Q1; ++j) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < Q1; ++l) t = fma(Ry[l * Q1 + j], HYb[i * Q1 + l], t);
          Fb[i * Q1 + j] = t;
        }
      // gauge dependence through z = (s_{K-1} c + u_{K-1} - u_K) / s_K
      double zx_bar[Q1], zy_bar[Q1];
#pragma unroll
      for (int i = 0; i < Q1; ++i) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < Q1; ++k) {
          double rb = 0.0;  // Rx-bar[k][i]
#pragma unroll
          for (int l = 0; l < Q1; ++l) rb = fma(fb_reg[k * Q1 + l], HY[i * Q1 + l], rb);
          t = fma(rb, dRx[k * Q1 + i], t);
        }
        zx_bar[i] = t;
      }
#pragma unroll
      for (int j = 0; j < Q1; ++j) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          double rb = 0.0;  // Ry-bar[l][j] = sum_i HYb[i][l] F[i][j]
#pragma unroll
          for (int i = 0; i < Q1; ++i) rb = fma(HYb[i * Q1 + l], F[i * Q1 + j], rb);
          t = fma(rb, dRy[l * Q1 + j], t);
        }
        zy_bar[j] = t;
      }
      // cotangents of the two gauges of the regauge
      double gux_k = 0.0, guy_k = 0.0, gs_k = 0.0;  // lambda_{K-1}
      double gux_1 = A.ag_out[node], guy_1 = A.ag_out[plane + node];
      double gT_1 = A.ag_out[2 * plane + node];
      double gs_1 = 0.0;
#pragma unroll
      for (int q = 0; q < Q1; ++q) {
        const double zx = fma(r, L::c(q), dx), zy = fma(r, L::c(q), dy);
        gux_k += zx_bar[q] * inv_s1;
        gux_1 -= zx_bar[q] * inv_s1;
        guy_k += zy_bar[q] * inv_s1;
        guy_1 -= zy_bar[q] * inv_s1;
        gs_k += (zx_bar[q] + zy_bar[q]) * L::c(q) * inv_s1;
        gs_1 -= (zx_bar[q] * zx + zy_bar[q] * zy) * inv_s1;
      }
      // s = sqrt(T / T_L)
      gT_1 += gs_1 * L::inv_TL / (2.0 * G1.s);
      double rho_bar_next = rho_bar;  // cotangent of rho_K

      // 2c. passes backwards: corrector moments, then advection
#pragma unroll 1
      for (int k = K - 1; k >= 0; --k) {
        const double Tk = hist(k, 2);
        const Gauge G{hist(k, 0), hist(k, 1), sqrt(Tk * L::inv_TL), Tk};
        // moments of pass k from its gauges (eqs. 10-12, peculiar frame)
        const double dux = hist(k + 1, 0) - G.ux, duy = hist(k + 1, 1) - G.uy;
        const double mxr = dux / G.s, myr = duy / G.s;  // mx / rho, my / rho
        const double rho_k1 = hist(k + 1, 3);
        const double e2r =
            A.isothermal ? 0.0 : (2.0 * hist(k + 1, 2) + dux * dux + duy * duy) / (G.s * G.s);
        // cotangents of lambda_{k+1}
        double gux_n = gux_1, guy_n = guy_1, gT_n = gT_1, grho_n = rho_bar_next;
        double gux = gux_n, guy = guy_n, gs = 0.0, gT = 0.0;
        double dux_b = gux_n, duy_b = guy_n, mx_b, my_b, e2_b = 0.0, rho_b = grho_n;
        if (A.isothermal) {
          gT += gT_n;
        } else {
          dux_b -= gT_n * dux;
          duy_b -= gT_n * duy;
          gs += gT_n * G.s * e2r;
          e2_b = 0.5 * gT_n * G.s * G.s / rho_k1;
          rho_b -= 0.5 * gT_n * G.s * G.s * e2r / rho_k1;
        }
        gs += dux_b * mxr + duy_b * myr;
        mx_b = dux_b * G.s / rho_k1;
        my_b = duy_b * G.s / rho_k1;
        rho_b -= (dux_b * dux + duy_b * duy) / rho_k1;
        if (k < K - 1) {
#pragma unroll
          for (int p = 0; p < Q; ++p) Fb[p] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < Q1; ++i)
#pragma unroll
          for (int j = 0; j < Q1; ++j)
            Fb[i * Q1 + j] += rho_b + mx_b * L::c(i) + my_b * L::c(j) +
                              e2_b * (L::c(i) * L::c(i) + L::c(j) * L::c(j));
        if (k == K - 1) {
          gux += gux_k;
          guy += guy_k;
          gs += gs_k;
        }
        {
          // the lane's y speeds; the lanes of a node sum their contributions
          // to the gauge cotangent
          double dgx = 0.0, dgy = 0.0, dgs = 0.0;
          adjoint_pass<Q1, FT, WX, WY, WN>(c, G, Fb, part * (Q1 / YS), (part + 1) * (Q1 / YS), dgx,
                                           dgy, dgs);
#pragma unroll
          for (int off = 1; off < YS; off <<= 1) {
            dgx += __shfl_xor(dgx, off);
            dgy += __shfl_xor(dgy, off);
            dgs += __shfl_xor(dgs, off);
          }
          gux += dgx;
          guy += dgy;
          gs += dgs;
        }
        gT += gs * L::inv_TL / (2.0 * G.s);
        gux_1 = gux;
        guy_1 = guy;
        gT_1 = gT;
        rho_bar_next = 0.0;
      }

      // 3. seed
      double sux = 0.0, suy = 0.0, sT = 0.0;
      if (A.seed_mode == 0) {
        sux = gux_1;
        suy = guy_1;
        sT = gT_1;
      } else if (A.seed_mode == 2) {
        sux = -gux_1;
        suy = -guy_1;
        sT = gT_1;
      } else {
        sT = A.isothermal ? gT_1 : 0.0;
      }
      if (part == 0) {  // once per node
        atomicAdd(&A.ag_in[node], sux);
        atomicAdd(&A.ag_in[plane + node], suy);
        atomicAdd(&A.ag_in[2 * plane + node], sT);
      }
    }

    __syncthreads();
    // map the window's cotangents back to each node's own gauge and add them
    for (int k = tid; k < WN; k += NT) {
      const int wy = k / WX, wx = k - wy * WX;
      const size_t src = (size_t)wrap_index(wy0 + wy, A.ny, A.bc_y) * A.nx +
                         wrap_index(wx0 + wx, A.nx, A.bc_x);
      double ab[Q];
      bool any = false;
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        ab[p] = s_acc[p * WN + k];
        any = any || (ab[p] != 0.0);
      }
      if (!any) continue;
      double f[Q];
#pragma unroll
      for (int p = 0; p < Q; ++p) f[p] = double(fin[(size_t)p * plane + src]);
      const double ss = sqrt(gin[2 * plane + src] * L::inv_TL);
      const double r = ss * inv_sB;
      const double dx = (gin[src] - uxB) * inv_sB, dy = (gin[plane + src] - uyB) * inv_sB;
      double Gx[Q], Gy[Q], dGx[Q], dGy[Q];
      transfer_factor<Q1, double>(r, dx, Gx);
      transfer_factor<Q1, double>(r, dy, Gy);
      transfer_factor_deriv<Q1>(r, dx, dGx);
      transfer_factor_deriv<Q1>(r, dy, dGy);
      // f^B[k][l] = sum_i Gx[k][i] sum_j Gy[l][j] f[i][j]
      double HYs[Q], HYb[Q];
#pragma unroll
      for (int i = 0; i < Q1; ++i)
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          double h = 0.0, hb = 0.0;
#pragma unroll
          for (int j = 0; j < Q1; ++j) h = fma(Gy[l * Q1 + j], f[i * Q1 + j], h);
#pragma unroll
          for (int kk = 0; kk < Q1; ++kk) hb = fma(Gx[kk * Q1 + i], ab[kk * Q1 + l], hb);
          HYs[i * Q1 + l] = h;
          HYb[i * Q1 + l] = hb;
        }
#pragma unroll
      for (int i = 0; i < Q1; ++i)
#pragma unroll
        for (int j = 0; j < Q1; ++j) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < Q1; ++l) t = fma(Gy[l * Q1 + j], HYb[i * Q1 + l], t);
          atomicAdd(&A.af_in[(size_t)(i * Q1 + j) * plane + src], t);
        }
      // source gauge: z = (s_s c + u_s - u_B) / s_B
      double zsx = 0.0, zsy = 0.0, zsc = 0.0;
#pragma unroll
      for (int i = 0; i < Q1; ++i) {
        double t = 0.0;
#pragma unroll
        for (int kk = 0; kk < Q1; ++kk) {
          double rb = 0.0;
#pragma unroll
          for (int l = 0; l < Q1; ++l) rb = fma(ab[kk * Q1 + l], HYs[i * Q1 + l], rb);
          t = fma(rb, dGx[kk * Q1 + i], t);
        }
        zsx += t;
        zsc = fma(t, L::c(i), zsc);
      }
#pragma unroll
      for (int j = 0; j < Q1; ++j) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          double rb = 0.0;
#pragma unroll
          for (int i = 0; i < Q1; ++i) rb = fma(HYb[i * Q1 + l], f[i * Q1 + j], rb);
          t = fma(rb, dGy[l * Q1 + j], t);
        }
        zsy += t;
        zsc = fma(t, L::c(j), zsc);
      }
      atomicAdd(&A.ag_in[src], zsx * inv_sB);
      atomicAdd(&A.ag_in[plane + src], zsy * inv_sB);
      atomicAdd(&A.ag_in[2 * plane + src], zsc * inv_sB * L::inv_TL / (2.0 * ss));
    }
    __syncthreads();  // LDS of this tile is free
  }  // tile loop

  // d/dtau of the block's tiles (every lane of a node holds it)
  if (YS > 1 && (tid & (YS - 1))) tau_bar = 0.0;
  if (A.adj_tau) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) tau_bar += __shfl_xor(tau_bar, off);
    if ((tid & 63) == 0 && tau_bar != 0.0) atomicAdd(A.adj_tau, tau_bar);
  }
  // the last block out resets the queue for the next launch on the stream
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(&A.queue->done, 1u) == gridDim.x - 1) {
      atomicExch(&A.queue->next, 0u);
      atomicExch(&A.queue->done, 0u);
    }
  }
}

__global__ void k_zero_f64(double* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Adjoint tiles, halo 4, 256 threads.  YS = 1: 16 x 16 nodes, one lane each
// (24 x 24 window, two FP64 plane sets: 144 KiB of LDS, one block per CU).
// YS = 2: 16 x 8 nodes, two lanes each (24 x 16 window, 96 KiB); YS = 4:
// 16 x 4 nodes, four lanes each (24 x 12 window): less serial work per lane,
// for grids too small to fill the device with one lane per node.
// Persistent grid: one block per resident slot, at most one per tile.
template <int Q1, class FT, int YS>
hipError_t launch_adjoint_ys(const AdjArgs& a, hipStream_t s) {
  constexpr int TX = 16, TY = 16 / YS, H = 4;
  constexpr int kMaxDev = 64;
  static int resident[kMaxDev] = {0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  if (resident[dev] == 0) {
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&k_step_adjoint<Q1, FT, TX, TY, H, YS>),
        TX * TY * YS, 0);
    if (e != hipSuccess) return e;
    resident[dev] = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  }
  const long long tiles = (long long)((a.nx + TX - 1) / TX) * ((a.ny + TY - 1) / TY);
  const int nblk = (int)(tiles < resident[dev] ? tiles : resident[dev]);
  hipLaunchKernelGGL((k_step_adjoint<Q1, FT, TX, TY, H, YS>), dim3(nblk), dim3(TX * TY * YS), 0,
                     s, a);
  return hipGetLastError();
}

// Lanes per node from the grid: four while the one-lane tiles would not give
// every other CU one, two while they would not give every CU two
// (POND_ADJOINT_LANES = 1, 2 or 4 forces the choice, for tests).
template <int Q1, class FT>
hipError_t launch_adjoint_t(const AdjArgs& a, hipStream_t s) {
  if constexpr (Q1 % 2 == 0) {
    const char* env = getenv("POND_ADJOINT_LANES");
    const int forced = env ? atoi(env) : 0;
    if (forced == 2) return launch_adjoint_ys<Q1, FT, 2>(a, s);
    if (forced == 4) return launch_adjoint_ys<Q1, FT, 4>(a, s);
    if (forced != 1) {
      int dev = 0, cus = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      const long long tiles1 = (long long)((a.nx + 15) / 16) * ((a.ny + 15) / 16);
      if (2 * tiles1 < cus) return launch_adjoint_ys<Q1, FT, 4>(a, s);
      if (tiles1 < 2LL * cus) return launch_adjoint_ys<Q1, FT, 2>(a, s);
    }
  }
  return launch_adjoint_ys<Q1, FT, 1>(a, s);
}

}  // namespace

hipError_t launch_adjoint(const pond_config& c, const void* f_in, const double* g_in,
                          const uint8_t* iters, const double* tape, const double* tape_f,
                          int tape_slots, const double* adj_f_out, const double* adj_g_out,
                          double* adj_f_in, double* adj_g_in, double* adj_tau, TileQueue* queue,
                          hipStream_t s) {
  const size_t plane = (size_t)c.nx * c.ny;
  const size_t nf = plane * c.q1d * c.q1d, ng = plane * 3;
  hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, adj_f_in, nf);
  hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, adj_g_in, ng);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  AdjArgs a;
  a.nx = c.nx;
  a.ny = c.ny;
  a.bc_x = c.bc_x;
  a.bc_y = c.bc_y;
  a.seed_mode = c.seed_mode;
  a.isothermal = c.isothermal;
  a.tau = c.tau;
  a.f_in = f_in;
  a.g_in = g_in;
  a.iters = iters;
  a.tape = tape;
  a.tape_f = tape_f;
  a.tape_slots = tape_slots;
  a.af_out = adj_f_out;
  a.ag_out = adj_g_out;
  a.af_in = adj_f_in;
  a.ag_in = adj_g_in;
  a.adj_tau = adj_tau;
  a.queue = queue;
  const bool f64 = c.precision == POND_F64;
  if (c.q1d == 4) return f64 ? launch_adjoint_t<4, double>(a, s) : launch_adjoint_t<4, float>(a, s);
  return f64 ? launch_adjoint_t<3, double>(a, s) : launch_adjoint_t<3, float>(a, s);
}

}  // namespace pond
