// The fused PonD time step on gfx950: propagation with the predictor-corrector
// gauge iteration (eqs. 6-16, App. E), regauge and BGK collision (eqs. 17-18).
//
// Mapping.  One lane owns one node; a wave covers a 32 x 2 tile of nodes.
//
// Common-frame halo window.  A block of TX x TY nodes stages a
// (TX + 2H) x (TY + 2H) window of the state at t - dt in LDS, placed around the
// stencils of the block's seed gauges (a uniform drift shifts the window
// instead of widening it).  While staging, every window node's populations are
// moved from the node's own gauge into one reference gauge lambda_B of the
// block (the mean seed gauge) by eq. (4).  Transfer matrices compose
// (G_{B->n} G_{s->B} = G_{s->n}), so inside the pass loop the transform of a
// collocation point s into the node's gauge lambda_n is G_{B->n} applied to
// the staged f^B_s: the per-axis factors of G_{B->n} are built once per node
// and pass.  A wave walks the union of its lanes' stencil columns (relative
// to each lane's node); per y speed a column's four rows are read from LDS,
// contracted with the y row of G_{B->n} and summed with their y weights, and
// the four x speeds share the result.  A collocation point outside the window
// is read from HBM and transformed directly with G_{s->n}.  After staging the
// lanes iterate independently up to the bulk-pass cap; nodes still iterating
// then go to a list that the block's 16-lane groups finish (the tail).
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>

#include "pond_device.hpp"
#include "pond_internal.hpp"

// A wave's node tile is 32 x 2: the lanes of a wave read a collocation point
// from 32 consecutive window columns of two rows, free of LDS bank conflicts
// (8 x 8 tiles spend about half of the LDS cycles in conflicts).
constexpr int kWaveTX = 32;

namespace pond {
namespace {

template <int Q1, class FT, int TX, int TY, int H>
struct TileShape {
  static constexpr int WX = TX + 2 * H;
  static constexpr int WY = TY + 2 * H;
  static constexpr int WN = WX * WY;
  static constexpr int NT = TX * TY;
  static constexpr int NW = NT / 64;
  static constexpr size_t lds_bytes = (size_t)Win<Q1, FT, WN>::size * sizeof(FT);
  static constexpr int WTX = kWaveTX;
  static constexpr int WTY = 64 / WTX;  // wave tile
  static_assert(TX % WTX == 0 && TY % WTY == 0, "waves tile the block");
  static_assert(lds_bytes + 1024 <= 160 * 1024, "window exceeds the 160 KiB LDS of a CU");
};

// Floor of a departure coordinate as int, saturated so that absurd gauges
// (non-finite or |x| > 1e9) cannot overflow the conversion.
__device__ __forceinline__ int sat_floor(double x) {
  x = fmin(fmax(x, -1.0e9), 1.0e9);
  return isfinite(x) ? int(floor(x)) : 0;
}

// Block reduction: minimum of four ints, sum of four doubles.
template <int NW>
__device__ __forceinline__ void block_reduce(int v[4], double a[4], int* s_i, double* s_d) {
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

// Row of G_{B->n} (or any transfer row) rounded to the arithmetic type.
template <int Q1, class FT>
__device__ __forceinline__ void row_to(const LagRow& P, double r, double d, FT* out) {
  double row[Q1];
  transfer_row_coef<Q1>(P, r, d, row);
#pragma unroll
  for (int q = 0; q < Q1; ++q) out[q] = FT(row[q]);
}

// Speed and Lagrange coefficients for a lane-varying index.
template <int Q1>
__device__ __forceinline__ double speed_lane(int i) {
  double c = Lat<Q1>::c(0);
#pragma unroll
  for (int k = 1; k < Q1; ++k) c = i == k ? Lat<Q1>::c(k) : c;
  return c;
}
template <int Q1>
__device__ __forceinline__ LagRow lag_row_lane(int k) {
  constexpr LagCoef<Q1> C{};
  LagRow P{C.v[0][0], C.v[0][1], C.v[0][2], C.v[0][3]};
#pragma unroll
  for (int kk = 1; kk < Q1; ++kk) {
    const bool t = k == kk;
    P.l0 = t ? C.v[kk][0] : P.l0;
    P.l1 = t ? C.v[kk][1] : P.l1;
    P.l2 = t ? C.v[kk][2] : P.l2;
    P.l3 = t ? C.v[kk][3] : P.l3;
  }
  return P;
}

// a4 for a collocation point read from HBM: the direct transform G_{s->n}
// with rows Pi, Pj at the node gauge (ux, uy, 1/inv_s).
template <int Q1, class FT>
__device__ __forceinline__ FT pair_value_hbm(const StepArgs& A, int gx, int gy, const LagRow& Pi,
                                             const LagRow& Pj, double ux, double uy, double inv_s) {
  using L = Lat<Q1>;
  const size_t plane = (size_t)A.nx * A.ny;
  const FT* __restrict__ fin = static_cast<const FT*>(A.f_in);
  const size_t src = (size_t)wrap_index(gy, A.ny, A.bc_y) * A.nx + wrap_index(gx, A.nx, A.bc_x);
  const double r = sqrt(A.g_in[2 * plane + src] * L::inv_TL) * inv_s;
  FT f[Q1 * Q1];
#pragma unroll
  for (int p = 0; p < Q1 * Q1; ++p) f[p] = fin[(size_t)p * plane + src];
  double gxr[Q1], gyr[Q1];
  transfer_row_coef<Q1>(Pi, r, (A.g_in[src] - ux) * inv_s, gxr);
  transfer_row_coef<Q1>(Pj, r, (A.g_in[plane + src] - uy) * inv_s, gyr);
  FT t = FT(0);
#pragma unroll
  for (int ip = 0; ip < Q1; ++ip) {
    FT h = FT(0);
#pragma unroll
    for (int jp = 0; jp < Q1; ++jp) h += FT(gyr[jp]) * f[ip * Q1 + jp];
    t += FT(gxr[ip]) * h;
  }
  return t;
}

// a4: [G_{lambda_s -> lambda_n} f_s]_(i,j) for the collocation point (gx, gy):
// G_{B->n} rows (gbx, gby) on the staged window, or the direct transform of
// the HBM state outside it (rows Pi, Pj at the node gauge (ux, uy, 1/inv_s)).
template <int Q1, class FT, int WX, int WY, int WN>
__device__ __forceinline__ FT pair_value(const StepArgs& A, const FT* s_f, int wx0, int wy0, int gx,
                                         int gy, const FT* gbx, const FT* gby, const LagRow& Pi,
                                         const LagRow& Pj, double ux, double uy, double inv_s) {
  const int lx = gx - wx0, ly = gy - wy0;
  FT t = FT(0);
  if ((unsigned)lx < (unsigned)WX && (unsigned)ly < (unsigned)WY) {
    using W = Win<Q1, FT, WN>;
    const int k = ly * WX + lx;
    FT f[Q1 * Q1];
    W::load(s_f, k * W::G, k * W::G + W::NGH * W::GS, f);
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) {
      FT h = FT(0);
#pragma unroll
      for (int jp = 0; jp < Q1; ++jp) h += gby[jp] * f[ip * Q1 + jp];
      t += gbx[ip] * h;
    }
  } else {
    t = pair_value_hbm<Q1, FT>(A, gx, gy, Pi, Pj, ux, uy, inv_s);
  }
  return t;
}

// a4 + a5 for one collocation point (gx, gy) of a column, y weight aym:
// on the LDS window the y contraction with the G_{B->n} row gby is weighted
// and summed over the column's rows into hc (the x rows of G_{B->n} are
// applied once per column by the caller, they do not depend on the row);
// outside it the point is read from HBM, transformed directly with the rows
// of G_{s->n} (which depend on the point's own gauge) and added to acc with
// the x weights wx.
template <int Q1, class FT, int WX, int WY, int WN>
__device__ __forceinline__ void column_point(const StepArgs& A, const FT* s_f, int wx0, int wy0,
                                             int gx, int gy, bool need, FT aym, const FT* wx,
                                             const FT* gby, const LagRow& Pj, double ux,
                                             double uy, double inv_s, FT* hc, FT* acc) {
  using L = Lat<Q1>;
  const int lx = gx - wx0, ly = gy - wy0;
  if (need && (unsigned)lx < (unsigned)WX && (unsigned)ly < (unsigned)WY) {
    using W = Win<Q1, FT, WN>;
    const int k = ly * WX + lx;
    // all loads first, so that they are in flight together
    FT f[Q1 * Q1];
    W::load(s_f, k * W::G, k * W::G + W::NGH * W::GS, f);
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) {
      FT v = FT(0);
#pragma unroll
      for (int jp = 0; jp < Q1; ++jp) v += gby[jp] * f[ip * Q1 + jp];
      hc[ip] += aym * v;
    }
  } else if (need) {
    const size_t plane = (size_t)A.nx * A.ny;
    const FT* __restrict__ fin = static_cast<const FT*>(A.f_in);
    const size_t src = (size_t)wrap_index(gy, A.ny, A.bc_y) * A.nx + wrap_index(gx, A.nx, A.bc_x);
    FT f[Q1 * Q1];
#pragma unroll
    for (int p = 0; p < Q1 * Q1; ++p) f[p] = fin[(size_t)p * plane + src];
    const double r = sqrt(A.g_in[2 * plane + src] * L::inv_TL) * inv_s;
    const double dx = (A.g_in[src] - ux) * inv_s;
    double gyr[Q1];
    transfer_row_coef<Q1>(Pj, r, (A.g_in[plane + src] - uy) * inv_s, gyr);
    FT h[Q1];
#pragma unroll
    for (int ip = 0; ip < Q1; ++ip) {
      FT v = FT(0);
#pragma unroll
      for (int jp = 0; jp < Q1; ++jp) v += FT(gyr[jp]) * f[ip * Q1 + jp];
      h[ip] = v;
    }
#pragma unroll
    for (int i = 0; i < Q1; ++i) {
      double gxr[Q1];
      transfer_row<Q1>(i, r, dx, gxr);
      FT v = FT(0);
#pragma unroll
      for (int ip = 0; ip < Q1; ++ip) v += FT(gxr[ip]) * h[ip];
      acc[i] += (wx[i] * aym) * v;
    }
  }
}

// a4 + a5 on the LDS window for the four rows of one stencil column and JB y
// speeds, the lane's whole column inside the window for each (node index
// k[b] of speed b's first row): the y contractions with the G_{B->n} rows
// gby[b], weighted by ayw[b] and summed into hc[b].  Row m of every speed is
// taken before row m + 1 (the speeds' rows are independent, so their reads
// are in flight together).  The second base of the reads is opaque to the
// optimiser, so that every read takes its group and row from the instruction
// offset.  In FP64 a scheduling barrier keeps each row's reads with the row:
// left free, the scheduler hoists the reads of all four rows and holds them
// at once, which measured slower; FP32 gains from it.
template <int Q1, int JB, class FT, int WX, int WN>
__device__ __forceinline__ void window_columns(const FT* s_f, const int* k, const FT (*ayw)[4],
                                               const FT (*gby)[Q1], FT (*hc)[Q1]) {
  using W = Win<Q1, FT, WN>;
  constexpr int Q = Q1 * Q1;
  int e[JB], eh[JB];
#pragma unroll
  for (int b = 0; b < JB; ++b) {
    e[b] = k[b] * W::G;
    eh[b] = e[b] + W::NGH * W::GS;
    asm volatile("" : "+v"(eh[b]));
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int b = 0; b < JB; ++b) {
      FT f[Q];
      W::load(s_f, e[b] + m * WX * W::G, eh[b] + m * WX * W::G, f);
#pragma unroll
      for (int ip = 0; ip < Q1; ++ip) {
        FT v = FT(0);
#pragma unroll
        for (int jp = 0; jp < Q1; ++jp) v += gby[b][jp] * f[ip * Q1 + jp];
        hc[b][ip] += ayw[b][m] * v;
      }
    }
    if constexpr (sizeof(FT) == 8) {
      if (m < 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

constexpr int kContinue = 0, kDone = 1, kBad = 2;

// a6 + a7: corrector gauge from the moments of the pass (peculiar frame of
// the pass gauge (ux, uy, s)) and the App. E test.
template <int Q1>
__device__ __forceinline__ int corrector(const StepArgs& A, double s, double ux, double uy, double T,
                                         double rho, double mx, double my, double e2,
                                         unsigned passes, double& rho1, double& ux1, double& uy1,
                                         double& T1, unsigned& flags) {
  using L = Lat<Q1>;
  const double dux = s * mx / rho, duy = s * my / rho;
  rho1 = rho;
  ux1 = ux + dux;
  uy1 = uy + duy;
  T1 = A.isothermal ? T : 0.5 * (s * s * e2 / rho - (dux * dux + duy * duy));
  if (!(rho1 > 0.0) || !(T1 > 0.0) || !isfinite(rho1) || !isfinite(ux1) || !isfinite(uy1) ||
      !isfinite(T1))
    return kBad;
  if (A.fixed_iter > 0) return (int)passes >= A.fixed_iter ? kDone : kContinue;
  bool conv = fabs(ux1 - ux) < A.eps_abs + A.eps_rel * fabs(ux1) &&
              fabs(uy1 - uy) < A.eps_abs + A.eps_rel * fabs(uy1);
  if (!A.isothermal) {
    const double s1 = sqrt(T1 * L::inv_TL);
    conv = conv && fabs(s1 - s) < A.eps_abs + A.eps_rel * fabs(s1);
  }
  if (conv) return kDone;
  if ((int)passes >= A.max_iter) {
    flags |= POND_ITERS_NONCONVERGED;
    return kDone;
  }
  return kContinue;
}

// NaN output of a node whose corrector moments were not physical.
template <int Q1, class FT>
__device__ __forceinline__ void store_bad(const StepArgs& A, FT* fout, size_t plane, size_t node,
                                          int p0, int p1) {
  const double qnan = __builtin_nan("");
  for (int p = p0; p < p1; ++p) fout[(size_t)p * plane + node] = FT(qnan);
  if (p0 == 0) {
    A.g_out[node] = qnan;
    A.g_out[plane + node] = qnan;
    A.g_out[2 * plane + node] = qnan;
  }
}

// ---- tail: finishing the block's unconverged nodes with groups of 16 lanes ----
// Lane p of a group owns population (i, j) = (p / q, p % q) of the group's
// node.  The group reduces the corrector moments with butterfly shuffles and
// gathers the populations of the regauge with shuffles.  Every lane of the wave
// runs this together (the shuffles span the wave); each group takes the next
// node of the block's list (count entries, the next one at *s_next) as soon
// as its own node has finished, so the groups of a wave do not wait for the
// wave's slowest node.  Collocation points come from the block's LDS window
// (pair_value, HBM outside it).  A node's final pass count raises the pass
// maximum of the wave that deferred it (s_wmax) and, when the step keeps
// statistics, its bin of the block's pass histogram s_hist.
template <int Q1, class FT, int WX, int WY, int WN, int TX, int WTX, int WTY>
__device__ __forceinline__ void tail_wave(const StepArgs& A, const FT* s_f, int wx0, int wy0,
                                          double uxB, double uyB, double sB, int bx0, int by0,
                                          unsigned count, const unsigned* s_list,
                                          unsigned* s_next, unsigned* s_wmax, unsigned* s_hist,
                                          unsigned long long& c_nc, unsigned long long& c_nb,
                                          unsigned long long& c_sp, unsigned long long& c_mp) {
  constexpr int Q = Q1 * Q1;
  using L = Lat<Q1>;
  const size_t plane = (size_t)A.nx * A.ny;
  FT* __restrict__ fout = static_cast<FT*>(A.f_out);
  int lane = threadIdx.x & 63;
  // Opaque to the optimiser: keeps the per-lane rows below from being hoisted
  // out of the block's tile loop (where they would stay live through the bulk
  // passes and cost registers).
  asm volatile("" : "+v"(lane));
  const int p = lane & 15;
  const bool pop = p < Q;
  const int pi = pop ? p / Q1 : 0, pj = pop ? p % Q1 : 0;
  const double ci = speed_lane<Q1>(pi), cj = speed_lane<Q1>(pj);
  const LagRow Pi = lag_row_lane<Q1>(pi), Pj = lag_row_lane<Q1>(pj);
  const int base = lane & ~15;
  bool has = false, exhausted = false, gdone = true, bad = false;
  unsigned passes = 0, flags = 0;
  int X = 0, Y = 0, lw = 0;
  size_t node = 0;
  FT fij = FT(0);
  double ux = 0.0, uy = 0.0, T = L::TL;
  double rho1 = 0.0, ux1 = 0.0, uy1 = 0.0, T1 = L::TL;
  for (;;) {
    // a group without a node takes the next entry of the list; a deferred
    // node's gauge went through its output gauge slot (read with
    // L1-bypassing loads)
    if (!has && !exhausted) {
      unsigned e = 0;
      if (p == 0) e = atomicAdd(s_next, 1u);
      e = __shfl(e, base);
      if (e < count) {
        const unsigned ent = s_list[e];
        const int ltid = (int)(ent & 0xFFFF);
        lw = ltid >> 6;
        const int ll = ltid & 63;
        X = bx0 + (lw % (TX / WTX)) * WTX + (ll % WTX);
        Y = by0 + (lw / (TX / WTX)) * WTY + (ll / WTX);
        node = (size_t)Y * A.nx + X;
        passes = ent >> 16;
        flags = 0;
        bad = false;
        gdone = false;
        has = true;
        ux = __hip_atomic_load(&A.g_out[node], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uy = __hip_atomic_load(&A.g_out[plane + node], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        T = __hip_atomic_load(&A.g_out[2 * plane + node], __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
        rho1 = 0.0;
        ux1 = ux;
        uy1 = uy;
        T1 = T;
      } else {
        exhausted = true;
      }
    }
    if (__all(!has)) break;
    // one predictor-corrector pass for the groups still iterating
    double s = 0.0;
    const bool iter = has && !gdone;
    if (iter) {
      ++passes;
      s = sqrt(T * L::inv_TL);
      const double inv_s = 1.0 / s;
      const double rB = sB * inv_s;
      const double xd = double(X) - (s * ci + ux), yd = double(Y) - (s * cj + uy);
      const double fl = floor(xd), fly = floor(yd);
      double ax[4], ay[4];
      interp_weights(xd - (fl - 1.0), ax);
      interp_weights(yd - (fly - 1.0), ay);
      const int x0 = sat_floor(fl) - 1, y0 = sat_floor(fly) - 1;
      FT gbx[Q1], gby[Q1];
      row_to<Q1, FT>(Pi, rB, (uxB - ux) * inv_s, gbx);
      row_to<Q1, FT>(Pj, rB, (uyB - uy) * inv_s, gby);
      FT acc = FT(0);
      using W = Win<Q1, FT, WN>;
      const int ly0 = y0 - wy0;
      const bool rows_in = (unsigned)ly0 <= (unsigned)(WY - 4);
#pragma unroll 1
      for (int n = 0; n < 4; ++n) {
        const double axn = n == 0 ? ax[0] : n == 1 ? ax[1] : n == 2 ? ax[2] : ax[3];
        FT col = FT(0);
        const int lx = x0 + n - wx0;
        if (rows_in && (unsigned)lx < (unsigned)WX) {
          // the column's four rows inside the window: one straight run
          const int e = (ly0 * WX + lx) * W::G;
          int eh = e + W::NGH * W::GS;
          asm volatile("" : "+v"(eh));
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            FT f[Q];
            W::load(s_f, e + m * WX * W::G, eh + m * WX * W::G, f);
            FT t = FT(0);
#pragma unroll
            for (int ip = 0; ip < Q1; ++ip) {
              FT h = FT(0);
#pragma unroll
              for (int jp = 0; jp < Q1; ++jp) h += gby[jp] * f[ip * Q1 + jp];
              t += gbx[ip] * h;
            }
            col += FT(ay[m]) * t;
          }
        } else {
#pragma unroll
          for (int m = 0; m < 4; ++m)
            col += FT(ay[m]) * pair_value<Q1, FT, WX, WY, WN>(A, s_f, wx0, wy0, x0 + n, y0 + m,
                                                              gbx, gby, Pi, Pj, ux, uy, inv_s);
        }
        acc += FT(axn) * col;
      }
      fij = pop ? acc : FT(0);
    }
    // a6 over the 16 lanes of the group (compensated pairwise sums; in
    // FP32 the products with the speeds are split exactly as in the one-lane
    // form, and the speeds are held as FP32 pairs)
    const bool live = iter && pop;
    FT v[4], er[4];
    {
#pragma clang fp contract(off)
      v[0] = live ? fij : FT(0);
      v[1] = live ? FT(ci) * fij : FT(0);
      v[2] = live ? FT(cj) * fij : FT(0);
      v[3] = live ? FT(ci * ci + cj * cj) * fij : FT(0);
      er[0] = er[1] = er[2] = er[3] = FT(0);
      if constexpr (sizeof(FT) == 4) {
        const double cv[3] = {ci, cj, ci * ci + cj * cj};
#pragma unroll
        for (int k = 1; k < 4; ++k) {
          const float hi = split_hi(cv[k - 1]), lo = split_lo(cv[k - 1]);
          er[k] = live ? fmaf(hi, fij, -v[k]) + lo * fij : 0.0f;
        }
      }
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const FT ov = __shfl_xor(v[k], off), oe = __shfl_xor(er[k], off);
          const FT t = v[k] + ov;
          const FT bp = t - v[k];
          er[k] += oe + ((v[k] - (t - bp)) + (ov - bp));
          v[k] = t;
        }
      }
    }
    if (iter) {
      const int verdict = corrector<Q1>(A, s, ux, uy, T, double(v[0]) + double(er[0]),
                                        double(v[1]) + double(er[1]), double(v[2]) + double(er[2]),
                                        double(v[3]) + double(er[3]), passes, rho1, ux1, uy1, T1,
                                        flags);
      if (verdict != kBad && A.tape && p == 0) {
        const size_t t = (size_t)passes * 4 * plane + node;
        A.tape[t] = ux1;
        A.tape[t + plane] = uy1;
        A.tape[t + 2 * plane] = T1;
        A.tape[t + 3 * plane] = rho1;
      }
      if (verdict == kBad) {
        bad = true;
        gdone = true;
      } else if (verdict == kDone) {
        gdone = true;
      } else {
        ux = ux1;
        uy = uy1;
        T = T1;
      }
    }
    // a8 + a9 + a10 for the groups whose node has finished; every lane
    // joins the shuffles
    if (!__any(has && gdone)) continue;
    FT fr = FT(0);
    {
      const double s0 = sqrt(T * L::inv_TL), s1 = sqrt(T1 * L::inv_TL);
      const double inv_s1 = 1.0 / s1, r = s0 * inv_s1;
      double ry[Q1], rx[Q1];
      transfer_row_coef<Q1>(Pj, r, (uy - uy1) * inv_s1, ry);  // row l = pj of Ry
      transfer_row_coef<Q1>(Pi, r, (ux - ux1) * inv_s1, rx);  // row k = pi of Rx
      FT h = FT(0);  // Hm(pi, l = pj) = sum_j Ry[l][j] F(pi, j)
#pragma unroll
      for (int jj = 0; jj < Q1; ++jj) h += FT(ry[jj]) * __shfl(fij, base + pi * Q1 + jj);
#pragma unroll
      for (int ii = 0; ii < Q1; ++ii) fr += FT(rx[ii]) * __shfl(h, base + ii * Q1 + pj);
    }
    if (has && gdone) {
      if (bad) {
        if (pop) store_bad<Q1, FT>(A, fout, plane, node, p, p + 1);
        flags |= POND_ITERS_BAD;
      } else if (pop) {
        if (A.tape_f) A.tape_f[(size_t)p * plane + node] = double(fij);
        const FT feq = FT(rho1 * (L::w(pi) * L::w(pj)));
        fout[(size_t)p * plane + node] = fr + FT(1.0 / A.tau) * (feq - fr);
        if (p == 0) {
          A.g_out[node] = ux1;
          A.g_out[plane + node] = uy1;
          A.g_out[2 * plane + node] = T1;
        }
      }
      if (p == 0) {
        if (A.iters) A.iters[node] = (uint8_t)((passes & POND_ITERS_MASK) | flags);
        atomicMax(&s_wmax[lw], passes);
        if (A.counters) atomicAdd(&s_hist[passes & POND_ITERS_MASK], 1u);
        c_nc += (flags & POND_ITERS_NONCONVERGED) ? 1 : 0;
        c_nb += (flags & POND_ITERS_BAD) ? 1 : 0;
        c_sp += passes;
        c_mp = passes > c_mp ? passes : c_mp;
      }
    }
    if (has && gdone) has = false;
  }
}

// Tile cost keys: the sum over the tile's waves of the most passes a node of
// the wave took.  One key bin per thread of the block: NT / 64 waves of at
// most 63 passes keep the keys below NT.
template <int NT>
constexpr unsigned kKeyBins = NT;

// Counting sort of the tiles by key, largest first, into order[] (one block,
// NT threads, 3 NT words of LDS).  Tiles with equal keys land in any
// order; the step's results do not depend on the order of its tiles.
template <int NT>
__device__ void order_tiles(const uint16_t* keys, unsigned* order, unsigned ntiles,
                            unsigned* lds) {
  static_assert(NT >= (int)kKeyBins<NT>, "one thread per key bin");
  unsigned* hist = lds;
  unsigned* scan = lds + kKeyBins<NT>;
  unsigned* start = lds + 2 * kKeyBins<NT>;
  const int tid = threadIdx.x;
  if (tid < (int)kKeyBins<NT>) hist[tid] = 0u;
  __syncthreads();
  for (unsigned t = tid; t < ntiles; t += NT) atomicAdd(&hist[keys[t]], 1u);
  __syncthreads();
  // inclusive scan over bins in decreasing key order (Hillis-Steele)
  unsigned v = tid < (int)kKeyBins<NT> ? hist[kKeyBins<NT> - 1 - tid] : 0u;
  for (unsigned off = 1; off < kKeyBins<NT>; off <<= 1) {
    if (tid < (int)kKeyBins<NT>) scan[tid] = v;
    __syncthreads();
    if (tid < (int)kKeyBins<NT> && (unsigned)tid >= off) v += scan[tid - off];
    __syncthreads();
  }
  if (tid < (int)kKeyBins<NT>) start[kKeyBins<NT> - 1 - tid] = v - hist[kKeyBins<NT> - 1 - tid];
  __syncthreads();
  for (unsigned t = tid; t < ntiles; t += NT) order[atomicAdd(&start[keys[t]], 1u)] = t;
}

// Waves per SIMD the registers are sized for (the launch bound's second
// argument): two (256 VGPRs: one 8-wave D2Q16 FP64 block or two 4-wave
// blocks per CU); FP32-mixed D2Q9 three (168 VGPRs, 33 spilled, three
// blocks per CU, measured 8-10 % faster than two; D2Q9 FP64 at three spills
// 139 registers).
template <int Q1, class FT>
constexpr int kStepWavesPerSIMD = sizeof(FT) == 4 && Q1 == 3 ? 3 : 2;

template <int Q1, class FT, int TX, int TY, int H>
__global__ void __launch_bounds__(TX * TY, (kStepWavesPerSIMD<Q1, FT>))
k_step(StepArgs A) {
  constexpr int Q = Q1 * Q1;
  using L = Lat<Q1>;
  using TS = TileShape<Q1, FT, TX, TY, H>;
  constexpr int WX = TS::WX, WY = TS::WY, WN = TS::WN, NT = TS::NT;
  __shared__ __align__(16) FT s_f[Win<Q1, FT, WN>::size];
  __shared__ int s_ri[4 * TS::NW];
  __shared__ double s_rd[4 * TS::NW];
  __shared__ unsigned s_list[NT];  // deferred nodes: local index | passes << 16
  __shared__ unsigned s_tail[2];   // list length, next entry to take
  __shared__ unsigned s_tile;
  __shared__ unsigned s_g;             // queue position of the current tile
  __shared__ unsigned s_pref, s_pref_tile;  // next tile taken ahead (s_pref: position or ~0)
  __shared__ unsigned s_arrive;        // waves done with the bulk passes of the tile
  // seed gauges (u_x, u_y, T rows of the tile) of the tile taken ahead, and that tile
  __shared__ __align__(16) double s_seed[Q1 == 4 && sizeof(FT) == 8 ? 3 * TY * TX : 2];
  __shared__ unsigned s_seed_tile;
  __shared__ unsigned s_last;          // this block is the last one out
  __shared__ unsigned s_wmax[TS::NW];  // per wave: maximum passes of its nodes
  __shared__ unsigned s_hist[POND_ITERS_MASK + 1];  // nodes per pass count (statistics)

  const int tid = threadIdx.x;
  // D2Q16 blocks take their next tile ahead (below; measured neutral to
  // slower for D2Q9), in FP64 with its seed gauges (1-2 % slower in
  // FP32-mixed)
  constexpr bool kTakeAhead = Q1 == 4;
  constexpr bool kStageSeeds = kTakeAhead && sizeof(FT) == 8;
  const int ntx = (A.nx + TX - 1) / TX;
  const unsigned ntiles = (unsigned)ntx * (unsigned)((A.ny + TY - 1) / TY);
  const bool keyed = A.tile_keys && ntiles <= A.tile_cap;  // tile arrays fit this grid
  if (tid < TS::NW) s_wmax[tid] = 0u;
  if (tid <= POND_ITERS_MASK) s_hist[tid] = 0u;
  if (tid == 0) {
    s_pref = ~0u;
    s_seed_tile = ~0u;
  }

  // Persistent blocks: each block takes tiles from the queue until it is
  // empty, so the cost spread between tiles (passes cluster along fronts) is
  // balanced over all CUs without the hardware dispatcher.
  for (;;) {
    if (tid == 0) {
      if (kTakeAhead && s_pref != ~0u) {  // taken while the previous tile finished
        s_g = s_pref;
        s_tile = s_pref_tile;
        s_pref = ~0u;
      } else {
        const unsigned g = atomicAdd(&A.queue->next, 1u);
        s_g = g;
        s_tile = (keyed && A.tile_order && g < ntiles) ? A.tile_order[g] : g;
      }
    }
    if (tid < 2) s_tail[tid] = 0u;
    if (tid == 2) s_arrive = 0u;
    __syncthreads();
    const unsigned tile = s_tile;
    if (tile >= ntiles) break;
    const int ty = (int)(tile / (unsigned)ntx), tx = (int)tile - ty * ntx;
    const int bx0 = tx * TX, by0 = ty * TY;
    // thread index made opaque per tile, so that nothing derived from it is
    // hoisted out of the tile loop and held in registers through the passes
    int tl = tid;
    asm volatile("" : "+v"(tl));
    const int wave = tl >> 6, lane = tl & 63;
    constexpr int WTX = TS::WTX, WTY = TS::WTY;
    const int X = bx0 + (wave % (TX / WTX)) * WTX + (lane % WTX);
    const int Y = by0 + (wave / (TX / WTX)) * WTY + (lane / WTX);
    const bool active = (X < A.nx) && (Y < A.ny);
    const size_t plane = (size_t)A.nx * A.ny;
    const FT* __restrict__ fin = static_cast<const FT*>(A.f_in);
    const double* __restrict__ gin = A.g_in;

    // a1: seed gauge (eqs. 7-8) or the alternative seeds.
    double ux = 0.0, uy = 0.0, T = L::TL;
    size_t node = 0;
    const bool seeds_staged = kStageSeeds && s_seed_tile == tile;
    if (active) {
      node = (size_t)Y * A.nx + X;
      if (seeds_staged) {
        const int k = (Y - by0) * TX + (X - bx0);
        ux = s_seed[k];
        uy = s_seed[TY * TX + k];
        T = s_seed[2 * TY * TX + k];
      } else {
        ux = gin[node];
        uy = gin[plane + node];
        T = gin[2 * plane + node];
      }
      if (A.seed_mode == 1) {
        ux = 0.0;
        uy = 0.0;
        if (!A.isothermal) T = L::TL;
      } else if (A.seed_mode == 2) {
        ux = -ux;
        uy = -uy;
      }
      if (A.tape) {
        A.tape[node] = ux;
        A.tape[plane + node] = uy;
        A.tape[2 * plane + node] = T;
      }
    }

    // ---- window placement and reference gauge from the seed gauges ----
    int wx0, wy0;
    double uxB, uyB, sB;
    {
      int v[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
      double a[4] = {0.0, 0.0, 0.0, 0.0};
      const double s0 = sqrt(T * L::inv_TL);
      const double sp = s0 * L::c(Q1 - 1);
      if (active && isfinite(sp) && s0 > 0.0 && isfinite(ux) && isfinite(uy) &&
          fabs(ux) < 1e9 && fabs(uy) < 1e9) {
        v[0] = sat_floor(double(X) - ux - sp) - 2;
        v[1] = -(sat_floor(double(X) - ux + sp) + 3);
        v[2] = sat_floor(double(Y) - uy - sp) - 2;
        v[3] = -(sat_floor(double(Y) - uy + sp) + 3);
        a[0] = ux;
        a[1] = uy;
        a[2] = s0;
        a[3] = 1.0;
      }
      block_reduce<TS::NW>(v, a, s_ri, s_rd);
      if (a[3] > 0.0) {
        uxB = a[0] / a[3];
        uyB = a[1] / a[3];
        sB = a[2] / a[3];
      } else {  // no usable seed in the block: any reference gauge is exact
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

#ifdef POND_LDS_POISON
    // checking build: every window value that the staging below does not
    // write reads as NaN, so a read of an unstaged value shows in the output
    for (int k = tid; k < Win<Q1, FT, WN>::size; k += NT) s_f[k] = FT(__builtin_nan(""));
    __syncthreads();
#endif
    // ---- stage the window in the reference gauge (eq. 4, G_{s->B}) ----
    {
      const double inv_sB = 1.0 / sB;
      // the reads of a thread's next window node are issued before the
      // current one is transformed, so that their latency overlaps it
      FT fn[Q];
      double gn[3];
      auto fetch = [&](int k) {
        const int wy = k / WX, wx = k - wy * WX;
        const int sx = wrap_index(wx0 + wx, A.nx, A.bc_x);
        const int sy = wrap_index(wy0 + wy, A.ny, A.bc_y);
        const size_t src = (size_t)sy * A.nx + sx;
#pragma unroll
        for (int p = 0; p < Q; ++p) fn[p] = fin[(size_t)p * plane + src];
#pragma unroll
        for (int c = 0; c < 3; ++c) gn[c] = gin[c * plane + src];
      };
      if (tid < WN) fetch(tid);
      for (int k = tid; k < WN; k += NT) {
        FT f[Q];
#pragma unroll
        for (int p = 0; p < Q; ++p) f[p] = fn[p];
        const double gux = gn[0], guy = gn[1], gT = gn[2];
        if (k + NT < WN) fetch(k + NT);
        // the transfer factors are built in FP64 and applied in the
        // arithmetic type (FP32-mixed: rounded, then FP32 contractions)
        const double ss = sqrt(gT * L::inv_TL);
        const double r = ss * inv_sB;
        double Gxd[Q], Gyd[Q];
        transfer_factor<Q1, double>(r, (gux - uxB) * inv_sB, Gxd);
        transfer_factor<Q1, double>(r, (guy - uyB) * inv_sB, Gyd);
        FT Gx[Q], Gy[Q];
#pragma unroll
        for (int p = 0; p < Q; ++p) {
          Gx[p] = FT(Gxd[p]);
          Gy[p] = FT(Gyd[p]);
        }
        FT Hm[Q];  // Hm[i][l] = sum_j Gy[l][j] f[i][j]
#pragma unroll
        for (int i = 0; i < Q1; ++i)
#pragma unroll
          for (int l = 0; l < Q1; ++l) {
            FT h = FT(0);
#pragma unroll
            for (int j = 0; j < Q1; ++j) h = fma(Gy[l * Q1 + j], f[i * Q1 + j], h);
            Hm[i * Q1 + l] = h;
          }
        using W = Win<Q1, FT, WN>;
        typename W::V tv[W::NG];  // one 16-byte LDS write per group
#pragma unroll
        for (int kk = 0; kk < Q1; ++kk)
#pragma unroll
          for (int l = 0; l < Q1; ++l) {
            FT t = FT(0);
#pragma unroll
            for (int i = 0; i < Q1; ++i) t = fma(Gx[kk * Q1 + i], Hm[i * Q1 + l], t);
            const int p = kk * Q1 + l;
            tv[p / W::G][p % W::G] = t;
          }
#pragma unroll
        for (int g = 0; g < W::NG; ++g) {
          if constexpr (W::NG * W::G > Q) {  // padding of the last group
            if (g == W::NG - 1) {
#pragma unroll
              for (int c = Q % W::G; c < W::G; ++c) tv[g][c] = FT(0);
            }
          }
          *reinterpret_cast<typename W::V*>(s_f + g * W::GS + k * W::G) = tv[g];
        }
      }
    }
    __syncthreads();

    // adaptive runs move nodes still unconverged after bulk_cap passes to the
    // block tail
    const bool capped = A.fixed_iter == 0 && A.bulk_cap > 0 && A.bulk_cap < A.max_iter;
    // step counters of this lane for the tile (its own node if finished in
    // the bulk phase, plus the nodes it finishes as a tail-group leader)
    unsigned long long c_nc = 0, c_nb = 0, c_sp = 0, c_mp = 0;
    FT* __restrict__ fout = static_cast<FT*>(A.f_out);

    unsigned passes = 0;
    unsigned flags = 0;
    bool deferred = false;
    if (active) {
      FT ft[Q];
      double ux1 = ux, uy1 = uy, T1 = T, rho1 = 0.0;
      bool bad = false;
      for (;;) {
        ++passes;
        const double s = sqrt(T * L::inv_TL);
        const double inv_s = 1.0 / s;
        // a4 (window part): G_{B->n} rows are l_k(rB c + dB) per axis.
        const double rB = sB * inv_s;
        const double dBx = (uxB - ux) * inv_s, dBy = (uyB - uy) * inv_s;

        // a2 + a3 (x axis) for every x speed: departure columns x0_i (as offsets
        // o_i = x0_i - X), weights, and the rows of G_{B->n} along x.
        int o[Q1];
        double xdv[Q1];  // departure abscissae (weights per column)
        FT gbx[Q1][Q1];
        int lo = INT_MAX, hi = INT_MIN;
        bool has = false, far = false;
#pragma unroll
        for (int i = 0; i < Q1; ++i) {
          const double xd = double(X) - (s * L::c(i) + ux);
          const double fl = floor(xd);
          xdv[i] = xd;
          o[i] = sat_floor(fl) - 1 - X;
          double row[Q1];
          transfer_row<Q1>(i, rB, dBx, row);
#pragma unroll
          for (int ip = 0; ip < Q1; ++ip) gbx[i][ip] = FT(row[ip]);
          if (isfinite(xd)) {
            lo = o[i] < lo ? o[i] : lo;
            hi = o[i] + 3 > hi ? o[i] + 3 : hi;
            has = true;
            far = far || o[i] < -kFarColumns || o[i] > kFarColumns;
          }
        }
        // A departure point further than kFarColumns nodes away (|v| dt of
        // hundreds of nodes) would stretch the wave's column walk: such a node
        // finishes in the block tail, which walks its own stencils.
        if (far) {
          --passes;
          deferred = true;
          break;
        }
        // The wave walks the union of its lanes' stencil columns (the same for
        // every y speed); every collocation point of a column is read from LDS
        // once per y speed and its y contraction is shared by the four x
        // speeds (each with its own weight, zero where the column is outside
        // that speed's stencil).
        if (!wave_column_range(lo, hi, has, lo, hi)) hi = lo - 1;
        // y speeds are taken in groups of JB (a group's rows are read
        // interleaved): D2Q16 two groups of two (measured faster than one or
        // four per group), D2Q9 one group of three.
        constexpr int JB = Q1 % 2 == 0 ? 2 : 3;
        if constexpr (sizeof(FT) == 4) {
          // FP32-mixed: one column walk for every group (a column's x weights
          // serve them all; measured faster than a walk per group)
          constexpr int NG = Q1 / JB;
          FT ayw[Q1][4];
          int y0[Q1], ly0[Q1];
          bool rows_in[Q1];
          FT gby[Q1][Q1];
          bool all_in[NG];
#pragma unroll
          for (int g = 0; g < NG; ++g) all_in[g] = true;
#pragma unroll
          for (int j = 0; j < Q1; ++j) {
            // a2 + a3 (y axis): the departure ordinate depends on c_j only.
            const double yd = double(Y) - (s * L::c(j) + uy);
            const double fly = floor(yd);
            const double ty = yd - (fly - 1.0);
#pragma unroll
            for (int m = 0; m < 4; ++m) ayw[j][m] = FT(interp_weight_at(m, ty));
            y0[j] = sat_floor(fly) - 1;
            ly0[j] = y0[j] - wy0;
            rows_in[j] = (unsigned)ly0[j] <= (unsigned)(WY - 4);
            all_in[j / JB] = all_in[j / JB] && rows_in[j];
            row_to<Q1, FT>(lag_row<Q1>(j), rB, dBy, gby[j]);
          }
          FT acc[Q1][Q1];  // acc[j][i]: population (i, j) of the pass
#pragma unroll
          for (int j = 0; j < Q1; ++j)
#pragma unroll
            for (int i = 0; i < Q1; ++i) acc[j][i] = FT(0);
#pragma unroll 1
          for (int rel = lo; rel <= hi; ++rel) {
            FT wx[Q1];
            bool need = false;
            const double px = double(X + rel);
#pragma unroll
            for (int i = 0; i < Q1; ++i) {
              bool in;
              wx[i] = lagrange_weight<FT>(px - xdv[i], in);
              need = need || in;
            }
            if (!__any(need)) continue;
            const int lx = X + rel - wx0;
            const bool col_in = (unsigned)lx < (unsigned)WX;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
              const int j0 = g * JB;
              FT hc[JB][Q1];
#pragma unroll
              for (int b = 0; b < JB; ++b)
#pragma unroll
                for (int ip = 0; ip < Q1; ++ip) hc[b][ip] = FT(0);
              if (need && all_in[g] && col_in) {
                int kk[JB];
#pragma unroll
                for (int b = 0; b < JB; ++b) kk[b] = ly0[j0 + b] * WX + lx;
                window_columns<Q1, JB, FT, WX, WN>(s_f, kk, &ayw[j0], &gby[j0], hc);
              } else if (need) {
#pragma unroll
                for (int b = 0; b < JB; ++b) {
                  const int j = j0 + b;
                  // with one speed per group this path means the column leaves the window
                  if (JB > 1 && rows_in[j] && col_in) {
                    const int kq = ly0[j] * WX + lx;
                    window_columns<Q1, 1, FT, WX, WN>(s_f, &kq, &ayw[j], &gby[j], &hc[b]);
                  } else {
                    const LagRow Pj = lag_row<Q1>(j);
#pragma unroll 1
                    for (int m = 0; m < 4; ++m) {
                      const FT aym = m == 0   ? ayw[j][0]
                                     : m == 1 ? ayw[j][1]
                                     : m == 2 ? ayw[j][2]
                                              : ayw[j][3];
                      column_point<Q1, FT, WX, WY, WN>(A, s_f, wx0, wy0, X + rel, y0[j] + m,
                                                       true, aym, wx, gby[j], Pj, ux, uy, inv_s,
                                                       hc[b], acc[j]);
                    }
                  }
                }
              }
#pragma unroll
              for (int b = 0; b < JB; ++b)
#pragma unroll
                for (int i = 0; i < Q1; ++i) {
                  FT v = FT(0);
#pragma unroll
                  for (int ip = 0; ip < Q1; ++ip) v += gbx[i][ip] * hc[b][ip];
                  acc[j0 + b][i] += wx[i] * v;
                }
            }
          }
#pragma unroll
          for (int i = 0; i < Q1; ++i)
#pragma unroll
            for (int j = 0; j < Q1; ++j) ft[i * Q1 + j] = acc[j][i];
        } else {
          // FP64: one column walk per group, half the y state in registers
          // (the one-walk form spills here and measured slower)
#pragma unroll 1
          for (int j0 = 0; j0 < Q1; j0 += JB) {
            FT ayw[JB][4];
            int ly0[JB];  // first stencil row of each speed, window-relative
            bool rows_in[JB];
            FT gby[JB][Q1];
            FT acc_row[JB][Q1];
            bool all_in = true;
#pragma unroll
            for (int b = 0; b < JB; ++b) {
              // a2 + a3 (y axis): the departure ordinate depends on c_j only.
              const int j = j0 + b;
              const double yd = double(Y) - (s * speed_rt<Q1>(j) + uy);
              const double fly = floor(yd);
              const double ty = yd - (fly - 1.0);
#pragma unroll
              for (int m = 0; m < 4; ++m) ayw[b][m] = FT(interp_weight_at(m, ty));
              ly0[b] = sat_floor(fly) - 1 - wy0;
              rows_in[b] = (unsigned)ly0[b] <= (unsigned)(WY - 4);
              all_in = all_in && rows_in[b];
              row_to<Q1, FT>(lag_row<Q1>(j), rB, dBy, gby[b]);
#pragma unroll
              for (int i = 0; i < Q1; ++i) acc_row[b][i] = FT(0);
            }
#pragma unroll 1
            for (int rel = lo; rel <= hi; ++rel) {
              // x speeds whose stencil no lane of the wave reaches at this
              // column skip their weight and x contraction (wave-uniform
              // branches; about half of them at any column)
              FT wx[Q1];
              bool wneed[Q1];
              bool need = false;
              const double px = double(X + rel);
#pragma unroll
              for (int i = 0; i < Q1; ++i) {
                const double u = px - xdv[i];
                const bool in = fabs(u) < 2.0;
                wneed[i] = __any(in);
                wx[i] = FT(0);
                if (wneed[i]) {
                  bool in2;
                  wx[i] = lagrange_weight<FT>(u, in2);
                }
                need = need || in;
              }
              if (!__any(need)) continue;
              FT hc[JB][Q1];
#pragma unroll
              for (int b = 0; b < JB; ++b)
#pragma unroll
                for (int ip = 0; ip < Q1; ++ip) hc[b][ip] = FT(0);
              const int lx = X + rel - wx0;
              const bool col_in = (unsigned)lx < (unsigned)WX;
              if (need && all_in && col_in) {
                int kk[JB];
#pragma unroll
                for (int b = 0; b < JB; ++b) kk[b] = ly0[b] * WX + lx;
                window_columns<Q1, JB, FT, WX, WN>(s_f, kk, ayw, gby, hc);
              } else if (need) {
#pragma unroll
                for (int b = 0; b < JB; ++b) {
                  // with one speed per walk this path means the column leaves the window
                  if (JB > 1 && rows_in[b] && col_in) {
                    const int kk = ly0[b] * WX + lx;
                    window_columns<Q1, 1, FT, WX, WN>(s_f, &kk, &ayw[b], &gby[b], &hc[b]);
                  } else {
                    const LagRow Pj = lag_row<Q1>(j0 + b);  // (rare path: rebuilt here)
#pragma unroll 1
                    for (int m = 0; m < 4; ++m) {
                      const FT aym = m == 0   ? ayw[b][0]
                                     : m == 1 ? ayw[b][1]
                                     : m == 2 ? ayw[b][2]
                                              : ayw[b][3];
                      column_point<Q1, FT, WX, WY, WN>(A, s_f, wx0, wy0, X + rel,
                                                       ly0[b] + wy0 + m, true, aym, wx, gby[b],
                                                       Pj, ux, uy, inv_s, hc[b], acc_row[b]);
                    }
                  }
                }
              }
#pragma unroll
              for (int i = 0; i < Q1; ++i) {
                if (!wneed[i]) continue;
#pragma unroll
                for (int b = 0; b < JB; ++b) {
                  FT v = FT(0);
#pragma unroll
                  for (int ip = 0; ip < Q1; ++ip) v += gbx[i][ip] * hc[b][ip];
                  acc_row[b][i] += wx[i] * v;
                }
              }
            }
#pragma unroll
            for (int b = 0; b < JB; ++b)
#pragma unroll
              for (int i = 0; i < Q1; ++i)
#pragma unroll
                for (int jj = 0; jj < Q1; ++jj)
                  if (jj == j0 + b) ft[i * Q1 + jj] = acc_row[b][i];
          }
        }

        // a6: moments in the peculiar frame of lambda_n.  FP64: plain fused
        // sums (rounding ~1e-16 of the moments, far below the App. E
        // tolerances).  FP32-mixed: FP32 accumulation compensated as a
        // Dot2 dot product: the products with the speeds split exactly,
        // the speeds held as FP32 pairs, the sums by TwoSum.
        double r0, mx, my, e2;
        if constexpr (sizeof(FT) == 8) {
          r0 = mx = my = e2 = 0.0;
#pragma unroll
          for (int i = 0; i < Q1; ++i)
#pragma unroll
            for (int j = 0; j < Q1; ++j) {
              const double fv = ft[i * Q1 + j];
              r0 += fv;
              mx = fma(L::c(i), fv, mx);
              my = fma(L::c(j), fv, my);
              e2 = fma(L::c(i) * L::c(i) + L::c(j) * L::c(j), fv, e2);
            }
        } else {
          // Row sums S_i = sum_j f_ij and column sums C_j = sum_i f_ij, each
          // with its TwoSum error; then rho = sum S_i and the speed-weighted
          // moments sum_i c_i S_i, sum_j c_j C_j, sum_i c_i^2 S_i +
          // sum_j c_j^2 C_j as Dot2 sums (a sum's error term enters with
          // the plain product): Q1 products per moment instead of Q.
          FT S[Q1], Se[Q1], C[Q1], Ce[Q1];
#pragma unroll
          for (int k = 0; k < Q1; ++k) {
            S[k] = ft[k * Q1];
            C[k] = ft[k];
            Se[k] = Ce[k] = FT(0);
          }
#pragma unroll
          for (int i = 0; i < Q1; ++i)
#pragma unroll
            for (int j = 0; j < Q1; ++j) {
              if (j > 0) two_sum_acc(S[i], Se[i], ft[i * Q1 + j]);
              if (i > 0) two_sum_acc(C[j], Ce[j], ft[i * Q1 + j]);
            }
          FT a0 = S[0], a0c = Se[0], ax = 0, axc = 0, ay = 0, ayc = 0, ae = 0, aec = 0;
#pragma unroll
          for (int k = 0; k < Q1; ++k) {
            const double ck = L::c(k), ck2 = ck * ck;
            if (k > 0) {
              two_sum_acc(a0, a0c, S[k]);
              a0c += Se[k];
            }
            dot2_acc(ax, axc, split_hi(ck), split_lo(ck), S[k]);
            axc = fma(FT(ck), Se[k], axc);
            dot2_acc(ay, ayc, split_hi(ck), split_lo(ck), C[k]);
            ayc = fma(FT(ck), Ce[k], ayc);
            dot2_acc(ae, aec, split_hi(ck2), split_lo(ck2), S[k]);
            dot2_acc(ae, aec, split_hi(ck2), split_lo(ck2), C[k]);
            aec = fma(FT(ck2), Se[k] + Ce[k], aec);
          }
          r0 = double(a0) + double(a0c);
          mx = double(ax) + double(axc);
          my = double(ay) + double(ayc);
          e2 = double(ae) + double(aec);
        }
        const int verdict = corrector<Q1>(A, s, ux, uy, T, r0, mx, my, e2, passes, rho1, ux1,
                                          uy1, T1, flags);
        if (verdict == kBad) {
          bad = true;
          break;
        }
        if (A.tape) {
          const size_t t = (size_t)passes * 4 * plane + node;
          A.tape[t] = ux1;
          A.tape[t + plane] = uy1;
          A.tape[t + 2 * plane] = T1;
          A.tape[t + 3 * plane] = rho1;
        }
        if (verdict == kDone) break;
        ux = ux1;
        uy = uy1;
        T = T1;
        if (capped && (int)passes >= A.bulk_cap) {
          deferred = true;  // continue in the tail with gauge (ux, uy, T)
          break;
        }
      }

      if (!deferred) {
        if (bad) {
          store_bad<Q1, FT>(A, fout, plane, node, 0, Q);
          flags |= POND_ITERS_BAD;
        } else {
          if (A.tape_f) {
#pragma unroll
            for (int p = 0; p < Q; ++p) A.tape_f[(size_t)p * plane + node] = double(ft[p]);
          }
          // a8: f^{lambda_n} -> lambda_{n+1}, one full Kronecker transform.
          const double s = sqrt(T * L::inv_TL), s1 = sqrt(T1 * L::inv_TL);
          const double inv_s1 = 1.0 / s1, r = s * inv_s1;
          double Rx[Q], Ry[Q];
          transfer_factor<Q1, double>(r, (ux - ux1) * inv_s1, Rx);
          transfer_factor<Q1, double>(r, (uy - uy1) * inv_s1, Ry);
          FT Hm[Q];  // Hm[i][l] = sum_j Ry[l][j] ft[i][j]
#pragma unroll
          for (int i = 0; i < Q1; ++i)
#pragma unroll
            for (int l = 0; l < Q1; ++l) {
              FT h = FT(0);
#pragma unroll
              for (int j = 0; j < Q1; ++j) h += FT(Ry[l * Q1 + j]) * ft[i * Q1 + j];
              Hm[i * Q1 + l] = h;
            }
          // a9: BGK towards rho W (eq. 18), a10: store.
          const FT omega = FT(1.0 / A.tau);
#pragma unroll
          for (int k = 0; k < Q1; ++k)
#pragma unroll
            for (int l = 0; l < Q1; ++l) {
              FT fr = FT(0);
#pragma unroll
              for (int i = 0; i < Q1; ++i) fr += FT(Rx[k * Q1 + i]) * Hm[i * Q1 + l];
              const FT feq = FT(rho1 * (L::w(k) * L::w(l)));
              fout[(size_t)(k * Q1 + l) * plane + node] = fr + omega * (feq - fr);
            }
          A.g_out[node] = ux1;
          A.g_out[plane + node] = uy1;
          A.g_out[2 * plane + node] = T1;
        }
        if (A.iters) A.iters[node] = (uint8_t)((passes & POND_ITERS_MASK) | flags);
        if (A.counters) atomicAdd(&s_hist[passes & POND_ITERS_MASK], 1u);
        c_nc += (flags & POND_ITERS_NONCONVERGED) ? 1 : 0;
        c_nb += (flags & POND_ITERS_BAD) ? 1 : 0;
        c_sp += passes;
        c_mp = passes > c_mp ? passes : c_mp;
      }
    }

    {  // cost key of the tile: per wave, the most passes of its nodes so far
      const int wm = wave_max_nonneg((int)passes);
      if (lane == 0) s_wmax[wave] = (unsigned)wm;
    }

    // ---- block tail: unconverged nodes, 16 lanes each, all waves of the block ----
    // A deferred node's next gauge goes through its output gauge slot (read
    // back with L1-bypassing loads after the barrier); its local index and pass
    // count go to an LDS list that the block's 16-lane groups drain.
    {
      if (deferred) {
        A.g_out[node] = ux;
        A.g_out[plane + node] = uy;
        A.g_out[2 * plane + node] = T;
        const unsigned slot = atomicAdd(&s_tail[0], 1u);
        s_list[slot] = (unsigned)tid | (passes << 16);
      }
      // The first wave done with its bulk passes takes the block's next tile
      // from the queue while the others finish (its wait for the queue is
      // then off the block's path), unless the queue is within two tiles per
      // block of its end, where a held tile would wait for this block.
      // The same wave copies that tile's seed gauges into LDS with direct
      // global-to-LDS loads (no registers held; full tiles on an even-width,
      // 16-byte aligned gauge array only), so that the tile starts without
      // that read either.
      if constexpr (kTakeAhead) {
        unsigned first = 0u;
        if (lane == 0) first = atomicAdd(&s_arrive, 1u) == 0u && s_g + 2u * gridDim.x < ntiles;
        if (__shfl(first, 0)) {
          unsigned tn = 0u;
          if (lane == 0) {
            const unsigned gn = atomicAdd(&A.queue->next, 1u);
            tn = (keyed && A.tile_order && gn < ntiles) ? A.tile_order[gn] : gn;
            s_pref_tile = tn;
            s_pref = gn;
          }
          tn = __shfl(tn, 0);
          const int tyn = (int)(tn / (unsigned)ntx), txn = (int)tn - tyn * ntx;
          const int bxn = txn * TX, byn = tyn * TY;
          const bool dma = kStageSeeds && tn < ntiles && bxn + TX <= A.nx && byn + TY <= A.ny &&
                           (A.nx & 1) == 0 && (reinterpret_cast<uintptr_t>(gin) & 15u) == 0u;
          if (dma) {
            // rows r = 0 .. 3 TY - 1 (gauge component r / TY, tile row r % TY) of TX
            // doubles; one load moves 64 lanes x 16 bytes = four rows, lane l to
            // LDS bytes 16 l onwards
            static_assert(TX == 32 && (3 * TY) % 4 == 0, "four gauge rows per load");
            const int rr = lane >> 4, cc = (lane & 15) * 2;
#pragma unroll 1
            for (int k = 0; k < 3 * TY / 4; ++k) {
              const int r = 4 * k + rr, comp = r / TY, ly = r - comp * TY;
              const double* src = gin + (size_t)comp * plane + (size_t)(byn + ly) * A.nx + bxn + cc;
              __builtin_amdgcn_global_load_lds(
                  (const void __attribute__((address_space(1)))*)src,
                  (void __attribute__((address_space(3)))*)(s_seed + 4 * k * TX), 16, 0, 0);
            }
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the copies are in LDS
          }
          if (lane == 0) s_seed_tile = dma ? tn : ~0u;
        }
      }
      __threadfence_block();
      __syncthreads();
      const unsigned count = s_tail[0];
      if (count)
        tail_wave<Q1, FT, WX, WY, WN, TX, WTX, WTY>(A, s_f, wx0, wy0, uxB, uyB, sB, bx0, by0,
                                                     count, s_list, &s_tail[1], s_wmax, s_hist,
                                                     c_nc, c_nb, c_sp, c_mp);
    }
    if (A.counters) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        c_nc += __shfl_xor(c_nc, off);
        c_nb += __shfl_xor(c_nb, off);
        c_sp += __shfl_xor(c_sp, off);
        const unsigned long long o = __shfl_xor(c_mp, off);
        c_mp = o > c_mp ? o : c_mp;
      }
      if (lane == 0) {
        if (c_nc) atomicAdd(&A.counters->nonconverged, c_nc);
        if (c_nb) atomicAdd(&A.counters->bad, c_nb);
        atomicAdd(&A.counters->sum_passes, c_sp);
        atomicMax(&A.counters->max_passes, c_mp);
      }
    }
    __syncthreads();  // LDS of this tile is free
    if (tid == 0) {
      unsigned key = 0;
#pragma unroll
      for (int w = 0; w < TS::NW; ++w) {
        key += s_wmax[w];
        s_wmax[w] = 0u;
      }
      if (keyed)
        A.tile_keys[tile] = (uint16_t)(key < kKeyBins<NT> ? key : kKeyBins<NT> - 1);
    }
  }  // tile loop

  // The block's pass histogram is complete: its last updates precede the
  // barriers of the final loop iteration.
  if (A.counters && tid <= POND_ITERS_MASK && s_hist[tid])
    atomicAdd(&A.counters->hist[tid], (unsigned long long)s_hist[tid]);

  // The last block out orders the tiles for the next launch by this step's
  // keys and resets the queue.  Every block has taken its last tile before it
  // counts itself out, so the order array is no longer read.  The flag has an
  // LDS word of its own: a wave still about to read s_tile must not see it.
  if (tid == 0) {
    __threadfence();
    s_last = atomicAdd(&A.queue->done, 1u) == gridDim.x - 1 ? 1u : 0u;
  }
  __syncthreads();
  if (s_last) {
    __threadfence();
    if (keyed && A.tile_order_next)
      order_tiles<NT>(A.tile_keys, A.tile_order_next, ntiles, reinterpret_cast<unsigned*>(s_f));
    if (tid == 0) {
      atomicExch(&A.queue->next, 0u);
      atomicExch(&A.queue->done, 0u);
    }
  }
}

// Tile shapes (TX x TY nodes per block, halo H).  D2Q16 FP64: 32 x 16
// nodes, a 42 x 26 window of 140 KiB of LDS (one block of 8 waves per CU, 2
// waves per SIMD).  Otherwise 32 x 8 nodes: D2Q16 FP32-mixed a 42 x 18
// window of 48 KiB, two blocks of 4 waves per CU (2 waves per SIMD; smaller
// tiles balance the passes better than 32 x 16, and 3 waves per SIMD with
// registers capped at 168 measured slower once two y speeds share a column
// walk); D2Q9 FP64 a 40 x 16 window of 51 KiB, two blocks per CU (about 1 %
// faster than one block on 32 x 16 tiles); D2Q9 FP32-mixed three blocks.
template <int Q1, class FT>
struct StepTile {
  static constexpr int TX = 32, TY = sizeof(FT) == 8 && Q1 == 4 ? 16 : 8, H = Q1 == 4 ? 5 : 4;
};

// Persistent grid: as many blocks as the device holds at once (CUs x blocks
// per CU), never more than there are tiles.
template <int Q1, class FT>
hipError_t launch_step_t(const StepArgs& a, hipStream_t s) {
  using ST = StepTile<Q1, FT>;
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
        &per_cu, reinterpret_cast<const void*>(&k_step<Q1, FT, ST::TX, ST::TY, ST::H>),
        ST::TX * ST::TY, 0);
    if (e != hipSuccess) return e;
    resident[dev] = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  }
  const long long tiles =
      (long long)((a.nx + ST::TX - 1) / ST::TX) * ((a.ny + ST::TY - 1) / ST::TY);
  const int nblk = (int)(tiles < resident[dev] ? tiles : resident[dev]);
  hipLaunchKernelGGL((k_step<Q1, FT, ST::TX, ST::TY, ST::H>), dim3(nblk), dim3(ST::TX * ST::TY), 0,
                     s, a);
  return hipGetLastError();
}

template <int Q1, class FT>
unsigned tile_count_t(const pond_config& c) {
  using ST = StepTile<Q1, FT>;
  return (unsigned)(((c.nx + ST::TX - 1) / ST::TX) * (long long)((c.ny + ST::TY - 1) / ST::TY));
}

}  // namespace

unsigned step_tile_count(const pond_config& c) {
  if (c.q1d == 3)
    return c.precision == POND_F64 ? tile_count_t<3, double>(c) : tile_count_t<3, float>(c);
  return c.precision == POND_F64 ? tile_count_t<4, double>(c) : tile_count_t<4, float>(c);
}

hipError_t launch_step(const pond_config& c, const StepArgs& a, hipStream_t s) {
  const bool f64 = c.precision == POND_F64;
  if (c.q1d == 4) return f64 ? launch_step_t<4, double>(a, s) : launch_step_t<4, float>(a, s);
  return f64 ? launch_step_t<3, double>(a, s) : launch_step_t<3, float>(a, s);
}

}  // namespace pond
