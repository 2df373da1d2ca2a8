// The fused PonD time step on gfx950: propagation with the predictor-corrector
// gauge iteration (eqs. 6-16, App. E), regauge and BGK collision (eqs. 17-18).
//
// Mapping.  One lane owns one node; a wave covers an 8 x 8 tile of nodes
// (nodes that need many predictor-corrector passes cluster along fronts, and
// square wave tiles cut the number of waves a front crosses).  A block of
// TX x TY nodes first stages a halo window of the state at t - dt in LDS:
// populations f (FT) and the gauge (u_x, u_y, sqrt(theta)) (double) of
// (TX + 2H) x (TY + 2H) nodes, placed around the stencils of the block's seed
// gauges (so a fast uniform drift shifts the window instead of widening it).
// The pass loop then gathers every collocation point from LDS; a point outside
// the window (a corrector pass that moved far, or a block whose stencils span
// more than the window) is read from HBM instead.  After the staging barrier
// the lanes iterate independently.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>

#include "pond_device.hpp"
#include "pond_internal.hpp"

namespace pond {
namespace {

template <int Q1, class FT, int TX, int TY, int H>
struct TileShape {
  static constexpr int WX = TX + 2 * H;
  static constexpr int WY = TY + 2 * H;
  static constexpr int WN = WX * WY;
  static constexpr int NT = TX * TY;
  static constexpr int NW = NT / 64;
  static constexpr size_t lds_bytes = (size_t)Q1 * Q1 * WN * sizeof(FT) + 3 * WN * sizeof(double);
  static_assert(TX % 8 == 0 && TY % 8 == 0, "waves are 8 x 8 node tiles");
  static_assert(lds_bytes + 64 <= 160 * 1024, "window exceeds the 160 KiB LDS of a CU");
};

// Block-wide minimum of four ints (maxima are passed negated).
template <int NW>
__device__ __forceinline__ void block_min4(int v[4], int* s_red) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int o = __shfl_xor(v[k], off);
      v[k] = o < v[k] ? o : v[k];
    }
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s_red[k * NW + (threadIdx.x >> 6)] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int m = s_red[k * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) m = s_red[k * NW + w] < m ? s_red[k * NW + w] : m;
    v[k] = m;
  }
}

// Floor of a departure coordinate as int, saturated so that absurd gauges
// (non-finite or |x| > 1e9) cannot overflow the conversion.
__device__ __forceinline__ int sat_floor(double x) {
  x = fmin(fmax(x, -1.0e9), 1.0e9);
  return isfinite(x) ? int(floor(x)) : 0;
}

template <int Q1, class FT, int TX, int TY, int H>
__global__ void __launch_bounds__(TX * TY)
k_step(StepArgs A) {
  constexpr int Q = Q1 * Q1;
  using L = Lat<Q1>;
  using TS = TileShape<Q1, FT, TX, TY, H>;
  constexpr int WX = TS::WX, WY = TS::WY, WN = TS::WN, NT = TS::NT;
  __shared__ FT s_f[Q * WN];
  __shared__ double s_g[3 * WN];
  __shared__ int s_red[4 * TS::NW];

  // Block -> tile: blocks are dealt to the 8 XCDs round-robin; renumber so
  // that consecutive tiles (which share halo data) run on the same XCD.
  const int nbx = gridDim.x, nblk = gridDim.x * gridDim.y;
  int b = blockIdx.y * nbx + blockIdx.x;
  if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  const int bx0 = (b % nbx) * TX, by0 = (b / nbx) * TY;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int X = bx0 + (wave % (TX / 8)) * 8 + (lane & 7);
  const int Y = by0 + (wave / (TX / 8)) * 8 + (lane >> 3);
  const bool active = (X < A.nx) && (Y < A.ny);
  const size_t plane = (size_t)A.nx * A.ny;
  const FT* __restrict__ fin = static_cast<const FT*>(A.f_in);
  const double* __restrict__ gin = A.g_in;

  // a1: seed gauge (eqs. 7-8) or the alternative seeds.
  double ux = 0.0, uy = 0.0, T = L::TL;
  size_t node = 0;
  if (active) {
    node = (size_t)Y * A.nx + X;
    ux = gin[node];
    uy = gin[plane + node];
    T = gin[2 * plane + node];
    if (A.seed_mode == 1) {
      ux = 0.0;
      uy = 0.0;
      if (!A.isothermal) T = L::TL;
    } else if (A.seed_mode == 2) {
      ux = -ux;
      uy = -uy;
    }
  }

  // ---- window placement from the seed stencils (one node of margin) ----
  int wx0, wy0;
  {
    int v[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
    const double sp = sqrt(T * L::inv_TL) * L::c(Q1 - 1);
    if (active && isfinite(sp) && isfinite(ux) && isfinite(uy)) {
      v[0] = sat_floor(double(X) - ux - sp) - 2;
      v[1] = -(sat_floor(double(X) - ux + sp) + 3);
      v[2] = sat_floor(double(Y) - uy - sp) - 2;
      v[3] = -(sat_floor(double(Y) - uy + sp) + 3);
    }
    block_min4<TS::NW>(v, s_red);
    if (v[0] == INT_MAX) {  // no usable seed in the block: centre on the tile
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
  // ---- stage the window (rows of the window are coalesced along x) ----
  for (int k = tid; k < WN; k += NT) {
    const int wy = k / WX, wx = k - wy * WX;
    const int sx = wrap_index(wx0 + wx, A.nx, A.bc_x);
    const int sy = wrap_index(wy0 + wy, A.ny, A.bc_y);
    const size_t src = (size_t)sy * A.nx + sx;
#pragma unroll
    for (int p = 0; p < Q; ++p) s_f[p * WN + k] = fin[(size_t)p * plane + src];
    s_g[k] = gin[src];
    s_g[WN + k] = gin[plane + src];
    s_g[2 * WN + k] = sqrt(gin[2 * plane + src] * L::inv_TL);
  }
  __syncthreads();

  unsigned passes = 0;
  unsigned flags = 0;
  if (active) {
    FT ft[Q];
    double ux1 = ux, uy1 = uy, T1 = T, rho1 = 0.0;
    bool bad = false;
    for (;;) {
      ++passes;
      const double s = sqrt(T * L::inv_TL);
      const double inv_s = 1.0 / s;
      const double uxs = ux * inv_s, uys = uy * inv_s;
#pragma unroll
      for (int p = 0; p < Q; ++p) ft[p] = FT(0);

      // (x speed i, stencil column n, y speed j, stencil row m) one at a time;
      // the four indices are wave-uniform, so the loops stay rolled and one
      // collocation point is live in registers.
#pragma unroll 1
      for (int i = 0; i < Q1; ++i) {
        // a2 + a3 (x axis): the departure abscissa depends on c_i only.
        const double xd = double(X) - (s * speed_rt<Q1>(i) + ux);
        const LagRow Pi = lag_row<Q1>(i);
        const double fl = floor(xd);
        double ax[4];
        interp_weights(xd - (fl - 1.0), ax);
        const int x0 = sat_floor(fl) - 1;
        FT acc_row[Q1];
#pragma unroll
        for (int j = 0; j < Q1; ++j) acc_row[j] = FT(0);
#pragma unroll 1
        for (int n = 0; n < 4; ++n) {
          const int gx = x0 + n;
          const int lx = gx - wx0;
          const bool in_x = (unsigned)lx < (unsigned)WX;
          const double axn = n == 0 ? ax[0] : n == 1 ? ax[1] : n == 2 ? ax[2] : ax[3];
#pragma unroll 1
          for (int j = 0; j < Q1; ++j) {
            // a2 + a3 (y axis)
            const double yd = double(Y) - (s * speed_rt<Q1>(j) + uy);
            const LagRow Pj = lag_row<Q1>(j);
            const double fly = floor(yd);
            double ay[4];
            interp_weights(yd - (fly - 1.0), ay);
            const int y0 = sat_floor(fly) - 1;
            FT acc_j = FT(0);
#pragma unroll 1
            for (int m = 0; m < 4; ++m) {
              const int gy = y0 + m;
              const int ly = gy - wy0;
              const double aym = m == 0 ? ay[0] : m == 1 ? ay[1] : m == 2 ? ay[2] : ay[3];
              // the collocation point (gx, gy): LDS window or HBM
              FT fs[Q];
              double sux, suy, ss;
              if (in_x && (unsigned)ly < (unsigned)WY) {
                const int k = ly * WX + lx;
#pragma unroll
                for (int p = 0; p < Q; ++p) fs[p] = s_f[p * WN + k];
                sux = s_g[k];
                suy = s_g[WN + k];
                ss = s_g[2 * WN + k];
              } else {
                const int sx = wrap_index(gx, A.nx, A.bc_x);
                const int sy = wrap_index(gy, A.ny, A.bc_y);
                const size_t src = (size_t)sy * A.nx + sx;
#pragma unroll
                for (int p = 0; p < Q; ++p) fs[p] = fin[(size_t)p * plane + src];
                sux = gin[src];
                suy = gin[plane + src];
                ss = sqrt(gin[2 * plane + src] * L::inv_TL);
              }
              // a4: rows i and j of the transfer factors, z = r c + d
              const double r = ss * inv_s;
              double gxr[Q1], gyr[Q1];
              transfer_row_coef<Q1>(Pi, r, fma(sux, inv_s, -uxs), gxr);
              transfer_row_coef<Q1>(Pj, r, fma(suy, inv_s, -uys), gyr);
              FT acc = FT(0);
#pragma unroll
              for (int ip = 0; ip < Q1; ++ip) {
                FT h = FT(0);
#pragma unroll
                for (int jp = 0; jp < Q1; ++jp) h += FT(gyr[jp]) * fs[ip * Q1 + jp];
                acc += FT(gxr[ip]) * h;
              }
              // a5: interpolation weight of this collocation point
              acc_j += FT(axn * aym) * acc;
            }
#pragma unroll
            for (int jj = 0; jj < Q1; ++jj)
              if (jj == j) acc_row[jj] += acc_j;
          }
        }
#pragma unroll
        for (int ii = 0; ii < Q1; ++ii)
          if (ii == i) {
#pragma unroll
            for (int j = 0; j < Q1; ++j) ft[ii * Q1 + j] = acc_row[j];
          }
      }

      // a6: moments in the peculiar frame of lambda_n (compensated sums).
      FT r0 = 0, r0c = 0, mx = 0, mxc = 0, my = 0, myc = 0, e2 = 0, e2c = 0;
#pragma unroll
      for (int i = 0; i < Q1; ++i)
#pragma unroll
        for (int j = 0; j < Q1; ++j) {
          const FT fv = ft[i * Q1 + j];
          two_sum_acc(r0, r0c, fv);
          two_sum_acc(mx, mxc, FT(L::c(i)) * fv);
          two_sum_acc(my, myc, FT(L::c(j)) * fv);
          two_sum_acc(e2, e2c, FT(L::c(i) * L::c(i) + L::c(j) * L::c(j)) * fv);
        }
      const double rho = double(r0) + double(r0c);
      const double dux = s * (double(mx) + double(mxc)) / rho;
      const double duy = s * (double(my) + double(myc)) / rho;
      rho1 = rho;
      ux1 = ux + dux;
      uy1 = uy + duy;
      T1 = A.isothermal ? T
                        : 0.5 * (s * s * (double(e2) + double(e2c)) / rho - (dux * dux + duy * duy));
      if (!(rho1 > 0.0) || !(T1 > 0.0) || !isfinite(rho1) || !isfinite(ux1) || !isfinite(uy1) ||
          !isfinite(T1)) {
        bad = true;
        break;
      }
      bool done;
      if (A.fixed_iter > 0) {
        done = (int)passes >= A.fixed_iter;
      } else {
        // a7: App. E, each of u_x, u_y, sqrt(theta) separately.
        bool conv = fabs(ux1 - ux) < A.eps_abs + A.eps_rel * fabs(ux1) &&
                    fabs(uy1 - uy) < A.eps_abs + A.eps_rel * fabs(uy1);
        if (!A.isothermal) {
          const double s1 = sqrt(T1 * L::inv_TL);
          conv = conv && fabs(s1 - s) < A.eps_abs + A.eps_rel * fabs(s1);
        }
        done = conv || (int)passes >= A.max_iter;
        if (!conv && done) flags |= POND_ITERS_NONCONVERGED;
      }
      if (done) break;
      ux = ux1;
      uy = uy1;
      T = T1;
    }

    FT* __restrict__ fout = static_cast<FT*>(A.f_out);
    if (bad) {
      flags |= POND_ITERS_BAD;
      const double qnan = __builtin_nan("");
#pragma unroll
      for (int p = 0; p < Q; ++p) fout[(size_t)p * plane + node] = FT(qnan);
      A.g_out[node] = qnan;
      A.g_out[plane + node] = qnan;
      A.g_out[2 * plane + node] = qnan;
    } else {
      // a8: f^{lambda_n} -> lambda_{n+1}, one full Kronecker transform.
      const double s = sqrt(T * L::inv_TL), s1 = sqrt(T1 * L::inv_TL);
      const double inv_s1 = 1.0 / s1, r = s * inv_s1;
      FT Hm[Q];  // Hm[i][l] = sum_j Ry[l][j] ft[i][j]
#pragma unroll
      for (int l = 0; l < Q1; ++l) {
        double ry[Q1];
        transfer_row<Q1>(l, r, (uy - uy1) * inv_s1, ry);
#pragma unroll
        for (int i = 0; i < Q1; ++i) {
          FT h = FT(0);
#pragma unroll
          for (int j = 0; j < Q1; ++j) h += FT(ry[j]) * ft[i * Q1 + j];
          Hm[i * Q1 + l] = h;
        }
      }
      // a9: BGK towards rho W (eq. 18), a10: store.
      const FT omega = FT(1.0 / A.tau);
#pragma unroll
      for (int k = 0; k < Q1; ++k) {
        double rx[Q1];
        transfer_row<Q1>(k, r, (ux - ux1) * inv_s1, rx);
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          FT fr = FT(0);
#pragma unroll
          for (int i = 0; i < Q1; ++i) fr += FT(rx[i]) * Hm[i * Q1 + l];
          const FT feq = FT(rho1 * (L::w(k) * L::w(l)));
          fout[(size_t)(k * Q1 + l) * plane + node] = fr + omega * (feq - fr);
        }
      }
      A.g_out[node] = ux1;
      A.g_out[plane + node] = uy1;
      A.g_out[2 * plane + node] = T1;
    }
    if (A.iters) A.iters[node] = (uint8_t)((passes & POND_ITERS_MASK) | flags);
  }

  if (A.counters) {
    unsigned long long nc = (flags & POND_ITERS_NONCONVERGED) ? 1ull : 0ull;
    unsigned long long nb = (flags & POND_ITERS_BAD) ? 1ull : 0ull;
    unsigned long long sp = passes;
    unsigned long long mp = passes;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      nc += __shfl_xor(nc, off);
      nb += __shfl_xor(nb, off);
      sp += __shfl_xor(sp, off);
      const unsigned long long o = __shfl_xor(mp, off);
      mp = o > mp ? o : mp;
    }
    if (lane == 0) {
      if (nc) atomicAdd(&A.counters->nonconverged, nc);
      if (nb) atomicAdd(&A.counters->bad, nb);
      atomicAdd(&A.counters->sum_passes, sp);
      atomicMax(&A.counters->max_passes, mp);
    }
  }
}

// Tile shapes: TX x TY nodes per block, halo H.  FP64: 16 x 16, H = 5
// (26 x 26 window, 103 KiB LDS, one block per CU).  FP32-mixed: same window
// in 59 KiB (two blocks per CU).
template <int Q1, class FT>
struct StepTile;
template <> struct StepTile<4, double> { static constexpr int TX = 16, TY = 16, H = 5; };
template <> struct StepTile<4, float> { static constexpr int TX = 16, TY = 16, H = 5; };
template <> struct StepTile<3, double> { static constexpr int TX = 16, TY = 16, H = 4; };
template <> struct StepTile<3, float> { static constexpr int TX = 16, TY = 16, H = 4; };

template <int Q1, class FT>
hipError_t launch_step_t(const StepArgs& a, hipStream_t s) {
  using ST = StepTile<Q1, FT>;
  dim3 block(ST::TX * ST::TY);
  dim3 grid((a.nx + ST::TX - 1) / ST::TX, (a.ny + ST::TY - 1) / ST::TY);
  hipLaunchKernelGGL((k_step<Q1, FT, ST::TX, ST::TY, ST::H>), grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(const pond_config& c, const StepArgs& a, hipStream_t s) {
  const bool f64 = c.precision == POND_F64;
  if (c.q1d == 4) return f64 ? launch_step_t<4, double>(a, s) : launch_step_t<4, float>(a, s);
  return f64 ? launch_step_t<3, double>(a, s) : launch_step_t<3, float>(a, s);
}

}  // namespace pond
