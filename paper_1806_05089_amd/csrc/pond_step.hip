// The fused PonD time step on gfx950: propagation with the predictor-corrector
// gauge iteration (eqs. 6-16, App. E), regauge and BGK collision (eqs. 17-18).
//
// Mapping.  One lane owns one node; a wave covers an 8 x 8 tile of nodes
// (nodes that need many predictor-corrector passes cluster along fronts, and
// square wave tiles cut the number of waves a front crosses).
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
// and pass, and a (population, collocation point) pair costs 16 LDS reads and
// 20 multiply-adds.  A collocation point outside the window is read from HBM
// and transformed directly with G_{s->n}.  After staging the lanes iterate
// independently (no further barriers).
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
  static constexpr size_t lds_bytes = (size_t)Q1 * Q1 * WN * sizeof(FT);
  static_assert(TX % 8 == 0 && TY % 8 == 0, "waves are 8 x 8 node tiles");
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

template <int Q1, class FT, int TX, int TY, int H>
__global__ void __launch_bounds__(TX * TY)
k_step(StepArgs A) {
  constexpr int Q = Q1 * Q1;
  using L = Lat<Q1>;
  using TS = TileShape<Q1, FT, TX, TY, H>;
  constexpr int WX = TS::WX, WY = TS::WY, WN = TS::WN, NT = TS::NT;
  __shared__ FT s_f[Q * WN];
  __shared__ int s_ri[4 * TS::NW];
  __shared__ double s_rd[4 * TS::NW];

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

  // ---- stage the window in the reference gauge (eq. 4, G_{s->B}) ----
  {
    const double inv_sB = 1.0 / sB;
    for (int k = tid; k < WN; k += NT) {
      const int wy = k / WX, wx = k - wy * WX;
      const int sx = wrap_index(wx0 + wx, A.nx, A.bc_x);
      const int sy = wrap_index(wy0 + wy, A.ny, A.bc_y);
      const size_t src = (size_t)sy * A.nx + sx;
      double f[Q];
#pragma unroll
      for (int p = 0; p < Q; ++p) f[p] = double(fin[(size_t)p * plane + src]);
      const double ss = sqrt(gin[2 * plane + src] * L::inv_TL);
      const double r = ss * inv_sB;
      double Gx[Q], Gy[Q];
      transfer_factor<Q1, double>(r, (gin[src] - uxB) * inv_sB, Gx);
      transfer_factor<Q1, double>(r, (gin[plane + src] - uyB) * inv_sB, Gy);
      double Hm[Q];  // Hm[i][l] = sum_j Gy[l][j] f[i][j]
#pragma unroll
      for (int i = 0; i < Q1; ++i)
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          double h = 0.0;
#pragma unroll
          for (int j = 0; j < Q1; ++j) h = fma(Gy[l * Q1 + j], f[i * Q1 + j], h);
          Hm[i * Q1 + l] = h;
        }
#pragma unroll
      for (int kk = 0; kk < Q1; ++kk)
#pragma unroll
        for (int l = 0; l < Q1; ++l) {
          double t = 0.0;
#pragma unroll
          for (int i = 0; i < Q1; ++i) t = fma(Gx[kk * Q1 + i], Hm[i * Q1 + l], t);
          s_f[(kk * Q1 + l) * WN + k] = FT(t);
        }
    }
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
      // a4 (window part): G_{B->n} rows are l_k(rB c + dB) per axis.
      const double rB = sB * inv_s;
      const double dBx = (uxB - ux) * inv_s, dBy = (uyB - uy) * inv_s;

      // (y speed j, x speed i, stencil column n) are wave-uniform rolled
      // loops; the four stencil rows of one column are unrolled.
#pragma unroll 1
      for (int j = 0; j < Q1; ++j) {
        // a2 + a3 (y axis): the departure ordinate depends on c_j only.
        const double yd = double(Y) - (s * speed_rt<Q1>(j) + uy);
        const double fly = floor(yd);
        double ay[4];
        interp_weights(yd - (fly - 1.0), ay);
        const int y0 = sat_floor(fly) - 1;
        const int ly0 = y0 - wy0;
        const LagRow Pj = lag_row<Q1>(j);
        FT gby[Q1];
        {
          double row[Q1];
          transfer_row_coef<Q1>(Pj, rB, dBy, row);
#pragma unroll
          for (int jp = 0; jp < Q1; ++jp) gby[jp] = FT(row[jp]);
        }
#pragma unroll 1
        for (int i = 0; i < Q1; ++i) {
          // a2 + a3 (x axis)
          const double xd = double(X) - (s * speed_rt<Q1>(i) + ux);
          const double fl = floor(xd);
          double ax[4];
          interp_weights(xd - (fl - 1.0), ax);
          const int x0 = sat_floor(fl) - 1;
          const LagRow Pi = lag_row<Q1>(i);
          FT gbx[Q1];
          {
            double row[Q1];
            transfer_row_coef<Q1>(Pi, rB, dBx, row);
#pragma unroll
            for (int ip = 0; ip < Q1; ++ip) gbx[ip] = FT(row[ip]);
          }
          FT acc_ij = FT(0);
#pragma unroll 1
          for (int n = 0; n < 4; ++n) {
            const int lx = x0 + n - wx0;
            const bool in_x = (unsigned)lx < (unsigned)WX;
            const double axn = n == 0 ? ax[0] : n == 1 ? ax[1] : n == 2 ? ax[2] : ax[3];
            FT col = FT(0);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const int ly = ly0 + m;
              FT val;
              if (in_x && (unsigned)ly < (unsigned)WY) {
                // a4 + a5: [G_{B->n} f^B_s]_(i,j) from the staged window
                const int k = ly * WX + lx;
                FT t = FT(0);
#pragma unroll
                for (int ip = 0; ip < Q1; ++ip) {
                  FT h = FT(0);
#pragma unroll
                  for (int jp = 0; jp < Q1; ++jp) h += gby[jp] * s_f[(ip * Q1 + jp) * WN + k];
                  t += gbx[ip] * h;
                }
                val = t;
              } else {
                // outside the window: [G_{s->n} f_s]_(i,j) from HBM
                const int sx = wrap_index(x0 + n, A.nx, A.bc_x);
                const int sy = wrap_index(y0 + m, A.ny, A.bc_y);
                const size_t src = (size_t)sy * A.nx + sx;
                const double r = sqrt(gin[2 * plane + src] * L::inv_TL) * inv_s;
                double gxr[Q1], gyr[Q1];
                transfer_row_coef<Q1>(Pi, r, fma(gin[src], inv_s, -uxs), gxr);
                transfer_row_coef<Q1>(Pj, r, fma(gin[plane + src], inv_s, -uys), gyr);
                FT t = FT(0);
#pragma unroll
                for (int ip = 0; ip < Q1; ++ip) {
                  FT h = FT(0);
#pragma unroll
                  for (int jp = 0; jp < Q1; ++jp)
                    h += FT(gyr[jp]) * fin[(size_t)(ip * Q1 + jp) * plane + src];
                  t += FT(gxr[ip]) * h;
                }
                val = t;
              }
              // a5: weight of row m
              col += FT(ay[m]) * val;
            }
            acc_ij += FT(axn) * col;
          }
#pragma unroll
          for (int ii = 0; ii < Q1; ++ii)
#pragma unroll
            for (int jj = 0; jj < Q1; ++jj)
              if (ii == i && jj == j) ft[ii * Q1 + jj] = acc_ij;
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

// Tile shapes (TX x TY nodes per block, halo H).  D2Q16: 32 x 16 nodes with a
// 42 x 26 window: 140 KiB of LDS in FP64 (one block, 8 waves per CU) and
// 70 KiB in FP32 (two blocks per CU).
#ifndef POND_TILE_X
#define POND_TILE_X 32
#endif
#ifndef POND_TILE_Y
#define POND_TILE_Y 16
#endif
#ifndef POND_HALO
#define POND_HALO 5
#endif
template <int Q1, class FT>
struct StepTile {
  static constexpr int TX = POND_TILE_X, TY = POND_TILE_Y, H = Q1 == 4 ? POND_HALO : 4;
};

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
