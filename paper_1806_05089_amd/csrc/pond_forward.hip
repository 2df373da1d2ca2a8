// Forward kernels of the PonD time step on gfx950: equilibrium initialisation,
// the fused step (propagation + predictor-corrector + BGK) and the moments.
//
// Layout in HBM: structure-of-arrays planes, row-major [ny][nx]:
//   f[p][y][x], p = i*q + j   populations in the node's own gauge (FT)
//   g[k][y][x], k = ux, uy, T the node's gauge (double)
// One lane owns one node; a wave covers 64 consecutive x nodes of one row, so
// every gather of a (population, collocation point) pair reads 64 neighbouring
// words of one plane.
#include <hip/hip_runtime.h>
#include <math.h>

#include "pond_device.hpp"
#include "pond_internal.hpp"

namespace pond {
namespace {

constexpr int kBlockX = 64;
constexpr int kBlockY = 4;

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

// ------------------------------------------------------------------ init
template <int Q1, class FT>
__global__ void __launch_bounds__(256)
k_init(int nx, int ny, const double* __restrict__ rho, const double* __restrict__ ux,
       const double* __restrict__ uy, const double* __restrict__ T, FT* __restrict__ f,
       double* __restrict__ g, uint8_t* __restrict__ iters, unsigned long long* bad) {
  const size_t plane = (size_t)nx * ny;
  const size_t node = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= plane) return;
  const double r = rho[node], u = ux[node], v = uy[node], t = T[node];
#pragma unroll
  for (int i = 0; i < Q1; ++i)
#pragma unroll
    for (int j = 0; j < Q1; ++j)
      f[(size_t)(i * Q1 + j) * plane + node] = FT(r * (Lat<Q1>::w(i) * Lat<Q1>::w(j)));
  g[node] = u;
  g[plane + node] = v;
  g[2 * plane + node] = t;
  if (iters) iters[node] = 0;
  const bool ok = (r > 0.0) && (t > 0.0) && finite(r) && finite(u) && finite(v) && finite(t);
  if (!ok) atomicAdd(bad, 1ull);
}

// ------------------------------------------------------------------ step
// One lane = one node.  Every pass of the predictor-corrector loop:
//   a2  particle velocities v = sqrt(theta_n) c + u_n           (eqs. 1, 9)
//   a3  departure points x - v dt, stencil origin floor - 1,
//       per-axis Lagrange weights                              (eq. 6, App. C)
//   a4  gauge transform of every collocation point into lambda_n,
//       one row of each per-axis factor                        (eq. 4)
//   a5  weighted sum over the 4 x 4 stencil                    (eq. 5)
//   a6  corrector moments in the peculiar frame of lambda_n     (eqs. 10-12)
//   a7  App. E convergence test on u_x, u_y, sqrt(theta)
// then a8 regauge into lambda_{n+1}, a9 BGK, a10 store.
template <int Q1, class FT>
__global__ void __launch_bounds__(kBlockX * kBlockY)
k_step(StepArgs A) {
  constexpr int Q = Q1 * Q1;
  using L = Lat<Q1>;
  const int X = blockIdx.x * kBlockX + threadIdx.x;
  const int Y = blockIdx.y * kBlockY + threadIdx.y;
  const bool active = (X < A.nx) && (Y < A.ny);
  const size_t plane = (size_t)A.nx * A.ny;
  const FT* __restrict__ fin = static_cast<const FT*>(A.f_in);
  const double* __restrict__ gin = A.g_in;

  unsigned passes = 0;
  unsigned flags = 0;
  if (active) {
    const size_t node = (size_t)Y * A.nx + X;
    // a1: seed gauge (eqs. 7-8) or the alternative seeds.
    double ux = gin[node], uy = gin[plane + node], T = gin[2 * plane + node];
    if (A.seed_mode == 1) {
      ux = 0.0;
      uy = 0.0;
      if (!A.isothermal) T = L::TL;
    } else if (A.seed_mode == 2) {
      ux = -ux;
      uy = -uy;
    }

    FT ft[Q];
    double ux1 = ux, uy1 = uy, T1 = T, rho1 = 0.0;
    bool bad = false;
    for (;;) {
      ++passes;
      const double s = sqrt(T * L::inv_TL);
      const double inv_s = 1.0 / s;
#pragma unroll
      for (int p = 0; p < Q; ++p) ft[p] = FT(0);

      // One (x speed i, stencil column n, y speed j, stencil row m) at a
      // time; all four indices are wave-uniform, so the loops stay rolled and
      // only one collocation point is live in registers.
#pragma unroll 1
      for (int i = 0; i < Q1; ++i) {
        // a2 + a3 (x axis): the departure abscissa depends on c_i only.
        const double xd = double(X) - (s * speed_rt<Q1>(i) + ux);
        const double fl = floor(xd);
        double ax[4];
        interp_weights(xd - (fl - 1.0), ax);
        const int x0 = int(fl) - 1;
        FT acc_row[Q1];
#pragma unroll
        for (int j = 0; j < Q1; ++j) acc_row[j] = FT(0);
#pragma unroll 1
        for (int n = 0; n < 4; ++n) {
          const int sx = wrap_index(x0 + n, A.nx, A.bc_x);
          const double axn = n == 0 ? ax[0] : n == 1 ? ax[1] : n == 2 ? ax[2] : ax[3];
#pragma unroll 1
          for (int j = 0; j < Q1; ++j) {
            // a2 + a3 (y axis)
            const double yd = double(Y) - (s * speed_rt<Q1>(j) + uy);
            const double fly = floor(yd);
            double ay[4];
            interp_weights(yd - (fly - 1.0), ay);
            const int y0 = int(fly) - 1;
            FT acc_j = FT(0);
#pragma unroll 1
            for (int m = 0; m < 4; ++m) {
              const int sy = wrap_index(y0 + m, A.ny, A.bc_y);
              const double aym = m == 0 ? ay[0] : m == 1 ? ay[1] : m == 2 ? ay[2] : ay[3];
              // a4: rows i and j of the transfer factors of this point
              const size_t src = (size_t)sy * A.nx + sx;
              const double sux = gin[src], suy = gin[plane + src], sT = gin[2 * plane + src];
              const double r = sqrt(sT * L::inv_TL) * inv_s;
              double gx[Q1], gy[Q1];
              transfer_row_rt<Q1>(i, r, (sux - ux) * inv_s, gx);
              transfer_row_rt<Q1>(j, r, (suy - uy) * inv_s, gy);
              FT acc = FT(0);
#pragma unroll
              for (int ip = 0; ip < Q1; ++ip) {
                FT h = FT(0);
#pragma unroll
                for (int jp = 0; jp < Q1; ++jp) h += FT(gy[jp]) * fin[(size_t)(ip * Q1 + jp) * plane + src];
                acc += FT(gx[ip]) * h;
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
      T1 = A.isothermal ? T : 0.5 * (s * s * (double(e2) + double(e2c)) / rho - (dux * dux + duy * duy));
      if (!(rho1 > 0.0) || !(T1 > 0.0) || !finite(rho1) || !finite(ux1) || !finite(uy1) ||
          !finite(T1)) {
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
      FT H[Q];  // H[i][l] = sum_j Ry[l][j] ft[i][j]
#pragma unroll
      for (int l = 0; l < Q1; ++l) {
        double ry[Q1];
        transfer_row<Q1>(l, r, (uy - uy1) * inv_s1, ry);
#pragma unroll
        for (int i = 0; i < Q1; ++i) {
          FT h = FT(0);
#pragma unroll
          for (int j = 0; j < Q1; ++j) h += FT(ry[j]) * ft[i * Q1 + j];
          H[i * Q1 + l] = h;
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
          for (int i = 0; i < Q1; ++i) fr += FT(rx[i]) * H[i * Q1 + l];
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
    if (__lane_id() == 0) {
      if (nc) atomicAdd(&A.counters->nonconverged, nc);
      if (nb) atomicAdd(&A.counters->bad, nb);
      atomicAdd(&A.counters->sum_passes, sp);
      atomicMax(&A.counters->max_passes, mp);
    }
  }
}

// --------------------------------------------------------------- moments
template <int Q1, class FT>
__global__ void __launch_bounds__(256)
k_moments(int nx, int ny, const FT* __restrict__ f, const double* __restrict__ g,
          double* __restrict__ rho, double* __restrict__ ux, double* __restrict__ uy,
          double* __restrict__ T, double* __restrict__ Mmn) {
  using L = Lat<Q1>;
  const size_t plane = (size_t)nx * ny;
  const size_t node = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= plane) return;
  const double gu = g[node], gv = g[plane + node], gT = g[2 * plane + node];
  const double s = sqrt(gT * L::inv_TL);
  double fl[Q1 * Q1];
#pragma unroll
  for (int p = 0; p < Q1 * Q1; ++p) fl[p] = double(f[(size_t)p * plane + node]);
  double r0 = 0, mx = 0, my = 0, e2 = 0;
#pragma unroll
  for (int i = 0; i < Q1; ++i)
#pragma unroll
    for (int j = 0; j < Q1; ++j) {
      const double fv = fl[i * Q1 + j];
      r0 += fv;
      mx += L::c(i) * fv;
      my += L::c(j) * fv;
      e2 += (L::c(i) * L::c(i) + L::c(j) * L::c(j)) * fv;
    }
  const double du = s * mx / r0, dv = s * my / r0;
  if (rho) rho[node] = r0;
  if (ux) ux[node] = gu + du;
  if (uy) uy[node] = gv + dv;
  if (T) T[node] = 0.5 * (s * s * e2 / r0 - (du * du + dv * dv));
  if (Mmn) {
    // Raw moments of eq. (2): sum_p f_p v_x^m v_y^n.
#pragma unroll
    for (int m = 0; m < Q1; ++m)
#pragma unroll
      for (int n = 0; n < Q1; ++n) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < Q1; ++i) {
          const double vx = s * L::c(i) + gu;
          double px = 1.0;
#pragma unroll
          for (int e = 0; e < m; ++e) px *= vx;
#pragma unroll
          for (int j = 0; j < Q1; ++j) {
            const double vy = s * L::c(j) + gv;
            double py = 1.0;
#pragma unroll
            for (int e = 0; e < n; ++e) py *= vy;
            acc += fl[i * Q1 + j] * px * py;
          }
        }
        Mmn[(size_t)(m * Q1 + n) * plane + node] = acc;
      }
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

template <int Q1, class FT>
hipError_t launch_step_t(const StepArgs& a, hipStream_t s) {
  dim3 block(kBlockX, kBlockY);
  dim3 grid((a.nx + kBlockX - 1) / kBlockX, (a.ny + kBlockY - 1) / kBlockY);
  hipLaunchKernelGGL((k_step<Q1, FT>), grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_init(const pond_config& c, const double* rho, const double* ux,
                       const double* uy, const double* T, void* f, double* g, uint8_t* iters,
                       unsigned long long* bad_count, hipStream_t s) {
  const size_t plane = (size_t)c.nx * c.ny;
  dim3 block(256), grid((unsigned)((plane + 255) / 256));
  const bool f64 = c.precision == POND_F64;
  if (c.q1d == 4) {
    if (f64) hipLaunchKernelGGL((k_init<4, double>), grid, block, 0, s, c.nx, c.ny, rho, ux, uy, T, (double*)f, g, iters, bad_count);
    else hipLaunchKernelGGL((k_init<4, float>), grid, block, 0, s, c.nx, c.ny, rho, ux, uy, T, (float*)f, g, iters, bad_count);
  } else {
    if (f64) hipLaunchKernelGGL((k_init<3, double>), grid, block, 0, s, c.nx, c.ny, rho, ux, uy, T, (double*)f, g, iters, bad_count);
    else hipLaunchKernelGGL((k_init<3, float>), grid, block, 0, s, c.nx, c.ny, rho, ux, uy, T, (float*)f, g, iters, bad_count);
  }
  return hipGetLastError();
}

hipError_t launch_step(const pond_config& c, const StepArgs& a, hipStream_t s) {
  const bool f64 = c.precision == POND_F64;
  if (c.q1d == 4) return f64 ? launch_step_t<4, double>(a, s) : launch_step_t<4, float>(a, s);
  return f64 ? launch_step_t<3, double>(a, s) : launch_step_t<3, float>(a, s);
}

hipError_t launch_moments(const pond_config& c, const void* f, const double* g, double* rho,
                          double* ux, double* uy, double* T, double* Mmn, hipStream_t s) {
  const size_t plane = (size_t)c.nx * c.ny;
  dim3 block(256), grid((unsigned)((plane + 255) / 256));
  const bool f64 = c.precision == POND_F64;
  if (c.q1d == 4) {
    if (f64) hipLaunchKernelGGL((k_moments<4, double>), grid, block, 0, s, c.nx, c.ny, (const double*)f, g, rho, ux, uy, T, Mmn);
    else hipLaunchKernelGGL((k_moments<4, float>), grid, block, 0, s, c.nx, c.ny, (const float*)f, g, rho, ux, uy, T, Mmn);
  } else {
    if (f64) hipLaunchKernelGGL((k_moments<3, double>), grid, block, 0, s, c.nx, c.ny, (const double*)f, g, rho, ux, uy, T, Mmn);
    else hipLaunchKernelGGL((k_moments<3, float>), grid, block, 0, s, c.nx, c.ny, (const float*)f, g, rho, ux, uy, T, Mmn);
  }
  return hipGetLastError();
}

}  // namespace pond
