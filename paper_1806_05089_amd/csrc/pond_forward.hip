// Bandwidth-bound kernels around the PonD step on gfx950: equilibrium
// initialisation, macroscopic moments and a counter fill.
//
// Layout in HBM: structure-of-arrays planes, row-major [ny][nx]:
//   f[p][y][x], p = i*q + j   populations in the node's own gauge (FT)
//   g[k][y][x], k = ux, uy, T the node's gauge (double)
#include <hip/hip_runtime.h>
#include <math.h>

#include "pond_device.hpp"
#include "pond_internal.hpp"

namespace pond {
namespace {

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

// ------------------------------------------------ transpose of the init
// f_p = rho W_p (eq. (17)) is linear in rho and does not depend on the gauge
// (the populations live in the node's own gauge), so the cotangent of rho is
// the W-weighted sum of the population cotangents and the gauge cotangents
// are those of g.
template <int Q1>
__global__ void __launch_bounds__(256)
k_init_adjoint(size_t plane, const double* __restrict__ adj_f, const double* __restrict__ adj_g,
               double* __restrict__ adj_rho, double* __restrict__ adj_ux,
               double* __restrict__ adj_uy, double* __restrict__ adj_T) {
  const size_t node = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= plane) return;
  if (adj_rho) {
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < Q1; ++i)
#pragma unroll
      for (int j = 0; j < Q1; ++j)
        a = fma(Lat<Q1>::w(i) * Lat<Q1>::w(j), adj_f[(size_t)(i * Q1 + j) * plane + node], a);
    adj_rho[node] = a;
  }
  if (adj_ux) adj_ux[node] = adj_g[node];
  if (adj_uy) adj_uy[node] = adj_g[plane + node];
  if (adj_T) adj_T[node] = adj_g[2 * plane + node];
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
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

hipError_t launch_init_adjoint(const pond_config& c, const double* adj_f, const double* adj_g,
                               double* adj_rho, double* adj_ux, double* adj_uy, double* adj_T,
                               hipStream_t s) {
  const size_t plane = (size_t)c.nx * c.ny;
  dim3 block(256), grid((unsigned)((plane + 255) / 256));
  if (c.q1d == 4)
    hipLaunchKernelGGL((k_init_adjoint<4>), grid, block, 0, s, plane, adj_f, adj_g, adj_rho,
                       adj_ux, adj_uy, adj_T);
  else
    hipLaunchKernelGGL((k_init_adjoint<3>), grid, block, 0, s, plane, adj_f, adj_g, adj_rho,
                       adj_ux, adj_uy, adj_T);
  return hipGetLastError();
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
