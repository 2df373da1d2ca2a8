// Internal launch interface between the C ABI (pond_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pond.h"

namespace pond {

// Device counters of one step (reset before the step by a fill kernel).
struct StepCounters {
  unsigned long long nonconverged;
  unsigned long long bad;
  unsigned long long sum_passes;
  unsigned long long max_passes;
};

struct StepArgs {
  int nx, ny;
  int bc_x, bc_y;
  int max_iter, fixed_iter, seed_mode, isothermal;
  int bulk_cap;  // adaptive mode: passes run one lane per node before the
                 // block's unconverged nodes move to the 16-lane tail
                 // (0 or >= max_iter: no tail)
  double tau, eps_abs, eps_rel;
  const void* f_in;
  const double* g_in;
  void* f_out;
  double* g_out;
  uint8_t* iters;
  StepCounters* counters;  // nullable
};

hipError_t launch_init(const pond_config& c, const double* rho, const double* ux,
                       const double* uy, const double* T, void* f, double* g, uint8_t* iters,
                       unsigned long long* bad_count, hipStream_t s);
hipError_t launch_step(const pond_config& c, const StepArgs& a, hipStream_t s);
hipError_t launch_moments(const pond_config& c, const void* f, const double* g, double* rho,
                          double* ux, double* uy, double* T, double* Mmn, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_adjoint(const pond_config& c, const void* f_in, const double* g_in,
                          const uint8_t* iters, const double* adj_f_out, const double* adj_g_out,
                          double* adj_f_in, double* adj_g_in, double* adj_tau, hipStream_t s);

}  // namespace pond
