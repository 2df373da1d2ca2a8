// Internal launch interface between the C ABI (pond_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pond.h"

namespace pond {

// Device counters of one step (reset before the step by a fill kernel):
// totals, then the number of nodes per pass count (index = passes, 0..63).
struct StepCounters {
  unsigned long long nonconverged;
  unsigned long long bad;
  unsigned long long sum_passes;
  unsigned long long max_passes;
  unsigned long long hist[POND_ITERS_MASK + 1];
};
constexpr int kStepCounterWords = (int)(sizeof(StepCounters) / sizeof(unsigned long long));

// Tile queue of the persistent step kernel: blocks take tiles in order from
// `next`; the last block to finish resets both fields to zero, so the queue is
// ready for the next launch on the same stream.
struct TileQueue {
  unsigned next;
  unsigned done;
};

// Device memory the library keeps per (device, stream): the step statistics
// and the tile queue.  Zeroed once when allocated.
struct StreamSlot {
  StepCounters counters;
  TileQueue queue;
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
  TileQueue* queue;
  // Tile order: tiles are taken in the order tile_order[0..ntiles) (nullable:
  // row-major).  Each tile writes its cost key to tile_keys (nullable), and the
  // last block writes the order for the next step, costliest first, to
  // tile_order_next (nullable; may equal tile_order).
  uint16_t* tile_keys;
  const unsigned* tile_order;
  unsigned* tile_order_next;
  // Entries the three tile arrays hold; the kernel uses them only when its
  // tile count fits (the tiles are then taken row-major and not keyed).
  unsigned tile_cap;
  // Pass history for the adjoint (nullable, both or neither).  With N nodes,
  // tape[(k * 4 + c) * N + node] holds for k = 0 the seed gauge (c = 0, 1, 2:
  // u_x, u_y, T) and for k >= 1 the gauge after pass k (c = 0, 1, 2) and the
  // density of pass k (c = 3), for k up to the node's pass count (at most
  // max_iter, or fixed_iter); tape_f[p * N + node] holds population p of the
  // node's last pass, in the gauge of that pass.  Bad nodes leave it unset.
  double* tape;
  double* tape_f;
};

hipError_t launch_init(const pond_config& c, const double* rho, const double* ux,
                       const double* uy, const double* T, void* f, double* g, uint8_t* iters,
                       unsigned long long* bad_count, hipStream_t s);
hipError_t launch_step(const pond_config& c, const StepArgs& a, hipStream_t s);
unsigned step_tile_count(const pond_config& c);
hipError_t launch_moments(const pond_config& c, const void* f, const double* g, double* rho,
                          double* ux, double* uy, double* T, double* Mmn, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
// Transpose of the equilibrium initialisation (eq. (17)): adj_rho = sum_p W_p
// adj_f_p, the gauge cotangents pass through.  Every output is nullable.
hipError_t launch_init_adjoint(const pond_config& c, const double* adj_f, const double* adj_g,
                               double* adj_rho, double* adj_ux, double* adj_uy, double* adj_T,
                               hipStream_t s);
// Adjoint of one step; iters, tape and tape_f are the pass counts and the
// pass history that a step with the same input and configuration recorded
// (tape_slots gauge slots per node: nodes with more passes get no derivative).
hipError_t launch_adjoint(const pond_config& c, const void* f_in, const double* g_in,
                          const uint8_t* iters, const double* tape, const double* tape_f,
                          int tape_slots, const double* adj_f_out, const double* adj_g_out,
                          double* adj_f_in, double* adj_g_in, double* adj_tau, TileQueue* queue,
                          hipStream_t s);

}  // namespace pond
