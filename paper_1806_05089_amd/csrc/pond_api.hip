// C ABI of libpond: argument checks, buffer ping-pong and kernel launches.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <string>

#include "pond.h"
#include "pond_internal.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(POND_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Device memory kept per (device, stream): step statistics, the step
// kernel's tile queue, and the tile cost keys and tile order that one step
// leaves for the next (a scheduling hint: results do not depend on it).  Work
// on one stream runs in order, so a slot is never used by two kernels at
// once.  Allocated on the first call on a stream (the arrays grow with the
// grid) and held until the process ends.
struct Slot {
  pond::StreamSlot* dev = nullptr;
  uint16_t* keys = nullptr;
  unsigned* order = nullptr;
  size_t cap = 0;           // tiles the arrays hold
  int order_nx = -1;        // grid and tile count whose tile order `order` holds
  int order_ny = -1;
  unsigned order_tiles = 0;
};
std::mutex g_mutex;
std::map<std::pair<int, void*>, Slot> g_slots;

int slot_for_stream(hipStream_t s, Slot** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_mutex);
  Slot& sl = g_slots[std::make_pair(dev, static_cast<void*>(s))];
  if (!sl.dev) {
    pond::StreamSlot* p = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&p), sizeof(pond::StreamSlot));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(stream slot)");
    e = hipMemset(p, 0, sizeof(pond::StreamSlot));
    if (e != hipSuccess) {
      (void)hipFree(p);
      return hip_fail(e, "hipMemset(stream slot)");
    }
    sl.dev = p;
  }
  *out = &sl;
  return POND_OK;
}

// Tile key and order arrays for `ntiles` tiles.  Growing them waits for the
// stream, since a kernel in flight may still use the old arrays.
int ensure_tile_arrays(Slot* sl, size_t ntiles, hipStream_t s) {
  if (sl->cap >= ntiles) return POND_OK;
  hipError_t e;
  if (sl->cap) {
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "pond_step sync");
    (void)hipFree(sl->keys);
    (void)hipFree(sl->order);
    sl->keys = nullptr;
    sl->order = nullptr;
    sl->cap = 0;
  }
  sl->order_nx = sl->order_ny = -1;
  e = hipMalloc(reinterpret_cast<void**>(&sl->keys), ntiles * sizeof(uint16_t));
  if (e == hipSuccess)
    e = hipMalloc(reinterpret_cast<void**>(&sl->order), ntiles * sizeof(unsigned));
  if (e != hipSuccess) {
    (void)hipFree(sl->keys);
    sl->keys = nullptr;
    sl->order = nullptr;
    return hip_fail(e, "hipMalloc(tile arrays)");
  }
  sl->cap = ntiles;
  return POND_OK;
}

// Passes a node runs one lane per node before an unconverged node moves to the
// block's 16-lane tail (POND_BULK_CAP overrides the default).  From sweeps on
// the 1024^2 Riemann flow: D2Q16 FP64 7, D2Q9 FP64 9, FP32-mixed 5.
int bulk_cap(const pond_config& c) {
  static int env = [] {
    const char* e = getenv("POND_BULK_CAP");
    return e ? atoi(e) : -1;
  }();
  if (env >= 0) return env;
  if (c.precision != POND_F64) return 5;
  return c.q1d == 3 ? 9 : 7;
}

size_t f_bytes(const pond_config& c) {
  const size_t plane = (size_t)c.nx * c.ny;
  return plane * c.q1d * c.q1d * (c.precision == POND_F64 ? sizeof(double) : sizeof(float));
}
size_t g_bytes(const pond_config& c) { return (size_t)c.nx * c.ny * 3 * sizeof(double); }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

int check_config(const pond_config* c) {
  if (!c) return fail(POND_E_NULL, "config is NULL");
  if (c->nx < 1 || c->ny < 1) return fail(POND_E_INVALID, "nx and ny must be >= 1");
  if ((long long)c->nx * c->ny > (1ll << 31))
    return fail(POND_E_INVALID, "grid larger than 2^31 nodes");
  if (c->q1d != 3 && c->q1d != 4) return fail(POND_E_INVALID, "q1d must be 3 (D2Q9) or 4 (D2Q16)");
  if (c->precision != POND_F64 && c->precision != POND_F32_MIXED)
    return fail(POND_E_INVALID, "precision must be POND_F64 or POND_F32_MIXED");
  if (c->isothermal != 0 && c->isothermal != 1) return fail(POND_E_INVALID, "isothermal must be 0 or 1");
  if ((c->bc_x != POND_PERIODIC && c->bc_x != POND_ZERO_GRADIENT) ||
      (c->bc_y != POND_PERIODIC && c->bc_y != POND_ZERO_GRADIENT))
    return fail(POND_E_INVALID, "bc must be POND_PERIODIC or POND_ZERO_GRADIENT");
  if (c->max_iter < 1 || c->max_iter > POND_ITERS_MASK)
    return fail(POND_E_INVALID, "max_iter must be in 1..63");
  if (c->fixed_iter < 0 || c->fixed_iter > POND_ITERS_MASK)
    return fail(POND_E_INVALID, "fixed_iter must be in 0..63");
  if (c->seed_mode < 0 || c->seed_mode > 2) return fail(POND_E_INVALID, "seed_mode must be 0, 1 or 2");
  if (!(c->tau > 0.0) || !(c->tau < 1e30)) return fail(POND_E_INVALID, "tau must be finite and > 0");
  if (!(c->eps_abs >= 0.0) || !(c->eps_rel >= 0.0))
    return fail(POND_E_INVALID, "eps_abs and eps_rel must be >= 0");
  return POND_OK;
}

// Calls that run the step: in FP32-mixed mode with adaptive passes the App. E
// tolerances must be reachable in FP32 (the FP64 defaults would run every
// node to max_iter).
int check_step_tolerances(const pond_config* c, const char* who) {
  constexpr double kEpsF32 = 1.1920928955078125e-07;  // 2^-23
  if (c->precision == POND_F32_MIXED && c->fixed_iter == 0 &&
      !(c->eps_abs >= kEpsF32 || c->eps_rel >= kEpsF32))
    return fail(POND_E_INVALID, std::string(who) +
                                    ": FP32-mixed adaptive passes need max(eps_abs, eps_rel) >= "
                                    "2^-23 (FP32 resolution), e.g. 1e-6 / 1e-5");
  return POND_OK;
}

// Arguments of one step launch on a slot's queue and tile arrays (the state
// buffers, counters and pass history are set by the caller).
pond::StepArgs step_args(const pond_config& c, Slot* slot) {
  pond::StepArgs a;
  a.nx = c.nx;
  a.ny = c.ny;
  a.bc_x = c.bc_x;
  a.bc_y = c.bc_y;
  a.max_iter = c.max_iter;
  a.fixed_iter = c.fixed_iter;
  a.seed_mode = c.seed_mode;
  a.isothermal = c.isothermal;
  a.bulk_cap = bulk_cap(c);
  a.tau = c.tau;
  a.eps_abs = c.eps_abs;
  a.eps_rel = c.eps_rel;
  a.f_in = nullptr;
  a.g_in = nullptr;
  a.f_out = nullptr;
  a.g_out = nullptr;
  a.iters = nullptr;
  a.counters = nullptr;
  a.queue = &slot->dev->queue;
  a.tile_keys = slot->keys;
  a.tile_order = nullptr;
  a.tile_order_next = slot->order;
  a.tile_cap = (unsigned)slot->cap;
  a.tape = nullptr;
  a.tape_f = nullptr;
  return a;
}

// Launches one step; the tile order left by the previous step on the stream is
// used when it belongs to the same grid and tile count (the tile shape depends
// on the precision and the lattice).
hipError_t launch_step_on(const pond_config& c, Slot* slot, pond::StepArgs& a, hipStream_t s) {
  const unsigned ntiles = pond::step_tile_count(c);
  const bool ordered =
      slot->order_nx == c.nx && slot->order_ny == c.ny && slot->order_tiles == ntiles;
  a.tile_order = ordered ? slot->order : nullptr;
  const hipError_t e = pond::launch_step(c, a, s);
  if (e != hipSuccess) {
    slot->order_nx = slot->order_ny = -1;
    return e;
  }
  slot->order_nx = c.nx;
  slot->order_ny = c.ny;
  slot->order_tiles = ntiles;
  return hipSuccess;
}

// Pass history of one step (layout of StepArgs::tape / tape_f, one block):
// (kslots * 4 + Q) * N doubles, kslots = 1 + the most passes a node can take.
struct TapeLayout {
  int kslots;
  size_t tape_f_offset;  // bytes
  size_t total;          // bytes
};
TapeLayout tape_layout(const pond_config& c) {
  TapeLayout t;
  const size_t plane = (size_t)c.nx * c.ny;
  t.kslots = 1 + (c.fixed_iter > 0 ? c.fixed_iter : c.max_iter);
  t.tape_f_offset = (size_t)t.kslots * 4 * plane * sizeof(double);
  t.total = t.tape_f_offset + (size_t)c.q1d * c.q1d * plane * sizeof(double);
  return t;
}

// Caller workspace of pond_step_adjoint: the recorded step's pass history,
// then its output state (f, g, iters), each part aligned to 256 bytes.
struct AdjointWorkspace {
  size_t f_offset, g_offset, iters_offset, total;  // bytes
};
AdjointWorkspace adjoint_workspace(const pond_config& c) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  AdjointWorkspace w;
  w.f_offset = up(tape_layout(c).total);
  w.g_offset = w.f_offset + up(f_bytes(c));
  w.iters_offset = w.g_offset + up(g_bytes(c));
  w.total = w.iters_offset + up((size_t)c.nx * c.ny);
  return w;
}

// One step from (in_f, in_g) with its pass history written to `tape`.
hipError_t record_step(const pond_config& c, Slot* slot, const void* in_f, const double* in_g,
                       void* out_f, double* out_g, uint8_t* out_iters, char* tape,
                       hipStream_t s) {
  pond::StepArgs a = step_args(c, slot);
  a.f_in = in_f;
  a.g_in = in_g;
  a.f_out = out_f;
  a.g_out = out_g;
  a.iters = out_iters;
  a.tape = reinterpret_cast<double*>(tape);
  a.tape_f = reinterpret_cast<double*>(tape + tape_layout(c).tape_f_offset);
  return launch_step_on(c, slot, a, s);
}

// adj_in must not overlap the adjoint's inputs (nor the tape, if given).
int check_adjoint_aliasing(const pond_config& c, const pond_state* in, const pond_state* adj_out,
                           const pond_state* adj_in, const void* tape) {
  const size_t plane = (size_t)c.nx * c.ny;
  const size_t afb = plane * c.q1d * c.q1d * sizeof(double), agb = g_bytes(c);
  const size_t fb = f_bytes(c), tb = tape_layout(c).total;
  if (overlap(adj_in->f, afb, adj_out->f, afb) || overlap(adj_in->g, agb, adj_out->g, agb) ||
      overlap(adj_in->f, afb, in->f, fb) || overlap(adj_in->g, agb, in->g, agb) ||
      overlap(adj_in->f, afb, adj_in->g, agb) ||
      (tape && (overlap(adj_in->f, afb, tape, tb) || overlap(adj_in->g, agb, tape, tb))))
    return fail(POND_E_ALIAS, "pond_step_adjoint: adj_in overlaps another buffer");
  return POND_OK;
}

// The adjoint kernel on a recorded step (pass counts `iters`, history `tape`).
int launch_adjoint_on(const pond_config& c, Slot* slot, const pond_state* in,
                      const uint8_t* iters, const char* tape, const pond_state* adj_out,
                      pond_state* adj_in, double* adj_tau, hipStream_t s) {
  const TapeLayout t = tape_layout(c);
  const hipError_t e = pond::launch_adjoint(
      c, in->f, in->g, iters, reinterpret_cast<const double*>(tape),
      reinterpret_cast<const double*>(tape + t.tape_f_offset), t.kslots,
      (const double*)adj_out->f, adj_out->g, (double*)adj_in->f, adj_in->g, adj_tau,
      &slot->dev->queue, s);
  if (e == hipErrorNotSupported) return fail(POND_E_UNSUPPORTED, "pond_step_adjoint: not available");
  if (e != hipSuccess) return hip_fail(e, "pond_step_adjoint launch");
  return POND_OK;
}

// ---- scratch of pond_step_noalloc: one fixed device array per GPU ----
// Layout: step counters at 0, the tile queue at 1 KiB, the tile cost keys at
// 2 KiB (uint16 per tile), the tile order after them (uint32 per tile).
constexpr size_t kNoAllocTiles = 65536;  // 4096^2 in both precisions
constexpr size_t kScratchQueue = 1024;
constexpr size_t kScratchKeys = 2048;
constexpr size_t kScratchOrder = kScratchKeys + kNoAllocTiles * sizeof(uint16_t);
constexpr size_t kScratchBytes = kScratchOrder + kNoAllocTiles * sizeof(unsigned);
static_assert(sizeof(pond::StepCounters) <= kScratchQueue, "counters fit their part");
static_assert(sizeof(pond::TileQueue) <= kScratchKeys - kScratchQueue, "queue fits its part");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per device: the scratch array's device address (from hipGetSymbolAddress;
// the array's name is a host-side stand-in, never a device address) and the
// grid whose tile order the array holds.
struct NoAllocDevice {
  char* ptr = nullptr;
  int order_nx = -1, order_ny = -1;
  unsigned order_tiles = 0;
};
std::mutex g_noalloc_mutex;
std::map<int, NoAllocDevice> g_noalloc;

int noalloc_scratch(NoAllocDevice** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_noalloc_mutex);
  NoAllocDevice& d = g_noalloc[dev];
  if (!d.ptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    d.ptr = static_cast<char*>(p);
  }
  *out = &d;
  return POND_OK;
}

}  // namespace

extern "C" {

const char* pond_last_error(void) { return g_last_error.c_str(); }

int pond_abi_version(void) { return 201; }

int pond_init(const pond_config* cfg, const double* rho, const double* ux, const double* uy,
              const double* T, pond_state* out, void* hip_stream) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!rho || !ux || !uy || !T) return fail(POND_E_NULL, "pond_init: a field pointer is NULL");
  if (!out || !out->f || !out->g) return fail(POND_E_NULL, "pond_init: output state is NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Slot* slot = nullptr;
  if ((rc = slot_for_stream(s, &slot))) return rc;
  pond::StepCounters* cnt = &slot->dev->counters;
  hipError_t e = pond::launch_zero_u64(&cnt->bad, 1, s);
  if (e != hipSuccess) return hip_fail(e, "pond_init zero");
  e = pond::launch_init(*cfg, rho, ux, uy, T, out->f, out->g, out->iters, &cnt->bad, s);
  if (e != hipSuccess) return hip_fail(e, "pond_init launch");
  unsigned long long bad = 0;
  e = hipMemcpyAsync(&bad, &cnt->bad, sizeof(bad), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "pond_init copy");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "pond_init sync");
  if (bad) {
    char buf[128];
    snprintf(buf, sizeof(buf), "pond_init: %llu nodes with rho <= 0, T <= 0 or non-finite values", bad);
    return fail(POND_E_STATE, buf);
  }
  return POND_OK;
}

int pond_step(const pond_config* cfg, pond_state* in, pond_state* out, int32_t nsteps,
              void* hip_stream, pond_stats* stats) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if ((rc = check_step_tolerances(cfg, "pond_step"))) return rc;
  if (!in || !out || !in->f || !in->g || !out->f || !out->g)
    return fail(POND_E_NULL, "pond_step: a state buffer is NULL");
  if (nsteps < 1) return fail(POND_E_INVALID, "pond_step: nsteps must be >= 1");
  const size_t fb = f_bytes(*cfg), gb = g_bytes(*cfg);
  if (overlap(in->f, fb, out->f, fb) || overlap(in->g, gb, out->g, gb) ||
      overlap(in->f, fb, out->g, gb) || overlap(in->g, gb, out->f, fb))
    return fail(POND_E_ALIAS, "pond_step: input and output state overlap");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Slot* slot = nullptr;
  if ((rc = slot_for_stream(s, &slot))) return rc;
  pond::StepCounters* cnt = stats ? &slot->dev->counters : nullptr;
  if ((rc = ensure_tile_arrays(slot, pond::step_tile_count(*cfg), s))) return rc;

  pond::StepArgs a = step_args(*cfg, slot);
  a.iters = out->iters;

  const void* src_f = in->f;
  const double* src_g = in->g;
  hipError_t e;
  for (int k = 0; k < nsteps; ++k) {
    const bool to_out = (k % 2 == 0);
    void* dst_f = to_out ? out->f : in->f;
    double* dst_g = to_out ? out->g : in->g;
    const bool last = (k == nsteps - 1);
    a.f_in = src_f;
    a.g_in = src_g;
    a.f_out = dst_f;
    a.g_out = dst_g;
    a.counters = (last && cnt) ? cnt : nullptr;
    if (a.counters) {
      e = pond::launch_zero_u64(reinterpret_cast<unsigned long long*>(cnt),
                                pond::kStepCounterWords, s);
      if (e != hipSuccess) return hip_fail(e, "pond_step zero counters");
    }
    e = launch_step_on(*cfg, slot, a, s);
    if (e != hipSuccess) return hip_fail(e, "pond_step launch");
    src_f = dst_f;
    src_g = dst_g;
  }
  if (nsteps % 2 == 0) {
    // The last step wrote `in`; move the result to `out`.
    e = hipMemcpyAsync(out->f, in->f, fb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out->g, in->g, gb, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "pond_step final copy");
  }
  if (stats) {
    pond::StepCounters h;
    e = hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pond_step stats");
    stats->nonconverged = (int64_t)h.nonconverged;
    stats->bad_state = (int64_t)h.bad;
    stats->max_iters = (int32_t)h.max_passes;
    stats->mean_iters = (double)h.sum_passes / ((double)cfg->nx * cfg->ny);
    for (int k = 0; k <= POND_ITERS_MASK; ++k) stats->iter_hist[k] = (int64_t)h.hist[k];
  }
  return POND_OK;
}

int pond_moments(const pond_config* cfg, const pond_state* state, double* rho, double* ux,
                 double* uy, double* T, double* Mmn, void* hip_stream) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!state || !state->f || !state->g) return fail(POND_E_NULL, "pond_moments: state is NULL");
  hipError_t e = pond::launch_moments(*cfg, state->f, state->g, rho, ux, uy, T, Mmn,
                                      static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "pond_moments launch");
  return POND_OK;
}

int pond_tape_bytes(const pond_config* cfg, int64_t* bytes) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!bytes) return fail(POND_E_NULL, "pond_tape_bytes: bytes is NULL");
  *bytes = (int64_t)tape_layout(*cfg).total;
  return POND_OK;
}

int pond_step_record(const pond_config* cfg, const pond_state* in, pond_state* out, void* tape,
                     void* hip_stream) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if ((rc = check_step_tolerances(cfg, "pond_step_record"))) return rc;
  if (!in || !out || !in->f || !in->g || !out->f || !out->g || !out->iters || !tape)
    return fail(POND_E_NULL, "pond_step_record: a required buffer is NULL");
  const size_t fb = f_bytes(*cfg), gb = g_bytes(*cfg), plane = (size_t)cfg->nx * cfg->ny;
  const size_t tb = tape_layout(*cfg).total;
  if (overlap(in->f, fb, out->f, fb) || overlap(in->g, gb, out->g, gb) ||
      overlap(in->f, fb, out->g, gb) || overlap(in->g, gb, out->f, fb) ||
      overlap(tape, tb, in->f, fb) || overlap(tape, tb, in->g, gb) ||
      overlap(tape, tb, out->f, fb) || overlap(tape, tb, out->g, gb) ||
      overlap(tape, tb, out->iters, plane))
    return fail(POND_E_ALIAS, "pond_step_record: buffers overlap");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Slot* slot = nullptr;
  if ((rc = slot_for_stream(s, &slot))) return rc;
  if ((rc = ensure_tile_arrays(slot, pond::step_tile_count(*cfg), s))) return rc;
  const hipError_t e = record_step(*cfg, slot, in->f, in->g, out->f, out->g, out->iters,
                                   static_cast<char*>(tape), s);
  if (e != hipSuccess) return hip_fail(e, "pond_step_record launch");
  return POND_OK;
}

int pond_step_adjoint_recorded(const pond_config* cfg, const pond_state* in,
                               const pond_state* out_fwd, const void* tape,
                               const pond_state* adj_out, pond_state* adj_in, double* adj_tau,
                               void* hip_stream) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if ((rc = check_step_tolerances(cfg, "pond_step_adjoint_recorded"))) return rc;
  if (!in || !out_fwd || !tape || !adj_out || !adj_in || !in->f || !in->g || !out_fwd->iters ||
      !adj_out->f || !adj_out->g || !adj_in->f || !adj_in->g)
    return fail(POND_E_NULL, "pond_step_adjoint_recorded: a required buffer is NULL");
  if ((rc = check_adjoint_aliasing(*cfg, in, adj_out, adj_in, tape))) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Slot* slot = nullptr;
  if ((rc = slot_for_stream(s, &slot))) return rc;
  return launch_adjoint_on(*cfg, slot, in, out_fwd->iters, static_cast<const char*>(tape),
                           adj_out, adj_in, adj_tau, s);
}

int pond_workspace_bytes(const pond_config* cfg, int32_t op, int64_t* bytes) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!bytes) return fail(POND_E_NULL, "pond_workspace_bytes: bytes is NULL");
  if (op == POND_OP_STEP) {
    *bytes = 0;
  } else if (op == POND_OP_STEP_ADJOINT) {
    *bytes = (int64_t)adjoint_workspace(*cfg).total;
  } else {
    return fail(POND_E_INVALID, "pond_workspace_bytes: op must be POND_OP_STEP or POND_OP_STEP_ADJOINT");
  }
  return POND_OK;
}

int pond_step_adjoint(const pond_config* cfg, const pond_state* in, const pond_state* out_fwd,
                      const pond_state* adj_out, pond_state* adj_in, double* adj_tau,
                      void* workspace, int64_t workspace_bytes, void* hip_stream) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if ((rc = check_step_tolerances(cfg, "pond_step_adjoint"))) return rc;
  if (!in || !out_fwd || !adj_out || !adj_in || !in->f || !in->g || !out_fwd->iters ||
      !adj_out->f || !adj_out->g || !adj_in->f || !adj_in->g || !workspace)
    return fail(POND_E_NULL, "pond_step_adjoint: a required buffer is NULL");
  const AdjointWorkspace w = adjoint_workspace(*cfg);
  if (workspace_bytes < 0 || (size_t)workspace_bytes < w.total)
    return fail(POND_E_INVALID, "pond_step_adjoint: workspace smaller than "
                                "pond_workspace_bytes(cfg, POND_OP_STEP_ADJOINT)");
  if (reinterpret_cast<uintptr_t>(workspace) % 16 != 0)
    return fail(POND_E_INVALID, "pond_step_adjoint: workspace must be 16-byte aligned");
  if ((rc = check_adjoint_aliasing(*cfg, in, adj_out, adj_in, nullptr))) return rc;
  const size_t fb = f_bytes(*cfg), gb = g_bytes(*cfg);
  const size_t afb = (size_t)cfg->nx * cfg->ny * cfg->q1d * cfg->q1d * sizeof(double);
  if (overlap(workspace, w.total, in->f, fb) || overlap(workspace, w.total, in->g, gb) ||
      overlap(workspace, w.total, adj_out->f, afb) || overlap(workspace, w.total, adj_out->g, gb) ||
      overlap(workspace, w.total, adj_in->f, afb) || overlap(workspace, w.total, adj_in->g, gb))
    return fail(POND_E_ALIAS, "pond_step_adjoint: workspace overlaps another buffer");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Slot* slot = nullptr;
  if ((rc = slot_for_stream(s, &slot))) return rc;
  if ((rc = ensure_tile_arrays(slot, pond::step_tile_count(*cfg), s))) return rc;
  // The step is run again with its pass history recorded (it reproduces
  // out_fwd bit for bit) into the caller's workspace: tape, output state.
  char* m = static_cast<char*>(workspace);
  void* sf = m + w.f_offset;
  double* sg = reinterpret_cast<double*>(m + w.g_offset);
  uint8_t* siters = reinterpret_cast<uint8_t*>(m + w.iters_offset);
  const hipError_t e = record_step(*cfg, slot, in->f, in->g, sf, sg, siters, m, s);
  if (e != hipSuccess) return hip_fail(e, "pond_step_adjoint step launch");
  return launch_adjoint_on(*cfg, slot, in, siters, m, adj_out, adj_in, adj_tau, s);
}

int pond_init_adjoint(const pond_config* cfg, const double* adj_f, const double* adj_g,
                      double* adj_rho, double* adj_ux, double* adj_uy, double* adj_T,
                      void* hip_stream) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!adj_f || !adj_g) return fail(POND_E_NULL, "pond_init_adjoint: adj_f or adj_g is NULL");
  const size_t plane = (size_t)cfg->nx * cfg->ny;
  const size_t afb = plane * cfg->q1d * cfg->q1d * sizeof(double), agb = g_bytes(*cfg);
  double* outs[4] = {adj_rho, adj_ux, adj_uy, adj_T};
  for (double* o : outs)
    if (o && (overlap(o, plane * sizeof(double), adj_f, afb) ||
              overlap(o, plane * sizeof(double), adj_g, agb)))
      return fail(POND_E_ALIAS, "pond_init_adjoint: an output overlaps adj_f or adj_g");
  const hipError_t e = pond::launch_init_adjoint(*cfg, adj_f, adj_g, adj_rho, adj_ux, adj_uy,
                                                 adj_T, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "pond_init_adjoint launch");
  return POND_OK;
}

int pond_step_noalloc(const pond_config* cfg, pond_state* in, pond_state* out, int32_t nsteps,
                      void* hip_stream, pond_stats* stats) {
  g_last_error.clear();
  int rc = check_config(cfg);
  if (rc) return rc;
  if ((rc = check_step_tolerances(cfg, "pond_step_noalloc"))) return rc;
  if (!in || !out || !in->f || !in->g || !out->f || !out->g)
    return fail(POND_E_NULL, "pond_step_noalloc: a state buffer is NULL");
  if (nsteps < 1) return fail(POND_E_INVALID, "pond_step_noalloc: nsteps must be >= 1");
  const unsigned ntiles = pond::step_tile_count(*cfg);
  if (ntiles > kNoAllocTiles) {
    char buf[160];
    snprintf(buf, sizeof(buf),
             "pond_step_noalloc: %u step tiles exceed the fixed scratch (%zu tiles: 4096 x 4096 "
             "nodes); use pond_step", ntiles, kNoAllocTiles);
    return fail(POND_E_INVALID, buf);
  }
  const size_t fb = f_bytes(*cfg), gb = g_bytes(*cfg);
  if (overlap(in->f, fb, out->f, fb) || overlap(in->g, gb, out->g, gb) ||
      overlap(in->f, fb, out->g, gb) || overlap(in->g, gb, out->f, fb))
    return fail(POND_E_ALIAS, "pond_step_noalloc: input and output state overlap");
  NoAllocDevice* d = nullptr;
  if ((rc = noalloc_scratch(&d))) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  pond::StepCounters* cnt = reinterpret_cast<pond::StepCounters*>(d->ptr);
  pond::TileQueue* queue = reinterpret_cast<pond::TileQueue*>(d->ptr + kScratchQueue);
  // The array keeps the last call's contents: the queue must start empty.
  hipError_t e = pond::launch_zero_u64(reinterpret_cast<unsigned long long*>(queue), 1, s);
  if (e != hipSuccess) return hip_fail(e, "pond_step_noalloc zero queue");

  pond::StepArgs a;
  a.nx = cfg->nx;
  a.ny = cfg->ny;
  a.bc_x = cfg->bc_x;
  a.bc_y = cfg->bc_y;
  a.max_iter = cfg->max_iter;
  a.fixed_iter = cfg->fixed_iter;
  a.seed_mode = cfg->seed_mode;
  a.isothermal = cfg->isothermal;
  a.bulk_cap = bulk_cap(*cfg);
  a.tau = cfg->tau;
  a.eps_abs = cfg->eps_abs;
  a.eps_rel = cfg->eps_rel;
  a.iters = out->iters;
  a.queue = queue;
  a.tile_keys = reinterpret_cast<uint16_t*>(d->ptr + kScratchKeys);
  a.tile_order_next = reinterpret_cast<unsigned*>(d->ptr + kScratchOrder);
  a.tile_cap = (unsigned)kNoAllocTiles;
  a.tape = nullptr;
  a.tape_f = nullptr;

  const void* src_f = in->f;
  const double* src_g = in->g;
  for (int k = 0; k < nsteps; ++k) {
    const bool to_out = (k % 2 == 0);
    void* dst_f = to_out ? out->f : in->f;
    double* dst_g = to_out ? out->g : in->g;
    a.f_in = src_f;
    a.g_in = src_g;
    a.f_out = dst_f;
    a.g_out = dst_g;
    a.counters = (k == nsteps - 1 && stats) ? cnt : nullptr;
    if (a.counters) {
      e = pond::launch_zero_u64(reinterpret_cast<unsigned long long*>(cnt),
                                pond::kStepCounterWords, s);
      if (e != hipSuccess) return hip_fail(e, "pond_step_noalloc zero counters");
    }
    {
      // the order left in the array is a permutation of this grid's tiles
      // only if the last call on this device had the same grid and tile count
      std::lock_guard<std::mutex> lock(g_noalloc_mutex);
      const bool ordered = d->order_nx == cfg->nx && d->order_ny == cfg->ny &&
                           d->order_tiles == ntiles;
      a.tile_order = ordered ? a.tile_order_next : nullptr;
      e = pond::launch_step(*cfg, a, s);
      d->order_nx = e == hipSuccess ? cfg->nx : -1;
      d->order_ny = e == hipSuccess ? cfg->ny : -1;
      d->order_tiles = ntiles;
    }
    if (e != hipSuccess) return hip_fail(e, "pond_step_noalloc launch");
    src_f = dst_f;
    src_g = dst_g;
  }
  if (nsteps % 2 == 0) {
    e = hipMemcpyAsync(out->f, in->f, fb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out->g, in->g, gb, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "pond_step_noalloc final copy");
  }
  if (stats) {
    pond::StepCounters h;
    e = hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pond_step_noalloc stats");
    stats->nonconverged = (int64_t)h.nonconverged;
    stats->bad_state = (int64_t)h.bad;
    stats->max_iters = (int32_t)h.max_passes;
    stats->mean_iters = (double)h.sum_passes / ((double)cfg->nx * cfg->ny);
    for (int k = 0; k <= POND_ITERS_MASK; ++k) stats->iter_hist[k] = (int64_t)h.hist[k];
  }
  return POND_OK;
}

}  // extern "C"
