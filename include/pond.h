/*
 * libpond -- C ABI of the Particles-on-Demand (PonD) time step on AMD gfx950.
 *
 * The method is that of Dorschner, Boesch and Karlin, "Particles-on-Demand for
 * Kinetic Theory" (arXiv:1806.05089).  The state of the solver is, at every
 * node of an equidistant periodic or bounded 2-D mesh (dx = dt = 1, App. C and
 * the statement that dt = 1 is used throughout), the Q populations expressed in
 * the node's own gauge lambda = {u, T} together with that gauge (main text,
 * definition of f^lambda and of the limit gauge, eqs. (13)-(16)).
 *
 * Speed sets are tensor products of q one-dimensional speeds: q = 4 (D2Q16,
 * roots of the probabilists' Hermite polynomial He_4, T_L = 1) or q = 3 (D2Q9
 * of App. A, T_L = 1/3).  Population p = i*q + j carries the speed (c_i, c_j).
 *
 * Conventions shared by every call:
 *   - All array arguments are DEVICE pointers owned by the caller, laid out as
 *     structure-of-arrays planes, row-major [ny][nx] (x fastest).
 *   - Every call is asynchronous on the given hipStream_t (passed as void*;
 *     NULL = the default stream) unless stated otherwise.
 *   - Return value: POND_OK (0) on success, a negative POND_E_* code otherwise;
 *     pond_last_error() then returns a message (thread-local).  A failed
 *     argument check launches nothing.
 *   - Physical failures inside a step (no convergence, T <= 0, rho <= 0,
 *     non-finite values) are not errors: they are counted in pond_stats and
 *     marked in the per-node iteration plane.
 *   - Library-held device memory: the first pond_init / pond_step /
 *     pond_step_adjoint on a (device, stream) pair allocates and zeroes a small
 *     slot for it (step statistics, the step kernel's tile queue, and one cost
 *     key and one order entry per tile of 32 x 16 nodes for D2Q16 in FP64,
 *     32 x 8 otherwise: 6 bytes per tile, 12-24 KiB at 1024^2, grown after a
 *     stream synchronisation when a larger grid appears); it is held until the
 *     process ends.  A step leaves its tiles' costs there, and the next step
 *     on the same stream takes the costliest tiles first: a scheduling hint
 *     only, results do not depend on that order (every call is a pure
 *     function of its inputs).  Scratch of a size that grows with the grid
 *     and the pass cap (the adjoint's) is the caller's: see
 *     pond_workspace_bytes.  Calls on one stream run in order; concurrent
 *     calls on different streams use different slots.
 *   - HIP graph capture: pond_step (without stats) and pond_step_adjoint
 *     record kernels and device copies only, no memset.  Make one call on the
 *     capturing stream before capture (it allocates the stream's slot) and
 *     capture at most the grid size used then.
 */
#ifndef POND_H_
#define POND_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  POND_OK = 0,
  POND_E_INVALID = -1,     /* a configuration value is out of range           */
  POND_E_NULL = -2,        /* a required pointer is NULL                      */
  POND_E_ALIAS = -3,       /* input and output buffers overlap                */
  POND_E_STATE = -4,       /* pond_init found rho <= 0, T <= 0 or non-finite  */
  POND_E_HIP = -5,         /* a HIP runtime call failed                       */
  POND_E_UNSUPPORTED = -6  /* valid request that the library does not provide */
};

enum { POND_F64 = 0, POND_F32_MIXED = 1 };
enum { POND_OP_STEP = 0, POND_OP_STEP_ADJOINT = 1 }; /* pond_workspace_bytes */
enum { POND_PERIODIC = 0, POND_ZERO_GRADIENT = 1 };

/* Bits of the per-node iteration plane written by pond_step. */
#define POND_ITERS_MASK 0x3F        /* predictor-corrector passes, 1..63        */
#define POND_ITERS_NONCONVERGED 0x40 /* the pass cap was hit before App. E's test */
#define POND_ITERS_BAD 0x80          /* rho <= 0, T <= 0 or non-finite: output NaN */

typedef struct {
  int32_t nx, ny;     /* nodes per axis, >= 1                                   */
  int32_t q1d;        /* 4: D2Q16; 3: D2Q9 (App. A)                             */
  int32_t precision;  /* POND_F64: f in double; POND_F32_MIXED: f in float      */
  int32_t isothermal; /* 1: T frozen at the node's stored value, eq. (12) dropped */
  int32_t bc_x, bc_y; /* POND_PERIODIC or POND_ZERO_GRADIENT (stencil index clamp) */
  int32_t max_iter;   /* cap on predictor-corrector passes, 1..63 (adaptive mode) */
  int32_t fixed_iter; /* 0: adaptive (App. E test); n > 0: exactly n passes       */
  int32_t seed_mode;  /* seed gauge: 0 own gauge at t - dt (eqs. (7)-(8));
                         1 {0, T_L}; 2 {-u, T} (the seed-independence experiment) */
  double tau;         /* BGK: 2 beta = 1 / tau, eq. (18); nu = T (tau - 1/2) dt    */
  double eps_abs;     /* App. E tolerances (paper: 1e-12, 1e-10 in FP64)          */
  double eps_rel;
} pond_config;

typedef struct {
  void* f;        /* [q*q][ny][nx] populations in the node's own gauge:
                     double for POND_F64, float for POND_F32_MIXED            */
  double* g;      /* [3][ny][nx] gauge per node: u_x, u_y, T (double always)   */
  uint8_t* iters; /* [ny][nx] written by pond_step (POND_ITERS_* bits); nullable */
} pond_state;

typedef struct {
  int64_t nonconverged; /* nodes that hit max_iter in the last step             */
  int64_t bad_state;    /* nodes with rho <= 0, T <= 0 or non-finite values      */
  int32_t max_iters;    /* largest pass count over the grid in the last step     */
  double mean_iters;    /* mean pass count per node in the last step             */
  int64_t iter_hist[POND_ITERS_MASK + 1]; /* nodes per pass count n = 1..63 in
                           the last step (index n; index 0 stays 0): the
                           per-node predictor-corrector iteration counts of
                           App. E as one histogram; sums to nx * ny          */
} pond_stats;

/*
 * Equilibrium initial state (the paper leaves it open; eq. (17) gives the
 * equilibrium of the co-moving gauge): f_p = rho W_i W_j in the gauge
 * {u(x), T(x)}, g = (u_x, u_y, T).
 * rho, ux, uy, T: [ny][nx] double device arrays.  out->f, out->g required;
 * out->iters, if given, is set to 0.
 * Checks every node on the device and returns POND_E_STATE if rho <= 0, T <= 0
 * or a value is non-finite; this check synchronises the stream.
 */
int pond_init(const pond_config* cfg, const double* rho, const double* ux, const double* uy,
              const double* T, pond_state* out, void* hip_stream);

/*
 * nsteps >= 1 PonD time steps (propagation with the predictor-corrector gauge
 * iteration, eqs. (6)-(16) and App. E, then BGK collision, eqs. (17)-(18)).
 * `in` is the state at t - dt, `out` receives the state after nsteps steps.
 * in->f/g and out->f/g must not overlap (the semi-Lagrangian gather reads the
 * whole field at t - dt).  With nsteps == 1 `in` is only read.  With
 * nsteps > 1 the call ping-pongs between the two states, so in->f and in->g
 * are WRITTEN (they hold step nsteps - 1 or nsteps afterwards); a caller that
 * needs them intact passes a copy.
 * out->iters (nullable) receives the pass count and status bits of the last step.
 * stats (HOST pointer, nullable): if given, filled for the last step; the call
 * then synchronises the stream before returning.
 * In POND_F32_MIXED mode with adaptive passes (fixed_iter == 0) the App. E
 * tolerances must be reachable in FP32: max(eps_abs, eps_rel) below 2^-23
 * (FP32 machine epsilon) is rejected with POND_E_INVALID (the paper's FP64
 * values 1e-12 / 1e-10 would run every node to max_iter); the same holds for
 * pond_step_record and both adjoint calls.
 * Tuning (environment, read once per process; results agree to rounding):
 * POND_BULK_CAP = n sets how many passes a node runs one lane per node before
 * an unconverged node is finished by 16 lanes (default D2Q16 FP64 7, D2Q9
 * FP64 9, FP32-mixed 5; 0 or n >= max_iter: never); POND_ADJOINT_LANES = 1, 2 or 4
 * fixes the lanes per node of the adjoint kernels (default: by grid size).
 */
int pond_step(const pond_config* cfg, pond_state* in, pond_state* out, int32_t nsteps,
              void* hip_stream, pond_stats* stats);

/*
 * Macroscopic fields of a state: rho = sum f, rho u = sum v f, 2 rho T + rho|u|^2
 * = sum |v|^2 f with v = sqrt(T_g / T_L) c + u_g of the node's own gauge g
 * (eqs. (10)-(12)).  Mmn (nullable): the raw moments of eq. (2),
 * [m*q + n][ny][nx] for m, n < q.  Every output pointer is nullable.
 */
int pond_moments(const pond_config* cfg, const pond_state* state, double* rho, double* ux,
                 double* uy, double* T, double* Mmn, void* hip_stream);

/*
 * Caller workspace for an operation, written to *bytes (host pointer):
 *   POND_OP_STEP          0 (pond_step needs none beyond the stream slot);
 *   POND_OP_STEP_ADJOINT  the pass history of one step plus one output
 *                         state: ((K + 1) * 4 + q1d^2) * nx * ny * 8 bytes
 *                         (K = fixed_iter, or max_iter in adaptive mode),
 *                         + f, g and iters of one state, each part rounded up
 *                         to 256 bytes.
 * POND_E_INVALID for another op.
 */
int pond_workspace_bytes(const pond_config* cfg, int32_t op, int64_t* bytes);

/*
 * Vector-Jacobian product of one pond_step (nsteps = 1) about the forward pass
 * in -> out_fwd, the unrolled predictor-corrector iteration differentiated
 * with its pass counts fixed (the computed map; eqs. (4)-(18) taken
 * backwards).  The call first runs that step again from `in` with the same
 * configuration, recording every node's pass gauges, densities and last-pass
 * populations in the caller's workspace (the step is deterministic, so this
 * run reproduces out_fwd bit for bit), then the adjoint kernel.  out_fwd is
 * the caller's forward result; it must be given (with iters) but is not read.
 * adj_out: cotangents of (f, g) at t (adj_out->f is double in both precisions).
 * adj_in:  receives the cotangents of (f, g) at t - dt (double); it is
 *          overwritten, not accumulated.  Must not overlap the other buffers.
 * adj_tau (device double*, nullable): d/dtau of <adj_out, out> is ADDED to it.
 * workspace: device memory owned by the caller, 16-byte aligned, at least
 *          pond_workspace_bytes(cfg, POND_OP_STEP_ADJOINT) bytes
 *          (workspace_bytes gives its size; smaller: POND_E_INVALID); it must
 *          not overlap the other buffers (POND_E_ALIAS) and is scratch only:
 *          its contents are undefined after the call.
 */
int pond_step_adjoint(const pond_config* cfg, const pond_state* in, const pond_state* out_fwd,
                      const pond_state* adj_out, pond_state* adj_in, double* adj_tau,
                      void* workspace, int64_t workspace_bytes, void* hip_stream);

/*
 * Transpose of pond_init (the equilibrium f_p = rho W_p of eq. (17), in the
 * gauge {u, T}): from cotangents adj_f [q1d^2][ny][nx] and adj_g [3][ny][nx]
 * (double device arrays), adj_rho = sum_p W_p adj_f_p and adj_ux, adj_uy,
 * adj_T = the three planes of adj_g ([ny][nx] double device arrays, each
 * nullable, overwritten; they must not overlap adj_f or adj_g).
 */
int pond_init_adjoint(const pond_config* cfg, const double* adj_f, const double* adj_g,
                      double* adj_rho, double* adj_ux, double* adj_uy, double* adj_T,
                      void* hip_stream);

/*
 * Recorded steps, for callers that run the step themselves before the adjoint
 * (a checkpointed rollout replays each segment anyway): pond_step_record is
 * one pond_step (nsteps = 1, same arithmetic, same out) that also writes the
 * pass history the adjoint needs -- every node's seed gauge, the gauge and
 * density after each predictor-corrector pass (eqs. (10)-(16)) and the
 * populations of its last pass -- to `tape`; pond_step_adjoint_recorded is
 * pond_step_adjoint about that step, reading the tape instead of running the
 * step again.
 *
 * pond_tape_bytes: the tape's size for cfg, written to *bytes (host pointer):
 *   ((K + 1) * 4 + q1d^2) * nx * ny * 8 bytes, K = fixed_iter, or max_iter in
 *   adaptive mode.
 * pond_step_record: tape (device, caller-owned, pond_tape_bytes bytes) must
 *   not overlap the states; out->iters is required.  POND_E_ALIAS / _NULL as
 *   for pond_step.
 * pond_step_adjoint_recorded: `tape` and out_fwd->iters as written by
 *   pond_step_record(cfg, in, out_fwd, tape) with the same cfg; a tape of
 *   another step gives a meaningless result (nodes whose pass count does not
 *   fit the tape carry no derivative; nothing is read outside it).  Other
 *   arguments as for pond_step_adjoint; adj_in must not overlap the tape.
 */
int pond_tape_bytes(const pond_config* cfg, int64_t* bytes);
int pond_step_record(const pond_config* cfg, const pond_state* in, pond_state* out, void* tape,
                     void* hip_stream);
int pond_step_adjoint_recorded(const pond_config* cfg, const pond_state* in,
                               const pond_state* out_fwd, const void* tape,
                               const pond_state* adj_out, pond_state* adj_in, double* adj_tau,
                               void* hip_stream);

/*
 * pond_step for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, arithmetic and results as pond_step (bit for bit); it calls no
 * hipMalloc / hipFree and allocates nothing through any library.  Its step
 * counters, tile queue and tile cost/order arrays live in one fixed device
 * array of the library (about 386 KiB per GPU, held until the process ends),
 * sized for at most 65,536 step tiles (tiles of 32 x 16 nodes for D2Q16 in
 * POND_F64, 32 x 8 otherwise: any grid up to 4096 x 4096); a larger grid is
 * rejected with POND_E_INVALID.  The queue is cleared by a fill kernel at
 * every call (no memset).  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (different streams, or threads) race and are
 * not supported; calls in order on one stream are.
 */
int pond_step_noalloc(const pond_config* cfg, pond_state* in, pond_state* out, int32_t nsteps,
                      void* hip_stream, pond_stats* stats);

/* Message for the last nonzero return on this thread ("" if none). */
const char* pond_last_error(void);

/* ABI version of this header (major * 100 + minor).  101 added the recorded
 * steps (pond_tape_bytes, pond_step_record, pond_step_adjoint_recorded); 200:
 * the pass histogram in pond_stats, pond_step_adjoint on caller workspace
 * (pond_workspace_bytes), pond_init_adjoint, `in` of pond_step not const;
 * 201 adds pond_step_noalloc. */
int pond_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* POND_H_ */
