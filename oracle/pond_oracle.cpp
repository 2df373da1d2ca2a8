// Plain, slow, FP64 CPU oracle of the Particles-on-Demand (PonD) time step.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load this library.  It shares no code,
// header, table or constant generator with the HIP path.
//
// Every function follows the paper (Dorschner, Boesch, Karlin, "Particles-on-
// Demand for Kinetic Theory", arXiv:1806.05089) in its order and notation:
//   * particle velocities v_i = sqrt(theta) c_i + u        -- eq. (1), eq. (9)
//   * moments M_mn of eq. (2), matched between gauges       -- eq. (3)
//   * transfer matrix G = M_{lambda'}^{-1} M_lambda          -- eq. (4)
//   * reconstruction from collocation points                -- eq. (5), App. C
//   * semi-Lagrangian advection at x - v_i dt               -- eq. (6)
//   * seed gauge = gauge of the node at t - dt              -- eqs. (7)-(8)
//   * corrector moments rho, u, T                           -- eqs. (10)-(12)
//   * predictor-corrector iteration and its stopping test   -- eqs. (13)-(16), App. E
//   * BGK relaxation to rho W_i in the co-moving gauge      -- eqs. (17)-(18)
//
// Readings of the paper taken here (each one is listed in the design notes):
//   * D2Q16 (q = 4 per axis): c = -/+ sqrt(3 -/+ sqrt 6) (roots of the
//     probabilists' Hermite polynomial He_4), T_L = 1, 1-D weights
//     (3 +/- sqrt 6)/12 (the larger weight on the inner speed).  D2Q9 (q = 3):
//     c = -1, 0, 1, T_L = 1/3, W = 1/6, 2/3, 1/6 (App. A).
//   * Moments are matched in the basis ((v_x - u'_x)/sqrt(theta'))^m
//     ((v_y - u'_y)/sqrt(theta'))^n, m, n < q.  It spans the same polynomial
//     space as the monomials of eq. (2), so G is the same matrix; this basis
//     keeps the linear system well conditioned at any Mach number.
//   * The transfer matrix factorises into per-axis q x q factors (the
//     Kronecker form of App. B); oracle_transfer_2d builds the explicit
//     Q x Q system for the test that pins this factorisation.
//   * After the last predictor-corrector pass n, the populations f^{lambda_n}
//     are moved into the gauge lambda_{n+1} by eq. (4) before collision, and
//     lambda_{n+1} is stored.  rho in eq. (18) is rho_{n+1} of eq. (10).
//   * Convergence test of App. E with |phi_{n+1}| on the right-hand side, for
//     phi in {u_x, u_y, sqrt(theta)} (isothermal: {u_x, u_y}).
//   * Isothermal variant: T is frozen at the node's stored temperature and
//     eq. (12) is not evaluated.
//   * Nodes whose corrector moments give rho <= 0, T <= 0 or a non-finite
//     value are flagged and their output is NaN.
//
// Scalar type S is double or std::complex<double>; with the latter the whole
// step is evaluated in complex arithmetic for complex-step differentiation
// (Squire & Trapp 1998): every branch (floor, convergence test, pivoting)
// decides on real parts only.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

inline double re(double x) { return x; }
inline double re(const cplx& x) { return x.real(); }
inline bool finite_re(double x) { return std::isfinite(x); }
inline bool finite_re(const cplx& x) { return std::isfinite(x.real()) && std::isfinite(x.imag()); }

template <class S> S nan_value() { return S(std::numeric_limits<double>::quiet_NaN()); }

// ---------------------------------------------------------------- lattice
// App. A (D2Q9) and the Gauss-Hermite rule with 4 points (D2Q16).
struct Lattice {
  int q;
  double c[4];
  double w[4];
  double TL;
};

bool make_lattice(int q, Lattice* L) {
  L->q = q;
  if (q == 4) {
    const double r6 = std::sqrt(6.0);
    const double xi1 = std::sqrt(3.0 - r6), xi2 = std::sqrt(3.0 + r6);
    const double w_in = (3.0 + r6) / 12.0, w_out = (3.0 - r6) / 12.0;
    L->c[0] = -xi2; L->c[1] = -xi1; L->c[2] = xi1; L->c[3] = xi2;
    L->w[0] = w_out; L->w[1] = w_in; L->w[2] = w_in; L->w[3] = w_out;
    L->TL = 1.0;
    return true;
  }
  if (q == 3) {
    L->c[0] = -1.0; L->c[1] = 0.0; L->c[2] = 1.0; L->c[3] = 0.0;
    L->w[0] = 1.0 / 6.0; L->w[1] = 2.0 / 3.0; L->w[2] = 1.0 / 6.0; L->w[3] = 0.0;
    L->TL = 1.0 / 3.0;
    return true;
  }
  return false;
}

struct Cfg {
  int q;          // speeds per axis (4: D2Q16, 3: D2Q9)
  int isothermal; // 1: temperature frozen, eq. (12) dropped
  int bc_x, bc_y; // 0: periodic, 1: zero gradient (index clamp)
  int max_iter;   // cap on predictor-corrector passes (adaptive mode)
  int fixed_iter; // >0: exactly this many passes, no convergence test
  int seed_mode;  // 0: own gauge at t-dt (eqs. 7-8); 1: {0, T_L}; 2: {-u, T}
  double eps_abs, eps_rel;
};

// ------------------------------------------------------- linear algebra
// Solve A X = B for X (n x n, n x m), Gaussian elimination with partial
// pivoting on |Re| of the pivot column.  A and B are overwritten.
template <class S>
void solve_dense(int n, int m, S* A, S* B) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    double best = std::fabs(re(A[col * n + col]));
    for (int r = col + 1; r < n; ++r) {
      double v = std::fabs(re(A[r * n + col]));
      if (v > best) { best = v; piv = r; }
    }
    if (piv != col) {
      for (int k = 0; k < n; ++k) std::swap(A[col * n + k], A[piv * n + k]);
      for (int k = 0; k < m; ++k) std::swap(B[col * m + k], B[piv * m + k]);
    }
    for (int r = col + 1; r < n; ++r) {
      S fac = A[r * n + col] / A[col * n + col];
      for (int k = col; k < n; ++k) A[r * n + k] -= fac * A[col * n + k];
      for (int k = 0; k < m; ++k) B[r * m + k] -= fac * B[col * m + k];
    }
  }
  for (int col = n - 1; col >= 0; --col) {
    for (int k = 0; k < m; ++k) {
      S acc = B[col * m + k];
      for (int r = col + 1; r < n; ++r) acc -= A[col * n + r] * B[r * m + k];
      B[col * m + k] = acc / A[col * n + col];
    }
  }
}

// -------------------------------------------------------- transfer (eq. 4)
// Per-axis factor of G_{lambda}^{lambda'}: G1[k*q + i] maps source population
// i (speed c_i in gauge {u, theta}) onto target population k (gauge
// {u', theta'}).  Matching sum_i f_i v_i^p = sum_k f'_k v'_k^p for p < q,
// written in the target-centred variable z = (v - u') / sqrt(theta'):
//   sum_k G1[k,i] c_k^p = z_i^p,   z_i = (sqrt(theta) c_i + u - u') / sqrt(theta').
template <class S>
void transfer_1d(const Lattice& L, S s_src, S u_src, S s_dst, S u_dst, S* G1) {
  const int q = L.q;
  S A[16], B[16];
  for (int p = 0; p < q; ++p) {
    for (int k = 0; k < q; ++k) {
      double cp = 1.0;
      for (int e = 0; e < p; ++e) cp *= L.c[k];
      A[p * q + k] = S(cp);
    }
    for (int i = 0; i < q; ++i) {
      S z = (s_src * L.c[i] + u_src - u_dst) / s_dst;
      S zp = S(1.0);
      for (int e = 0; e < p; ++e) zp *= z;
      B[p * q + i] = zp;
    }
  }
  solve_dense<S>(q, q, A, B);
  for (int k = 0; k < q * q; ++k) G1[k] = B[k];
}

// Apply the Kronecker transfer G = Gx (x) Gy to a population vector in the
// x-major order p = i*q + j (App. B: f'_(k,l) = sum_{i,j} Gx[k,i] Gy[l,j] f_(i,j)).
template <class S>
S transfer_component(int q, const S* Gx, const S* Gy, const S* f, int k, int l) {
  S acc = S(0.0);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) acc += Gx[k * q + i] * Gy[l * q + j] * f[i * q + j];
  return acc;
}

// ------------------------------------------------- reconstruction (App. C)
// Third-order Lagrange weight of collocation point n in {0..3} at local
// coordinate t = x - x0 (x0 = floor(x) - 1).
template <class S>
S lagrange_weight(S t, int n) {
  S a = S(1.0);
  for (int k = 0; k < 4; ++k) {
    if (k == n) continue;
    a *= (t - double(k)) / double(n - k);
  }
  return a;
}

inline int wrap_index(long long i, int n, int bc) {
  if (bc == 0) {
    long long r = i % n;
    if (r < 0) r += n;
    return int(r);
  }
  if (i < 0) return 0;
  if (i >= n) return n - 1;
  return int(i);
}

// ------------------------------------------------------------ one node
// One PonD step at node (X, Y): propagation with the predictor-corrector
// gauge iteration (eqs. 6-16), then BGK collision (eq. 18).
// f: [Q][ny][nx], g: [3][ny][nx] (u_x, u_y, T), both at t - dt.
// Returns 0 (converged / fixed), 1 (hit max_iter), 2 (bad state).
template <class S>
int step_node(const Cfg& cfg, const Lattice& L, int nx, int ny, const S* f, const S* g,
              S tau, long long X, long long Y, S* fo, S* go, int* passes_out) {
  const int q = L.q, Q = q * q;
  const long long plane = (long long)nx * ny;
  const long long node = Y * nx + X;

  // Seed gauge, eqs. (7)-(8) (modes 1 and 2: the alternative seeds of the
  // seed-independence experiment).
  S ux = g[0 * plane + node], uy = g[1 * plane + node], T = g[2 * plane + node];
  if (cfg.seed_mode == 1) {
    ux = S(0.0); uy = S(0.0);
    if (!cfg.isothermal) T = S(L.TL);
  } else if (cfg.seed_mode == 2) {
    ux = -ux; uy = -uy;
  }

  S ft[16];
  S ux1 = ux, uy1 = uy, T1 = T, rho1 = S(0.0);
  int passes = 0;
  int status = 0;
  for (;;) {
    ++passes;
    const S sq = std::sqrt(T / L.TL);  // sqrt(theta_n)
    // Advection at the departure points, eq. (6), with the reconstruction
    // formula eq. (5) / App. C.
    for (int i = 0; i < q; ++i) {
      for (int j = 0; j < q; ++j) {
        const S vx = sq * L.c[i] + ux;
        const S vy = sq * L.c[j] + uy;
        const S xd = double(X) - vx;  // dt = 1
        const S yd = double(Y) - vy;
        const long long fx = (long long)std::floor(re(xd));
        const long long fy = (long long)std::floor(re(yd));
        const long long x0 = fx - 1, y0 = fy - 1;
        const S tx = xd - double(x0), ty = yd - double(y0);
        S acc = S(0.0);
        for (int m = 0; m < 4; ++m) {
          for (int n = 0; n < 4; ++n) {
            const S a = lagrange_weight(tx, n) * lagrange_weight(ty, m);
            const int sx = wrap_index(x0 + n, nx, cfg.bc_x);
            const int sy = wrap_index(y0 + m, ny, cfg.bc_y);
            const long long sn = (long long)sy * nx + sx;
            const S sux = g[0 * plane + sn], suy = g[1 * plane + sn], sT = g[2 * plane + sn];
            const S ss = std::sqrt(sT / L.TL);
            S Gx[16], Gy[16], fs[16];
            transfer_1d<S>(L, ss, sux, sq, ux, Gx);
            transfer_1d<S>(L, ss, suy, sq, uy, Gy);
            for (int p = 0; p < Q; ++p) fs[p] = f[p * plane + sn];
            acc += a * transfer_component<S>(q, Gx, Gy, fs, i, j);
          }
        }
        ft[i * q + j] = acc;
      }
    }
    // Corrector moments, eqs. (10)-(12), with the velocities of eq. (9).
    S rho = S(0.0), jx = S(0.0), jy = S(0.0), e2 = S(0.0);
    for (int i = 0; i < q; ++i) {
      for (int j = 0; j < q; ++j) {
        const S vx = sq * L.c[i] + ux;
        const S vy = sq * L.c[j] + uy;
        const S fv = ft[i * q + j];
        rho += fv;
        jx += vx * fv;
        jy += vy * fv;
        e2 += (vx * vx + vy * vy) * fv;
      }
    }
    rho1 = rho;
    ux1 = jx / rho;
    uy1 = jy / rho;
    if (cfg.isothermal) {
      T1 = T;
    } else {
      T1 = (e2 - rho * (ux1 * ux1 + uy1 * uy1)) / (2.0 * rho);  // D = 2
    }
    if (!(re(rho1) > 0.0) || !(re(T1) > 0.0) || !finite_re(rho1) || !finite_re(ux1) ||
        !finite_re(uy1) || !finite_re(T1)) {
      status = 2;
      break;
    }
    bool done;
    if (cfg.fixed_iter > 0) {
      done = passes >= cfg.fixed_iter;
    } else {
      // App. E: |phi_{n+1} - phi_n| < eps_abs + eps_rel |phi_{n+1}|, each phi.
      auto ok = [&](S a_new, S a_old) {
        return std::fabs(re(a_new) - re(a_old)) < cfg.eps_abs + cfg.eps_rel * std::fabs(re(a_new));
      };
      bool conv = ok(ux1, ux) && ok(uy1, uy);
      if (!cfg.isothermal) conv = conv && ok(std::sqrt(T1 / L.TL), sq);
      done = conv || passes >= cfg.max_iter;
      if (!conv && done) status = 1;
    }
    if (done) break;
    ux = ux1; uy = uy1; T = T1;
  }
  *passes_out = passes;
  if (status == 2) {
    for (int p = 0; p < Q; ++p) fo[p] = nan_value<S>();
    go[0] = go[1] = go[2] = nan_value<S>();
    return status;
  }

  // Move f^{lambda_n} into lambda_{n+1} (eq. 4), then BGK (eq. 18) with
  // f^eq = rho W_i (eq. 17), 2 beta = 1 / tau.
  const S sq_n = std::sqrt(T / L.TL), sq_1 = std::sqrt(T1 / L.TL);
  S Gx[16], Gy[16];
  transfer_1d<S>(L, sq_n, ux, sq_1, ux1, Gx);
  transfer_1d<S>(L, sq_n, uy, sq_1, uy1, Gy);
  const S two_beta = S(1.0) / tau;
  for (int k = 0; k < q; ++k) {
    for (int l = 0; l < q; ++l) {
      const S fr = transfer_component<S>(q, Gx, Gy, ft, k, l);
      const S feq = rho1 * (L.w[k] * L.w[l]);
      fo[k * q + l] = fr + two_beta * (feq - fr);
    }
  }
  go[0] = ux1; go[1] = uy1; go[2] = T1;
  return status;
}

template <class S>
void step_all(const Cfg& cfg, const Lattice& L, int nx, int ny, const S* f, const S* g, S tau,
              S* fo, S* go, int32_t* iters, int32_t* status) {
  const int Q = L.q * L.q;
  const long long plane = (long long)nx * ny;
#pragma omp parallel for schedule(dynamic, 1)
  for (int Y = 0; Y < ny; ++Y) {
    for (int X = 0; X < nx; ++X) {
      S fl[16], gl[3];
      int passes = 0;
      const int st = step_node<S>(cfg, L, nx, ny, f, g, tau, X, Y, fl, gl, &passes);
      const long long node = (long long)Y * nx + X;
      for (int p = 0; p < Q; ++p) fo[p * plane + node] = fl[p];
      for (int k = 0; k < 3; ++k) go[k * plane + node] = gl[k];
      if (iters) iters[node] = passes;
      if (status) status[node] = st;
    }
  }
}

template <class S>
void moments_all(const Lattice& L, long long nnode, const S* f, const S* g, S* rho, S* ux, S* uy,
                 S* T, S* Mmn) {
  const int q = L.q, Q = q * q;
#pragma omp parallel for schedule(static)
  for (long long node = 0; node < nnode; ++node) {
    const S gux = g[0 * nnode + node], guy = g[1 * nnode + node], gT = g[2 * nnode + node];
    const S sq = std::sqrt(gT / L.TL);
    S r = S(0.0), jx = S(0.0), jy = S(0.0), e2 = S(0.0);
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        const S vx = sq * L.c[i] + gux, vy = sq * L.c[j] + guy;
        const S fv = f[(long long)(i * q + j) * nnode + node];
        r += fv; jx += vx * fv; jy += vy * fv; e2 += (vx * vx + vy * vy) * fv;
      }
    const S u = jx / r, v = jy / r;
    if (rho) rho[node] = r;
    if (ux) ux[node] = u;
    if (uy) uy[node] = v;
    if (T) T[node] = (e2 - r * (u * u + v * v)) / (2.0 * r);
    if (Mmn) {
      // Raw moments of eq. (2), m, n < q, stored [m*q + n][node].
      for (int m = 0; m < q; ++m)
        for (int n = 0; n < q; ++n) {
          S acc = S(0.0);
          for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
              const S vx = sq * L.c[i] + gux, vy = sq * L.c[j] + guy;
              S px = S(1.0), py = S(1.0);
              for (int e = 0; e < m; ++e) px *= vx;
              for (int e = 0; e < n; ++e) py *= vy;
              acc += f[(long long)(i * q + j) * nnode + node] * px * py;
            }
          Mmn[(long long)(m * q + n) * nnode + node] = acc;
        }
    }
  }
}

Cfg make_cfg(int q, int isothermal, int bc_x, int bc_y, int max_iter, int fixed_iter,
             int seed_mode, double eps_abs, double eps_rel) {
  Cfg c;
  c.q = q; c.isothermal = isothermal; c.bc_x = bc_x; c.bc_y = bc_y;
  c.max_iter = max_iter; c.fixed_iter = fixed_iter; c.seed_mode = seed_mode;
  c.eps_abs = eps_abs; c.eps_rel = eps_rel;
  return c;
}

void split(const cplx* a, double* r, double* im, long long n) {
  for (long long k = 0; k < n; ++k) { r[k] = a[k].real(); im[k] = a[k].imag(); }
}
std::vector<cplx> join(const double* r, const double* im, long long n) {
  std::vector<cplx> v(n);
  for (long long k = 0; k < n; ++k) v[k] = cplx(r[k], im ? im[k] : 0.0);
  return v;
}

}  // namespace

// ======================================================================
// C ABI of the oracle (its own; loaded by the test suite through ctypes).
// Arrays are C-contiguous float64; f is [Q][ny][nx] with population index
// p = i*q + j (i: x speed index, j: y speed index); g is [3][ny][nx].
// ======================================================================
extern "C" {

int oracle_lattice(int q, double* c, double* w, double* TL) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  for (int k = 0; k < q; ++k) { c[k] = L.c[k]; w[k] = L.w[k]; }
  *TL = L.TL;
  return 0;
}

// Per-axis transfer factor, G1[k*q+i]; gauges given as (u, T).
int oracle_transfer_1d(int q, double u_src, double T_src, double u_dst, double T_dst, double* G1) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  transfer_1d<double>(L, std::sqrt(T_src / L.TL), u_src, std::sqrt(T_dst / L.TL), u_dst, G1);
  return 0;
}

// Explicit Q x Q transfer matrix of eq. (4) built from the 2-D moment system
// (moments (m, n), m, n < q, in the target-centred basis), G[p_out*Q + p_in].
int oracle_transfer_2d(int q, double ux_src, double uy_src, double T_src, double ux_dst,
                       double uy_dst, double T_dst, double* G) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  const int Q = q * q;
  const double ss = std::sqrt(T_src / L.TL), sd = std::sqrt(T_dst / L.TL);
  std::vector<double> A(Q * Q), B(Q * Q);
  for (int m = 0; m < q; ++m)
    for (int n = 0; n < q; ++n) {
      const int row = m * q + n;
      for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
          const int col = i * q + j;
          A[row * Q + col] = std::pow(L.c[i], m) * std::pow(L.c[j], n);
          const double zx = (ss * L.c[i] + ux_src - ux_dst) / sd;
          const double zy = (ss * L.c[j] + uy_src - uy_dst) / sd;
          B[row * Q + col] = std::pow(zx, m) * std::pow(zy, n);
        }
    }
  solve_dense<double>(Q, Q, A.data(), B.data());
  for (int k = 0; k < Q * Q; ++k) G[k] = B[k];
  return 0;
}

double oracle_lagrange_weight(double t, int n) { return lagrange_weight<double>(t, n); }

// Equilibrium initialisation: f = rho W_i in the gauge {u(x), T(x)}.
int oracle_init(int q, int nx, int ny, const double* rho, const double* ux, const double* uy,
                const double* T, double* f, double* g) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  const long long plane = (long long)nx * ny;
  for (long long node = 0; node < plane; ++node) {
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) f[(long long)(i * q + j) * plane + node] = rho[node] * L.w[i] * L.w[j];
    g[node] = ux[node];
    g[plane + node] = uy[node];
    g[2 * plane + node] = T[node];
  }
  return 0;
}

// One PonD step over the whole grid.  iters/status may be null.
int oracle_step(int q, int nx, int ny, int isothermal, int bc_x, int bc_y, int max_iter,
                int fixed_iter, int seed_mode, double tau, double eps_abs, double eps_rel,
                const double* f, const double* g, double* fo, double* go, int32_t* iters,
                int32_t* status) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  Cfg cfg = make_cfg(q, isothermal, bc_x, bc_y, max_iter, fixed_iter, seed_mode, eps_abs, eps_rel);
  step_all<double>(cfg, L, nx, ny, f, g, tau, fo, go, iters, status);
  return 0;
}

// One PonD step evaluated at selected nodes only (flat indices y*nx + x).
// fo: [Q][nsel], go: [3][nsel].
int oracle_step_nodes(int q, int nx, int ny, int isothermal, int bc_x, int bc_y, int max_iter,
                      int fixed_iter, int seed_mode, double tau, double eps_abs, double eps_rel,
                      const double* f, const double* g, long long nsel, const int64_t* sel,
                      double* fo, double* go, int32_t* iters, int32_t* status) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  Cfg cfg = make_cfg(q, isothermal, bc_x, bc_y, max_iter, fixed_iter, seed_mode, eps_abs, eps_rel);
  const int Q = q * q;
#pragma omp parallel for schedule(dynamic, 16)
  for (long long k = 0; k < nsel; ++k) {
    const long long node = sel[k];
    double fl[16], gl[3];
    int passes = 0;
    const int st = step_node<double>(cfg, L, nx, ny, f, g, tau, node % nx, node / nx, fl, gl, &passes);
    for (int p = 0; p < Q; ++p) fo[p * nsel + k] = fl[p];
    for (int c = 0; c < 3; ++c) go[c * nsel + k] = gl[c];
    if (iters) iters[k] = passes;
    if (status) status[k] = st;
  }
  return 0;
}

// rho, u, T from the populations and their gauge (eqs. 10-12 evaluated with
// the node's own velocities); Mmn (nullable): raw moments of eq. (2).
int oracle_moments(int q, int nx, int ny, const double* f, const double* g, double* rho,
                   double* ux, double* uy, double* T, double* Mmn) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  moments_all<double>(L, (long long)nx * ny, f, g, rho, ux, uy, T, Mmn);
  return 0;
}

// ---- complex-step variants (real and imaginary parts in separate arrays) ----
int oracle_init_cs(int q, int nx, int ny, const double* rho_r, const double* rho_i,
                   const double* ux_r, const double* ux_i, const double* uy_r, const double* uy_i,
                   const double* T_r, const double* T_i, double* f_r, double* f_i, double* g_r,
                   double* g_i) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  const long long plane = (long long)nx * ny;
  for (long long node = 0; node < plane; ++node) {
    const cplx r(rho_r[node], rho_i[node]);
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        const cplx v = r * (L.w[i] * L.w[j]);
        f_r[(long long)(i * q + j) * plane + node] = v.real();
        f_i[(long long)(i * q + j) * plane + node] = v.imag();
      }
    g_r[node] = ux_r[node]; g_i[node] = ux_i[node];
    g_r[plane + node] = uy_r[node]; g_i[plane + node] = uy_i[node];
    g_r[2 * plane + node] = T_r[node]; g_i[2 * plane + node] = T_i[node];
  }
  return 0;
}

int oracle_step_cs(int q, int nx, int ny, int isothermal, int bc_x, int bc_y, int max_iter,
                   int fixed_iter, int seed_mode, double tau_r, double tau_i, double eps_abs,
                   double eps_rel, const double* f_r, const double* f_i, const double* g_r,
                   const double* g_i, double* fo_r, double* fo_i, double* go_r, double* go_i,
                   int32_t* iters, int32_t* status) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  Cfg cfg = make_cfg(q, isothermal, bc_x, bc_y, max_iter, fixed_iter, seed_mode, eps_abs, eps_rel);
  const long long plane = (long long)nx * ny;
  const int Q = q * q;
  std::vector<cplx> f = join(f_r, f_i, Q * plane), g = join(g_r, g_i, 3 * plane);
  std::vector<cplx> fo(Q * plane), go(3 * plane);
  step_all<cplx>(cfg, L, nx, ny, f.data(), g.data(), cplx(tau_r, tau_i), fo.data(), go.data(),
                 iters, status);
  split(fo.data(), fo_r, fo_i, Q * plane);
  split(go.data(), go_r, go_i, 3 * plane);
  return 0;
}

int oracle_moments_cs(int q, int nx, int ny, const double* f_r, const double* f_i,
                      const double* g_r, const double* g_i, double* rho_r, double* rho_i,
                      double* ux_r, double* ux_i, double* uy_r, double* uy_i, double* T_r,
                      double* T_i) {
  Lattice L;
  if (!make_lattice(q, &L)) return -1;
  const long long plane = (long long)nx * ny;
  const int Q = q * q;
  std::vector<cplx> f = join(f_r, f_i, Q * plane), g = join(g_r, g_i, 3 * plane);
  std::vector<cplx> r(plane), u(plane), v(plane), T(plane);
  moments_all<cplx>(L, plane, f.data(), g.data(), r.data(), u.data(), v.data(), T.data(), nullptr);
  split(r.data(), rho_r, rho_i, plane);
  split(u.data(), ux_r, ux_i, plane);
  split(v.data(), uy_r, uy_i, plane);
  split(T.data(), T_r, T_i, plane);
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads of the following calls (n >= 1); returns the previous count.
int oracle_set_num_threads(int n) {
  const int prev = oracle_num_threads();
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#endif
  return prev;
}

}  // extern "C"
