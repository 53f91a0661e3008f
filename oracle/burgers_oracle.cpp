// CPU oracle for the viscous-Burgers explicit and BTCS steppers.
//
// TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check and the benchmark's CPU
// baseline leg load this library.  It shares no source, header or generated table with the device path.
//
// Plain loops in the paper's order and notation, compiled with -O2 -ffp-contract=off so that every
// expression rounds exactly as written (no fused multiply-add).  Templated on the working type: the
// FP64 instantiation is the reference; the FP32 one runs the same steps in single precision.
//
// Paper: Potluri et al., "Explicit and implicit finite difference solvers implemented in JAX for shock
// wave physics" (arXiv 2601.12204).  Equation numbers below are the paper's.
//
// Readings of the paper that this file takes (each is listed with its reason in the design notes):
//  * N stored nodes.  Periodic: x_i = i dx, dx = L / N, node N is node 0 (eq. 18).  Dirichlet:
//    dx = L / (N - 1), nodes 0 and N-1 carry a and b (eqs. 16-17) and the interior is updated.
//  * Diffusion is (u_{i+1} + u_{i-1}) - 2 u_i (eqs. 4 and 21; eqs. 5, 6, 9 carry a sign slip).
//  * Convection is upwinded by the sign of u_i: backward difference for u_i >= 0 (eq. 3) and forward
//    difference for u_i < 0 (the text following eq. 3).  With c = r u_i this is
//    max(c,0) (u_i - u_{i-1}) + min(c,0) (u_{i+1} - u_i).
//  * BTCS (Sec. 2.4, eq. 23): the spatial operator is taken at t^{n+1} with its convective coefficient
//    lagged at u^n, so each step is one linear tridiagonal solve A u^{n+1} = u^n, cyclic for periodic
//    boundaries (Sherman-Morrison) and plain for Dirichlet (boundary values moved to the right side).
//  * CFL (eqs. 7-8): dt = sigma * min(dx / umax, dx^2 / (2 nu)).
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

enum { PERIODIC = 0, DIRICHLET = 1 };
enum { SCHEME_EXPLICIT = 0, SCHEME_BTCS = 1 };

// Sec. 2.2: grid spacing for N stored nodes.
double grid_dx(int64_t n, double length, int bc) {
  return bc == PERIODIC ? length / (double)n : length / (double)(n - 1);
}

// ---------------------------------------------------------------------------------------------------
// Explicit forward-Euler step, eq. 21 with the upwind direction chosen by the sign of u_i (text after
// eq. 3).  r = dt/dx, D = nu dt/dx^2.  Dirichlet nodes 0 and n-1 are set to a and b; the interior
// update at i = 1 and i = n-2 reads the boundary values a and b as its neighbours.
// Updates the nodes i0 <= i < i1 of out from u.
template <typename T>
void explicit_range(int64_t n, int bc, T a, T b, T r, T D, const T* u, T* out, int64_t i0, int64_t i1) {
  const T zero = 0;
  const T two = 2;
  for (int64_t i = i0; i < i1; ++i) {
    if (bc == DIRICHLET && (i == 0 || i == n - 1)) {
      out[i] = (i == 0) ? a : b;
      continue;
    }
    T um, up;
    if (bc == PERIODIC) {
      um = u[i == 0 ? n - 1 : i - 1];
      up = u[i == n - 1 ? 0 : i + 1];
    } else {
      um = (i == 1) ? a : u[i - 1];
      up = (i == n - 2) ? b : u[i + 1];
    }
    T ui = u[i];
    T c = r * ui;                      // local Courant number
    T cpos = c > zero ? c : zero;      // max(c, 0): backward difference
    T cneg = c < zero ? c : zero;      // min(c, 0): forward difference
    T lap = (up + um) - two * ui;      // eq. 4 numerator
    out[i] = ((ui - cpos * (ui - um)) - cneg * (up - ui)) + D * lap;
  }
}

template <typename T>
void explicit_step(int64_t n, int bc, T a, T b, T r, T D, const T* u, T* out) {
  explicit_range(n, bc, a, b, r, D, u, out, 0, n);
}

// ---------------------------------------------------------------------------------------------------
// BTCS assembly, Sec. 2.4 and eq. 23.  Row i of A u^{n+1} = u^n with the coefficient c_i = r u_i^n
// lagged at the old level:
//   sub   l_i = -(D + max(c_i, 0))
//   diag  d_i = 1 + 2D + |c_i|
//   super p_i = min(c_i, 0) - D
//   rhs_i = u_i^n
// Periodic: rows 0..n-1, the corners are l_0 (row 0, column n-1) and p_{n-1} (row n-1, column 0).
// Dirichlet: rows for the unknowns 1..n-2; the known boundary values move to the right side.
// Returns the number of rows m.
template <typename T>
int64_t btcs_assemble(int64_t n, int bc, T a, T b, T r, T D, const T* u, T* l, T* d, T* p, T* rhs) {
  const T zero = 0, one = 1, two = 2;
  int64_t first = bc == PERIODIC ? 0 : 1;
  int64_t m = bc == PERIODIC ? n : n - 2;
  for (int64_t k = 0; k < m; ++k) {
    T ui = u[first + k];
    T c = r * ui;
    T cpos = c > zero ? c : zero;
    T cneg = c < zero ? c : zero;
    T cabs = c < zero ? -c : c;
    l[k] = -(D + cpos);
    d[k] = (one + two * D) + cabs;
    p[k] = cneg - D;
    rhs[k] = ui;
  }
  if (bc == DIRICHLET) {
    rhs[0] = rhs[0] - l[0] * a;
    rhs[m - 1] = rhs[m - 1] - p[m - 1] * b;
  }
  return m;
}

// Thomas algorithm (Gaussian elimination without pivoting) for rows k = 0..m-1 with sub-diagonal l,
// diagonal d, super-diagonal p; l[0] and p[m-1] are not part of the matrix.
template <typename T>
void thomas(int64_t m, const T* l, const T* d, const T* p, const T* rhs, T* x, T* cw, T* yw) {
  cw[0] = p[0] / d[0];
  yw[0] = rhs[0] / d[0];
  for (int64_t k = 1; k < m; ++k) {
    T den = d[k] - l[k] * cw[k - 1];
    cw[k] = p[k] / den;
    yw[k] = (rhs[k] - l[k] * yw[k - 1]) / den;
  }
  x[m - 1] = yw[m - 1];
  for (int64_t k = m - 2; k >= 0; --k) x[k] = yw[k] - cw[k] * x[k + 1];
}

// Cyclic tridiagonal solve by the Sherman-Morrison formula (Press et al., Numerical Recipes, Sec. 2.7):
// A = B + w v^T with w = (g, 0, ..., 0, alpha), v = (1, 0, ..., 0, beta / g), g = -d_0,
// beta = A[0][m-1] = l_0, alpha = A[m-1][0] = p_{m-1}.  B is tridiagonal with
// B_00 = d_0 - g and B_{m-1,m-1} = d_{m-1} - alpha beta / g.  Solve B y = rhs and B z = w, then
// x = y - (v.y) / (1 + v.z) z.  Requires m >= 3.
template <typename T>
void cyclic_solve(int64_t m, const T* l, const T* d, const T* p, const T* rhs, T* x) {
  std::vector<T> dd(d, d + m), w(m, T(0)), y(m), z(m), cw(m), yw(m);
  const T g = -d[0];
  const T beta = l[0];
  const T alpha = p[m - 1];
  dd[0] = d[0] - g;
  dd[m - 1] = d[m - 1] - alpha * beta / g;
  w[0] = g;
  w[m - 1] = alpha;
  thomas(m, l, dd.data(), p, rhs, y.data(), cw.data(), yw.data());
  thomas(m, l, dd.data(), p, w.data(), z.data(), cw.data(), yw.data());
  const T vy = y[0] + beta * y[m - 1] / g;
  const T vz = z[0] + beta * z[m - 1] / g;
  const T fact = vy / (T(1) + vz);
  for (int64_t k = 0; k < m; ++k) x[k] = y[k] - fact * z[k];
}

// One BTCS step: assemble (lagged coefficients), solve, write boundary nodes.
template <typename T>
void btcs_step(int64_t n, int bc, T a, T b, T r, T D, const T* u, T* out) {
  std::vector<T> l(n), d(n), p(n), rhs(n), cw(n), yw(n);
  int64_t m = btcs_assemble(n, bc, a, b, r, D, u, l.data(), d.data(), p.data(), rhs.data());
  if (bc == PERIODIC) {
    cyclic_solve(m, l.data(), d.data(), p.data(), rhs.data(), out);
  } else {
    thomas(m, l.data(), d.data(), p.data(), rhs.data(), out + 1, cw.data(), yw.data());
    out[0] = a;
    out[n - 1] = b;
  }
}

// Advance one instance nsteps times with fixed dt.
template <typename T>
void run_one(int64_t n, int bc, int scheme, T a, T b, T r, T D, T* u, int64_t nsteps) {
  std::vector<T> tmp(n);
  for (int64_t s = 0; s < nsteps; ++s) {
    if (scheme == SCHEME_EXPLICIT) explicit_step(n, bc, a, b, r, D, u, tmp.data());
    else btcs_step(n, bc, a, b, r, D, u, tmp.data());
    std::memcpy(u, tmp.data(), sizeof(T) * (size_t)n);
  }
}

// Batched run; scalars per instance are given in FP64 and cast to T (the cast is the only rounding
// of r and D in the FP32 path, identical to what the device side receives).
template <typename T>
void run_batch(int64_t count, const int64_t* offsets, const int32_t* bc, const int32_t* scheme,
               const double* r, const double* D, const double* a, const double* b, T* u,
               int64_t nsteps, int nthreads) {
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int64_t i = 0; i < count; ++i) {
    run_one<T>(offsets[i + 1] - offsets[i], bc[i], scheme[i], (T)a[i], (T)b[i], (T)r[i], (T)D[i],
               u + offsets[i], nsteps);
  }
}

// Explicit steps of one large instance with the nodes split over threads (each node's update reads
// only the previous level, so the split does not change any result).
template <typename T>
void run_explicit_parallel(int64_t n, int bc, double a, double b, double r, double D, T* u,
                           int64_t nsteps, int nthreads) {
  std::vector<T> tmp(n);
  T* src = u;
  T* dst = tmp.data();
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
  nthreads = 1;
#endif
  const int64_t chunk = 1 << 15;
  const int64_t nchunks = (n + chunk - 1) / chunk;
  for (int64_t s = 0; s < nsteps; ++s) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int64_t c = 0; c < nchunks; ++c) {
      explicit_range<T>(n, bc, (T)a, (T)b, (T)r, (T)D, src, dst, c * chunk, std::min(n, (c + 1) * chunk));
    }
    std::swap(src, dst);
  }
  if (src != u) std::memcpy(u, src, sizeof(T) * (size_t)n);
}

// Cole-Hopf closed form for the sawtooth problem on [0, 2 pi]: with phi the periodic heat kernel
// started at t = -1 and moving with speed 4,
//   u = 4 - 2 nu phi_x / phi,  phi = sum_k exp(-(x - 4t - 2 pi k)^2 / (4 nu (t+1))),
// evaluated as 4 + sum_k w_k (xi - 2 pi k) / (t + 1) with xi = (x - 4t) mod 2 pi and w the normalised
// (log-sum-exp) image weights over k = -2..3.
double cole_hopf_point(double x, double t, double nu) {
  const double two_pi = 2.0 * M_PI;
  double xi = std::fmod(x - 4.0 * t, two_pi);
  if (xi < 0) xi += two_pi;
  double e[6], s[6];
  double emax = -INFINITY;
  for (int j = 0; j < 6; ++j) {
    int k = j - 2;
    s[j] = xi - two_pi * k;
    e[j] = -(s[j] * s[j]) / (4.0 * nu * (t + 1.0));
    emax = std::max(emax, e[j]);
  }
  double num = 0, den = 0;
  for (int j = 0; j < 6; ++j) {
    double w = std::exp(e[j] - emax);
    num += w * s[j];
    den += w;
  }
  return 4.0 + (num / den) / (t + 1.0);
}

}  // namespace

extern "C" {

double oracle_dx(int64_t n, double length, int bc) { return grid_dx(n, length, bc); }

// r = dt / dx and D = nu dt / dx^2 in FP64 (Sec. 2.2-2.3).
void oracle_ratios(int64_t n, double length, double nu, double dt, int bc, double* r, double* D) {
  const double dx = grid_dx(n, length, bc);
  *r = dt / dx;
  *D = nu * dt / (dx * dx);
}

// eqs. 7-8 with safety factor sigma: dt = sigma * min(dx / umax, dx^2 / (2 nu)); a zero umax or nu
// removes that limit.
double oracle_cfl_dt(int64_t n, double length, double nu, int bc, double umax, double sigma) {
  const double dx = grid_dx(n, length, bc);
  double lim = INFINITY;
  if (umax > 0) lim = std::min(lim, dx / umax);
  if (nu > 0) lim = std::min(lim, dx * dx / (2.0 * nu));
  return sigma * lim;
}

void oracle_explicit_step_f64(int64_t n, int bc, double a, double b, double r, double D,
                              const double* u, double* out) {
  explicit_step<double>(n, bc, a, b, r, D, u, out);
}
void oracle_explicit_step_f32(int64_t n, int bc, double a, double b, double r, double D,
                              const float* u, float* out) {
  explicit_step<float>(n, bc, (float)a, (float)b, (float)r, (float)D, u, out);
}

int64_t oracle_btcs_assemble_f64(int64_t n, int bc, double a, double b, double r, double D,
                                 const double* u, double* l, double* d, double* p, double* rhs) {
  return btcs_assemble<double>(n, bc, a, b, r, D, u, l, d, p, rhs);
}

void oracle_thomas_f64(int64_t m, const double* l, const double* d, const double* p,
                       const double* rhs, double* x) {
  std::vector<double> cw(m), yw(m);
  thomas<double>(m, l, d, p, rhs, x, cw.data(), yw.data());
}

void oracle_cyclic_f64(int64_t m, const double* l, const double* d, const double* p,
                       const double* rhs, double* x) {
  cyclic_solve<double>(m, l, d, p, rhs, x);
}

void oracle_btcs_step_f64(int64_t n, int bc, double a, double b, double r, double D,
                          const double* u, double* out) {
  btcs_step<double>(n, bc, a, b, r, D, u, out);
}
void oracle_btcs_step_f32(int64_t n, int bc, double a, double b, double r, double D,
                          const float* u, float* out) {
  btcs_step<float>(n, bc, (float)a, (float)b, (float)r, (float)D, u, out);
}

void oracle_run_f64(int64_t count, const int64_t* offsets, const int32_t* bc, const int32_t* scheme,
                    const double* r, const double* D, const double* a, const double* b, double* u,
                    int64_t nsteps, int nthreads) {
  run_batch<double>(count, offsets, bc, scheme, r, D, a, b, u, nsteps, nthreads);
}
void oracle_run_f32(int64_t count, const int64_t* offsets, const int32_t* bc, const int32_t* scheme,
                    const double* r, const double* D, const double* a, const double* b, float* u,
                    int64_t nsteps, int nthreads) {
  run_batch<float>(count, offsets, bc, scheme, r, D, a, b, u, nsteps, nthreads);
}

void oracle_run_explicit_large_f64(int64_t n, int bc, double a, double b, double r, double D,
                                   double* u, int64_t nsteps, int nthreads) {
  run_explicit_parallel<double>(n, bc, a, b, r, D, u, nsteps, nthreads);
}

void oracle_cole_hopf(int64_t m, const double* x, double t, double nu, double* out) {
  for (int64_t i = 0; i < m; ++i) out[i] = cole_hopf_point(x[i], t, nu);
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
