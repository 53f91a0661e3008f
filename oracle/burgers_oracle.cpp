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
enum { SCHEME_EXPLICIT = 0, SCHEME_BTCS = 1, SCHEME_RK4 = 2, SCHEME_CN = 3, SCHEME_NEWTON = 4 };

// Newton-Raphson iterations per implicit central-convection step (a fixed count; see newton_step).
constexpr int kNewtonIters = 4;

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
// Classical fourth-order Runge-Kutta step (Sec. 2.7.1, eq. 22) over the spatial operator of eq. 21.
// K(v) = dt L(v) is the increment eq. 21 adds to v in one forward-Euler step:
//   K_i(v) = D ((v_{i+1} + v_{i-1}) - 2 v_i) - (max(c,0) (v_i - v_{i-1}) + min(c,0) (v_{i+1} - v_i)),
// c = r v_i, upwinded as in the explicit step.  The stages are the classical ones,
//   K1 = K(u), K2 = K(u + K1/2), K3 = K(u + K2/2), K4 = K(u + K3),
// and u' = u + (K1 + 2 K2 + 2 K3 + K4) / 6, summed left to right (eq. 22 with dt folded into K).
// Dirichlet nodes carry a and b in every stage and have K = 0.
template <typename T>
void rk4_increment(int64_t n, int bc, T a, T b, T r, T D, const T* v, T* K) {
  const T zero = 0, two = 2;
  for (int64_t i = 0; i < n; ++i) {
    if (bc == DIRICHLET && (i == 0 || i == n - 1)) {
      K[i] = zero;
      continue;
    }
    T um, up;
    if (bc == PERIODIC) {
      um = v[i == 0 ? n - 1 : i - 1];
      up = v[i == n - 1 ? 0 : i + 1];
    } else {
      um = (i == 1) ? a : v[i - 1];
      up = (i == n - 2) ? b : v[i + 1];
    }
    T vi = v[i];
    T c = r * vi;
    T cpos = c > zero ? c : zero;
    T cneg = c < zero ? c : zero;
    T lap = (up + um) - two * vi;
    K[i] = D * lap - (cpos * (vi - um) + cneg * (up - vi));
  }
}

template <typename T>
void rk4_step(int64_t n, int bc, T a, T b, T r, T D, const T* u, T* out) {
  const T half = (T)0.5, two = 2, six = 6;
  std::vector<T> K1(n), K2(n), K3(n), K4(n), v(n);
  rk4_increment(n, bc, a, b, r, D, u, K1.data());
  for (int64_t i = 0; i < n; ++i) v[i] = u[i] + half * K1[i];
  rk4_increment(n, bc, a, b, r, D, v.data(), K2.data());
  for (int64_t i = 0; i < n; ++i) v[i] = u[i] + half * K2[i];
  rk4_increment(n, bc, a, b, r, D, v.data(), K3.data());
  for (int64_t i = 0; i < n; ++i) v[i] = u[i] + K3[i];
  rk4_increment(n, bc, a, b, r, D, v.data(), K4.data());
  for (int64_t i = 0; i < n; ++i) out[i] = u[i] + (((K1[i] + two * K2[i]) + two * K3[i]) + K4[i]) / six;
  if (bc == DIRICHLET) {
    out[0] = a;
    out[n - 1] = b;
  }
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

// One Crank-Nicolson step (the paper names Crank-Nicolson beside BTCS among its implicit schemes,
// Sec. 2.2), with the same lagged upwind/central operator as BTCS:  write the BTCS matrix as A = I + N,
// N's row i = (-(D + max(c_i,0)), 2D + |c_i|, min(c_i,0) - D), c_i = r u_i^n; then
//   (I + N/2) u^{n+1} = (I - N/2) u^n,
// i.e. rows (N_sub/2, 1 + N_diag/2, N_sup/2) and right-hand side u_i - (N u^n)_i / 2, cyclic for
// periodic instances; Dirichlet values enter both sides as in BTCS.
template <typename T>
void cn_step(int64_t n, int bc, T a, T b, T r, T D, const T* u, T* out) {
  const T zero = 0, one = 1, two = 2, half = (T)0.5;
  std::vector<T> l(n), d(n), p(n), rhs(n), cw(n), yw(n);
  const int64_t first = bc == PERIODIC ? 0 : 1;
  const int64_t m = bc == PERIODIC ? n : n - 2;
  for (int64_t k = 0; k < m; ++k) {
    const int64_t i = first + k;
    T um, up;
    if (bc == PERIODIC) {
      um = u[i == 0 ? n - 1 : i - 1];
      up = u[i == n - 1 ? 0 : i + 1];
    } else {
      um = (i == 1) ? a : u[i - 1];
      up = (i == n - 2) ? b : u[i + 1];
    }
    const T ui = u[i];
    const T c = r * ui;
    const T cpos = c > zero ? c : zero;
    const T cneg = c < zero ? c : zero;
    const T cabs = c < zero ? -c : c;
    const T nl = -(D + cpos);
    const T nd = two * D + cabs;
    const T np = cneg - D;
    l[k] = half * nl;
    d[k] = one + half * nd;
    p[k] = half * np;
    rhs[k] = ui - half * ((nl * um + nd * ui) + np * up);
  }
  if (bc == PERIODIC) {
    cyclic_solve(m, l.data(), d.data(), p.data(), rhs.data(), out);
  } else {
    rhs[0] = rhs[0] - l[0] * a;
    rhs[m - 1] = rhs[m - 1] - p[m - 1] * b;
    thomas(m, l.data(), d.data(), p.data(), rhs.data(), out + 1, cw.data(), yw.data());
    out[0] = a;
    out[n - 1] = b;
  }
}

// Fully implicit step with central convection (Sec. 2.4, eqs. 10-14): solve F(x) = 0 with
//   F_i(x) = (x_i - u_i) + ((r/2) x_i (x_{i+1} - x_{i-1}) - D ((x_{i+1} + x_{i-1}) - 2 x_i)),
// r = dt/dx, D = nu dt/dx^2 (eq. 11 with dt folded in), by Newton-Raphson from x = u: J(x) delta = -F(x),
// x = x + delta (eqs. 12-13).  J is tridiagonal (eq. 14), cyclic for periodic instances:
//   J_{i,i-1} = -(r/2) x_i - D,  J_{i,i} = (1 + 2D) + (r/2)(x_{i+1} - x_{i-1}),  J_{i,i+1} = (r/2) x_i - D
// (eq. 15 is garbled; these are the derivatives of eq. 11).  Dirichlet values are fixed and enter F.
// `iters` iterations, no pivoting (the Jacobian is diagonally dominant while the cell Peclet number
// (r/2)|x_i| / D stays below 1 and the step is moderate).
template <typename T>
void newton_step(int64_t n, int bc, T a, T b, T r, T D, const T* u, T* out, int iters) {
  const T one = 1, two = 2, half_r = r / two;
  std::vector<T> x(u, u + n), l(n), d(n), p(n), rhs(n), dx(n), cw(n), yw(n);
  if (bc == DIRICHLET) {
    x[0] = a;
    x[n - 1] = b;
  }
  const int64_t first = bc == PERIODIC ? 0 : 1;
  const int64_t m = bc == PERIODIC ? n : n - 2;
  for (int it = 0; it < iters; ++it) {
    for (int64_t k = 0; k < m; ++k) {
      const int64_t i = first + k;
      const T xm = x[i == 0 ? n - 1 : i - 1];
      const T xp = x[i == n - 1 ? 0 : i + 1];
      const T xi = x[i];
      const T F = (xi - u[i]) + (half_r * xi * (xp - xm) - D * ((xp + xm) - two * xi));
      l[k] = -(half_r * xi) - D;
      d[k] = (one + two * D) + half_r * (xp - xm);
      p[k] = half_r * xi - D;
      rhs[k] = -F;
    }
    if (bc == PERIODIC) {
      cyclic_solve(m, l.data(), d.data(), p.data(), rhs.data(), dx.data());
    } else {
      thomas(m, l.data(), d.data(), p.data(), rhs.data(), dx.data(), cw.data(), yw.data());
    }
    for (int64_t k = 0; k < m; ++k) x[first + k] = x[first + k] + dx[k];
  }
  std::copy(x.begin(), x.end(), out);
}

// Advance one instance nsteps times with fixed dt.
template <typename T>
void run_one(int64_t n, int bc, int scheme, T a, T b, T r, T D, T* u, int64_t nsteps) {
  std::vector<T> tmp(n);
  for (int64_t s = 0; s < nsteps; ++s) {
    if (scheme == SCHEME_EXPLICIT) explicit_step(n, bc, a, b, r, D, u, tmp.data());
    else if (scheme == SCHEME_RK4) rk4_step(n, bc, a, b, r, D, u, tmp.data());
    else if (scheme == SCHEME_CN) cn_step(n, bc, a, b, r, D, u, tmp.data());
    else if (scheme == SCHEME_NEWTON) newton_step(n, bc, a, b, r, D, u, tmp.data(), kNewtonIters);
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


// ---------------------------------------------------------------------------------------------------
// Differentiation of the steppers (the paper computes gradients with respect to initial data by
// reverse-mode AD through its solvers, Sec. 2.7.1 and 2.7.3).  Written out by hand for the discrete
// steps above.  The upwind switch is differentiated on its u_i >= 0 branch at u_i = 0 (H = [u_i >= 0]),
// and dt is a constant.  The viscosity enters through D = nu dt/dx^2 only, so dD = dnu dt/dx^2.
// Dirichlet boundary nodes are constants: they carry no tangent and receive no adjoint.

// Neighbour values of node i as the explicit step reads them (Dirichlet: node 1 reads a, node n-2
// reads b); `um_state`/`up_state` tell whether the neighbour is a state node (carries a tangent).
void neighbours(int64_t n, int bc, int64_t i, int64_t& im, int64_t& ip, bool& um_state, bool& up_state) {
  if (bc == PERIODIC) {
    im = i == 0 ? n - 1 : i - 1;
    ip = i == n - 1 ? 0 : i + 1;
    um_state = up_state = true;
  } else {
    im = i - 1;
    ip = i + 1;
    um_state = i != 1;
    up_state = i != n - 2;
  }
}

// Tangent-linear explicit step: dout = d(u')/du . du + d(u')/dD . dD.
void explicit_tangent(int64_t n, int bc, double a, double b, double r, double D, const double* u,
                      const double* du, double dD, double* dout) {
  for (int64_t i = 0; i < n; ++i) {
    if (bc == DIRICHLET && (i == 0 || i == n - 1)) { dout[i] = 0.0; continue; }
    int64_t im, ip;
    bool ms, ps;
    neighbours(n, bc, i, im, ip, ms, ps);
    const double um = ms ? u[im] : a, up = ps ? u[ip] : b;
    const double dum = ms ? du[im] : 0.0, dup = ps ? du[ip] : 0.0;
    const double ui = u[i], dui = du[i];
    const double lap = (up + um) - 2.0 * ui;
    const double dlap = (dup + dum) - 2.0 * dui;
    double v;
    if (ui >= 0) {   // u' = u - r u (u - um) + D lap
      v = dui - r * dui * (ui - um) - r * ui * (dui - dum);
    } else {         // u' = u - r u (up - u) + D lap
      v = dui - r * dui * (up - ui) - r * ui * (dup - dui);
    }
    dout[i] = v + D * dlap + dD * lap;
  }
}

// Adjoint explicit step: lam = (d u'/du)^T lamp; returns lamp . d(u')/dD.
double explicit_adjoint(int64_t n, int bc, double a, double b, double r, double D, const double* u,
                        const double* lamp, double* lam) {
  for (int64_t i = 0; i < n; ++i) lam[i] = 0.0;
  double gD = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (bc == DIRICHLET && (i == 0 || i == n - 1)) continue;
    int64_t im, ip;
    bool ms, ps;
    neighbours(n, bc, i, im, ip, ms, ps);
    const double um = ms ? u[im] : a, up = ps ? u[ip] : b;
    const double ui = u[i], li = lamp[i];
    double self, left, right;   // coefficients of du_i, du_{i-1}, du_{i+1} in du'_i
    if (ui >= 0) {
      self = 1.0 - r * (ui - um) - r * ui - 2.0 * D;
      left = r * ui + D;
      right = D;
    } else {
      self = 1.0 - r * (up - ui) + r * ui - 2.0 * D;
      left = D;
      right = D - r * ui;
    }
    lam[i] += self * li;
    if (ms) lam[im] += left * li;
    if (ps) lam[ip] += right * li;
    gD += li * ((up + um) - 2.0 * ui);
  }
  return gD;
}

// Shared pieces of the BTCS derivatives for x = u^{n+1} solving A(y) x = y (y = u^n), written on the
// full rows with the Dirichlet boundary values standing in as x_0 = a, x_{n-1} = b:
//   G_i = r [H (x_i - x_{i-1}) + (1 - H)(x_{i+1} - x_i)]   (derivative of row i of A x w.r.t. y_i)
//   (L x)_i = 2 x_i - x_{i-1} - x_{i+1}                     (derivative of row i of A x w.r.t. D)
void btcs_g_and_l(int64_t n, int bc, double a, double b, double r, const double* y, const double* x,
                  std::vector<double>& G, std::vector<double>& Lx) {
  G.assign(n, 0.0);
  Lx.assign(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    if (bc == DIRICHLET && (i == 0 || i == n - 1)) continue;
    double xm, xp;
    if (bc == PERIODIC) {
      xm = x[i == 0 ? n - 1 : i - 1];
      xp = x[i == n - 1 ? 0 : i + 1];
    } else {
      xm = i == 1 ? a : x[i - 1];
      xp = i == n - 2 ? b : x[i + 1];
    }
    G[i] = y[i] >= 0 ? r * (x[i] - xm) : r * (xp - x[i]);
    Lx[i] = (2.0 * x[i] - xm) - xp;
  }
}

// Solve A z = f (transpose = false) or A^T z = f (transpose = true) for the BTCS matrix of state y,
// over the unknown nodes; z and f are full-length node arrays (Dirichlet ends ignored, z ends = 0).
void btcs_matrix_solve(int64_t n, int bc, double r, double D, const double* y, const double* f, double* z,
                       bool transpose) {
  std::vector<double> l(n), d(n), p(n), rhs(n), cw(n), yw(n);
  // assemble with a = b = 0: only the matrix is needed here
  const int64_t m = btcs_assemble<double>(n, bc, 0.0, 0.0, r, D, y, l.data(), d.data(), p.data(), rhs.data());
  const int64_t first = bc == PERIODIC ? 0 : 1;
  for (int64_t k = 0; k < m; ++k) rhs[k] = f[first + k];
  std::vector<double> tl(m), tp(m);
  if (transpose) {   // (A^T)_{k,k-1} = p_{k-1}, (A^T)_{k,k+1} = l_{k+1}, corners swapped likewise
    for (int64_t k = 0; k < m; ++k) {
      tl[k] = bc == PERIODIC ? p[(k - 1 + m) % m] : (k > 0 ? p[k - 1] : 0.0);
      tp[k] = bc == PERIODIC ? l[(k + 1) % m] : (k + 1 < m ? l[k + 1] : 0.0);
    }
  } else {
    for (int64_t k = 0; k < m; ++k) { tl[k] = l[k]; tp[k] = p[k]; }
  }
  std::vector<double> sol(m);
  if (bc == PERIODIC) cyclic_solve<double>(m, tl.data(), d.data(), tp.data(), rhs.data(), sol.data());
  else thomas<double>(m, tl.data(), d.data(), tp.data(), rhs.data(), sol.data(), cw.data(), yw.data());
  for (int64_t i = 0; i < n; ++i) z[i] = 0.0;
  for (int64_t k = 0; k < m; ++k) z[first + k] = sol[k];
}

// Tangent-linear BTCS step: A dx = dy - G dy - dD L x.
void btcs_tangent(int64_t n, int bc, double a, double b, double r, double D, const double* y,
                  const double* x, const double* dy, double dD, double* dx) {
  std::vector<double> G, Lx, f(n);
  btcs_g_and_l(n, bc, a, b, r, y, x, G, Lx);
  for (int64_t i = 0; i < n; ++i) f[i] = dy[i] - G[i] * dy[i] - dD * Lx[i];
  btcs_matrix_solve(n, bc, r, D, y, f.data(), dx, false);
}

// Adjoint BTCS step: mu = A^{-T} lamp; lam = (1 - G) mu; returns -mu . L x (the D-derivative).
double btcs_adjoint(int64_t n, int bc, double a, double b, double r, double D, const double* y,
                    const double* x, const double* lamp, double* lam) {
  std::vector<double> G, Lx, mu(n);
  btcs_g_and_l(n, bc, a, b, r, y, x, G, Lx);
  btcs_matrix_solve(n, bc, r, D, y, lamp, mu.data(), true);
  double gD = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    lam[i] = (1.0 - G[i]) * mu[i];
    gD -= mu[i] * Lx[i];
  }
  return gD;
}

// Forward states u^0..u^nsteps of one instance.
std::vector<std::vector<double>> forward_states(int64_t n, int bc, int scheme, double a, double b, double r,
                                                double D, const double* u0, int64_t nsteps) {
  std::vector<std::vector<double>> st(nsteps + 1, std::vector<double>(n));
  for (int64_t i = 0; i < n; ++i) st[0][i] = u0[i];
  for (int64_t s = 0; s < nsteps; ++s) {
    if (scheme == SCHEME_EXPLICIT) explicit_step<double>(n, bc, a, b, r, D, st[s].data(), st[s + 1].data());
    else btcs_step<double>(n, bc, a, b, r, D, st[s].data(), st[s + 1].data());
  }
  return st;
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
void oracle_newton_step_f64(int64_t n, int bc, double a, double b, double r, double D, const double* u,
                            double* out, int iters) {
  newton_step<double>(n, bc, a, b, r, D, u, out, iters);
}
void oracle_newton_step_f32(int64_t n, int bc, double a, double b, double r, double D, const float* u,
                            float* out, int iters) {
  newton_step<float>(n, bc, (float)a, (float)b, (float)r, (float)D, u, out, iters);
}
int oracle_newton_iters() { return kNewtonIters; }
void oracle_cn_step_f64(int64_t n, int bc, double a, double b, double r, double D, const double* u,
                        double* out) {
  cn_step<double>(n, bc, a, b, r, D, u, out);
}
void oracle_cn_step_f32(int64_t n, int bc, double a, double b, double r, double D, const float* u,
                        float* out) {
  cn_step<float>(n, bc, (float)a, (float)b, (float)r, (float)D, u, out);
}
void oracle_rk4_step_f64(int64_t n, int bc, double a, double b, double r, double D, const double* u,
                         double* out) {
  rk4_step<double>(n, bc, a, b, r, D, u, out);
}
void oracle_rk4_step_f32(int64_t n, int bc, double a, double b, double r, double D, const float* u,
                         float* out) {
  rk4_step<float>(n, bc, (float)a, (float)b, (float)r, (float)D, u, out);
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


// Reverse sweep through nsteps steps of each instance (all forward states kept).  lamT = dJ/du_T;
// writes grad_u0 = dJ/du0 and grad_nu[i] = dJ/dnu_i; dtdx2[i] = dt/dx^2 = dD/dnu.
void oracle_adjoint_run(int64_t count, const int64_t* offsets, const int32_t* bc, const int32_t* scheme,
                        const double* r, const double* D, const double* a, const double* b,
                        const double* dtdx2, const double* u0, const double* lamT, int64_t nsteps,
                        double* grad_u0, double* grad_nu, int nthreads) {
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int64_t i = 0; i < count; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    auto st = forward_states(n, bc[i], scheme[i], a[i], b[i], r[i], D[i], u0 + offsets[i], nsteps);
    std::vector<double> lam(lamT + offsets[i], lamT + offsets[i] + n), prev(n);
    double gD = 0.0;
    for (int64_t s = nsteps - 1; s >= 0; --s) {
      if (scheme[i] == SCHEME_EXPLICIT)
        gD += explicit_adjoint(n, bc[i], a[i], b[i], r[i], D[i], st[s].data(), lam.data(), prev.data());
      else
        gD += btcs_adjoint(n, bc[i], a[i], b[i], r[i], D[i], st[s].data(), st[s + 1].data(), lam.data(),
                           prev.data());
      lam.swap(prev);
    }
    if (bc[i] == DIRICHLET) { lam[0] = 0.0; lam[n - 1] = 0.0; }
    for (int64_t k = 0; k < n; ++k) grad_u0[offsets[i] + k] = lam[k];
    grad_nu[i] = gD * dtdx2[i];
  }
}

// Tangent-linear sweep: du_T from du0 and dnu[i].
void oracle_tangent_run(int64_t count, const int64_t* offsets, const int32_t* bc, const int32_t* scheme,
                        const double* r, const double* D, const double* a, const double* b,
                        const double* dtdx2, const double* u0, const double* du0, const double* dnu,
                        int64_t nsteps, double* duT, int nthreads) {
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int64_t i = 0; i < count; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    auto st = forward_states(n, bc[i], scheme[i], a[i], b[i], r[i], D[i], u0 + offsets[i], nsteps);
    std::vector<double> du(du0 + offsets[i], du0 + offsets[i] + n), nxt(n);
    if (bc[i] == DIRICHLET) { du[0] = 0.0; du[n - 1] = 0.0; }
    const double dD = dnu[i] * dtdx2[i];
    for (int64_t s = 0; s < nsteps; ++s) {
      if (scheme[i] == SCHEME_EXPLICIT)
        explicit_tangent(n, bc[i], a[i], b[i], r[i], D[i], st[s].data(), du.data(), dD, nxt.data());
      else
        btcs_tangent(n, bc[i], a[i], b[i], r[i], D[i], st[s].data(), st[s + 1].data(), du.data(), dD, nxt.data());
      du.swap(nxt);
    }
    for (int64_t k = 0; k < n; ++k) duT[offsets[i] + k] = du[k];
  }
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
