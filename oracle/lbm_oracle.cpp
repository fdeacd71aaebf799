// FP64 CPU oracle for the immersed-boundary lattice Boltzmann step.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library. The product path (the
// HIP library and its Python binding) never calls, links or imports it, and
// it shares no code, header or table with that path.
//
// What is computed (paper: Sec. III-A robot model, Sec. III-B "GPU-accelerated
// localized fluid-structure interaction", Eq. (2) and Eq. (3)):
//   * a D3Q27 lattice Boltzmann approximation of the Navier-Stokes equations
//     of Eq. (2), BGK collision with relaxation time tau,
//   * the fictitious body force of an accelerating, rotating frame, Eq. (3),
//     added to the collision by Guo's forcing scheme,
//   * open x faces by non-equilibrium extrapolation (Sec. III-B, Simulation:
//     the domain boundary treatment taken from Zhao-Li 2002),
//   * the immersed surface as uniformly sampled Lagrangian markers (Sec. III-B,
//     Simulation), coupled two-way by the immersed boundary method: velocity
//     interpolation with Peskin's 4-point smoothed delta kernel, explicit
//     direct forcing, force spreading with the same kernel,
//   * marker positions and velocities by linear blend skinning of bone
//     transforms (Sec. III-A),
//   * the fluid's force, torque and power on the body (the external
//     generalized force of Eq. (1)).
// The paper gives no lattice, collision, forcing or delta-kernel details; the
// readings used here are the ones listed in the design notes of the
// repository, and the header comments of each function say which it takes.
//
// Everything is double precision and deliberately plain: each stage of a step
// is its own pass over the grid or the markers, in the order
//   skin -> moments and unforced velocity -> interpolate -> direct forcing
//   (-> multi-direct-forcing passes) -> spread -> collide interior nodes ->
//   boundary planes -> stream -> wrench.
// Lattice sweeps are parallel over z with OpenMP; per-node arithmetic does
// not depend on the thread count. Marker sums are sequential in marker order.
//
// Parity pins: see tests/test_oracle_*.py (the power term and the open faces'
// outflow and density extrapolation in tests/test_oracle_pins.py). Nothing
// here is "parity unpinned" except the fish thrust and power series, which
// have no closed form.

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------- forward mode ------
// Dual number v + d e (e^2 = 0): carrying d through every operation gives the
// exact directional derivative of the computation (forward-mode
// differentiation). The step below is written once over a scalar type T;
// T = double is the oracle itself, T = Dual its tangent. Branches (stencil
// base, kernel support, face tests) depend on values only.
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline Dual operator+(double a, Dual b) { return Dual(a) + b; }
inline Dual operator+(Dual a, double b) { return a + Dual(b); }
inline Dual operator-(double a, Dual b) { return Dual(a) - b; }
inline Dual operator-(Dual a, double b) { return a - Dual(b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual &operator+=(Dual &a, Dual b) { return a = a + b; }
inline double val(double x) { return x; }
inline double val(const Dual &x) { return x.v; }
inline double tsqrt(double x) { return std::sqrt(x); }
inline Dual tsqrt(Dual x) {
  const double r = std::sqrt(x.v);
  return Dual(r, x.d / (2.0 * r));
}

// ---------------------------------------------------------------- lattice --
// D3Q27: velocities c_i in {-1,0,1}^3, index i = (cx+1) + 3(cy+1) + 9(cz+1).
// Weights by |c|^2: 8/27, 2/27, 1/54, 1/216; sound speed squared 1/3.
struct D3Q27 {
  int c[27][3];
  double w[27];
  D3Q27() {
    for (int i = 0; i < 27; ++i) {
      c[i][0] = i % 3 - 1;
      c[i][1] = (i / 3) % 3 - 1;
      c[i][2] = i / 9 - 1;
      int s = c[i][0] * c[i][0] + c[i][1] * c[i][1] + c[i][2] * c[i][2];
      w[i] = (s == 0) ? 8.0 / 27.0 : (s == 1) ? 2.0 / 27.0 : (s == 2) ? 1.0 / 54.0 : 1.0 / 216.0;
    }
  }
};
const D3Q27 L;

// Second-order equilibrium f^eq_i = w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u].
template <class T>
void equilibrium(T rho, const T u[3], T feq[27]) {
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < 27; ++i) {
    T cu = (double)L.c[i][0] * u[0] + (double)L.c[i][1] * u[1] + (double)L.c[i][2] * u[2];
    feq[i] = L.w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

template <class A, class B, class C>
void cross(const A a[3], const B b[3], C out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

}  // namespace

extern "C" {

// ------------------------------------------------------------ C structs ----
// Boundary codes of a face; an axis is periodic on both faces or open on both.
enum { OR_BC_PERIODIC = 0, OR_BC_VELOCITY = 1, OR_BC_OUTFLOW = 2 };
// Immersed-boundary schemes: explicit direct forcing (with mdf_iters - 1
// multi-direct-forcing passes), or the implicit velocity correction solved by
// mdf_iters conjugate-gradient steps.
enum { OR_IB_DIRECT = 0, OR_IB_IMPLICIT = 1 };
// Collisions: BGK, or the two-relaxation-time collision (see Relax).
enum { OR_COLLIDE_BGK = 0, OR_COLLIDE_TRT = 1 };
// Immersed-wall condition: no-slip (the marker takes the body velocity), or
// slip (Sec. III-B: a Neumann condition, the wall only stops flow through it:
// the forcing acts on the velocity component along the surface normal).
enum { OR_WALL_NO_SLIP = 0, OR_WALL_SLIP = 1 };

struct OrParams {
  int32_t nx, ny, nz;
  int32_t bc_lo, bc_hi;  // x = 0 and x = nx-1; both periodic or both open
  int32_t mdf_iters;     // >= 1; direct forcing: 1 is plain explicit; implicit: CG steps
  double tau;
  double ib_alpha;       // direct-forcing gain
  int32_t bc_y[2];       // y = 0 and y = ny-1 (0: periodic, the default)
  int32_t bc_z[2];       // z = 0 and z = nz-1
  int32_t ib_scheme;     // OR_IB_*
  int32_t collision;     // OR_COLLIDE_*
  double trt_lambda;     // TRT: Lambda = (tau - 1/2)(tau- - 1/2) > 0
  int32_t wall_mode;     // OR_WALL_*
};

// Frame of reference for one step (Eq. (3)): linear acceleration of the
// frame origin (p-double-dot), angular velocity (r-dot) and angular
// acceleration (r-double-dot) as vectors in frame coordinates, the origin x0
// about which x' = x - x0 is measured, and the prescribed velocity on each
// open x face that carries a velocity condition.
struct OrFrame {
  double acc[3];
  double omega[3];
  double alpha[3];
  double origin[3];
  double u_lo[3];
  double u_hi[3];
};

// Skinned marker set. Each marker follows two bones with linear blend
// weights (Sec. III-A: linear blend skinning). Arrays are structure-of-arrays.
struct OrMarkers {
  int32_t n;
  int32_t nbones;
  const double *xrest;   // [3][n] rest-pose positions, lattice units
  const int32_t *bone;   // [2][n]
  const double *weight;  // [2][n]
  const double *dv;      // [n]  marker volume (surface area share x 1 cell)
  const double *nrest;   // [3][n] rest-pose outward unit normals (slip walls; may be null otherwise)
};

}  // extern "C"

namespace {

// Peskin's 4-point smoothed delta function (one axis). C^1, with discrete
// partition of unity, zero first moment and sum of squares 3/8.
template <class T>
T phi(T r) {
  T a = val(r) < 0.0 ? -r : r;
  if (val(a) <= 1.0) return (3.0 - 2.0 * a + tsqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
  if (val(a) <= 2.0) return (5.0 - 2.0 * a - tsqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
  return T(0.0);
}

// Eq. (3) frame force per unit mass without its velocity-dependent Coriolis
// part: a0(x) = -acc - alpha x x' - omega x (omega x x'), with x' = x - x0.
void frame_accel_static(const OrFrame *fr, const double *x, double *a0) {
  double xp[3] = {x[0] - fr->origin[0], x[1] - fr->origin[1], x[2] - fr->origin[2]};
  double ax[3], wx[3], wwx[3];
  cross(fr->alpha, xp, ax);
  cross(fr->omega, xp, wx);
  cross(fr->omega, wx, wwx);
  for (int a = 0; a < 3; ++a) a0[a] = -fr->acc[a] - ax[a] - wwx[a];
}

// Fluid velocity at a node. With Guo forcing the velocity is
//   u = (m + F/2) / rho,  F = g + rho * a_ni(x, u),
// and a_ni (Eq. (3)) contains the Coriolis term -2 omega x u, so u is defined
// implicitly. Writing b = m/rho + g/(2 rho) + a0/2 the definition reads
// u + omega x u = b, a 3x3 linear system whose exact solution is
//   u = (b - omega x b + (omega.b) omega) / (1 + |omega|^2).
// Returns u and the total force density F used by the collision.
template <class T>
void node_velocity(T rho, const T *m, const T *g, const OrFrame *fr, const double *x, T *u, T *F) {
  double a0[3];
  frame_accel_static(fr, x, a0);
  T b[3];
  for (int a = 0; a < 3; ++a) b[a] = m[a] / rho + g[a] / (2.0 * rho) + 0.5 * a0[a];
  T wb[3];
  cross(fr->omega, b, wb);
  T wdotb = fr->omega[0] * b[0] + fr->omega[1] * b[1] + fr->omega[2] * b[2];
  double w2 = fr->omega[0] * fr->omega[0] + fr->omega[1] * fr->omega[1] + fr->omega[2] * fr->omega[2];
  for (int a = 0; a < 3; ++a) u[a] = (b[a] - wb[a] + wdotb * fr->omega[a]) / (1.0 + w2);
  T wu[3];
  cross(fr->omega, u, wu);
  for (int a = 0; a < 3; ++a) F[a] = g[a] + rho * (a0[a] - 2.0 * wu[a]);
}

// Relaxation of the collision. BGK: one rate 1/tau. TRT (the two-relaxation-
// time member of the multiple-relaxation-time family): the parts of f even
// and odd in c relax at their own rates, omega+ = 1/tau (it sets the
// viscosity, nu = (tau - 1/2)/3) and omega- = 1/tau- with
// (tau - 1/2)(tau- - 1/2) = Lambda.
struct Relax {
  bool trt;
  double tau;     // BGK relaxation time; TRT: tau+
  double wp, wm;  // omega+, omega-
};

Relax relax_bgk(double tau) { return Relax{false, tau, 1.0 / tau, 1.0 / tau}; }
Relax relax_trt(double tau, double lambda) {
  const double tm = 0.5 + lambda / (tau - 0.5);
  return Relax{true, tau, 1.0 / tau, 1.0 / tm};
}

// Opposite velocity: c_opp(i) = -c_i.
int opposite(int i) {
  for (int j = 0; j < 27; ++j)
    if (L.c[j][0] == -L.c[i][0] && L.c[j][1] == -L.c[i][1] && L.c[j][2] == -L.c[i][2]) return j;
  return -1;
}

// Guo's source term without its relaxation prefactor:
//   S_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F.
template <class T>
void guo_source(const T u[3], const T F[3], T S[27]) {
  for (int i = 0; i < 27; ++i) {
    T cu = (double)L.c[i][0] * u[0] + (double)L.c[i][1] * u[1] + (double)L.c[i][2] * u[2];
    T s = 0.0;
    for (int a = 0; a < 3; ++a) s += (3.0 * ((double)L.c[i][a] - u[a]) + 9.0 * cu * (double)L.c[i][a]) * F[a];
    S[i] = L.w[i] * s;
  }
}

// TRT update of populations h towards e with source S: with x+_i and x-_i the
// parts of x even and odd in c, (x_i + x_opp(i))/2 and (x_i - x_opp(i))/2,
//   h*_i = h_i - omega+ (h+_i - e+_i) - omega- (h-_i - e-_i)
//          + (1 - omega+/2) S+_i + (1 - omega-/2) S-_i.
template <class T>
void trt_update(const Relax &rx, const T *h, const T *e, const T *S, T *out) {
  for (int i = 0; i < 27; ++i) {
    const int j = opposite(i);
    const T hp = 0.5 * (h[i] + h[j]), hm = 0.5 * (h[i] - h[j]);
    const T ep = 0.5 * (e[i] + e[j]), em = 0.5 * (e[i] - e[j]);
    const T sp = 0.5 * (S[i] + S[j]), sm = 0.5 * (S[i] - S[j]);
    out[i] = h[i] - rx.wp * (hp - ep) - rx.wm * (hm - em) + (1.0 - 0.5 * rx.wp) * sp + (1.0 - 0.5 * rx.wm) * sm;
  }
}

// Collision with Guo's forcing term at one node. BGK:
//   f*_i = f_i - (f_i - f^eq_i(rho,u)) / tau
//          + (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F;
// TRT: trt_update with e = f^eq(rho, u) and S = Guo's source.
template <class T>
void collide_node(const T *f, const T *g, const OrFrame *fr, const double *x, const Relax &rx, T *fout, T *u_out,
                  T *F_out) {
  T rho = 0.0, m[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 27; ++i) {
    rho += f[i];
    for (int a = 0; a < 3; ++a) m[a] += f[i] * (double)L.c[i][a];
  }
  T u[3], F[3];
  node_velocity(rho, m, g, fr, x, u, F);
  T feq[27];
  equilibrium(rho, u, feq);
  if (rx.trt) {
    T S[27];
    guo_source(u, F, S);
    trt_update(rx, f, feq, S, fout);
  } else {
    const double tau = rx.tau;
    double pref = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < 27; ++i) {
      T cu = (double)L.c[i][0] * u[0] + (double)L.c[i][1] * u[1] + (double)L.c[i][2] * u[2];
      T s = 0.0;
      for (int a = 0; a < 3; ++a) s += (3.0 * ((double)L.c[i][a] - u[a]) + 9.0 * cu * (double)L.c[i][a]) * F[a];
      fout[i] = f[i] - (f[i] - feq[i]) / tau + pref * L.w[i] * s;
    }
  }
  if (u_out)
    for (int a = 0; a < 3; ++a) u_out[a] = u[a];
  if (F_out)
    for (int a = 0; a < 3; ++a) F_out[a] = F[a];
}

// Linear blend skinning (Sec. III-A): X = sum_b w_b (R_b xrest + t_b) and
// U = sum_b w_b (Rdot_b xrest + tdot_b). A bone pose is 24 numbers: R (3x3,
// row-major), t (3), Rdot (3x3, row-major), tdot (3).
template <class T>
void skin(const OrMarkers *mk, const T *poses, T *X, T *U) {
  const int n = mk->n;
  for (int k = 0; k < n; ++k) {
    double xr[3] = {mk->xrest[k], mk->xrest[n + k], mk->xrest[2 * n + k]};
    T x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 2; ++j) {
      int b = mk->bone[j * n + k];
      double wgt = mk->weight[j * n + k];
      const T *P = poses + 24 * b;
      for (int a = 0; a < 3; ++a) {
        T px = P[3 * a] * xr[0] + P[3 * a + 1] * xr[1] + P[3 * a + 2] * xr[2] + P[9 + a];
        T pv = P[12 + 3 * a] * xr[0] + P[12 + 3 * a + 1] * xr[1] + P[12 + 3 * a + 2] * xr[2] + P[21 + a];
        x[a] += wgt * px;
        v[a] += wgt * pv;
      }
    }
    for (int a = 0; a < 3; ++a) {
      X[a * n + k] = x[a];
      U[a * n + k] = v[a];
    }
  }
}

// Skinned outward normals: n_k = N(sum_b w_kb R_b nrest_k), N() scaling to
// unit length (the bones' rotations act on the rest normal; their
// translations do not).
template <class T>
void skin_normals(const OrMarkers *mk, const T *poses, T *Nout) {
  const int n = mk->n;
  for (int k = 0; k < n; ++k) {
    double nr[3] = {mk->nrest[k], mk->nrest[n + k], mk->nrest[2 * n + k]};
    T v[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 2; ++j) {
      int b = mk->bone[j * n + k];
      double wgt = mk->weight[j * n + k];
      const T *P = poses + 24 * b;
      for (int a = 0; a < 3; ++a) v[a] += wgt * (P[3 * a] * nr[0] + P[3 * a + 1] * nr[1] + P[3 * a + 2] * nr[2]);
    }
    T len = tsqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int a = 0; a < 3; ++a) Nout[a * n + k] = v[a] / len;
  }
}

}  // namespace

extern "C" {

int or_abi_version(void) { return 5; }

// Threads a parallel lattice sweep uses.
int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads later lattice sweeps use (timing on one core); n >= 1.
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

void or_lattice(int32_t *c, double *w) {
  for (int i = 0; i < 27; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
    w[i] = L.w[i];
  }
}

void or_equilibrium(double rho, const double *u, double *feq) { equilibrium(rho, u, feq); }

// Equilibrium populations of a whole field: rho [n], u [3][n] -> f [27][n].
void or_equilibrium_field(const double *rho, const double *u, int64_t n, double *f) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    double uk[3] = {u[k], u[n + k], u[2 * n + k]}, feq[27];
    equilibrium(rho[k], uk, feq);
    for (int i = 0; i < 27; ++i) f[i * n + k] = feq[i];
  }
}

double or_phi(double r) { return phi(r); }

void or_frame_accel_static(const OrFrame *fr, const double *x, double *a0) { frame_accel_static(fr, x, a0); }

void or_node_velocity(double rho, const double *m, const double *g, const OrFrame *fr, const double *x, double *u,
                      double *F) {
  node_velocity(rho, m, g, fr, x, u, F);
}

void or_collide_node(const double *f, const double *g, const OrFrame *fr, const double *x, double tau, double *fout,
                     double *u_out, double *F_out) {
  collide_node(f, g, fr, x, relax_bgk(tau), fout, u_out, F_out);
}

// The TRT collision at one node (tests): tau = tau+, lambda = Lambda.
void or_collide_node_trt(const double *f, const double *g, const OrFrame *fr, const double *x, double tau,
                         double lambda, double *fout, double *u_out, double *F_out) {
  collide_node(f, g, fr, x, relax_trt(tau, lambda), fout, u_out, F_out);
}

void or_skin(const OrMarkers *mk, const double *poses, double *X, double *U) { skin(mk, poses, X, U); }

// Skinned outward normals [3][n] (tests); the marker set must carry nrest.
int or_skin_normals(const OrMarkers *mk, const double *poses, double *N) {
  if (!mk || !mk->nrest) return -1;
  skin_normals(mk, poses, N);
  return 0;
}

}  // extern "C"

namespace {

inline int wrap(int i, int n) { return ((i % n) + n) % n; }

struct Grid {
  int nx, ny, nz;
  bool per[3];     // axis periodic; otherwise both of its faces are open
  int bc[3][2];    // face conditions (low, high) of each open axis
  size_t ncell() const { return (size_t)nx * ny * nz; }
  size_t idx(int x, int y, int z) const { return (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z); }
  int n(int a) const { return a == 0 ? nx : (a == 1 ? ny : nz); }
};

// The grid of a parameter set; false if an axis has one periodic and one open face.
bool make_grid(const OrParams *p, Grid &G) {
  const int32_t b[3][2] = {{p->bc_lo, p->bc_hi}, {p->bc_y[0], p->bc_y[1]}, {p->bc_z[0], p->bc_z[1]}};
  G.nx = p->nx;
  G.ny = p->ny;
  G.nz = p->nz;
  for (int a = 0; a < 3; ++a) {
    G.per[a] = b[a][0] == OR_BC_PERIODIC;
    if (G.per[a] != (b[a][1] == OR_BC_PERIODIC)) return false;
    G.bc[a][0] = b[a][0];
    G.bc[a][1] = b[a][1];
  }
  return true;
}

// The 4x4x4 stencil of a marker: nodes floor(X)-1 .. floor(X)+2 per axis,
// indices wrapped on periodic axes. Returns false if a node falls outside a
// non-periodic axis (the caller rejects such markers beforehand).
template <class T>
bool stencil(const Grid &G, const T X[3], int nodes[3][4], T wts[3][4]) {
  for (int a = 0; a < 3; ++a) {
    int base = (int)std::floor(val(X[a])) - 1;
    for (int s = 0; s < 4; ++s) {
      int j = base + s;
      wts[a][s] = phi(X[a] - (double)j);
      if (G.per[a]) {
        j = wrap(j, G.n(a));
      } else if (j < 0 || j >= G.n(a)) {
        return false;
      }
      nodes[a][s] = j;
    }
  }
  return true;
}

// U_k = sum over the stencil of field(x) delta_h(x - X_k), delta_h the
// tensor product of phi. field is [ncomp][cells].
template <class T>
void interpolate(const Grid &G, const T *field, int ncomp, const T *X, int n, T *out) {
  for (int k = 0; k < n; ++k) {
    T Xk[3] = {X[k], X[n + k], X[2 * n + k]};
    int nodes[3][4];
    T w[3][4];
    stencil(G, Xk, nodes, w);
    for (int c = 0; c < ncomp; ++c) out[c * n + k] = 0.0;
    for (int sz = 0; sz < 4; ++sz)
      for (int sy = 0; sy < 4; ++sy)
        for (int sx = 0; sx < 4; ++sx) {
          T d = w[0][sx] * w[1][sy] * w[2][sz];
          size_t id = G.idx(nodes[0][sx], nodes[1][sy], nodes[2][sz]);
          for (int c = 0; c < ncomp; ++c) out[c * n + k] += field[c * G.ncell() + id] * d;
        }
  }
}

// g(x) = sum_k Fdv_k delta_h(x - X_k), with Fdv = F_k dV_k. g is [3][cells]
// and is overwritten.
template <class T>
void spread(const Grid &G, const T *X, int n, const T *Fdv, T *g) {
  std::fill(g, g + 3 * G.ncell(), T(0.0));
  for (int k = 0; k < n; ++k) {
    T Xk[3] = {X[k], X[n + k], X[2 * n + k]};
    int nodes[3][4];
    T w[3][4];
    stencil(G, Xk, nodes, w);
    for (int sz = 0; sz < 4; ++sz)
      for (int sy = 0; sy < 4; ++sy)
        for (int sx = 0; sx < 4; ++sx) {
          T d = w[0][sx] * w[1][sy] * w[2][sz];
          size_t id = G.idx(nodes[0][sx], nodes[1][sy], nodes[2][sz]);
          for (int c = 0; c < 3; ++c) g[c * G.ncell() + id] += Fdv[c * n + k] * d;
        }
  }
}

// Density, momentum and the velocity with force field g (no g: pass zeros)
// at every node. rho is [cells], u is [3][cells].
template <class T>
void node_fields(const Grid &G, const T *f, const T *g, const OrFrame *fr, T *rho, T *u) {
  const size_t N = G.ncell();
#pragma omp parallel for schedule(static)
  for (int z = 0; z < G.nz; ++z)
    for (int y = 0; y < G.ny; ++y)
      for (int x = 0; x < G.nx; ++x) {
        size_t id = G.idx(x, y, z);
        T r = 0.0, m[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < 27; ++i) {
          T fi = f[i * N + id];
          r += fi;
          for (int a = 0; a < 3; ++a) m[a] += fi * (double)L.c[i][a];
        }
        T gg[3] = {0.0, 0.0, 0.0};
        if (g)
          for (int a = 0; a < 3; ++a) gg[a] = g[a * N + id];
        double pos[3] = {(double)x, (double)y, (double)z};
        T uu[3], F[3];
        node_velocity(r, m, gg, fr, pos, uu, F);
        rho[id] = r;
        for (int a = 0; a < 3; ++a) u[a * N + id] = uu[a];
      }
}

// Inward step of node (x, y, z) along each axis: +1 on an open low face, -1 on
// an open high face, 0 elsewhere. A node with any nonzero step is a boundary
// node; its inward neighbour (node + step) is the node it extrapolates from.
bool boundary_step(const Grid &G, int x, int y, int z, int d[3]) {
  const int c[3] = {x, y, z};
  bool any = false;
  for (int a = 0; a < 3; ++a) {
    d[a] = 0;
    if (G.per[a]) continue;
    if (c[a] == 0) d[a] = 1;
    else if (c[a] == G.n(a) - 1) d[a] = -1;
    any = any || d[a] != 0;
  }
  return any;
}

// Face condition that sets a boundary node's velocity: its first velocity face
// in the order x low, x high, y low, y high, z low, z high (0: none, then the
// node is an outflow node); *face_u is that face's velocity (u_hi for the x
// high face, u_lo for every other face: in the local moving domain every
// open face sees the same far field).
int boundary_velocity(const Grid &G, const OrFrame *fr, const int d[3], const double **face_u) {
  for (int a = 0; a < 3; ++a)
    for (int side = 0; side < 2; ++side) {
      if (d[a] != (side == 0 ? 1 : -1)) continue;
      if (G.bc[a][side] == OR_BC_VELOCITY) {
        *face_u = (a == 0 && side == 1) ? fr->u_hi : fr->u_lo;
        return 1;
      }
    }
  return 0;
}

}  // namespace

extern "C" {

// Interpolation of a [ncomp][cells] field to n markers (tests).
int or_interpolate(const OrParams *p, const double *field, int ncomp, const double *X, int n, double *out) {
  Grid G;
  if (!make_grid(p, G)) return -1;
  interpolate(G, field, ncomp, X, n, out);
  return 0;
}

// Spreading of n marker forces Fdv = F dV onto g [3][cells] (tests).
int or_spread(const OrParams *p, const double *X, int n, const double *Fdv, double *g) {
  Grid G;
  if (!make_grid(p, G)) return -1;
  spread(G, X, n, Fdv, g);
  return 0;
}

// Density and unforced velocity u* (frame force included, immersed-boundary
// force excluded) of the pre-collision state f. This is the velocity field
// the step interpolates to the markers and the one reported as "the velocity".
int or_macros(const OrParams *p, const double *f, const OrFrame *fr, double *rho, double *u) {
  Grid G;
  if (!make_grid(p, G)) return -1;
  node_fields(G, f, (const double *)nullptr, fr, rho, u);
  return 0;
}

}  // extern "C"

namespace {

// Implicit velocity correction (the implicit immersed-boundary variant the
// paper cites in its Introduction, Wu and Shu's velocity correction). The
// marker forces G_k = F_k dV_k are the ones whose spread force, added to the
// fluid velocity, brings the interpolated velocity to the body velocity at
// every marker:
//   interp(u*) + interp(M spread(G) / (2 rho)) = U,
// with M = (I + [omega]x)^-1 the Coriolis solve that defines the fluid
// velocity. M is the same 3x3 matrix at every node, so the system separates:
//   S G = (I + [omega]x) (U - U*),   S = interp . (1 / (2 rho)) . spread,
// one scalar system per component with the symmetric positive semidefinite
// S (S_kl = sum_x delta(x - X_k) delta(x - X_l) / (2 rho(x))). Each component
// is solved by `iters` steps of conjugate gradients from G = 0, with the
// diagonal preconditioner 2 rho_k: for a uniform density the diagonal of S is
// (3/8)^3 / (2 rho) (the 4-point kernel's squared weights sum to 3/8 along
// each axis), and a constant factor in a preconditioner does not change the
// iterates. Guards: alpha = 0 when p.Sp is not positive (nothing left to
// correct), beta = 0 when the previous r.z is 0.
//   rho [cells] node density; X, U, Ustar [3][nm]; rhok [nm]; G [3][nm] out.
template <class T>
void implicit_forces(const Grid &G, const T *rho, const T *X, const T *U, const T *Ustar, const T *rhok,
                     const OrFrame *fr, int nm, int iters, T *Gout) {
  const size_t N = G.ncell();
  std::vector<T> r(3 * nm), z(3 * nm), p(3 * nm), q(3 * nm), g(3 * N), h(3 * N);
  for (int k = 0; k < nm; ++k) {
    T R[3], wR[3];
    for (int a = 0; a < 3; ++a) R[a] = U[a * nm + k] - Ustar[a * nm + k];
    cross(fr->omega, R, wR);
    for (int a = 0; a < 3; ++a) r[a * nm + k] = R[a] + wR[a];
  }
  T rz[3];
  for (int a = 0; a < 3; ++a) {
    rz[a] = 0.0;
    for (int k = 0; k < nm; ++k) {
      const size_t i = (size_t)a * nm + k;
      z[i] = 2.0 * rhok[k] * r[i];
      p[i] = z[i];
      Gout[i] = 0.0;
      rz[a] += r[i] * z[i];
    }
  }
  for (int it = 0; it < iters; ++it) {
    // q = S p
    spread(G, X, nm, p.data(), g.data());
    for (int a = 0; a < 3; ++a)
      for (size_t id = 0; id < N; ++id) h[a * N + id] = g[a * N + id] / (2.0 * rho[id]);
    interpolate(G, h.data(), 3, X, nm, q.data());
    for (int a = 0; a < 3; ++a) {
      T pq = 0.0;
      for (int k = 0; k < nm; ++k) pq += p[a * nm + k] * q[a * nm + k];
      const T alpha = val(pq) > 0.0 ? rz[a] / pq : T(0.0);
      T rz_new = 0.0;
      for (int k = 0; k < nm; ++k) {
        const size_t i = (size_t)a * nm + k;
        Gout[i] += alpha * p[i];
        r[i] = r[i] - alpha * q[i];
        z[i] = 2.0 * rhok[k] * r[i];
        rz_new += r[i] * z[i];
      }
      const T beta = val(rz[a]) != 0.0 ? rz_new / rz[a] : T(0.0);
      for (int k = 0; k < nm; ++k) p[a * nm + k] = z[a * nm + k] + beta * p[a * nm + k];
      rz[a] = rz_new;
    }
  }
}

// Implicit velocity correction on a slip wall: one unknown per marker, the
// normal force G_k = gamma_k n_k, chosen so that the interpolated velocity
// with the spread force has the body's normal velocity at every marker:
//   n_k . [interp(u* + spread(G) / (2 rho)) - U]_k = 0,
// i.e. (N^T S N) gamma = N^T (U - U*), N stacking the unit normals. N^T S N
// is symmetric positive semidefinite when the frame does not rotate (the
// Coriolis solve would make it unsymmetric; rotating frames are rejected).
// Conjugate gradients as in implicit_forces, on the scalars gamma.
template <class T>
void implicit_forces_slip(const Grid &G, const T *rho, const T *X, const T *U, const T *Ustar, const T *rhok,
                          const T *Nk, int nm, int iters, T *Gout) {
  const size_t N = G.ncell();
  std::vector<T> r(nm), z(nm), p(nm), q(nm), gam(nm, T(0.0)), pv(3 * nm), qv(3 * nm), g(3 * N), h(3 * N);
  T rz = 0.0;
  for (int k = 0; k < nm; ++k) {
    r[k] = 0.0;
    for (int a = 0; a < 3; ++a) r[k] += Nk[a * nm + k] * (U[a * nm + k] - Ustar[a * nm + k]);
    z[k] = 2.0 * rhok[k] * r[k];
    p[k] = z[k];
    rz += r[k] * z[k];
  }
  for (int it = 0; it < iters; ++it) {
    for (int k = 0; k < nm; ++k)
      for (int a = 0; a < 3; ++a) pv[a * nm + k] = p[k] * Nk[a * nm + k];
    spread(G, X, nm, pv.data(), g.data());
    for (int a = 0; a < 3; ++a)
      for (size_t id = 0; id < N; ++id) h[a * N + id] = g[a * N + id] / (2.0 * rho[id]);
    interpolate(G, h.data(), 3, X, nm, qv.data());
    T pq = 0.0;
    for (int k = 0; k < nm; ++k) {
      q[k] = 0.0;
      for (int a = 0; a < 3; ++a) q[k] += Nk[a * nm + k] * qv[a * nm + k];
      pq += p[k] * q[k];
    }
    const T alpha = val(pq) > 0.0 ? rz / pq : T(0.0);
    T rz_new = 0.0;
    for (int k = 0; k < nm; ++k) {
      gam[k] += alpha * p[k];
      r[k] = r[k] - alpha * q[k];
      z[k] = 2.0 * rhok[k] * r[k];
      rz_new += r[k] * z[k];
    }
    const T beta = val(rz) != 0.0 ? rz_new / rz : T(0.0);
    for (int k = 0; k < nm; ++k) p[k] = z[k] + beta * p[k];
    rz = rz_new;
  }
  for (int k = 0; k < nm; ++k)
    for (int a = 0; a < 3; ++a) Gout[a * nm + k] = gam[k] * Nk[a * nm + k];
}

// Advance the pre-collision populations f [27][nz][ny][nx] by nsteps steps.
//   poses  : [nsteps][nbones][24] bone poses for each step (may be null when
//            markers is null)
//   frames : [nsteps]
//   wrench : [nsteps][8] or null: force (3), torque about the frame origin
//            (3), power, thrust-free spare slot = 0
//   X, U, F: [3][n] or null: marker positions, velocities and direct-forcing
//            force densities of the LAST step
// Returns 0, or -4 when a marker's stencil leaves the domain across an open
// face, or -1 on bad arguments.
template <class T>
int run(const OrParams *p, T *f, const OrMarkers *mk, const T *poses, const OrFrame *frames, int nsteps, T *wrench,
        T *Xout, T *Uout, T *Fout, const double *gext = nullptr) {
  if (!p || !f || p->nx < 4 || p->ny < 4 || p->nz < 4 || !(p->tau > 0.5)) return -1;
  Grid G;
  if (!make_grid(p, G)) return -1;
  if (p->mdf_iters < 1 || (p->ib_scheme != OR_IB_DIRECT && p->ib_scheme != OR_IB_IMPLICIT)) return -1;
  const size_t N = G.ncell();
  const double tau = p->tau;
  if (p->collision != OR_COLLIDE_BGK && p->collision != OR_COLLIDE_TRT) return -1;
  if (p->collision == OR_COLLIDE_TRT && !(p->trt_lambda > 0.0 && std::isfinite(p->trt_lambda))) return -1;
  const Relax rx = p->collision == OR_COLLIDE_TRT ? relax_trt(tau, p->trt_lambda) : relax_bgk(tau);
  const int nm = mk ? mk->n : 0;
  if (p->wall_mode != OR_WALL_NO_SLIP && p->wall_mode != OR_WALL_SLIP) return -1;
  const bool slip = p->wall_mode == OR_WALL_SLIP && nm > 0;
  if (slip && !mk->nrest) return -1;

  std::vector<T> fpost(27 * N), rho(N), ustar(3 * N), g(3 * N, T(0.0));
  std::vector<T> X(3 * nm), U(3 * nm), Fk(3 * nm), Fdv(3 * nm), Ustar(3 * nm), rhok(nm), Uk(3 * nm);
  std::vector<T> Nk(slip ? 3 * nm : 0);
  std::vector<T> ufull(3 * N);
  // direct-forcing increment alpha 2 rho_k (U_k - V_k) at marker k, or with a
  // slip wall only its component along the normal, alpha 2 rho_k ((U_k - V_k).n_k) n_k
  auto forcing = [&](const std::vector<T> &V, int k, T out[3]) {
    T d[3];
    for (int a = 0; a < 3; ++a) d[a] = U[a * nm + k] - V[a * nm + k];
    if (slip) {
      T dn = d[0] * Nk[k] + d[1] * Nk[nm + k] + d[2] * Nk[2 * nm + k];
      for (int a = 0; a < 3; ++a) d[a] = dn * Nk[a * nm + k];
    }
    for (int a = 0; a < 3; ++a) out[a] = p->ib_alpha * 2.0 * rhok[k] * d[a];
  };

  for (int step = 0; step < nsteps; ++step) {
    const OrFrame *fr = &frames[step];

    // (1) marker positions and velocities for this step
    if (nm > 0) {
      skin(mk, poses + (size_t)step * mk->nbones * 24, X.data(), U.data());
      if (slip) skin_normals(mk, poses + (size_t)step * mk->nbones * 24, Nk.data());
      for (int a = 0; a < 3; ++a)
        if (!G.per[a])
          for (int k = 0; k < nm; ++k)
            if (!(val(X[a * nm + k]) >= 2.0 && val(X[a * nm + k]) < G.n(a) - 3.0)) return -4;
    }

    // (2) density and unforced velocity at every node
    node_fields(G, (const T *)f, (const T *)nullptr, fr, rho.data(), ustar.data());

    // (3)-(5) interpolation, direct forcing, spreading
    std::fill(g.begin(), g.end(), T(0.0));
    if (nm > 0) {
      interpolate(G, ustar.data(), 3, X.data(), nm, Ustar.data());
      interpolate(G, rho.data(), 1, X.data(), nm, rhok.data());
      if (p->ib_scheme == OR_IB_IMPLICIT && slip) {
        const double *w = fr->omega;
        if (w[0] != 0.0 || w[1] != 0.0 || w[2] != 0.0) return -1;  // unsymmetric system: not supported
        implicit_forces_slip(G, rho.data(), X.data(), U.data(), Ustar.data(), rhok.data(), Nk.data(), nm,
                             p->mdf_iters, Fdv.data());
        for (int k = 0; k < nm; ++k)
          for (int a = 0; a < 3; ++a) Fk[a * nm + k] = Fdv[a * nm + k] / mk->dv[k];
      } else if (p->ib_scheme == OR_IB_IMPLICIT) {
        implicit_forces(G, rho.data(), X.data(), U.data(), Ustar.data(), rhok.data(), fr, nm, p->mdf_iters,
                        Fdv.data());
        for (int k = 0; k < nm; ++k)
          for (int a = 0; a < 3; ++a) Fk[a * nm + k] = Fdv[a * nm + k] / mk->dv[k];
      } else {
        for (int k = 0; k < nm; ++k) {
          T inc[3];
          forcing(Ustar, k, inc);
          for (int a = 0; a < 3; ++a) Fk[a * nm + k] = inc[a];
        }
        for (int it = 1; it < p->mdf_iters; ++it) {
          // multi-direct forcing: spread the current force, re-interpolate the
          // velocity that includes it, add the remaining correction
          for (int k = 0; k < nm; ++k)
            for (int a = 0; a < 3; ++a) Fdv[a * nm + k] = Fk[a * nm + k] * mk->dv[k];
          spread(G, X.data(), nm, Fdv.data(), g.data());
          node_fields(G, f, g.data(), fr, rho.data(), ufull.data());
          interpolate(G, ufull.data(), 3, X.data(), nm, Uk.data());
          for (int k = 0; k < nm; ++k) {
            T inc[3];
            forcing(Uk, k, inc);
            for (int a = 0; a < 3; ++a) Fk[a * nm + k] += inc[a];
          }
        }
        for (int k = 0; k < nm; ++k)
          for (int a = 0; a < 3; ++a) Fdv[a * nm + k] = Fk[a * nm + k] * mk->dv[k];
      }
      spread(G, X.data(), nm, Fdv.data(), g.data());
    }
    // a prescribed body-force density field, added to the immersed force (tests)
    if (gext)
      for (size_t i = 0; i < 3 * N; ++i) g[i] += gext[i];

    // (6) BGK + Guo collision on every node that is not an open boundary node
#pragma omp parallel for schedule(static)
    for (int z = 0; z < G.nz; ++z)
      for (int y = 0; y < G.ny; ++y)
        for (int x = 0; x < G.nx; ++x) {
          int d[3];
          if (boundary_step(G, x, y, z, d)) continue;
          size_t id = G.idx(x, y, z);
          T fl[27], fo[27];
          for (int i = 0; i < 27; ++i) fl[i] = f[i * N + id];
          T gg[3] = {g[id], g[N + id], g[2 * N + id]};
          double pos[3] = {(double)x, (double)y, (double)z};
          collide_node(fl, gg, fr, pos, rx, fo, (T *)nullptr, (T *)nullptr);
          for (int i = 0; i < 27; ++i) fpost[i * N + id] = fo[i];
        }

    // (7) open faces by non-equilibrium extrapolation. Boundary node x_b
    // takes its inward neighbour x_f's density and non-equilibrium part:
    //   f*_i(x_b) = f^eq_i(rho_f, u_b) + (1 - 1/tau) (f_i(x_f) - f^eq_i(rho_f, u_f))
    //               + (1 - 1/(2 tau)) w_i [3 (c_i - u_b) + 9 (c_i.u_b) c_i] . F_b
    // x_f is x_b moved one node inward along each open axis it lies on (a
    // diagonal neighbour on edges and corners); u_f is x_f's fluid velocity
    // (with its force half-term, the same definition the collision uses); u_b
    // is the prescribed velocity of x_b's velocity face, or u_f when it lies on
    // outflow faces only; F_b = rho_f a_ni(x_b, u_b) is the frame force alone
    // (markers never reach a boundary node).
    if (!(G.per[0] && G.per[1] && G.per[2])) {
#pragma omp parallel for schedule(static)
      for (int z = 0; z < G.nz; ++z)
        for (int y = 0; y < G.ny; ++y)
          for (int x = 0; x < G.nx; ++x) {
            int d[3];
            if (!boundary_step(G, x, y, z, d)) continue;
            const int xf = x + d[0], yf = y + d[1], zf = z + d[2];
            size_t idf = G.idx(xf, yf, zf), idb = G.idx(x, y, z);
            T fl[27], r = 0.0, m[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < 27; ++i) {
              fl[i] = f[i * N + idf];
              r += fl[i];
              for (int a = 0; a < 3; ++a) m[a] += fl[i] * (double)L.c[i][a];
            }
            T gf[3] = {g[idf], g[N + idf], g[2 * N + idf]};
            double posf[3] = {(double)xf, (double)yf, (double)zf};
            double posb[3] = {(double)x, (double)y, (double)z};
            T uf[3], Ff[3];
            node_velocity(r, m, gf, fr, posf, uf, Ff);
            const double *uface = nullptr;
            const int vel = boundary_velocity(G, fr, d, &uface);
            T ub[3];
            for (int a = 0; a < 3; ++a) ub[a] = vel ? T(uface[a]) : uf[a];
            double a0[3];
            T wu[3], Fb[3];
            frame_accel_static(fr, posb, a0);
            cross(fr->omega, ub, wu);
            for (int a = 0; a < 3; ++a) Fb[a] = r * (a0[a] - 2.0 * wu[a]);
            T feq_b[27], feq_f[27];
            equilibrium(r, ub, feq_b);
            equilibrium(r, uf, feq_f);
            if (rx.trt) {
              // TRT: the non-equilibrium part's even and odd halves relax at
              // their own rates, f*(x_b) = trt_update of h = f^eq(u_b) + f(x_f) -
              // f^eq(u_f) towards f^eq(u_b) with the source at (u_b, F_b)
              T h[27], Sb[27], out[27];
              for (int i = 0; i < 27; ++i) h[i] = feq_b[i] + (fl[i] - feq_f[i]);
              guo_source(ub, Fb, Sb);
              trt_update(rx, h, feq_b, Sb, out);
              for (int i = 0; i < 27; ++i) fpost[i * N + idb] = out[i];
            } else {
              double pref = 1.0 - 1.0 / (2.0 * tau);
              for (int i = 0; i < 27; ++i) {
                T cu = (double)L.c[i][0] * ub[0] + (double)L.c[i][1] * ub[1] + (double)L.c[i][2] * ub[2];
                T s = 0.0;
                for (int a = 0; a < 3; ++a)
                  s += (3.0 * ((double)L.c[i][a] - ub[a]) + 9.0 * cu * (double)L.c[i][a]) * Fb[a];
                fpost[i * N + idb] = feq_b[i] + (1.0 - 1.0 / tau) * (fl[i] - feq_f[i]) + pref * L.w[i] * s;
              }
            }
          }
    }

    // (8) streaming: f_i(x, n+1) = f*_i(x - c_i, n). Periodic axes wrap; a
    // source outside an open face is replaced by the nearest node on it (those
    // values are never used: extrapolation overwrites the boundary nodes).
#pragma omp parallel for schedule(static)
    for (int z = 0; z < G.nz; ++z)
      for (int y = 0; y < G.ny; ++y)
        for (int x = 0; x < G.nx; ++x)
          for (int i = 0; i < 27; ++i) {
            int sc[3] = {x - L.c[i][0], y - L.c[i][1], z - L.c[i][2]};
            for (int a = 0; a < 3; ++a) {
              const int na = G.n(a);
              sc[a] = G.per[a] ? wrap(sc[a], na) : (sc[a] < 0 ? 0 : (sc[a] >= na ? na - 1 : sc[a]));
            }
            f[i * N + G.idx(x, y, z)] = fpost[i * N + G.idx(sc[0], sc[1], sc[2])];
          }

    // (9) the fluid's force, torque and power on the body: the body exerts
    // F_k dV_k on the fluid, so the fluid exerts the opposite on the body.
    if (wrench) {
      T *wr = wrench + 8 * (size_t)step;
      for (int j = 0; j < 8; ++j) wr[j] = 0.0;
      for (int k = 0; k < nm; ++k) {
        T Fb[3] = {-Fdv[k], -Fdv[nm + k], -Fdv[2 * nm + k]};
        T r[3] = {X[k] - fr->origin[0], X[nm + k] - fr->origin[1], X[2 * nm + k] - fr->origin[2]};
        T t[3];
        cross(r, Fb, t);
        for (int a = 0; a < 3; ++a) {
          wr[a] += Fb[a];
          wr[3 + a] += t[a];
        }
        wr[6] += Fdv[k] * U[k] + Fdv[nm + k] * U[nm + k] + Fdv[2 * nm + k] * U[2 * nm + k];
      }
    }
  }
  if (nm > 0) {
    if (Xout) std::copy(X.begin(), X.end(), Xout);
    if (Uout) std::copy(U.begin(), U.end(), Uout);
    if (Fout) std::copy(Fk.begin(), Fk.end(), Fout);
  }
  return 0;
}


}  // namespace

extern "C" {

int or_run(const OrParams *p, double *f, const OrMarkers *mk, const double *poses, const OrFrame *frames,
           int nsteps, double *wrench, double *Xout, double *Uout, double *Fout) {
  return run(p, f, mk, poses, frames, nsteps, wrench, Xout, Uout, Fout);
}

// nsteps steps with no body and a constant body-force density field
// g [3][cells] added at every node (tests of the bulk forcing).
int or_run_forced(const OrParams *p, double *f, const OrFrame *frames, int nsteps, const double *g) {
  return run(p, f, (const OrMarkers *)nullptr, (const double *)nullptr, frames, nsteps, (double *)nullptr,
             (double *)nullptr, (double *)nullptr, (double *)nullptr, g);
}

// Forward-mode tangent of or_run with respect to the bone poses: the same
// step in dual numbers, with the initial populations and the frames held
// fixed. poses_d [nsteps][nbones][24] is the direction (d pose / d theta for
// a parameter theta); f is advanced in place as by or_run, f_d [27][cells]
// receives d f / d theta, wrench and wrench_d [nsteps][8] the wrench and its
// derivative. Same return codes as or_run.
int or_run_tangent(const OrParams *p, double *f, double *f_d, const OrMarkers *mk, const double *poses,
                   const double *poses_d, const OrFrame *frames, int nsteps, double *wrench, double *wrench_d) {
  if (!p || !f || !mk || !poses || !poses_d || !frames || nsteps < 0) return -1;
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  const size_t np = (size_t)nsteps * mk->nbones * 24;
  std::vector<Dual> fd(27 * N), pd(np), wd(8 * (size_t)nsteps);
  for (size_t q = 0; q < 27 * N; ++q) fd[q] = Dual(f[q]);
  for (size_t q = 0; q < np; ++q) pd[q] = Dual(poses[q], poses_d[q]);
  const int rc = run(p, fd.data(), mk, pd.data(), frames, nsteps, wd.data(), (Dual *)nullptr, (Dual *)nullptr,
                     (Dual *)nullptr);
  for (size_t q = 0; q < 27 * N; ++q) {
    f[q] = fd[q].v;
    if (f_d) f_d[q] = fd[q].d;
  }
  for (size_t q = 0; q < 8 * (size_t)nsteps; ++q) {
    if (wrench) wrench[q] = wd[q].v;
    if (wrench_d) wrench_d[q] = wd[q].d;
  }
  return rc;
}

}  // extern "C"
