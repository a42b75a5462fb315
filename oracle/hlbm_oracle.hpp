// Oracle for the fused HLBM stream-collide step -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU implementation of one time step of the homogenized
// hybrid recursive-regularized LBM with Smagorinsky LES and the Spalding wall
// model ("Efficient Wall-Modelled Large Eddy Simulation of Rotors using
// Homogenized Lattice Boltzmann Methods", Sec. 2.2 "Homogenized Lattice
// Boltzmann Method", Sec. 2.2.1 "Turbulent Wall Model", Sec. 2.2.2
// "Fluid-Structure Interaction", Sec. 3).  Only tests/, the smoke entry point
// and the CPU baseline of the benchmark may load it; the product path never
// does.  It shares no code with the HIP library.
//
// Every formula is written out as its definition: full Hermite tensor
// contractions over a,b,c in {x,y,z}, whole-grid phases, no fusion.  All
// arithmetic is templated on the scalar so the same code runs in double,
// std::complex<double> (complex-step derivatives) and Dual<N> (forward-mode
// Jacobians used by the oracle adjoint).
#pragma once
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

namespace oracle {

// ---------------------------------------------------------------- scalars
template <int N>
struct Dual {
  double v;
  double g[N];
  Dual() : v(0) { for (int k = 0; k < N; ++k) g[k] = 0; }
  Dual(double x) : v(x) { for (int k = 0; k < N; ++k) g[k] = 0; }
};
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v + b.v; for (int k = 0; k < N; ++k) r.g[k] = a.g[k] + b.g[k]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v - b.v; for (int k = 0; k < N; ++k) r.g[k] = a.g[k] - b.g[k]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) { Dual<N> r; r.v = -a.v; for (int k = 0; k < N; ++k) r.g[k] = -a.g[k]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v * b.v; for (int k = 0; k < N; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v / b.v; for (int k = 0; k < N; ++k) r.g[k] = (a.g[k] * b.v - a.v * b.g[k]) / (b.v * b.v); return r; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> inline Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> inline Dual<N> sqrt(const Dual<N>& a) { Dual<N> r; r.v = std::sqrt(a.v); for (int k = 0; k < N; ++k) r.g[k] = a.g[k] / (2.0 * r.v); return r; }
template <int N> inline Dual<N> exp(const Dual<N>& a) { Dual<N> r; r.v = std::exp(a.v); for (int k = 0; k < N; ++k) r.g[k] = a.g[k] * r.v; return r; }
template <int N> inline Dual<N> log(const Dual<N>& a) { Dual<N> r; r.v = std::log(a.v); for (int k = 0; k < N; ++k) r.g[k] = a.g[k] / a.v; return r; }

inline double re(double x) { return x; }
inline double re(const std::complex<double>& x) { return x.real(); }
template <int N> inline double re(const Dual<N>& x) { return x.v; }

// ------------------------------------------------------------ constants
// Velocity sets.  D3Q27: c in {-1,0,1}^3, canonical order
// i = 9(cx+1) + 3(cy+1) + (cz+1), weights 8/27, 2/27, 1/54, 1/216 by |c|^2.
// D3Q19 (the paper's stencil, Sec. 2.2, Fig. 2): the same order restricted
// to |c|^2 <= 2, weights 1/3, 1/18, 1/36.  Q is the largest set (array
// bounds); a lattice's own count is q.
constexpr int Q = 27;
constexpr double CS2 = 1.0 / 3.0;

struct Lattice {
  int q;
  int c[Q][3];
  double w[Q];
  explicit Lattice(int nq) : q(0) {
    for (int i = 0; i < 27; ++i) {
      const int cx = i / 9 - 1, cy = (i / 3) % 3 - 1, cz = i % 3 - 1;
      const int n2 = cx * cx + cy * cy + cz * cz;
      if (nq == 19 && n2 == 3) continue;
      c[q][0] = cx; c[q][1] = cy; c[q][2] = cz;
      if (nq == 19) w[q] = n2 == 0 ? 1.0 / 3.0 : n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
      else w[q] = n2 == 0 ? 8.0 / 27.0 : n2 == 1 ? 2.0 / 27.0 : n2 == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
      ++q;
    }
  }
  // Second Hermite polynomial H^(2)_ab = c_a c_b - cs^2 delta_ab.
  double H2(int i, int a, int b) const { return c[i][a] * c[i][b] - (a == b ? CS2 : 0.0); }
  // Third Hermite polynomial H^(3)_abc = c_a c_b c_c - cs^2 (c_a d_bc + c_b d_ac + c_c d_ab).
  double H3(int i, int a, int b, int cc) const {
    return c[i][a] * c[i][b] * c[i][cc] -
           CS2 * (c[i][a] * (b == cc) + c[i][b] * (a == cc) + c[i][cc] * (a == b));
  }
  // Third-order term of a Hermite expansion at velocity i for the
  // coefficient tensor a3 (Sec. 2.2: equilibrium and recursive f^(1)).
  // D3Q27 holds every third-order polynomial: the full series term
  // H3 : a3 / (6 cs^6).  D3Q19 holds neither H_aaa (zero on any velocity
  // set in {-1,0,1}) nor H_xyz, and its H_aab, H_ccb are not orthogonal
  // under its weights; the recursive-regularized schemes the paper builds on
  // (Coreixas et al. 2017, Jacob et al. 2018) project onto the orthogonal
  // pairs H_aab + H_ccb and H_aab - H_ccb (b the odd index, a and c the
  // other two axes), whose D3Q19 norms are 2 cs^6 and 6 cs^6.
  template <class T>
  T third(int i, const T a3[3][3][3]) const {
    T s = T(0.0);
    if (q == 27) {
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          for (int cc = 0; cc < 3; ++cc) s = s + H3(i, a, b, cc) * a3[a][b][cc];
      return s / (6.0 * CS2 * CS2 * CS2);
    }
    for (int b = 0; b < 3; ++b) {
      const int a = b == 0 ? 1 : 0, cc = b == 2 ? 1 : 2;
      const double hp = H3(i, a, a, b) + H3(i, cc, cc, b), hm = H3(i, a, a, b) - H3(i, cc, cc, b);
      s = s + hp * (a3[a][a][b] + a3[cc][cc][b]) / (2.0 * CS2 * CS2 * CS2) +
          hm * (a3[a][a][b] - a3[cc][cc][b]) / (6.0 * CS2 * CS2 * CS2);
    }
    return s;
  }
};

inline const Lattice& lattice(int q) {
  static const Lattice L27(27), L19(19);
  return q == 19 ? L19 : L27;
}
inline const Lattice& lat() { return lattice(27); }

// ------------------------------------------------------------ parameters
struct Params {
  double tau0;        // molecular relaxation time (> 1/2)
  double cs_smag;     // Smagorinsky constant C_S
  double eps_h;       // width of the porosity transition band (lattice units)
  int transition;     // 0: tanh transition, 1: linear s(phi) = phi/eps_h + 1/2
  int wall_model;     // 0 off, 1 on
  double E, kappa;    // Spalding constants
  double y_s;         // sampling distance
  double tol;         // Newton stop tolerance on |f(u^{j+1}) - f(u^j)|
  int maxit;          // Newton iteration cap
  double u_in[3];     // inflow velocity
  double turb_I;      // inflow turbulence intensity (std of each component / |u_in|)
  uint64_t seed;      // inflow noise seed
  double fd_share;    // 1 - sigma in an element's cells off the wall (hybrid f~(1)); 0: sigma = 1
};

// Reference grid of a moving element (Sec. 3.1: the element is voxelized
// once in its own inertial reference grid, and that grid is embedded into
// the lattice porosity at the element's position and orientation each
// step): the signed distance phi (positive inside) at body coordinates
// o + h (i, j, k), stored [k][j][i], body axes the radial direction of blade
// 0, the tangential direction e x e_r and the rotor axis e.
struct RefGrid {
  std::vector<double> phi;
  int n[3];
  double h, o[3];
};

struct Rotor {
  double center[3], axis[3];
  double R, r_hub, chord, thick, twist_root, twist_tip, omega, phase0;
  int n_blades, tag;
  double inertia;     // moment of inertia about the axis; 0: prescribed rotation
  double torque_gen;  // opposing (generator) torque of a coupled rotor
  const RefGrid* grid = nullptr;  // replaces the flat-plate blades and hub when set
};

// ------------------------------------------------------------ equilibrium
// Third-order Hermite equilibrium (Sec. 2.2, equilibrium definition) with
// a0^(n) = rho u^n: the Hermite series 1/(n! cs^(2n)) H^(n):a^(n), its
// third-order term as the lattice holds it (Lattice::third).
template <class T>
void equilibrium(const T& rho, const T u[3], T feq[Q], const Lattice& L = lat()) {
  T a3[3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int cc = 0; cc < 3; ++cc) a3[a][b][cc] = u[a] * u[b] * u[cc];
  for (int i = 0; i < L.q; ++i) {
    T s1 = T(0.0), s2 = T(0.0);
    for (int a = 0; a < 3; ++a) {
      s1 = s1 + double(L.c[i][a]) * u[a];
      for (int b = 0; b < 3; ++b) s2 = s2 + L.H2(i, a, b) * u[a] * u[b];
    }
    feq[i] = L.w[i] * rho * (1.0 + s1 / CS2 + s2 / (2.0 * CS2 * CS2) + L.third(i, a3));
  }
}

// Moments: rho = sum f, j = sum c f, P = sum c c f.  m = (rho, jx, jy, jz,
// Pxx, Pyy, Pzz, Pxy, Pxz, Pyz).
template <class T>
void moments_of(const T f[Q], T m[10], const Lattice& L = lat()) {
  for (int k = 0; k < 10; ++k) m[k] = T(0.0);
  for (int i = 0; i < L.q; ++i) {
    const int* c = L.c[i];
    m[0] = m[0] + f[i];
    m[1] = m[1] + double(c[0]) * f[i];
    m[2] = m[2] + double(c[1]) * f[i];
    m[3] = m[3] + double(c[2]) * f[i];
    m[4] = m[4] + double(c[0] * c[0]) * f[i];
    m[5] = m[5] + double(c[1] * c[1]) * f[i];
    m[6] = m[6] + double(c[2] * c[2]) * f[i];
    m[7] = m[7] + double(c[0] * c[1]) * f[i];
    m[8] = m[8] + double(c[0] * c[2]) * f[i];
    m[9] = m[9] + double(c[1] * c[2]) * f[i];
  }
}

inline void sym_index(int a, int b, int& k) {
  // index of P_ab in the 6-vector (xx, yy, zz, xy, xz, yz)
  if (a == b) { k = a; return; }
  int lo = a < b ? a : b, hi = a < b ? b : a;
  k = (lo == 0 && hi == 1) ? 3 : (lo == 0 && hi == 2) ? 4 : 5;
}

// ------------------------------------------------------------ collision
// One cell of the homogenized update (Sec. 2.2, eq. hlbm):
//   u_hat = (1-d) u + d (uB + uwm)                          (eq. convexVelocity, Sec. 2.2.1 last paragraph)
//   Pi    = P - rho cs^2 I - rho u_hat u_hat                  (non-equilibrium stress, recomputed from moments)
//   tau   = 1/2 [tau0 + sqrt(tau0^2 + 18 sqrt2 Cs^2 |Pi| / rho)]   (eq. tauEff with eqs. sgsStress/turbVisc)
//   f1    = w [H2:Pi/(2cs^4) + H3:a1^(3)/(6cs^6)], a1^(3)_abc = u_a Pi_bc + u_b Pi_ac + u_c Pi_ab (recursive)
//   f1fd  = w rho tau / cs^2 H2:S                             (FD non-equilibrium)
//   f*    = feq(rho, u_hat) + (1 - 1/tau) [sigma f1 - (1-sigma) f1fd]
//   dP    = j - rho u_hat    (momentum handed to the solid this step)
template <class T>
void collide_cell(const T m[10], const T& d, const double uB[3], const T uwm[3], const T Swm[6],
                  double sigma, double tau0, double Cs, T fstar[Q], T dP[3], const Lattice& L = lat()) {
  using std::sqrt;
  const T rho = m[0];
  T u[3], uh[3];
  for (int a = 0; a < 3; ++a) u[a] = m[1 + a] / rho;
  for (int a = 0; a < 3; ++a) uh[a] = (1.0 - d) * u[a] + d * (uB[a] + uwm[a]);
  T P[3][3], Pi[3][3], S[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      int k; sym_index(a, b, k);
      P[a][b] = m[4 + k];
      S[a][b] = Swm[k];
      Pi[a][b] = P[a][b] - rho * uh[a] * uh[b] - (a == b ? rho * CS2 : T(0.0));
    }
  T qq = T(0.0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) qq = qq + Pi[a][b] * Pi[a][b];
  T qn = re(qq) > 0.0 ? sqrt(qq) : T(0.0);
  const T tau = 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * std::sqrt(2.0) * Cs * Cs * qn / rho));
  T a3[3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) a3[a][b][c] = uh[a] * Pi[b][c] + uh[b] * Pi[a][c] + uh[c] * Pi[a][b];
  T feq[Q];
  equilibrium(rho, uh, feq, L);
  for (int i = 0; i < L.q; ++i) {
    T h2pi = T(0.0), h2s = T(0.0);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        h2pi = h2pi + L.H2(i, a, b) * Pi[a][b];
        h2s = h2s + L.H2(i, a, b) * S[a][b];
      }
    T f1 = L.w[i] * (h2pi / (2.0 * CS2 * CS2) + L.third(i, a3));
    T f1fd = L.w[i] * rho * tau / CS2 * h2s;
    T ftil = sigma * f1 - (1.0 - sigma) * f1fd;
    fstar[i] = feq[i] + (1.0 - 1.0 / tau) * ftil;
  }
  for (int a = 0; a < 3; ++a) dP[a] = m[1 + a] - rho * uh[a];
}

// ------------------------------------------------------------ wall model
// Truncated Spalding law (Sec. 2.2.1, eq. spalding) with the exponential's
// argument capped at 80 so that an overshooting iterate stays finite.
template <class T>
T spalding_bracket(const T& k) {
  using std::exp;
  T ek = re(k) > 80.0 ? T(std::exp(80.0)) : exp(k);
  return ek - 1.0 - k - k * k / 2.0 - k * k * k / 6.0;
}
template <class T>
T spalding_dbracket(const T& k) {  // d/dk of the bracket (the capped exponential is constant)
  using std::exp;
  T ek = re(k) > 80.0 ? T(0.0) : exp(k);
  return ek - 1.0 - k - k * k / 2.0;
}

// Counters of the wall model: Newton iterations for u_tau and cells solved;
// the safeguards of the Newton iterations (a non-positive iterate halved,
// an exponential argument capped at 80), which the parity cases must never
// reach; wall cells whose tangential slip lies within a factor two of the
// 1e-6 activity bound (where FP32 and FP64 could take different branches).
struct WallStats {
  int64_t newton_iters = 0;
  int64_t calls = 0;
  int64_t halvings = 0;
  int64_t capped = 0;
  int64_t near_threshold = 0;
};

// Newton-Raphson with the paper's stop rule |f(u^{j+1}) - f(u^j)| < tol, at most
// maxit iterations (Sec. 2.2.1); a non-positive iterate is replaced by half the
// previous one (counted in *halvings).
template <class T, class F, class DF>
T newton(T u, F f, DF df, double tol, int maxit, int* iters, int* halvings = nullptr) {
  T fu = f(u);
  int it = 0;
  for (; it < maxit; ++it) {
    T un = u - fu / df(u);
    if (re(un) <= 0.0) {
      un = 0.5 * u;
      if (halvings) ++*halvings;
    }
    T fn = f(un);
    bool done = std::fabs(re(fn) - re(fu)) < tol;
    u = un;
    fu = fn;
    if (done) { ++it; break; }
  }
  if (iters) *iters = it;
  return u;
}

// Implicit wall function for the friction velocity (eq. implicitWF):
//   f(ut) = p + (1/E) bracket(kappa p) - y ut / nu,  p = U / ut.
template <class T>
T wall_f(const T& ut, const T& U, double y, double nu, double E, double kappa) {
  T p = U / ut;
  return p + spalding_bracket(kappa * p) / E - y * ut / nu;
}
template <class T>
T wall_df(const T& ut, const T& U, double y, double nu, double E, double kappa) {
  T p = U / ut;
  return -(p / ut) * (1.0 + kappa * spalding_dbracket(kappa * p) / E) - y / nu;
}

template <class T>
struct WallOut {
  T uwm[3];
  T S[6];
  T utau;
  bool active;
  int iters_tau, iters_plus;
  double slip;          // tangential slip U (also for an inactive cell)
  int halvings, capped; // Newton safeguards taken (both solves)
};

// Wall model at one wall cell (Sec. 2.2.1 and Sec. 3.2):
//   v = u_s - u_w, v_t its tangential part, U = |v_t|, t = v_t / U;
//   u_tau from the implicit wall function at the sampling distance y_s, guess
//   u_tau^prev (cell active last step) or sqrt(nu U / y_s) (eq. guess);
//   u+ at the cell from the Spalding law at y1+ = y1 u_tau / nu;
//   u_wm = u_tau u+ t;  S = 1/2 (U - u_tau u+)/(y_s - y1) (t n^T + n t^T).
template <class T>
WallOut<T> wall_model_cell(const T us[3], const double uw[3], const double n[3], double y1,
                           const T& utau_prev, bool prev_active, const Params& p, double nu) {
  using std::sqrt;
  WallOut<T> o;
  T v[3];
  for (int a = 0; a < 3; ++a) v[a] = us[a] - uw[a];
  T vn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  T vt[3];
  for (int a = 0; a < 3; ++a) vt[a] = v[a] - vn * n[a];
  T U2 = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2];
  o.iters_tau = o.iters_plus = 0;
  o.halvings = o.capped = 0;
  o.slip = std::sqrt(re(U2));
  // below a tangential slip of 1e-6 lattice units (2e-5 of the free-stream
  // speed of the rotor workloads) the wall law is not applied: the slip
  // direction t is undefined as U -> 0 (on a rotor axis U vanishes by
  // symmetry), and the bound lies above FP32 rounding noise in U
  if (!(std::sqrt(re(U2)) >= 1e-6)) {
    o.active = false;
    for (int a = 0; a < 3; ++a) o.uwm[a] = T(0.0);
    for (int k = 0; k < 6; ++k) o.S[k] = T(0.0);
    o.utau = T(0.0);
    return o;
  }
  T U = sqrt(U2);
  T t[3];
  for (int a = 0; a < 3; ++a) t[a] = vt[a] / U;
  const double ys = p.y_s, E = p.E, kap = p.kappa;
  T guess = prev_active ? utau_prev : sqrt(nu * U / ys);
  // an evaluation whose exponential argument exceeds 80 takes the cap
  auto cap = [&](const T& k) { if (re(k) > 80.0) ++o.capped; };
  T ut = newton(
      guess, [&](const T& x) { cap(kap * (U / x)); return wall_f(x, U, ys, nu, E, kap); },
      [&](const T& x) { return wall_df(x, U, ys, nu, E, kap); }, p.tol, p.maxit, &o.iters_tau, &o.halvings);
  // u+ at the cell: Newton on Spalding's law from the two-layer estimate
  // min(y+, ln(E max(y+,1))/kappa) (viscous sublayer below y+ ~ 11, log law above)
  using std::log;
  T yp = y1 * ut / nu;
  T yl = re(yp) > 1.0 ? yp : T(1.0);
  T ulog = log(E * yl) / kap;
  T up0 = re(ulog) < re(yp) ? ulog : yp;
  T up = newton(
      up0, [&](const T& x) { cap(kap * x); return x + spalding_bracket(kap * x) / E - yp; },
      [&](const T& x) { return 1.0 + kap * spalding_dbracket(kap * x) / E; }, p.tol, p.maxit,
      &o.iters_plus, &o.halvings);
  T q = ut * up;
  for (int a = 0; a < 3; ++a) o.uwm[a] = q * t[a];
  T dudn = (U - q) / (ys - y1);
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      int k; sym_index(a, b, k);
      o.S[k] = 0.5 * dudn * (t[a] * n[b] + n[a] * t[b]);
    }
  o.utau = ut;
  o.active = true;
  return o;
}

// ------------------------------------------------------------ geometry
// Rotor made of flat-plate blades with linear twist plus a hub sphere, given
// as a signed distance phi (positive inside the solid).  The porosity follows
// the lattice-porosity definition of Sec. 2.2.2 (d = 0 for phi <= -eps/2,
// s(phi) inside the band, 1 for phi >= eps/2).
struct Frame { double e[3], e1[3], e2[3]; };

inline Frame rotor_frame(const Rotor& r) {
  Frame F;
  double n = std::sqrt(r.axis[0] * r.axis[0] + r.axis[1] * r.axis[1] + r.axis[2] * r.axis[2]);
  for (int a = 0; a < 3; ++a) F.e[a] = r.axis[a] / n;
  double a0[3] = {1, 0, 0};
  if (std::fabs(F.e[0]) >= 0.9) { a0[0] = 0; a0[1] = 1; }
  double ae = a0[0] * F.e[0] + a0[1] * F.e[1] + a0[2] * F.e[2];
  double e1[3];
  for (int a = 0; a < 3; ++a) e1[a] = a0[a] - ae * F.e[a];
  double n1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (int a = 0; a < 3; ++a) F.e1[a] = e1[a] / n1;
  F.e2[0] = F.e[1] * F.e1[2] - F.e[2] * F.e1[1];
  F.e2[1] = F.e[2] * F.e1[0] - F.e[0] * F.e1[2];
  F.e2[2] = F.e[0] * F.e1[1] - F.e[1] * F.e1[0];
  return F;
}

// Signed distance (positive inside) of rotor r turned to angle theta (blade
// b at theta + 2 pi b / n_blades) and its gradient.
inline double rotor_phi_at(const Rotor& r, const Frame& F, const double x[3], double theta, double grad[3]);

// Signed distance of rotor r at time step n of its prescribed rotation.
inline double rotor_phi(const Rotor& r, const Frame& F, const double x[3], int64_t n, double grad[3]) {
  return rotor_phi_at(r, F, x, r.phase0 + r.omega * double(n), grad);
}

// The body of a reference grid at rotor angle theta: the point's body
// coordinates p (projections on blade 0's radial and tangential directions
// and on the axis), grid coordinates u = (p - o) / h, and the trilinear
// interpolant of the eight surrounding samples; its gradient is that of the
// interpolant, taken back to the lattice frame.  A point outside the grid
// is not in the body (phi = -1e300, gradient zero).
inline double grid_phi_at(const RefGrid& G, const Frame& F, const double rel[3], double theta, double grad[3]) {
  for (int a = 0; a < 3; ++a) grad[a] = 0.0;
  const double ct = std::cos(theta), st = std::sin(theta);
  double axes[3][3];
  for (int a = 0; a < 3; ++a) {
    axes[0][a] = ct * F.e1[a] + st * F.e2[a];
    axes[1][a] = -st * F.e1[a] + ct * F.e2[a];
    axes[2][a] = F.e[a];
  }
  int i0[3];
  double f[3];
  for (int k = 0; k < 3; ++k) {
    const double p = rel[0] * axes[k][0] + rel[1] * axes[k][1] + rel[2] * axes[k][2];
    const double u = (p - G.o[k]) / G.h;
    if (!(u >= 0.0 && u <= double(G.n[k] - 1))) return -1e300;
    int i = int(std::floor(u));
    if (i > G.n[k] - 2) i = G.n[k] - 2;
    i0[k] = i;
    f[k] = u - double(i);
  }
  double phi = 0.0, du[3] = {0.0, 0.0, 0.0};
  for (int corner = 0; corner < 8; ++corner) {
    const int b[3] = {corner & 1, (corner >> 1) & 1, (corner >> 2) & 1};
    const double v = G.phi[((size_t)(i0[2] + b[2]) * G.n[1] + (i0[1] + b[1])) * G.n[0] + (i0[0] + b[0])];
    double w[3], dw[3];
    for (int k = 0; k < 3; ++k) {
      w[k] = b[k] ? f[k] : 1.0 - f[k];
      dw[k] = b[k] ? 1.0 : -1.0;
    }
    phi += w[0] * w[1] * w[2] * v;
    du[0] += dw[0] * w[1] * w[2] * v;
    du[1] += w[0] * dw[1] * w[2] * v;
    du[2] += w[0] * w[1] * dw[2] * v;
  }
  for (int a = 0; a < 3; ++a) grad[a] = (du[0] * axes[0][a] + du[1] * axes[1][a] + du[2] * axes[2][a]) / G.h;
  return phi;
}

inline double rotor_phi_at(const Rotor& r, const Frame& F, const double x[3], double theta, double grad[3]) {
  double rel[3] = {x[0] - r.center[0], x[1] - r.center[1], x[2] - r.center[2]};
  if (r.grid) return grid_phi_at(*r.grid, F, rel, theta, grad);
  double dist = std::sqrt(rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2]);
  // hub sphere
  double best = r.r_hub - dist;
  for (int a = 0; a < 3; ++a) grad[a] = dist > 0 ? -rel[a] / dist : 0.0;
  const double ax = rel[0] * F.e[0] + rel[1] * F.e[1] + rel[2] * F.e[2];
  const double two_pi = 6.283185307179586476925286766559;
  for (int b = 0; b < r.n_blades; ++b) {
    double th = theta + two_pi * double(b) / double(r.n_blades);
    double ct = std::cos(th), st = std::sin(th);
    double er[3], ep[3];
    for (int a = 0; a < 3; ++a) {
      er[a] = ct * F.e1[a] + st * F.e2[a];
      ep[a] = -st * F.e1[a] + ct * F.e2[a];
    }
    double rr = rel[0] * er[0] + rel[1] * er[1] + rel[2] * er[2];
    double qq = rel[0] * ep[0] + rel[1] * ep[1] + rel[2] * ep[2];
    double span = r.R - r.r_hub;
    double frac = (rr - r.r_hub) / span;
    double dbeta = 0.0;
    if (frac <= 0.0) frac = 0.0;
    else if (frac >= 1.0) frac = 1.0;
    else dbeta = (r.twist_tip - r.twist_root) / span;
    double beta = r.twist_root + (r.twist_tip - r.twist_root) * frac;
    double cb = std::cos(beta), sb = std::sin(beta);
    double s = -cb * qq + sb * ax;   // chord coordinate
    double h = cb * ax + sb * qq;    // thickness coordinate
    double p[3] = {rr - 0.5 * (r.R + r.r_hub), s, h};
    double half[3] = {0.5 * span, 0.5 * r.chord, 0.5 * r.thick};
    double q[3], qp[3];
    double qpn2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      q[k] = std::fabs(p[k]) - half[k];
      qp[k] = q[k] > 0 ? q[k] : 0.0;
      qpn2 += qp[k] * qp[k];
    }
    int kmax = 0;
    for (int k = 1; k < 3; ++k) if (q[k] > q[kmax]) kmax = k;
    double sdf = std::sqrt(qpn2) + (q[kmax] < 0 ? q[kmax] : 0.0);
    double phi = -sdf;
    if (phi > best) {
      best = phi;
      // gradient of sdf with respect to (p_r, s, h)
      double gp[3] = {0, 0, 0};
      if (qpn2 > 0) {
        double qn = std::sqrt(qpn2);
        for (int k = 0; k < 3; ++k) gp[k] = (p[k] >= 0 ? 1.0 : -1.0) * qp[k] / qn;
      } else {
        gp[kmax] = p[kmax] >= 0 ? 1.0 : -1.0;
      }
      // chain rule through r = rel.er, s(rel), h(rel) including the twist
      double gs_r = dbeta * (sb * qq + cb * ax);
      double gh_r = dbeta * (-sb * ax + cb * qq);
      for (int a = 0; a < 3; ++a) {
        double dr = er[a];
        double ds = -cb * ep[a] + sb * F.e[a] + gs_r * er[a];
        double dh = cb * F.e[a] + sb * ep[a] + gh_r * er[a];
        grad[a] = -(gp[0] * dr + gp[1] * ds + gp[2] * dh);
      }
    }
  }
  return best;
}

inline double transition_s(double phi, double eps, int kind) {
  if (phi <= -0.5 * eps) return 0.0;
  if (phi >= 0.5 * eps) return 1.0;
  if (kind == 1) return phi / eps + 0.5;
  return 0.5 * (1.0 + std::tanh(4.0 * phi / eps) / std::tanh(2.0));
}

// ------------------------------------------------------------ counter RNG
// splitmix64 (Steele, Lea, Flood 2014): output k of the generator seeded with s
// is mix(s + (k+1) * golden).  Gaussians from pairs of uniforms by Box-Muller.
inline uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
inline double inflow_gaussian(uint64_t seed, int64_t n, int y, int z, int comp, int ny, int nz) {
  uint64_t base = ((((uint64_t)n * (uint64_t)ny + (uint64_t)y) * (uint64_t)nz + (uint64_t)z) * 3ULL + (uint64_t)comp) * 2ULL;
  double u1 = 1.0 - (double)(splitmix64_at(seed, base) >> 11) * 0x1.0p-53;
  double u2 = (double)(splitmix64_at(seed, base + 1) >> 11) * 0x1.0p-53;
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586476925286766559 * u2);
}

}  // namespace oracle
