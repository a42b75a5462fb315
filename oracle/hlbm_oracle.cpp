// C interface of the oracle -- TEST INFRASTRUCTURE ONLY (see hlbm_oracle.hpp).
//
// Host FP64 buffers throughout; field layout [component][z][y][x] with x
// fastest; population order i = 9(cx+1) + 3(cy+1) + (cz+1).
#include "hlbm_oracle_sim.hpp"

#include <cstdio>
#include <memory>

using namespace oracle;

extern "C" {

struct or_params {
  double tau0, cs_smag, eps_h;
  int32_t transition, wall_model;
  double E, kappa, y_s, tol;
  int32_t maxit, pad0;
  double u_in[3];
  double turb_I;
  uint64_t seed;
  double fd_share;
};

struct or_rotor {
  double center[3], axis[3];
  double R, r_hub, chord, thick, twist_root, twist_tip, omega, phase0;
  int32_t n_blades, tag;
  double inertia, torque_gen;
};

static Params to_params(const or_params* q) {
  Params p{};
  p.tau0 = q->tau0; p.cs_smag = q->cs_smag; p.eps_h = q->eps_h; p.transition = q->transition;
  p.wall_model = q->wall_model; p.E = q->E; p.kappa = q->kappa; p.y_s = q->y_s; p.tol = q->tol;
  p.maxit = q->maxit; for (int a = 0; a < 3; ++a) p.u_in[a] = q->u_in[a];
  p.turb_I = q->turb_I; p.seed = q->seed;
  p.fd_share = q->fd_share;
  return p;
}

static Rotor to_rotor(const or_rotor* r) {
  Rotor o{};
  for (int a = 0; a < 3; ++a) { o.center[a] = r->center[a]; o.axis[a] = r->axis[a]; }
  o.R = r->R; o.r_hub = r->r_hub; o.chord = r->chord; o.thick = r->thick;
  o.twist_root = r->twist_root; o.twist_tip = r->twist_tip; o.omega = r->omega; o.phase0 = r->phase0;
  o.n_blades = r->n_blades; o.tag = r->tag;
  o.inertia = r->inertia; o.torque_gen = r->torque_gen;
  return o;
}

typedef Sim<double> SimD;

void* oracle_create(int nx, int ny, int nz, int bc_x) {
  if (nx < 2 || ny < 1 || nz < 1) return nullptr;
  return new SimD(nx, ny, nz, bc_x);
}
// The same on velocity set q (27 or 19).
void* oracle_create_q(int nx, int ny, int nz, int bc_x, int q) {
  if (nx < 2 || ny < 1 || nz < 1 || (q != 27 && q != 19)) return nullptr;
  return new SimD(nx, ny, nz, bc_x, q);
}
void oracle_destroy(void* h) { delete (SimD*)h; }
void oracle_set_threads(void* h, int n) { ((SimD*)h)->nthreads = n > 0 ? n : 1; }

int oracle_set_params(void* h, const or_params* q) {
  if (!(q->tau0 > 0.5) || q->maxit < 1 || !(q->eps_h > 0) || !(q->fd_share >= 0 && q->fd_share <= 1)) return 1;
  ((SimD*)h)->p = to_params(q);
  return 0;
}
int oracle_set_rotors(void* h, const or_rotor* r, int n) {
  std::vector<Rotor> v;
  for (int k = 0; k < n; ++k) {
    if (r[k].tag < 1 || r[k].tag > 15 || r[k].n_blades < 0) return 1;
    v.push_back(to_rotor(&r[k]));
  }
  ((SimD*)h)->set_rotors(v.data(), n);
  return 0;
}
int oracle_set_porosity_field(void* h, const double* d, const uint8_t* tag) {
  SimD* s = (SimD*)h;
  if (d) s->d_static.assign(d, d + s->N); else s->d_static.clear();
  if (tag) s->tag_static.assign(tag, tag + s->N); else s->tag_static.clear();
  return 0;
}
int oracle_set_solid_velocity(void* h, const double* uB) {
  SimD* s = (SimD*)h;
  if (uB) s->uB_static.assign(uB, uB + 3 * s->N); else s->uB_static.clear();
  return 0;
}
int oracle_set_control(void* h, const double* dd) {
  SimD* s = (SimD*)h;
  if (dd) s->dd.assign(dd, dd + s->N); else s->dd.clear();
  return 0;
}
int oracle_set_tag_frame(void* h, int tag, const double* c, const double* axis) {
  SimD* s = (SimD*)h;
  if (tag < 1 || tag > 15) return 1;
  double n = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
  if (!(n > 0)) return 1;
  for (int a = 0; a < 3; ++a) { s->tag_center[tag][a] = c[a]; s->tag_axis[tag][a] = axis[a] / n; }
  return 0;
}
int oracle_init_equilibrium(void* h, const double* rho, const double* u) {
  ((SimD*)h)->init_equilibrium(rho, u);
  return 0;
}
int oracle_step(void* h, int64_t n) {
  SimD* s = (SimD*)h;
  for (int64_t k = 0; k < n; ++k) s->do_step();
  return 0;
}
int64_t oracle_get_step(void* h) { return ((SimD*)h)->step; }
// Angle and angular velocity of each rotor at the current step.
int oracle_rotor_state(void* h, double* theta, double* omega) {
  SimD* s = (SimD*)h;
  for (size_t k = 0; k < s->rotors.size(); ++k) {
    theta[k] = s->angle(k, s->step);
    omega[k] = s->speed(k);
  }
  return int(s->rotors.size());
}

// rho, u of the pre-collision populations f(x, n) and the homogenized velocity
// u_hat of the collision at step n (u_hat = post-collision momentum / rho);
// the lattice state is left untouched.
int oracle_moments(void* h, double* rho, double* u, double* uhat) {
  SimD* s = (SimD*)h;
  s->geometry(s->step);
  s->pull(s->step);
  s->moments();
  const int64_t N = s->N;
  for (int64_t c = 0; c < N; ++c) {
    if (rho) rho[c] = s->mom[c];
    if (u) for (int a = 0; a < 3; ++a) u[(size_t)a * N + c] = s->u[(size_t)a * N + c];
  }
  if (uhat) {
    std::vector<double> ut = s->utau;
    std::vector<uint8_t> ac = s->active;
    WallStats ws = s->wstats;
    if (s->p.wall_model) s->wall_model();
    else { s->uwm.assign(3 * N, 0.0); }
    for (int64_t c = 0; c < N; ++c)
      for (int a = 0; a < 3; ++a)
        uhat[(size_t)a * N + c] = (1.0 - s->d[c]) * s->u[(size_t)a * N + c] +
                                  s->d[c] * (s->g_uB[3 * c + a] + s->uwm[(size_t)a * N + c]);
    s->utau = ut; s->active = ac; s->wstats = ws;
  }
  return 0;
}

int oracle_get_populations(void* h, double* dst) {
  SimD* s = (SimD*)h;
  std::memcpy(dst, s->h.data(), sizeof(double) * s->q * s->N);
  return 0;
}
int oracle_set_populations(void* h, const double* src) {
  SimD* s = (SimD*)h;
  std::memcpy(s->h.data(), src, sizeof(double) * s->q * s->N);
  return 0;
}
int oracle_get_wall_state(void* h, double* utau, uint8_t* active) {
  SimD* s = (SimD*)h;
  if (utau) std::memcpy(utau, s->utau.data(), sizeof(double) * s->N);
  if (active) std::memcpy(active, s->active.data(), s->N);
  return 0;
}
int oracle_set_wall_state(void* h, const double* utau, const uint8_t* active, int64_t step) {
  SimD* s = (SimD*)h;
  std::memcpy(s->utau.data(), utau, sizeof(double) * s->N);
  std::memcpy(s->active.data(), active, s->N);
  s->step = step;
  return 0;
}
int oracle_history(void* h, int64_t from, int64_t to, double* dst) {
  SimD* s = (SimD*)h;
  int64_t n = (int64_t)s->hist.size() / HIST;
  if (from < 0 || to > n || from > to) return 1;
  std::memcpy(dst, s->hist.data() + from * HIST, sizeof(double) * HIST * (to - from));
  return 0;
}
int64_t oracle_history_len(void* h) { return (int64_t)((SimD*)h)->hist.size() / HIST; }
void oracle_clear_history(void* h) {
  SimD* s = (SimD*)h;
  s->hist.clear();
  s->hist_scale.clear();
  s->hist_me.clear();
  s->hist_me_scale.clear();
}
// Per recorded step [from, to) and tag 1..15: sum of |dP| and of |r x dP|
// over the tag's cells (30 doubles per step).
int oracle_history_scale(void* h, int64_t from, int64_t to, double* dst) {
  SimD* s = (SimD*)h;
  int64_t n = (int64_t)s->hist_scale.size() / 30;
  if (from < 0 || to > n || from > to) return 1;
  std::memcpy(dst, s->hist_scale.data() + from * 30, sizeof(double) * 30 * (to - from));
  return 0;
}
// Momentum-exchange forces of the recorded steps [from, to) of a run with the
// estimator switched on (oracle_set_force_mode), 45 doubles per step: tags
// 1..15 x F_ME[3].
void oracle_set_force_mode(void* h, int mode) { ((SimD*)h)->with_me = (mode & 1) != 0; }
int64_t oracle_history_me_len(void* h) { return (int64_t)((SimD*)h)->hist_me.size() / 45; }
// Per recorded step and tag: the sum of the magnitudes of the link terms of
// the momentum-exchange force (15 doubles per step).
int oracle_history_me_scale(void* h, int64_t from, int64_t to, double* dst) {
  SimD* s = (SimD*)h;
  int64_t n = (int64_t)s->hist_me_scale.size() / 15;
  if (from < 0 || to > n || from > to) return 1;
  std::memcpy(dst, s->hist_me_scale.data() + from * 15, sizeof(double) * 15 * (to - from));
  return 0;
}
int oracle_history_me(void* h, int64_t from, int64_t to, double* dst) {
  SimD* s = (SimD*)h;
  int64_t n = (int64_t)s->hist_me.size() / 45;
  if (from < 0 || to > n || from > to) return 1;
  std::memcpy(dst, s->hist_me.data() + from * 45, sizeof(double) * 45 * (to - from));
  return 0;
}
// Newton halvings, exponential caps and near-threshold slips since creation.
void oracle_wall_safeguards(void* h, int64_t* out) {
  const WallStats& w = ((SimD*)h)->wstats;
  out[0] = w.halvings;
  out[1] = w.capped;
  out[2] = w.near_threshold;
}
// Trilinear sample of a scalar field q ([z][y][x]) at X with the wall model's
// boundary handling (periodic y, z; x periodic or clamped).
double oracle_trilinear(const double* q, int nx, int ny, int nz, int bc_x, const double* X) {
  return trilinear(q, nx, ny, nz, bc_x, X);
}
int64_t oracle_wall_newton_iters(void* h) { return ((SimD*)h)->wstats.newton_iters; }
int64_t oracle_wall_calls(void* h) { return ((SimD*)h)->wstats.calls; }

// Geometry of the current step: porosity d (incl. control), tag, wall-cell
// flag, signed distance of the nearest rotor, outward normal, solid velocity.
int oracle_geometry(void* h, double* d, uint8_t* tag, uint8_t* wall, double* phi, double* n, double* uB) {
  SimD* s = (SimD*)h;
  s->geometry(s->step);
  const int64_t N = s->N;
  for (int64_t c = 0; c < N; ++c) {
    if (d) d[c] = s->d[c];
    if (tag) tag[c] = s->g_tag[c];
    if (wall) wall[c] = s->g_wall[c];
    if (phi) phi[c] = s->g_phi[c];
    for (int a = 0; a < 3; ++a) {
      if (n) n[(size_t)a * N + c] = s->g_n[3 * c + a];
      if (uB) uB[(size_t)a * N + c] = s->g_uB[3 * c + a];
    }
  }
  return 0;
}

// ----------------------------------------------------- cell-level entry points
void oracle_lattice(int32_t* c, double* w) {
  const Lattice& L = lat();
  for (int i = 0; i < L.q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
    w[i] = L.w[i];
  }
}
// Velocities and weights of set q (27 or 19); returns its size.
int oracle_lattice_q(int q, int32_t* c, double* w) {
  const Lattice& L = lattice(q);
  for (int i = 0; i < L.q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
    w[i] = L.w[i];
  }
  return L.q;
}
void oracle_equilibrium(double rho, const double* u, double* feq) { equilibrium(rho, u, feq); }
void oracle_equilibrium_q(int q, double rho, const double* u, double* feq) { equilibrium(rho, u, feq, lattice(q)); }
void oracle_collide_cell(const double* m, double d, const double* uB, const double* uwm, const double* S,
                         double sigma, double tau0, double Cs, double* fstar, double* dP) {
  collide_cell(m, d, uB, uwm, S, sigma, tau0, Cs, fstar, dP);
}
void oracle_collide_cell_q(int q, const double* m, double d, const double* uB, const double* uwm, const double* S,
                           double sigma, double tau0, double Cs, double* fstar, double* dP) {
  collide_cell(m, d, uB, uwm, S, sigma, tau0, Cs, fstar, dP, lattice(q));
}
void oracle_moments_of(const double* f, double* m) { moments_of(f, m); }
void oracle_moments_of_q(int q, const double* f, double* m) { moments_of(f, m, lattice(q)); }
double oracle_spalding_yplus(double up, double E, double kappa) { return up + spalding_bracket(kappa * up) / E; }
// out = (uwm[3], S[6], utau, active, Newton halvings, exponential caps);
// returns Newton iterations for u_tau.
int oracle_wall_cell(const double* us, const double* uw, const double* n, double y1, double utau_prev,
                     int prev_active, const or_params* q, double* out, int* iters_plus) {
  Params p = to_params(q);
  double nu = CS2 * (p.tau0 - 0.5);
  WallOut<double> o = wall_model_cell(us, uw, n, y1, utau_prev, prev_active != 0, p, nu);
  for (int a = 0; a < 3; ++a) out[a] = o.uwm[a];
  for (int k = 0; k < 6; ++k) out[3 + k] = o.S[k];
  out[9] = o.utau;
  out[10] = o.active ? 1.0 : 0.0;
  out[11] = o.halvings;
  out[12] = o.capped;
  if (iters_plus) *iters_plus = o.iters_plus;
  return o.iters_tau;
}
double oracle_rotor_phi(const or_rotor* r, const double* x, int64_t n, double* grad) {
  Rotor ro = to_rotor(r);
  Frame F = rotor_frame(ro);
  return rotor_phi(ro, F, x, n, grad);
}
double oracle_transition(double phi, double eps, int kind) { return transition_s(phi, eps, kind); }
int oracle_set_rotor_grid(void* h, int k, const double* phi, int n0, int n1, int n2, double spacing,
                          const double* origin) {
  if (k < 0 || k >= 8) return 1;
  if (phi && (n0 < 2 || n1 < 2 || n2 < 2 || !(spacing > 0) || !origin)) return 1;
  const int n[3] = {n0, n1, n2};
  ((SimD*)h)->set_grid(k, phi, n, spacing, origin);
  return 0;
}
// Distance and gradient of a reference-grid body of rotor r at angle theta.
double oracle_grid_rotor_phi(const or_rotor* r, const double* phi, int n0, int n1, int n2, double spacing,
                             const double* origin, const double* x, double theta, double* grad) {
  RefGrid G;
  G.phi.assign(phi, phi + (size_t)n0 * n1 * n2);
  G.n[0] = n0; G.n[1] = n1; G.n[2] = n2;
  G.h = spacing;
  for (int a = 0; a < 3; ++a) G.o[a] = origin[a];
  Rotor ro = to_rotor(r);
  ro.grid = &G;
  return rotor_phi_at(ro, rotor_frame(ro), x, theta, grad);
}
double oracle_gaussian(uint64_t seed, int64_t n, int y, int z, int comp, int ny, int nz) {
  return inflow_gaussian(seed, n, y, z, comp, ny, nz);
}
uint64_t oracle_splitmix64(uint64_t seed, uint64_t k) { return splitmix64_at(seed, k); }

}  // extern "C"
