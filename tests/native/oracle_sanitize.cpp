// Drives the oracle through its C interface on small cases that reach every
// phase (rotor geometry, inflow turbulence, outflow, wall model, static
// porosity, control, the adjoint with checkpoints and the complex-step
// derivative), for a build with AddressSanitizer and UndefinedBehavior-
// Sanitizer.  Exit status 0 and "done" on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

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
void* oracle_create(int nx, int ny, int nz, int bc_x);
void oracle_destroy(void* h);
int oracle_set_params(void* h, const or_params* q);
int oracle_set_rotors(void* h, const or_rotor* r, int n);
int oracle_set_porosity_field(void* h, const double* d, const uint8_t* tag);
int oracle_set_control(void* h, const double* dd);
int oracle_init_equilibrium(void* h, const double* rho, const double* u);
int oracle_step(void* h, int64_t n);
int oracle_moments(void* h, double* rho, double* u, double* uhat);
int64_t oracle_history_len(void* h);
int oracle_history(void* h, int64_t from, int64_t to, double* dst);
int oracle_history_scale(void* h, int64_t from, int64_t to, double* dst);
void oracle_wall_safeguards(void* h, int64_t* out);
int oracle_adjoint_run(void* h, int64_t nsteps, int64_t t0, int64_t t1, int obj_tag, int ckpt_every, double* J,
                       double* G);
int oracle_complex_step_J(void* h, int64_t nsteps, int64_t t0, int64_t t1, int obj_tag, int64_t cell, double hstep,
                          double* J, double* dJ);
double oracle_trilinear(const double* q, int nx, int ny, int nz, int bc_x, const double* X);
}

int main() {
  const int nx = 20, ny = 16, nz = 14;
  const int64_t N = int64_t(nx) * ny * nz;
  or_params p{};
  p.tau0 = 0.52; p.cs_smag = 0.1; p.eps_h = 2.0; p.transition = 0; p.wall_model = 1;
  p.E = 9.8; p.kappa = 0.41; p.y_s = 3.0; p.tol = 1e-4; p.maxit = 10;
  p.u_in[0] = 0.05; p.turb_I = 0.05; p.seed = 9;
  or_rotor r{};
  r.center[0] = 6.3; r.center[1] = 8.2; r.center[2] = 6.9;
  r.axis[0] = 1.0;
  r.R = 5.0; r.r_hub = 1.2; r.chord = 2.5; r.thick = 2.0;
  r.twist_root = 0.35; r.twist_tip = 0.09; r.omega = 0.06; r.phase0 = 0.2;
  r.n_blades = 3; r.tag = 2;
  void* h = oracle_create(nx, ny, nz, 1);
  if (!h || oracle_set_params(h, &p) || oracle_set_rotors(h, &r, 1)) return 1;
  std::vector<double> d(N, 0.0), dd(N, 0.0), u(3 * N, 0.0), rho(N), uh(3 * N);
  std::vector<uint8_t> tag(N, 0);
  for (int64_t c = 0; c < N; ++c) {
    const int x = int(c % nx);
    if (x == nx - 3) { d[c] = 0.5; tag[c] = 1; }
    u[c] = 0.05;
    dd[c] = 1e-4 * double(c % 7);
  }
  oracle_set_porosity_field(h, d.data(), tag.data());
  oracle_set_control(h, dd.data());
  oracle_init_equilibrium(h, nullptr, u.data());
  oracle_step(h, 4);
  oracle_moments(h, rho.data(), u.data(), uh.data());
  const int64_t nh = oracle_history_len(h);
  std::vector<double> hist(91 * nh), scl(30 * nh);
  if (oracle_history(h, 0, nh, hist.data()) || oracle_history_scale(h, 0, nh, scl.data())) return 2;
  int64_t safe[3];
  oracle_wall_safeguards(h, safe);
  double J = 0.0, dJ = 0.0, Jc = 0.0;
  std::vector<double> G(N);
  if (oracle_adjoint_run(h, 5, 1, 5, 0, 2, &J, G.data())) return 3;
  if (oracle_complex_step_J(h, 3, 0, 3, 2, N / 2, 1e-30, &Jc, &dJ)) return 4;
  const double X[3] = {nx - 0.3, -0.4, nz + 0.2};
  const double q = oracle_trilinear(rho.data(), nx, ny, nz, 1, X);
  oracle_destroy(h);
  std::printf("J %.6e G[0] %.3e q %.6f safeguards %lld %lld %lld\n", J, G[0], q, (long long)safe[0],
              (long long)safe[1], (long long)safe[2]);
  if (!std::isfinite(J) || !std::isfinite(q)) return 5;
  std::printf("done\n");
  return 0;
}
