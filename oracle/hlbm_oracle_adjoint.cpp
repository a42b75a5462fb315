// Discrete adjoint of the oracle time stepping -- TEST INFRASTRUCTURE ONLY.
//
// Objective: J = 1/(t1 - t0) * sum over steps n in [t0, t1) (counted from the
// start of the run) of the axial torque e_k . T_k(n) of the selected tag
// (0 = all tags), T_k = sum_{tag k} (x - x_k) x dP with dP = j - rho u_hat the
// momentum handed to the solid (Sec. 2.2.2, force integration per tag).
// Control: the porosity offset delta_d added to d in every cell.  The
// gradient G = dJ/d(delta_d) is the exact derivative of the discrete map,
// Newton iterations of the wall model included as executed (their stop
// decisions held fixed), computed in reverse with checkpoints.
//
// Local Jacobians come from forward-mode dual numbers through the same
// templated cell functions the forward oracle uses; the reverse sweep only
// transposes them.  The complex-step entry point differentiates the forward
// oracle directly and pins this adjoint.
#include "hlbm_oracle_sim.hpp"

#include <array>
#include <complex>

using namespace oracle;

namespace {

struct Snapshot {
  std::vector<double> h, utau;
  std::vector<uint8_t> active;
  int64_t step;
};

Snapshot snap(const Sim<double>& s) { return Snapshot{s.h, s.utau, s.active, s.step}; }
void restore(Sim<double>& s, const Snapshot& z) {
  s.h = z.h;
  s.utau = z.utau;
  s.active = z.active;
  s.step = z.step;
}

typedef Dual<20> D20;
typedef Dual<4> D4;

// Reverse of one step n.  Inputs: the lattice holding the state at n, the
// adjoint lam of the post-collision state of step n and UT of the friction
// velocity state written by step n.  Outputs: lam_out (adjoint of the state
// at n), UT_out (adjoint of the friction velocity state read by step n); G
// accumulates dJ/d(delta_d).
void adjoint_step(Sim<double>& s, int64_t n, double obj_weight, int obj_tag, const std::vector<double>& lam,
                  const std::vector<double>& UT, std::vector<double>& lam_out, std::vector<double>& UT_out,
                  double* G) {
  const Lattice& L = *s.lat_;
  const int q = s.q;
  const int64_t N = s.N;
  const int nx = s.nx, ny = s.ny, nz = s.nz;
  s.geometry(n);
  s.pull(n);
  s.moments();
  const Params& p = s.p;
  const double nu = CS2 * (p.tau0 - 0.5);
  // ---- wall model values and Jacobians (inputs: probe velocity, u_tau^prev)
  std::vector<double> uwm(3 * N, 0.0), Swm(6 * N, 0.0), sig(N, 1.0);
  std::vector<double> Jw;             // per wall cell: 10 outputs x 4 inputs
  std::vector<int64_t> wcells;
  std::vector<std::array<double, 3>> xs_of;
  if (p.wall_model) {
    for (int64_t c = 0; c < N; ++c) {
      if (!s.g_wall[c]) continue;
      const int x = int(c % nx), y = int((c / nx) % ny), z = int(c / ((int64_t)nx * ny));
      const Rotor& R = s.rotors[s.g_rot[c]];
      const Frame& F = s.frames[s.g_rot[c]];
      const double* nn = &s.g_n[3 * c];
      const double y1 = -s.g_phi[c];
      double xw[3], xs[3];
      const double X[3] = {double(x), double(y), double(z)};
      for (int a = 0; a < 3; ++a) { xw[a] = X[a] - y1 * nn[a]; xs[a] = xw[a] + p.y_s * nn[a]; }
      double rel[3] = {xw[0] - R.center[0], xw[1] - R.center[1], xw[2] - R.center[2]};
      double uw[3] = {R.omega * (F.e[1] * rel[2] - F.e[2] * rel[1]), R.omega * (F.e[2] * rel[0] - F.e[0] * rel[2]),
                      R.omega * (F.e[0] * rel[1] - F.e[1] * rel[0])};
      double us[3];
      s.sample_u(xs, us);
      D4 usd[3];
      for (int a = 0; a < 3; ++a) { usd[a] = D4(us[a]); usd[a].g[a] = 1.0; }
      D4 utp(s.utau[c]);
      utp.g[3] = 1.0;
      WallOut<D4> o = wall_model_cell(usd, uw, nn, y1, utp, s.active[c] != 0, p, nu);
      if (!o.active) continue;
      for (int a = 0; a < 3; ++a) uwm[(size_t)a * N + c] = o.uwm[a].v;
      for (int k = 0; k < 6; ++k) Swm[(size_t)k * N + c] = o.S[k].v;
      sig[c] = 0.0;
      wcells.push_back(c);
      xs_of.push_back({xs[0], xs[1], xs[2]});
      for (int a = 0; a < 3; ++a) for (int r = 0; r < 4; ++r) Jw.push_back(o.uwm[a].g[r]);
      for (int k = 0; k < 6; ++k) for (int r = 0; r < 4; ++r) Jw.push_back(o.S[k].g[r]);
      for (int r = 0; r < 4; ++r) Jw.push_back(o.utau.g[r]);
    }
  }
  // ---- hybrid non-equilibrium off the wall: sigma = 1 - fd_share and the
  // central-difference strain of the pre-collision velocity in the element
  // cells that are not active wall cells (as in the forward step)
  std::vector<int64_t> fdcells;
  if (p.fd_share > 0.0) {
    s.sigma = sig;
    s.Swm = Swm;
    s.fd_strain();
    for (int64_t c = 0; c < N; ++c)
      if (s.sigma[c] != sig[c]) fdcells.push_back(c);
    sig = s.sigma;
    Swm = s.Swm;
  }
  // ---- collision adjoint per cell
  std::vector<double> mbar(10 * N, 0.0), uwbar(3 * N, 0.0), Sbar(6 * N, 0.0);
#pragma omp parallel for num_threads(s.nthreads) schedule(static)
  for (int64_t c = 0; c < N; ++c) {
    const int x = int(c % nx), y = int((c / nx) % ny), z = int(c / ((int64_t)nx * ny));
    double fbar[Q];
    for (int i = 0; i < q; ++i) fbar[i] = lam[(size_t)i * N + c];
    double pbar[3] = {0, 0, 0};
    const int t = s.g_tag[c];
    if (obj_weight != 0.0 && t != 0 && (obj_tag == 0 || obj_tag == t)) {
      const double r[3] = {x - s.tag_center[t][0], y - s.tag_center[t][1], z - s.tag_center[t][2]};
      const double* e = s.tag_axis[t];
      pbar[0] = obj_weight * (e[1] * r[2] - e[2] * r[1]);
      pbar[1] = obj_weight * (e[2] * r[0] - e[0] * r[2]);
      pbar[2] = obj_weight * (e[0] * r[1] - e[1] * r[0]);
    }
    D20 m[10], dd, uw3[3], S6[6], fs[Q], dp[3];
    for (int k = 0; k < 10; ++k) { m[k] = D20(s.mom[(size_t)k * N + c]); m[k].g[k] = 1.0; }
    dd = D20(s.d[c]);
    dd.g[10] = 1.0;
    for (int a = 0; a < 3; ++a) { uw3[a] = D20(uwm[(size_t)a * N + c]); uw3[a].g[11 + a] = 1.0; }
    for (int k = 0; k < 6; ++k) { S6[k] = D20(Swm[(size_t)k * N + c]); S6[k].g[14 + k] = 1.0; }
    collide_cell(m, dd, &s.g_uB[3 * c], uw3, S6, sig[c], p.tau0, p.cs_smag, fs, dp, L);
    double xbar[20] = {0};
    for (int r = 0; r < 20; ++r) {
      double acc = 0.0;
      for (int i = 0; i < q; ++i) acc += fbar[i] * fs[i].g[r];
      for (int a = 0; a < 3; ++a) acc += pbar[a] * dp[a].g[r];
      xbar[r] = acc;
    }
    for (int k = 0; k < 10; ++k) mbar[(size_t)k * N + c] = xbar[k];
    G[c] += xbar[10];
    for (int a = 0; a < 3; ++a) uwbar[(size_t)a * N + c] = xbar[11 + a];
    for (int k = 0; k < 6; ++k) Sbar[(size_t)k * N + c] = xbar[14 + k];
  }
  // ---- wall model adjoint: probe velocity -> the 8 probe corners' velocities
  std::fill(UT_out.begin(), UT_out.end(), 0.0);
  std::vector<double> ubar(3 * N, 0.0);
  for (size_t w = 0; w < wcells.size(); ++w) {
    const int64_t c = wcells[w];
    const double* J = &Jw[w * 40];
    double out_bar[10];
    for (int a = 0; a < 3; ++a) out_bar[a] = uwbar[(size_t)a * N + c];
    for (int k = 0; k < 6; ++k) out_bar[3 + k] = Sbar[(size_t)k * N + c];
    out_bar[9] = UT[c];
    double in_bar[4] = {0, 0, 0, 0};
    for (int o = 0; o < 10; ++o)
      for (int r = 0; r < 4; ++r) in_bar[r] += out_bar[o] * J[o * 4 + r];
    UT_out[c] += in_bar[3];
    // trilinear weights of the probe, as in Sim::sample_u
    const double* X = xs_of[w].data();
    int i0[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) { double fl = std::floor(X[a]); i0[a] = (int)fl; fr[a] = X[a] - fl; }
    for (int corner = 0; corner < 8; ++corner) {
      int qd[3];
      double wgt = 1.0;
      for (int a = 0; a < 3; ++a) {
        int bit = (corner >> a) & 1;
        qd[a] = i0[a] + bit;
        wgt *= bit ? fr[a] : 1.0 - fr[a];
      }
      qd[1] = Sim<double>::wrap(qd[1], ny);
      qd[2] = Sim<double>::wrap(qd[2], nz);
      if (s.bc_x == 0) qd[0] = Sim<double>::wrap(qd[0], nx);
      else qd[0] = qd[0] < 0 ? 0 : (qd[0] > nx - 1 ? nx - 1 : qd[0]);
      const int64_t cc = s.idx(qd[0], qd[1], qd[2]);
      for (int a = 0; a < 3; ++a) ubar[(size_t)a * N + cc] += wgt * in_bar[a];
    }
  }
  // ---- the strain of the hybrid cells: S_ab = (d_a u_b + d_b u_a) / 2 with
  // d_b u_a = (u_a(x + e_b) - u_a(x - e_b)) / 2 -> velocity adjoints of the
  // neighbours (the same neighbour rules as the forward strain)
  for (const int64_t c : fdcells) {
    const int x = int(c % nx), y = int((c / nx) % ny), z = int(c / ((int64_t)nx * ny));
    const int xm = s.bc_x == 0 ? Sim<double>::wrap(x - 1, nx) : (x > 0 ? x - 1 : 0);
    const int xp = s.bc_x == 0 ? Sim<double>::wrap(x + 1, nx) : (x < nx - 1 ? x + 1 : nx - 1);
    int64_t nb[3][2];
    nb[0][0] = s.idx(xm, y, z);
    nb[0][1] = s.idx(xp, y, z);
    nb[1][0] = s.idx(x, Sim<double>::wrap(y - 1, ny), z);
    nb[1][1] = s.idx(x, Sim<double>::wrap(y + 1, ny), z);
    nb[2][0] = s.idx(x, y, Sim<double>::wrap(z - 1, nz));
    nb[2][1] = s.idx(x, y, Sim<double>::wrap(z + 1, nz));
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        int k;
        sym_index(a, b, k);
        // adjoint of d_b u_a: S_aa = d_a u_a; S_ab = (d_b u_a + d_a u_b) / 2
        const double dub = (a == b ? 1.0 : 0.5) * Sbar[(size_t)k * N + c];
        ubar[(size_t)a * N + nb[b][1]] += 0.5 * dub;
        ubar[(size_t)a * N + nb[b][0]] -= 0.5 * dub;
      }
  }
  // ---- u = j / rho into the moment adjoints, then moments -> populations
  std::fill(lam_out.begin(), lam_out.end(), 0.0);
  std::vector<double> mu((size_t)Q * N);
#pragma omp parallel for num_threads(s.nthreads) schedule(static)
  for (int64_t c = 0; c < N; ++c) {
    double mb[10];
    for (int k = 0; k < 10; ++k) mb[k] = mbar[(size_t)k * N + c];
    const double rho = s.mom[c];
    for (int a = 0; a < 3; ++a) {
      const double ub = ubar[(size_t)a * N + c];
      const double j = s.mom[(size_t)(1 + a) * N + c];
      mb[0] -= ub * j / (rho * rho);
      mb[1 + a] += ub / rho;
    }
    for (int i = 0; i < q; ++i) {
      const int* ci = L.c[i];
      mu[(size_t)i * N + c] = mb[0] + ci[0] * mb[1] + ci[1] * mb[2] + ci[2] * mb[3] + ci[0] * ci[0] * mb[4] +
                              ci[1] * ci[1] * mb[5] + ci[2] * ci[2] * mb[6] + ci[0] * ci[1] * mb[7] +
                              ci[0] * ci[2] * mb[8] + ci[1] * ci[2] * mb[9];
    }
  }
  // ---- transpose of the pull: f_i(x) = state_i(x - c_i) (inflow: no state)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t c = s.idx(x, y, z);
        for (int i = 0; i < q; ++i) {
          int xs = x - L.c[i][0];
          const int ys = Sim<double>::wrap(y - L.c[i][1], ny), zs = Sim<double>::wrap(z - L.c[i][2], nz);
          if (s.bc_x == 0) xs = Sim<double>::wrap(xs, nx);
          else if (xs < 0) continue;
          else if (xs > nx - 1) xs = nx - 1;
          lam_out[(size_t)i * N + s.idx(xs, ys, zs)] += mu[(size_t)i * N + c];
        }
      }
}

}  // namespace

extern "C" {

// Forward nsteps from the current state recording J over steps [t0, t1) of the
// run, then the reverse sweep; G[c] = dJ/d(delta_d)(c).  The lattice ends in
// the forward final state.
int oracle_adjoint_run(void* hp, int64_t nsteps, int64_t t0, int64_t t1, int obj_tag, int ckpt_every, double* J_out,
                       double* G) {
  Sim<double>& s = *(Sim<double>*)hp;
  if (nsteps < 1 || t0 < 0 || t1 <= t0 || t1 > nsteps || ckpt_every < 1) return 1;
  for (const Rotor& r : s.rotors)
    if (r.inertia > 0) return 1;     // and for prescribed rotations
  const int64_t n0 = s.step, N = s.N;
  s.obj_on = true;
  s.obj_t0 = n0 + t0;
  s.obj_t1 = n0 + t1;
  s.obj_tag = obj_tag;
  s.J = 0.0;
  std::vector<Snapshot> ck;
  for (int64_t k = 0; k < nsteps; ++k) {
    if (k % ckpt_every == 0) ck.push_back(snap(s));
    s.do_step();
  }
  s.obj_on = false;
  *J_out = s.J;
  const Snapshot fin = snap(s);
  const size_t hist_len = s.hist.size(), scale_len = s.hist_scale.size();
  const double wgt = 1.0 / double(t1 - t0);
  std::vector<double> lam((size_t)Q * N, 0.0), lam2((size_t)Q * N), UT(N, 0.0), UT2(N);
  for (int64_t c = 0; c < N; ++c) G[c] = 0.0;
  for (int64_t seg = (int64_t)ck.size() - 1; seg >= 0; --seg) {
    restore(s, ck[seg]);
    const int64_t a = seg * ckpt_every, b = std::min<int64_t>(nsteps, a + ckpt_every);
    std::vector<Snapshot> states;
    for (int64_t k = a; k < b; ++k) {
      states.push_back(snap(s));
      if (k + 1 < b) s.do_step();
    }
    for (int64_t k = b - 1; k >= a; --k) {
      restore(s, states[k - a]);
      const double w = (k >= t0 && k < t1) ? wgt : 0.0;
      adjoint_step(s, n0 + k, w, obj_tag, lam, UT, lam2, UT2, G);
      lam.swap(lam2);
      UT.swap(UT2);
    }
  }
  restore(s, fin);
  s.hist.resize(hist_len);
  s.hist_scale.resize(scale_len);
  return 0;
}

// (J, dJ/d(delta_d at cell)) by the complex-step method: the forward oracle run
// in complex arithmetic with delta_d(cell) += i h.  The lattice is unchanged.
int oracle_complex_step_J(void* hp, int64_t nsteps, int64_t t0, int64_t t1, int obj_tag, int64_t cell, double hstep,
                          double* J, double* dJ) {
  typedef std::complex<double> C;
  const Sim<double>& s = *(const Sim<double>*)hp;
  if (cell < 0 || cell >= s.N || t1 <= t0 || t0 < 0) return 1;
  for (const Rotor& r : s.rotors)
    if (r.inertia > 0) return 1;  // prescribed rotations only
  Sim<C> z(s.nx, s.ny, s.nz, s.bc_x, s.q);
  z.p = s.p;
  z.set_rotors(s.rotors.data(), (int)s.rotors.size());
  for (int t = 0; t < NTAG; ++t)
    for (int a = 0; a < 3; ++a) { z.tag_center[t][a] = s.tag_center[t][a]; z.tag_axis[t][a] = s.tag_axis[t][a]; }
  z.d_static = s.d_static;
  z.uB_static = s.uB_static;
  z.tag_static = s.tag_static;
  z.nthreads = s.nthreads;
  z.dd.assign(s.N, C(0.0));
  for (int64_t c = 0; c < s.N && !s.dd.empty(); ++c) z.dd[c] = C(s.dd[c]);
  z.dd[cell] += C(0.0, hstep);
  for (size_t k = 0; k < s.h.size(); ++k) z.h[k] = C(s.h[k]);
  for (int64_t c = 0; c < s.N; ++c) z.utau[c] = C(s.utau[c]);
  z.active = s.active;
  z.step = s.step;
  z.obj_on = true;
  z.obj_t0 = s.step + t0;
  z.obj_t1 = s.step + t1;
  z.obj_tag = obj_tag;
  z.J = C(0.0);
  for (int64_t k = 0; k < nsteps; ++k) z.do_step();
  *J = z.J.real();
  *dJ = z.J.imag() / hstep;
  return 0;
}

}  // extern "C"
