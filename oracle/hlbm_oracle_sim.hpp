// Whole-lattice oracle time stepping -- TEST INFRASTRUCTURE ONLY.
//
// One step n -> n+1, phase by phase over the whole grid (the order of the
// algorithm of Sec. 3.2, read for a pull scheme):
//   1. geometry of every rotor at step n (porosity, tag, normal, wall distance)
//   2. pre-collision populations f(x,n) = f*(x - c_i, n-1) with the outer
//      boundaries (periodic y,z; periodic or inflow/outflow in x)
//   3. moments rho, j, P of f(x,n)
//   4. wall model on the wall cells
//   5. collision of every cell, momentum handed to each tagged solid
//   6. the post-collision populations become the new state.
// The state is f*(x) of the previous step, held as h = f* - w.
#pragma once
#include "hlbm_oracle.hpp"

namespace oracle {

constexpr int NTAG = 16;         // tags 0..15; tag 0 means "no solid element"
constexpr int HIST = 1 + 15 * 6; // per step: mass, then (F, T) for tags 1..15

// Trilinear interpolation of a cell-centred field q (layout [z][y][x]) at
// point X (Sec. 3.2: the wall model samples the velocity at a configurable
// distance from the wall): the eight cells around X weighted by products of
// the fractional offsets, y and z periodic, x periodic or clamped to the
// first and last plane (inflow/outflow lattices).
template <class T>
T trilinear(const T* q, int nx, int ny, int nz, int bc_x, const double X[3]) {
  const int n3[3] = {nx, ny, nz};
  int i0[3];
  double fr[3];
  for (int a = 0; a < 3; ++a) { double fl = std::floor(X[a]); i0[a] = (int)fl; fr[a] = X[a] - fl; }
  T acc = T(0.0);
  for (int corner = 0; corner < 8; ++corner) {
    int c[3];
    double wgt = 1.0;
    for (int a = 0; a < 3; ++a) {
      int bit = (corner >> a) & 1;
      c[a] = i0[a] + bit;
      wgt *= bit ? fr[a] : 1.0 - fr[a];
    }
    for (int a = 1; a < 3; ++a) c[a] = ((c[a] % n3[a]) + n3[a]) % n3[a];
    if (bc_x == 0) c[0] = ((c[0] % nx) + nx) % nx;
    else c[0] = c[0] < 0 ? 0 : (c[0] > nx - 1 ? nx - 1 : c[0]);
    acc = acc + wgt * q[((int64_t)c[2] * ny + c[1]) * nx + c[0]];
  }
  return acc;
}

template <class T>
struct Sim {
  int nx = 0, ny = 0, nz = 0, bc_x = 0;  // bc_x: 0 periodic, 1 inflow at x=0 / outflow at x=nx-1
  int64_t N = 0;
  Params p{};
  std::vector<Rotor> rotors;
  std::vector<RefGrid> grids = std::vector<RefGrid>(8);  // reference grid per rotor index (empty: none)
  std::vector<Frame> frames;
  // rotation of each rotor: angle and angular velocity of the current step
  // (prescribed: phase0 + omega n and omega; coupled: the rigid-body state)
  std::vector<double> theta, Omega;
  std::vector<double> d_static, uB_static;
  std::vector<uint8_t> tag_static;
  std::vector<T> dd;                      // porosity control added to d
  double tag_center[NTAG][3]{}, tag_axis[NTAG][3]{};
  const Lattice* lat_ = &lattice(27);     // velocity set
  int q = 27;
  std::vector<T> h;                       // [q][N] post-collision state minus weights
  std::vector<T> utau;                    // wall state per cell
  std::vector<uint8_t> active;
  int64_t step = 0;
  std::vector<double> hist;               // HIST doubles per recorded step
  // per recorded step and tag 1..15: sum over the tag's cells of |dP| and of
  // |(x - x_c) x dP| (the scales of the force and torque sums)
  std::vector<double> hist_scale;
  // per recorded step and tag 1..15: the momentum-exchange force (3 doubles)
  // and the sum of the magnitudes of its link terms (its scale)
  std::vector<double> hist_me, hist_me_scale;
  bool with_me = false;
  WallStats wstats;
  int nthreads = 1;

  // objective: J += sum over steps in [t0,t1) of axial torque of obj_tag (0 = all tags), / (t1-t0)
  bool obj_on = false;
  int64_t obj_t0 = 0, obj_t1 = 0;
  int obj_tag = 0;
  T J = T(0.0);

  // per-step work arrays
  std::vector<double> g_phi, g_n, g_uB, g_dbase;
  std::vector<int> g_rot;
  std::vector<uint8_t> g_tag, g_wall;
  std::vector<T> f, mom, u, uwm, Swm, dP, d;
  std::vector<double> sigma;

  Sim(int nx_, int ny_, int nz_, int bcx, int nq = 27) : nx(nx_), ny(ny_), nz(nz_), bc_x(bcx) {
    N = (int64_t)nx * ny * nz;
    lat_ = &lattice(nq);
    q = lat_->q;
    h.assign((size_t)q * N, T(0.0));
    utau.assign(N, T(0.0));
    active.assign(N, 0);
    for (int t = 0; t < NTAG; ++t) {
      tag_center[t][0] = 0.5 * (nx - 1); tag_center[t][1] = 0.5 * (ny - 1); tag_center[t][2] = 0.5 * (nz - 1);
      tag_axis[t][0] = 1; tag_axis[t][1] = 0; tag_axis[t][2] = 0;
    }
  }

  int64_t idx(int x, int y, int z) const { return ((int64_t)z * ny + y) * nx + x; }
  static int wrap(int a, int n) { a %= n; return a < 0 ? a + n : a; }

  // Reference grid of rotor index k (copied); an empty phi removes it.
  void set_grid(int k, const double* phi, const int n[3], double h, const double o[3]) {
    RefGrid& G = grids[k];
    G.phi.clear();
    if (phi) {
      G.phi.assign(phi, phi + (size_t)n[0] * n[1] * n[2]);
      for (int a = 0; a < 3; ++a) { G.n[a] = n[a]; G.o[a] = o[a]; }
      G.h = h;
    }
    if ((size_t)k < rotors.size()) rotors[k].grid = G.phi.empty() ? nullptr : &G;
  }

  void set_rotors(const Rotor* r, int n) {
    rotors.assign(r, r + n);
    for (size_t k = 0; k < rotors.size() && k < grids.size(); ++k)
      rotors[k].grid = grids[k].phi.empty() ? nullptr : &grids[k];
    reset_rotation();
    frames.clear();
    for (auto& ro : rotors) {
      frames.push_back(rotor_frame(ro));
      const Frame& F = frames.back();
      for (int a = 0; a < 3; ++a) { tag_center[ro.tag][a] = ro.center[a]; tag_axis[ro.tag][a] = F.e[a]; }
    }
  }

  // The rotation state at the current step: prescribed angles, coupled
  // rotors starting from their prescribed angle and speed.
  void reset_rotation() {
    theta.assign(rotors.size(), 0.0);
    Omega.assign(rotors.size(), 0.0);
    for (size_t k = 0; k < rotors.size(); ++k) {
      theta[k] = rotors[k].phase0 + rotors[k].omega * double(step);
      Omega[k] = rotors[k].omega;
    }
  }
  double angle(size_t k, int64_t n) const {
    return rotors[k].inertia > 0 ? theta[k] : rotors[k].phase0 + rotors[k].omega * double(n);
  }
  double speed(size_t k) const { return rotors[k].inertia > 0 ? Omega[k] : rotors[k].omega; }

  // Two-way coupling of a rotor with inertia I (the structure update of the
  // FSI time loop, Sec. 3.2, for a rigid rotation about the fixed axis):
  // I dOmega/dt = e . T - T_gen with the torque T the fluid handed to the
  // rotor in step n, explicit: Omega_{n+1} = Omega_n + (e . T_n - T_gen) / I,
  // theta_{n+1} = theta_n + Omega_n.
  void evolve_rotors(const double* rec) {
    for (size_t k = 0; k < rotors.size(); ++k) {
      const Rotor& r = rotors[k];
      if (!(r.inertia > 0)) continue;
      const double* Tq = rec + 4 + 6 * (r.tag - 1);
      const double* e = frames[k].e;
      const double Tax = e[0] * Tq[0] + e[1] * Tq[1] + e[2] * Tq[2];
      const double Om1 = Omega[k] + (Tax - r.torque_gen) / r.inertia;
      theta[k] = theta[k] + Omega[k];
      Omega[k] = Om1;
    }
  }

  // -------------------------------------------------- 1. geometry
  void geometry(int64_t n) {
    g_phi.assign(N, -1e300); g_n.assign(3 * N, 0.0); g_uB.assign(3 * N, 0.0); g_dbase.assign(N, 0.0);
    g_rot.assign(N, -1); g_tag.assign(N, 0); g_wall.assign(N, 0);
    d.assign(N, T(0.0));
    const double eps = p.eps_h;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int64_t c = idx(x, y, z);
          const double X[3] = {double(x), double(y), double(z)};
          double best = -1e300, bgrad[3] = {0, 0, 0};
          int brot = -1;
          for (size_t k = 0; k < rotors.size(); ++k) {
            double gr[3];
            double ph = rotor_phi_at(rotors[k], frames[k], X, angle(k, n), gr);
            if (ph > best) { best = ph; brot = (int)k; for (int a = 0; a < 3; ++a) bgrad[a] = gr[a]; }
          }
          double drot = brot >= 0 ? transition_s(best, eps, p.transition) : 0.0;
          double ds = d_static.empty() ? 0.0 : d_static[c];
          g_dbase[c] = ds > drot ? ds : drot;
          g_phi[c] = best;
          if (drot > 0.0) {
            const Rotor& R = rotors[brot];
            const Frame& F = frames[brot];
            g_rot[c] = brot;
            g_tag[c] = (uint8_t)R.tag;
            double rel[3] = {X[0] - R.center[0], X[1] - R.center[1], X[2] - R.center[2]};
            // uB = Omega e x (x - x_c)
            const double om = speed(brot);
            g_uB[3 * c + 0] = om * (F.e[1] * rel[2] - F.e[2] * rel[1]);
            g_uB[3 * c + 1] = om * (F.e[2] * rel[0] - F.e[0] * rel[2]);
            g_uB[3 * c + 2] = om * (F.e[0] * rel[1] - F.e[1] * rel[0]);
            double gn = std::sqrt(bgrad[0] * bgrad[0] + bgrad[1] * bgrad[1] + bgrad[2] * bgrad[2]);
            if (gn > 0) for (int a = 0; a < 3; ++a) g_n[3 * c + a] = -bgrad[a] / gn;
            if (p.wall_model && best > -0.5 * eps && best < 0.0 && gn > 0) g_wall[c] = 1;
          } else {
            g_tag[c] = tag_static.empty() ? 0 : tag_static[c];
            if (!uB_static.empty())
              for (int a = 0; a < 3; ++a) g_uB[3 * c + a] = uB_static[(size_t)a * N + c];
          }
          d[c] = T(g_dbase[c]) + (dd.empty() ? T(0.0) : dd[c]);
        }
  }

  // -------------------------------------------------- 2. pull with boundaries
  void inflow_velocity(int64_t n, int y, int z, double uin[3]) const {
    double mag = std::sqrt(p.u_in[0] * p.u_in[0] + p.u_in[1] * p.u_in[1] + p.u_in[2] * p.u_in[2]);
    for (int a = 0; a < 3; ++a) {
      uin[a] = p.u_in[a];
      if (p.turb_I != 0.0) uin[a] += p.turb_I * mag * inflow_gaussian(p.seed, n, y, z, a, ny, nz);
    }
  }

  void pull(int64_t n) {
    const Lattice& L = *lat_;
    f.assign((size_t)q * N, T(0.0));
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int64_t c = idx(x, y, z);
          for (int i = 0; i < q; ++i) {
            int xs = x - L.c[i][0];
            int ys = wrap(y - L.c[i][1], ny), zs = wrap(z - L.c[i][2], nz);
            if (bc_x == 0) {
              xs = wrap(xs, nx);
            } else if (xs < 0) {
              double uin[3];
              inflow_velocity(n, ys, zs, uin);
              T ui[3] = {T(uin[0]), T(uin[1]), T(uin[2])};
              T feq[Q];
              equilibrium(T(1.0), ui, feq, L);
              f[(size_t)i * N + c] = feq[i];
              continue;
            } else if (xs > nx - 1) {
              xs = nx - 1;
            }
            f[(size_t)i * N + c] = L.w[i] + h[(size_t)i * N + idx(xs, ys, zs)];
          }
        }
  }

  // -------------------------------------------------- 3. moments
  void moments() {
    mom.assign((size_t)10 * N, T(0.0));
    u.assign((size_t)3 * N, T(0.0));
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t c = 0; c < N; ++c) {
      T fc[Q], m[10];
      for (int i = 0; i < q; ++i) fc[i] = f[(size_t)i * N + c];
      moments_of(fc, m, *lat_);
      for (int k = 0; k < 10; ++k) mom[(size_t)k * N + c] = m[k];
      for (int a = 0; a < 3; ++a) u[(size_t)a * N + c] = m[1 + a] / m[0];
    }
  }

  // trilinear interpolation of the fluid velocity at a point
  void sample_u(const double X[3], T us[3]) const {
    for (int a = 0; a < 3; ++a) us[a] = trilinear(&u[(size_t)a * N], nx, ny, nz, bc_x, X);
  }

  // -------------------------------------------------- 4. wall model
  void wall_model() {
    uwm.assign((size_t)3 * N, T(0.0));
    Swm.assign((size_t)6 * N, T(0.0));
    sigma.assign(N, 1.0);
    const double nu = CS2 * (p.tau0 - 0.5);
    std::vector<T> ut_new(N, T(0.0));
    std::vector<uint8_t> act_new(N, 0);
    int64_t iters = 0, calls = 0, halv = 0, capd = 0, near = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(+ : iters, calls, halv, capd, near)
    for (int64_t c = 0; c < N; ++c) {
      if (!g_wall[c]) continue;
      const int x = int(c % nx), y = int((c / nx) % ny), z = int(c / ((int64_t)nx * ny));
      const Rotor& R = rotors[g_rot[c]];
      const Frame& F = frames[g_rot[c]];
      const double* nn = &g_n[3 * c];
      const double y1 = -g_phi[c];
      double xw[3], xs[3];
      const double X[3] = {double(x), double(y), double(z)};
      for (int a = 0; a < 3; ++a) { xw[a] = X[a] - y1 * nn[a]; xs[a] = xw[a] + p.y_s * nn[a]; }
      double rel[3] = {xw[0] - R.center[0], xw[1] - R.center[1], xw[2] - R.center[2]};
      const double om = speed(g_rot[c]);
      double uw[3] = {om * (F.e[1] * rel[2] - F.e[2] * rel[1]),
                      om * (F.e[2] * rel[0] - F.e[0] * rel[2]),
                      om * (F.e[0] * rel[1] - F.e[1] * rel[0])};
      T us[3];
      sample_u(xs, us);
      WallOut<T> o = wall_model_cell(us, uw, nn, y1, utau[c], active[c] != 0, p, nu);
      halv += o.halvings;
      capd += o.capped;
      if (o.slip >= 0.5e-6 && o.slip <= 2e-6) near += 1;
      if (o.active) {
        for (int a = 0; a < 3; ++a) uwm[(size_t)a * N + c] = o.uwm[a];
        for (int k = 0; k < 6; ++k) Swm[(size_t)k * N + c] = o.S[k];
        sigma[c] = 0.0;
        ut_new[c] = o.utau;
        act_new[c] = 1;
        iters += o.iters_tau;
        calls += 1;
      }
    }
    wstats.newton_iters += iters;
    wstats.calls += calls;
    wstats.halvings += halv;
    wstats.capped += capd;
    wstats.near_threshold += near;
    utau.swap(ut_new);
    active.swap(act_new);
  }

  // -------------------------------------------------- 5. collision + 6. new state
  void collide_and_record() {
    const Lattice& L = *lat_;
    dP.assign((size_t)3 * N, T(0.0));
    std::vector<T> rho(N);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t c = 0; c < N; ++c) {
      T m[10], fs[Q], dp[3], uw3[3], S6[6];
      for (int k = 0; k < 10; ++k) m[k] = mom[(size_t)k * N + c];
      for (int a = 0; a < 3; ++a) uw3[a] = uwm[(size_t)a * N + c];
      for (int k = 0; k < 6; ++k) S6[k] = Swm[(size_t)k * N + c];
      collide_cell(m, d[c], &g_uB[3 * c], uw3, S6, sigma[c], p.tau0, p.cs_smag, fs, dp, L);
      for (int i = 0; i < q; ++i) h[(size_t)i * N + c] = fs[i] - L.w[i];
      for (int a = 0; a < 3; ++a) dP[(size_t)a * N + c] = dp[a];
      rho[c] = m[0];
    }
    // fixed (z, y, x) order FP64 sums
    std::vector<double> rec(HIST, 0.0), scl(2 * 15, 0.0);
    T Tax = T(0.0);
    T mass = T(0.0);
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int64_t c = idx(x, y, z);
          mass = mass + rho[c];
          const int t = g_tag[c];
          if (t == 0) continue;
          const T dp[3] = {dP[c], dP[(size_t)N + c], dP[(size_t)2 * N + c]};
          const double r[3] = {x - tag_center[t][0], y - tag_center[t][1], z - tag_center[t][2]};
          const T tq[3] = {r[1] * dp[2] - r[2] * dp[1], r[2] * dp[0] - r[0] * dp[2], r[0] * dp[1] - r[1] * dp[0]};
          double* o = &rec[1 + 6 * (t - 1)];
          for (int a = 0; a < 3; ++a) { o[a] += re(dp[a]); o[3 + a] += re(tq[a]); }
          scl[2 * (t - 1)] += std::sqrt(re(dp[0]) * re(dp[0]) + re(dp[1]) * re(dp[1]) + re(dp[2]) * re(dp[2]));
          scl[2 * (t - 1) + 1] += std::sqrt(re(tq[0]) * re(tq[0]) + re(tq[1]) * re(tq[1]) + re(tq[2]) * re(tq[2]));
          if (obj_on && (obj_tag == 0 || obj_tag == t))
            Tax = Tax + tag_axis[t][0] * tq[0] + tag_axis[t][1] * tq[1] + tag_axis[t][2] * tq[2];
        }
    rec[0] = re(mass);
    hist.insert(hist.end(), rec.begin(), rec.end());
    evolve_rotors(rec.data());
    hist_scale.insert(hist_scale.end(), scl.begin(), scl.end());
    if (with_me) momentum_exchange();
    if (obj_on && step >= obj_t0 && step < obj_t1) J = J + Tax / double(obj_t1 - obj_t0);
  }

  // Momentum-exchange force on each tagged element (Sec. 2.2.2, the
  // momentum-exchange sum after Wen et al. 2014, read per link): the links
  // join a cell x of tag 0 to a neighbour x_b = x + c_i of tag T != 0; the
  // link carries f*_i(x) into the element and f*_ibar(x_b) out of it, and
  // hands the element (c_i - u_s) f*_i(x) + (c_i + u_s) f*_ibar(x_b), u_s
  // the solid velocity of x_b (Galilean-invariant form).  Post-collision
  // populations of this step, tags of this step; x faces of an
  // inflow/outflow lattice have no links beyond them.  A tag-0 cell next to
  // several elements gives its links to the element of its first such
  // neighbour in velocity order.
  void momentum_exchange() {
    const Lattice& L = *lat_;
    std::vector<double> me(15 * 3, 0.0), mes(15, 0.0);
    auto neighbour = [&](int x, int y, int z, int i, int64_t& cn) {
      int xn = x + L.c[i][0];
      const int yn = wrap(y + L.c[i][1], ny), zn = wrap(z + L.c[i][2], nz);
      if (bc_x == 0) xn = wrap(xn, nx);
      else if (xn < 0 || xn > nx - 1) return false;
      cn = idx(xn, yn, zn);
      return true;
    };
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int64_t c = idx(x, y, z);
          const int t = g_tag[c];
          int tme = t;
          double acc[3] = {0.0, 0.0, 0.0}, mag = 0.0;
          for (int i = 0; i < q; ++i) {
            if (L.c[i][0] == 0 && L.c[i][1] == 0 && L.c[i][2] == 0) continue;
            int64_t cn;
            if (!neighbour(x, y, z, i, cn)) continue;
            const int tn = g_tag[cn];
            const double fs = re(h[(size_t)i * N + c]) + L.w[i];
            double term[3];
            if (t != 0 && tn == 0) {
              // outflow of x across a link of its element: (u_s(x) - c_i) f*_i(x)
              for (int a = 0; a < 3; ++a) term[a] = (g_uB[3 * c + a] - L.c[i][a]) * fs;
            } else if (t == 0 && tn != 0) {
              if (tme == 0) tme = tn;
              if (tn != tme) continue;
              // inflow into the element: (c_i - u_s(x_b)) f*_i(x)
              for (int a = 0; a < 3; ++a) term[a] = (L.c[i][a] - g_uB[3 * cn + a]) * fs;
            } else {
              continue;
            }
            for (int a = 0; a < 3; ++a) acc[a] += term[a];
            mag += std::sqrt(term[0] * term[0] + term[1] * term[1] + term[2] * term[2]);
          }
          if (tme != 0) {
            for (int a = 0; a < 3; ++a) me[3 * (tme - 1) + a] += acc[a];
            mes[tme - 1] += mag;
          }
        }
    hist_me.insert(hist_me.end(), me.begin(), me.end());
    hist_me_scale.insert(hist_me_scale.end(), mes.begin(), mes.end());
  }

  // Hybrid non-equilibrium off the wall (Sec. 2.2: f~(1) = sigma f(1) -
  // (1 - sigma) f(1,FD), f(1,FD) from a non-local finite-difference strain):
  // in the cells of an element (tag != 0) that are not active wall cells,
  // sigma = 1 - fd_share and S = S^FD, the central difference of the
  // pre-collision velocity u = j / rho, S_ab = (d_a u_b + d_b u_a) / 2,
  // d_b u_a = (u_a(x + e_b) - u_a(x - e_b)) / 2, y and z periodic, x periodic
  // or clamped to the first and last plane.
  void fd_strain() {
    const double sig = 1.0 - p.fd_share;
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int64_t c = idx(x, y, z);
          if (g_tag[c] == 0 || sigma[c] != 1.0) continue;
          int64_t nb[3][2];
          const int xm = bc_x == 0 ? wrap(x - 1, nx) : (x > 0 ? x - 1 : 0);
          const int xp = bc_x == 0 ? wrap(x + 1, nx) : (x < nx - 1 ? x + 1 : nx - 1);
          nb[0][0] = idx(xm, y, z);
          nb[0][1] = idx(xp, y, z);
          nb[1][0] = idx(x, wrap(y - 1, ny), z);
          nb[1][1] = idx(x, wrap(y + 1, ny), z);
          nb[2][0] = idx(x, y, wrap(z - 1, nz));
          nb[2][1] = idx(x, y, wrap(z + 1, nz));
          T du[3][3];  // du[a][b] = d_b u_a
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
              du[a][b] = 0.5 * (u[(size_t)a * N + nb[b][1]] - u[(size_t)a * N + nb[b][0]]);
          for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) {
              int k;
              sym_index(a, b, k);
              Swm[(size_t)k * N + c] = 0.5 * (du[a][b] + du[b][a]);
            }
          sigma[c] = sig;
        }
  }

  void do_step() {
    geometry(step);
    pull(step);
    moments();
    if (p.wall_model) wall_model();
    else { uwm.assign((size_t)3 * N, T(0.0)); Swm.assign((size_t)6 * N, T(0.0)); sigma.assign(N, 1.0); }
    if (p.fd_share > 0.0) fd_strain();
    collide_and_record();
    ++step;
  }

  void init_equilibrium(const double* rho, const double* uu) {
    const Lattice& L = *lat_;
    for (int64_t c = 0; c < N; ++c) {
      T r = T(rho ? rho[c] : 1.0);
      T u3[3];
      for (int a = 0; a < 3; ++a) u3[a] = T(uu ? uu[(size_t)a * N + c] : 0.0);
      T feq[Q];
      equilibrium(r, u3, feq, L);
      for (int i = 0; i < q; ++i) h[(size_t)i * N + c] = feq[i] - L.w[i];
    }
    std::fill(utau.begin(), utau.end(), T(0.0));
    std::fill(active.begin(), active.end(), 0);
    step = 0;
    reset_rotation();
    hist.clear();
    hist_scale.clear();
    hist_me.clear();
    hist_me_scale.clear();
  }
};

}  // namespace oracle
