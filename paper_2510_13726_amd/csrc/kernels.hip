// HIP kernels of libhlbm for gfx950 (CDNA4, wave64).
//
//  k_wall_geometry  wall model of a step (probe interpolation, Newton) in the
//                   first workgroups, rotor porosity embedding and inflow
//                   plane of the next step in the others; the adjoint
//                   instantiation adds the adjoint wall step
//  k_geometry       the geometry alone (first step of a run)
//  k_sweep          fused pull-stream + moments + HLBM collision + store, with
//                   per-tag force/torque partials on FSI workgroups
//  k_reduce_l1/l2   deterministic reduction of the partials into the history
//  k_adj_sweep      reverse sweep of the discrete adjoint
// plus initialisation, conversion and bookkeeping kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <utility>

#include "hlbm_internal.h"
#include "launch.h"
#include "lbm_cell.h"

namespace hlbm {

// ================================================================ helpers
__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// f(integral_constant<int, 0>) ... f(integral_constant<int, N - 1>): loop
// bodies whose velocity index is a compile-time constant.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Pre-collision deviations h_i = f_i - w_i of cell (x, y, z):
// f_i(x) = f*_i(x - c_i) with periodic y, z; in x periodic, or the
// equilibrium inflow ghost plane at x = -1 (precomputed for the step in
// `ghost`, [9][nz][ny] for the velocities with c_x = +1) and the
// zero-gradient copy at x = nx.
template <class ST, class CT, bool kPeriodicX, int Q = 27>
__device__ __forceinline__ void pull_cell(const ST* __restrict__ src, const Geometry& g, int x, int y, int z,
                                          const CT* __restrict__ ghost, CT h[Q]) {
  const int zp = z + 1 == g.nz ? 0 : z + 1, zm = z == 0 ? g.nz - 1 : z - 1;
  const int yp = y + 1 == g.ny ? 0 : y + 1, ym = y == 0 ? g.ny - 1 : y - 1;
  int xp, xm;
  if (kPeriodicX) {
    xp = x + 1 == g.nx ? 0 : x + 1;
    xm = x == 0 ? g.nx - 1 : x - 1;
  } else {
    xp = x + 1 == g.nx ? x : x + 1;  // outflow: copy of the last plane
    xm = x == 0 ? 0 : x - 1;         // inflow plane is replaced below
  }
  // source of velocity c is x - c: c = -1 -> +1 neighbour, c = +1 -> -1 neighbour
  const int64_t rb[3][3] = {{(int64_t(zp) * g.ny + yp) * g.row, (int64_t(zp) * g.ny + y) * g.row, (int64_t(zp) * g.ny + ym) * g.row},
                            {(int64_t(z) * g.ny + yp) * g.row, (int64_t(z) * g.ny + y) * g.row, (int64_t(z) * g.ny + ym) * g.row},
                            {(int64_t(zm) * g.ny + yp) * g.row, (int64_t(zm) * g.ny + y) * g.row, (int64_t(zm) * g.ny + ym) * g.row}};
  const uint32_t ox[3] = {pop_x<Q>(xp), pop_x<Q>(x), pop_x<Q>(xm)};
  static_for<Q>([&](auto I) {
    constexpr int i = I;
    const ST* p = src + rb[czq<Q>(i) + 1][cyq<Q>(i) + 1];
    const uint32_t o = (ox[cxq<Q>(i) + 1] + uint32_t(i * kTileX)) * uint32_t(sizeof(ST));
    h[i] = CT(wq<Q>(i)) * Store<ST>::template load<CT>(at_bytes(p, o));
  });
  if (!kPeriodicX && x == 0) {
    // the inflow plane holds the nine c_x = +1 directions by m = 3 (c_y + 1) + (c_z + 1)
    const uint32_t pz[3] = {uint32_t(zp) * g.ny, uint32_t(z) * g.ny, uint32_t(zm) * g.ny};
    const uint32_t py[3] = {uint32_t(yp), uint32_t(y), uint32_t(ym)};
    const int64_t plane = int64_t(g.ny) * g.nz;
    static_for<9>([&](auto M) {
      constexpr int m = M;
      constexpr int k = kq<Q>(1, m / 3 - 1, m % 3 - 1);
      if constexpr (k >= 0) h[k] = ghost[m * plane + pz[m % 3] + py[m / 3]];
    });
  }
}

// Byte pointers into global memory (address space 1), so that a pointer
// kept in scalar registers through an empty asm stays a global pointer.
typedef __attribute__((address_space(1))) const char* gconst_bytes;
typedef __attribute__((address_space(1))) char* gbytes;

// pull_cell for a wave whose 64 lanes share y and z (uniform values): the
// y/z part of every source address is a scalar, the per-lane part is one of
// three x offsets, so each load is a scalar base plus a 32-bit lane offset.
template <class ST, class CT, bool kPeriodicX, int Q = 27>
__device__ __forceinline__ void pull_row(const ST* __restrict__ src, const Geometry& g, int x, int y, int z,
                                         const CT* __restrict__ ghost, CT h[Q]) {
  const int zp = z + 1 == g.nz ? 0 : z + 1, zm = z == 0 ? g.nz - 1 : z - 1;
  const int yp = y + 1 == g.ny ? 0 : y + 1, ym = y == 0 ? g.ny - 1 : y - 1;
  int xp, xm;
  if (kPeriodicX) {
    xp = x + 1 == g.nx ? 0 : x + 1;
    xm = x == 0 ? g.nx - 1 : x - 1;
  } else {
    xp = x + 1 == g.nx ? x : x + 1;  // outflow: copy of the last plane
    xm = x == 0 ? 0 : x - 1;         // inflow plane is replaced below
  }
  // The velocities with the same (c_y, c_z) read the same source row
  // (y - c_y, z - c_z), each from the run of its own index.  Each of the
  // nine rows gets one wave-uniform base (its start); a lane adds one of
  // three 32-bit offsets, its source cell in the row plus the first run of
  // the velocities with its c_x, and the load the velocity's rank among those
  // runs as its immediate offset.
  constexpr uint32_t es = sizeof(ST), run = kTileX * es;
  const uint64_t rs = uint64_t(g.row) * es;
  // index [c + 1] of each array: source z - c_z, y - c_y, x - c_x
  const uint64_t zb[3] = {uint64_t(zp) * g.ny * rs, uint64_t(z) * g.ny * rs, uint64_t(zm) * g.ny * rs};
  const uint64_t yb[3] = {uint64_t(yp) * rs, uint64_t(y) * rs, uint64_t(ym) * rs};
  const uint32_t ox[3] = {pop_x<Q>(xp) * es + xgroup_of<Q>(0) * run, pop_x<Q>(x) * es + xgroup_of<Q>(1) * run,
                          pop_x<Q>(xm) * es + xgroup_of<Q>(2) * run};
  gconst_bytes p = (gconst_bytes)src;
  static_for<9>([&](auto R) {
    constexpr int b = R / 3, a = R % 3;  // c_y + 1, c_z + 1
    gconst_bytes q = p + (zb[a] + yb[b]);
    // kept in scalar registers: each load is this base plus a lane offset
    asm("" : "+s"(q));
    static_for<3>([&](auto J) {
      constexpr int j = J;
      constexpr int k = kq<Q>(j - 1, b - 1, a - 1);
      if constexpr (k >= 0) {
        constexpr uint32_t rank = uint32_t(k - xgroup_of<Q>(j));
        h[k] = CT(wq<Q>(k)) * Store<ST>::template load<CT>((const ST*)(q + ox[j] + rank * run));
      }
    });
  });
  if (!kPeriodicX && x == 0) {
    const int64_t plane = int64_t(g.ny) * g.nz;
    const int64_t pz[3] = {int64_t(zp) * g.ny, int64_t(z) * g.ny, int64_t(zm) * g.ny};
    const int py[3] = {yp, y, ym};
    static_for<9>([&](auto M) {
      constexpr int m = M;
      constexpr int k = kq<Q>(1, m / 3 - 1, m % 3 - 1);
      if constexpr (k >= 0) h[k] = ghost[m * plane + pz[m % 3] + py[m / 3]];
    });
  }
}

// Position (z, tile row, tile column) of sweep tile blk, and its index in
// lattice order ((z nty + ty) ntx + tx, the index of its FSI slot and mass
// partial).  Bands of `band` tile rows along y are swept one after the
// other, each z plane by plane, so that the three z planes that read a
// source row are swept close together in time.  Tile ids and counts fit
// 32 bits (fewer than 2^31 cells, 256 per tile).
struct TileId {
  int z, ty, tx;
  uint32_t canon;
};
__device__ __forceinline__ TileId tile_id(const Geometry& g, uint32_t blk) {
  const uint32_t ntx = uint32_t(g.ntx);
  uint32_t ty0, rem, z, ri;
  if (blk < g.full_tiles) {
    const uint32_t b = udiv(blk, g.by_band);
    rem = blk - b * (g.band * ntx * uint32_t(g.nz));
    z = udiv(rem, g.by_bandrow);
    rem -= z * (g.band * ntx);
    ty0 = b * g.band;
  } else {
    // the last band, of nty - (full bands) band rows
    const uint32_t rows = uint32_t(g.nty) - (g.full_tiles / (ntx * uint32_t(g.nz)));
    rem = blk - g.full_tiles;
    z = udiv(rem, g.by_tailrow);
    rem -= z * (rows * ntx);
    ty0 = uint32_t(g.nty) - rows;
  }
  ri = udiv(rem, g.by_ntx);
  const uint32_t ty = ty0 + ri, tx = rem - ri * ntx;
  return TileId{int(z), int(ty), int(tx), (z * uint32_t(g.nty) + ty) * ntx + tx};
}

// Inflow ghost plane of step n: h_i = f^eq_i(1, u_in(n, y, z)) - w_i for the
// nine velocities with c_x = +1, u_in = U + I |U| xi with seeded normals xi.
// Cell k = z ny + y of the plane; ghost64 (nullable) gets the FP64 values.
template <class CT, int Q = 27>
__device__ __forceinline__ void inflow_plane_cell(const Geometry& g, const Model& m, int64_t n, int64_t k,
                                                  CT* __restrict__ ghost, double* __restrict__ ghost64) {
  const int64_t plane = int64_t(g.ny) * g.nz;
  const int z = int(k / g.ny), y = int(k - int64_t(z) * g.ny);
  double u[3] = {m.u_in[0], m.u_in[1], m.u_in[2]};
  if (m.turb_amp != 0.0)
    for (int a = 0; a < 3; ++a) u[a] += m.turb_amp * inflow_normal(m.seed, n, y, z, a, g.ny, g.nz);
  // the c_x = +1 directions, by m = 3 (c_y + 1) + (c_z + 1)
  CT ge[Q];
  equilibrium_dev_unit<CT, Q>(CT(u[0]), CT(u[1]), CT(u[2]), ge);
  static_for<9>([&](auto M) {
    constexpr int kk = kq<Q>(1, M / 3 - 1, M % 3 - 1);
    if constexpr (kk >= 0) ghost[M * plane + k] = CT(wq<Q>(kk)) * ge[kk];
  });
  if (ghost64) {
    double gd[Q];
    equilibrium_dev_unit<double, Q>(u[0], u[1], u[2], gd);
    static_for<9>([&](auto M) {
      constexpr int kk = kq<Q>(1, M / 3 - 1, M % 3 - 1);
      if constexpr (kk >= 0) ghost64[M * plane + k] = wq<Q>(kk) * gd[kk];
    });
  }
}

template <class CT, int Q>
__global__ __launch_bounds__(256) void k_prologue(Geometry g, Model m, int64_t n, CT* __restrict__ ghost,
                                                  double* __restrict__ ghost64) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g.bc_x == 0 || k >= int64_t(g.ny) * g.nz) return;
  inflow_plane_cell<CT, Q>(g, m, n, k, ghost, ghost64);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ================================================================ geometry
// Signed distance (positive inside) of a rotor at step n: hub sphere united
// with flat-plate blades (box in blade coordinates r, chord s, thickness h;
// pitch beta(r) linear from root to tip).  The value pass returns the
// distance and the piece attaining it (-1 hub, b blade b); the gradient pass
// differentiates that piece (the same arithmetic as the value pass).
struct RotorPhi {
  double phi;
  int piece;
  double sb, cb;  // sin and cos of the winning blade's pitch at the point
};

// Blade b in its own frame: radial r, tangential q, axial a of the point;
// box coordinates p and the pitch derivative dbeta.
struct BladeFrame {
  double er[3], ep[3], rr, qq, ax, p[3], sb, cb, dbeta;
};
__device__ __forceinline__ void blade_frame(const RotorDev& r, double ct, double st, const double rel[3], double ax,
                                            BladeFrame& f) {
  for (int a = 0; a < 3; ++a) {
    f.er[a] = ct * r.e1[a] + st * r.e2[a];
    f.ep[a] = -st * r.e1[a] + ct * r.e2[a];
  }
  f.rr = rel[0] * f.er[0] + rel[1] * f.er[1] + rel[2] * f.er[2];
  f.qq = rel[0] * f.ep[0] + rel[1] * f.ep[1] + rel[2] * f.ep[2];
  f.ax = ax;
}
// with_pitch: compute sin and cos of the pitch, else take f.sb, f.cb as given
__device__ __forceinline__ void blade_box(const RotorDev& r, BladeFrame& f, bool with_pitch = true) {
  const double span = r.R - r.r_hub;
  double frac = (f.rr - r.r_hub) / span;
  f.dbeta = 0.0;
  if (frac <= 0.0) frac = 0.0;
  else if (frac >= 1.0) frac = 1.0;
  else f.dbeta = (r.tw_tip - r.tw_root) / span;
  if (with_pitch) {
    const double beta = r.tw_root + (r.tw_tip - r.tw_root) * frac;
    sincos(beta, &f.sb, &f.cb);
  }
  f.p[0] = f.rr - 0.5 * (r.R + r.r_hub);
  f.p[1] = -f.cb * f.qq + f.sb * f.ax;
  f.p[2] = f.cb * f.ax + f.sb * f.qq;
}

// Reference-grid body (Sec. 3.1: the element voxelized once on its own
// grid, embedded at its current position and orientation every step).  The
// body frame turns with blade 0: e_r = cos(theta) e1 + sin(theta) e2, e_t =
// e x e_r, and the axis e.  A point's body coordinates, divided into grid
// units, give its cell (the last cell for a point on the far face) and the
// fractions inside it; a point off the grid is not in the body.
struct GridCell {
  const double* v;  // sample of the cell's lowest corner
  double f[3];
  double ax[3][3];  // e_r, e_t, e
};
__device__ __forceinline__ bool grid_cell(const RotorDev& r, double ct, double st, const double rel[3], GridCell& s) {
  for (int a = 0; a < 3; ++a) {
    s.ax[0][a] = ct * r.e1[a] + st * r.e2[a];
    s.ax[1][a] = -st * r.e1[a] + ct * r.e2[a];
    s.ax[2][a] = r.e[a];
  }
  int i[3];
  for (int k = 0; k < 3; ++k) {
    const double p = rel[0] * s.ax[k][0] + rel[1] * s.ax[k][1] + rel[2] * s.ax[k][2];
    const double u = (p - r.go[k]) / r.gh;
    if (!(u >= 0.0 && u <= double(r.gn[k] - 1))) return false;
    const int c = min(int(floor(u)), r.gn[k] - 2);
    i[k] = c;
    s.f[k] = u - double(c);
  }
  s.v = r.grid + (int64_t(i[2]) * r.gn[1] + i[1]) * r.gn[0] + i[0];
  return true;
}
// The eight corner samples of a cell, v[z][y][x].
__device__ __forceinline__ void grid_corners(const RotorDev& r, const GridCell& s, double v[2][2][2]) {
  const int64_t sy = r.gn[0], sz = int64_t(r.gn[0]) * r.gn[1];
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy) {
      v[dz][dy][0] = s.v[dz * sz + dy * sy];
      v[dz][dy][1] = s.v[dz * sz + dy * sy + 1];
    }
}
// Trilinear interpolant: along the first axis, then the second, the third.
__device__ __forceinline__ double grid_value(const RotorDev& r, const GridCell& s) {
  double v[2][2][2];
  grid_corners(r, s, v);
  double w[2];
  for (int dz = 0; dz < 2; ++dz) {
    const double a0 = v[dz][0][0] + s.f[0] * (v[dz][0][1] - v[dz][0][0]);
    const double a1 = v[dz][1][0] + s.f[0] * (v[dz][1][1] - v[dz][1][0]);
    w[dz] = a0 + s.f[1] * (a1 - a0);
  }
  return w[0] + s.f[2] * (w[1] - w[0]);
}
// Gradient of that interpolant in the lattice frame.
__device__ __forceinline__ void grid_gradient(const RotorDev& r, const GridCell& s, double grad[3]) {
  double v[2][2][2];
  grid_corners(r, s, v);
  const double fx = s.f[0], fy = s.f[1], fz = s.f[2];
  double d[3] = {0.0, 0.0, 0.0};  // derivatives with respect to the three fractions
  for (int dz = 0; dz < 2; ++dz) {
    const double wz = dz ? fz : 1.0 - fz, sz = dz ? 1.0 : -1.0;
    for (int dy = 0; dy < 2; ++dy) {
      const double wy = dy ? fy : 1.0 - fy, sy = dy ? 1.0 : -1.0;
      const double lo = v[dz][dy][0], hi = v[dz][dy][1];
      const double along = lo + fx * (hi - lo);
      d[0] += wy * wz * (hi - lo);
      d[1] += sy * wz * along;
      d[2] += wy * sz * along;
    }
  }
  const double ih = 1.0 / r.gh;
  for (int a = 0; a < 3; ++a) grad[a] = (d[0] * s.ax[0][a] + d[1] * s.ax[1][a] + d[2] * s.ax[2][a]) * ih;
}

__device__ __forceinline__ RotorPhi rotor_phi(const RotorDev& r, const double* ctab, const double* stab, double x,
                                              double y, double z, double cut) {
  RotorPhi o;
  const double rel[3] = {x - r.c[0], y - r.c[1], z - r.c[2]};
  if (r.grid) {
    GridCell s;
    o.sb = 0.0;
    o.cb = 1.0;
    if (grid_cell(r, ctab[0], stab[0], rel, s)) {
      o.phi = grid_value(r, s);
      o.piece = 0;
    } else {
      o.phi = -1e300;
      o.piece = -2;
    }
    return o;
  }
  const double dist = sqrt(rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2]);
  o.phi = r.r_hub - dist;
  o.piece = -1;
  o.sb = 0.0;
  o.cb = 1.0;
  const double ax = rel[0] * r.e[0] + rel[1] * r.e[1] + rel[2] * r.e[2];
  const double span = r.R - r.r_hub;
  const double half[3] = {0.5 * span, 0.5 * r.chord, 0.5 * r.thick};
  // the blade lies within r_hub <= r <= R and q^2 + a^2 <= (c/2)^2 + (t/2)^2:
  // a point farther than `cut` from that slab cannot reach phi > -cut
  const double hc = 0.5 * sqrt(r.chord * r.chord + r.thick * r.thick) + cut;
  for (int b = 0; b < r.nb; ++b) {
    BladeFrame f;
    blade_frame(r, ctab[b], stab[b], rel, ax, f);
    if (f.rr < r.r_hub - cut || f.rr > r.R + cut || f.qq * f.qq + ax * ax > hc * hc) continue;
    blade_box(r, f);
    double q[3], qn2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      q[k] = fabs(f.p[k]) - half[k];
      const double qp = q[k] > 0 ? q[k] : 0.0;
      qn2 += qp * qp;
    }
    // largest component (first on ties), selected without indexing
    double qm = q[0];
    if (q[1] > qm) qm = q[1];
    if (q[2] > qm) qm = q[2];
    const double phi = -(sqrt(qn2) + (qm < 0 ? qm : 0.0));
    if (phi > o.phi) {
      o.phi = phi;
      o.piece = b;
      o.sb = f.sb;
      o.cb = f.cb;
    }
  }
  return o;
}

// Gradient of the rotor distance at (x, y, z) for the piece found by rotor_phi
// (with the pitch sine and cosine that pass computed there).
__device__ __forceinline__ void rotor_grad(const RotorDev& r, const double* ctab, const double* stab, double x,
                                           double y, double z, const RotorPhi& w, double grad[3]) {
  const int piece = w.piece;
  const double rel[3] = {x - r.c[0], y - r.c[1], z - r.c[2]};
  if (r.grid) {
    GridCell s;
    if (grid_cell(r, ctab[0], stab[0], rel, s)) grid_gradient(r, s, grad);
    else grad[0] = grad[1] = grad[2] = 0.0;
    return;
  }
  const double dist = sqrt(rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2]);
  if (piece < 0) {
    for (int a = 0; a < 3; ++a) grad[a] = dist > 0 ? -rel[a] / dist : 0.0;
    return;
  }
  const double ax = rel[0] * r.e[0] + rel[1] * r.e[1] + rel[2] * r.e[2];
  const double span = r.R - r.r_hub;
  const double half[3] = {0.5 * span, 0.5 * r.chord, 0.5 * r.thick};
  BladeFrame f;
  blade_frame(r, ctab[piece], stab[piece], rel, ax, f);
  f.sb = w.sb;
  f.cb = w.cb;
  blade_box(r, f, false);
  double q[3], qp[3], qn2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    q[k] = fabs(f.p[k]) - half[k];
    qp[k] = q[k] > 0 ? q[k] : 0.0;
    qn2 += qp[k] * qp[k];
  }
  int km = 0;
  if (q[1] > q[0]) km = 1;
  if (q[2] > (km == 1 ? q[1] : q[0])) km = 2;
  double gp[3] = {0.0, 0.0, 0.0};
  if (qn2 > 0) {
    const double qn = sqrt(qn2);
    for (int k = 0; k < 3; ++k) gp[k] = (f.p[k] >= 0 ? 1.0 : -1.0) * qp[k] / qn;
  } else {
    for (int k = 0; k < 3; ++k) gp[k] = k == km ? (f.p[k] >= 0 ? 1.0 : -1.0) : 0.0;
  }
  const double gs = f.dbeta * (f.sb * f.qq + f.cb * ax);
  const double gh = f.dbeta * (-f.sb * ax + f.cb * f.qq);
  for (int a = 0; a < 3; ++a) {
    const double ds = -f.cb * f.ep[a] + f.sb * r.e[a] + gs * f.er[a];
    const double dh = f.cb * r.e[a] + f.sb * f.ep[a] + gh * f.er[a];
    grad[a] = -(gp[0] * f.er[a] + gp[1] * ds + gp[2] * dh);
  }
}

// Lattice porosity of a signed distance (Def. Lattice Porosity).
__device__ __forceinline__ double transition(double phi, double eps, int kind) {
  if (phi <= -0.5 * eps) return 0.0;
  if (phi >= 0.5 * eps) return 1.0;
  if (kind == 1) return phi / eps + 0.5;
  return 0.5 * (1.0 + tanh(4.0 * phi / eps) / tanh(2.0));
}

__device__ __forceinline__ int rotor_of_slot(const RotorTable& rt, int64_t s) {
  int k = 0;
  for (int j = 1; j < rt.n; ++j)
    if (s >= rt.r[j].off) k = j;
  return k;
}

__device__ __forceinline__ void slot_cell(const RotorDev& r, int64_t s, int& x, int& y, int& z) {
  const uint32_t l = uint32_t(s - r.off);  // box slots fit in 32 bits
  const uint32_t pl = uint32_t(r.bn[0]) * uint32_t(r.bn[1]);
  const uint32_t lz = l / pl, rem = l - lz * pl;
  const uint32_t ly = rem / uint32_t(r.bn[0]);
  z = r.b0[2] + int(lz);
  y = r.b0[1] + int(ly);
  x = r.b0[0] + int(rem - ly * uint32_t(r.bn[0]));
}

__device__ __forceinline__ bool in_box(const RotorDev& r, int x, int y, int z) {
  return x >= r.b0[0] && x < r.b0[0] + r.bn[0] && y >= r.b0[1] && y < r.b0[1] + r.bn[1] && z >= r.b0[2] &&
         z < r.b0[2] + r.bn[2];
}

// ---------------------------------------------------------------- wall model
// Forward-mode dual numbers with K directions: differentiate the wall model
// exactly as executed.  Four directions (probe velocity, previous friction
// velocity) for the model, two (tangential slip U, previous friction
// velocity) inside the Newton solves, which depend on those two only.
namespace dual {
template <int K>
struct Dual {
  double v, g[K];
};
template <int K> __device__ __forceinline__ Dual<K> mk(double v) { Dual<K> r; r.v = v; for (int q = 0; q < K; ++q) r.g[q] = 0.0; return r; }
template <int K> __device__ __forceinline__ Dual<K> operator+(Dual<K> a, Dual<K> b) { Dual<K> r; r.v = a.v + b.v; for (int q = 0; q < K; ++q) r.g[q] = a.g[q] + b.g[q]; return r; }
template <int K> __device__ __forceinline__ Dual<K> operator-(Dual<K> a, Dual<K> b) { Dual<K> r; r.v = a.v - b.v; for (int q = 0; q < K; ++q) r.g[q] = a.g[q] - b.g[q]; return r; }
template <int K> __device__ __forceinline__ Dual<K> operator*(Dual<K> a, Dual<K> b) { Dual<K> r; r.v = a.v * b.v; for (int q = 0; q < K; ++q) r.g[q] = a.g[q] * b.v + a.v * b.g[q]; return r; }
template <int K> __device__ __forceinline__ Dual<K> operator/(Dual<K> a, Dual<K> b) {
  Dual<K> r; r.v = a.v / b.v;
  const double ib = 1.0 / (b.v * b.v);
  for (int q = 0; q < K; ++q) r.g[q] = (a.g[q] * b.v - a.v * b.g[q]) * ib;
  return r;
}
template <int K> __device__ __forceinline__ Dual<K> operator+(Dual<K> a, double b) { return a + mk<K>(b); }
template <int K> __device__ __forceinline__ Dual<K> operator-(Dual<K> a, double b) { return a - mk<K>(b); }
template <int K> __device__ __forceinline__ Dual<K> operator-(double a, Dual<K> b) { return mk<K>(a) - b; }
template <int K> __device__ __forceinline__ Dual<K> operator*(double a, Dual<K> b) { return mk<K>(a) * b; }
template <int K> __device__ __forceinline__ Dual<K> operator*(Dual<K> a, double b) { return a * mk<K>(b); }
template <int K> __device__ __forceinline__ Dual<K> operator/(Dual<K> a, double b) { return a / mk<K>(b); }
template <int K> __device__ __forceinline__ Dual<K> operator/(double a, Dual<K> b) { return mk<K>(a) / b; }
template <int K> __device__ __forceinline__ Dual<K> operator+(double a, Dual<K> b) { return mk<K>(a) + b; }
template <int K> __device__ __forceinline__ Dual<K> sqrt(Dual<K> a) { Dual<K> r; r.v = ::sqrt(a.v); for (int q = 0; q < K; ++q) r.g[q] = a.g[q] / (2.0 * r.v); return r; }
template <int K> __device__ __forceinline__ Dual<K> exp(Dual<K> a) { Dual<K> r; r.v = ::exp(a.v); for (int q = 0; q < K; ++q) r.g[q] = a.g[q] * r.v; return r; }
template <int K> __device__ __forceinline__ Dual<K> log(Dual<K> a) { Dual<K> r; r.v = ::log(a.v); for (int q = 0; q < K; ++q) r.g[q] = a.g[q] / a.v; return r; }
template <int K> __device__ __forceinline__ double val(Dual<K> a) { return a.v; }
template <int K> __device__ __forceinline__ Dual<K> rcp_nr(Dual<K> a) { return 1.0 / a; }
template <int K> __device__ __forceinline__ Dual<K> div_nr(Dual<K> a, Dual<K> b) { return a / b; }
using D4 = Dual<4>;
using D2 = Dual<2>;
using D1 = Dual<1>;
}  // namespace dual
using dual::D4;
using dual::D2;
using dual::D1;
// FP64 reciprocal and quotient for the positive or negative, normal operands
// of the wall law (no zeros, infinities or denormals): the hardware
// reciprocal estimate refined by two Newton-Raphson steps for 1/x,
// r <- r + r (1 - x r), each of which squares the relative error; the
// quotient q = a r then gets one residual correction q <- q + r (a - b q).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double div_nr(double a, double b) {
  const double r = rcp_nr(b);
  const double q = a * r;
  return fma(r, fma(-b, q, a), q);
}
using dual::rcp_nr;
using dual::div_nr;
__device__ __forceinline__ double val(double a) { return a; }
using dual::val;
template <class R> struct Cst;
template <> struct Cst<double> { __device__ static double make(double v) { return v; } };
template <int K> struct Cst<dual::Dual<K>> { __device__ static dual::Dual<K> make(double v) { return dual::mk<K>(v); } };
template <class R> __device__ __forceinline__ R cst(double v) { return Cst<R>::make(v); }

// The Newton solves of the wall model in plain FP64, or with the two
// directions (U, u_tau^prev) when the model carries four: seeds and the
// chain rule back to the model's directions.
template <class R> struct NewtonType { using type = R; };
template <> struct NewtonType<D4> { using type = D2; };
__device__ __forceinline__ double seed_newton(double a, int) { return a; }
__device__ __forceinline__ D2 seed_newton(const D4& a, int dir) {
  D2 r;
  r.v = a.v;
  r.g[0] = dir == 0 ? 1.0 : 0.0;
  r.g[1] = dir == 1 ? 1.0 : 0.0;
  return r;
}
__device__ __forceinline__ double lift_newton(double a, double, double) { return a; }
__device__ __forceinline__ D4 lift_newton(const D2& a, const D4& U, const D4& utp) {
  D4 r;
  r.v = a.v;
  for (int q = 0; q < 4; ++q) r.g[q] = a.g[0] * U.g[q] + a.g[1] * utp.g[q];
  return r;
}

// Truncated Spalding bracket e^k - 1 - k - k^2/2 - k^3/6 (eq. spalding) with
// the exponential capped at e^80, and its derivative.
template <class R>
__device__ __forceinline__ R spalding_bracket(R k) {
  const R ek = val(k) > 80.0 ? cst<R>(::exp(80.0)) : exp(k);
  return ek - 1.0 - k - k * k * 0.5 - k * k * k / 6.0;
}
template <class R>
__device__ __forceinline__ R spalding_dbracket(R k) {
  const R ek = val(k) > 80.0 ? cst<R>(0.0) : exp(k);
  return ek - 1.0 - k - k * k * 0.5;
}

// Newton iteration of Sec. 2.2.1 (stop when |f(u^{j+1}) - f(u^j)| < tol or
// after maxit steps, halving a non-positive iterate, counted in halvings).
template <class R, class F>
__device__ __forceinline__ R newton(R u, F&& fdf, double tol, int maxit, int& iters, int& halvings) {
  R fu, du;
  fdf(u, fu, du);
  int it = 0;
  for (; it < maxit; ++it) {
    R un = u - div_nr(fu, du);
    if (val(un) <= 0.0) {
      un = 0.5 * u;
      ++halvings;
    }
    R fn, dn;
    fdf(un, fn, dn);
    const bool done = fabs(val(fn) - val(fu)) < tol;
    u = un;
    fu = fn;
    du = dn;
    if (done) {
      ++it;
      break;
    }
  }
  iters = it;
  return u;
}

// Tangential slip U and its direction t of the probe velocity us relative
// to the wall velocity uw (outward normal nn).  False when U is below 1e-6
// (cell treated as a plain cell): the slip direction is undefined as the
// slip vanishes (by symmetry on a rotor axis), and the bound sits above FP32
// rounding noise in the probe velocity.
template <class R>
__device__ __forceinline__ bool wall_slip(const R us[3], const double uw[3], const double nn[3], R& U, R t[3]) {
  R v[3] = {us[0] - uw[0], us[1] - uw[1], us[2] - uw[2]};
  const R vn = v[0] * nn[0] + v[1] * nn[1] + v[2] * nn[2];
  R vt[3] = {v[0] - vn * nn[0], v[1] - vn * nn[1], v[2] - vn * nn[2]};
  const R U2 = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2];
  if (!(::sqrt(val(U2)) >= 1e-6)) return false;
  U = sqrt(U2);
  const R iU = 1.0 / U;
  for (int a = 0; a < 3; ++a) t[a] = vt[a] * iU;
  return true;
}

// The two Newton solves: u_tau from the slip U (guess: the previous u_tau,
// else the laminar estimate), then u+ at y1+.  safe: Newton halvings and
// evaluations whose exponential argument took the cap at 80.
struct Safeguards {
  int halvings = 0, caps = 0;
};
template <class RN>
__device__ __forceinline__ void wall_newtons(RN Un, RN utpn, bool prev_active, double y1, const Model& m, RN& utn,
                                             RN& upn, int& it1, Safeguards& safe) {
  const double E = m.E, kap = m.kappa;
  // the Newton chains run on one lane per wall cell: every division is a
  // long dependent sequence in FP64, so the constants enter as reciprocals
  const double sixth = 1.0 / 6.0;
  const RN guess = prev_active ? utpn : sqrt(m.nu_ys * Un);
  utn = newton(
      guess,
      [&](RN u, RN& f, RN& df) {
        const RN iu = rcp_nr(u);
        const RN p = Un * iu;
        const RN k = kap * p;
        if (val(k) > 80.0) ++safe.caps;
        const RN ek = val(k) > 80.0 ? cst<RN>(::exp(80.0)) : exp(k);
        const RN dek = val(k) > 80.0 ? cst<RN>(0.0) : ek;
        const RN poly = 1.0 + k + k * k * 0.5;
        f = p + (ek - poly - k * k * k * sixth) * m.inv_E - m.ys_nu * u;
        df = 0.0 - (p * iu) * (1.0 + m.kappa_E * (dek - poly)) - m.ys_nu;
      },
      m.tol, m.maxit, it1, safe.halvings);
  const RN yp = y1 * utn * m.inv_nu;
  const RN ylog = val(yp) > 1.0 ? yp : cst<RN>(1.0);
  const RN ulog = log(E * ylog) * m.inv_kappa;
  int it2 = 0;
  upn = newton(
      val(ulog) < val(yp) ? ulog : yp,
      [&](RN u, RN& f, RN& df) {
        const RN k = kap * u;
        if (val(k) > 80.0) ++safe.caps;
        const RN ek = val(k) > 80.0 ? cst<RN>(::exp(80.0)) : exp(k);
        const RN dek = val(k) > 80.0 ? cst<RN>(0.0) : ek;
        const RN poly = 1.0 + k + k * k * 0.5;
        f = u + (ek - poly - k * k * k * sixth) * m.inv_E - yp;
        df = 1.0 + m.kappa_E * (dek - poly);
      },
      m.tol, m.maxit, it2, safe.halvings);
}

// u_wm = u_tau u+ t, S_wm = (U - u_tau u+) / (2 (y_s - y1)) (t n + n t), u_tau.
template <class R>
__device__ __forceinline__ void wall_outputs(R U, const R t[3], R qv, R ut, const double nn[3], double y1,
                                             const Model& m, R out[10]) {
  const R hd = 0.5 * ((U - qv) / (m.y_s - y1));
  out[0] = qv * t[0];
  out[1] = qv * t[1];
  out[2] = qv * t[2];
  out[3] = hd * (t[0] * nn[0] + nn[0] * t[0]);
  out[4] = hd * (t[1] * nn[1] + nn[1] * t[1]);
  out[5] = hd * (t[2] * nn[2] + nn[2] * t[2]);
  out[6] = hd * (t[0] * nn[1] + nn[0] * t[1]);
  out[7] = hd * (t[0] * nn[2] + nn[0] * t[2]);
  out[8] = hd * (t[1] * nn[2] + nn[1] * t[2]);
  out[9] = ut;
}

// Wall model of one cell given its probe velocity us, wall velocity uw,
// outward normal nn, wall distance y1 and the previous friction velocity:
// out = (u_wm[3], S[6] as xx yy zz xy xz yz, u_tau); false for a plain cell.
template <class R>
__device__ __forceinline__ bool wall_solve(const R us[3], const double uw[3], const double nn[3], double y1,
                                           R utp, bool prev_active, const Model& m, R out[10], int& it1,
                                           Safeguards& safe) {
  it1 = 0;
  R U, t[3];
  if (!wall_slip<R>(us, uw, nn, U, t)) return false;
  using RN = typename NewtonType<R>::type;
  RN utn, upn;
  wall_newtons<RN>(seed_newton(U, 0), seed_newton(utp, 1), prev_active, y1, m, utn, upn, it1, safe);
  wall_outputs<R>(U, t, lift_newton(utn * upn, U, utp), lift_newton(utn, U, utp), nn, y1, m, out);
  return true;
}

// Probe corner `corner` (0..7) of wall slot s at list position w: its cell
// and trilinear weight, the cell position and the foot-point wall velocity.
struct Probe {
  int x, y, z;        // wall cell
  int q[3];           // this lane's corner cell
  double wgt;
  double y1, nn[3], uw[3];
};
__device__ __forceinline__ Probe probe_of(const RotorDev& R, const Geometry& g, const Model& m,
                                          const double* __restrict__ geo, int64_t total, int64_t s, int64_t w,
                                          int corner, bool periodic_x) {
  Probe p;
  slot_cell(R, s, p.x, p.y, p.z);
  p.y1 = -geo[w];
  p.nn[0] = geo[total + w]; p.nn[1] = geo[2 * total + w]; p.nn[2] = geo[3 * total + w];
  const double X[3] = {double(p.x), double(p.y), double(p.z)};
  double xw[3], xs[3];
  for (int a = 0; a < 3; ++a) {
    xw[a] = X[a] - p.y1 * p.nn[a];
    xs[a] = xw[a] + m.y_s * p.nn[a];
  }
  const double rw[3] = {xw[0] - R.c[0], xw[1] - R.c[1], xw[2] - R.c[2]};
  p.uw[0] = R.omega * (R.e[1] * rw[2] - R.e[2] * rw[1]);
  p.uw[1] = R.omega * (R.e[2] * rw[0] - R.e[0] * rw[2]);
  p.uw[2] = R.omega * (R.e[0] * rw[1] - R.e[1] * rw[0]);
  p.wgt = 1.0;
  for (int a = 0; a < 3; ++a) {
    const double fl = floor(xs[a]);
    const int bit = (corner >> a) & 1;
    const double fr = xs[a] - fl;
    p.q[a] = int(fl) + bit;
    p.wgt *= bit ? fr : 1.0 - fr;
  }
  p.q[1] = ((p.q[1] % g.ny) + g.ny) % g.ny;
  p.q[2] = ((p.q[2] % g.nz) + g.nz) % g.nz;
  if (periodic_x) p.q[0] = ((p.q[0] % g.nx) + g.nx) % g.nx;
  else p.q[0] = p.q[0] < 0 ? 0 : (p.q[0] > g.nx - 1 ? g.nx - 1 : p.q[0]);
  return p;
}

// Trilinear probe velocity summed over the eight lanes of a group in a fixed order.
__device__ __forceinline__ void group8_sum(double us[3]) {
  const int base = int(threadIdx.x & 63) & ~7;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = __shfl(us[a], base + j, 64);
    us[a] = ((o[0] + o[1]) + (o[2] + o[3])) + ((o[4] + o[5]) + (o[6] + o[7]));
  }
}

// Wall model (Sec. 2.2.1, Sec. 3.2) on the listed wall cells, eight lanes per
// cell: lane j pulls the populations of probe corner j and forms its
// velocity; the trilinear sum is reduced over the eight lanes; lane 0 runs
// the two Newton solves and writes u_wm, S_wm, sigma and the u_tau state.
// Adjoint of the torque objective with respect to the momentum exchange of
// a cell of tag t: d(e . (r x dP)) / d dP = e x r, weighted by w.
// Probe-velocity adjoints are summed in fixed point (fix_split / fix_merge),
// so that the sum of the scattered contributions does not depend on the
// order of the atomic additions and the gradient is reproducible bit for
// bit.  Accumulators [3 q + k][N] for component q, piece k; a value outside
// the range raises bit 1 of flag.
__device__ __forceinline__ void fix_add(unsigned long long* acc, int64_t N, int64_t c, int q, double v,
                                        int32_t* flag) {
  long long p[3];
  if (!fix_split(v, p)) {
    atomicOr(flag, 2);
    return;
  }
  unsigned long long* b = acc + int64_t(3 * q) * N + c;
  atomicAdd(b, (unsigned long long)p[0]);
  atomicAdd(b + N, (unsigned long long)p[1]);
  atomicAdd(b + 2 * N, (unsigned long long)p[2]);
}

// The sum of component q at cell c as FP64; the accumulators are zeroed.
__device__ __forceinline__ double fix_take(unsigned long long* acc, int64_t N, int64_t c, int q) {
  unsigned long long* b = acc + int64_t(3 * q) * N + c;
  const long long s2 = (long long)b[0], s1 = (long long)b[N], s0 = (long long)b[2 * N];
  b[0] = 0ull;
  b[N] = 0ull;
  b[2 * N] = 0ull;
  return fix_merge(s2, s1, s0);
}

template <class CT>
__device__ __forceinline__ void objective_dp(const RotorTable& rt, int t, int obj_tag, double w, int x, int y, int z,
                                             CT pb[3]) {
  pb[0] = pb[1] = pb[2] = CT(0);
  if (w == 0.0 || t == 0 || (obj_tag != 0 && obj_tag != t)) return;
  const double* fr = rt.frame[t];
  const double rx = x - fr[0], ry = y - fr[1], rz = z - fr[2];
  // d(e . (r x dP)) / d dP = e x r
  pb[0] = CT(w * (fr[4] * rz - fr[5] * ry));
  pb[1] = CT(w * (fr[5] * rx - fr[3] * rz));
  pb[2] = CT(w * (fr[3] * ry - fr[4] * rx));
}

template <class CT>
struct WallArgs {
  const RotorTable* rot;
  Geometry g;
  Model m;
  int64_t total;             // box slots
  const void* src;           // state of the step (storage type)
  const double* geo;         // [4][total] of the step's geometry
  const int32_t* wlist;
  const int32_t* wcount;
  const double* ut_prev;
  const uint8_t* act_prev;
  double* ut_new;
  uint8_t* act_new;
  CT* wall_out;              // [10][total]
  unsigned long long* stats; // Newton statistics (count_stats != 0)
  const double* ghost;       // FP64 inflow plane of the step
  int32_t count_stats;
  // adjoint instantiation only: the transposed wall-model Jacobian applied
  // at each active wall cell (the adjoint wall step)
  const CT* lam_in;          // adjoint of the state after the step (blocked layout)
  const CT* side_in;         // outflow share of lam_in on the last x plane (nullable)
  const CT* d_eff;
  const uint8_t* tag;
  const CT* ghost_ct;        // inflow plane in the compute type
  const double* ut_bar_in;   // adjoint of the friction velocity written by the step
  double* ut_bar_out;        // adjoint of the friction velocity read by the step
  unsigned long long* ubar;  // probe-velocity adjoints in fixed point ([9][N], fix_add)
  int32_t* flag;             // bit 1: a probe-velocity adjoint outside the fixed-point range
  double obj_w;              // weight of this step's torque in J
  int32_t obj_tag;
};

// Workgroup `blk` of `nblk` doing the wall model: a persistent loop over the
// device-side wall-cell count.  kAdj: also the adjoint wall step of the
// discrete adjoint: the wall model with its 10 x 4 Jacobian (dual numbers),
// the collision VJP at the wall cell for the adjoint of (u_wm, S), the
// transposed Jacobian giving the adjoints of the probe velocity (scattered to
// the eight probe corners with the trilinear weights) and of u_tau^prev.
template <class ST, class CT, bool kPeriodicX, bool kAdj, int Q = 27>
__device__ __forceinline__ void wall_cells(const WallArgs<CT>& a, uint32_t blk, uint32_t nblk) {
  const RotorTable& rt = *a.rot;
  const Geometry& g = a.g;
  const Model& m = a.m;
  const int64_t total = a.total;
  const ST* __restrict__ src = static_cast<const ST*>(a.src);
  const double* __restrict__ geo = a.geo;
  const int32_t* __restrict__ wlist = a.wlist;
  const double* __restrict__ ut_prev = a.ut_prev;
  const uint8_t* __restrict__ act_prev = a.act_prev;
  double* __restrict__ ut_new = a.ut_new;
  uint8_t* __restrict__ act_new = a.act_new;
  CT* __restrict__ wall_out = a.wall_out;
  const int corner = threadIdx.x & 7;
  const int count = *a.wcount;
  // each wave takes 8 consecutive list entries per iteration; the trip count
  // is uniform over the wave so that every lane takes part in the shuffles
  const int64_t wave = (int64_t(blk) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t(nblk) * blockDim.x) >> 6;
  const int64_t lw = (threadIdx.x & 63) >> 3;
  // the first entry is read before the count arrives: the list holds total
  // entries, so the clamped read is in bounds, and lanes past the count only
  // compute on a valid (stale) entry whose results are dropped
  const int64_t w0 = wave * 8 + lw < total ? wave * 8 + lw : total - 1;
  const int32_t s0 = min(wlist[w0], int32_t(total - 1));
  for (int64_t wb = wave * 8; wb < count; wb += nwaves * 8) {
    const int64_t w = wb + lw;
    const bool live = w < count;
    const int64_t wr = wb == wave * 8 ? w0 : (live ? w : wb);
    // every entry is a box slot; the clamp keeps a corrupt entry in bounds
    const int64_t s = wb == wave * 8 ? s0 : min(wlist[wr], int32_t(total - 1));
    // state of the previous step, loaded early (used by the Newton guess)
    const double utp = ut_prev[s];
    const bool actp = act_prev[s] != 0;
    const RotorDev& R = rt.r[rotor_of_slot(rt, s)];
    const Probe pr = probe_of(R, g, m, geo, total, s, wr, corner, kPeriodicX);
    double h[Q];
    pull_cell<ST, double, kPeriodicX, Q>(src, g, pr.q[0], pr.q[1], pr.q[2], a.ghost, h);
    const Moments<double> mo = moments_q<Q, double>(h);
    const double rho = 1.0 + mo.drho;
    double us[3] = {pr.wgt * (mo.jx / rho), pr.wgt * (mo.jy / rho), pr.wgt * (mo.jz / rho)};
    group8_sum(us);
    int it1 = 0, done = 0;
    Safeguards safe;
    double usb[3] = {0.0, 0.0, 0.0};
    // adjoint: the model with its 10 x 4 Jacobian with respect to (us,
    // u_tau^prev).  The Newton solves depend on (U, u_tau^prev) only; lanes
    // 0 and 1 of the group run them with one derivative direction each (the
    // same value chain), and lane 0 takes lane 1's derivatives.
    D4 o4[kAdj ? 10 : 1] = {};
    bool slip = false;
    if constexpr (kAdj) {
      D4 ud[3];
      for (int q = 0; q < 3; ++q) { ud[q] = dual::mk<4>(us[q]); ud[q].g[q] = 1.0; }
      D4 up = dual::mk<4>(utp);
      up.g[3] = 1.0;
      D4 Ud, td[3];
      D1 ut1{}, up1{};
      if (corner < 2 && live) {
        slip = wall_slip<D4>(ud, pr.uw, pr.nn, Ud, td);
        if (slip) {
          D1 Un, utpn;
          Un.v = Ud.v;
          Un.g[0] = corner == 0 ? 1.0 : 0.0;
          utpn.v = utp;
          utpn.g[0] = corner == 1 ? 1.0 : 0.0;
          wall_newtons<D1>(Un, utpn, actp, pr.y1, m, ut1, up1, it1, safe);
        }
      }
      const int lead = int(threadIdx.x & 63) & ~7;
      const double dut = __shfl(ut1.g[0], lead + 1, 64), dup = __shfl(up1.g[0], lead + 1, 64);
      if (corner == 0 && live && slip) {
        D2 ut2, up2;
        ut2.v = ut1.v; ut2.g[0] = ut1.g[0]; ut2.g[1] = dut;
        up2.v = up1.v; up2.g[0] = up1.g[0]; up2.g[1] = dup;
        wall_outputs<D4>(Ud, td, lift_newton(ut2 * up2, Ud, up), lift_newton(ut2, Ud, up), pr.nn, pr.y1, m, o4);
      }
    }
    if (corner == 0 && live) {
      const int64_t T = total;
      bool active;
      double out[10];
      if constexpr (kAdj) {
        active = slip;
        for (int q = 0; q < 10; ++q) out[q] = o4[q].v;
      } else {
        active = wall_solve<double>(us, pr.uw, pr.nn, pr.y1, utp, actp, m, out, it1, safe);
      }
      if (!active) {
        for (int q = 0; q < 9; ++q) wall_out[q * T + s] = CT(0);
        wall_out[9 * T + s] = CT(1);
        act_new[s] = 0;
      } else {
        for (int q = 0; q < 9; ++q) wall_out[q * T + s] = CT(out[q]);
        wall_out[9 * T + s] = CT(0);
        ut_new[s] = out[9];
        act_new[s] = 1;
        done = 1;
      }
      if constexpr (kAdj) {
        if (active) {
          const int x = pr.x, y = pr.y, z = pr.z;
          const int64_t c = (int64_t(z) * g.ny + y) * g.nx + x;
          CT hc[Q];
          pull_cell<ST, CT, kPeriodicX, Q>(src, g, x, y, z, a.ghost_ct, hc);
          const Moments<CT> mc = moments_q<Q, CT>(hc);
          // adjoint of the state after the step at this cell; on the last
          // x plane lam_in also holds the outflow share of the c_x = -1 states
          const bool fix = !kPeriodicX && a.side_in && x == g.nx - 1;
          const int64_t k = int64_t(z) * g.ny + y, plane = int64_t(g.ny) * g.nz;
          CT gb[Q];
          for (int i = 0; i < Q; ++i) {
            CT l = a.lam_in[pop_at<Q>(g, i, x, y, z)];
            if (fix && i < xgroup_of<Q>(1)) l += a.side_in[i * plane + k];
            gb[i] = CT(wq<Q>(i)) * l;
          }
          // the FSI inputs of the cell as the sweep of the step read them
          const uint8_t tb = a.tag[c];
          const CT d = a.d_eff[c];
          const double rx = x - R.c[0], ry = y - R.c[1], rz = z - R.c[2];
          const CT b[3] = {CT(R.omega * (R.e[1] * rz - R.e[2] * ry)) + CT(out[0]),
                           CT(R.omega * (R.e[2] * rx - R.e[0] * rz)) + CT(out[1]),
                           CT(R.omega * (R.e[0] * ry - R.e[1] * rx)) + CT(out[2])};
          CT S[6];
          for (int q = 0; q < 6; ++q) S[q] = CT(out[3 + q]);
          CT pb[3];
          objective_dp<CT>(rt, tb & kTagMask, a.obj_tag, a.obj_w, x, y, z, pb);
          Moments<CT> mb;
          CT db, bb[3], Sb[6];
          collide_vjp<CT, Q>(mc, d, b[0], b[1], b[2], CT(0), S, CT(m.tau0), CT(m.smag), gb, pb, mb, db, bb, Sb);
          double ob[10];
          for (int q = 0; q < 3; ++q) ob[q] = double(bb[q]);
          for (int q = 0; q < 6; ++q) ob[3 + q] = double(Sb[q]);
          ob[9] = a.ut_bar_in[s];
          double ib[4] = {0.0, 0.0, 0.0, 0.0};
          for (int q = 0; q < 10; ++q)
            for (int r = 0; r < 4; ++r) ib[r] += ob[q] * o4[q].g[r];
          usb[0] = ib[0]; usb[1] = ib[1]; usb[2] = ib[2];
          a.ut_bar_out[s] = ib[3];
        }
      }
    }
    if constexpr (kAdj) {
      // broadcast the probe adjoint of the group's lane 0 and scatter per corner
      const int lead = int(threadIdx.x & 63) & ~7;
      double v[3];
      for (int q = 0; q < 3; ++q) v[q] = __shfl(usb[q], lead, 64);
      if (live && (v[0] != 0.0 || v[1] != 0.0 || v[2] != 0.0)) {
        const int64_t cc = (int64_t(pr.q[2]) * g.ny + pr.q[1]) * g.nx + pr.q[0];
        for (int q = 0; q < 3; ++q) fix_add(a.ubar, g.N, cc, q, pr.wgt * v[q], a.flag);
      }
    }
    // Newton statistics (diagnostics steps): one atomic per wave; the
    // safeguards of the solves run by lane 0 of each group
    if (a.count_stats) {
      const bool lead_live = corner == 0 && live;
      int a1 = it1, a2 = done, a3 = lead_live ? safe.halvings : 0, a4 = lead_live ? safe.caps : 0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        a1 += __shfl_xor(a1, o, 64);
        a2 += __shfl_xor(a2, o, 64);
        a3 += __shfl_xor(a3, o, 64);
        a4 += __shfl_xor(a4, o, 64);
      }
      if ((threadIdx.x & 63) == 0 && a2) {
        atomicAdd(&a.stats[0], (unsigned long long)a1);
        atomicAdd(&a.stats[1], (unsigned long long)a2);
      }
      if ((threadIdx.x & 63) == 0 && (a3 | a4)) {
        atomicAdd(&a.stats[2], (unsigned long long)a3);
        atomicAdd(&a.stats[3], (unsigned long long)a4);
      }
    }
  }
}

template <class ST, class CT, bool kPeriodicX, bool kAdj, int Q>
__global__ __launch_bounds__(256) void k_wall(WallArgs<CT> a) {
  wall_cells<ST, CT, kPeriodicX, kAdj, Q>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- geometry
// One launch per step over the rotor boxes' slots (one lane per slot): the
// rotor geometry of the step (porosity, tag, wall flag, normal and wall
// distance) and the wall-model work list; extra workgroups write the step's
// inflow plane.
template <class CT>
struct GeoArgs {
  const RotorTable* rot;
  Geometry g;
  Model m;
  const BladeTrig* trig;     // blade angles of the step
  int64_t total;             // box slots
  const CT* d_static;
  const uint8_t* tag_static;
  const CT* dd;              // nullable
  CT* d_eff;
  uint8_t* tag;
  double* geo;               // [4][total]: phi, n of the listed wall cells, by list position
  uint8_t* act_new;          // wall-state slots, reset to inactive
  int32_t* wlist;
  int32_t* wcount;           // this launch's counter (zero on entry)
  int32_t* wcount_next;      // the next launch's counter, zeroed here
  int64_t step;              // inflow plane of the step (extra workgroups)
  CT* ghost;
  double* ghost64;
  int32_t ghost_blocks;
  // growth layer (nullable): evaluate the rotor distance only on the slots
  // with mark_in == key; mark for the next step (key + 1) the slots within
  // one cell of every evaluated slot whose distance exceeds -mark_cut
  const long long* mark_in;
  long long* mark_out;
  long long key;
  double mark_cut;
  // per geometry workgroup: rotor distances evaluated and box slots visited
  // since creation ([2 bid], [2 bid + 1]; each entry written by one
  // workgroup per launch, so no atomics)
  unsigned long long* gstats;
};

// Workgroup `bid` of the geometry work: box slots first, then the extra
// workgroups of the inflow plane.
template <class CT, int Q = 27>
__device__ __forceinline__ void geometry_block(const GeoArgs<CT>& a, uint32_t bid) {
  const Geometry& g = a.g;
  const Model& m = a.m;
  const uint32_t nbw = uint32_t((a.total + 255) / 256);
  if (bid >= nbw) {
    const int64_t plane = int64_t(g.ny) * g.nz;
    const int64_t k = (int64_t(bid) - nbw) * 256 + threadIdx.x;
    if (k < plane) inflow_plane_cell<CT, Q>(g, m, a.step, k, a.ghost, a.ghost64);
    return;
  }
  __shared__ int wl_count, wl_base, n_eval, n_live;
  if (threadIdx.x == 0) {
    wl_count = 0;
    n_eval = 0;
    n_live = 0;
    if (bid == 0) *a.wcount_next = 0;
  }
  __syncthreads();
  const int64_t s0 = int64_t(bid) * blockDim.x + threadIdx.x;
  const bool live = s0 < a.total;
  const int64_t s = live ? s0 : a.total - 1;
  const RotorTable& rt = *a.rot;
  const int k = rotor_of_slot(rt, s);
  int x, y, z;
  slot_cell(rt.r[k], s, x, y, z);
  const int64_t c = (int64_t(z) * g.ny + y) * g.nx + x;
  double best = -1e300, gr[3] = {0, 0, 0};
  int br = -1;
  RotorPhi win{};
  // growth layer: a slot outside it is fluid for every rotor at this step
  const bool eval = !a.mark_in || a.mark_in[s] == a.key;
  for (int j = 0; eval && j < rt.n; ++j) {
    if (!in_box(rt.r[j], x, y, z)) continue;
    RotorPhi p = rotor_phi(rt.r[j], a.trig->c[j], a.trig->s[j], double(x), double(y), double(z), 0.5 * m.eps_h + 1.0);
    if (p.phi > best) {
      best = p.phi;
      br = j;
      win = p;
    }
  }
  {
    // counts of the wave into the workgroup's (one LDS atomic per wave)
    const unsigned long long be = __ballot(live && eval), bl = __ballot(live);
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&n_eval, int(__popcll(be)));
      atomicAdd(&n_live, int(__popcll(bl)));
    }
  }
  if (live && a.mark_out && best > -a.mark_cut) {
    // the slots of this box within one cell form the next step's layer
    const RotorDev& R = rt.r[k];
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int xn = x + dx, yn = y + dy, zn = z + dz;
          if (!in_box(R, xn, yn, zn)) continue;
          const int64_t sn = R.off + (int64_t(zn - R.b0[2]) * R.bn[1] + (yn - R.b0[1])) * R.bn[0] + (xn - R.b0[0]);
          a.mark_out[sn] = a.key + 1;
        }
  }
  // the normal is needed by wall-cell candidates only (band -eps_h/2 < phi < 0)
  if (br >= 0 && m.wall_model && best > -0.5 * m.eps_h && best < 0.0)
    rotor_grad(rt.r[br], a.trig->c[br], a.trig->s[br], double(x), double(y), double(z), win, gr);
  const double drot = br >= 0 ? transition(best, m.eps_h, m.transition) : 0.0;
  const double ds = double(a.d_static[c]);
  const double base = ds > drot ? ds : drot;
  if (live) a.d_eff[c] = CT(base) + (a.dd ? a.dd[c] : CT(0));
  const double gn = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
  uint8_t tb;
  if (drot > 0.0) {
    tb = uint8_t(rt.r[br].tag) | kRotorBit;
    if (m.wall_model && best > -0.5 * m.eps_h && best < 0.0 && gn > 0) tb |= kWallBit;
  } else {
    tb = a.tag_static[c];
  }
  if (live) {
    a.tag[c] = tb;
    a.act_new[s] = 0;
  }
  // wall cells of this box's own rotor go to the work list: ranks from an
  // LDS counter, one global atomic per workgroup
  const bool mine = live && (tb & kWallBit) && br == k;
  int rank = 0;
  if (mine) rank = atomicAdd(&wl_count, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    wl_base = wl_count ? atomicAdd(a.wcount, wl_count) : 0;
    if (a.gstats) {
      a.gstats[2 * bid] += (unsigned long long)n_eval;
      a.gstats[2 * bid + 1] += (unsigned long long)n_live;
    }
  }
  __syncthreads();
  if (!mine) return;
  // the wall cell's distance and normal beside its list entry, so that the
  // wall model reads both with one dependent load
  const int64_t pos = wl_base + rank;
  const double inv = 1.0 / gn;
  a.wlist[pos] = int32_t(s);
  a.geo[pos] = best;
  a.geo[a.total + pos] = -gr[0] * inv;
  a.geo[2 * a.total + pos] = -gr[1] * inv;
  a.geo[3 * a.total + pos] = -gr[2] * inv;
}

template <class CT, int Q>
__global__ __launch_bounds__(256) void k_geometry(GeoArgs<CT> a) {
  geometry_block<CT, Q>(a, blockIdx.x);
}

// The wall model of one step (workgroups [0, wall_blocks)) and the geometry
// of the next step (the remaining workgroups) in one launch: the two are
// independent when the geometry writes the other buffer set, and both are
// latency-bound chains that overlap well.
template <class ST, class CT, bool kPeriodicX, bool kAdj, int Q>
__global__ __launch_bounds__(256) void k_wall_geometry(WallArgs<CT> w, GeoArgs<CT> ga, uint32_t wall_blocks) {
  if (blockIdx.x < wall_blocks) wall_cells<ST, CT, kPeriodicX, kAdj, Q>(w, blockIdx.x, wall_blocks);
  else geometry_block<CT, Q>(ga, blockIdx.x - wall_blocks);
}

// ================================================================ fused sweep
template <class CT>
struct SweepArgs {
  const void* src;
  void* dst;
  Geometry g;
  Model m;
  const int32_t* blk_slot;
  const CT* d_eff;
  const uint8_t* tag;
  const CT* wall_out;
  int64_t bbox_total;
  const RotorTable* rot;
  const CT* uB_static;
  double* partial;
  double* mass_part;
  int32_t* flag;
  const CT* ghost;
  int64_t step;
  int64_t nblocks;
  CT* out_rho;
  CT* out_u;
  CT* out_uhat;
  // finite-difference strain (nullable fd_u: off)
  const CT* fd_u;
  const int32_t* near_index;
  CT fd_share;
};

// The velocity field of the finite-difference strain: the pre-collision
// velocity of the cells of the listed tiles ([index][3][kBlock]).
template <class CT>
struct FdField {
  const CT* fd_u;
  const int32_t* near_index;
};

// Pre-collision velocity component a of cell (x, y, z) from the velocity
// buffer of the listed tiles.
template <class CT>
__device__ __forceinline__ CT fd_velocity(const Geometry& g, const FdField<CT>& f, int a, int x, int y, int z) {
  const int64_t canon = (int64_t(z) * g.nty + y / kTileY) * g.ntx + x / kTileX;
  const int32_t k = f.near_index[canon];
  return f.fd_u[(int64_t(k) * 3 + a) * kBlock + (y % kTileY) * kTileX + (x % kTileX)];
}

// Neighbours of the central differences: y, z periodic, x periodic or
// clamped to the first and last plane.
template <bool kPeriodicX>
__device__ __forceinline__ void fd_stencil(const Geometry& g, int x, int y, int z, int& xm, int& xp, int& ym, int& yp,
                                           int& zm, int& zp) {
  if (kPeriodicX) {
    xm = x == 0 ? g.nx - 1 : x - 1;
    xp = x + 1 == g.nx ? 0 : x + 1;
  } else {
    xm = x == 0 ? 0 : x - 1;
    xp = x + 1 == g.nx ? x : x + 1;
  }
  ym = y == 0 ? g.ny - 1 : y - 1;
  yp = y + 1 == g.ny ? 0 : y + 1;
  zm = z == 0 ? g.nz - 1 : z - 1;
  zp = z + 1 == g.nz ? 0 : z + 1;
}

// Central-difference strain S_ab = (d_a u_b + d_b u_a) / 2 of the
// pre-collision velocity at (x, y, z), d_b u_a = (u_a(x + e_b) - u_a(x - e_b))
// / 2.  Order xx, yy, zz, xy, xz, yz.
template <class CT, bool kPeriodicX>
__device__ __forceinline__ void fd_strain(const Geometry& g, const FdField<CT>& f, int x, int y, int z, CT S[6]) {
  int xm, xp, ym, yp, zm, zp;
  fd_stencil<kPeriodicX>(g, x, y, z, xm, xp, ym, yp, zm, zp);
  CT d[3][3];  // d[a][b] = d_b u_a
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d[a][0] = CT(0.5) * (fd_velocity(g, f, a, xp, y, z) - fd_velocity(g, f, a, xm, y, z));
    d[a][1] = CT(0.5) * (fd_velocity(g, f, a, x, yp, z) - fd_velocity(g, f, a, x, ym, z));
    d[a][2] = CT(0.5) * (fd_velocity(g, f, a, x, y, zp) - fd_velocity(g, f, a, x, y, zm));
  }
  S[0] = d[0][0];
  S[1] = d[1][1];
  S[2] = d[2][2];
  S[3] = CT(0.5) * (d[0][1] + d[1][0]);
  S[4] = CT(0.5) * (d[0][2] + d[2][0]);
  S[5] = CT(0.5) * (d[1][2] + d[2][1]);
}

// One workgroup = kBlock consecutive cells.  Every cell pulls its 27
// populations, forms the moments, collides and writes its 27 post-collision
// values (kMoments: writes rho, u, u_hat instead).  Workgroups that touch a
// porous region (blk_slot >= 0) read porosity and tags, apply the
// homogenized velocity and the wall model outputs and reduce the momentum
// handed to each tag; the others run the plain bulk collision.
template <class ST, class CT, bool kPeriodicX, bool kMoments, int Q = 27>
__device__ __forceinline__ void sweep_tile(const SweepArgs<CT>& a, uint32_t blk, double (&lds)[4][kPartial]) {
  const Geometry& g = a.g;
  // tile (tx, ty, z): 64 consecutive x-cells per wave, 4 y-rows per workgroup
  // tile ids and counts fit 32 bits (fewer than 2^31 cells, 256 per tile)
  const TileId ti = tile_id(g, blk);
  const int z = ti.z, ty = ti.ty, tx = ti.tx;
  const int xr = tx * kTileX + int(threadIdx.x & (kTileX - 1));
  // one row per wave: y is uniform over the wave
  const int yr = __builtin_amdgcn_readfirstlane(ty * kTileY + int(threadIdx.x >> 6));
  const bool row_ok = yr < g.ny;
  const bool valid = xr < g.nx && row_ok;
  const int x = valid ? xr : 0, y = row_ok ? yr : 0;
  const int64_t c = (int64_t(z) * g.ny + y) * g.nx + x;
  const int32_t slot = a.blk_slot[ti.canon];

  CT h[Q];
  pull_row<ST, CT, kPeriodicX, Q>(static_cast<const ST*>(a.src), g, x, y, z, a.ghost, h);
  const Moments<CT> mo = moments_q<Q, CT>(h);
  const CT rho = CT(1) + mo.drho;
  const CT irho = rcp_ct(rho);
  const CT ux = mo.jx * irho, uy = mo.jy * irho, uz = mo.jz * irho;
  const CT tau0 = CT(a.m.tau0), smag = CT(a.m.smag);

  CT g2[Q];
  if (slot < 0) {
    if (kMoments) {
      if (valid) {
        a.out_rho[c] = rho;
        a.out_u[c] = ux; a.out_u[g.N + c] = uy; a.out_u[2 * g.N + c] = uz;
        if (a.out_uhat) { a.out_uhat[c] = ux; a.out_uhat[g.N + c] = uy; a.out_uhat[2 * g.N + c] = uz; }
      }
      return;
    }
    const CT S0[6] = {CT(0), CT(0), CT(0), CT(0), CT(0), CT(0)};
    collide<CT, false, Q>(mo, rho, ux, uy, uz, CT(1), S0, tau0, smag, g2);
  } else {
    CT d = CT(0);
    uint8_t tb = 0;
    if (valid) {
      d = a.d_eff[c];
      tb = a.tag[c];
    }
    const int t = tb & kTagMask;
    CT bx = CT(0), by = CT(0), bz = CT(0);
    const RotorTable& rt = *a.rot;
    int rk = -1;
    if (tb & kRotorBit) {
      rk = rt.tag2rot[t];
      const RotorDev& R = rt.r[rk];
      const double rx = x - R.c[0], ry = y - R.c[1], rz = z - R.c[2];
      bx = CT(R.omega * (R.e[1] * rz - R.e[2] * ry));
      by = CT(R.omega * (R.e[2] * rx - R.e[0] * rz));
      bz = CT(R.omega * (R.e[0] * ry - R.e[1] * rx));
    } else if (a.uB_static && valid) {
      bx = a.uB_static[c]; by = a.uB_static[g.N + c]; bz = a.uB_static[2 * g.N + c];
    }
    CT S[6] = {CT(0), CT(0), CT(0), CT(0), CT(0), CT(0)};
    CT sigma = CT(1);
    if (tb & kWallBit) {
      const RotorDev& R = rt.r[rk];
      const int64_t ws = R.off + (int64_t(z - R.b0[2]) * R.bn[1] + (y - R.b0[1])) * R.bn[0] + (x - R.b0[0]);
      const int64_t T = a.bbox_total;
      bx += a.wall_out[ws];
      by += a.wall_out[T + ws];
      bz += a.wall_out[2 * T + ws];
#pragma unroll
      for (int q = 0; q < 6; ++q) S[q] = a.wall_out[(3 + q) * T + ws];
      sigma = a.wall_out[9 * T + ws];
    }
    // hybrid non-equilibrium off the wall: element cells that are not
    // active wall cells take sigma = 1 - fd_share and the non-local strain
    if (!kMoments && a.fd_u && t != 0 && sigma == CT(1) && valid) {
      sigma = CT(1) - a.fd_share;
      fd_strain<CT, kPeriodicX>(g, FdField<CT>{a.fd_u, a.near_index}, x, y, z, S);
    }
    const CT hx = ux + d * (bx - ux), hy = uy + d * (by - uy), hz = uz + d * (bz - uz);
    if (kMoments) {
      if (valid) {
        a.out_rho[c] = rho;
        a.out_u[c] = ux; a.out_u[g.N + c] = uy; a.out_u[2 * g.N + c] = uz;
        if (a.out_uhat) { a.out_uhat[c] = hx; a.out_uhat[g.N + c] = hy; a.out_uhat[2 * g.N + c] = hz; }
      }
      return;
    }
    collide<CT, true, Q>(mo, rho, hx, hy, hz, sigma, S, tau0, smag, g2);
    // momentum handed to the solid and its torque, per tag (FP64)
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (t != 0 && valid) {
      const double px = double(mo.jx - rho * hx), py = double(mo.jy - rho * hy), pz = double(mo.jz - rho * hz);
      const double* fr = rt.frame[t];
      const double rx = x - fr[0], ry = y - fr[1], rz = z - fr[2];
      v[0] = px; v[1] = py; v[2] = pz;
      v[3] = ry * pz - rz * py;
      v[4] = rz * px - rx * pz;
      v[5] = rx * py - ry * px;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (!__syncthreads_or(t != 0 && valid)) {
      // no tagged cell in this tile: its partial is zero
      if (threadIdx.x < kPartial) a.partial[int64_t(slot) * kPartial + threadIdx.x] = 0.0;
    } else {
    for (int q = threadIdx.x; q < 4 * kPartial; q += kBlock) (&lds[0][0])[q] = 0.0;
    __syncthreads();
    const int tt = (t != 0 && valid) ? t : 0;
    uint64_t pending = __ballot(tt != 0);
    while (pending) {
      const int l0 = __ffsll((long long)pending) - 1;
      const int cur = __shfl(tt, l0, 64);
      const bool mine = tt == cur;
      double s6[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) s6[q] = wave_sum(mine ? v[q] : 0.0);
      if (lane == 0)
        for (int q = 0; q < 6; ++q) lds[wv][cur * 6 + q] = s6[q];
      pending &= ~__ballot(mine);
    }
    __syncthreads();
    if (threadIdx.x < kPartial) {
      const int q = threadIdx.x;
      a.partial[int64_t(slot) * kPartial + q] = (lds[0][q] + lds[1][q]) + (lds[2][q] + lds[3][q]);
    }
    }
  }
  if (!kMoments) {
    if (valid) {
      // this wave's block: contiguous, Q runs of kTileX cells
      // one scalar base per group of runs that the 12-bit immediate offset
      // of a store reaches (FP16 32 runs, FP32 16, FP64 8)
      constexpr int run = kTileX * sizeof(ST), per = 4096 / run;
      const gbytes p = (gbytes)(static_cast<ST*>(a.dst) + (int64_t(z) * g.ny + y) * g.row + int64_t(tx) * (Q * kTileX));
      const uint32_t o = uint32_t(x % kTileX) * uint32_t(sizeof(ST));
#pragma unroll
      for (int i0 = 0; i0 < Q; i0 += per) {
        gbytes q = p + int64_t(i0) * run;
        asm("" : "+s"(q));
#pragma unroll
        for (int i = i0; i < Q && i < i0 + per; ++i) Store<ST>::template store<CT>((ST*)(q + o + (i - i0) * run), g2[i]);
      }
    }
    // a non-finite density raises the flag (steps that check)
    if (a.flag && valid && !(rho == rho && fabs(double(rho)) < 1e300)) atomicOr(a.flag, 1);
    if (a.mass_part) {
      const double mrho = valid ? double(rho) : 0.0;
      const double ws = wave_sum(mrho);
      __syncthreads();
      if ((threadIdx.x & 63) == 0) lds[0][threadIdx.x >> 6] = ws;
      __syncthreads();
      if (threadIdx.x == 0) a.mass_part[ti.canon] = (lds[0][0] + lds[0][1]) + (lds[0][2] + lds[0][3]);
    }
  }
}

// Tile of workgroup i.  Consecutive workgroups are dispatched round-robin
// over the eight XCDs (i mod 8), each with its own L2: XCD k gets whole rows
// of ntx tiles, so the blocks that the x-shifted loads of neighbouring tiles
// share are fetched into one L2, while the eight XCDs sweep eight adjacent
// tile rows of the lattice at a time.  Workgroups past the last full group
// of eight rows keep lattice order.
__device__ __forceinline__ uint32_t tile_of(uint32_t i, const Geometry& g) {
  if (i >= g.grouped) return i;
  const uint32_t ntx = uint32_t(g.ntx);
  const uint32_t r = i - udiv(i, g.by_span) * (8u * ntx);
  return i - r + (r % 8u) * ntx + r / 8u;
}

template <class ST, class CT, bool kPeriodicX, bool kMoments, int Q>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs<CT> a) {
  __shared__ double lds[4][kPartial];
  const uint32_t blk = tile_of(blockIdx.x, a.g);
  sweep_tile<ST, CT, kPeriodicX, kMoments, Q>(a, blk, lds);
}

// Force / torque / mass reduction, level 1: workgroup (b, j) sums the force
// partials b, b + G, ... of step slice j and the mass partials of its chunk,
// in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_l1(const double* __restrict__ partial, int32_t nslots,
                                                   const double* __restrict__ mass_part, int64_t nmass, int64_t n0,
                                                   int32_t diag_every, double* __restrict__ l1,
                                                   double* __restrict__ ml1) {
  __shared__ double s[2][kPartial];
  __shared__ double sm[256];
  const int G = gridDim.x, b = blockIdx.x, j = blockIdx.y;
  const int64_t n = n0 + j;
  const bool diag = diag_every > 0 && n % diag_every == 0;
  const double* P = partial + int64_t(j) * (nslots > 0 ? nslots : 1) * kPartial;
  const double* M = mass_part + int64_t(j) * nmass;
  const int k = threadIdx.x % kPartial, r = threadIdx.x / kPartial;  // r in {0, 1, 2}; row 2 idle
  if (r < 2) {
    double acc = 0.0;
#pragma unroll 4
    for (int32_t sl = b + r * G; sl < nslots; sl += 2 * G) acc += P[int64_t(sl) * kPartial + k];
    s[r][k] = acc;
  }
  double macc = 0.0;
  if (diag) {
    const int64_t per = (nmass + G - 1) / G;
    const int64_t lo = int64_t(b) * per, hi = lo + per < nmass ? lo + per : nmass;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) macc += M[i];
  }
  sm[threadIdx.x] = macc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  double* L1 = l1 + (int64_t(j) * G + b) * kPartial;
  if (threadIdx.x < kPartial) L1[threadIdx.x] = s[0][threadIdx.x] + s[1][threadIdx.x];
  if (threadIdx.x == 0) ml1[int64_t(j) * G + b] = sm[0];
}

// Level 2: workgroup j adds the G level-1 results of slice j in order into
// the record of step n0 + j.
__global__ __launch_bounds__(256) void k_reduce_l2(const double* __restrict__ l1, const double* __restrict__ ml1,
                                                   int G, int64_t n0, int32_t diag_every, double* __restrict__ hist,
                                                   int64_t hist_cap) {
  __shared__ double s[2][kPartial];
  const int j = blockIdx.x;
  const int64_t n = n0 + j;
  const bool diag = diag_every > 0 && n % diag_every == 0;
  const double* L1 = l1 + int64_t(j) * G * kPartial;
  const double* M1 = ml1 + int64_t(j) * G;
  double* rec = hist + (n % hist_cap) * kHist;
  const int k = threadIdx.x % kPartial, r = threadIdx.x / kPartial;
  if (r < 2) {
    double acc = 0.0;
#pragma unroll 4
    for (int q = r; q < G; q += 2) acc += L1[int64_t(q) * kPartial + k];
    s[r][k] = acc;
  }
  __syncthreads();
  if (threadIdx.x >= 6 && threadIdx.x < kPartial) rec[1 + threadIdx.x - 6] = s[0][threadIdx.x] + s[1][threadIdx.x];
  if (threadIdx.x == 255) {
    if (diag) {
      double acc = 0.0;
      for (int q = 0; q < G; ++q) acc += M1[q];
      rec[0] = acc;
    } else {
      rec[0] = __builtin_nan("");
    }
  }
}

// ---------------------------------------------------------------- finite-difference strain
// Pre-collision velocity u = j / rho of the cells of each listed tile (the
// FSI tiles and their neighbours) into fd_u, for the strain of the sweep.
template <class ST, class CT, bool kPeriodicX, int Q>
__global__ __launch_bounds__(kBlock) void k_fd_velocity(const ST* __restrict__ src, Geometry g,
                                                        const CT* __restrict__ ghost,
                                                        const int32_t* __restrict__ tiles, CT* __restrict__ fd_u) {
  const uint32_t canon = uint32_t(tiles[blockIdx.x]);
  const uint32_t ntx = uint32_t(g.ntx), tpz = ntx * uint32_t(g.nty);
  const int z = int(canon / tpz);
  const uint32_t rem = canon - uint32_t(z) * tpz;
  const int ty = int(rem / ntx), tx = int(rem - uint32_t(ty) * ntx);
  const int xr = tx * kTileX + int(threadIdx.x & (kTileX - 1));
  const int yr = __builtin_amdgcn_readfirstlane(ty * kTileY + int(threadIdx.x >> 6));
  const bool row_ok = yr < g.ny;
  const int x = xr < g.nx && row_ok ? xr : 0, y = row_ok ? yr : 0;
  CT h[Q];
  pull_row<ST, CT, kPeriodicX, Q>(src, g, x, y, z, ghost, h);
  const Moments<CT> mo = moments_q<Q, CT>(h);
  const CT irho = rcp_ct(CT(1) + mo.drho);
  CT* o = fd_u + int64_t(blockIdx.x) * 3 * kBlock + threadIdx.x;
  o[0] = mo.jx * irho;
  o[kBlock] = mo.jy * irho;
  o[2 * kBlock] = mo.jz * irho;
}

// ---------------------------------------------------------------- momentum exchange
// Solid velocity of a cell with tag byte tb: rigid rotation of its rotor,
// else the static solid velocity (if any), else zero.
template <class CT>
__device__ __forceinline__ void solid_velocity(const RotorTable& rt, uint8_t tb, const CT* uB_static, int64_t N,
                                               int64_t c, int x, int y, int z, double u[3]) {
  if (tb & kRotorBit) {
    const RotorDev& R = rt.r[rt.tag2rot[tb & kTagMask]];
    const double rx = x - R.c[0], ry = y - R.c[1], rz = z - R.c[2];
    u[0] = R.omega * (R.e[1] * rz - R.e[2] * ry);
    u[1] = R.omega * (R.e[2] * rx - R.e[0] * rz);
    u[2] = R.omega * (R.e[0] * ry - R.e[1] * rx);
  } else if (uB_static) {
    u[0] = double(uB_static[c]);
    u[1] = double(uB_static[N + c]);
    u[2] = double(uB_static[2 * N + c]);
  } else {
    u[0] = u[1] = u[2] = 0.0;
  }
}

template <class CT>
struct MeArgs {
  const void* state;         // post-collision populations of the step
  Geometry g;
  const uint8_t* tag;        // tags of the step
  const RotorTable* rot;
  const CT* uB_static;       // nullable
  const int32_t* fsi_tiles;  // lattice-order tile of each slot
  double* partial;           // [slot][kMePartial]
};

// Momentum-exchange force of the step (Sec. 2.2.2, per link between a tag-0
// cell and a cell of an element, Galilean-invariant form), one workgroup per
// tile of the list (FSI tiles and their neighbours): each cell adds the terms of its own post-collision populations
// on its links -- an element's cell (c_i of the link pointing out of the
// element) (u_s - c_i) f*_i, a tag-0 cell (c_i pointing into the element)
// (c_i - u_s(x + c_i)) f*_i -- and the tile reduces them per tag in FP64.
template <class ST, class CT, bool kPeriodicX, int Q>
__global__ __launch_bounds__(kBlock) void k_momentum_exchange(MeArgs<CT> a) {
  __shared__ double lds[4][kMePartial];
  const Geometry& g = a.g;
  const int32_t slot = blockIdx.x;
  const uint32_t canon = uint32_t(a.fsi_tiles[slot]);
  const uint32_t ntx = uint32_t(g.ntx), tpz = ntx * uint32_t(g.nty);
  const int z = int(canon / tpz);
  const uint32_t rem = canon - uint32_t(z) * tpz;
  const int ty = int(rem / ntx), tx = int(rem - uint32_t(ty) * ntx);
  const int x = tx * kTileX + int(threadIdx.x & (kTileX - 1));
  const int y = ty * kTileY + int(threadIdx.x >> 6);
  const bool valid = x < g.nx && y < g.ny;
  const RotorTable& rt = *a.rot;
  const ST* __restrict__ st = static_cast<const ST*>(a.state);
  double acc[3] = {0.0, 0.0, 0.0};
  int tme = 0;
  if (valid) {
    const int64_t c = (int64_t(z) * g.ny + y) * g.nx + x;
    const uint8_t tb = a.tag[c];
    const int t = tb & kTagMask;
    tme = t;
    double us[3] = {0.0, 0.0, 0.0};
    if (t != 0) solid_velocity<CT>(rt, tb, a.uB_static, g.N, c, x, y, z, us);
    static_for<Q>([&](auto I) {
      constexpr int i = I;
      constexpr int cx = cxq<Q>(i), cy = cyq<Q>(i), cz = czq<Q>(i);
      if constexpr (cx != 0 || cy != 0 || cz != 0) {
        int xn = x + cx;
        const int yn = wrapi(y + cy, g.ny), zn = wrapi(z + cz, g.nz);
        bool in = true;
        if (kPeriodicX) xn = wrapi(xn, g.nx);
        else in = xn >= 0 && xn < g.nx;
        if (in) {
          const int64_t cn = (int64_t(zn) * g.ny + yn) * g.nx + xn;
          const uint8_t tbn = a.tag[cn];
          const int tn = tbn & kTagMask;
          if ((t != 0 && tn == 0) || (t == 0 && tn != 0 && (tme == 0 || tn == tme))) {
            const double f = wq<Q>(i) * (1.0 + Store<ST>::template load<double>(st + pop_at<Q>(g, i, x, y, z)));
            if (t != 0) {
              acc[0] += (us[0] - cx) * f;
              acc[1] += (us[1] - cy) * f;
              acc[2] += (us[2] - cz) * f;
            } else {
              tme = tn;
              double un[3];
              solid_velocity<CT>(rt, tbn, a.uB_static, g.N, cn, xn, yn, zn, un);
              acc[0] += (cx - un[0]) * f;
              acc[1] += (cy - un[1]) * f;
              acc[2] += (cz - un[2]) * f;
            }
          }
        }
      }
    });
  }
  // per-tag sums over the tile in a fixed order: waves by ballot, then LDS
  for (int q = threadIdx.x; q < 4 * kMePartial; q += kBlock) (&lds[0][0])[q] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t pending = __ballot(tme != 0);
  while (pending) {
    const int l0 = __ffsll((long long)pending) - 1;
    const int cur = __shfl(tme, l0, 64);
    const bool mine = tme == cur;
    double s3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) s3[k] = wave_sum(mine ? acc[k] : 0.0);
    if (lane == 0)
      for (int k = 0; k < 3; ++k) lds[wv][cur * 3 + k] = s3[k];
    pending &= ~__ballot(mine);
  }
  __syncthreads();
  if (threadIdx.x < kMePartial) {
    const int q = threadIdx.x;
    a.partial[int64_t(slot) * kMePartial + q] = (lds[0][q] + lds[1][q]) + (lds[2][q] + lds[3][q]);
  }
}

// Momentum-exchange reduction, level 1: workgroup (b, j) sums the partials
// b, b + G, ... of step slice j (five rows of slots, then the rows in order).
__global__ __launch_bounds__(256) void k_reduce_me_l1(const double* __restrict__ partial, int32_t nslots,
                                                      double* __restrict__ l1) {
  __shared__ double s[5][kMePartial];
  const int G = gridDim.x, b = blockIdx.x, j = blockIdx.y;
  const double* P = partial + int64_t(j) * (nslots > 0 ? nslots : 1) * kMePartial;
  const int k = threadIdx.x % kMePartial, r = threadIdx.x / kMePartial;  // r in 0..5; row 5 idle
  if (r < 5) {
    double acc = 0.0;
    for (int32_t sl = b + r * G; sl < nslots; sl += 5 * G) acc += P[int64_t(sl) * kMePartial + k];
    s[r][k] = acc;
  }
  __syncthreads();
  if (threadIdx.x < kMePartial)
    l1[(int64_t(j) * G + b) * kMePartial + threadIdx.x] =
        (((s[0][threadIdx.x] + s[1][threadIdx.x]) + s[2][threadIdx.x]) + s[3][threadIdx.x]) + s[4][threadIdx.x];
}

// Level 2: workgroup j adds the G level-1 results of slice j in order into
// the momentum-exchange record of step n0 + j (tags 1..15).
__global__ __launch_bounds__(64) void k_reduce_me_l2(const double* __restrict__ l1, int G, int64_t n0,
                                                     double* __restrict__ hist_me, int64_t hist_cap) {
  const int j = blockIdx.x, k = threadIdx.x;
  if (k < 3 || k >= kMePartial) return;
  double acc = 0.0;
  for (int q = 0; q < G; ++q) acc += l1[(int64_t(j) * G + q) * kMePartial + k];
  hist_me[((n0 + j) % hist_cap) * kHistMe + (k - 3)] = acc;
}

// ---------------------------------------------------------------- state I/O
template <class ST, class CT, int Q>
__global__ __launch_bounds__(256) void k_init_eq(ST* __restrict__ dst, Geometry g, const CT* __restrict__ rho,
                                                 const CT* __restrict__ u) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const CT r = rho ? rho[c] : CT(1);
  const CT ux = u ? u[c] : CT(0), uy = u ? u[g.N + c] : CT(0), uz = u ? u[2 * g.N + c] : CT(0);
  CT ge[Q];
  equilibrium_dev<CT, Q>(r, ux, uy, uz, ge);
  const int x = int(c % g.nx), y = int((c / g.nx) % g.ny), z = int(c / (int64_t(g.nx) * g.ny));
#pragma unroll
  for (int i = 0; i < Q; ++i) Store<ST>::template store<CT>(dst + pop_at<Q>(g, i, x, y, z), ge[i]);
}

template <class ST, int Q>
__global__ __launch_bounds__(256) void k_get_pop(const ST* __restrict__ src, Geometry g, double* __restrict__ dst) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = int(c % g.nx), y = int((c / g.nx) % g.ny), z = int(c / (int64_t(g.nx) * g.ny));
  static_for<Q>([&](auto I) {
    constexpr int i = I;
    dst[int64_t(i) * g.N + c] = wq<Q>(i) * Store<ST>::template load<double>(src + pop_at<Q>(g, i, x, y, z));
  });
}

template <class ST, int Q>
__global__ __launch_bounds__(256) void k_set_pop(ST* __restrict__ dst, Geometry g, const double* __restrict__ src) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = int(c % g.nx), y = int((c / g.nx) % g.ny), z = int(c / (int64_t(g.nx) * g.ny));
  static_for<Q>([&](auto I) {
    constexpr int i = I;
    Store<ST>::template store<double>(dst + pop_at<Q>(g, i, x, y, z), src[int64_t(i) * g.N + c] / wq<Q>(i));
  });
}

template <class ST, int Q>
__global__ __launch_bounds__(256) void k_get_pop_at(const ST* __restrict__ src, Geometry g,
                                                    const int64_t* __restrict__ cells, int64_t count,
                                                    double* __restrict__ dst) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int64_t c = cells[k];
  if (c < 0 || c >= g.N) {
    for (int i = 0; i < Q; ++i) dst[k * Q + i] = __builtin_nan("");
    return;
  }
  const int x = int(c % g.nx), y = int((c / g.nx) % g.ny), z = int(c / (int64_t(g.nx) * g.ny));
  static_for<Q>([&](auto I) {
    constexpr int i = I;
    dst[k * Q + i] = wq<Q>(i) * Store<ST>::template load<double>(src + pop_at<Q>(g, i, x, y, z));
  });
}

// Every element of a population buffer (cells and the unused tail of the
// last block of each row) set to the rest state g = 0.
template <class ST>
__global__ __launch_bounds__(256) void k_fill_rest(ST* __restrict__ dst, int64_t count) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < count) Store<ST>::template store<double>(dst + e, 0.0);
}

// FSI workgroups (bit 0): any cell in a rotor box, or with static porosity,
// tag or control.  Reach workgroups (bit 1): within the wall model's probe
// stencil around a rotor box (periodic in y, z); they run the plain path but
// are swept after the wall model, and the adjoint gathers probe adjoints there.
template <class CT>
__global__ __launch_bounds__(256) void k_mark(const RotorTable* __restrict__ rtp, Geometry g,
                                              const CT* __restrict__ d_static, const uint8_t* __restrict__ tag_static,
                                              const CT* __restrict__ dd, int32_t* __restrict__ blk) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int64_t nxy = int64_t(g.nx) * g.ny;
  const int z = int(c / nxy);
  const int64_t r = c - int64_t(z) * nxy;
  const int y = int(r / g.nx), x = int(r - int64_t(y) * g.nx);
  bool fsi = d_static[c] != CT(0) || tag_static[c] != 0 || (dd && dd[c] != CT(0));
  bool reach = false;
  const RotorTable& rt = *rtp;
  for (int j = 0; j < rt.n; ++j) {
    const RotorDev& rr = rt.r[j];
    fsi = fsi || in_box(rr, x, y, z);
    const int lx = x - rr.mb0[0];
    const int ly = ((y - rr.mb0[1]) % g.ny + g.ny) % g.ny, lz = ((z - rr.mb0[2]) % g.nz + g.nz) % g.nz;
    const bool inx = g.bc_x == 0 ? (((lx % g.nx) + g.nx) % g.nx < rr.mbn[0] || rr.mbn[0] >= g.nx)
                                 : (lx >= 0 && lx < rr.mbn[0]);
    reach = reach || (inx && (ly < rr.mbn[1] || rr.mbn[1] >= g.ny) && (lz < rr.mbn[2] || rr.mbn[2] >= g.nz));
  }
  const int bits = (fsi ? 1 : 0) | (reach ? 2 : 0);
  if (bits) atomicOr(&blk[(int64_t(z) * g.nty + y / kTileY) * g.ntx + x / kTileX], bits);
}

// d_eff = d_static + control everywhere (rotor boxes are overwritten each step),
// tag = static tag.
template <class CT>
__global__ __launch_bounds__(256) void k_refill(Geometry g, const CT* __restrict__ d_static,
                                                const uint8_t* __restrict__ tag_static, const CT* __restrict__ dd,
                                                CT* __restrict__ d_eff, uint8_t* __restrict__ tag) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  d_eff[c] = d_static[c] + (dd ? dd[c] : CT(0));
  tag[c] = tag_static[c];
}


// ================================================================ adjoint
// Reverse of step n (discrete adjoint).  The state adjoint lam is the
// derivative of the objective with respect to the stored post-collision
// populations f*_i (not the normalized deviations), in compute type.
template <class CT>
struct AdjArgs {
  const void* src;          // state at step n (storage type)
  const CT* lam_in;         // adjoint of the state after step n (blocked layout)
  CT* lam_out;              // adjoint of the state at step n (blocked layout)
  CT* side;                 // outflow side buffer of this step [9][nz][ny]
  const CT* side_in;        // that of the next step, nullable: see k_adj_sweep
  Geometry g;
  Model m;
  const int32_t* blk_slot;
  const CT* d_eff;
  const uint8_t* tag;
  const CT* wall_out;
  int64_t bbox_total;
  const RotorTable* rot;
  const CT* uB_static;
  const CT* ghost;
  unsigned long long* ubar; // probe-velocity adjoints scattered by the wall cells (fixed point); zeroed here
  double* G;                // dJ/d(delta_d), accumulated
  double obj_w;             // weight of this step's torque in J (0 outside the window)
  int32_t obj_tag;
  int64_t nblocks;
  double* zero;             // zeroed by the workgroups past nblocks
  int64_t nzero;
  // finite-difference strain of the step (nullable fd_u: off)
  const CT* fd_u;
  const int32_t* near_index;
  CT fd_share;
  const int32_t* tiles;     // the FSI tiles and their neighbours
  int32_t* flag;
};

// Homogenization inputs of an FSI cell: porosity, b = u^B + u_wm, S, sigma.
template <class CT>
__device__ __forceinline__ void fsi_inputs(const AdjArgs<CT>& a, const RotorTable& rt, int64_t c, int x, int y, int z,
                                           uint8_t tb, CT& d, CT b[3], CT S[6], CT& sigma) {
  d = a.d_eff[c];
  b[0] = b[1] = b[2] = CT(0);
  for (int q = 0; q < 6; ++q) S[q] = CT(0);
  sigma = CT(1);
  const int t = tb & kTagMask;
  if (tb & kRotorBit) {
    const RotorDev& R = rt.r[rt.tag2rot[t]];
    const double rx = x - R.c[0], ry = y - R.c[1], rz = z - R.c[2];
    b[0] = CT(R.omega * (R.e[1] * rz - R.e[2] * ry));
    b[1] = CT(R.omega * (R.e[2] * rx - R.e[0] * rz));
    b[2] = CT(R.omega * (R.e[0] * ry - R.e[1] * rx));
    if (tb & kWallBit) {
      const int64_t ws = R.off + (int64_t(z - R.b0[2]) * R.bn[1] + (y - R.b0[1])) * R.bn[0] + (x - R.b0[0]);
      const int64_t T = a.bbox_total;
      b[0] += a.wall_out[ws];
      b[1] += a.wall_out[T + ws];
      b[2] += a.wall_out[2 * T + ws];
      for (int q = 0; q < 6; ++q) S[q] = a.wall_out[(3 + q) * T + ws];
      sigma = a.wall_out[9 * T + ws];
    }
  } else if (a.uB_static) {
    b[0] = a.uB_static[c]; b[1] = a.uB_static[a.g.N + c]; b[2] = a.uB_static[2 * a.g.N + c];
  }
}

// Local part of a reverse step at cell (x, y, z) (index c): the moments of
// the state and the collision VJP from the adjoint of the next state at the
// cell (with the outflow share on the last plane), under the FSI inputs of
// the forward step when the tile is an FSI tile.  Returns whether the cell
// took the finite-difference strain (sigma = 1 - fd_share): the element
// cells that are not active wall cells.
template <class ST, class CT, bool kPeriodicX, int Q>
__device__ __forceinline__ bool adj_local(const AdjArgs<CT>& a, int x, int y, int z, int64_t c, bool fsi,
                                          Moments<CT>& mo, Moments<CT>& mb, CT& db, CT Sb[6]) {
  const Geometry& g = a.g;
  CT h[Q];
  pull_row<ST, CT, kPeriodicX, Q>(static_cast<const ST*>(a.src), g, x, y, z, a.ghost, h);
  mo = moments_q<Q, CT>(h);
  // lam in the blocked layout of the populations: this wave's block
  constexpr uint32_t cs = sizeof(CT);
  const uint64_t rs = uint64_t(g.row) * cs;
  const uint32_t o4 = pop_x<Q>(x) * cs;
  CT gb[Q];
  {
    typedef __attribute__((address_space(1))) const char* gcb;
    gcb q = (gcb)a.lam_in + (uint64_t(z) * g.ny + y) * rs;
#pragma unroll
    for (int i = 0; i < Q; ++i) gb[i] = *(const CT*)(q + (o4 + uint32_t(i * kTileX) * cs));
  }
  if (!kPeriodicX && a.side_in && x == g.nx - 1) {
    const int64_t k = int64_t(z) * g.ny + y, plane = int64_t(g.ny) * g.nz;
    for (int i = 0; i < xgroup_of<Q>(1); ++i) gb[i] += a.side_in[i * plane + k];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) gb[i] *= CT(wq<Q>(i));
  CT d = CT(0), b[3] = {CT(0), CT(0), CT(0)}, S[6] = {CT(0), CT(0), CT(0), CT(0), CT(0), CT(0)}, sigma = CT(1);
  CT pb[3] = {CT(0), CT(0), CT(0)};
  bool fd = false;
  if (fsi) {
    const RotorTable& rt = *a.rot;
    const uint8_t tb = a.tag[c];
    fsi_inputs(a, rt, c, x, y, z, tb, d, b, S, sigma);
    if (a.fd_u && (tb & kTagMask) != 0 && sigma == CT(1)) {
      sigma = CT(1) - a.fd_share;
      fd_strain<CT, kPeriodicX>(g, FdField<CT>{a.fd_u, a.near_index}, x, y, z, S);
      fd = true;
    }
    objective_dp<CT>(rt, tb & kTagMask, a.obj_tag, a.obj_w, x, y, z, pb);
  } else if (a.uB_static) {
    b[0] = a.uB_static[c]; b[1] = a.uB_static[g.N + c]; b[2] = a.uB_static[2 * g.N + c];
  }
  CT bb[3];
  collide_vjp<CT, Q>(mo, d, b[0], b[1], b[2], sigma, S, CT(a.m.tau0), CT(a.m.smag), gb, pb, mb, db, bb, Sb);
  return fd;
}

// Velocity adjoints of the finite-difference strain, one workgroup per
// listed tile (the FSI tiles and their neighbours; the neighbours exit).  At
// a cell that took the strain, the collision VJP gives the adjoint of S;
// S_ab = (d_a u_b + d_b u_a) / 2 with d_b u_a = (u_a(x + e_b) - u_a(x - e_b))
// / 2 hands it to the pre-collision velocities of the six neighbours, summed
// in fixed point with the probe-velocity adjoints; the adjoint sweep of the
// step gathers them.
template <class ST, class CT, bool kPeriodicX, int Q>
__global__ __launch_bounds__(kBlock) void k_adj_fd(AdjArgs<CT> a) {
  const Geometry& g = a.g;
  const uint32_t canon = uint32_t(a.tiles[blockIdx.x]);
  if (a.blk_slot[canon] < 0) return;
  const uint32_t ntx = uint32_t(g.ntx), tpz = ntx * uint32_t(g.nty);
  const int z = int(canon / tpz);
  const uint32_t rem = canon - uint32_t(z) * tpz;
  const int ty = int(rem / ntx), tx = int(rem - uint32_t(ty) * ntx);
  const int xr = tx * kTileX + int(threadIdx.x & (kTileX - 1));
  const int yr = __builtin_amdgcn_readfirstlane(ty * kTileY + int(threadIdx.x >> 6));
  if (xr >= g.nx || yr >= g.ny) return;
  const int x = xr, y = yr;
  const int64_t c = (int64_t(z) * g.ny + y) * g.nx + x;
  if ((a.tag[c] & kTagMask) == 0) return;
  Moments<CT> mo, mb;
  CT db, Sb[6];
  if (!adj_local<ST, CT, kPeriodicX, Q>(a, x, y, z, c, true, mo, mb, db, Sb)) return;
  int xm, xp, ym, yp, zm, zp;
  fd_stencil<kPeriodicX>(g, x, y, z, xm, xp, ym, yp, zm, zp);
  const int64_t cp[3] = {(int64_t(z) * g.ny + y) * g.nx + xp, (int64_t(z) * g.ny + yp) * g.nx + x,
                         (int64_t(zp) * g.ny + y) * g.nx + x};
  const int64_t cm[3] = {(int64_t(z) * g.ny + y) * g.nx + xm, (int64_t(z) * g.ny + ym) * g.nx + x,
                         (int64_t(zm) * g.ny + y) * g.nx + x};
  // adjoint of d_b u_a: S_aa = d_a u_a, S_ab = (d_b u_a + d_a u_b) / 2
  const double s0 = double(Sb[0]), s1 = double(Sb[1]), s2 = double(Sb[2]);
  const double s3 = 0.5 * double(Sb[3]), s4 = 0.5 * double(Sb[4]), s5 = 0.5 * double(Sb[5]);
  const double dbar[3][3] = {{s0, s3, s4}, {s3, s1, s5}, {s4, s5, s2}};
  for (int q = 0; q < 3; ++q)
    for (int e = 0; e < 3; ++e) {
      const double v = 0.5 * dbar[q][e];
      if (v == 0.0) continue;
      fix_add(a.ubar, g.N, cp[e], q, v, a.flag);
      fix_add(a.ubar, g.N, cm[e], q, -v, a.flag);
    }
}

// Adjoint sweep over all cells: collision VJP from the local adjoint of the
// next state, the probe-velocity adjoints gathered from the wall cells (and
// from the finite-difference strain), and the transpose of the pull
// (lam_out_i(x - c_i) = mu_i(x)).  Outflow: the state at (nx-1, y', z') with
// c_x = -1 is read by (nx-2, .) and by the clamped read of (nx-1, .); the
// second share goes to `side`, and the reader of lam (this sweep of the
// previous step, and the adjoint wall step) adds it on the last plane.
// Workgroups past nblocks zero `zero`.
template <class ST, class CT, bool kPeriodicX, int Q = 27>
__global__ __launch_bounds__(kBlock) void k_adj_sweep(AdjArgs<CT> a) {
  const Geometry& g = a.g;
  if (int64_t(blockIdx.x) >= a.nblocks) {
    const int64_t k = (int64_t(blockIdx.x) - a.nblocks) * kBlock + threadIdx.x;
    if (k < a.nzero) a.zero[k] = 0.0;
    return;
  }
  const uint32_t blk = tile_of(blockIdx.x, g);
  const TileId ti = tile_id(g, blk);
  const int z = ti.z, ty = ti.ty, tx = ti.tx;
  const int xr = tx * kTileX + int(threadIdx.x & (kTileX - 1));
  // one row per wave: y is uniform over the wave
  const int yr = __builtin_amdgcn_readfirstlane(ty * kTileY + int(threadIdx.x >> 6));
  if (xr >= g.nx || yr >= g.ny) return;
  const int x = xr, y = yr;
  const int64_t c = (int64_t(z) * g.ny + y) * g.nx + x;
  double ub[3] = {0.0, 0.0, 0.0};
  const int32_t slot = a.blk_slot[ti.canon];
  const bool fsi = slot >= 0, gather = slot != -1;
  if (gather) {
    for (int q = 0; q < 3; ++q) {
      ub[q] = fix_take(a.ubar, g.N, c, q);
    }
  }
  Moments<CT> mo, mb;
  CT db, Sb[6];
  (void)adj_local<ST, CT, kPeriodicX, Q>(a, x, y, z, c, fsi, mo, mb, db, Sb);
  if (gather) {
    // velocity u = j / rho at this cell, sampled by wall-cell probes and
    // by the finite-difference strain of its neighbours
    const CT rho = CT(1) + mo.drho, irho = rcp_ct(rho);
    const CT ju = CT(ub[0]) * mo.jx + CT(ub[1]) * mo.jy + CT(ub[2]) * mo.jz;
    mb.drho -= ju * irho * irho;
    mb.jx += CT(ub[0]) * irho;
    mb.jy += CT(ub[1]) * irho;
    mb.jz += CT(ub[2]) * irho;
  }
  constexpr uint32_t cs = sizeof(CT);
  const uint64_t rs = uint64_t(g.row) * cs;
  a.G[c] += double(db);
  // transpose of the pull: the state read by f_i(x) is at x - c_i
  const int zp = z + 1 == g.nz ? 0 : z + 1, zm = z == 0 ? g.nz - 1 : z - 1;
  const int yp = y + 1 == g.ny ? 0 : y + 1, ym = y == 0 ? g.ny - 1 : y - 1;
  int xp, xm;
  if (kPeriodicX) {
    xp = x + 1 == g.nx ? 0 : x + 1;
    xm = x == 0 ? g.nx - 1 : x - 1;
  } else {
    xp = x + 1 == g.nx ? x : x + 1;
    xm = x == 0 ? 0 : x - 1;
  }
  const uint64_t rz[3] = {uint64_t(zp) * g.ny, uint64_t(z) * g.ny, uint64_t(zm) * g.ny};
  const uint32_t ry[3] = {uint32_t(yp), uint32_t(y), uint32_t(ym)};
  const uint32_t ox[3] = {pop_x<Q>(xp) * cs, pop_x<Q>(x) * cs, pop_x<Q>(xm) * cs};
  const int64_t plane = int64_t(g.ny) * g.nz;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = cxq<Q>(i), cy = cyq<Q>(i), cz = czq<Q>(i);
    const CT mu = mb.drho + CT(cx) * mb.jx + CT(cy) * mb.jy + CT(cz) * mb.jz + CT(cx * cx) * mb.pxx +
                  CT(cy * cy) * mb.pyy + CT(cz * cz) * mb.pzz + CT(cx * cy) * mb.pxy + CT(cx * cz) * mb.pxz +
                  CT(cy * cz) * mb.pyz;
    typedef __attribute__((address_space(1))) char* gb_t;
    gb_t base = (gb_t)a.lam_out + ((rz[cz + 1] + ry[cy + 1]) * rs + uint64_t(i * kTileX) * cs);
    if (!kPeriodicX) {
      if (cx == 1 && x == 0) {
        continue;  // read the inflow ghost, not the state
      }
      if (cx == -1 && x == g.nx - 1) {
        // clamped outflow read of (nx-1, y - cy, z - cz): also read by (nx-2, ...)
        a.side[(i) * plane + int64_t(zp * (cz == -1) + z * (cz == 0) + zm * (cz == 1)) * g.ny +
               (yp * (cy == -1) + y * (cy == 0) + ym * (cy == 1))] = mu;
        continue;
      }
    }
    *(CT*)(base + ox[cx + 1]) = mu;
  }
  if (!kPeriodicX) {
    // states nobody reads: (nx-1, *) for c_x = +1 and (0, *) for c_x = -1
    if (x == g.nx - 1)
      for (int i = xgroup_of<Q>(2); i < Q; ++i) a.lam_out[pop_at<Q>(g, i, x, y, z)] = CT(0);
    if (x == 0)
      for (int i = 0; i < xgroup_of<Q>(1); ++i) a.lam_out[pop_at<Q>(g, i, x, y, z)] = CT(0);
  }
}

// ================================================================ static workspace
// Device memory of the lattices created by hlbm_lattice_create_static.  In
// host code the array's name is not a device address: kernels and copies get
// the address that hipGetSymbolAddress returns on each device.
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

hipError_t static_workspace(void** ptr) {
  constexpr int kDevices = 64;
  static void* addr[kDevices] = {};
  static std::mutex lock;
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(lock);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// ================================================================ launchers
static inline dim3 grid1(int64_t n, int b) { return dim3(unsigned((n + b - 1) / b)); }

template <class F>
static hipError_t by_types(int storage, int compute, F&& f) {
  if (compute == 0 && storage == 0) return f((double*)nullptr, (double*)nullptr);
  if (compute == 1 && storage == 1) return f((float*)nullptr, (float*)nullptr);
  if (compute == 1 && storage == 2) return f((_Float16*)nullptr, (float*)nullptr);
  if (compute == 1 && storage == 3) return f((bf16_t*)nullptr, (float*)nullptr);
  return hipErrorInvalidValue;
}

// f(integral_constant<int, Q>) for the lattice's velocity set.
template <class F>
static hipError_t by_q(int q, F&& f) {
  if (q == 19) return f(std::integral_constant<int, 19>{});
  return f(std::integral_constant<int, 27>{});
}

template <class F>
static hipError_t by_compute(int compute, F&& f) {
  if (compute == 0) return f((double*)nullptr);
  if (compute == 1) return f((float*)nullptr);
  return hipErrorInvalidValue;
}

// Arguments of the geometry launch of `step` and its workgroup count.
template <class CT>
static GeoArgs<CT> geo_args(const Launch& L, int64_t step, const BladeTrig* trig, int epoch, uint8_t* act_new,
                            bool with_ghost, int64_t* blocks) {
  const int64_t nbw = L.nrot > 0 ? (L.bbox_total + 255) / 256 : 0;
  const int64_t plane = int64_t(L.g.ny) * L.g.nz;
  const int64_t nghost = (with_ghost && L.g.bc_x != 0) ? (plane + 255) / 256 : 0;
  GeoArgs<CT> a{};
  a.rot = L.rot; a.g = L.g; a.m = L.m; a.trig = trig; a.total = nbw > 0 ? L.bbox_total : 0;
  a.d_static = (const CT*)L.d_static; a.tag_static = L.tag_static; a.dd = (const CT*)L.dd;
  a.d_eff = (CT*)L.d_eff; a.tag = L.tag; a.geo = L.geo; a.act_new = act_new; a.wlist = L.wlist;
  a.wcount = L.wcount + epoch % kCounters; a.wcount_next = L.wcount + (epoch + 1) % kCounters;
  a.step = step; a.ghost = (CT*)L.ghost;
  // the wall model samples in FP64: also fill the FP64 plane when it differs
  a.ghost64 = (L.compute != 0 && L.nrot > 0) ? L.ghost64 : nullptr;
  a.ghost_blocks = int32_t(nghost);
  a.gstats = L.gstats;
  if (L.gmark && nbw > 0) {
    // two mark arrays by step parity: a launch reads the marks of the
    // previous step's launch and writes those of the next step
    a.mark_in = L.guse ? L.gmark + (step & 1) * L.bbox_total : nullptr;
    a.mark_out = L.gmark + ((step + 1) & 1) * L.bbox_total;
    a.key = (L.ggen << 40) | (long long)(step & ((1ll << 40) - 1));
    a.mark_cut = 0.5 * L.m.eps_h + 1.0;
  }
  *blocks = nbw + nghost;
  return a;
}

hipError_t launch_geometry(const Launch& L, int64_t step, const BladeTrig* trig, int epoch, uint8_t* act_new,
                           bool with_ghost) {
  return by_compute(L.compute, [&](auto* ct) {
    using CT = std::remove_pointer_t<decltype(ct)>;
    int64_t blocks = 0;
    const GeoArgs<CT> a = geo_args<CT>(L, step, trig, epoch, act_new, with_ghost, &blocks);
    if (blocks == 0) return hipSuccess;
    return by_q(L.q, [&](auto QC) {
      hipLaunchKernelGGL((k_geometry<CT, QC.value>), dim3(unsigned(blocks)), dim3(256), 0, L.stream, a);
      return hipGetLastError();
    });
  });
}

hipError_t launch_wall(const Launch& L, const void* src, const double* ut_prev, const uint8_t* act_prev,
                       double* ut_new, uint8_t* act_new, int epoch, const AdjLaunch* adj, int count_stats,
                       const NextGeometry* next) {
  if (L.nrot == 0 || L.bbox_total == 0) {
    if (!next) return hipSuccess;
    return launch_geometry(*next->L, next->step, next->trig, next->epoch, next->act_new, next->with_ghost);
  }
  // persistent grid over the (device-side) wall-cell count, 32 cells per workgroup
  int64_t wall_blocks = (L.bbox_total + 31) / 32;
  if (wall_blocks > 1024) wall_blocks = 1024;
  return by_types(L.storage, L.compute, [&](auto* st, auto* ct) {
    using ST = std::remove_pointer_t<decltype(st)>;
    using CT = std::remove_pointer_t<decltype(ct)>;
    WallArgs<CT> w{};
    w.rot = L.rot; w.g = L.g; w.m = L.m; w.total = L.bbox_total; w.src = src; w.geo = L.geo; w.wlist = L.wlist;
    w.wcount = L.wcount + epoch % kCounters; w.ut_prev = ut_prev; w.act_prev = act_prev; w.ut_new = ut_new;
    w.act_new = act_new; w.wall_out = (CT*)L.wall_out; w.stats = L.stats; w.ghost = L.ghost64;
    w.count_stats = count_stats;
    if (adj) {
      w.lam_in = (const CT*)adj->lam_in; w.side_in = (const CT*)adj->side_in;
      w.d_eff = (const CT*)L.d_eff; w.tag = L.tag; w.ghost_ct = (const CT*)L.ghost;
      w.ut_bar_in = adj->ut_bar_in; w.ut_bar_out = adj->ut_bar_out; w.ubar = adj->ubar; w.flag = L.flag;
      w.obj_w = adj->obj_w; w.obj_tag = adj->obj_tag;
    }
    int64_t geo_blocks = 0;
    GeoArgs<CT> ga{};
    if (next)
      ga = geo_args<CT>(*next->L, next->step, next->trig, next->epoch, next->act_new, next->with_ghost, &geo_blocks);
    auto go = [&](auto wall_kernel, auto fused_kernel) {
      if (geo_blocks == 0)
        hipLaunchKernelGGL(wall_kernel, dim3(unsigned(wall_blocks)), dim3(256), 0, L.stream, w);
      else
        hipLaunchKernelGGL(fused_kernel, dim3(unsigned(wall_blocks + geo_blocks)), dim3(256), 0, L.stream, w, ga,
                           uint32_t(wall_blocks));
    };
    (void)by_q(L.q, [&](auto QC) {
      constexpr int Q = QC.value;
      if (L.g.bc_x == 0) {
        if (adj) go(k_wall<ST, CT, true, true, Q>, k_wall_geometry<ST, CT, true, true, Q>);
        else go(k_wall<ST, CT, true, false, Q>, k_wall_geometry<ST, CT, true, false, Q>);
      } else {
        if (adj) go(k_wall<ST, CT, false, true, Q>, k_wall_geometry<ST, CT, false, true, Q>);
        else go(k_wall<ST, CT, false, false, Q>, k_wall_geometry<ST, CT, false, false, Q>);
      }
      return hipSuccess;
    });
    return hipGetLastError();
  });
}

template <class CT>
static SweepArgs<CT> sweep_args(const Launch& L, const void* src, void* dst, int64_t step) {
  SweepArgs<CT> a{};
  a.src = src; a.dst = dst; a.g = L.g; a.m = L.m;
  a.blk_slot = L.blk_slot; a.d_eff = (const CT*)L.d_eff; a.tag = L.tag;
  a.wall_out = (const CT*)L.wall_out; a.bbox_total = L.bbox_total; a.rot = L.rot;
  a.uB_static = (const CT*)L.uB_static; a.partial = L.partial; a.mass_part = nullptr; a.flag = nullptr;
  a.step = step; a.nblocks = L.nblocks;
  a.ghost = (const CT*)L.ghost;
  if (L.m.fd_share > 0.0 && L.fd_u) {
    a.fd_u = (const CT*)L.fd_u;
    a.near_index = L.near_index;
    a.fd_share = CT(L.m.fd_share);
  }
  return a;
}

hipError_t launch_sweep(const Launch& L, const void* src, void* dst, int64_t step, bool diag, bool check) {
  if (L.nblocks == 0) return hipSuccess;
  return by_types(L.storage, L.compute, [&](auto* st, auto* ct) {
    using ST = std::remove_pointer_t<decltype(st)>;
    using CT = std::remove_pointer_t<decltype(ct)>;
    SweepArgs<CT> a = sweep_args<CT>(L, src, dst, step);
    if (diag) a.mass_part = L.mass_part;
    if (check) a.flag = L.flag;
    return by_q(L.q, [&](auto QC) {
      constexpr int Q = QC.value;
      if (L.g.bc_x == 0)
        hipLaunchKernelGGL((k_sweep<ST, CT, true, false, Q>), dim3(unsigned(L.nblocks)), dim3(kBlock), L.sweep_lds,
                           L.stream, a);
      else
        hipLaunchKernelGGL((k_sweep<ST, CT, false, false, Q>), dim3(unsigned(L.nblocks)), dim3(kBlock), L.sweep_lds,
                           L.stream, a);
      return hipGetLastError();
    });
  });
}

hipError_t launch_moments(const Launch& L, const void* src, int64_t step, void* rho, void* u, void* uhat) {
  return by_types(L.storage, L.compute, [&](auto* st, auto* ct) {
    using ST = std::remove_pointer_t<decltype(st)>;
    using CT = std::remove_pointer_t<decltype(ct)>;
    SweepArgs<CT> a = sweep_args<CT>(L, src, nullptr, step);
    a.out_rho = (CT*)rho; a.out_u = (CT*)u; a.out_uhat = (CT*)uhat;
    return by_q(L.q, [&](auto QC) {
      constexpr int Q = QC.value;
      if (L.g.bc_x == 0)
        hipLaunchKernelGGL((k_sweep<ST, CT, true, true, Q>), dim3(unsigned(L.nblocks)), dim3(kBlock), 0, L.stream, a);
      else
        hipLaunchKernelGGL((k_sweep<ST, CT, false, true, Q>), dim3(unsigned(L.nblocks)), dim3(kBlock), 0, L.stream, a);
      return hipGetLastError();
    });
  });
}

hipError_t launch_prologue(const Launch& L, int64_t step) {
  const int64_t plane = int64_t(L.g.ny) * L.g.nz;
  if (L.g.bc_x == 0) return hipSuccess;
  // the wall model samples in FP64: also fill the FP64 plane when it differs
  double* g64 = (L.compute != 0 && L.nrot > 0) ? L.ghost64 : nullptr;
  return by_compute(L.compute, [&](auto* ct) {
    using CT = std::remove_pointer_t<decltype(ct)>;
    return by_q(L.q, [&](auto QC) {
      hipLaunchKernelGGL((k_prologue<CT, QC.value>), grid1(plane, 256), dim3(256), 0, L.stream, L.g, L.m, step,
                         (CT*)L.ghost, g64);
      return hipGetLastError();
    });
  });
}

hipError_t launch_finalize(const Launch& L, int64_t n0, int32_t count, int32_t nslots, int32_t diag_every,
                           int32_t me_slots) {
  const int G = kPartL1;
  if (me_slots >= 0 && L.me_partial) {
    hipLaunchKernelGGL(k_reduce_me_l1, dim3(G, unsigned(count)), dim3(256), 0, L.stream, L.me_partial, me_slots,
                       L.me_l1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_me_l2, dim3(unsigned(count)), dim3(64), 0, L.stream, L.me_l1, G, n0, L.hist_me,
                       L.hist_cap);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_reduce_l1, dim3(G, unsigned(count)), dim3(256), 0, L.stream, L.partial, nslots, L.mass_part,
                     L.nblocks, n0, diag_every, L.part_l1, L.mass_l1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_l2, dim3(unsigned(count)), dim3(256), 0, L.stream, L.part_l1, L.mass_l1, G, n0,
                     diag_every, L.hist, L.hist_cap);
  return hipGetLastError();
}

hipError_t launch_fd_velocity(const Launch& L, const void* src, int64_t) {
  if (L.nnear <= 0 || !L.fd_u) return hipSuccess;
  return by_types(L.storage, L.compute, [&](auto* st, auto* ct) {
    using ST = std::remove_pointer_t<decltype(st)>;
    using CT = std::remove_pointer_t<decltype(ct)>;
    return by_q(L.q, [&](auto QC) {
      constexpr int Q = QC.value;
      if (L.g.bc_x == 0)
        hipLaunchKernelGGL((k_fd_velocity<ST, CT, true, Q>), dim3(unsigned(L.nnear)), dim3(kBlock), 0, L.stream,
                           (const ST*)src, L.g, (const CT*)L.ghost, L.fsi_tiles, (CT*)L.fd_u);
      else
        hipLaunchKernelGGL((k_fd_velocity<ST, CT, false, Q>), dim3(unsigned(L.nnear)), dim3(kBlock), 0, L.stream,
                           (const ST*)src, L.g, (const CT*)L.ghost, L.fsi_tiles, (CT*)L.fd_u);
      return hipGetLastError();
    });
  });
}

hipError_t launch_momentum_exchange(const Launch& L, const void* state, int32_t nslots, double* me_partial) {
  if (nslots <= 0 || !L.fsi_tiles) return hipSuccess;
  return by_types(L.storage, L.compute, [&](auto* st, auto* ct) {
    using ST = std::remove_pointer_t<decltype(st)>;
    using CT = std::remove_pointer_t<decltype(ct)>;
    MeArgs<CT> a{};
    a.state = state; a.g = L.g; a.tag = L.tag; a.rot = L.rot; a.uB_static = (const CT*)L.uB_static;
    a.fsi_tiles = L.fsi_tiles; a.partial = me_partial;
    return by_q(L.q, [&](auto QC) {
      constexpr int Q = QC.value;
      if (L.g.bc_x == 0)
        hipLaunchKernelGGL((k_momentum_exchange<ST, CT, true, Q>), dim3(unsigned(nslots)), dim3(kBlock), 0, L.stream,
                           a);
      else
        hipLaunchKernelGGL((k_momentum_exchange<ST, CT, false, Q>), dim3(unsigned(nslots)), dim3(kBlock), 0,
                           L.stream, a);
      return hipGetLastError();
    });
  });
}

template <class CT>
static AdjArgs<CT> adj_args(const Launch& L, const AdjLaunch& A) {
  AdjArgs<CT> a{};
  a.src = A.src; a.lam_in = (const CT*)A.lam_in; a.lam_out = (CT*)A.lam_out; a.side = (CT*)A.side;
  a.side_in = (const CT*)A.side_in;
  a.g = L.g; a.m = L.m; a.blk_slot = L.blk_slot; a.d_eff = (const CT*)L.d_eff; a.tag = L.tag;
  a.wall_out = (const CT*)L.wall_out; a.bbox_total = L.bbox_total; a.rot = L.rot;
  a.uB_static = (const CT*)L.uB_static; a.ghost = (const CT*)L.ghost; a.ubar = A.ubar; a.G = A.G;
  a.obj_w = A.obj_w; a.obj_tag = A.obj_tag; a.nblocks = L.nblocks;
  a.zero = A.zero; a.nzero = A.zero ? A.nzero : 0;
  if (L.m.fd_share > 0.0 && L.fd_u) {
    a.fd_u = (const CT*)L.fd_u;
    a.near_index = L.near_index;
    a.fd_share = CT(L.m.fd_share);
  }
  a.tiles = L.fsi_tiles;
  a.flag = L.flag;
  return a;
}

hipError_t launch_adjoint_fd(const Launch& L, const AdjLaunch& A) {
  if (!(L.m.fd_share > 0.0) || !L.fd_u || L.nnear <= 0) return hipSuccess;
  return by_types(L.storage, L.compute, [&](auto* st, auto* ct) {
    using ST = std::remove_pointer_t<decltype(st)>;
    using CT = std::remove_pointer_t<decltype(ct)>;
    AdjArgs<CT> a = adj_args<CT>(L, A);
    return by_q(L.q, [&](auto QC) {
      constexpr int Q = QC.value;
      if (L.g.bc_x == 0)
        hipLaunchKernelGGL((k_adj_fd<ST, CT, true, Q>), dim3(unsigned(L.nnear)), dim3(kBlock), 0, L.stream, a);
      else
        hipLaunchKernelGGL((k_adj_fd<ST, CT, false, Q>), dim3(unsigned(L.nnear)), dim3(kBlock), 0, L.stream, a);
      return hipGetLastError();
    });
  });
}

hipError_t launch_adjoint_sweep(const Launch& L, const AdjLaunch& A) {
  return by_types(L.storage, L.compute, [&](auto* st, auto* ct) {
    using ST = std::remove_pointer_t<decltype(st)>;
    using CT = std::remove_pointer_t<decltype(ct)>;
    AdjArgs<CT> a = adj_args<CT>(L, A);
    const int64_t nzb = A.zero ? (A.nzero + kBlock - 1) / kBlock : 0;
    const dim3 grid(unsigned(L.nblocks + nzb));
    return by_q(L.q, [&](auto QC) {
      constexpr int Q = QC.value;
      if (L.g.bc_x == 0) hipLaunchKernelGGL((k_adj_sweep<ST, CT, true, Q>), grid, dim3(kBlock), 0, L.stream, a);
      else hipLaunchKernelGGL((k_adj_sweep<ST, CT, false, Q>), grid, dim3(kBlock), 0, L.stream, a);
      return hipGetLastError();
    });
  });
}

hipError_t launch_init_equilibrium(const Launch& L, void* dst, const void* rho, const void* u) {
  return by_types(L.storage, L.compute, [&](auto* st, auto* ct) {
    using ST = std::remove_pointer_t<decltype(st)>;
    using CT = std::remove_pointer_t<decltype(ct)>;
    return by_q(L.q, [&](auto QC) {
      hipLaunchKernelGGL((k_init_eq<ST, CT, QC.value>), grid1(L.g.N, 256), dim3(256), 0, L.stream, (ST*)dst, L.g,
                         (const CT*)rho, (const CT*)u);
      return hipGetLastError();
    });
  });
}

hipError_t launch_get_populations(const Launch& L, const void* src, double* dst) {
  return by_types(L.storage, L.compute, [&](auto* st, auto*) {
    using ST = std::remove_pointer_t<decltype(st)>;
    return by_q(L.q, [&](auto QC) {
      hipLaunchKernelGGL((k_get_pop<ST, QC.value>), grid1(L.g.N, 256), dim3(256), 0, L.stream, (const ST*)src, L.g,
                         dst);
      return hipGetLastError();
    });
  });
}

hipError_t launch_set_populations(const Launch& L, void* dst, const double* src) {
  return by_types(L.storage, L.compute, [&](auto* st, auto*) {
    using ST = std::remove_pointer_t<decltype(st)>;
    return by_q(L.q, [&](auto QC) {
      hipLaunchKernelGGL((k_set_pop<ST, QC.value>), grid1(L.g.N, 256), dim3(256), 0, L.stream, (ST*)dst, L.g, src);
      return hipGetLastError();
    });
  });
}

hipError_t launch_get_populations_at(const Launch& L, const void* src, const int64_t* cells, int64_t count,
                                     double* dst) {
  if (count == 0) return hipSuccess;
  return by_types(L.storage, L.compute, [&](auto* st, auto*) {
    using ST = std::remove_pointer_t<decltype(st)>;
    return by_q(L.q, [&](auto QC) {
      hipLaunchKernelGGL((k_get_pop_at<ST, QC.value>), grid1(count, 256), dim3(256), 0, L.stream, (const ST*)src, L.g,
                         cells, count, dst);
      return hipGetLastError();
    });
  });
}

// Two-way rotor coupling, one lane per rotor (the structure update of the
// FSI time loop, Sec. 3.2, for a rigid rotation about the fixed axis):
// I (Omega_{n+1} - Omega_n) = e . T_n - T_gen and theta_{n+1} = theta_n +
// Omega_n, T_n the torque record of step n.  Writes the speed of step m into
// the rotor table (read by the solid velocity of the sweep, the wall model
// and the momentum exchange) and the blade angles of steps m and m + 1 (read
// by the geometry, which the wall launch of step m computes for m + 1).
__global__ __launch_bounds__(64) void k_couple(RotorTable* __restrict__ rt, RotorDyn* __restrict__ dyn,
                                               const double* __restrict__ hist, int64_t hist_cap, int64_t rec,
                                               int64_t m) {
  const int k = threadIdx.x;
  if (k >= rt->n) return;
  RotorDev& R = rt->r[k];
  double th0, th1;
  if (R.inertia > 0.0) {
    double th = dyn->theta[k], om = dyn->omega[k];
    if (rec >= 0) {
      const double* T = hist + (rec % hist_cap) * kHist + 4 + 6 * (R.tag - 1);
      const double Tax = R.e[0] * T[0] + R.e[1] * T[1] + R.e[2] * T[2];
      const double om1 = om + (Tax - R.tgen) / R.inertia;
      th = th + om;
      om = om1;
      dyn->theta[k] = th;
      dyn->omega[k] = om;
    }
    R.omega = om;
    th0 = th;
    th1 = th + om;
  } else {
    th0 = R.phase0 + R.omega * double(m);
    th1 = R.phase0 + R.omega * double(m + 1);
  }
  BladeTrig& a = dyn->trig[m & 1];
  BladeTrig& b = dyn->trig[(m + 1) & 1];
  for (int j = 0; j < R.nb; ++j) {
    const double off = 6.283185307179586476925286766559 * double(j) / double(R.nb);
    a.c[k][j] = cos(th0 + off);
    a.s[k][j] = sin(th0 + off);
    b.c[k][j] = cos(th1 + off);
    b.s[k][j] = sin(th1 + off);
  }
}

hipError_t launch_couple(const Launch& L, int64_t rec, int64_t m) {
  if (!L.dyn || L.nrot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_couple, dim3(1), dim3(64), 0, L.stream, L.rot, L.dyn, (const double*)L.hist, L.hist_cap, rec,
                     m);
  return hipGetLastError();
}

// Plain streaming copy: one 16 B element per thread, non-temporal loads and
// stores.  This is the fastest copy form measured here (32.6 GB buffers:
// 82 % of 8 TB/s, against 78 % with plain loads and stores and 70 % with
// four elements per thread).  Launched in chunks of 2^30 elements.
typedef float float4v __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(const float4v* __restrict__ src, float4v* __restrict__ dst,
                                                     int64_t n16) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t stream) {
  constexpr int64_t kChunk = int64_t(1) << 30;
  const int64_t n16 = bytes / 16;
  for (int64_t o = 0; o < n16; o += kChunk) {
    const int64_t m = std::min(kChunk, n16 - o);
    hipLaunchKernelGGL(k_stream_copy, dim3(unsigned((m + 255) / 256)), dim3(256), 0, stream,
                       static_cast<const float4v*>(src) + o, static_cast<float4v*>(dst) + o, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fill_rest(const Launch& L, void* dst) {
  return by_types(L.storage, L.compute, [&](auto* st, auto*) {
    using ST = std::remove_pointer_t<decltype(st)>;
    const int64_t count = L.g.row * L.g.ny * L.g.nz;
    hipLaunchKernelGGL(k_fill_rest<ST>, grid1(count, 256), dim3(256), 0, L.stream, (ST*)dst, count);
    return hipGetLastError();
  });
}

hipError_t launch_mark_blocks(const Launch& L) {
  hipError_t e = hipMemsetAsync(L.blk_slot, 0, sizeof(int32_t) * L.nblocks, L.stream);
  if (e != hipSuccess) return e;
  return by_compute(L.compute, [&](auto* ct) {
    using CT = std::remove_pointer_t<decltype(ct)>;
    hipLaunchKernelGGL(k_mark<CT>, grid1(L.g.N, 256), dim3(256), 0, L.stream, L.rot, L.g, (const CT*)L.d_static,
                       L.tag_static, (const CT*)L.dd, L.blk_slot);
    return hipGetLastError();
  });
}

hipError_t launch_refill_porosity(const Launch& L) {
  return by_compute(L.compute, [&](auto* ct) {
    using CT = std::remove_pointer_t<decltype(ct)>;
    hipLaunchKernelGGL(k_refill<CT>, grid1(L.g.N, 256), dim3(256), 0, L.stream, L.g, (const CT*)L.d_static,
                       L.tag_static, (const CT*)L.dd, (CT*)L.d_eff, L.tag);
    return hipGetLastError();
  });
}

}  // namespace hlbm
