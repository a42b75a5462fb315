// C ABI of libhlbm: validation, workspace layout, the host step loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hlbm.h"
#include "hlbm_internal.h"
#include "launch.h"

using namespace hlbm;

namespace {

std::string g_create_error;

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int elem_size(int t) { return t == HLBM_F64 ? 8 : t == HLBM_F32 ? 4 : 2; }

bool desc_ok(const hlbm_desc* d, std::string* why) {
  if (!d) { *why = "desc is NULL"; return false; }
  if (d->nx < 2 || d->ny < 1 || d->nz < 1) { *why = "lattice needs nx >= 2, ny >= 1, nz >= 1"; return false; }
  const int64_t N = int64_t(d->nx) * d->ny * d->nz;
  if (N >= (int64_t(1) << 31)) { *why = "lattice above 2^31 cells"; return false; }
  if (d->compute != HLBM_F64 && d->compute != HLBM_F32) { *why = "compute must be F64 or F32"; return false; }
  if (d->storage < HLBM_F64 || d->storage > HLBM_BF16) { *why = "unknown storage type"; return false; }
  if (d->compute == HLBM_F64 && d->storage != HLBM_F64) { *why = "F64 compute needs F64 storage"; return false; }
  if (d->compute == HLBM_F32 && d->storage == HLBM_F64) { *why = "F64 storage needs F64 compute"; return false; }
  if (d->bc_x != HLBM_BC_PERIODIC && d->bc_x != HLBM_BC_INFLOW_OUTFLOW) { *why = "unknown bc_x"; return false; }
  if (d->bbox_cells < 0 || d->history < 0) { *why = "negative bbox_cells or history"; return false; }
  if (d->velocities != 0 && d->velocities != 27 && d->velocities != 19) {
    *why = "velocities must be 27 (or 0) or 19";
    return false;
  }
  return true;
}

// Velocities of the lattice's set: 27 or 19.
int vel_of(const hlbm_desc* d) { return d->velocities == 19 ? 19 : 27; }

int64_t cells_of(const hlbm_desc* d) { return int64_t(d->nx) * d->ny * d->nz; }

// Population elements per (y, z) row in the blocked layout: the row's x
// extent rounded up to whole blocks of kTileX cells, q populations each.
int64_t pop_row(const hlbm_desc* d) { return int64_t((d->nx + kTileX - 1) / kTileX) * vel_of(d) * kTileX; }
// Elements of one population buffer.
int64_t pop_elems(const hlbm_desc* d) { return pop_row(d) * d->ny * d->nz; }

// Force-partial slots of the workspace (kPartial FP64 each): one step's FSI
// workgroups take at most one slot per sweep workgroup; up to kMaxBatch
// steps' worth, capped at 2^20 slots (768 MiB) unless one step needs more.
int64_t partial_slots(int64_t nblocks) {
  return std::min<int64_t>(int64_t(kMaxBatch) * nblocks, std::max<int64_t>(nblocks, int64_t(1) << 20));
}


struct Layout {
  int64_t d_eff, d_effb, d_static, tag, tagb, tag_static, uB, dd, blk, partial, partl1, mass, massl1, wlist, wlistb,
      wcount, flag, stats, rot, geo, geob, ut0, ut1, act0, act1, act2, wall, hist, ghost, ghost64, ghostb, ghost64b,
      trig, lam0, lam1, utb0, utb1, ubar, side, sideb, scr_ut, scr_act, scr_actb, fsi_tiles, me_partial, me_l1,
      hist_me, near_index, fd_u, dyn, gmark, gstats, total;
};

Layout layout(const hlbm_desc* d) {
  Layout L{};
  const int64_t N = cells_of(d);
  const int cs = elem_size(d->compute);
  const int64_t nb = int64_t((d->nx + kTileX - 1) / kTileX) * ((d->ny + kTileY - 1) / kTileY) * d->nz;
  const int64_t B = d->bbox_cells;
  const int64_t H = d->history > 0 ? d->history : 1024;
  int64_t o = 0;
  // every section gets at least one aligned block, so sections never alias
  auto take = [&](int64_t bytes) { int64_t at = o; o = align_up(o + std::max<int64_t>(bytes, 1), kAlign); return at; };
  // porosity, tags, box geometry and wall list in two sets, by step parity
  L.d_eff = take(N * cs);
  L.d_effb = take(N * cs);
  L.d_static = take(N * cs);
  L.tag = take(N);
  L.tagb = take(N);
  L.tag_static = take(N);
  L.uB = take((d->flags & HLBM_WITH_SOLID_VELOCITY) ? 3 * N * cs : 0);
  L.dd = take((d->flags & HLBM_WITH_CONTROL) ? N * cs : 0);
  L.blk = take(nb * 4);
  L.partial = take(partial_slots(nb) * kPartial * 8);
  L.partl1 = take(int64_t(kMaxBatch) * kPartL1 * kPartial * 8);
  L.mass = take(int64_t(kMaxBatch) * nb * 8);
  L.massl1 = take(int64_t(kMaxBatch) * kPartL1 * 8);
  L.wlist = take(B * 4);
  L.wlistb = take(B * 4);
  L.wcount = take(64);
  L.flag = take(64);
  L.stats = take(64);
  L.rot = take(sizeof(RotorTable));
  L.geo = take(4 * B * 8);
  L.geob = take(4 * B * 8);
  L.ut0 = take(B * 8);
  L.ut1 = take(B * 8);
  L.act0 = take(B);
  L.act1 = take(B);
  L.act2 = take(B);
  L.wall = take(kWallOut * B * cs);
  L.hist = take(H * kHist * 8);
  const int64_t plane = int64_t(d->ny) * d->nz;
  L.ghost = take(d->bc_x == HLBM_BC_INFLOW_OUTFLOW ? 9 * plane * cs : 0);
  L.ghost64 = take(d->bc_x == HLBM_BC_INFLOW_OUTFLOW ? 9 * plane * 8 : 0);
  L.ghostb = take(d->bc_x == HLBM_BC_INFLOW_OUTFLOW ? 9 * plane * cs : 0);
  L.ghost64b = take(d->bc_x == HLBM_BC_INFLOW_OUTFLOW ? 9 * plane * 8 : 0);
  L.trig = take(d->bbox_cells > 0 ? int64_t(kTrigSteps) * int64_t(sizeof(BladeTrig)) : 0);
  L.dyn = take(d->bbox_cells > 0 ? int64_t(sizeof(RotorDyn)) : 0);
  L.gmark = take(2 * B * 8);
  L.gstats = take(2 * ((B + 255) / 256) * 8);
  const bool adj = (d->flags & HLBM_WITH_ADJOINT) != 0;
  const int64_t lam_bytes = adj ? pop_elems(d) * cs : 0;
  L.lam0 = take(lam_bytes);
  L.lam1 = take(lam_bytes);
  L.utb0 = take(adj ? B * 8 : 0);
  L.utb1 = take(adj ? B * 8 : 0);
  L.ubar = take(adj ? 9 * N * 8 : 0);
  L.side = take(adj ? 9 * plane * cs : 0);
  L.sideb = take(adj ? 9 * plane * cs : 0);
  L.scr_ut = take(adj ? B * 8 : 0);
  L.scr_act = take(adj ? B : 0);
  L.scr_actb = take(adj ? B : 0);
  const bool me = (d->flags & HLBM_WITH_MOMENTUM_EXCHANGE) != 0;
  const bool fd = (d->flags & HLBM_WITH_FD_STRAIN) != 0;
  L.fsi_tiles = take(me || fd ? nb * 4 : 0);
  L.near_index = take(fd ? nb * 4 : 0);
  L.fd_u = take(fd ? nb * 3 * kBlock * cs : 0);
  L.me_partial = take(me ? partial_slots(nb) * kMePartial * 8 : 0);
  L.me_l1 = take(me ? int64_t(kMaxBatch) * kPartL1 * kMePartial * 8 : 0);
  L.hist_me = take(me ? H * kHistMe * 8 : 0);
  L.total = o;
  return L;
}

struct RotorBox { int32_t b0[3], bn[3]; };

// Fixed box around the rotor's swept cylinder plus a margin (the transition
// band eps_h/2 and one cell for the rasterized box).
bool rotor_box(const hlbm_desc* d, const hlbm_rotor& r, double margin, RotorBox* box, std::string* why,
               bool clip = false) {
  const double an = std::sqrt(r.axis[0] * r.axis[0] + r.axis[1] * r.axis[1] + r.axis[2] * r.axis[2]);
  if (!(an > 0)) { *why = "rotor axis is zero"; return false; }
  const double hc = std::sqrt(0.25 * r.chord * r.chord + 0.25 * r.thick * r.thick);
  const double rc = std::max(std::sqrt(r.R * r.R + hc * hc), r.r_hub);
  const double ha = std::max(hc, r.r_hub);
  const double m = margin;
  const int n3[3] = {d->nx, d->ny, d->nz};
  for (int k = 0; k < 3; ++k) {
    const double e = r.axis[k] / an;
    const double ext = ha * std::fabs(e) + rc * std::sqrt(std::max(0.0, 1.0 - e * e));
    int lo = int(std::floor(r.center[k] - ext - m));
    int hi = int(std::ceil(r.center[k] + ext + m));
    if (clip) {
      // capacity bound: the solid itself must fit, the margin is clipped
      if (r.center[k] - ext < 0 || r.center[k] + ext > n3[k] - 1) { *why = "rotor leaves the domain"; return false; }
      lo = lo < 0 ? 0 : lo;
      hi = hi > n3[k] - 1 ? n3[k] - 1 : hi;
    }
    if (lo < 0 || hi > n3[k] - 1) { *why = "rotor bounding box leaves the domain"; return false; }
    box->b0[k] = lo;
    box->bn[k] = hi - lo + 1;
  }
  return true;
}

// Height (tile rows) of the bands of the sweep order.  A z plane of up to
// 1024 tiles (about four per CU) fits in the workgroups in flight, so plane
// after plane already sweeps the three z planes that read a source row
// together, and the plain lattice order (one band) is fastest; a larger
// plane is swept in bands of 8 tile rows through all z.  Measured on one
// fixed allocation on MI355X (the population buffers reused, so that the
// spread between allocations drops out): 256x128x128 (128 tiles per plane)
// 154.7 us with one band against 163-166 us with bands of 1-16 rows;
// 1536x768x256 (4608 tiles per plane) 11.74 ms with bands of 8 rows against
// 11.87 ms (1 row) and 11.96 ms (one band); 1024x512x384 7.41 ms against
// 7.51 ms and 7.88 ms.  HLBM_TILE_BAND overrides the choice (measurement
// runs).
uint32_t tile_band(const hlbm_desc* d, int32_t nty) {
  if (const char* e = std::getenv("HLBM_TILE_BAND")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1) return uint32_t(std::min<long>(v, nty));
  }
  const int64_t ntx = (d->nx + kTileX - 1) / kTileX;
  return ntx * nty > 1024 ? uint32_t(std::min<int32_t>(8, nty)) : uint32_t(nty);
}

// Dynamic LDS of a sweep workgroup, which caps the workgroups resident on a
// CU (160 KB of LDS each; the sweep itself holds under 4 KB).  Without a
// cap, the FP32 sweep runs five per CU (its registers allow five waves per
// SIMD).  On lattices of more than 2^18 tiles the FP32 sweep is faster with
// four per CU, measured on one lattice with the cap switched every 43-83 steps
// (four rounds, two allocations): D3Q27 at 1536x768x256 11.56-11.58 against
// 11.72-11.73 ms and 10.94-10.99 against 11.07-11.11 ms, at 1024x512x384
// 7.72 against 7.83 ms; D3Q19 at 1536x768x256 7.73-7.76 against 7.86-7.91
// ms.  Three per CU is slower (D3Q27 12.32 and 11.79 ms on the same two
// allocations).  FP16 and BF16 storage, closer to the ALU bound, gain
// nothing or slow down with a cap.  HLBM_SWEEP_WG_PER_CU = 3 or 4 sets the
// cap, 0 removes it (measurement runs).
uint32_t sweep_lds(const hlbm_desc* d, int64_t tiles) {
  int cap = 0;
  if (d->storage == HLBM_F32 && tiles > (int64_t(1) << 18)) cap = 4;
  if (const char* e = std::getenv("HLBM_SWEEP_WG_PER_CU")) cap = int(std::strtol(e, nullptr, 10));
  if (cap != 3 && cap != 4) return 0;
  return uint32_t(163840 / cap - 4096);
}

void set_tile_band(Geometry* g, uint32_t band) {
  const uint32_t ntx = uint32_t(g->ntx), nz = uint32_t(g->nz), nty = uint32_t(g->nty);
  g->band = band;
  g->full_tiles = (nty / band) * band * ntx * nz;
  const uint32_t tail = nty - (nty / band) * band;
  g->by_ntx = make_udiv(ntx);
  g->by_bandrow = make_udiv(band * ntx);
  g->by_band = make_udiv(band * ntx * nz);
  g->by_tailrow = make_udiv(std::max(tail, 1u) * ntx);
}

}  // namespace

struct hlbm_lattice {
  hlbm_desc desc{};
  hipStream_t stream = nullptr;
  Layout lay{};
  Launch L{};
  void* pop[2] = {nullptr, nullptr};
  int cur = 0;                 // pop[cur] holds the state
  char* ws = nullptr;           // the caller's workspace
  // geometry buffer sets (porosity, tags, box geometry, wall list) by step parity
  struct GeoSet {
    void* d_eff;
    uint8_t* tag;
    double* geo;
    int32_t* wlist;
  } set[2] = {};
  double* ut[2] = {nullptr, nullptr};
  int wcur = 0;                // ut[wcur] holds the friction-velocity state
  // wall-model activity of the state (act[acur]), of the next state, and of
  // the one after it, which the geometry of the next step resets while the
  // wall model of this step runs
  uint8_t* act[3] = {nullptr, nullptr, nullptr};
  int acur = 0;
  RotorTable rot{};
  std::vector<hlbm_rotor> rotors;
  // reference grids by rotor index (caller memory)
  struct GridRef {
    const double* phi = nullptr;
    int32_t n[3] = {0, 0, 0};
    double h = 0.0, o[3] = {0.0, 0.0, 0.0};
  } grids[kMaxRotors];
  hlbm_params params{};
  bool have_params = false;
  int32_t nslots = 0;
  int32_t nme = 0;             // tiles of the momentum-exchange launch
  int64_t step = 0;
  int64_t hist_start = 0;      // first step recorded since init
  int64_t hist_cap = 0;
  std::string err;
  // forward record of the discrete adjoint
  struct Record {
    bool valid = false;
    int64_t n0 = 0, nsteps = 0, t0 = 0, t1 = 0;
    int32_t obj_tag = 0, ckpt_every = 1;
    char* ckpt = nullptr;
    double J = 0.0;
  } rec;
  int wc_epoch = 0;  // wall-list counter of the next geometry launch (0 .. kCounters - 1)
  // the geometry of step ahead_step (counter ahead_epoch) is already in its
  // buffer set, computed by the previous step's wall-model launch; -1: none
  int64_t ahead_step = -1;
  int ahead_epoch = 0;
  // steps swept but not yet reduced: pending steps from pend_n0; their force
  // partials are slices of `batch` steps in the partial buffer
  int64_t pend_n0 = 0;
  int32_t pending = 0, batch = 1;
  // blade angles on the device for steps [trig_base, trig_base + kTrigSteps)
  BladeTrig* trig_host = nullptr;  // pinned staging buffer
  hipEvent_t trig_ev = nullptr;
  int64_t trig_base = -1;
  void* ghost[2] = {nullptr, nullptr};
  double* ghost64[2] = {nullptr, nullptr};
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof[4];
  std::vector<hipEvent_t> pool;
  int static_dev = -1;         // device whose static workspace this lattice uses, -1: caller's workspace
  bool coupled = false;        // a rotor turns with the fluid torque (inertia > 0)
  // growth layer of the rotor geometry: allowed by the environment, usable
  // for the current rotors, generation of the rotor / parameter state, and
  // the step and generation of the last geometry launch
  bool growth_env = false, growth_ok = false;
  long long gen = 1;
  int64_t geo_prev = -2;
  long long geo_prev_gen = 0;
  long long* gmark = nullptr;
};

namespace {

// Devices whose static workspace is in use by a lattice (one at a time).
std::mutex g_static_lock;
bool g_static_busy[64] = {};
bool static_claim(int dev) {
  std::lock_guard<std::mutex> g(g_static_lock);
  if (dev < 0 || dev >= 64 || g_static_busy[dev]) return false;
  g_static_busy[dev] = true;
  return true;
}
void static_release(int dev) {
  std::lock_guard<std::mutex> g(g_static_lock);
  if (dev >= 0 && dev < 64) g_static_busy[dev] = false;
}

int fail(hlbm_handle h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_create_error = msg;
  return code;
}
int hip_fail(hlbm_handle h, hipError_t e, const char* where) {
  return fail(h, HLBM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

void set_model(hlbm_handle h) {
  const hlbm_params& p = h->params;
  Model& m = h->L.m;
  m.tau0 = p.tau0;
  m.smag = 18.0 * std::sqrt(2.0) * p.cs_smag * p.cs_smag;
  m.eps_h = p.eps_h;
  m.transition = p.transition;
  m.wall_model = p.wall_model;
  m.E = p.E; m.kappa = p.kappa; m.y_s = p.y_s; m.tol = p.tol;
  m.nu = (p.tau0 - 0.5) / 3.0;
  m.inv_E = 1.0 / p.E;
  m.kappa_E = p.kappa / p.E;
  m.inv_kappa = 1.0 / p.kappa;
  m.inv_nu = 1.0 / m.nu;
  m.ys_nu = p.y_s / m.nu;
  m.nu_ys = m.nu / p.y_s;
  m.maxit = p.maxit;
  for (int a = 0; a < 3; ++a) m.u_in[a] = p.u_in[a];
  const double mag = std::sqrt(p.u_in[0] * p.u_in[0] + p.u_in[1] * p.u_in[1] + p.u_in[2] * p.u_in[2]);
  m.turb_amp = p.turb_I * mag;
  m.seed = p.seed;
  m.fd_share = p.fd_share;
}

// The launch state with the geometry buffer set and inflow plane of step n.
Launch launch_of(hlbm_handle h, int64_t n) {
  Launch L = h->L;
  const auto& q = h->set[n & 1];
  L.d_eff = q.d_eff;
  L.tag = q.tag;
  L.geo = q.geo;
  L.wlist = q.wlist;
  L.ghost = h->ghost[n & 1];
  L.ghost64 = h->ghost64[n & 1];
  return L;
}
void select_step(hlbm_handle h, int64_t n) { h->L = launch_of(h, n); }

int next_epoch(hlbm_handle h) {
  const int e = h->wc_epoch;
  h->wc_epoch = (e + 1) % kCounters;
  return e;
}

// Static porosity and tags (plus the control field) into both buffer sets.
// Growth layer of the rotor geometry (Sec. 3.1, Fig. fsialgo): a geometry
// launch of step n evaluates the rotor distance only on the box slots that
// the launch of step n - 1 marked (the cells within one cell of those whose
// distance lay within one cell of the transition band), when that launch ran
// under the same rotors and parameters.  Every launch marks for the next.
void growth_for(hlbm_handle h, Launch* L, int64_t n) {
  if (!h->growth_ok) {
    L->gmark = nullptr;
    L->guse = 0;
    return;
  }
  L->gmark = h->gmark;
  L->ggen = h->gen;
  L->guse = (h->geo_prev == n - 1 && h->geo_prev_gen == h->gen) ? 1 : 0;
  h->geo_prev = n;
  h->geo_prev_gen = h->gen;
}

// After a change of the rotors or parameters: the marks of earlier launches
// no longer apply.  The layer is used for prescribed rotations whose surface
// moves at most half a cell per step (|omega| (R + eps_h/2 + 1) <= 1/2): the
// best of the 26 neighbours of a cell then lies at least 0.88 cells deeper
// in the transition band, more than the motion.
void growth_update(hlbm_handle h) {
  ++h->gen;
  bool ok = h->growth_env && h->gmark && h->rot.n > 0;
  for (int k = 0; k < h->rot.n && ok; ++k) {
    const RotorDev& r = h->rot.r[k];
    // the layer's reach assumes a distance that changes by at most one per
    // cell; the interpolant of a reference grid can be steeper near creases
    if (r.inertia > 0 || r.grid || !(std::fabs(r.omega) * (r.R + 0.5 * h->params.eps_h + 1.0) <= 0.5)) ok = false;
  }
  h->growth_ok = ok;
}

hipError_t refill_porosity(hlbm_handle h) {
  h->ahead_step = -1;
  ++h->gen;
  for (int p = 0; p < 2; ++p) {
    hipError_t e = launch_refill_porosity(launch_of(h, p));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Zero the wall-list counters and restart their rotation: a geometry launch
// counts from zero into its own counter, also after a call that changed the
// rotor boxes or skipped the geometry (no rotors).
hipError_t reset_counters(hlbm_handle h) {
  h->wc_epoch = 0;
  h->ahead_step = -1;
  return hipMemsetAsync(h->L.wcount, 0, sizeof(int32_t) * kCounters, h->stream);
}

// Carry the wall-model state (u_tau, active) of every cell that lies in the
// box of the same rotor in both tables from the old slot layout to the new
// one (the state is per cell); cells new to a box start inactive.  Host
// round trip, set-up time only.
int remap_wall_state(hlbm_handle h, const RotorTable& old_t, int64_t old_total, const RotorTable& new_t,
                     int64_t new_total) {
  std::vector<double> ut_old(std::max<int64_t>(old_total, 1)), ut_new(std::max<int64_t>(new_total, 1), 0.0);
  std::vector<uint8_t> ac_old(std::max<int64_t>(old_total, 1)), ac_new(std::max<int64_t>(new_total, 1), 0);
  hipError_t e = hipSuccess;
  if (old_total > 0) {
    e = hipMemcpyAsync(ut_old.data(), h->ut[h->wcur], old_total * 8, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ac_old.data(), h->act[h->acur], old_total, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "read wall state");
  }
  for (int k = 0; k < new_t.n && k < old_t.n; ++k) {
    const RotorDev& a = old_t.r[k];
    const RotorDev& b = new_t.r[k];
    for (int z = 0; z < b.bn[2]; ++z)
      for (int y = 0; y < b.bn[1]; ++y)
        for (int x = 0; x < b.bn[0]; ++x) {
          const int X = b.b0[0] + x, Y = b.b0[1] + y, Z = b.b0[2] + z;
          const int ox = X - a.b0[0], oy = Y - a.b0[1], oz = Z - a.b0[2];
          if (ox < 0 || oy < 0 || oz < 0 || ox >= a.bn[0] || oy >= a.bn[1] || oz >= a.bn[2]) continue;
          const int64_t so = a.off + (int64_t(oz) * a.bn[1] + oy) * a.bn[0] + ox;
          const int64_t sn = b.off + (int64_t(z) * b.bn[1] + y) * b.bn[0] + x;
          ut_new[sn] = ut_old[so];
          ac_new[sn] = ac_old[so];
        }
  }
  const int64_t B = std::max<int64_t>(new_total, 1);
  e = hipMemcpyAsync(h->ut[h->wcur], ut_new.data(), B * 8, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->act[h->acur], ac_new.data(), B, hipMemcpyHostToDevice, h->stream);
  for (int k = 1; k < 3 && e == hipSuccess; ++k) e = hipMemsetAsync(h->act[(h->acur + k) % 3], 0, B, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "write wall state");
  return HLBM_OK;
}

bool same_boxes(const RotorTable& a, const RotorTable& b) {
  if (a.n != b.n) return false;
  for (int k = 0; k < a.n; ++k)
    for (int q = 0; q < 3; ++q)
      if (a.r[k].b0[q] != b.r[k].b0[q] || a.r[k].bn[q] != b.r[k].bn[q] || a.r[k].mb0[q] != b.r[k].mb0[q] ||
          a.r[k].mbn[q] != b.r[k].mbn[q])
        return false;
  return true;
}

// Mark FSI workgroups and number them (host round trip; set-up time only).
int rebuild_slots(hlbm_handle h) {
  hipError_t e = launch_mark_blocks(h->L);
  if (e != hipSuccess) return hip_fail(h, e, "mark blocks");
  std::vector<int32_t> flags(h->L.nblocks);
  e = hipMemcpyAsync(flags.data(), h->L.blk_slot, sizeof(int32_t) * flags.size(), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "read block flags");
  // slot >= 0: FSI path (porosity, tags, wall-model outputs, force partial);
  // -2: plain path within the wall model's probe reach, where the adjoint
  // gathers the probe-velocity adjoints; -1: plain path.
  // momentum-exchange tiles: the FSI tiles and their neighbours (a cell next
  // to an element's cell lies in the same tile or an adjacent one)
  std::vector<int32_t> tiles;
  if (h->L.fsi_tiles) {
    const Geometry& g = h->L.g;
    const int ntx = g.ntx, nty = g.nty, nz = g.nz;
    std::vector<uint8_t> near(flags.size(), 0);
    for (size_t b = 0; b < flags.size(); ++b) {
      if (!(flags[b] & 1)) continue;
      const int tz = int(b / (size_t(ntx) * nty)), r = int(b % (size_t(ntx) * nty));
      const int ty = r / ntx, tx = r % ntx;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            int X = tx + dx;
            if (g.bc_x == 0) X = (X + ntx) % ntx;
            else if (X < 0 || X >= ntx) continue;
            const int Y = (ty + dy + nty) % nty, Z = (tz + dz + nz) % nz;
            near[(size_t(Z) * nty + Y) * ntx + X] = 1;
          }
    }
    for (size_t b = 0; b < near.size(); ++b)
      if (near[b]) tiles.push_back(int32_t(b));
  }
  int32_t n = 0;
  for (auto& f : flags) f = (f & 1) ? n++ : (f & 2) ? -2 : -1;
  // the finite-difference strain of an FSI tile's cells reads the velocity
  // of the neighbouring tiles' cells: the adjoint gathers there too
  if (h->L.near_index)
    for (const int32_t b : tiles)
      if (flags[size_t(b)] == -1) flags[size_t(b)] = -2;
  h->nslots = n;
  h->nme = (h->desc.flags & HLBM_WITH_MOMENTUM_EXCHANGE) ? int32_t(tiles.size()) : 0;
  h->L.nnear = h->L.near_index ? int32_t(tiles.size()) : 0;
  if (h->L.fsi_tiles && !tiles.empty()) {
    e = hipMemcpyAsync(const_cast<int32_t*>(h->L.fsi_tiles), tiles.data(), sizeof(int32_t) * tiles.size(),
                       hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "write FSI neighbourhood tile list");
  }
  if (h->L.near_index) {
    std::vector<int32_t> index(flags.size(), -1);
    for (size_t k = 0; k < tiles.size(); ++k) index[size_t(tiles[k])] = int32_t(k);
    e = hipMemcpyAsync(h->L.near_index, index.data(), sizeof(int32_t) * index.size(), hipMemcpyHostToDevice,
                       h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "write tile index");
  }
  // as many steps of slices as the partial buffer holds, at most kMaxBatch
  h->batch = int32_t(std::max<int64_t>(
      1, std::min<int64_t>(kMaxBatch, partial_slots(h->L.nblocks) / std::max<int32_t>(std::max(n, h->nme), 1))));
  e = hipMemcpyAsync(h->L.blk_slot, flags.data(), sizeof(int32_t) * flags.size(), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "write block slots");
  return HLBM_OK;
}

// Start the coupled rotors at the current step from their phase0 and omega.
int restart_rotation(hlbm_handle h) {
  if (!h->L.dyn) return HLBM_OK;
  double st[2 * kMaxRotors] = {0};
  for (int k = 0; k < h->rot.n; ++k) {
    st[k] = h->rot.r[k].phase0 + h->rot.r[k].omega * double(h->step);
    st[kMaxRotors + k] = h->rot.r[k].omega;
  }
  hipError_t e = hipMemcpyAsync(h->L.dyn, st, sizeof(st), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "restart rotor rotation");
  return HLBM_OK;
}

// The device rotor table with the coupled rotors' current speed and the
// blade angles of the current step and the next.
int upload_rotors(hlbm_handle h) {
  hipError_t e = hipMemcpyAsync(h->L.rot, &h->rot, sizeof(RotorTable), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess && h->coupled) e = launch_couple(h->L, -1, h->step);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "upload rotor table");
  return HLBM_OK;
}

// Build the rotor table (frames, boxes, pools); validates capacity.
int build_rotor_table(hlbm_handle h, const hlbm_rotor* r, int32_t n, RotorTable* out, int64_t* total) {
  RotorTable t = h->rot;  // keeps tag frames of static tags
  t.n = n;
  for (int k = 0; k < kTags; ++k) t.tag2rot[k] = -1;
  int64_t off = 0;
  for (int k = 0; k < n; ++k) {
    const hlbm_rotor& q = r[k];
    if (q.tag < 1 || q.tag > 15) return fail(h, HLBM_ERR_INVALID, "rotor tag must be 1..15");
    if (t.tag2rot[q.tag] >= 0) return fail(h, HLBM_ERR_INVALID, "rotor tags must be distinct");
    if (q.n_blades < 0 || q.n_blades > HLBM_MAX_BLADES) return fail(h, HLBM_ERR_INVALID, "n_blades out of range");
    if (!(q.R > q.r_hub) || !(q.r_hub >= 0) || !(q.chord > 0) || !(q.thick > 0))
      return fail(h, HLBM_ERR_INVALID, "rotor needs R > r_hub >= 0, chord > 0, thick > 0");
    if (!(q.inertia >= 0) || !std::isfinite(q.inertia) || !std::isfinite(q.torque_gen) || !std::isfinite(q.omega) ||
        !std::isfinite(q.phase0))
      return fail(h, HLBM_ERR_INVALID, "rotor needs a finite inertia >= 0, torque_gen, omega and phase0");
    RotorBox box;
    std::string why;
    if (!rotor_box(&h->desc, q, 0.5 * h->params.eps_h + 1.0, &box, &why)) return fail(h, HLBM_ERR_INVALID, why);
    RotorDev& d = t.r[k];
    const double an = std::sqrt(q.axis[0] * q.axis[0] + q.axis[1] * q.axis[1] + q.axis[2] * q.axis[2]);
    for (int a = 0; a < 3; ++a) { d.c[a] = q.center[a]; d.e[a] = q.axis[a] / an; }
    double a0[3] = {1, 0, 0};
    if (std::fabs(d.e[0]) >= 0.9) { a0[0] = 0; a0[1] = 1; }
    const double ae = a0[0] * d.e[0] + a0[1] * d.e[1] + a0[2] * d.e[2];
    double e1[3];
    for (int a = 0; a < 3; ++a) e1[a] = a0[a] - ae * d.e[a];
    const double n1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int a = 0; a < 3; ++a) d.e1[a] = e1[a] / n1;
    d.e2[0] = d.e[1] * d.e1[2] - d.e[2] * d.e1[1];
    d.e2[1] = d.e[2] * d.e1[0] - d.e[0] * d.e1[2];
    d.e2[2] = d.e[0] * d.e1[1] - d.e[1] * d.e1[0];
    d.R = q.R; d.r_hub = q.r_hub; d.chord = q.chord; d.thick = q.thick;
    d.tw_root = q.twist_root; d.tw_tip = q.twist_tip; d.omega = q.omega; d.phase0 = q.phase0;
    d.nb = q.n_blades; d.tag = q.tag;
    d.inertia = q.inertia; d.tgen = q.torque_gen;
    const auto& G = h->grids[k];
    if (G.phi && q.n_blades < 1)
      return fail(h, HLBM_ERR_INVALID, "a rotor with a reference grid needs n_blades >= 1 (blade 0 orients it)");
    d.grid = G.phi;
    for (int a = 0; a < 3; ++a) { d.gn[a] = G.n[a]; d.go[a] = G.o[a]; }
    d.gpad = 0;
    d.gh = G.h;
    for (int a = 0; a < 3; ++a) { d.b0[a] = box.b0[a]; d.bn[a] = box.bn[a]; }
    // FSI workgroups also cover the wall model's probe corners (reach y_s + 1
    // beyond the box; periodic in y and z), where the adjoint gathers the
    // probe-velocity adjoints
    const int reach = h->params.wall_model ? int(std::ceil(h->params.y_s)) + 2 : 0;
    for (int a = 0; a < 3; ++a) { d.mb0[a] = box.b0[a] - reach; d.mbn[a] = box.bn[a] + 2 * reach; }
    d.cells = int64_t(box.bn[0]) * box.bn[1] * box.bn[2];
    d.off = off;
    off += d.cells;
    t.tag2rot[q.tag] = k;
    for (int a = 0; a < 3; ++a) { t.frame[q.tag][a] = d.c[a]; t.frame[q.tag][3 + a] = d.e[a]; }
  }
  if (off > h->desc.bbox_cells)
    return fail(h, HLBM_ERR_INVALID, "rotor boxes need " + std::to_string(off) + " cells, workspace holds " +
                                         std::to_string(h->desc.bbox_cells));
  *out = t;
  *total = off;
  return HLBM_OK;
}

bool params_ok(const hlbm_params* p, std::string* why) {
  if (!p) { *why = "params is NULL"; return false; }
  if (!(p->tau0 > 0.5)) { *why = "tau0 must exceed 1/2"; return false; }
  if (!(p->cs_smag >= 0)) { *why = "cs_smag must be >= 0"; return false; }
  if (!(p->eps_h > 0)) { *why = "eps_h must be > 0"; return false; }
  if (p->transition != HLBM_TRANSITION_TANH && p->transition != HLBM_TRANSITION_LINEAR) { *why = "bad transition"; return false; }
  if (p->maxit < 1 || p->maxit > 100) { *why = "maxit must be 1..100"; return false; }
  if (p->wall_model && (!(p->E > 0) || !(p->kappa > 0) || !(p->y_s > 0.5 * p->eps_h) || !(p->tol > 0))) {
    *why = "wall model needs E > 0, kappa > 0, tol > 0, y_s > eps_h/2";
    return false;
  }
  if (!(p->turb_I >= 0) || p->diag_every < 0) { *why = "turb_I and diag_every must be >= 0"; return false; }
  if (p->force_mode < 0 || p->force_mode > 1) { *why = "force_mode must be 0 or 1"; return false; }
  if (!(p->fd_share >= 0.0 && p->fd_share <= 1.0)) { *why = "fd_share must be in [0, 1]"; return false; }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->u_in[a])) { *why = "u_in not finite"; return false; }
  return true;
}

}  // namespace

extern "C" {

int64_t hlbm_population_bytes(const hlbm_desc* d) {
  std::string why;
  if (!desc_ok(d, &why)) return -1;
  return pop_elems(d) * elem_size(d->storage);
}

int64_t hlbm_workspace_bytes(const hlbm_desc* d) {
  std::string why;
  if (!desc_ok(d, &why)) return -1;
  return layout(d).total;
}

int64_t hlbm_rotor_bbox_cells(const hlbm_desc* d, const hlbm_rotor* r, int32_t n) {
  std::string why;
  if (!desc_ok(d, &why) || n < 0 || (n > 0 && !r)) return -1;
  int64_t total = 0;
  for (int k = 0; k < n; ++k) {
    RotorBox b;
    // the widest band the workspace allows for: eps_h <= 4 cells
    if (!rotor_box(d, r[k], 0.5 * 4.0 + 1.0, &b, &why, true)) return -1;
    total += int64_t(b.bn[0]) * b.bn[1] * b.bn[2];
  }
  return total;
}

int hlbm_lattice_create(const hlbm_desc* d, void* pop_a, void* pop_b, void* ws, hlbm_handle* out) {
  std::string why;
  if (!out) return fail(nullptr, HLBM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!desc_ok(d, &why)) return fail(nullptr, HLBM_ERR_INVALID, why);
  if (!pop_a || !pop_b || !ws) return fail(nullptr, HLBM_ERR_INVALID, "population or workspace pointer is NULL");
  if (pop_a == pop_b) return fail(nullptr, HLBM_ERR_INVALID, "the two population buffers must differ");
  hlbm_handle h = new hlbm_lattice();
  h->desc = *d;
  h->stream = static_cast<hipStream_t>(d->stream);
  h->lay = layout(d);
  h->pop[0] = pop_a;
  h->pop[1] = pop_b;
  h->hist_cap = d->history > 0 ? d->history : 1024;
  char* base = static_cast<char*>(ws);
  Launch& L = h->L;
  L.stream = h->stream;
  L.storage = d->storage;
  L.compute = d->compute;
  L.q = vel_of(d);
  L.g.nx = d->nx; L.g.ny = d->ny; L.g.nz = d->nz; L.g.bc_x = d->bc_x;
  L.g.N = cells_of(d);
  L.g.row = pop_row(d);
  L.g.ntx = (d->nx + kTileX - 1) / kTileX;
  L.g.nty = (d->ny + kTileY - 1) / kTileY;
  L.nblocks = int64_t(L.g.ntx) * L.g.nty * d->nz;
  L.g.by_ntx = make_udiv(uint32_t(L.g.ntx));
  set_tile_band(&L.g, tile_band(d, L.g.nty));
  L.sweep_lds = sweep_lds(d, int64_t(L.g.ntx) * L.g.nty * L.g.nz);
  L.g.by_span = make_udiv(8u * uint32_t(L.g.ntx));
  L.g.grouped = uint32_t(L.nblocks / (8 * int64_t(L.g.ntx)) * (8 * int64_t(L.g.ntx)));
  const Layout& Y = h->lay;
  h->ws = base;
  h->set[0] = {base + Y.d_eff, reinterpret_cast<uint8_t*>(base + Y.tag), reinterpret_cast<double*>(base + Y.geo),
               reinterpret_cast<int32_t*>(base + Y.wlist)};
  h->set[1] = {base + Y.d_effb, reinterpret_cast<uint8_t*>(base + Y.tagb), reinterpret_cast<double*>(base + Y.geob),
               reinterpret_cast<int32_t*>(base + Y.wlistb)};
  L.d_eff = h->set[0].d_eff;
  L.d_static = base + Y.d_static;
  L.tag = h->set[0].tag;
  L.tag_static = reinterpret_cast<uint8_t*>(base + Y.tag_static);
  L.uB_static = nullptr;
  L.dd = nullptr;
  L.blk_slot = reinterpret_cast<int32_t*>(base + Y.blk);
  L.partial = reinterpret_cast<double*>(base + Y.partial);
  L.part_l1 = reinterpret_cast<double*>(base + Y.partl1);
  L.mass_part = reinterpret_cast<double*>(base + Y.mass);
  L.mass_l1 = reinterpret_cast<double*>(base + Y.massl1);
  L.wlist = h->set[0].wlist;
  L.wcount = reinterpret_cast<int32_t*>(base + Y.wcount);
  L.flag = reinterpret_cast<int32_t*>(base + Y.flag);
  L.stats = reinterpret_cast<unsigned long long*>(base + Y.stats);
  L.rot = reinterpret_cast<RotorTable*>(base + Y.rot);
  L.nrot = 0;
  L.bbox_total = 0;
  L.geo = h->set[0].geo;
  h->ut[0] = reinterpret_cast<double*>(base + Y.ut0);
  h->ut[1] = reinterpret_cast<double*>(base + Y.ut1);
  h->act[0] = reinterpret_cast<uint8_t*>(base + Y.act0);
  h->act[1] = reinterpret_cast<uint8_t*>(base + Y.act1);
  h->act[2] = reinterpret_cast<uint8_t*>(base + Y.act2);
  L.wall_out = base + Y.wall;
  L.hist = reinterpret_cast<double*>(base + Y.hist);
  L.hist_cap = h->hist_cap;
  const bool with_me = (d->flags & HLBM_WITH_MOMENTUM_EXCHANGE) != 0;
  const bool with_fd = (d->flags & HLBM_WITH_FD_STRAIN) != 0;
  L.fsi_tiles = (with_me || with_fd) ? reinterpret_cast<int32_t*>(base + Y.fsi_tiles) : nullptr;
  L.near_index = with_fd ? reinterpret_cast<int32_t*>(base + Y.near_index) : nullptr;
  L.fd_u = with_fd ? base + Y.fd_u : nullptr;
  L.nnear = 0;
  L.me_partial = with_me ? reinterpret_cast<double*>(base + Y.me_partial) : nullptr;
  L.me_l1 = with_me ? reinterpret_cast<double*>(base + Y.me_l1) : nullptr;
  L.hist_me = with_me ? reinterpret_cast<double*>(base + Y.hist_me) : nullptr;
  h->ghost[0] = base + Y.ghost;
  h->ghost[1] = base + Y.ghostb;
  h->ghost64[0] = reinterpret_cast<double*>(base + Y.ghost64);
  h->ghost64[1] = reinterpret_cast<double*>(base + Y.ghost64b);
  if (L.compute == HLBM_F64) {
    h->ghost64[0] = reinterpret_cast<double*>(h->ghost[0]);
    h->ghost64[1] = reinterpret_cast<double*>(h->ghost[1]);
  }
  L.ghost = h->ghost[0];
  L.ghost64 = h->ghost64[0];
  L.trig_tab = d->bbox_cells > 0 ? reinterpret_cast<BladeTrig*>(base + Y.trig) : nullptr;
  L.dyn = d->bbox_cells > 0 ? reinterpret_cast<RotorDyn*>(base + Y.dyn) : nullptr;
  h->gmark = d->bbox_cells > 0 ? reinterpret_cast<long long*>(base + Y.gmark) : nullptr;
  L.gmark = nullptr;
  L.ggen = 0;
  L.guse = 0;
  L.gstats = d->bbox_cells > 0 ? reinterpret_cast<unsigned long long*>(base + Y.gstats) : nullptr;
  // opt-in: on MI355X marking the layer costs more than the distance
  // evaluations it saves (the fused wall-and-geometry launch took 31.3 us
  // with it and 24.5 us without at 256x128x128, 190 and 179 us at
  // 1536x768x256)
  if (const char* g = std::getenv("HLBM_GROWTH_LAYER")) h->growth_env = std::strcmp(g, "1") == 0;
  // defaults: Smagorinsky-free BGK-like relaxation at tau0 = 1 until set_params
  hlbm_params p{};
  p.tau0 = 1.0; p.cs_smag = 0.0; p.eps_h = 2.0; p.transition = HLBM_TRANSITION_TANH; p.wall_model = 0;
  p.E = 9.8; p.kappa = 0.41; p.y_s = 3.0; p.tol = 1e-4; p.maxit = 10; p.diag_every = 1;
  h->params = p;
  set_model(h);
  for (int k = 0; k < kTags; ++k) {
    h->rot.tag2rot[k] = -1;
    h->rot.frame[k][0] = 0.5 * (d->nx - 1); h->rot.frame[k][1] = 0.5 * (d->ny - 1); h->rot.frame[k][2] = 0.5 * (d->nz - 1);
    h->rot.frame[k][3] = 1; h->rot.frame[k][4] = 0; h->rot.frame[k][5] = 0;
  }
  h->rot.n = 0;
  hipError_t e = hipMemsetAsync(ws, 0, Y.total, h->stream);
  if (e == hipSuccess) e = launch_fill_rest(L, h->pop[0]);
  if (e == hipSuccess) e = launch_fill_rest(L, h->pop[1]);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    hip_fail(nullptr, e, "create");
    delete h;
    return HLBM_ERR_HIP;
  }
  int rc = upload_rotors(h);
  if (rc == HLBM_OK) rc = rebuild_slots(h);
  if (rc != HLBM_OK) {
    g_create_error = h->err;
    delete h;
    return rc;
  }
  *out = h;
  return HLBM_OK;
}

void hlbm_lattice_destroy(hlbm_handle h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  for (auto& v : h->prof)
    for (auto& p : v) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  for (auto e : h->pool) (void)hipEventDestroy(e);
  if (h->trig_ev) (void)hipEventDestroy(h->trig_ev);
  if (h->trig_host) {
    if (h->static_dev >= 0) delete[] h->trig_host;
    else (void)hipHostFree(h->trig_host);
  }
  if (h->static_dev >= 0) static_release(h->static_dev);
  delete h;
}

int hlbm_lattice_create_static(const hlbm_desc* d, void* pop_a, void* pop_b, hlbm_handle* out) {
  std::string why;
  if (!out) return fail(nullptr, HLBM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!desc_ok(d, &why)) return fail(nullptr, HLBM_ERR_INVALID, why);
  const int64_t need = layout(d).total;
  if (need > kStaticWorkspaceBytes)
    return fail(nullptr, HLBM_ERR_INVALID,
                "lattice needs " + std::to_string(need) + " bytes of workspace; the static workspace holds " +
                    std::to_string(kStaticWorkspaceBytes) + " (use hlbm_lattice_create with a workspace buffer)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "create static");
  if (!static_claim(dev)) return fail(nullptr, HLBM_ERR_STATE, "another lattice uses the static workspace of this device");
  void* ws = nullptr;
  e = static_workspace(&ws);
  if (e != hipSuccess) {
    static_release(dev);
    return hip_fail(nullptr, e, "static workspace address");
  }
  const int rc = hlbm_lattice_create(d, pop_a, pop_b, ws, out);
  if (rc != HLBM_OK) {
    static_release(dev);
    return rc;
  }
  (*out)->static_dev = dev;
  return HLBM_OK;
}

int hlbm_set_params(hlbm_handle h, const hlbm_params* p) {
  if (!h) return HLBM_ERR_INVALID;
  std::string why;
  if (!params_ok(p, &why)) return fail(h, HLBM_ERR_INVALID, why);
  if ((p->force_mode & 1) && !(h->desc.flags & HLBM_WITH_MOMENTUM_EXCHANGE))
    return fail(h, HLBM_ERR_STATE, "force_mode 1 needs a lattice created with HLBM_WITH_MOMENTUM_EXCHANGE");
  if (p->fd_share > 0.0 && !(h->desc.flags & HLBM_WITH_FD_STRAIN))
    return fail(h, HLBM_ERR_STATE, "fd_share > 0 needs a lattice created with HLBM_WITH_FD_STRAIN");
  const hlbm_params old = h->params;
  h->params = *p;
  if (!h->rotors.empty()) {
    RotorTable t;
    int64_t total;
    int rc = build_rotor_table(h, h->rotors.data(), int32_t(h->rotors.size()), &t, &total);
    if (rc != HLBM_OK) { h->params = old; return rc; }
    // the boxes depend on eps_h (transition band) and the marking boxes on
    // the wall model's probe reach: when they move, the per-cell wall state
    // follows its cells into the new slots, cells of the old boxes return to
    // the static field, and the wall lists restart
    const bool moved = !same_boxes(h->rot, t);
    const RotorTable old_t = h->rot;
    const int64_t old_total = h->L.bbox_total;
    if (moved && (rc = remap_wall_state(h, old_t, old_total, t, total)) != HLBM_OK) return rc;
    h->rot = t;
    h->L.bbox_total = total;
    if (moved) {
      hipError_t e = refill_porosity(h);
      if (e == hipSuccess) e = reset_counters(h);
      if (e != hipSuccess) return hip_fail(h, e, "reset rotor boxes");
    }
    if ((rc = upload_rotors(h)) != HLBM_OK) return rc;
    if ((rc = rebuild_slots(h)) != HLBM_OK) return rc;
  }
  set_model(h);
  growth_update(h);
  h->have_params = true;
  h->ahead_step = -1;
  h->rec.valid = false;
  return HLBM_OK;
}

int hlbm_set_rotors(hlbm_handle h, const hlbm_rotor* r, int32_t n) {
  if (!h) return HLBM_ERR_INVALID;
  if (n < 0 || n > HLBM_MAX_ROTORS || (n > 0 && !r)) return fail(h, HLBM_ERR_INVALID, "0 <= n <= 8 rotors");
  RotorTable t;
  int64_t total;
  int rc = build_rotor_table(h, r, n, &t, &total);
  if (rc != HLBM_OK) return rc;
  h->rot = t;
  h->trig_base = -1;  // the blade angles change with the rotors
  h->coupled = false;
  for (int k = 0; k < n; ++k) h->coupled = h->coupled || r[k].inertia > 0;
  if ((rc = restart_rotation(h)) != HLBM_OK) return rc;
  h->rotors.assign(r, r + n);
  h->L.nrot = n;
  h->L.bbox_total = total;
  growth_update(h);
  // reset cells of the old boxes to the static field, then re-mark
  hipError_t e = refill_porosity(h);
  if (e != hipSuccess) return hip_fail(h, e, "refill porosity");
  for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipMemsetAsync(h->act[k], 0, std::max<int64_t>(total, 1), h->stream);
  if (e == hipSuccess) e = reset_counters(h);
  if (e != hipSuccess) return hip_fail(h, e, "reset wall state");
  h->rec.valid = false;
  if ((rc = upload_rotors(h)) != HLBM_OK) return rc;
  return rebuild_slots(h);
}

int hlbm_set_rotor_grid(hlbm_handle h, int32_t rotor, const double* phi, int32_t n0, int32_t n1, int32_t n2,
                        double spacing, const double* origin) {
  if (!h) return HLBM_ERR_INVALID;
  if (rotor < 0 || rotor >= HLBM_MAX_ROTORS) return fail(h, HLBM_ERR_INVALID, "rotor index out of range");
  hlbm_lattice::GridRef G;
  if (phi) {
    if (n0 < 2 || n1 < 2 || n2 < 2 || int64_t(n0) * n1 * n2 > (int64_t(1) << 31))
      return fail(h, HLBM_ERR_INVALID, "reference grid needs 2 <= n0, n1, n2 and fewer than 2^31 samples");
    if (!(spacing > 0.0) || !std::isfinite(spacing) || !origin)
      return fail(h, HLBM_ERR_INVALID, "reference grid needs spacing > 0 and an origin");
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(origin[a])) return fail(h, HLBM_ERR_INVALID, "reference grid origin not finite");
    G.phi = phi;
    G.n[0] = n0; G.n[1] = n1; G.n[2] = n2;
    G.h = spacing;
    for (int a = 0; a < 3; ++a) G.o[a] = origin[a];
  }
  const hlbm_lattice::GridRef old = h->grids[rotor];
  h->grids[rotor] = G;
  if (rotor < int32_t(h->rotors.size())) {
    const std::vector<hlbm_rotor> r = h->rotors;
    const int rc = hlbm_set_rotors(h, r.data(), int32_t(r.size()));
    if (rc != HLBM_OK) h->grids[rotor] = old;
    return rc;
  }
  return HLBM_OK;
}

int hlbm_set_porosity_field(hlbm_handle h, const void* d, const uint8_t* tag) {
  if (!h) return HLBM_ERR_INVALID;
  const int64_t N = h->L.g.N;
  const int cs = elem_size(h->desc.compute);
  hipError_t e = d ? hipMemcpyAsync(h->L.d_static, d, N * cs, hipMemcpyDeviceToDevice, h->stream)
                   : hipMemsetAsync(h->L.d_static, 0, N * cs, h->stream);
  if (e == hipSuccess)
    e = tag ? hipMemcpyAsync(h->L.tag_static, tag, N, hipMemcpyDeviceToDevice, h->stream)
            : hipMemsetAsync(h->L.tag_static, 0, N, h->stream);
  if (e == hipSuccess) e = refill_porosity(h);
  if (e != hipSuccess) return hip_fail(h, e, "set porosity field");
  h->rec.valid = false;
  return rebuild_slots(h);
}

int hlbm_set_solid_velocity(hlbm_handle h, const void* uB) {
  if (!h) return HLBM_ERR_INVALID;
  if (!(h->desc.flags & HLBM_WITH_SOLID_VELOCITY)) return fail(h, HLBM_ERR_STATE, "created without HLBM_WITH_SOLID_VELOCITY");
  const int64_t bytes = 3 * h->L.g.N * elem_size(h->desc.compute);
  void* dst = h->ws + h->lay.uB;
  hipError_t e = uB ? hipMemcpyAsync(dst, uB, bytes, hipMemcpyDeviceToDevice, h->stream)
                    : hipMemsetAsync(dst, 0, bytes, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "set solid velocity");
  h->L.uB_static = uB ? dst : nullptr;
  return HLBM_OK;
}

int hlbm_set_control(hlbm_handle h, const void* dd) {
  if (!h) return HLBM_ERR_INVALID;
  if (!(h->desc.flags & HLBM_WITH_CONTROL)) return fail(h, HLBM_ERR_STATE, "created without HLBM_WITH_CONTROL");
  const int64_t bytes = h->L.g.N * elem_size(h->desc.compute);
  void* dst = h->ws + h->lay.dd;
  hipError_t e = dd ? hipMemcpyAsync(dst, dd, bytes, hipMemcpyDeviceToDevice, h->stream)
                    : hipMemsetAsync(dst, 0, bytes, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "set control");
  h->L.dd = dd ? dst : nullptr;
  e = refill_porosity(h);
  if (e != hipSuccess) return hip_fail(h, e, "refill porosity");
  h->rec.valid = false;  // a recorded forward run belongs to the old control
  return rebuild_slots(h);
}

int hlbm_set_tag_frame(hlbm_handle h, int32_t tag, const double center[3], const double axis[3]) {
  if (!h) return HLBM_ERR_INVALID;
  if (tag < 1 || tag > 15 || !center || !axis) return fail(h, HLBM_ERR_INVALID, "tag must be 1..15");
  if (h->rot.tag2rot[tag] >= 0) return fail(h, HLBM_ERR_INVALID, "tag belongs to a rotor");
  const double n = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
  if (!(n > 0)) return fail(h, HLBM_ERR_INVALID, "axis is zero");
  for (int a = 0; a < 3; ++a) { h->rot.frame[tag][a] = center[a]; h->rot.frame[tag][3 + a] = axis[a] / n; }
  return upload_rotors(h);
}

int hlbm_init_equilibrium(hlbm_handle h, const void* rho, const void* u) {
  if (!h) return HLBM_ERR_INVALID;
  hipError_t e = launch_init_equilibrium(h->L, h->pop[h->cur], rho, u);
  const int64_t B = std::max<int64_t>(h->L.bbox_total, 1);
  for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipMemsetAsync(h->act[k], 0, B, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "init equilibrium");
  h->ahead_step = -1;
  h->step = 0;
  h->hist_start = 0;
  h->rec.valid = false;
  ++h->gen;
  if (h->coupled) {
    int rc = restart_rotation(h);
    if (rc == HLBM_OK) rc = upload_rotors(h);
    if (rc != HLBM_OK) return rc;
  }
  return HLBM_OK;
}

}  // extern "C"

namespace {
// cos / sin of every blade angle phase0 + omega n + 2 pi b / n_blades at step n
BladeTrig blade_trig(hlbm_handle h, int64_t n) {
  BladeTrig t{};
  for (int k = 0; k < h->rot.n; ++k) {
    const RotorDev& r = h->rot.r[k];
    for (int b = 0; b < r.nb; ++b) {
      const double th = r.phase0 + r.omega * double(n) + 6.283185307179586476925286766559 * double(b) / double(r.nb);
      t.c[k][b] = std::cos(th);
      t.s[k][b] = std::sin(th);
    }
  }
  return t;
}

// Blade angles of step n on the device: the table holds kTrigSteps steps
// from trig_base; a step outside it reloads the table (host cos / sin, one
// asynchronous copy from a pinned buffer) from step n, or up to step n when
// n lies before the table, as in the reverse sweep of the adjoint.
hipError_t trig_of(hlbm_handle h, int64_t n, const BladeTrig** out) {
  *out = nullptr;
  if (h->rot.n == 0 || !h->L.trig_tab) return hipSuccess;
  if (h->coupled) {
    // written on the device for steps step and step + 1 (no adjoint with coupling)
    *out = h->L.dyn->trig + (n & 1);
    return hipSuccess;
  }
  if (h->trig_base < 0 || n < h->trig_base || n >= h->trig_base + kTrigSteps) {
    hipError_t e = hipSuccess;
    if (!h->trig_host) {
      // a lattice on the static workspace stages from ordinary host memory
      // (it makes no HIP allocation)
      if (h->static_dev >= 0) h->trig_host = new BladeTrig[kTrigSteps];
      else e = hipHostMalloc(reinterpret_cast<void**>(&h->trig_host), sizeof(BladeTrig) * kTrigSteps, 0);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&h->trig_ev, hipEventDisableTiming);
    } else {
      e = hipEventSynchronize(h->trig_ev);  // the previous copy has read the buffer
    }
    if (e != hipSuccess) return e;
    const int64_t base = (h->trig_base >= 0 && n < h->trig_base) ? std::max<int64_t>(0, n - (kTrigSteps - 1)) : n;
    for (int k = 0; k < kTrigSteps; ++k) h->trig_host[k] = blade_trig(h, base + k);
    e = hipMemcpyAsync(h->L.trig_tab, h->trig_host, sizeof(BladeTrig) * kTrigSteps, hipMemcpyHostToDevice,
                       h->stream);
    if (e == hipSuccess) e = hipEventRecord(h->trig_ev, h->stream);
    if (e != hipSuccess) return e;
    h->trig_base = base;
  }
  *out = h->L.trig_tab + (n - h->trig_base);
  return hipSuccess;
}

hipEvent_t take_event(hlbm_handle h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run one launch, bracketed by events when profiling is on.
template <class F>
hipError_t timed(hlbm_handle h, int kind, F&& f) {
  if (!h->profiling) return f();
  hipStream_t s = h->stream;
  hipEvent_t a = take_event(h), b = take_event(h);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e == hipSuccess) e = f();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  h->prof[kind].push_back({a, b});
  return e;
}
// Force / torque / mass records of the pending steps (one reduction launch
// pair for all of them).
hipError_t flush(hlbm_handle h) {
  if (h->pending == 0) return hipSuccess;
  const int32_t cnt = h->pending;
  h->pending = 0;
  return timed(h, HLBM_KERNEL_OTHER, [&] {
    return launch_finalize(h->L, h->pend_n0, cnt, h->nslots, h->params.diag_every,
                           (h->params.force_mode & 1) ? h->nme : -1);
  });
}

// A wall-model probe (and the pull around it) can reach the inflow plane
// when a rotor's marking box touches x = 0.
bool probe_reaches_inlet(hlbm_handle h) {
  if (h->L.g.bc_x == 0 || !h->params.wall_model) return false;
  for (int k = 0; k < h->rot.n; ++k)
    if (h->rot.r[k].mb0[0] <= 0) return true;
  return false;
}

// One forward step n from state `src` to `dst` with the wall-model state
// (ut_prev, act_prev) -> (ut_new, act_new): inflow plane, geometry (unless
// the previous step's wall-model launch computed it), wall model, sweep.
// act_ahead (nullable): the activity buffer of the state after the next
// step; given, the wall-model launch also computes the geometry of step
// n + 1, which resets it.
hipError_t forward_one(hlbm_handle h, int64_t n, const void* src, void* dst, const double* ut_prev,
                       const uint8_t* act_prev, double* ut_new, uint8_t* act_new, uint8_t* act_ahead,
                       bool record = true) {
  select_step(h, n);
  const bool diag = record && h->params.diag_every > 0 && n % h->params.diag_every == 0;
  const bool wall = h->params.wall_model && h->L.nrot > 0;
  // the inflow plane is written by the geometry launch, unless a wall-model
  // probe can reach the inlet: then it must be complete before the wall launch
  const bool inlet = probe_reaches_inlet(h);
  hipError_t e = hipSuccess;
  if (inlet) e = timed(h, HLBM_KERNEL_OTHER, [&] { return launch_prologue(h->L, n); });
  int epoch = h->ahead_epoch;
  if (h->ahead_step != n) {
    const BladeTrig* trig = nullptr;
    if (e == hipSuccess) e = trig_of(h, n, &trig);
    epoch = next_epoch(h);
    if (e == hipSuccess)
      e = timed(h, HLBM_KERNEL_RASTERIZE, [&] {
        growth_for(h, &h->L, n);
        return launch_geometry(h->L, n, trig, epoch, act_new, !inlet);
      });
  }
  h->ahead_step = -1;
  if (e == hipSuccess && wall) {
    NextGeometry ng{};
    Launch L1;
    if (act_ahead) {
      const BladeTrig* trig1 = nullptr;
      e = trig_of(h, n + 1, &trig1);
      L1 = launch_of(h, n + 1);
      growth_for(h, &L1, n + 1);
      ng = NextGeometry{&L1, n + 1, trig1, next_epoch(h), act_ahead, !inlet};
    }
    if (e == hipSuccess)
      e = timed(h, HLBM_KERNEL_WALL, [&] {
        return launch_wall(h->L, src, ut_prev, act_prev, ut_new, act_new, epoch, nullptr, diag ? 1 : 0,
                           act_ahead ? &ng : nullptr);
      });
    if (e == hipSuccess && act_ahead) {
      h->ahead_step = n + 1;
      h->ahead_epoch = ng.epoch;
    }
  }
  if (e == hipSuccess && h->params.fd_share > 0.0)
    e = timed(h, HLBM_KERNEL_OTHER, [&] { return launch_fd_velocity(h->L, src, n); });
  if (!record) {
    // a recomputed step: its records exist, the partials go unreduced
    if (e == hipSuccess) e = timed(h, HLBM_KERNEL_SWEEP, [&] { return launch_sweep(h->L, src, dst, n, false, false); });
    return e;
  }
  // force partials (and mass partials of a diagnostics step) into this step's slice
  if (e == hipSuccess && h->pending == h->batch) e = flush(h);
  if (h->pending == 0) h->pend_n0 = n;
  const int32_t j = h->pending;
  Launch Ls = h->L;
  Ls.partial = h->L.partial + int64_t(j) * std::max<int32_t>(h->nslots, 1) * kPartial;
  Ls.mass_part = h->L.mass_part + int64_t(j) * h->L.nblocks;
  const bool check = diag || h->params.check_nonfinite;
  if (e == hipSuccess) e = timed(h, HLBM_KERNEL_SWEEP, [&] { return launch_sweep(Ls, src, dst, n, diag, check); });
  if (e == hipSuccess && (h->params.force_mode & 1)) {
    double* mp = h->L.me_partial + int64_t(j) * std::max<int32_t>(h->nme, 1) * kMePartial;
    e = timed(h, HLBM_KERNEL_OTHER, [&] { return launch_momentum_exchange(h->L, dst, h->nme, mp); });
  }
  if (e == hipSuccess) ++h->pending;
  // a coupled rotor turns with this step's torque before the next step starts
  if (e == hipSuccess && h->coupled) {
    e = flush(h);
    if (e == hipSuccess) e = timed(h, HLBM_KERNEL_OTHER, [&] { return launch_couple(h->L, n, n + 1); });
  }
  return e;
}

int check_flag(hlbm_handle h) {
  int32_t flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, h->L.flag, 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "read non-finite flag");
  if (flag) {
    (void)hipMemsetAsync(h->L.flag, 0, 4, h->stream);
    return fail(h, HLBM_ERR_NONFINITE, "non-finite density before step " + std::to_string(h->step));
  }
  return HLBM_OK;
}

// Restartable state in the checkpoint / stack layout: populations, u_tau, active.
struct StateLayout {
  int64_t pops, ut, act, bytes;
};
StateLayout state_layout(hlbm_handle h) {
  StateLayout s;
  const int64_t B = h->L.bbox_total;
  s.pops = pop_elems(&h->desc) * elem_size(h->desc.storage);
  s.ut = align_up(s.pops, 256);
  s.act = s.ut + align_up(B * 8, 256);
  s.bytes = s.act + align_up(std::max<int64_t>(B, 1), 256);
  return s;
}

hipError_t copy_state_out(hlbm_handle h, char* dst) {
  const StateLayout s = state_layout(h);
  const int64_t B = h->L.bbox_total;
  hipError_t e = hipMemcpyAsync(dst, h->pop[h->cur], s.pops, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess && B) e = hipMemcpyAsync(dst + s.ut, h->ut[h->wcur], B * 8, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess && B) e = hipMemcpyAsync(dst + s.act, h->act[h->acur], B, hipMemcpyDeviceToDevice, h->stream);
  return e;
}

// Axial torque of the selected tags in a history record.
double axial_torque(hlbm_handle h, const double* rec, int32_t obj_tag) {
  double J = 0.0;
  for (int t = 1; t < kTags; ++t) {
    if (obj_tag != 0 && obj_tag != t) continue;
    const double* T = rec + 4 + 6 * (t - 1);
    J += h->rot.frame[t][3] * T[0] + h->rot.frame[t][4] * T[1] + h->rot.frame[t][5] * T[2];
  }
  return J;
}
}  // namespace

extern "C" {

}  // extern "C"

namespace {
// One recorded step of the lattice state (reductions left pending).
hipError_t step_one(hlbm_handle h) {
  const bool wall = h->params.wall_model && h->L.nrot > 0;
  const int a1 = (h->acur + 1) % 3, a2 = (h->acur + 2) % 3;
  hipError_t e = forward_one(h, h->step, h->pop[h->cur], h->pop[1 - h->cur], h->ut[h->wcur], h->act[h->acur],
                             h->ut[1 - h->wcur], h->act[a1], wall ? h->act[a2] : nullptr);
  if (e != hipSuccess) return e;
  h->cur = 1 - h->cur;
  if (wall) {
    h->wcur = 1 - h->wcur;
    h->acur = a1;
  }
  ++h->step;
  return hipSuccess;
}
}  // namespace

extern "C" {

int hlbm_step(hlbm_handle h, int64_t n) {
  if (!h) return HLBM_ERR_INVALID;
  if (n < 0) return fail(h, HLBM_ERR_INVALID, "n must be >= 0");
  for (int64_t k = 0; k < n; ++k) {
    hipError_t e = step_one(h);
    if (e != hipSuccess) return hip_fail(h, e, "step");
  }
  hipError_t ef = flush(h);
  if (ef != hipSuccess) return hip_fail(h, ef, "step");
  h->rec.valid = false;
  if (h->params.check_nonfinite) return check_flag(h);
  return HLBM_OK;
}

int64_t hlbm_checkpoint_bytes(hlbm_handle h, int64_t nsteps, int32_t ckpt_every) {
  if (!h || nsteps < 1 || ckpt_every < 1) return -1;
  return ((nsteps + ckpt_every - 1) / ckpt_every) * state_layout(h).bytes;
}

int64_t hlbm_adjoint_stack_bytes(hlbm_handle h, int32_t ckpt_every) {
  if (!h || ckpt_every < 1) return -1;
  return int64_t(ckpt_every) * state_layout(h).bytes;
}

int hlbm_forward_record(hlbm_handle h, int64_t nsteps, int64_t t0, int64_t t1, int32_t obj_tag, int32_t ckpt_every,
                        void* ckpt, int64_t ckpt_bytes, double* J) {
  if (!h) return HLBM_ERR_INVALID;
  if (!(h->desc.flags & HLBM_WITH_ADJOINT)) return fail(h, HLBM_ERR_STATE, "created without HLBM_WITH_ADJOINT");
  if (nsteps < 1 || t0 < 0 || t1 <= t0 || t1 > nsteps || ckpt_every < 1 || obj_tag < 0 || obj_tag > 15 || !ckpt || !J)
    return fail(h, HLBM_ERR_INVALID, "need 0 <= t0 < t1 <= nsteps, ckpt_every >= 1, 0 <= obj_tag <= 15");
  if (h->coupled) return fail(h, HLBM_ERR_STATE, "the adjoint is written for prescribed rotor rotations");
  if (ckpt_bytes < hlbm_checkpoint_bytes(h, nsteps, ckpt_every))
    return fail(h, HLBM_ERR_INVALID, "checkpoint buffer too small");
  const StateLayout sl = state_layout(h);
  const int64_t n0 = h->step;
  // steps run without synchronizing (reductions batched as in hlbm_step);
  // the window's records are read once per chunk of half the history ring
  const int64_t chunk = std::max<int64_t>(1, h->hist_cap / 2);
  std::vector<double> rec(size_t(std::min(chunk, nsteps)) * kHist);
  double acc = 0.0;
  int64_t done = 0;
  while (done < nsteps) {
    const int64_t m = std::min(chunk, nsteps - done);
    for (int64_t k = done; k < done + m; ++k) {
      if (k % ckpt_every == 0) {
        hipError_t e = copy_state_out(h, static_cast<char*>(ckpt) + (k / ckpt_every) * sl.bytes);
        if (e != hipSuccess) return hip_fail(h, e, "checkpoint");
      }
      hipError_t e = step_one(h);
      if (e != hipSuccess) return hip_fail(h, e, "forward record");
    }
    hipError_t e = flush(h);
    if (e != hipSuccess) return hip_fail(h, e, "forward record");
    // objective from the FP64 history of the chunk, summed in step order
    const int64_t lo = std::max(done, t0), hi = std::min(done + m, t1);
    if (hi > lo) {
      int rc = hlbm_history(h, n0 + lo, n0 + hi, rec.data());
      if (rc != HLBM_OK) return rc;
      for (int64_t k = lo; k < hi; ++k) acc += axial_torque(h, rec.data() + (k - lo) * kHist, obj_tag);
    }
    done += m;
  }
  if (h->params.check_nonfinite) {
    const int rc = check_flag(h);
    if (rc != HLBM_OK) return rc;
  }
  h->rec.valid = true;
  h->rec.n0 = n0;
  h->rec.nsteps = nsteps;
  h->rec.t0 = t0;
  h->rec.t1 = t1;
  h->rec.obj_tag = obj_tag;
  h->rec.ckpt_every = ckpt_every;
  h->rec.ckpt = static_cast<char*>(ckpt);
  h->rec.J = acc / double(t1 - t0);
  *J = h->rec.J;
  return HLBM_OK;
}

int hlbm_adjoint(hlbm_handle h, double gJ, double* G, void* stack, int64_t stack_bytes) {
  if (!h) return HLBM_ERR_INVALID;
  if (!h->rec.valid || h->step != h->rec.n0 + h->rec.nsteps)
    return fail(h, HLBM_ERR_STATE, "hlbm_adjoint needs a preceding hlbm_forward_record and no steps since");
  const int32_t ce = h->rec.ckpt_every;
  if (!G || !stack || stack_bytes < hlbm_adjoint_stack_bytes(h, ce))
    return fail(h, HLBM_ERR_INVALID, "G or stack missing, or stack too small");
  const StateLayout sl = state_layout(h);
  const Layout& Y = h->lay;
  char* ws = h->ws;
  void* lam[2] = {ws + Y.lam0, ws + Y.lam1};
  double* utb[2] = {reinterpret_cast<double*>(ws + Y.utb0), reinterpret_cast<double*>(ws + Y.utb1)};
  unsigned long long* ubar = reinterpret_cast<unsigned long long*>(ws + Y.ubar);
  void* side[2] = {ws + Y.side, ws + Y.sideb};
  double* scr_ut = reinterpret_cast<double*>(ws + Y.scr_ut);
  // activity written by the wall model of a reverse step, by step parity
  uint8_t* scr_act[2] = {reinterpret_cast<uint8_t*>(ws + Y.scr_act), reinterpret_cast<uint8_t*>(ws + Y.scr_actb)};
  const int64_t N = h->L.g.N, B = std::max<int64_t>(h->L.bbox_total, 1);
  const bool wall = h->params.wall_model && h->L.nrot > 0;
  const int cs = elem_size(h->desc.compute);
  const int64_t lam_bytes = pop_elems(&h->desc) * cs;
  hipError_t e = flush(h);
  if (e == hipSuccess) e = hipMemsetAsync(lam[0], 0, lam_bytes, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(utb[0], 0, B * 8, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(utb[1], 0, B * 8, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(ubar, 0, 9 * N * 8, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(G, 0, N * 8, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "adjoint init");
  const int64_t nseg = (h->rec.nsteps + ce - 1) / ce;
  int cur = 0;
  // the outflow share of lam (side) of the previous reverse step, if any
  bool have_side = false;
  const double w = gJ / double(h->rec.t1 - h->rec.t0);
  char* st = static_cast<char*>(stack);
  h->ahead_step = -1;
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t a = seg * ce, b = std::min<int64_t>(h->rec.nsteps, a + ce);
    // recompute the states of the segment into the stack; each wall-model
    // launch also computes the next step's geometry, the last one that of the
    // first reverse step
    e = hipMemcpyAsync(st, h->rec.ckpt + seg * sl.bytes, sl.bytes, hipMemcpyDeviceToDevice, h->stream);
    for (int64_t k = a; e == hipSuccess && k + 1 < b; ++k) {
      char* s0 = st + (k - a) * sl.bytes;
      char* s1 = s0 + sl.bytes;
      uint8_t* ahead = k + 2 < b ? reinterpret_cast<uint8_t*>(s1 + sl.bytes + sl.act) : scr_act[(h->rec.n0 + k + 1) & 1];
      e = forward_one(h, h->rec.n0 + k, s0, s1, reinterpret_cast<double*>(s0 + sl.ut),
                      reinterpret_cast<uint8_t*>(s0 + sl.act), reinterpret_cast<double*>(s1 + sl.ut),
                      reinterpret_cast<uint8_t*>(s1 + sl.act), wall ? ahead : nullptr, false);
    }
    if (e != hipSuccess) return hip_fail(h, e, "adjoint recompute");
    for (int64_t k = b - 1; k >= a; --k) {
      const int64_t n = h->rec.n0 + k;
      char* s0 = st + (k - a) * sl.bytes;
      const double* ut0 = reinterpret_cast<const double*>(s0 + sl.ut);
      const uint8_t* ac0 = reinterpret_cast<const uint8_t*>(s0 + sl.act);
      AdjLaunch A{};
      A.src = s0;
      A.lam_in = lam[cur];
      A.lam_out = lam[1 - cur];
      A.side = side[cur];
      A.side_in = have_side ? side[1 - cur] : nullptr;
      A.ubar = ubar;
      A.G = G;
      A.ut_bar_in = utb[cur];
      A.ut_bar_out = utb[1 - cur];
      A.obj_w = (k >= h->rec.t0 && k < h->rec.t1) ? w : 0.0;
      A.obj_tag = h->rec.obj_tag;
      // the adjoint of u_tau read by this step is consumed: zero it for the
      // writes of the next reverse step
      A.zero = wall ? utb[cur] : nullptr;
      A.nzero = B;
      // geometry and inflow of step n (unless computed ahead), then the wall
      // model with its adjoint, and the geometry of step n - 1 when it is in
      // this segment
      select_step(h, n);
      const bool inlet = probe_reaches_inlet(h);
      if (inlet) e = launch_prologue(h->L, n);
      int epoch = h->ahead_epoch;
      if (h->ahead_step != n) {
        const BladeTrig* trig = nullptr;
        if (e == hipSuccess) e = trig_of(h, n, &trig);
        epoch = next_epoch(h);
        growth_for(h, &h->L, n);
        if (e == hipSuccess) e = launch_geometry(h->L, n, trig, epoch, scr_act[n & 1], !inlet);
      }
      h->ahead_step = -1;
      if (e == hipSuccess && wall) {
        NextGeometry ng{};
        Launch L1;
        if (k > a) {
          const BladeTrig* trig1 = nullptr;
          e = trig_of(h, n - 1, &trig1);
          L1 = launch_of(h, n - 1);
          growth_for(h, &L1, n - 1);
          ng = NextGeometry{&L1, n - 1, trig1, next_epoch(h), scr_act[(n - 1) & 1], !inlet};
        }
        if (e == hipSuccess)
          e = launch_wall(h->L, s0, ut0, ac0, scr_ut, scr_act[n & 1], epoch, &A, 0, k > a ? &ng : nullptr);
        if (e == hipSuccess && k > a) {
          h->ahead_step = n - 1;
          h->ahead_epoch = ng.epoch;
        }
      }
      // the strain of the hybrid cells: velocity adjoints of their neighbours
      if (e == hipSuccess && h->params.fd_share > 0.0) {
        e = launch_fd_velocity(h->L, s0, n);
        if (e == hipSuccess) e = launch_adjoint_fd(h->L, A);
      }
      if (e == hipSuccess) e = launch_adjoint_sweep(h->L, A);
      if (e != hipSuccess) return hip_fail(h, e, "adjoint step");
      have_side = h->L.g.bc_x != 0;
      cur = 1 - cur;
    }
  }
  h->ahead_step = -1;
  int32_t flag = 0;
  e = hipMemcpyAsync(&flag, h->L.flag, 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "adjoint");
  if (flag & 2) {
    (void)hipMemsetAsync(h->L.flag, 0, 4, h->stream);
    return fail(h, HLBM_ERR_NONFINITE, "a probe-velocity adjoint is non-finite or beyond 2^40");
  }
  return HLBM_OK;
}

int64_t hlbm_get_step(hlbm_handle h) { return h ? h->step : -1; }

int hlbm_moments(hlbm_handle h, void* rho, void* u, void* uhat) {
  if (!h) return HLBM_ERR_INVALID;
  if (!rho || !u) return fail(h, HLBM_ERR_INVALID, "rho and u are required");
  const bool wall = h->params.wall_model && h->L.nrot > 0;
  select_step(h, h->step);
  const BladeTrig* trig = nullptr;
  hipError_t e = trig_of(h, h->step, &trig);
  const bool inlet = probe_reaches_inlet(h);
  if (e == hipSuccess && inlet) e = launch_prologue(h->L, h->step);
  // the wall model writes the next state slot, which is not committed here;
  // the geometry is computed afresh (and any computed ahead is dropped)
  h->ahead_step = -1;
  uint8_t* act_next = h->act[(h->acur + 1) % 3];
  const int epoch = next_epoch(h);
  growth_for(h, &h->L, h->step);
  if (e == hipSuccess) e = launch_geometry(h->L, h->step, trig, epoch, act_next, !inlet);
  if (e == hipSuccess && wall)
    e = launch_wall(h->L, h->pop[h->cur], h->ut[h->wcur], h->act[h->acur], h->ut[1 - h->wcur], act_next, epoch,
                    nullptr, 0);
  if (e == hipSuccess) e = launch_moments(h->L, h->pop[h->cur], h->step, rho, u, uhat);
  if (e != hipSuccess) return hip_fail(h, e, "moments");
  return HLBM_OK;
}

int hlbm_get_populations(hlbm_handle h, double* dst) {
  if (!h || !dst) return h ? fail(h, HLBM_ERR_INVALID, "dst is NULL") : HLBM_ERR_INVALID;
  hipError_t e = launch_get_populations(h->L, h->pop[h->cur], dst);
  if (e != hipSuccess) return hip_fail(h, e, "get populations");
  return HLBM_OK;
}

int hlbm_set_populations(hlbm_handle h, const double* src) {
  if (!h || !src) return h ? fail(h, HLBM_ERR_INVALID, "src is NULL") : HLBM_ERR_INVALID;
  hipError_t e = launch_set_populations(h->L, h->pop[h->cur], src);
  if (e != hipSuccess) return hip_fail(h, e, "set populations");
  h->rec.valid = false;
  return HLBM_OK;
}

int hlbm_get_populations_at(hlbm_handle h, const int64_t* cells, int64_t count, double* dst) {
  if (!h) return HLBM_ERR_INVALID;
  if (count < 0 || (count > 0 && (!cells || !dst))) return fail(h, HLBM_ERR_INVALID, "bad cell list");
  hipError_t e = launch_get_populations_at(h->L, h->pop[h->cur], cells, count, dst);
  if (e != hipSuccess) return hip_fail(h, e, "get populations at");
  return HLBM_OK;
}

// state blob: [int64 step, int64 bbox_total, magic, coupled, pad to 128, FP64 theta[8] omega[8]]
// [populations][u_tau][active]
int64_t hlbm_state_bytes(hlbm_handle h) {
  if (!h) return -1;
  const int64_t B = h->L.bbox_total;
  return 256 + pop_elems(&h->desc) * elem_size(h->desc.storage) + align_up(B * 8, 256) + align_up(B, 256);
}

int hlbm_get_state(hlbm_handle h, void* dst) {
  if (!h || !dst) return h ? fail(h, HLBM_ERR_INVALID, "dst is NULL") : HLBM_ERR_INVALID;
  char* p = static_cast<char*>(dst);
  const int64_t B = h->L.bbox_total;
  const int64_t pb = pop_elems(&h->desc) * elem_size(h->desc.storage);
  int64_t head[32] = {0};
  head[0] = h->step;
  head[1] = B;
  head[2] = 0x484c424d;  // "HLBM"
  head[3] = h->coupled ? 1 : 0;
  hipError_t e = hipMemcpyAsync(p, head, sizeof(head), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess && h->L.dyn)
    e = hipMemcpyAsync(p + 128, h->L.dyn, 2 * kMaxRotors * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(p + 256, h->pop[h->cur], pb, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess && B)
    e = hipMemcpyAsync(p + 256 + pb, h->ut[h->wcur], B * 8, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess && B)
    e = hipMemcpyAsync(p + 256 + pb + align_up(B * 8, 256), h->act[h->acur], B, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "get state");
  return HLBM_OK;
}

int hlbm_set_state(hlbm_handle h, const void* src) {
  if (!h || !src) return h ? fail(h, HLBM_ERR_INVALID, "src is NULL") : HLBM_ERR_INVALID;
  const char* p = static_cast<const char*>(src);
  int64_t head[32];
  hipError_t e = hipMemcpyAsync(head, p, sizeof(head), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "read state header");
  const int64_t B = h->L.bbox_total;
  if (head[2] != 0x484c424d || head[1] != B) return fail(h, HLBM_ERR_INVALID, "state blob does not match this lattice");
  const int64_t pb = pop_elems(&h->desc) * elem_size(h->desc.storage);
  e = hipMemcpyAsync(h->pop[h->cur], p + 256, pb, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess && B) e = hipMemcpyAsync(h->ut[h->wcur], p + 256 + pb, B * 8, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess && B)
    e = hipMemcpyAsync(h->act[h->acur], p + 256 + pb + align_up(B * 8, 256), B, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "set state");
  h->ahead_step = -1;
  h->step = head[0];
  h->hist_start = head[0];
  h->rec.valid = false;
  ++h->gen;
  if (h->coupled) {
    // the rotation saved with the state, or a restart from phase0 and omega
    // for a state saved without coupled rotors
    int rc = HLBM_OK;
    if (head[3]) {
      e = hipMemcpyAsync(h->L.dyn, p + 128, 2 * kMaxRotors * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "set rotor state");
    } else {
      rc = restart_rotation(h);
    }
    if (rc == HLBM_OK) rc = upload_rotors(h);
    if (rc != HLBM_OK) return rc;
  }
  return HLBM_OK;
}

}  // extern "C"

namespace {
// Records [from, to) of a device ring of `cap` records of `width` doubles
// into dst: one copy per contiguous piece of the ring (at most two).
hipError_t copy_ring(hipStream_t stream, const double* ring, int64_t cap, int width, int64_t from, int64_t to,
                     double* dst) {
  for (int64_t s = from; s < to;) {
    const int64_t slot = s % cap, n = std::min(to - s, cap - slot);
    const hipError_t e = hipMemcpyAsync(dst + (s - from) * width, ring + slot * width, n * width * 8,
                                        hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    s += n;
  }
  return hipSuccess;
}
}  // namespace

extern "C" {

int hlbm_history(hlbm_handle h, int64_t from, int64_t to, double* dst) {
  if (!h) return HLBM_ERR_INVALID;
  const int64_t lo = std::max(h->hist_start, h->step - h->hist_cap);
  if (from < lo || to > h->step || from > to || (to > from && !dst))
    return fail(h, HLBM_ERR_INVALID, "steps [" + std::to_string(from) + ", " + std::to_string(to) +
                                         ") not in the history ring [" + std::to_string(lo) + ", " +
                                         std::to_string(h->step) + ")");
  hipError_t e = copy_ring(h->stream, h->L.hist, h->hist_cap, kHist, from, to, dst);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "history");
  return HLBM_OK;
}

int hlbm_history_me(hlbm_handle h, int64_t from, int64_t to, double* dst) {
  if (!h) return HLBM_ERR_INVALID;
  if (!h->L.hist_me) return fail(h, HLBM_ERR_STATE, "created without HLBM_WITH_MOMENTUM_EXCHANGE");
  const int64_t lo = std::max(h->hist_start, h->step - h->hist_cap);
  if (from < lo || to > h->step || from > to || (to > from && !dst))
    return fail(h, HLBM_ERR_INVALID, "steps not in the history ring");
  hipError_t e = flush(h);
  if (e == hipSuccess) e = copy_ring(h->stream, h->L.hist_me, h->hist_cap, kHistMe, from, to, dst);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "momentum-exchange history");
  return HLBM_OK;
}

int hlbm_thrust_coefficient(hlbm_handle h, int32_t tag, int64_t from, int64_t to, int32_t source, double rho,
                            double u_inf, double radius, double* dst) {
  if (!h) return HLBM_ERR_INVALID;
  if (tag < 1 || tag > 15 || (source != 0 && source != 1) || !(rho > 0) || !(u_inf > 0) || !(radius > 0) ||
      (to > from && !dst))
    return fail(h, HLBM_ERR_INVALID, "need tag 1..15, source 0 or 1, rho, u_inf, radius > 0");
  const int64_t n = std::max<int64_t>(0, to - from);
  const int stride = source == 0 ? kHist : kHistMe;
  std::vector<double> rec(std::max<int64_t>(n, 1) * stride);
  const int rc = source == 0 ? hlbm_history(h, from, to, rec.data()) : hlbm_history_me(h, from, to, rec.data());
  if (rc != HLBM_OK) return rc;
  const double* e = &h->rot.frame[tag][3];
  const double q = 0.5 * rho * 3.14159265358979323846 * radius * radius * u_inf * u_inf;
  for (int64_t k = 0; k < n; ++k) {
    const double* F = rec.data() + k * stride + (source == 0 ? 1 + 6 * (tag - 1) : 3 * (tag - 1));
    dst[k] = (e[0] * F[0] + e[1] * F[1] + e[2] * F[2]) / q;
  }
  return HLBM_OK;
}

int hlbm_force_torque(hlbm_handle h, int32_t tag, double F[3], double T[3]) {
  if (!h) return HLBM_ERR_INVALID;
  if (tag < 1 || tag > 15 || !F || !T) return fail(h, HLBM_ERR_INVALID, "tag must be 1..15");
  if (h->step <= h->hist_start) return fail(h, HLBM_ERR_STATE, "no step taken yet");
  double rec[kHist];
  int rc = hlbm_history(h, h->step - 1, h->step, rec);
  if (rc != HLBM_OK) return rc;
  for (int a = 0; a < 3; ++a) { F[a] = rec[1 + 6 * (tag - 1) + a]; T[a] = rec[4 + 6 * (tag - 1) + a]; }
  return HLBM_OK;
}

int hlbm_geometry_stats(hlbm_handle h, int64_t* evaluated, int64_t* visited) {
  if (!h) return HLBM_ERR_INVALID;
  const int64_t nwg = (h->desc.bbox_cells + 255) / 256;
  std::vector<unsigned long long> s(size_t(2 * nwg), 0ull);
  hipError_t e = hipSuccess;
  if (nwg > 0 && h->L.gstats)
    e = hipMemcpyAsync(s.data(), h->L.gstats, sizeof(unsigned long long) * s.size(), hipMemcpyDeviceToHost,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "geometry stats");
  int64_t ev = 0, vis = 0;
  for (int64_t b = 0; b < nwg; ++b) {
    ev += int64_t(s[size_t(2 * b)]);
    vis += int64_t(s[size_t(2 * b + 1)]);
  }
  if (evaluated) *evaluated = ev;
  if (visited) *visited = vis;
  return HLBM_OK;
}

int hlbm_wall_stats(hlbm_handle h, int64_t* iters, int64_t* cells) {
  if (!h) return HLBM_ERR_INVALID;
  unsigned long long s[2];
  hipError_t e = hipMemcpyAsync(s, h->L.stats, sizeof(s), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "wall stats");
  if (iters) *iters = int64_t(s[0]);
  if (cells) *cells = int64_t(s[1]);
  return HLBM_OK;
}

int hlbm_wall_safeguards(hlbm_handle h, int64_t* halvings, int64_t* caps) {
  if (!h) return HLBM_ERR_INVALID;
  unsigned long long s[4];
  hipError_t e = hipMemcpyAsync(s, h->L.stats, sizeof(s), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "wall safeguards");
  if (halvings) *halvings = int64_t(s[2]);
  if (caps) *caps = int64_t(s[3]);
  return HLBM_OK;
}

int hlbm_rotor_state(hlbm_handle h, double* theta, double* omega) {
  if (!h) return HLBM_ERR_INVALID;
  const int n = h->rot.n;
  if (n > 0 && (!theta || !omega)) return fail(h, HLBM_ERR_INVALID, "theta and omega must not be NULL");
  double st[2 * kMaxRotors] = {0};
  if (h->coupled) {
    hipError_t e = hipMemcpyAsync(st, h->L.dyn, sizeof(st), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "rotor state");
  }
  for (int k = 0; k < n; ++k) {
    const RotorDev& r = h->rot.r[k];
    const bool c = r.inertia > 0;
    theta[k] = c ? st[k] : r.phase0 + r.omega * double(h->step);
    omega[k] = c ? st[kMaxRotors + k] : r.omega;
  }
  return n;
}

int hlbm_profile_enable(hlbm_handle h, int32_t enable) {
  if (!h) return HLBM_ERR_INVALID;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "profile enable");
  for (auto& v : h->prof) {
    for (auto& p : v) { h->pool.push_back(p.first); h->pool.push_back(p.second); }
    v.clear();
  }
  h->profiling = enable != 0;
  return HLBM_OK;
}

int hlbm_profile_read(hlbm_handle h, int32_t kernel, int64_t* launches, double* total_ms) {
  if (!h) return HLBM_ERR_INVALID;
  if (kernel < 0 || kernel > 3) return fail(h, HLBM_ERR_INVALID, "unknown kernel class");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "profile read");
  double sum = 0.0;
  for (auto& p : h->prof[kernel]) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, p.first, p.second);
    if (e != hipSuccess) return hip_fail(h, e, "event elapsed time");
    sum += ms;
  }
  if (launches) *launches = int64_t(h->prof[kernel].size());
  if (total_ms) *total_ms = sum;
  return HLBM_OK;
}

int hlbm_sweep_partition(hlbm_handle h, int64_t* fsi_cells, int64_t* bulk_cells) {
  if (!h) return HLBM_ERR_INVALID;
  std::vector<int32_t> slot(h->L.nblocks);
  hipError_t e = hipMemcpyAsync(slot.data(), h->L.blk_slot, sizeof(int32_t) * slot.size(), hipMemcpyDeviceToHost,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "partition");
  const Geometry& g = h->L.g;
  int64_t cnt[2] = {0, 0};
  for (int64_t b = 0; b < h->L.nblocks; ++b) {
    const int64_t tpz = int64_t(g.ntx) * g.nty;
    const int64_t rem = b % tpz;
    const int ty = int(rem / g.ntx), tx = int(rem % g.ntx);
    const int64_t cx = std::min<int64_t>(kTileX, g.nx - int64_t(tx) * kTileX);
    const int64_t cy = std::min<int64_t>(kTileY, g.ny - int64_t(ty) * kTileY);
    cnt[slot[b] >= 0 ? 0 : 1] += cx * cy;
  }
  if (fsi_cells) *fsi_cells = cnt[0];
  if (bulk_cells) *bulk_cells = cnt[1];
  return HLBM_OK;
}

int hlbm_stream_copy(const void* src, void* dst, int64_t bytes, void* stream) {
  if (bytes < 0 || bytes % 16 || (bytes > 0 && (!src || !dst)) || (reinterpret_cast<uintptr_t>(src) & 15) ||
      (reinterpret_cast<uintptr_t>(dst) & 15) || (bytes / 16 + 1023) / 1024 > int64_t(0x7fffffff))
    return HLBM_ERR_INVALID;
  hipError_t e = launch_stream_copy(src, dst, bytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? HLBM_OK : HLBM_ERR_HIP;
}

const char* hlbm_last_error(hlbm_handle h) { return h ? h->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
