// Host-side launchers of the libhlbm kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hlbm_internal.h"

namespace hlbm {

// Everything a launch needs, with raw device pointers carved from the
// caller's workspace.  Types of the typed fields follow storage / compute.
struct Launch {
  hipStream_t stream;        // the caller's stream
  int storage, compute;      // hlbm_dtype values
  int q;                     // velocity set: 27 or 19
  Geometry g;
  Model m;
  int64_t nblocks;           // sweep workgroups = ntx * nty * nz
  uint32_t sweep_lds;        // dynamic LDS of a sweep workgroup: caps the resident workgroups per CU
  BladeTrig* trig_tab;       // blade angles of kTrigSteps consecutive steps
  RotorDyn* dyn;             // coupled rotation state (nullable)
  // growth layer of the rotor geometry: marks [2][bbox_total] by step
  // parity (null: every box slot is evaluated), the generation of the rotor
  // and parameter state they belong to, and whether this launch reads them
  long long* gmark;
  long long ggen;
  int32_t guse;
  unsigned long long* gstats;  // [2][geometry workgroups]: distances evaluated, slots visited
  // fields
  void* d_eff;
  void* d_static;
  uint8_t* tag;
  uint8_t* tag_static;
  void* uB_static;           // nullable
  void* dd;                  // nullable
  int32_t* blk_slot;
  double* partial;
  double* part_l1;           // [kPartL1][kPartial]
  double* mass_part;
  double* mass_l1;           // [kPartL1]
  // d_eff, tag, geo and wlist point into the buffer set of the step being
  // launched: the sets alternate by step so that the geometry of step n + 1
  // can be written while step n reads its own
  int32_t* wlist;            // wall cells of the step (box slots)
  int32_t* wcount;           // [kCounters] wall-list counters, in turn by launch
  int32_t* flag;
  unsigned long long* stats; // [0] Newton iterations, [1] wall cells, [2] Newton halvings, [3] exponential caps
  RotorTable* rot;           // device copy
  int32_t nrot;
  int64_t bbox_total;
  double* geo;               // [4][bbox_total]: phi, n
  void* wall_out;            // [10][bbox_total] compute type
  double* hist;
  int64_t hist_cap;
  // momentum-exchange force (HLBM_WITH_MOMENTUM_EXCHANGE): the tiles of its
  // launch (lattice-order index; the FSI tiles and their neighbours), their
  // partials by step slice, level-1 results, history ring [hist_cap][kHistMe]
  const int32_t* fsi_tiles;
  // finite-difference strain (HLBM_WITH_FD_STRAIN): index of each tile in
  // that list (-1: not in it) and the pre-collision velocity of its cells,
  // [index][3][kBlock] in the compute type
  int32_t* near_index;
  void* fd_u;
  int32_t nnear;
  double* me_partial;
  double* me_l1;
  double* hist_me;
  void* ghost;               // inflow ghost plane [9][nz][ny], compute type
  double* ghost64;           // same in FP64 for the wall model
};

// Wall-list counters: a geometry launch of epoch e (0 <= e < kCounters)
// counts into counter e and zeroes counter e + 1 (mod kCounters) for the
// next launch.  Three of them let the geometry of one step run beside the
// wall model of the previous one, which still reads its own counter.
constexpr int kCounters = 3;

// Rotor geometry of the step on the box slots and the wall-cell list
// (counter `epoch`); with_ghost: also the step's inflow plane.
hipError_t launch_geometry(const Launch& L, int64_t step, const BladeTrig* trig, int epoch, uint8_t* act_new,
                           bool with_ghost);
// A geometry launch folded into a wall-model launch: the arguments of
// launch_geometry, with L giving the buffer set and inflow plane it writes
// (which the wall model must not read).
struct NextGeometry {
  const Launch* L;
  int64_t step;
  const BladeTrig* trig;
  int epoch;
  uint8_t* act_new;
  bool with_ghost;
};
struct AdjLaunch;
// Wall model of the listed wall cells of `epoch`; adj (nullable): also the
// adjoint wall step of a reverse step; next (nullable): a geometry launch run
// by further workgroups of the same launch.
hipError_t launch_wall(const Launch& L, const void* src, const double* ut_prev, const uint8_t* act_prev,
                       double* ut_new, uint8_t* act_new, int epoch, const AdjLaunch* adj = nullptr,
                       int count_stats = 1, const NextGeometry* next = nullptr);
// Step sweep of every cell: pull, moments, collision (porosity, solid and
// wall-model velocities in the FSI tiles), store, per-tag momentum partials.
// diag: also the step's mass partials; check: raise the non-finite flag for
// a non-finite density.
hipError_t launch_sweep(const Launch& L, const void* src, void* dst, int64_t step, bool diag, bool check);
hipError_t launch_prologue(const Launch& L, int64_t step);
// Records of steps n0 .. n0 + count - 1 from their partial slices (slice j:
// force partials at partial + j nslots kPartial, mass partials at
// mass_part + j nblocks); the mass of the steps that are not diagnostics
// steps is recorded as NaN.
// me_slots >= 0: also the momentum-exchange records from that many slots per step.
hipError_t launch_finalize(const Launch& L, int64_t n0, int32_t count, int32_t nslots, int32_t diag_every,
                           int32_t me_slots);
// Pre-collision velocity of the cells of the listed tiles (for the
// finite-difference strain of the step's sweep).
hipError_t launch_fd_velocity(const Launch& L, const void* src, int64_t step);
// Momentum-exchange partials of the step whose post-collision state is
// `state`, into me_partial (one slot per FSI tile).
hipError_t launch_momentum_exchange(const Launch& L, const void* state, int32_t nslots, double* me_partial);
// Rotor rotation for step m: rec >= 0 first advances every coupled rotor by
// the axial torque of history record rec; then each coupled rotor's speed
// goes into the rotor table and every rotor's blade angles of steps m and
// m + 1 into the parity slots of L.dyn.
hipError_t launch_couple(const Launch& L, int64_t rec, int64_t m);
hipError_t launch_moments(const Launch& L, const void* src, int64_t step, void* rho, void* u, void* uhat);
hipError_t launch_init_equilibrium(const Launch& L, void* dst, const void* rho, const void* u);
hipError_t launch_get_populations(const Launch& L, const void* src, double* dst);
hipError_t launch_set_populations(const Launch& L, void* dst, const double* src);
hipError_t launch_get_populations_at(const Launch& L, const void* src, const int64_t* cells, int64_t count,
                                     double* dst);
hipError_t launch_mark_blocks(const Launch& L);

// One reverse step of the discrete adjoint.
struct AdjLaunch {
  const void* src;          // state at the step (storage type)
  const void* lam_in;       // adjoint of the next state (compute type, blocked layout of the populations)
  void* lam_out;            // adjoint of this state
  void* side;               // outflow side buffer of this step [9][nz][ny]
  const void* side_in;      // that of the next step (added to lam_in on the last plane); nullable
  unsigned long long* ubar; // [9][N] fixed-point probe-velocity adjoints, zero except the wall scatter
  double* G;                // [N] FP64 gradient accumulator
  const double* ut_bar_in;  // adjoint of the friction velocity written by the step
  double* ut_bar_out;       // adjoint of the friction velocity read by the step
  double obj_w;
  int32_t obj_tag;
  double* zero;             // zeroed by the adjoint sweep (nullable), nzero doubles
  int64_t nzero;
};
// The adjoint wall step runs inside launch_wall (adj); with fd_share > 0,
// the velocity adjoints of the finite-difference strain (launch_adjoint_fd,
// after launch_fd_velocity of the step's state); then this sweep.
hipError_t launch_adjoint_fd(const Launch& L, const AdjLaunch& A);
hipError_t launch_adjoint_sweep(const Launch& L, const AdjLaunch& A);
hipError_t launch_refill_porosity(const Launch& L);
// Plain streaming copy (bytes a multiple of 16, 16-byte aligned pointers).
hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t stream);
hipError_t launch_fill_rest(const Launch& L, void* dst);

// Workspace for lattices created without a caller buffer: a file-scope
// device array of kStaticWorkspaceBytes on every GPU the library runs on,
// held until the process ends.  static_workspace returns its device address
// on the current device (looked up once per device).
constexpr int64_t kStaticWorkspaceBytes = int64_t(32) << 20;
hipError_t static_workspace(void** ptr);

}  // namespace hlbm
