/*
 * hlbm.h -- C ABI of the MI355X fused HLBM stream-collide library (libhlbm.so).
 *
 * The library advances the homogenized hybrid recursive-regularized lattice
 * Boltzmann method with Smagorinsky LES and a Spalding wall model on moving
 * porous rotors ("Efficient Wall-Modelled Large Eddy Simulation of Rotors
 * using Homogenized Lattice Boltzmann Methods", Sec. 2.2 eq. hlbm, Sec. 2.2.1,
 * Sec. 2.2.2, Sec. 3) on a D3Q27 lattice or on the paper's D3Q19 lattice
 * (Sec. 2.2, Fig. 2), on one gfx950 GPU.
 *
 * Conventions used by every entry point:
 *  - Cells (x, y, z), x fastest; linear cell index c = (z*ny + y)*nx + x.
 *    Fields are stored component-major: a 3-vector field is [3][nz][ny][nx].
 *  - Velocities c_i in {-1,0,1}^3, canonical order i = 9(cx+1)+3(cy+1)+(cz+1),
 *    opposite of i is 26-i, rest population 13; weights 8/27, 2/27, 1/54,
 *    1/216 by |c_i|^2 = 0, 1, 2, 3; lattice units dx = dt = 1, cs^2 = 1/3.
 *    D3Q19 (hlbm_desc.velocities = 19): the same order restricted to the 19
 *    velocities with |c_i|^2 <= 2 (index k = 0..18, opposite 18-k, rest 9),
 *    weights 1/3, 1/18, 1/36; its third-order Hermite terms are the
 *    projection onto H_aab + H_ccb and H_aab - H_ccb.
 *  - State between steps: the post-collision populations f*_i(x) of the
 *    previous step.  Step n pulls f_i(x, n) = f*_i(x - c_i) (the streaming of
 *    eq. hlbm), applies the outer boundaries, collides and stores f*(x).
 *    Canonical population arrays exchanged through this ABI hold
 *    h_i(x) = f*_i(x) - w_i in FP64, layout [q][nz][ny][nx] (q = 27 or 19).
 *  - Porosity convention of eq. convexVelocity: d = 1 solid, d = 0 fluid.
 *  - "device" pointers are HIP device memory on the lattice's device; "host"
 *    pointers are ordinary host memory.  The library never frees memory it
 *    did not allocate; all device memory is owned by the caller.
 *  - Every call returns HLBM_OK (0) or an error code; the message of the last
 *    error is available from hlbm_last_error().  Nothing throws across the
 *    ABI.  One handle may be used by one host thread at a time.
 *  - All work is enqueued on the stream given at creation; calls that return
 *    data to host memory synchronize that stream.
 */
#ifndef HLBM_H
#define HLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HLBM_Q 27
#define HLBM_MAX_ROTORS 8
#define HLBM_MAX_BLADES 8
#define HLBM_NUM_TAGS 16          /* tags 1..15 name solid elements; 0 = none */
#define HLBM_HIST_STRIDE 91       /* per step: mass, then (F[3], T[3]) for tags 1..15 */

enum hlbm_status {
  HLBM_OK = 0,
  HLBM_ERR_INVALID = 1,     /* bad argument or size; nothing was changed */
  HLBM_ERR_HIP = 2,         /* a HIP runtime call failed */
  HLBM_ERR_NONFINITE = 3,   /* a non-finite density was detected by the step */
  HLBM_ERR_STATE = 4        /* call not valid in the handle's current state */
};

enum hlbm_dtype { HLBM_F64 = 0, HLBM_F32 = 1, HLBM_F16 = 2, HLBM_BF16 = 3 };
enum hlbm_bc { HLBM_BC_PERIODIC = 0, HLBM_BC_INFLOW_OUTFLOW = 1 };
enum hlbm_transition { HLBM_TRANSITION_TANH = 0, HLBM_TRANSITION_LINEAR = 1 };

/* Optional workspace sections requested at creation. */
#define HLBM_WITH_SOLID_VELOCITY 1   /* reserve a static solid-velocity field */
#define HLBM_WITH_CONTROL 2          /* reserve a porosity control field (adjoint) */
#define HLBM_WITH_ADJOINT 4          /* reserve the discrete-adjoint work arrays */
#define HLBM_WITH_MOMENTUM_EXCHANGE 8 /* reserve the momentum-exchange force arrays */
#define HLBM_WITH_FD_STRAIN 16        /* reserve the finite-difference strain arrays */

typedef struct hlbm_lattice* hlbm_handle;

/* Lattice description.  storage: type of the stored populations (FP16/BF16
 * only with compute = HLBM_F32); compute: arithmetic type of the sweep
 * (HLBM_F64 or HLBM_F32).  bc_x: x faces periodic, or equilibrium inflow at
 * x = 0 and zero-gradient outflow at x = nx-1 (y and z are periodic).
 * velocities: 27 (or 0) for D3Q27, 19 for D3Q19.
 * bbox_cells: total cells of the rotors' bounding boxes the workspace must
 * hold (from hlbm_rotor_bbox_cells); history: steps kept in the force ring. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t storage;
  int32_t compute;
  int32_t bc_x;
  int32_t flags;
  int32_t velocities;
  int64_t bbox_cells;
  int64_t history;
  void* stream;              /* hipStream_t; NULL = the null stream */
} hlbm_desc;

/* Model parameters (Sec. 2.2, 2.2.1, 2.2.2).  tau0 > 1/2 molecular relaxation
 * time; cs_smag Smagorinsky constant; eps_h transition width of the lattice
 * porosity; transition HLBM_TRANSITION_*; wall model E, kappa, sampling
 * distance y_s, Newton tolerance tol on |f(u^{j+1}) - f(u^j)| and iteration
 * cap maxit; u_in inflow velocity, turb_I inflow turbulence intensity and its
 * seed; diag_every: every k-th step also reduces the total mass and checks
 * for non-finite densities (0 = never); check_nonfinite: every step checks
 * for non-finite densities (whatever diag_every is), and hlbm_step
 * synchronizes at its end and reports HLBM_ERR_NONFINITE; force_mode bit 0:
 * every step also records the momentum-exchange force of every element
 * (hlbm_history_me; needs HLBM_WITH_MOMENTUM_EXCHANGE); fd_share: the
 * hybrid non-equilibrium of Sec. 2.2, f~(1) = sigma f(1) - (1 - sigma)
 * f(1,FD), in the cells of an element (tag != 0) that are not active wall
 * cells, with sigma = 1 - fd_share and f(1,FD) from the central-difference
 * strain of the pre-collision velocity (y, z periodic; x periodic or clamped
 * to the first and last plane); 0 (the default) keeps sigma = 1 there;
 * fd_share > 0 needs HLBM_WITH_FD_STRAIN. */
typedef struct {
  double tau0, cs_smag, eps_h;
  int32_t transition, wall_model;
  double E, kappa, y_s, tol;
  int32_t maxit, diag_every;
  double u_in[3];
  double turb_I;
  uint64_t seed;
  int32_t check_nonfinite, force_mode;
  double fd_share;
} hlbm_params;

/* Rotor of n_blades flat-plate blades (chord x thick, from r_hub to R,
 * pitch twisted linearly from twist_root to twist_tip, radians) and a hub
 * sphere of radius r_hub, turning about axis through center at omega
 * rad/step from phase0; its cells carry tag (1..15).
 * inertia = 0: prescribed rotation, angle phase0 + omega n at step n.
 * inertia > 0: two-way coupling (the structure update of the FSI time loop,
 * Sec. 3.2, as a rigid rotation about the fixed axis): from angle phase0
 * and speed omega at the step hlbm_set_rotors is called, each step n turns
 * the rotor by theta_{n+1} = theta_n + Omega_n and drives it by the axial
 * torque e . T_n the fluid handed to it (hlbm_force_torque) against the
 * generator torque torque_gen: Omega_{n+1} = Omega_n + (e . T_n -
 * torque_gen) / inertia, all on the device.  The explicit update is stable
 * while inertia exceeds about half the moment of inertia of the fluid the
 * blades displace (added mass). */
typedef struct {
  double center[3], axis[3];
  double R, r_hub, chord, thick, twist_root, twist_tip, omega, phase0;
  int32_t n_blades, tag;
  double inertia, torque_gen;
} hlbm_rotor;

/* Bytes of one population buffer.  Its layout is internal (the canonical
 * arrays go through hlbm_get/set_populations): each (y, z) row is cut into
 * blocks of 64 consecutive x cells holding the q populations of those cells
 * as q runs of 64 values, the last block padded. */
int64_t hlbm_population_bytes(const hlbm_desc* desc);
/* Bytes of the workspace for this description. */
int64_t hlbm_workspace_bytes(const hlbm_desc* desc);
/* Cells of the fixed bounding boxes of these rotors (value for desc->bbox_cells). */
int64_t hlbm_rotor_bbox_cells(const hlbm_desc* desc, const hlbm_rotor* rotors, int32_t n);

/* Create a lattice on the current HIP device.  pop_a, pop_b: device buffers of
 * hlbm_population_bytes each; workspace: device buffer of
 * hlbm_workspace_bytes.  The handle borrows them until destroy.  The
 * lattice starts at rest (f* = w), step 0, no solids.  The environment
 * variable HLBM_TILE_BAND (a positive integer), read here, overrides the
 * number of tile rows per band of the sweep's tile order (for
 * measurements); results do not depend on it. */
int hlbm_lattice_create(const hlbm_desc* desc, void* pop_a, void* pop_b, void* workspace,
                        hlbm_handle* out);
/* Destroy a handle; never frees caller memory.  NULL is a no-op. */
void hlbm_lattice_destroy(hlbm_handle h);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as hlbm_lattice_create, but the workspace is the library's own static
 * device array of HLBM_STATIC_WORKSPACE_BYTES (32 MiB) on the current
 * device, which each device holds until the process ends.  No call on the
 * returned handle allocates device or pinned host memory.  The caller still
 * passes both population buffers.  HLBM_ERR_INVALID when
 * hlbm_workspace_bytes(desc) exceeds the array; HLBM_ERR_STATE while
 * another lattice on the device uses it (one at a time per device:
 * hlbm_lattice_destroy frees it for the next one).  The array keeps the
 * previous lattice's contents; creation clears it. */
#define HLBM_STATIC_WORKSPACE_BYTES (32 << 20)
int hlbm_lattice_create_static(const hlbm_desc* desc, void* pop_a, void* pop_b, hlbm_handle* out);

/* Parameters (validated: tau0 > 1/2, cs_smag >= 0, eps_h > 0, maxit >= 1).
 * With rotors set, a change of eps_h, y_s or the wall-model switch can move
 * the rotors' fixed boxes: cells leaving them return to the static field,
 * and the per-cell wall-model state (u_tau^prev, active, Sec. 2.2.1) of
 * every cell stays with that cell.  Invalidates a forward record. */
int hlbm_set_params(hlbm_handle h, const hlbm_params* p);

/* Rotors rasterized on the GPU every step (Sec. 3.1); n <= HLBM_MAX_ROTORS,
 * tags distinct, n_blades <= HLBM_MAX_BLADES, bounding boxes inside the
 * domain and within desc->bbox_cells.  n = 0 removes all rotors. */
int hlbm_set_rotors(hlbm_handle h, const hlbm_rotor* rotors, int32_t n);

/* Reference grid of rotor index `rotor` (Sec. 3.1: a moving element is
 * voxelized once on its own reference grid, which is embedded into the
 * lattice porosity at the element's position and orientation every step).
 * The grid replaces that rotor's flat-plate blades and hub sphere; its
 * axis, center, rotation, tag and the other rotor fields keep their meaning.
 * phi: device FP64 array [n2][n1][n0] (borrowed until replaced, removed or
 * the handle is destroyed), the signed distance (positive inside) at body
 * coordinates origin + spacing (i0, i1, i2).  Body axes: 0 the radial
 * direction of blade 0, cos(theta) e1 + sin(theta) e2 at rotor angle theta
 * (e1 the unit projection of x onto the plane normal to the axis, of y when
 * |axis_x| >= 0.9, e2 = axis x e1); 1 the tangential direction axis x
 * (axis 0); 2 the axis.  Each step the geometry samples phi trilinearly at
 * the body coordinates of the box cells and takes the wall normal from the
 * gradient of that interpolant; a cell off the grid is not in the body.
 * The solid (phi >= 0) must lie within the rotor's envelope (radius
 * sqrt(R^2 + (chord/2)^2 + (thick/2)^2) about the axis, axial half extent
 * max(sqrt((chord/2)^2 + (thick/2)^2), r_hub)), which sizes its box, and the
 * grid must reach eps_h/2 + 1 beyond the solid.  n0, n1, n2 >= 2, spacing >
 * 0, the rotor needs n_blades >= 1 (blade 0 orients the body).  phi = NULL
 * removes the grid.  The grid stays with the rotor index across
 * hlbm_set_rotors calls; when the index holds a rotor, this call re-applies
 * the rotors as hlbm_set_rotors does.  HLBM_ERR_INVALID for bad arguments. */
int hlbm_set_rotor_grid(hlbm_handle h, int32_t rotor, const double* phi, int32_t n0, int32_t n1, int32_t n2,
                        double spacing, const double* origin);

/* Static porosity field: the lattice porosity d of Def. Lattice Porosity
 * (Sec. 2.2.2) entering eq. convexVelocity, device, compute type, N values,
 * 0 <= d <= 1 (1 solid, 0 fluid), and the tag of the solid element each cell
 * belongs to (device, uint8, N values, 0..15; the per-element force and
 * torque of Sec. 2.2.2 sum over one tag); both are copied.  NULL d clears
 * the field (d = 0 everywhere), NULL tag sets tag 0.  Rotor cells override
 * both where a rotor covers them (d = max(static, rotor)).  Invalidates a
 * forward record. */
int hlbm_set_porosity_field(hlbm_handle h, const void* d, const uint8_t* tag);

/* Static solid velocity u^B of eq. convexVelocity (Sec. 2.2: the velocity
 * toward which the porosity drives a cell), device, compute type, [3][N],
 * used where the cell is not covered by a rotor (rotor cells take the rigid
 * rotation Omega e x (x - x_c) of Sec. 3.1); copied.  Needs
 * HLBM_WITH_SOLID_VELOCITY.  NULL resets to zero. */
int hlbm_set_solid_velocity(hlbm_handle h, const void* uB);

/* Porosity control delta_d (device, compute type, N values) added to the
 * porosity of every cell (d = max(d_static, d_rotor) + delta_d); copied.
 * Needs HLBM_WITH_CONTROL.  NULL resets to zero.  Invalidates a forward
 * record. */
int hlbm_set_control(hlbm_handle h, const void* dd);

/* Reference frame (torque centre, axis) of a tag set through the static
 * field; rotor tags use the rotor's centre and axis. */
int hlbm_set_tag_frame(hlbm_handle h, int32_t tag, const double center[3], const double axis[3]);

/* f* = f^eq(rho, u) (the third-order equilibrium of Sec. 2.2) in every
 * cell; rho (N) and u ([3][N]) device, compute type; NULL rho = 1, NULL u =
 * 0.  Resets the step counter, the wall-model state and the history. */
int hlbm_init_equilibrium(hlbm_handle h, const void* rho, const void* u);

/* Advance n >= 0 steps (asynchronous unless check_nonfinite is set).  A
 * step is the algorithm of Sec. 3.2: rotor geometry, wall model, fused
 * stream-collide sweep with force records.  The wall-model launch of each
 * step also computes the geometry of the next one (kept for the next call
 * unless a call in between changes the geometry inputs or reads moments);
 * results do not depend on how steps are split over calls. */
int hlbm_step(hlbm_handle h, int64_t n);

/* Current step counter. */
int64_t hlbm_get_step(hlbm_handle h);

/* Density and velocity of the pre-collision populations f(x, n) of the next
 * step (rho N, u [3][N]) and the homogenized velocity u_hat it collides to
 * ([3][N], eq. convexVelocity; nullable); device, compute type.  The lattice
 * state is not changed. */
int hlbm_moments(hlbm_handle h, void* rho, void* u, void* uhat);

/* Canonical state h = f* - w, FP64, device, [q][N]. */
int hlbm_get_populations(hlbm_handle h, double* dst);
int hlbm_set_populations(hlbm_handle h, const double* src);
/* Canonical state at selected cells: dst[k*q + i] for cell cells[k] (both
 * device); NaN for a cell index outside the lattice. */
int hlbm_get_populations_at(hlbm_handle h, const int64_t* cells, int64_t count, double* dst);

/* Complete restartable state (populations in storage format, wall-model
 * state, step counter) as an opaque blob of hlbm_state_bytes bytes (device). */
int64_t hlbm_state_bytes(hlbm_handle h);
int hlbm_get_state(hlbm_handle h, void* dst);
int hlbm_set_state(hlbm_handle h, const void* src);

/* Force F and torque T (about the tag's centre) handed to the solid with
 * this tag by the last step: the per-element force of Sec. 2.2.2 summed per
 * tag as in Sec. 3.1 (here the momentum j - rho u_hat each cell's collision
 * hands to the solid, eq. convexVelocity; T = sum (x - x_c) x that
 * momentum), FP64 sums in a fixed order, host (syncs).  HLBM_ERR_STATE
 * before the first step. */
int hlbm_force_torque(hlbm_handle h, int32_t tag, double F[3], double T[3]);
/* Records of steps [from, to) (absolute step numbers still in the ring),
 * HLBM_HIST_STRIDE doubles each, host (syncs): per step the total mass
 * sum rho, then for tags 1..15 the force and torque of hlbm_force_torque
 * (the per-step force history of the time loop of Sec. 3.2, the thrust and
 * torque histories of Sec. 4).  Mass is NaN on steps without diagnostics.
 * HLBM_ERR_INVALID for steps outside the ring. */
int hlbm_history(hlbm_handle h, int64_t from, int64_t to, double* dst);

/* Discrete adjoint of the time stepping (gradient of the time-averaged
 * rotor torque with respect to the porosity control delta_d), on either
 * velocity set.
 * Objective: J = 1/(t1-t0) sum over steps k in [t0, t1) of the record of
 * the axial torque e_tag . T_tag (obj_tag 0 = all tags), with T from the
 * momentum handed to the solid (Sec. 2.2.2).  Needs HLBM_WITH_ADJOINT.
 * hlbm_forward_record advances nsteps from the current state, storing a
 * restartable state every ckpt_every steps into ckpt (device, at least
 * hlbm_checkpoint_bytes), and returns J (host double).  hlbm_adjoint then
 * writes G = gJ dJ/d(delta_d) (device FP64, N values): it recomputes each
 * segment of ckpt_every steps into stack (device, hlbm_adjoint_stack_bytes)
 * and runs the reverse steps; Newton iterations of the wall model are
 * differentiated as executed, and with fd_share > 0 the central differences
 * of the hybrid cells' strain carry its adjoint to the neighbours'
 * velocities.  Prescribed rotations only: forward_record refuses a coupled
 * rotor (inertia > 0) with HLBM_ERR_STATE.  The lattice state is left
 * unchanged. */
int64_t hlbm_checkpoint_bytes(hlbm_handle h, int64_t nsteps, int32_t ckpt_every);
int64_t hlbm_adjoint_stack_bytes(hlbm_handle h, int32_t ckpt_every);
/* A record is invalidated by any call that steps the lattice or changes its
 * state or inputs (hlbm_step, set_state, set_populations,
 * init_equilibrium, set_params, set_rotors, set_porosity_field,
 * set_control): hlbm_adjoint then returns HLBM_ERR_STATE. */
int hlbm_forward_record(hlbm_handle h, int64_t nsteps, int64_t t0, int64_t t1, int32_t obj_tag, int32_t ckpt_every,
                        void* ckpt, int64_t ckpt_bytes, double* J);
int hlbm_adjoint(hlbm_handle h, double gJ, double* G, void* stack, int64_t stack_bytes);

/* Wall-model counters since creation, accumulated on diagnostics steps
 * (every diag_every-th step): Newton iterations for u_tau and wall cells
 * solved (host, syncs). */
int hlbm_wall_stats(hlbm_handle h, int64_t* newton_iters, int64_t* wall_cells);

/* Momentum-exchange force on each element (Sec. 2.2.2: the paper's
 * momentum-exchange sum after Wen et al., read per link and in its
 * Galilean-invariant form): over the links joining a cell x of tag 0 to a
 * neighbour x_b = x + c_i of tag T, F_T = sum (c_i - u_s) f*_i(x) +
 * (c_i + u_s) f*_ibar(x_b), post-collision populations of the step, u_s the
 * solid velocity at x_b; no links across the x faces of an inflow/outflow
 * lattice; a tag-0 cell next to several elements gives its links to the
 * first of them in velocity order.  It differs from hlbm_force_torque's
 * force (the momentum the collision hands to the solid) by the change of
 * the momentum inside the element, zero in a steady flow.  Records of steps
 * [from, to) in the history ring, 45 doubles each (tags 1..15 x F[3]), FP64
 * host (syncs); recorded while force_mode bit 0 is set, zero otherwise.
 * HLBM_ERR_STATE without HLBM_WITH_MOMENTUM_EXCHANGE. */
int hlbm_history_me(hlbm_handle h, int64_t from, int64_t to, double* dst);

/* Thrust coefficient (Def. Thrust Coefficient, Sec. 4) of element tag per
 * step of [from, to): C_T = T / (0.5 rho pi r^2 U^2) with T the axial force
 * e . F on the element (e the tag frame's axis), F the force of
 * hlbm_force_torque (source 0) or the momentum-exchange force (source 1);
 * rho, u_inf, radius the reference density, free-stream speed and rotor
 * radius (all > 0).  dst: to - from doubles, host (syncs). */
int hlbm_thrust_coefficient(hlbm_handle h, int32_t tag, int64_t from, int64_t to, int32_t source, double rho,
                            double u_inf, double radius, double* dst);

/* Safeguards of the wall model's Newton iterations (Sec. 2.2.1) taken since
 * creation on diagnostics steps: iterates that went non-positive and were
 * replaced by half the previous one, and evaluations whose exponential
 * argument exceeded 80 and took the cap (host, syncs).  Both stay zero on
 * well-posed runs. */
int hlbm_wall_safeguards(hlbm_handle h, int64_t* halvings, int64_t* caps);

/* Rotor geometry work since creation (host, syncs): box slots whose rotor
 * distance was evaluated, and box slots visited, over all geometry
 * launches.  The rasterization (Sec. 3.1) evaluates the distance on every
 * slot of the rotor boxes; with the environment variable
 * HLBM_GROWTH_LAYER=1, read at creation, only on the growth layer of Fig.
 * fsialgo: the cells within one cell of those whose distance lay within one
 * cell of the transition band at the previous step, while every rotor
 * rotates as prescribed with |omega| (R + eps_h/2 + 1) <= 1/2 (the surface
 * moves at most half a cell per step), no rotor has a reference grid (whose
 * interpolant may be steeper than a distance), and the previous step's geometry was
 * computed under the same rotors and parameters.  The result is the same
 * either way; the layer is off by default because marking it costs more
 * than the evaluations it saves. */
int hlbm_geometry_stats(hlbm_handle h, int64_t* evaluated, int64_t* visited);

/* Angle theta (rad) and angular velocity Omega (rad/step) of each rotor at
 * the current step, in the order of hlbm_set_rotors: prescribed rotors
 * phase0 + omega n and omega, coupled ones their state (see hlbm_rotor).
 * theta, omega: host arrays of at least the number of rotors (syncs).
 * Returns the number of rotors, or a negative error code.  The state of
 * coupled rotors travels in hlbm_get_state / hlbm_set_state; hlbm_set_rotors
 * and hlbm_init_equilibrium restart it from phase0 and omega. */
int hlbm_rotor_state(hlbm_handle h, double* theta, double* omega);

/* Opt-in kernel timing with HIP events recorded on the lattice's stream
 * around every launch of the given kernel class during hlbm_step
 * (HLBM_KERNEL_*).  hlbm_profile_enable(h, 1) starts a fresh count;
 * hlbm_profile_read synchronizes and returns the number of timed launches
 * and their summed duration in milliseconds.  For benchmarks and tests. */
/* SWEEP: stream-collide sweep; WALL: wall model (whose launch also computes
 * the rotor geometry and inflow plane of the next step); RASTERIZE: rotor
 * geometry (with the step's inflow plane) launched on its own, which happens
 * on the first step of a run and after a call that changes the geometry
 * inputs, or every step without the wall model; OTHER: batched force
 * reductions and separately launched inflow planes. */
enum hlbm_kernel { HLBM_KERNEL_SWEEP = 0, HLBM_KERNEL_WALL = 1, HLBM_KERNEL_RASTERIZE = 2, HLBM_KERNEL_OTHER = 3 };
int hlbm_profile_enable(hlbm_handle h, int32_t enable);
int hlbm_profile_read(hlbm_handle h, int32_t kernel, int64_t* launches, double* total_ms);
/* Cells of the sweep's porous (FSI) workgroups, which apply porosity, solid
 * and wall-model velocities and reduce the per-tag momentum, and of its
 * plain workgroups (host, syncs). */
int hlbm_sweep_partition(hlbm_handle h, int64_t* fsi_cells, int64_t* bulk_cells);
/* A plain streaming copy of `bytes` bytes from src to dst (device, 16-byte
 * aligned, bytes a multiple of 16, not overlapping), one 16 B element per
 * thread with non-temporal loads and stores, enqueued on `stream`
 * (hipStream_t, NULL = the null stream): the reference of the streaming bandwidth the sweep is measured
 * against in benchmarks.  HLBM_ERR_INVALID for a misaligned or negative
 * size; asynchronous. */
int hlbm_stream_copy(const void* src, void* dst, int64_t bytes, void* stream);

/* Message of the last error of this handle (or of the last failed create
 * when h is NULL).  Valid until the next call on the handle. */
const char* hlbm_last_error(hlbm_handle h);

#ifdef __cplusplus
}
#endif

#endif /* HLBM_H */
