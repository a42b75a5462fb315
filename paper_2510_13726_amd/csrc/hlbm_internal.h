// Internal device/host data structures of libhlbm (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlbm {

constexpr int kQ = 27;
constexpr int kTileX = 64;           // sweep workgroup: 64 x-cells (one wave) ...
constexpr int kTileY = 4;            // ... by 4 y-rows (4 waves)
constexpr int kBlock = kTileX * kTileY;
constexpr int kMaxRotors = 8;
constexpr int kMaxBlades = 8;
constexpr int kTags = 16;
constexpr int kHist = 91;            // mass + 15 x (F, T)
constexpr int kPartial = 96;         // per FSI block: [16 tags][F3, T3]
constexpr int kMassL1 = 256;         // first-level mass reduction width
constexpr int kPartL1 = 64;          // first-level force reduction width
constexpr int kMaxBatch = 8;         // steps whose reductions are launched together
constexpr int kWallOut = 10;         // u_wm[3], S[6], sigma per wall slot
constexpr int kMePartial = 48;       // per FSI block: [16 tags][F_ME 3]
constexpr int kHistMe = 45;          // 15 x F_ME

// Tag byte of a cell: bits 0-3 tag, bit 6 = covered by a rotor, bit 7 = wall cell.
constexpr uint8_t kTagMask = 0x0f;
constexpr uint8_t kRotorBit = 0x40;
constexpr uint8_t kWallBit = 0x80;

struct RotorDev {
  double c[3], e[3], e1[3], e2[3];
  double R, r_hub, chord, thick, tw_root, tw_tip, omega, phase0;
  int32_t nb, tag;
  int32_t b0[3], bn[3];   // bounding box origin and extent (cells)
  int32_t mb0[3], mbn[3]; // FSI marking box (box + probe reach, may wrap in y, z)
  int64_t off;            // first slot of this box in the box pools
  int64_t cells;          // bn[0]*bn[1]*bn[2]
  double inertia, tgen;   // coupled rotation (inertia > 0) and its generator torque
  // reference grid of the body (nullable): signed distance [gn2][gn1][gn0]
  // at body coordinates go + gh (i0, i1, i2)
  const double* grid;
  int32_t gn[3], gpad;
  double gh, go[3];
};

struct RotorTable {
  int32_t n;
  int32_t tag2rot[kTags];  // rotor index of a tag, -1 if none
  RotorDev r[kMaxRotors];
  double frame[kTags][6];  // per tag: torque centre, axis
};

struct Model {
  double tau0;
  double smag;         // 18 sqrt(2) C_S^2 (coefficient of the Smagorinsky root)
  double eps_h;
  int32_t transition, wall_model;
  double E, kappa, y_s, tol, nu;
  // reciprocals and ratios for the wall law (one division each, on the host)
  double inv_E, kappa_E, inv_kappa, inv_nu, ys_nu, nu_ys;
  int32_t maxit, pad;
  double u_in[3];
  double turb_amp;     // turb_I * |u_in|
  uint64_t seed;
  double fd_share;     // 1 - sigma off the wall in element cells
};

// Quotient of a 32-bit unsigned dividend by an invariant divisor d > 0 from
// one multiply-high, a subtraction and two shifts, exact for every dividend
// (Granlund and Montgomery, Division by invariant integers using
// multiplication, PLDI 1994, Sec. 4): with l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, t = mulhi(m, n),
// n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0).
struct Udiv {
  uint32_t m, s1, s2;
};
inline Udiv make_udiv(uint32_t d) {
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  // 2^l - d < 2^(l-1), so the product stays below 2^63
  const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
  return Udiv{uint32_t(m), l < 1 ? l : 1u, l > 1 ? l - 1 : 0u};
}
// Fixed-point form of a sum of FP64 values that is independent of the order
// of the terms: a value v with |v| < 2^40 is the integer X = round(v 2^64),
// split by magnitude into 32-bit pieces |X| = P2 2^64 + P1 2^32 + P0 and
// signed like v; each piece is summed in its own int64 accumulator (exact
// for fewer than 2^31 terms).  fix_split returns false (p untouched) for a
// value outside the range or not finite.
__host__ __device__ inline bool fix_split(double v, long long p[3]) {
  constexpr double k32 = 4294967296.0, k64 = 18446744073709551616.0;
  if (!(fabs(v) < 1099511627776.0)) return false;  // 2^40
  const double t = rint(fabs(v) * k64);
  const double p2 = floor(t / k64);
  const double r1 = t - p2 * k64;  // in [0, 2^64), exact
  const double p1 = floor(r1 / k32);
  const double p0 = r1 - p1 * k32;  // in [0, 2^32), exact
  const long long s = v < 0.0 ? -1 : 1;
  p[0] = s * (long long)p2;
  p[1] = s * (long long)p1;
  p[2] = s * (long long)p0;
  return true;
}

// The accumulated sum (s2 2^64 + s1 2^32 + s0) 2^-64 as FP64: the carries
// are normalized into H + F 2^-64 with F in [0, 2^64), and the magnitude is
// converted (one rounding of the fraction relative to the sum).
__host__ __device__ inline double fix_merge(long long s2, long long s1, long long s0) {
  const long long c0 = s0 >> 32;  // floor division by 2^32 (arithmetic shift)
  const unsigned long long l0 = (unsigned long long)(s0 - c0 * 4294967296ll);
  const long long m1 = s1 + c0;
  const long long c1 = m1 >> 32;
  const unsigned long long l1 = (unsigned long long)(m1 - c1 * 4294967296ll);
  const long long H = s2 + c1;
  const unsigned long long F = (l1 << 32) | l0;
  constexpr double k2m64 = 5.42101086242752217e-20;  // 2^-64
  if (H >= 0) return double(H) + double(F) * k2m64;
  if (F == 0) return double(H);
  return -(double(-(H + 1)) + double(0ull - F) * k2m64);
}

__host__ __device__ inline uint32_t udiv(uint32_t n, const Udiv& v) {
  const uint32_t t = uint32_t((uint64_t(v.m) * n) >> 32);
  return (t + ((n - t) >> v.s1)) >> v.s2;
}

struct Geometry {
  int32_t nx, ny, nz, bc_x;
  int64_t N;
  int64_t row;         // population elements per (y, z) row: ntx blocks of 27 x kTileX
  int32_t ntx, nty;    // sweep tiles along x and y
  // Sweep tile order: the rows of tiles along y are cut into bands of `band`
  // rows (the last band holds the remainder); band by band, z by z, the
  // band's rows, x fastest.  band = nty is the plain lattice order (z
  // slowest); band = 1 sweeps each row of tiles through all z.  Divisors:
  // ntx, band ntx, band ntx nz, the last band's rows times ntx, and 8 ntx
  // (eight tile rows); tiles in whole bands, tiles in whole groups of eight
  // rows.
  Udiv by_ntx, by_bandrow, by_band, by_tailrow, by_span;
  uint32_t band, full_tiles;
  uint32_t grouped;
};

// Blocked population layout: a row of the lattice is cut into blocks of
// kTileX consecutive x cells (one sweep wave); a block holds its cells' Q
// populations (27 or 19) as Q runs of kTileX values, so each of a wave's Q
// loads and Q stores touches one contiguous 256-byte run (FP32) of a few
// blocks.  Element (i, x, y, z) of a population buffer:
template <int Q = 27>
__host__ __device__ inline int64_t pop_at(const Geometry& g, int i, int x, int y, int z) {
  return (int64_t(z) * g.ny + y) * g.row + int64_t(x / kTileX) * (Q * kTileX) + i * kTileX + x % kTileX;
}
// Offset of cell x inside its row, population 0 (add i * kTileX for population i).
template <int Q = 27>
__host__ __device__ inline uint32_t pop_x(int x) {
  return uint32_t(x / kTileX) * uint32_t(Q * kTileX) + uint32_t(x % kTileX);
}

// cos and sin of every blade angle of every rotor at the current step
struct BladeTrig {
  double c[kMaxRotors][kMaxBlades];
  double s[kMaxRotors][kMaxBlades];
};
// Steps of blade angles held on the device at once (uploaded in chunks).
constexpr int kTrigSteps = 2048;

// Rotation of two-way coupled rotors, on the device: angle and angular
// velocity of every coupled rotor at the current step, and the blade angles
// of all rotors for the current step and the next, by step parity.
struct RotorDyn {
  double theta[kMaxRotors];
  double omega[kMaxRotors];
  BladeTrig trig[2];
};

}  // namespace hlbm
