// Per-cell arithmetic of the fused HLBM update, in the normalized deviation
// form used for storage: g_i = (f_i - w_i) / w_i.
//
// For the third-order Hermite equilibrium, the recursive-regularized
// non-equilibrium part and the FD part (Sec. 2.2, eq. hlbm and the
// definitions that follow it) the post-collision value divided by w_i is
//
//   f*_i / w_i = rho + 3 rho c.u + H2_i : B2 + H3_i : B3,
//   B2 = 9/2 rho u u + w' (9/2 sigma Pi - 3 (1 - sigma) rho tau S),
//   B3 = 9/2 (rho u u u + w' sigma a3),  a3_abc = u_a Pi_bc + u_b Pi_ac + u_c Pi_ab,
//   w' = 1 - 1/tau,  u = u_hat (eq. convexVelocity),
//
// (1/(2 cs^4) = 1/(6 cs^6) = 9/2 and 1/cs^2 = 3 with cs^2 = 1/3).  On the
// 27-velocity cube H3_aaa = 0, H3_aab = c_b (c_a^2 - 1/3) (three
// permutations) and H3_xyz = c_x c_y c_z (six), so with T_ab = 3 B3_aab
// (a != b), V_b = 3 rho u_b - sum_{a!=b} B3_aab and X = 6 B3_xyz
//
//   g*_i = E0 + sum_a c_a^2 B2_aa + 2 sum_{a<b} c_a c_b B2_ab          (even in c)
//        + sum_b c_b (V_b + sum_{a!=b} c_a^2 T_ab) + c_x c_y c_z X      (odd in c)
//   E0 = (rho - 1) - tr(B2)/3,
//
// evaluated once per pair of opposite velocities.  Everything is a small
// deviation, so FP32 keeps its relative precision.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlbm {

// ---------------------------------------------------------------- lattice
__host__ __device__ constexpr int cx_of(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz_of(int i) { return i % 3 - 1; }
__host__ __device__ constexpr double w_of(int i) {
  return (cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_of(i) * cz_of(i)) == 0   ? 8.0 / 27.0
         : (cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_of(i) * cz_of(i)) == 1 ? 2.0 / 27.0
         : (cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_of(i) * cz_of(i)) == 2 ? 1.0 / 54.0
                                                                                 : 1.0 / 216.0;
}
__host__ __device__ constexpr int idx_of(int cx, int cy, int cz) { return 9 * (cx + 1) + 3 * (cy + 1) + (cz + 1); }

// ---------------------------------------------------------------- storage
// Stored value of g = (f - w)/w: double, float, IEEE half (RNE) or bfloat16
// (RNE on the upper 16 bits of the float).
struct bf16_t { uint16_t bits; };

template <class ST> struct Store;
template <> struct Store<double> {
  template <class CT> __device__ static CT load(const double* p) { return CT(*p); }
  template <class CT> __device__ static void store(double* p, CT v) { __builtin_nontemporal_store(double(v), p); }
};
template <> struct Store<float> {
  template <class CT> __device__ static CT load(const float* p) { return CT(*p); }
  template <class CT> __device__ static void store(float* p, CT v) { __builtin_nontemporal_store(float(v), p); }
};
template <> struct Store<_Float16> {
  template <class CT> __device__ static CT load(const _Float16* p) { return CT(float(*p)); }
  template <class CT> __device__ static void store(_Float16* p, CT v) {
    __builtin_nontemporal_store(_Float16(float(v)), p);
  }
};
template <> struct Store<bf16_t> {
  template <class CT> __device__ static CT load(const bf16_t* p) {
    uint32_t b = uint32_t(*reinterpret_cast<const uint16_t*>(p)) << 16;
    return CT(__uint_as_float(b));
  }
  template <class CT> __device__ static void store(bf16_t* p, CT v) {
    float f = float(v);
    uint32_t b = __float_as_uint(f);
    uint32_t r = (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
    if ((b & 0x7fffffffu) > 0x7f800000u) r = (b >> 16) | 0x40u;  // keep NaN a NaN
    __builtin_nontemporal_store(uint16_t(r), reinterpret_cast<uint16_t*>(p));
  }
};

// Element at a uniform (scalar) base plus a 32-bit per-lane byte offset, so
// the compiler can use the scalar-base + 32-bit-offset global addressing.
template <class T>
__device__ __forceinline__ const T* at_bytes(const T* base, uint32_t byte_off) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ T* at_bytes(T* base, uint32_t byte_off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}

// ---------------------------------------------------------------- moments
// Deviation moments of h_i = f_i - w_i: drho = sum h, j = sum c h,
// p = sum c c h (so P = cs^2 I + p).
template <class CT>
struct Moments {
  CT drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
};

template <class CT>
__device__ __forceinline__ Moments<CT> moments_of(const CT h[27]) {
  // per (cy, cz) column: s = h- + h0 + h+, d = h+ - h-, a = h+ + h-
  CT s[9], d[9], a[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const CT hm = h[k], h0 = h[9 + k], hp = h[18 + k];
    a[k] = hp + hm;
    d[k] = hp - hm;
    s[k] = a[k] + h0;
  }
  Moments<CT> m;
  // k = 3(cy+1) + (cz+1)
  const CT sy_m = s[0] + s[1] + s[2], sy_0 = s[3] + s[4] + s[5], sy_p = s[6] + s[7] + s[8];
  m.drho = sy_m + sy_0 + sy_p;
  m.jy = sy_p - sy_m;
  m.pyy = sy_p + sy_m;
  const CT sz_m = s[0] + s[3] + s[6], sz_p = s[2] + s[5] + s[8];
  m.jz = sz_p - sz_m;
  m.pzz = sz_p + sz_m;
  m.pyz = (s[8] + s[0]) - (s[6] + s[2]);
  const CT dy_m = d[0] + d[1] + d[2], dy_0 = d[3] + d[4] + d[5], dy_p = d[6] + d[7] + d[8];
  m.jx = dy_m + dy_0 + dy_p;
  m.pxy = dy_p - dy_m;
  m.pxz = (d[2] + d[5] + d[8]) - (d[0] + d[3] + d[6]);
  m.pxx = (a[0] + a[1] + a[2]) + (a[3] + a[4] + a[5]) + (a[6] + a[7] + a[8]);
  return m;
}

// ---------------------------------------------------------------- reconstruction
template <class CT>
struct Coef {
  CT E0, Bxx, Byy, Bzz, Dxy, Dxz, Dyz;  // D = 2 B2 off-diagonal
  CT Vx, Vy, Vz;
  CT Tyx, Tzx, Txy, Tzy, Txz, Tyz;      // T_ab, a != b
  CT X;
};

// g*_i for all 27 velocities from the coefficients.
template <class CT>
__device__ __forceinline__ void reconstruct(const Coef<CT>& k, CT g[27]) {
  const CT ex = k.E0 + k.Bxx, ey = k.E0 + k.Byy, ez = k.E0 + k.Bzz;
  // faces
  g[idx_of(1, 0, 0)] = ex + k.Vx; g[idx_of(-1, 0, 0)] = ex - k.Vx;
  g[idx_of(0, 1, 0)] = ey + k.Vy; g[idx_of(0, -1, 0)] = ey - k.Vy;
  g[idx_of(0, 0, 1)] = ez + k.Vz; g[idx_of(0, 0, -1)] = ez - k.Vz;
  g[idx_of(0, 0, 0)] = k.E0;
  // edges
  const CT exy = ex + k.Byy, exz = ex + k.Bzz, eyz = ey + k.Bzz;
  const CT Wxy = k.Vx + k.Tyx, Wyx = k.Vy + k.Txy;
  const CT Wxz = k.Vx + k.Tzx, Wzx = k.Vz + k.Txz;
  const CT Wyz = k.Vy + k.Tzy, Wzy = k.Vz + k.Tyz;
  {
    const CT ep = exy + k.Dxy, em = exy - k.Dxy, op = Wxy + Wyx, om = Wxy - Wyx;
    g[idx_of(1, 1, 0)] = ep + op; g[idx_of(-1, -1, 0)] = ep - op;
    g[idx_of(1, -1, 0)] = em + om; g[idx_of(-1, 1, 0)] = em - om;
  }
  {
    const CT ep = exz + k.Dxz, em = exz - k.Dxz, op = Wxz + Wzx, om = Wxz - Wzx;
    g[idx_of(1, 0, 1)] = ep + op; g[idx_of(-1, 0, -1)] = ep - op;
    g[idx_of(1, 0, -1)] = em + om; g[idx_of(-1, 0, 1)] = em - om;
  }
  {
    const CT ep = eyz + k.Dyz, em = eyz - k.Dyz, op = Wyz + Wzy, om = Wyz - Wzy;
    g[idx_of(0, 1, 1)] = ep + op; g[idx_of(0, -1, -1)] = ep - op;
    g[idx_of(0, 1, -1)] = em + om; g[idx_of(0, -1, 1)] = em - om;
  }
  // corners
  const CT exyz = exy + k.Bzz;
  const CT Kx = Wxy + k.Tzx, Ky = Wyx + k.Tzy, Kz = Wzx + k.Tyz;
  {  // (1,1,1)
    const CT e = exyz + (k.Dxy + k.Dxz + k.Dyz), o = Kx + Ky + Kz + k.X;
    g[idx_of(1, 1, 1)] = e + o; g[idx_of(-1, -1, -1)] = e - o;
  }
  {  // (1,1,-1)
    const CT e = exyz + (k.Dxy - k.Dxz - k.Dyz), o = Kx + Ky - Kz - k.X;
    g[idx_of(1, 1, -1)] = e + o; g[idx_of(-1, -1, 1)] = e - o;
  }
  {  // (1,-1,1)
    const CT e = exyz + (-k.Dxy + k.Dxz - k.Dyz), o = Kx - Ky + Kz - k.X;
    g[idx_of(1, -1, 1)] = e + o; g[idx_of(-1, 1, -1)] = e - o;
  }
  {  // (1,-1,-1)
    const CT e = exyz + (-k.Dxy - k.Dxz + k.Dyz), o = Kx - Ky - Kz + k.X;
    g[idx_of(1, -1, -1)] = e + o; g[idx_of(-1, 1, 1)] = e - o;
  }
}

// Coefficients from rho, u (=u_hat), the symmetric tensor B2 and the third-
// order tensor 9/2 (rho u u u + w' sigma a3) given by its distinct components.
template <class CT>
__device__ __forceinline__ void finish_coef(Coef<CT>& k, CT drho, CT rho, CT ux, CT uy, CT uz,
                                            CT b2xx, CT b2yy, CT b2zz, CT b2xy, CT b2xz, CT b2yz,
                                            CT b3xxy, CT b3xxz, CT b3yyx, CT b3yyz, CT b3zzx, CT b3zzy,
                                            CT b3xyz) {
  k.Bxx = b2xx; k.Byy = b2yy; k.Bzz = b2zz;
  k.Dxy = CT(2) * b2xy; k.Dxz = CT(2) * b2xz; k.Dyz = CT(2) * b2yz;
  k.E0 = drho - (b2xx + b2yy + b2zz) * CT(1.0 / 3.0);
  // T_ab = 3 B3_aab: a = index appearing twice, b = once
  k.Txy = CT(3) * b3xxy; k.Txz = CT(3) * b3xxz;
  k.Tyx = CT(3) * b3yyx; k.Tyz = CT(3) * b3yyz;
  k.Tzx = CT(3) * b3zzx; k.Tzy = CT(3) * b3zzy;
  const CT r3 = CT(3) * rho;
  k.Vx = r3 * ux - (b3yyx + b3zzx);
  k.Vy = r3 * uy - (b3xxy + b3zzy);
  k.Vz = r3 * uz - (b3xxz + b3yyz);
  k.X = CT(6) * b3xyz;
}

// Normalized equilibrium deviation at rho = 1 (inflow ghost).
template <class CT>
__device__ __forceinline__ void equilibrium_dev_unit(CT ux, CT uy, CT uz, CT g[27]) {
  const CT c = CT(4.5);
  Coef<CT> k;
  finish_coef(k, CT(0), CT(1), ux, uy, uz, c * ux * ux, c * uy * uy, c * uz * uz, c * ux * uy, c * ux * uz,
              c * uy * uz, c * ux * ux * uy, c * ux * ux * uz, c * uy * uy * ux, c * uy * uy * uz,
              c * uz * uz * ux, c * uz * uz * uy, c * ux * uy * uz);
  reconstruct(k, g);
}

// Normalized equilibrium deviation at (rho, u).
template <class CT>
__device__ __forceinline__ void equilibrium_dev(CT rho, CT ux, CT uy, CT uz, CT g[27]) {
  const CT c = CT(4.5) * rho;
  Coef<CT> k;
  finish_coef(k, rho - CT(1), rho, ux, uy, uz, c * ux * ux, c * uy * uy, c * uz * uz, c * ux * uy, c * ux * uz,
              c * uy * uz, c * ux * ux * uy, c * ux * ux * uz, c * uy * uy * ux, c * uy * uy * uz,
              c * uz * uz * ux, c * uz * uz * uy, c * ux * uy * uz);
  reconstruct(k, g);
}

// Collision of one cell (Sec. 2.2, eq. hlbm).  Inputs: deviation moments m,
// homogenized velocity (ux, uy, uz), sigma and the wall strain S (used when
// sigma < 1), model constants.  Output: normalized post-collision deviations.
template <class CT, bool kWall>
__device__ __forceinline__ void collide(const Moments<CT>& m, CT rho, CT ux, CT uy, CT uz, CT sigma,
                                        const CT S[6], CT tau0, CT smag, CT g[27]) {
  const CT third = CT(1.0 / 3.0);
  const CT ru_x = rho * ux, ru_y = rho * uy, ru_z = rho * uz;
  const CT dd = m.drho * third;
  // Pi = P - rho cs^2 I - rho u u  with P = cs^2 I + p
  const CT Pxx = m.pxx - dd - ru_x * ux;
  const CT Pyy = m.pyy - dd - ru_y * uy;
  const CT Pzz = m.pzz - dd - ru_z * uz;
  const CT Pxy = m.pxy - ru_x * uy;
  const CT Pxz = m.pxz - ru_x * uz;
  const CT Pyz = m.pyz - ru_y * uz;
  const CT q2 = Pxx * Pxx + Pyy * Pyy + Pzz * Pzz + CT(2) * (Pxy * Pxy + Pxz * Pxz + Pyz * Pyz);
  const CT Q = sqrt(q2);
  const CT tau = CT(0.5) * (tau0 + sqrt(tau0 * tau0 + smag * Q / rho));
  const CT om = CT(1) - CT(1) / tau;
  const CT c45 = CT(4.5);
  CT b2xx, b2yy, b2zz, b2xy, b2xz, b2yz, os;
  if (kWall) {
    os = om * sigma;
    const CT fd = om * CT(3) * (CT(1) - sigma) * rho * tau;
    const CT pi = c45 * os;
    b2xx = c45 * ru_x * ux + pi * Pxx - fd * S[0];
    b2yy = c45 * ru_y * uy + pi * Pyy - fd * S[1];
    b2zz = c45 * ru_z * uz + pi * Pzz - fd * S[2];
    b2xy = c45 * ru_x * uy + pi * Pxy - fd * S[3];
    b2xz = c45 * ru_x * uz + pi * Pxz - fd * S[4];
    b2yz = c45 * ru_y * uz + pi * Pyz - fd * S[5];
  } else {
    os = om;
    b2xx = c45 * (ru_x * ux + om * Pxx);
    b2yy = c45 * (ru_y * uy + om * Pyy);
    b2zz = c45 * (ru_z * uz + om * Pzz);
    b2xy = c45 * (ru_x * uy + om * Pxy);
    b2xz = c45 * (ru_x * uz + om * Pxz);
    b2yz = c45 * (ru_y * uz + om * Pyz);
  }
  // 9/2 (rho u_a u_a u_b + w' sigma (2 u_a Pi_ab + u_b Pi_aa))
  const CT t = c45 * os;
  const CT b3xxy = c45 * ru_x * ux * uy + t * (CT(2) * ux * Pxy + uy * Pxx);
  const CT b3xxz = c45 * ru_x * ux * uz + t * (CT(2) * ux * Pxz + uz * Pxx);
  const CT b3yyx = c45 * ru_y * uy * ux + t * (CT(2) * uy * Pxy + ux * Pyy);
  const CT b3yyz = c45 * ru_y * uy * uz + t * (CT(2) * uy * Pyz + uz * Pyy);
  const CT b3zzx = c45 * ru_z * uz * ux + t * (CT(2) * uz * Pxz + ux * Pzz);
  const CT b3zzy = c45 * ru_z * uz * uy + t * (CT(2) * uz * Pyz + uy * Pzz);
  const CT b3xyz = c45 * ru_x * uy * uz + t * (ux * Pyz + uy * Pxz + uz * Pxy);
  Coef<CT> k;
  finish_coef(k, m.drho, rho, ux, uy, uz, b2xx, b2yy, b2zz, b2xy, b2xz, b2yz, b3xxy, b3xxz, b3yyx, b3yyz, b3zzx,
              b3zzy, b3xyz);
  reconstruct(k, g);
}

// ---------------------------------------------------------------- inflow noise
// splitmix64 output k of the generator seeded with s, and a Box-Muller normal
// from outputs 2j and 2j+1 for counter j = ((n ny + y) nz + z) 3 + comp.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double inflow_normal(uint64_t seed, int64_t n, int y, int z, int comp, int ny, int nz) {
  const uint64_t base =
      ((((uint64_t)n * (uint64_t)ny + (uint64_t)y) * (uint64_t)nz + (uint64_t)z) * 3ULL + (uint64_t)comp) * 2ULL;
  const double u1 = 1.0 - (double)(splitmix64_at(seed, base) >> 11) * 0x1.0p-53;
  const double u2 = (double)(splitmix64_at(seed, base + 1) >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

}  // namespace hlbm
