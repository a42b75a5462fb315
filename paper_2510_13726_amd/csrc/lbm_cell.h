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

// Velocity sets: D3Q27 (index i = idx_of(c)) and D3Q19, the paper's stencil
// (Sec. 2.2, Fig. 2): the 27-velocity order restricted to |c|^2 <= 2,
// weights 1/3, 1/18, 1/36.  k indexes a set's own velocities; opposite of k
// is Q - 1 - k in both.
template <int Q>
__host__ __device__ constexpr int i27_of(int k) {
  if (Q == 27) return k;
  int n = -1;
  for (int i = 0; i < 27; ++i) {
    const int c2 = cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_of(i) * cz_of(i);
    if (c2 <= 2 && ++n == k) return i;
  }
  return -1;
}
template <int Q> __host__ __device__ constexpr int cxq(int k) { return cx_of(i27_of<Q>(k)); }
template <int Q> __host__ __device__ constexpr int cyq(int k) { return cy_of(i27_of<Q>(k)); }
template <int Q> __host__ __device__ constexpr int czq(int k) { return cz_of(i27_of<Q>(k)); }
template <int Q>
__host__ __device__ constexpr double wq(int k) {
  if (Q == 27) return w_of(k);
  const int c2 = cxq<Q>(k) * cxq<Q>(k) + cyq<Q>(k) * cyq<Q>(k) + czq<Q>(k) * czq<Q>(k);
  return c2 == 0 ? 1.0 / 3.0 : c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
}
// Index of velocity (cx, cy, cz) in set Q; -1 if the set does not hold it.
template <int Q>
__host__ __device__ constexpr int kq(int cx, int cy, int cz) {
  for (int k = 0; k < Q; ++k)
    if (cxq<Q>(k) == cx && cyq<Q>(k) == cy && czq<Q>(k) == cz) return k;
  return -1;
}
// First index of the velocities with c_x = j - 1 (they are contiguous).
template <int Q>
__host__ __device__ constexpr int xgroup_of(int j) {
  return Q == 27 ? 9 * j : (j == 0 ? 0 : j == 1 ? 5 : 14);
}

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
  // FP32 -> BF16 in the hardware convert of gfx950 (round to nearest even,
  // a NaN stays a NaN)
  template <class CT> __device__ static void store(bf16_t* p, CT v) {
    const __bf16 b = static_cast<__bf16>(float(v));
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, b), reinterpret_cast<uint16_t*>(p));
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

// ---------------------------------------------------------------- rcp / sqrt
// Reciprocal and square root in the compute type: correctly rounded in FP64;
// in FP32 the hardware approximations (v_rcp_f32, v_sqrt_f32, about 1 ulp),
// far inside the FP32 tolerance and a fraction of the instructions of the
// correctly rounded sequences.
template <class T> __device__ __forceinline__ T rcp_ct(T x) { return T(1) / x; }
template <> __device__ __forceinline__ float rcp_ct<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <class T> __device__ __forceinline__ T sqrt_ct(T x) { return sqrt(x); }
template <> __device__ __forceinline__ float sqrt_ct<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

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

// Deviation moments over the D3Q19 velocities (h indexed by k of set 19).
template <class CT>
__device__ __forceinline__ Moments<CT> moments_of19(const CT h[19]) {
  Moments<CT> m{};
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const int cx = cxq<19>(k), cy = cyq<19>(k), cz = czq<19>(k);
    m.drho += h[k];
    if (cx) m.jx += CT(cx) * h[k];
    if (cy) m.jy += CT(cy) * h[k];
    if (cz) m.jz += CT(cz) * h[k];
    if (cx) m.pxx += h[k];
    if (cy) m.pyy += h[k];
    if (cz) m.pzz += h[k];
    if (cx * cy) m.pxy += CT(cx * cy) * h[k];
    if (cx * cz) m.pxz += CT(cx * cz) * h[k];
    if (cy * cz) m.pyz += CT(cy * cz) * h[k];
  }
  return m;
}
template <int Q, class CT>
__device__ __forceinline__ Moments<CT> moments_q(const CT* h) {
  if constexpr (Q == 27) return moments_of<CT>(h);
  else return moments_of19<CT>(h);
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

// D3Q19 reconstruction.  The 19 velocities do not hold H_xyz, and their
// third-order terms are the projection onto H_aab + H_ccb (norm 2 cs^6) and
// H_aab - H_ccb (norm 6 cs^6), b the odd index: with the same B3 = 9/2 (rho
// u u u + w' sigma a3) as the 27-velocity form this gives, per velocity,
//   face s e_b:            -2 s sum_{a != b} B3_aab
//   edge s_a e_a + s_b e_b: 2 s_b B3_aab + 2 s_a B3_bba
// so g*_i = E0 + sum_a c_a^2 B2_aa + 2 sum_{a<b} c_a c_b B2_ab + 3 rho c.u
// plus those terms.
template <class CT>
__device__ __forceinline__ void reconstruct19(CT drho, CT rho, CT ux, CT uy, CT uz, CT b2xx, CT b2yy, CT b2zz,
                                              CT b2xy, CT b2xz, CT b2yz, CT b3xxy, CT b3xxz, CT b3yyx, CT b3yyz,
                                              CT b3zzx, CT b3zzy, CT g[19]) {
  const CT E0 = drho - (b2xx + b2yy + b2zz) * CT(1.0 / 3.0);
  const CT r3 = CT(3) * rho;
  const CT Ux = r3 * ux, Uy = r3 * uy, Uz = r3 * uz;
  const CT ex = E0 + b2xx, ey = E0 + b2yy, ez = E0 + b2zz;
  g[kq<19>(0, 0, 0)] = E0;
  {
    const CT vx = Ux - CT(2) * (b3yyx + b3zzx), vy = Uy - CT(2) * (b3xxy + b3zzy), vz = Uz - CT(2) * (b3xxz + b3yyz);
    g[kq<19>(1, 0, 0)] = ex + vx; g[kq<19>(-1, 0, 0)] = ex - vx;
    g[kq<19>(0, 1, 0)] = ey + vy; g[kq<19>(0, -1, 0)] = ey - vy;
    g[kq<19>(0, 0, 1)] = ez + vz; g[kq<19>(0, 0, -1)] = ez - vz;
  }
  // edge (a, b): even E0 + B_aa + B_bb +- 2 B_ab, odd W_ab = U_a + 2 B3_bba
  auto edge = [&](CT eab, CT Dab, CT Wa, CT Wb, int ia_pp, int ia_mm, int ia_pm, int ia_mp) {
    const CT ep = eab + Dab, em = eab - Dab, op = Wa + Wb, om = Wa - Wb;
    g[ia_pp] = ep + op; g[ia_mm] = ep - op;
    g[ia_pm] = em + om; g[ia_mp] = em - om;
  };
  edge(ex + b2yy, CT(2) * b2xy, Ux + CT(2) * b3yyx, Uy + CT(2) * b3xxy, kq<19>(1, 1, 0), kq<19>(-1, -1, 0),
       kq<19>(1, -1, 0), kq<19>(-1, 1, 0));
  edge(ex + b2zz, CT(2) * b2xz, Ux + CT(2) * b3zzx, Uz + CT(2) * b3xxz, kq<19>(1, 0, 1), kq<19>(-1, 0, -1),
       kq<19>(1, 0, -1), kq<19>(-1, 0, 1));
  edge(ey + b2zz, CT(2) * b2yz, Uy + CT(2) * b3zzy, Uz + CT(2) * b3yyz, kq<19>(0, 1, 1), kq<19>(0, -1, -1),
       kq<19>(0, 1, -1), kq<19>(0, -1, 1));
}

// Normalized equilibrium deviation at (rho, u) on set Q (unit: rho = 1, the
// inflow ghost).
template <class CT, int Q = 27>
__device__ __forceinline__ void equilibrium_dev(CT rho, CT ux, CT uy, CT uz, CT g[Q]) {
  const CT c = CT(4.5) * rho;
  if constexpr (Q == 27) {
    Coef<CT> k;
    finish_coef(k, rho - CT(1), rho, ux, uy, uz, c * ux * ux, c * uy * uy, c * uz * uz, c * ux * uy, c * ux * uz,
                c * uy * uz, c * ux * ux * uy, c * ux * ux * uz, c * uy * uy * ux, c * uy * uy * uz,
                c * uz * uz * ux, c * uz * uz * uy, c * ux * uy * uz);
    reconstruct(k, g);
  } else {
    reconstruct19(rho - CT(1), rho, ux, uy, uz, c * ux * ux, c * uy * uy, c * uz * uz, c * ux * uy, c * ux * uz,
                  c * uy * uz, c * ux * ux * uy, c * ux * ux * uz, c * uy * uy * ux, c * uy * uy * uz,
                  c * uz * uz * ux, c * uz * uz * uy, g);
  }
}
template <class CT, int Q = 27>
__device__ __forceinline__ void equilibrium_dev_unit(CT ux, CT uy, CT uz, CT g[Q]) {
  equilibrium_dev<CT, Q>(CT(1), ux, uy, uz, g);
}

// Collision of one cell (Sec. 2.2, eq. hlbm).  Inputs: deviation moments m,
// homogenized velocity (ux, uy, uz), sigma and the wall strain S (used when
// sigma < 1), model constants.  Output: normalized post-collision deviations.
template <class CT, bool kWall, int NQ = 27>
__device__ __forceinline__ void collide(const Moments<CT>& m, CT rho, CT ux, CT uy, CT uz, CT sigma,
                                        const CT S[6], CT tau0, CT smag, CT g[NQ]) {
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
  const CT Q = sqrt_ct(q2);
  const CT tau = CT(0.5) * (tau0 + sqrt_ct(tau0 * tau0 + smag * Q * rcp_ct(rho)));
  const CT om = CT(1) - rcp_ct(tau);
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
  if constexpr (NQ == 27) {
    const CT b3xyz = c45 * ru_x * uy * uz + t * (ux * Pyz + uy * Pxz + uz * Pxy);
    Coef<CT> k;
    finish_coef(k, m.drho, rho, ux, uy, uz, b2xx, b2yy, b2zz, b2xy, b2xz, b2yz, b3xxy, b3xxz, b3yyx, b3yyz, b3zzx,
                b3zzy, b3xyz);
    reconstruct(k, g);
  } else {
    reconstruct19(m.drho, rho, ux, uy, uz, b2xx, b2yy, b2zz, b2xy, b2xz, b2yz, b3xxy, b3xxz, b3yyx, b3yyz, b3zzx,
                  b3zzy, g);
  }
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

namespace hlbm {

// ---------------------------------------------------------------- reverse mode
// Sums of the adjoint gbar over the velocities against the coefficient
// patterns of `reconstruct` (its transpose): E0 -> 1, B_aa -> c_a^2,
// D_ab -> c_a c_b, V_b -> c_b, T_ab -> c_a^2 c_b, X -> c_x c_y c_z.
template <class CT>
__device__ __forceinline__ Coef<CT> reconstruct_transpose(const CT gb[27]) {
  CT s[9], d[9], a[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const CT gm = gb[k], g0 = gb[9 + k], gp = gb[18 + k];
    a[k] = gp + gm;
    d[k] = gp - gm;
    s[k] = a[k] + g0;
  }
  // column k = 3(cy+1) + (cz+1)
  Coef<CT> c;
  const CT sy_m = s[0] + s[1] + s[2], sy_0 = s[3] + s[4] + s[5], sy_p = s[6] + s[7] + s[8];
  const CT sz_m = s[0] + s[3] + s[6], sz_p = s[2] + s[5] + s[8];
  c.E0 = sy_m + sy_0 + sy_p;
  c.Vy = sy_p - sy_m;
  c.Byy = sy_p + sy_m;
  c.Vz = sz_p - sz_m;
  c.Bzz = sz_p + sz_m;
  c.Dyz = (s[8] + s[0]) - (s[6] + s[2]);
  const CT dy_m = d[0] + d[1] + d[2], dy_0 = d[3] + d[4] + d[5], dy_p = d[6] + d[7] + d[8];
  const CT dz_m = d[0] + d[3] + d[6], dz_p = d[2] + d[5] + d[8];
  c.Vx = dy_m + dy_0 + dy_p;
  c.Dxy = dy_p - dy_m;
  c.Dxz = dz_p - dz_m;
  const CT ay_m = a[0] + a[1] + a[2], ay_0 = a[3] + a[4] + a[5], ay_p = a[6] + a[7] + a[8];
  c.Bxx = ay_m + ay_0 + ay_p;
  c.Txy = ay_p - ay_m;                               // sum cx^2 cy g
  c.Txz = (a[2] + a[5] + a[8]) - (a[0] + a[3] + a[6]);  // sum cx^2 cz g
  c.Tyx = dy_m + dy_p;                               // sum cy^2 cx g
  c.Tzx = dz_m + dz_p;                               // sum cz^2 cx g
  c.Tyz = (s[8] + s[2]) - (s[6] + s[0]);             // sum cy^2 cz g
  c.Tzy = (s[8] + s[6]) - (s[2] + s[0]);             // sum cz^2 cy g
  c.X = (d[8] + d[0]) - (d[6] + d[2]);               // sum cx cy cz g
  return c;
}

// Adjoints of the inputs of reconstruct19 (its transpose): E0, the
// odd-moment scale U = 3 rho u, B2 and the third-order coefficients B3_aab.
// Faces: g = (E0 + B_aa) +- (U_a - 2 sum_{c != a} B3_cca); edges (a, b):
// g = (E0 + B_aa + B_bb +- 2 B_ab) +- (U_a + 2 B3_bba) +- (U_b + 2 B3_aab).
template <class CT>
__device__ __forceinline__ void reconstruct19_transpose(const CT gb[19], CT& E0b, CT b2db[3], CT b2ob[3], CT Ub[3],
                                                        CT b3b[6]) {
  const CT exb = gb[kq<19>(1, 0, 0)] + gb[kq<19>(-1, 0, 0)], vxb = gb[kq<19>(1, 0, 0)] - gb[kq<19>(-1, 0, 0)];
  const CT eyb = gb[kq<19>(0, 1, 0)] + gb[kq<19>(0, -1, 0)], vyb = gb[kq<19>(0, 1, 0)] - gb[kq<19>(0, -1, 0)];
  const CT ezb = gb[kq<19>(0, 0, 1)] + gb[kq<19>(0, 0, -1)], vzb = gb[kq<19>(0, 0, 1)] - gb[kq<19>(0, 0, -1)];
  // edge (a, b): g_pp = ep + op, g_mm = ep - op, g_pm = em + om, g_mp = em - om
  auto edge_t = [&](int ipp, int imm, int ipm, int imp, CT& eb, CT& Db, CT& Wab, CT& Wbb) {
    const CT epb = gb[ipp] + gb[imm], opb = gb[ipp] - gb[imm];
    const CT emb = gb[ipm] + gb[imp], omb = gb[ipm] - gb[imp];
    eb = epb + emb;
    Db = epb - emb;
    Wab = opb + omb;
    Wbb = opb - omb;
  };
  CT exyb, Dxyb, Wx_xy, Wy_xy, exzb, Dxzb, Wx_xz, Wz_xz, eyzb, Dyzb, Wy_yz, Wz_yz;
  edge_t(kq<19>(1, 1, 0), kq<19>(-1, -1, 0), kq<19>(1, -1, 0), kq<19>(-1, 1, 0), exyb, Dxyb, Wx_xy, Wy_xy);
  edge_t(kq<19>(1, 0, 1), kq<19>(-1, 0, -1), kq<19>(1, 0, -1), kq<19>(-1, 0, 1), exzb, Dxzb, Wx_xz, Wz_xz);
  edge_t(kq<19>(0, 1, 1), kq<19>(0, -1, -1), kq<19>(0, 1, -1), kq<19>(0, -1, 1), eyzb, Dyzb, Wy_yz, Wz_yz);
  E0b = gb[kq<19>(0, 0, 0)] + exb + eyb + ezb + exyb + exzb + eyzb;
  b2db[0] = exb + exyb + exzb;
  b2db[1] = eyb + exyb + eyzb;
  b2db[2] = ezb + exzb + eyzb;
  b2ob[0] = CT(2) * Dxyb;
  b2ob[1] = CT(2) * Dxzb;
  b2ob[2] = CT(2) * Dyzb;
  Ub[0] = vxb + Wx_xy + Wx_xz;
  Ub[1] = vyb + Wy_xy + Wy_yz;
  Ub[2] = vzb + Wz_xz + Wz_yz;
  // b3 order xxy, xxz, yyx, yyz, zzx, zzy
  b3b[0] = CT(-2) * vyb + CT(2) * Wy_xy;
  b3b[1] = CT(-2) * vzb + CT(2) * Wz_xz;
  b3b[2] = CT(-2) * vxb + CT(2) * Wx_xy;
  b3b[3] = CT(-2) * vzb + CT(2) * Wz_yz;
  b3b[4] = CT(-2) * vxb + CT(2) * Wx_xz;
  b3b[5] = CT(-2) * vyb + CT(2) * Wy_yz;
}

// Vector-Jacobian product of `collide` (with the homogenized velocity
// u_hat = u + d (b - u), b = u^B + u_wm) and of the momentum handed to the
// solid dP = j - rho u_hat.  gb = adjoint of the normalized post-collision
// deviations (w_i times the adjoint of f*_i), pb = adjoint of dP.  Returns
// the adjoints of the deviation moments, of d and of b (= of u_wm) and S.
template <class CT, int NQ = 27>
__device__ __forceinline__ void collide_vjp(const Moments<CT>& m, CT d, CT bx, CT by, CT bz, CT sigma, const CT S[6],
                                            CT tau0, CT smag, const CT gb[NQ], const CT pb[3], Moments<CT>& mb,
                                            CT& db, CT bb[3], CT Sb[6]) {
  const CT third = CT(1.0 / 3.0), c45 = CT(4.5);
  // ---- forward intermediates
  const CT rho = CT(1) + m.drho, irho = rcp_ct(rho);
  const CT u[3] = {m.jx * irho, m.jy * irho, m.jz * irho};
  const CT e[3] = {bx - u[0], by - u[1], bz - u[2]};
  const CT uh[3] = {u[0] + d * e[0], u[1] + d * e[1], u[2] + d * e[2]};
  const CT ru[3] = {rho * uh[0], rho * uh[1], rho * uh[2]};
  const CT dd = m.drho * third;
  // Pi in the order xx, yy, zz, xy, xz, yz
  const CT P[6] = {m.pxx - dd - ru[0] * uh[0], m.pyy - dd - ru[1] * uh[1], m.pzz - dd - ru[2] * uh[2],
                   m.pxy - ru[0] * uh[1],      m.pxz - ru[0] * uh[2],      m.pyz - ru[1] * uh[2]};
  const CT q2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2] + CT(2) * (P[3] * P[3] + P[4] * P[4] + P[5] * P[5]);
  const CT Q = sqrt_ct(q2);
  const CT sarg = smag * Q * irho;
  const CT rr = sqrt_ct(tau0 * tau0 + sarg);
  const CT tau = CT(0.5) * (tau0 + rr);
  const CT om = CT(1) - rcp_ct(tau);
  const CT os = om * sigma;
  const CT fd = om * CT(3) * (CT(1) - sigma) * rho * tau;
  const CT pi = c45 * os, t = c45 * os;
  // ---- coefficient adjoints: E0 = drho - tr(B2)/3, the odd scale
  // U = 3 rho uh, B2 and B3 (b3 indexed (a twice, b once): xxy, xxz, yyx,
  // yyz, zzx, zzy, and xyz on D3Q27)
  CT b2b[6], b3xxy, b3xxz, b3yyx, b3yyz, b3zzx, b3zzy, b3xyz, drho_b, Ub[3];
  if constexpr (NQ == 27) {
    const Coef<CT> k = reconstruct_transpose(gb);
    // B_aa = b2_aa; D_ab = 2 b2_ab; T_ab = 3 b3_aab; V_b = U_b - sum_{a != b}
    // b3_aab; X = 6 b3_xyz
    b2b[0] = k.Bxx - k.E0 * third; b2b[1] = k.Byy - k.E0 * third; b2b[2] = k.Bzz - k.E0 * third;
    b2b[3] = CT(2) * k.Dxy; b2b[4] = CT(2) * k.Dxz; b2b[5] = CT(2) * k.Dyz;
    b3xxy = CT(3) * k.Txy - k.Vy; b3xxz = CT(3) * k.Txz - k.Vz;
    b3yyx = CT(3) * k.Tyx - k.Vx; b3yyz = CT(3) * k.Tyz - k.Vz;
    b3zzx = CT(3) * k.Tzx - k.Vx; b3zzy = CT(3) * k.Tzy - k.Vy;
    b3xyz = CT(6) * k.X;
    drho_b = k.E0;
    Ub[0] = k.Vx; Ub[1] = k.Vy; Ub[2] = k.Vz;
  } else {
    CT E0b, b2db[3], b2ob[3], b3b[6];
    reconstruct19_transpose<CT>(gb, E0b, b2db, b2ob, Ub, b3b);
    for (int a = 0; a < 3; ++a) {
      b2b[a] = b2db[a] - E0b * third;
      b2b[3 + a] = b2ob[a];
    }
    b3xxy = b3b[0]; b3xxz = b3b[1]; b3yyx = b3b[2]; b3yyz = b3b[3]; b3zzx = b3b[4]; b3zzy = b3b[5];
    b3xyz = CT(0);
    drho_b = E0b;
  }
  CT rho_b = CT(3) * (Ub[0] * uh[0] + Ub[1] * uh[1] + Ub[2] * uh[2]);
  CT uh_b[3] = {CT(3) * rho * Ub[0], CT(3) * rho * Ub[1], CT(3) * rho * Ub[2]};
  CT ru_b[3] = {CT(0), CT(0), CT(0)};
  CT Pb[6] = {CT(0), CT(0), CT(0), CT(0), CT(0), CT(0)};
  CT t_b = CT(0);
  // ---- B3_aab = 4.5 ru_a uh_a uh_b + t (2 uh_a Pi_ab + uh_b Pi_aa)
  // indices into P for Pi_ab: pair(a,b)
  auto b3_back = [&](int a, int b, int pab, CT g) {
    ru_b[a] += c45 * uh[a] * uh[b] * g;
    uh_b[a] += c45 * ru[a] * uh[b] * g + t * CT(2) * P[pab] * g;
    uh_b[b] += c45 * ru[a] * uh[a] * g + t * P[a] * g;
    t_b += (CT(2) * uh[a] * P[pab] + uh[b] * P[a]) * g;
    Pb[pab] += t * CT(2) * uh[a] * g;
    Pb[a] += t * uh[b] * g;
  };
  b3_back(0, 1, 3, b3xxy);
  b3_back(0, 2, 4, b3xxz);
  b3_back(1, 0, 3, b3yyx);
  b3_back(1, 2, 5, b3yyz);
  b3_back(2, 0, 4, b3zzx);
  b3_back(2, 1, 5, b3zzy);
  // B3_xyz = 4.5 ru_x uh_y uh_z + t (uh_x Pi_yz + uh_y Pi_xz + uh_z Pi_xy)
  ru_b[0] += c45 * uh[1] * uh[2] * b3xyz;
  uh_b[1] += c45 * ru[0] * uh[2] * b3xyz + t * P[4] * b3xyz;
  uh_b[2] += c45 * ru[0] * uh[1] * b3xyz + t * P[3] * b3xyz;
  uh_b[0] += t * P[5] * b3xyz;
  t_b += (uh[0] * P[5] + uh[1] * P[4] + uh[2] * P[3]) * b3xyz;
  Pb[5] += t * uh[0] * b3xyz;
  Pb[4] += t * uh[1] * b3xyz;
  Pb[3] += t * uh[2] * b3xyz;
  // ---- B2_ab = 4.5 ru_a uh_b + pi Pi_ab - fd S_ab
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  CT pi_b = CT(0), fd_b = CT(0);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const CT g = b2b[q];
    ru_b[ia[q]] += c45 * uh[ib[q]] * g;
    uh_b[ib[q]] += c45 * ru[ia[q]] * g;
    pi_b += P[q] * g;
    Pb[q] += pi * g;
    fd_b -= S[q] * g;
    Sb[q] = -fd * g;
  }
  // ---- relaxation: os = om sigma, pi = t = 4.5 os, fd = 3 om (1 - sigma) rho tau
  const CT os_b = c45 * (pi_b + t_b);
  CT om_b = sigma * os_b + CT(3) * (CT(1) - sigma) * rho * tau * fd_b;
  rho_b += CT(3) * om * (CT(1) - sigma) * tau * fd_b;
  CT tau_b = CT(3) * om * (CT(1) - sigma) * rho * fd_b;
  tau_b += om_b / (tau * tau);
  // tau = (tau0 + sqrt(tau0^2 + smag Q / rho)) / 2
  const CT sarg_b = CT(0.5) * tau_b / (CT(2) * rr);
  const CT Q_b = smag * sarg_b / rho;
  rho_b -= smag * Q * sarg_b / (rho * rho);
  if (Q > CT(0)) {
    const CT q2_b = Q_b / (CT(2) * Q);
    Pb[0] += CT(2) * P[0] * q2_b;
    Pb[1] += CT(2) * P[1] * q2_b;
    Pb[2] += CT(2) * P[2] * q2_b;
    Pb[3] += CT(4) * P[3] * q2_b;
    Pb[4] += CT(4) * P[4] * q2_b;
    Pb[5] += CT(4) * P[5] * q2_b;
  }
  // ---- Pi_aa = p_aa - drho/3 - ru_a uh_a, Pi_ab = p_ab - ru_a uh_b
  mb.pxx = Pb[0]; mb.pyy = Pb[1]; mb.pzz = Pb[2]; mb.pxy = Pb[3]; mb.pxz = Pb[4]; mb.pyz = Pb[5];
  drho_b -= (Pb[0] + Pb[1] + Pb[2]) * third;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    ru_b[ia[q]] -= uh[ib[q]] * Pb[q];
    uh_b[ib[q]] -= ru[ia[q]] * Pb[q];
  }
  // ---- dP = j - ru
  CT j_b[3] = {pb[0], pb[1], pb[2]};
#pragma unroll
  for (int a = 0; a < 3; ++a) ru_b[a] -= pb[a];
  // ---- ru = rho uh
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    rho_b += uh[a] * ru_b[a];
    uh_b[a] += rho * ru_b[a];
  }
  // ---- uh = u + d (b - u)
  CT u_b[3];
  db = CT(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u_b[a] = (CT(1) - d) * uh_b[a];
    db += e[a] * uh_b[a];
    bb[a] = d * uh_b[a];
  }
  // ---- u = j / rho
  CT ju = CT(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    j_b[a] += irho * u_b[a];
    ju += m.jx * (a == 0) * u_b[a] + m.jy * (a == 1) * u_b[a] + m.jz * (a == 2) * u_b[a];
  }
  rho_b -= irho * irho * ju;
  mb.drho = drho_b + rho_b;
  mb.jx = j_b[0]; mb.jy = j_b[1]; mb.jz = j_b[2];
}

}  // namespace hlbm
