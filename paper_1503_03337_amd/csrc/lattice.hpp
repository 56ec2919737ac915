// lattice.hpp -- compile-time lattices and the MRT collision of the
// incompressible D3Q14 / D3Q18 models (arXiv 1503.03337, Sec. 3 and
// Appendix B) and of the 26-velocity model the closing paragraph of
// Appendix B names (built by Sec. 3's construction), written for gfx950.
//
// The transforms m = T f and f* = f - T' N^-1 D are not stored as matrices:
// every T here factors into sums/differences of opposite axis pairs and
// small Walsh-Hadamard butterflies over the diagonal velocities (the 8
// corners form one 3-level butterfly; the 12 edges three 2-level ones, one
// per coordinate plane).  Each moment below is written as a combination of
// those partial sums; the combinations follow the rows of Eq. (T14), of the
// 18x18 T of Appendix B and of the 26x26 T of the 26-velocity model.  No
// MFMA: every entry of T is a small integer, so the transform is ~100-250
// add/sub per node.
#pragma once
#include <hip/hip_runtime.h>

namespace lbm {

template <int Q> struct Lattice;

// Sec. 3: six axis velocities, then the eight corners, x sign fastest.
template <> struct Lattice<14> {
  static constexpr int q = 14;
  static constexpr int cx[14] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
  static constexpr int cy[14] = {0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
  static constexpr int cz[14] = {0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
  static constexpr int opp[14] = {1, 0, 3, 2, 5, 4, 13, 12, 11, 10, 9, 8, 7, 6};
  // D3Q15 weights without the rest velocity (rest weight 2/9), by |c|^2.
  static constexpr double w_len[4] = {0.0, 1.0 / 9.0, 0.0, 1.0 / 72.0};
  static constexpr double w0 = 2.0 / 9.0;
  // squared row norms of T (T T' = diag(N))
  static constexpr int N[14] = {14, 168, 10, 40, 10, 40, 10, 40, 12, 4, 8, 8, 8, 8};
};

// Appendix B: six axis velocities, then the xy, xz and yz edges.
template <> struct Lattice<18> {
  static constexpr int q = 18;
  static constexpr int cx[18] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[18] = {0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[18] = {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
  static constexpr int opp[18] = {1, 0, 3, 2, 5, 4, 9, 8, 7, 6, 13, 12, 11, 10, 17, 16, 15, 14};
  static constexpr double w_len[4] = {0.0, 1.0 / 18.0, 1.0 / 36.0, 0.0};
  static constexpr double w0 = 1.0 / 3.0;
  static constexpr int N[18] = {18, 36, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8};
};

// The 26-velocity model: the 18 velocities of Appendix B in their order,
// then the 8 corners in the order of Sec. 3; D3Q27 weights (rest 8/27).
template <> struct Lattice<26> {
  static constexpr int q = 26;
  static constexpr int cx[26] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                 1, -1, 1, -1, 1, -1, 1, -1};
  static constexpr int cy[26] = {0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1,
                                 1, 1, -1, -1, 1, 1, -1, -1};
  static constexpr int cz[26] = {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1,
                                 1, 1, 1, 1, -1, -1, -1, -1};
  static constexpr int opp[26] = {1, 0, 3, 2, 5, 4, 9, 8, 7, 6, 13, 12, 11, 10, 17, 16, 15, 14,
                                  25, 24, 23, 22, 21, 20, 19, 18};
  static constexpr double w_len[4] = {0.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
  static constexpr double w0 = 8.0 / 27.0;
  static constexpr int N[26] = {26, 2340, 360, 18, 72, 72, 18, 72, 72, 18, 72, 72, 36,
                                72, 12,   24,  12, 12, 12, 24, 24, 24, 8,  8,  8,  8};
};

// |c_a|^2 (1 axis, 2 edge, 3 corner).
template <int Q>
__host__ __device__ constexpr int len2(int a) {
  return Lattice<Q>::cx[a] * Lattice<Q>::cx[a] + Lattice<Q>::cy[a] * Lattice<Q>::cy[a] +
         Lattice<Q>::cz[a] * Lattice<Q>::cz[a];
}

template <int Q>
__host__ __device__ constexpr double weight(int a) {
  return Lattice<Q>::w_len[len2<Q>(a)];
}

// Weight class of population a: 0 axis, 1 edge, 2 corner (the FP16
// deviation base 3 w_a p0 depends on nothing else).
template <int Q>
__host__ __device__ constexpr int wclass(int a) {
  return len2<Q>(a) - 1;
}

// Index of the velocity equal to c_a with the components of the axes in
// `mask` (bit 0 x, bit 1 y, bit 2 z) negated: the population a specular
// reflection off planes normal to those axes turns a into.
template <int Q>
__host__ __device__ constexpr int mirror(int a, int mask) {
  using L = Lattice<Q>;
  const int mx = (mask & 1) ? -L::cx[a] : L::cx[a];
  const int my = (mask & 2) ? -L::cy[a] : L::cy[a];
  const int mz = (mask & 4) ? -L::cz[a] : L::cz[a];
  for (int b = 0; b < Q; ++b)
    if (L::cx[b] == mx && L::cy[b] == my && L::cz[b] == mz) return b;
  return -1;
}

// k x + y in one instruction, for k a power of two (+-0.5, +-2, +-4): k x
// is then exact, so the fused result has the bits of the separate multiply
// and add.  Only such products are fused; every other product keeps its own
// rounding.
__device__ __forceinline__ float fma2(float k, float x, float y) { return __builtin_fmaf(k, x, y); }
__device__ __forceinline__ double fma2(double k, double x, double y) { return __builtin_fma(k, x, y); }

// Deviation units (DEV): the FP16 step kernels run the collision on
// g = (f - f_rest) 2^s, the stored deviation itself, where f_rest is the
// rest equilibrium at the reference pressure.  Every moment and equilibrium
// term that is linear in f (or in p, j, F) carries the factor 2^s and
// f_rest's share cancels exactly; a product of two such quantities (u u,
// u F) would carry 2^2s, so one factor of each product is taken times
// qs = 2^-s (exact: a power of two).  With DEV false qs is not used and the
// arithmetic is the plain one.
// Per-moment relaxation coefficients, pre-divided by the row norms:
//   sN_k = s_k / N_k,   hN_k = (1 - s_k/2) / N_k,
// so that d_k = D_k / N_k = sN_k (m_k - meq_k) - hN_k mF_k.
template <typename C> struct Relax {
  C sN[26];
  C hN[26];
};

// ---------------------------------------------------------------------------
// 14-velocity model.  Moments (Eq. (moment)):
//   0 P, 1 e, 2 jx, 3 qx, 4 jy, 5 qy, 6 jz, 7 qz, 8 3pxx, 9 pww, 10 pxy,
//   11 pyz, 12 pxz, 13 txyz.
// ---------------------------------------------------------------------------
template <typename C, bool FORCED, bool DEV = false>
__device__ __forceinline__ void collide14(C (&f)[14], const Relax<C>& r, const C (&F)[3],
                                          C qs = C(1)) {
  // forward: axis pairs
  const C ax = f[0] + f[1], dx = f[0] - f[1];
  const C ay = f[2] + f[3], dy = f[2] - f[3];
  const C az = f[4] + f[5], dz = f[4] - f[5];
  const C A = ax + ay + az;
  // forward: corner butterfly (x, then y, then z)
  const C cs1 = f[6] + f[7], cd1 = f[6] - f[7];
  const C cs2 = f[8] + f[9], cd2 = f[8] - f[9];
  const C cs3 = f[10] + f[11], cd3 = f[10] - f[11];
  const C cs4 = f[12] + f[13], cd4 = f[12] - f[13];
  const C pp = cs1 + cs2, py = cs1 - cs2, px = cd1 + cd2, pxy = cd1 - cd2;  // z = +1 layer
  const C mp = cs3 + cs4, my = cs3 - cs4, mx = cd3 + cd4, mxy = cd3 - cd4;  // z = -1 layer
  const C K0 = pp + mp, Kz = pp - mp, Ky = py + my, Kyz = py - my;
  const C Kx = px + mx, Kxz = px - mx, Kxy = pxy + mxy, Kxyz = pxy - mxy;

  const C mP = A + K0;
  const C me = fma2(C(-4), A, C(3) * K0);
  const C jx = dx + Kx, qx = fma2(C(-4), dx, Kx);
  const C jy = dy + Ky, qy = fma2(C(-4), dy, Ky);
  const C jz = dz + Kz, qz = fma2(C(-4), dz, Kz);
  const C pxx3 = fma2(C(2), ax, -ay) - az;
  const C pww = ay - az;

  // Eq. (hgl): u = j + F/2, p = 3/7 (P - |u|^2/3)
  C ux = jx, uy = jy, uz = jz;
  if (FORCED) {
    ux = fma2(C(0.5), F[0], ux);
    uy = fma2(C(0.5), F[1], uy);
    uz = fma2(C(0.5), F[2], uz);
  }
  const C uxq = DEV ? ux * qs : ux, uyq = DEV ? uy * qs : uy, uzq = DEV ? uz * qs : uz;
  const C uxx = uxq * ux, uyy = uyq * uy, uzz = uzq * uz;
  const C usq = uxx + uyy + uzz;
  const C p = (mP - usq * C(1.0 / 3.0)) * C(3.0 / 7.0);

  // d_k = sN_k (m_k - meq_k) - hN_k mF_k, Eq. (meq) equilibria
  C d0 = r.sN[0] * (mP - (C(7.0 / 3.0) * p + usq * C(1.0 / 3.0)));
  C d1e = r.sN[1] * (me - (usq - C(7) * p));
  C d2 = r.sN[2] * (jx - ux);
  C d3 = r.sN[3] * (qx + C(7.0 / 3.0) * ux);
  C d4 = r.sN[4] * (jy - uy);
  C d5 = r.sN[5] * (qy + C(7.0 / 3.0) * uy);
  C d6 = r.sN[6] * (jz - uz);
  C d7 = r.sN[7] * (qz + C(7.0 / 3.0) * uz);
  C d8 = r.sN[8] * (pxx3 - (C(3) * uxx - usq));
  C d9 = r.sN[9] * (pww - (uyy - uzz));
  C d10 = r.sN[10] * (Kxy - uxq * uy);
  C d11 = r.sN[11] * (Kyz - uyq * uz);
  C d12 = r.sN[12] * (Kxz - uxq * uz);
  C d13 = r.sN[13] * Kxyz;
  if (FORCED) {
    // m_F = (d m_eq / d u) . F
    const C Fx = F[0], Fy = F[1], Fz = F[2];
    const C w = uxq * Fx + uyq * Fy + uzq * Fz;
    d0 -= r.hN[0] * (C(2.0 / 3.0) * w);
    d1e -= r.hN[1] * (C(2) * w);
    d2 -= r.hN[2] * Fx;
    d3 -= r.hN[3] * (C(-7.0 / 3.0) * Fx);
    d4 -= r.hN[4] * Fy;
    d5 -= r.hN[5] * (C(-7.0 / 3.0) * Fy);
    d6 -= r.hN[6] * Fz;
    d7 -= r.hN[7] * (C(-7.0 / 3.0) * Fz);
    d8 -= r.hN[8] * fma2(C(-2), w, C(6) * uxq * Fx);
    d9 -= r.hN[9] * (C(2) * (uyq * Fy - uzq * Fz));
    d10 -= r.hN[10] * (uxq * Fy + uyq * Fx);
    d11 -= r.hN[11] * (uyq * Fz + uzq * Fy);
    d12 -= r.hN[12] * (uxq * Fz + uzq * Fx);
  }

  // back-transform f*_a = f_a - sum_k T_ka d_k, axis velocities
  const C bA = fma2(C(-4), d1e, d0);
  const C X = fma2(C(-4), d3, d2), Y = fma2(C(-4), d5, d4), Z = fma2(C(-4), d7, d6);
  f[0] -= fma2(C(2), d8, bA + X);
  f[1] -= fma2(C(2), d8, bA - X);
  const C yy = d9 - d8, zz = -(d8 + d9);
  f[2] -= (bA + Y) + yy;
  f[3] -= (bA - Y) + yy;
  f[4] -= (bA + Z) + zz;
  f[5] -= (bA - Z) + zz;
  // corners: inverse butterfly of W0 + cx Wx + cy Wy + cz Wz + cxcy Wxy + ...
  const C W0 = d0 + C(3) * d1e;
  const C Wx = d2 + d3, Wy = d4 + d5, Wz = d6 + d7;
  const C zp0 = W0 + Wz, zpx = Wx + d12, zpy = Wy + d11, zpxy = d10 + d13;
  const C zm0 = W0 - Wz, zmx = Wx - d12, zmy = Wy - d11, zmxy = d10 - d13;
  C a = zp0 + zpy, b = zpx + zpxy;
  f[6] -= a + b;
  f[7] -= a - b;
  a = zp0 - zpy;
  b = zpx - zpxy;
  f[8] -= a + b;
  f[9] -= a - b;
  a = zm0 + zmy;
  b = zmx + zmxy;
  f[10] -= a + b;
  f[11] -= a - b;
  a = zm0 - zmy;
  b = zmx - zmxy;
  f[12] -= a + b;
  f[13] -= a - b;
}

// ---------------------------------------------------------------------------
// 18-velocity model.  Moments (Eq. (d3q18moment)):
//   0 P, 1 e, 2 jx, 3 qx, 4 jy, 5 qy, 6 jz, 7 qz, 8 3pxx, 9 3pixx, 10 pww,
//   11 piww, 12 pxy, 13 pyz, 14 pxz, 15 tx, 16 ty, 17 tz.
// ---------------------------------------------------------------------------
template <typename C, bool FORCED, bool DEV = false>
__device__ __forceinline__ void collide18(C (&f)[18], const Relax<C>& r, const C (&F)[3],
                                          C qs = C(1)) {
  const C ax = f[0] + f[1], dx = f[0] - f[1];
  const C ay = f[2] + f[3], dy = f[2] - f[3];
  const C az = f[4] + f[5], dz = f[4] - f[5];
  const C A = ax + ay + az;
  // xy edges 6..9 in (cx, cy): (+,+) (-,+) (+,-) (-,-)
  C s = f[6] + f[7], d = f[6] - f[7], s_ = f[8] + f[9], d_ = f[8] - f[9];
  const C Sxy = s + s_, Yxy = s - s_, Xxy = d + d_, XYxy = d - d_;
  // xz edges 10..13 in (cx, cz)
  s = f[10] + f[11];
  d = f[10] - f[11];
  s_ = f[12] + f[13];
  d_ = f[12] - f[13];
  const C Sxz = s + s_, Zxz = s - s_, Xxz = d + d_, XZxz = d - d_;
  // yz edges 14..17 in (cy, cz)
  s = f[14] + f[15];
  d = f[14] - f[15];
  s_ = f[16] + f[17];
  d_ = f[16] - f[17];
  const C Syz = s + s_, Zyz = s - s_, Yyz = d + d_, YZyz = d - d_;

  const C E = Sxy + Sxz + Syz;
  const C mP = A + E;
  const C me = fma2(C(-2), A, E);
  const C ex = Xxy + Xxz, ey = Yxy + Yyz, ez = Zxz + Zyz;
  const C jx = dx + ex, qx = fma2(C(-4), dx, ex);
  const C jy = dy + ey, qy = fma2(C(-4), dy, ey);
  const C jz = dz + ez, qz = fma2(C(-4), dz, ez);
  const C axis_xx = fma2(C(2), ax, -ay) - az;
  const C edge_xx = fma2(C(-2), Syz, Sxy + Sxz);
  const C pxx3 = axis_xx + edge_xx;
  const C pixx3 = fma2(C(-2), axis_xx, edge_xx);
  const C axis_ww = ay - az, edge_ww = Sxy - Sxz;
  const C pww = axis_ww + edge_ww;
  const C piww = fma2(C(-2), axis_ww, edge_ww);
  const C tx = Xxy - Xxz, ty = Yyz - Yxy, tz = Zxz - Zyz;

  C ux = jx, uy = jy, uz = jz;
  if (FORCED) {
    ux = fma2(C(0.5), F[0], ux);
    uy = fma2(C(0.5), F[1], uy);
    uz = fma2(C(0.5), F[2], uz);
  }
  const C uxq = DEV ? ux * qs : ux, uyq = DEV ? uy * qs : uy, uzq = DEV ? uz * qs : uz;
  const C uxx = uxq * ux, uyy = uyq * uy, uzz = uzq * uz;
  const C usq = uxx + uyy + uzz;
  // Eq. (hgl) with w0 = 1/3: p = (P - |u|^2/2) / 2
  const C p = fma2(C(-0.5), usq, mP) * C(0.5);
  const C qxx = C(3) * uxx - usq, qww = uyy - uzz;

  C d0 = r.sN[0] * (mP - fma2(C(2), p, C(0.5) * usq));
  C d1e = r.sN[1] * (me - fma2(C(0.5), usq, -p));
  C d2 = r.sN[2] * (jx - ux);
  C d3 = r.sN[3] * (qx + C(2.0 / 3.0) * ux);
  C d4 = r.sN[4] * (jy - uy);
  C d5 = r.sN[5] * (qy + C(2.0 / 3.0) * uy);
  C d6 = r.sN[6] * (jz - uz);
  C d7 = r.sN[7] * (qz + C(2.0 / 3.0) * uz);
  C d8 = r.sN[8] * (pxx3 - qxx);
  C d9 = r.sN[9] * fma2(C(0.5), qxx, pixx3);
  C d10 = r.sN[10] * (pww - qww);
  C d11 = r.sN[11] * fma2(C(0.5), qww, piww);
  C d12 = r.sN[12] * (XYxy - uxq * uy);
  C d13 = r.sN[13] * (YZyz - uyq * uz);
  C d14 = r.sN[14] * (XZxz - uxq * uz);
  C d15 = r.sN[15] * tx;
  C d16 = r.sN[16] * ty;
  C d17 = r.sN[17] * tz;
  if (FORCED) {
    const C Fx = F[0], Fy = F[1], Fz = F[2];
    const C w = uxq * Fx + uyq * Fy + uzq * Fz;
    const C gxx = fma2(C(-2), w, C(6) * uxq * Fx);
    const C gww = uyq * Fy - uzq * Fz;
    d0 -= r.hN[0] * w;
    d1e -= r.hN[1] * w;
    d2 -= r.hN[2] * Fx;
    d3 -= r.hN[3] * (C(-2.0 / 3.0) * Fx);
    d4 -= r.hN[4] * Fy;
    d5 -= r.hN[5] * (C(-2.0 / 3.0) * Fy);
    d6 -= r.hN[6] * Fz;
    d7 -= r.hN[7] * (C(-2.0 / 3.0) * Fz);
    d8 -= r.hN[8] * gxx;
    d9 -= r.hN[9] * (C(-0.5) * gxx);
    d10 -= r.hN[10] * (C(2) * gww);
    d11 -= r.hN[11] * (-gww);
    d12 -= r.hN[12] * (uxq * Fy + uyq * Fx);
    d13 -= r.hN[13] * (uyq * Fz + uzq * Fy);
    d14 -= r.hN[14] * (uxq * Fz + uzq * Fx);
  }

  // back-transform, axis velocities (columns 1..6 of T)
  const C bA = fma2(C(-2), d1e, d0);
  const C X = fma2(C(-4), d3, d2), Y = fma2(C(-4), d5, d4), Z = fma2(C(-4), d7, d6);
  const C xx = fma2(C(2), d8, C(-4) * d9);
  const C yz_common = fma2(C(2), d9, -d8);  // -d8 + 2 d9
  const C ww = fma2(C(-2), d11, d10);
  const C yy = yz_common + ww, zz = yz_common - ww;
  f[0] -= (bA + X) + xx;
  f[1] -= (bA - X) + xx;
  f[2] -= (bA + Y) + yy;
  f[3] -= (bA - Y) + yy;
  f[4] -= (bA + Z) + zz;
  f[5] -= (bA - Z) + zz;
  // edges: value(s1,s2) = W0 + s1 W1 + s2 W2 + s1 s2 W12 per plane
  const C E0 = d0 + d1e, G = d8 + d9, H = d10 + d11;
  const C jqx = d2 + d3, jqy = d4 + d5, jqz = d6 + d7;
  {  // xy plane (cx, cy)
    const C W0 = E0 + G + H, W1 = jqx + d15, W2 = jqy - d16, W12 = d12;
    C a = W0 + W2, b = W1 + W12;
    f[6] -= a + b;
    f[7] -= a - b;
    a = W0 - W2;
    b = W1 - W12;
    f[8] -= a + b;
    f[9] -= a - b;
  }
  {  // xz plane (cx, cz)
    const C W0 = E0 + G - H, W1 = jqx - d15, W2 = jqz + d17, W12 = d14;
    C a = W0 + W2, b = W1 + W12;
    f[10] -= a + b;
    f[11] -= a - b;
    a = W0 - W2;
    b = W1 - W12;
    f[12] -= a + b;
    f[13] -= a - b;
  }
  {  // yz plane (cy, cz)
    const C W0 = fma2(C(-2), G, E0), W1 = jqy + d16, W2 = jqz - d17, W12 = d13;
    C a = W0 + W2, b = W1 + W12;
    f[14] -= a + b;
    f[15] -= a - b;
    a = W0 - W2;
    b = W1 - W12;
    f[16] -= a + b;
    f[17] -= a - b;
  }
}


// ---------------------------------------------------------------------------
// 26-velocity model.  Moments (Gram-Schmidt of the monomial rows by tensor
// order, Sec. 3's construction):
//   0 P, 1 e, 2 eps, 3 jx, 4 qx, 5 hx, 6 jy, 7 qy, 8 hy, 9 jz, 10 qz, 11 hz,
//   12 3pxx, 13 3pixx, 14 pww, 15 piww, 16 pxy, 17 pyz, 18 pxz, 19 pixy,
//   20 piyz, 21 pixz, 22 tx, 23 ty, 24 tz, 25 txyz.
// Basis rows: 1, 13|c|^2 - 27, (15|c|^4 - 61|c|^2 + 54)/2; c, (3|c|^2 - 7) c,
// (9|c|^4 - 39|c|^2 + 38) c / 2; 3c_x^2 - |c|^2, c_y^2 - c_z^2 and these
// times (3|c|^2 - 5); c_x c_y (...) and these times (3|c|^2 - 8); the
// third-order t rows of Appendix B and c_x c_y c_z.  Equilibria (T f_eq with
// the D3Q27 weights): P 19p/9 + 4|u|^2/9, e -18p + |u|^2, eps 3p - |u|^2,
// j u, q -2u, h u, the stresses as for 18 velocities with pi = -p, t 0.
// ---------------------------------------------------------------------------
template <typename C, bool FORCED, bool DEV = false>
__device__ __forceinline__ void collide26(C (&f)[26], const Relax<C>& r, const C (&F)[3],
                                          C qs = C(1)) {
  const C ax = f[0] + f[1], dx = f[0] - f[1];
  const C ay = f[2] + f[3], dy = f[2] - f[3];
  const C az = f[4] + f[5], dz = f[4] - f[5];
  const C A = ax + ay + az;
  // edges 6..17, per plane (as for 18 velocities)
  C s = f[6] + f[7], d = f[6] - f[7], s_ = f[8] + f[9], d_ = f[8] - f[9];
  const C Sxy = s + s_, Yxy = s - s_, Xxy = d + d_, XYxy = d - d_;
  s = f[10] + f[11];
  d = f[10] - f[11];
  s_ = f[12] + f[13];
  d_ = f[12] - f[13];
  const C Sxz = s + s_, Zxz = s - s_, Xxz = d + d_, XZxz = d - d_;
  s = f[14] + f[15];
  d = f[14] - f[15];
  s_ = f[16] + f[17];
  d_ = f[16] - f[17];
  const C Syz = s + s_, Zyz = s - s_, Yyz = d + d_, YZyz = d - d_;
  // corners 18..25 (as for 14 velocities): x, then y, then z
  const C cs1 = f[18] + f[19], cd1 = f[18] - f[19];
  const C cs2 = f[20] + f[21], cd2 = f[20] - f[21];
  const C cs3 = f[22] + f[23], cd3 = f[22] - f[23];
  const C cs4 = f[24] + f[25], cd4 = f[24] - f[25];
  const C pp = cs1 + cs2, py = cs1 - cs2, px = cd1 + cd2, pxy = cd1 - cd2;
  const C mp = cs3 + cs4, my = cs3 - cs4, mx = cd3 + cd4, mxy = cd3 - cd4;
  const C K0 = pp + mp, Kz = pp - mp, Ky = py + my, Kyz = py - my;
  const C Kx = px + mx, Kxz = px - mx, Kxy = pxy + mxy, Kxyz = pxy - mxy;

  const C E = Sxy + Sxz + Syz;
  const C mP = A + E + K0;
  const C me = (C(-14) * A - E) + C(12) * K0;
  const C meps = fma2(C(4), A - E, C(3) * K0);
  const C ex = Xxy + Xxz, ey = Yxy + Yyz, ez = Zxz + Zyz;
  const C jx = dx + ex + Kx, qx = fma2(C(-4), dx, fma2(C(2), Kx, -ex)),
          hx = fma2(C(4), dx, fma2(C(-2), ex, Kx));
  const C jy = dy + ey + Ky, qy = fma2(C(-4), dy, fma2(C(2), Ky, -ey)),
          hy = fma2(C(4), dy, fma2(C(-2), ey, Ky));
  const C jz = dz + ez + Kz, qz = fma2(C(-4), dz, fma2(C(2), Kz, -ez)),
          hz = fma2(C(4), dz, fma2(C(-2), ez, Kz));
  const C axis_xx = fma2(C(2), ax, -ay) - az;
  const C edge_xx = fma2(C(-2), Syz, Sxy + Sxz);
  const C pxx3 = axis_xx + edge_xx;
  const C pixx3 = fma2(C(-2), axis_xx, edge_xx);
  const C axis_ww = ay - az, edge_ww = Sxy - Sxz;
  const C pww = axis_ww + edge_ww;
  const C piww = fma2(C(-2), axis_ww, edge_ww);
  const C mpxy = XYxy + Kxy, mpyz = YZyz + Kyz, mpxz = XZxz + Kxz;
  const C mpixy = fma2(C(-2), XYxy, Kxy), mpiyz = fma2(C(-2), YZyz, Kyz),
          mpixz = fma2(C(-2), XZxz, Kxz);
  const C tx = Xxy - Xxz, ty = Yyz - Yxy, tz = Zxz - Zyz;

  C ux = jx, uy = jy, uz = jz;
  if (FORCED) {
    ux = fma2(C(0.5), F[0], ux);
    uy = fma2(C(0.5), F[1], uy);
    uz = fma2(C(0.5), F[2], uz);
  }
  const C uxq = DEV ? ux * qs : ux, uyq = DEV ? uy * qs : uy, uzq = DEV ? uz * qs : uz;
  const C uxx = uxq * ux, uyy = uyq * uy, uzz = uzq * uz;
  const C usq = uxx + uyy + uzz;
  // Eq. (hgl) with w0 = 8/27: p = 9/19 (P - 4/9 |u|^2)
  const C p = (mP - usq * C(4.0 / 9.0)) * C(9.0 / 19.0);
  const C qxx = C(3) * uxx - usq, qww = uyy - uzz;
  const C uxy = uxq * uy, uyz = uyq * uz, uxz = uxq * uz;

  C d0 = r.sN[0] * (mP - (C(19.0 / 9.0) * p + C(4.0 / 9.0) * usq));
  C d1 = r.sN[1] * (me - (usq - C(18) * p));
  C d2 = r.sN[2] * (meps - (C(3) * p - usq));
  C d3 = r.sN[3] * (jx - ux);
  C d4 = r.sN[4] * fma2(C(2), ux, qx);
  C d5 = r.sN[5] * (hx - ux);
  C d6 = r.sN[6] * (jy - uy);
  C d7 = r.sN[7] * fma2(C(2), uy, qy);
  C d8 = r.sN[8] * (hy - uy);
  C d9 = r.sN[9] * (jz - uz);
  C d10 = r.sN[10] * fma2(C(2), uz, qz);
  C d11 = r.sN[11] * (hz - uz);
  C d12 = r.sN[12] * (pxx3 - qxx);
  C d13 = r.sN[13] * (pixx3 + qxx);
  C d14 = r.sN[14] * (pww - qww);
  C d15 = r.sN[15] * (piww + qww);
  C d16 = r.sN[16] * (mpxy - uxy);
  C d17 = r.sN[17] * (mpyz - uyz);
  C d18 = r.sN[18] * (mpxz - uxz);
  C d19 = r.sN[19] * (mpixy + uxy);
  C d20 = r.sN[20] * (mpiyz + uyz);
  C d21 = r.sN[21] * (mpixz + uxz);
  C d22 = r.sN[22] * tx;
  C d23 = r.sN[23] * ty;
  C d24 = r.sN[24] * tz;
  C d25 = r.sN[25] * Kxyz;
  if (FORCED) {
    // m_F = (d m_eq / d u) . F
    const C Fx = F[0], Fy = F[1], Fz = F[2];
    const C w = uxq * Fx + uyq * Fy + uzq * Fz;
    const C gxx = fma2(C(-2), w, C(6) * uxq * Fx);
    const C gww = C(2) * (uyq * Fy - uzq * Fz);
    const C gxy = uxq * Fy + uyq * Fx, gyz = uyq * Fz + uzq * Fy, gxz = uxq * Fz + uzq * Fx;
    d0 -= r.hN[0] * (C(8.0 / 9.0) * w);
    d1 -= r.hN[1] * (C(2) * w);
    d2 -= r.hN[2] * (C(-2) * w);
    d3 -= r.hN[3] * Fx;
    d4 -= r.hN[4] * (C(-2) * Fx);
    d5 -= r.hN[5] * Fx;
    d6 -= r.hN[6] * Fy;
    d7 -= r.hN[7] * (C(-2) * Fy);
    d8 -= r.hN[8] * Fy;
    d9 -= r.hN[9] * Fz;
    d10 -= r.hN[10] * (C(-2) * Fz);
    d11 -= r.hN[11] * Fz;
    d12 -= r.hN[12] * gxx;
    d13 -= r.hN[13] * (-gxx);
    d14 -= r.hN[14] * gww;
    d15 -= r.hN[15] * (-gww);
    d16 -= r.hN[16] * gxy;
    d17 -= r.hN[17] * gyz;
    d18 -= r.hN[18] * gxz;
    d19 -= r.hN[19] * (-gxy);
    d20 -= r.hN[20] * (-gyz);
    d21 -= r.hN[21] * (-gxz);
  }

  // back-transform f*_a = f_a - sum_k T_ka d_k, axis velocities
  const C bA = fma2(C(4), d2, C(-14) * d1 + d0);
  const C X = fma2(C(4), d5 - d4, d3), Y = fma2(C(4), d8 - d7, d6),
          Z = fma2(C(4), d11 - d10, d9);
  const C xx = fma2(C(2), d12, C(-4) * d13);
  const C yz_common = fma2(C(2), d13, -d12);
  const C ww = fma2(C(-2), d15, d14);
  const C yy = yz_common + ww, zz = yz_common - ww;
  f[0] -= (bA + X) + xx;
  f[1] -= (bA - X) + xx;
  f[2] -= (bA + Y) + yy;
  f[3] -= (bA - Y) + yy;
  f[4] -= (bA + Z) + zz;
  f[5] -= (bA - Z) + zz;
  // edges: value(s1,s2) = W0 + s1 W1 + s2 W2 + s1 s2 W12 per plane
  const C E0 = fma2(C(-4), d2, d0 - d1), G = d12 + d13, H = d14 + d15;
  const C vx = fma2(C(-2), d5, d3 - d4), vy = fma2(C(-2), d8, d6 - d7),
          vz = fma2(C(-2), d11, d9 - d10);
  {  // xy plane (cx, cy)
    const C W0 = E0 + G + H, W1 = vx + d22, W2 = vy - d23, W12 = fma2(C(-2), d19, d16);
    C a = W0 + W2, b = W1 + W12;
    f[6] -= a + b;
    f[7] -= a - b;
    a = W0 - W2;
    b = W1 - W12;
    f[8] -= a + b;
    f[9] -= a - b;
  }
  {  // xz plane (cx, cz)
    const C W0 = E0 + G - H, W1 = vx - d22, W2 = vz + d24, W12 = fma2(C(-2), d21, d18);
    C a = W0 + W2, b = W1 + W12;
    f[10] -= a + b;
    f[11] -= a - b;
    a = W0 - W2;
    b = W1 - W12;
    f[12] -= a + b;
    f[13] -= a - b;
  }
  {  // yz plane (cy, cz)
    const C W0 = fma2(C(-2), G, E0), W1 = vy + d23, W2 = vz - d24, W12 = fma2(C(-2), d20, d17);
    C a = W0 + W2, b = W1 + W12;
    f[14] -= a + b;
    f[15] -= a - b;
    a = W0 - W2;
    b = W1 - W12;
    f[16] -= a + b;
    f[17] -= a - b;
  }
  // corners: inverse butterfly of W0 + cx Wx + cy Wy + cz Wz + cxcy Wxy + ...
  const C W0 = C(3) * d2 + (C(12) * d1 + d0);
  const C Wx = fma2(C(2), d4, d3 + d5), Wy = fma2(C(2), d7, d6 + d8),
          Wz = fma2(C(2), d10, d9 + d11);
  const C Wxy = d16 + d19, Wyz = d17 + d20, Wxz = d18 + d21;
  const C zp0 = W0 + Wz, zpx = Wx + Wxz, zpy = Wy + Wyz, zpxy = Wxy + d25;
  const C zm0 = W0 - Wz, zmx = Wx - Wxz, zmy = Wy - Wyz, zmxy = Wxy - d25;
  C a = zp0 + zpy, b = zpx + zpxy;
  f[18] -= a + b;
  f[19] -= a - b;
  a = zp0 - zpy;
  b = zpx - zpxy;
  f[20] -= a + b;
  f[21] -= a - b;
  a = zm0 + zmy;
  b = zmx + zmxy;
  f[22] -= a + b;
  f[23] -= a - b;
  a = zm0 - zmy;
  b = zmx - zmxy;
  f[24] -= a + b;
  f[25] -= a - b;
}

// ---------------------------------------------------------------------------
// Single-relaxation-time (LBGK) collision, the special case S = I/tau of the
// MRT models (Sec. 3: Lambda-hat = I/tau gives the iD3Q15 LBGK model of
// Sec. 2; Appendix B likewise for iD3Q19):
//   f*_a = f_a - (f_a - f_eq_a)/tau + (1 - 1/(2 tau)) src_a,
// f_eq from Eq. (edf), src_a = w_a [3 c.F + 9 (c.u)(c.F) - 3 u.F] the
// velocity-space form of the moment force (no transform needed).
// omega = 1/tau, hom = 1 - omega/2.
// ---------------------------------------------------------------------------
template <int Q, typename C, bool FORCED, bool DEV = false>
__device__ __forceinline__ void collide_bgk(C (&f)[Q], C omega, C hom, const C (&F)[3],
                                            C qs = C(1)) {
  using L = Lattice<Q>;
  C P = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    P += f[a];
    if (L::cx[a]) jx += L::cx[a] > 0 ? f[a] : -f[a];
    if (L::cy[a]) jy += L::cy[a] > 0 ? f[a] : -f[a];
    if (L::cz[a]) jz += L::cz[a] > 0 ? f[a] : -f[a];
  }
  C ux = jx, uy = jy, uz = jz;
  if (FORCED) {
    ux = fma2(C(0.5), F[0], ux);
    uy = fma2(C(0.5), F[1], uy);
    uz = fma2(C(0.5), F[2], uz);
  }
  const C uxq = DEV ? ux * qs : ux, uyq = DEV ? uy * qs : uy, uzq = DEV ? uz * qs : uz;
  const C usq = uxq * ux + uyq * uy + uzq * uz;
  // Eq. (hgl): p = (P - 3/2 w0 |u|^2) / (3 (1 - w0))
  const C p = (P - C(1.5 * L::w0) * usq) * C(1.0 / (3.0 * (1.0 - L::w0)));
  const C uF = FORCED ? uxq * F[0] + uyq * F[1] + uzq * F[2] : C(0);
  // (c.u)^2 and (c.u)(c.F) take 2^-s through their constant factor
  const C k45 = DEV ? C(4.5) * qs : C(4.5), k9 = DEV ? C(9) * qs : C(9);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const C w = C(weight<Q>(a));
    C cu = C(0), cF = C(0);
    if (L::cx[a]) { cu += L::cx[a] > 0 ? ux : -ux; if (FORCED) cF += L::cx[a] > 0 ? F[0] : -F[0]; }
    if (L::cy[a]) { cu += L::cy[a] > 0 ? uy : -uy; if (FORCED) cF += L::cy[a] > 0 ? F[1] : -F[1]; }
    if (L::cz[a]) { cu += L::cz[a] > 0 ? uz : -uz; if (FORCED) cF += L::cz[a] > 0 ? F[2] : -F[2]; }
    const C feq = w * (C(3) * p + C(3) * cu + k45 * cu * cu - C(1.5) * usq);
    C fa = f[a] - omega * (f[a] - feq);
    if (FORCED) fa += hom * (w * (C(3) * cF + k9 * cu * cF - C(3) * uF));
    f[a] = fa;
  }
}

template <int Q, typename C, bool FORCED, bool DEV = false>
__device__ __forceinline__ void collide(C (&f)[Q], const Relax<C>& r, const C (&F)[3],
                                        C qs = C(1)) {
  if constexpr (Q == 14)
    collide14<C, FORCED, DEV>(f, r, F, qs);
  else if constexpr (Q == 18)
    collide18<C, FORCED, DEV>(f, r, F, qs);
  else
    collide26<C, FORCED, DEV>(f, r, F, qs);
}

}  // namespace lbm
