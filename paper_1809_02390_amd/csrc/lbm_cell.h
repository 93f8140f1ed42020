// Per-node arithmetic of the self-tuning-EOS D2Q9 model, shared by every
// kernel of the library.  All functions are __host__ __device__ templates on
// the real type; the kernels instantiate them with float.
//
// Moment order (supplement Eq. 4): rho, e, eps, j_x, q_x, j_y, q_y, p_xx,
// p_xy.  Velocity order (supplement Eq. 3): rest, +x, +y, -x, -y, +x+y,
// -x+y, -x-y, +x-y.  Lattice units dx = dt = c = 1.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

// Scalars of one collision, precomputed on the host (FP64 -> T).
template <typename T>
struct Coef {
  T g2;        // G'^2 (force strength, main Eq. 12)
  T kp, rt;    // K' = K_EOS and R T of the CS pressure (main Eq. 20)
  T a, b4;     // a and b/4
  T kprt;      // K' R T
  T e_rho;     // G'^2/2 - K' a   : p_LBE = rho (K' R T Z + e_rho rho)
  T de_rho;    // G'^2 - 2 K' a   : d p_LBE / d rho = K' R T (rho Z)' + de_rho rho
  T alpha2, beta2;
  // 1 - s for the rows without off-diagonal coupling
  T one_m_seps, one_m_sq;
  // step (2) of supplement Sec. IV
  T k_seps_h;  // k s_eps / 2
  T h_sq_h;    // h s_q / 2
  T b_sq;      // b s_q
  T b_sq_h;    // b s_q / 2
  // step (3): 1 - s/2
  T om_e, om_eps, om_q, om_p;
  T two_om_e, two_om_p;  // 2 (1 - s/2)
  // step (4): nonzero entries of R, T, X (supplement Eqs. 34, 37, 40)
  T cR11, cR17, cR18, cT1, one_mk, twok_h, cX1;
  T cT1a, cT1b;  // cT1 (1 - k), cT1 (2k + h)
  T cR71, cR77, cT7, two_b, cX7;
  T cR81, cR88, cT8, cX8;
  // step (6)
  T s_e, kq2, s_eps, s_p;  // kq2 = k (s_e/2 - 1) s_eps
  T q1, q7;                // (s_e - kq2) G'^2 / 2 and s_p G'^2 / 12
  T q2, s_q;               // s_eps G'^2 / 2 and s_q
  // collide_scaled: the rows of m-bar - m times the diagonal of M^-1 = M^T D
  // (1/36 for e, eps; 1/12 for q; 1/4 for p_xx, p_xy) with the sign of the
  // corrections, folded into one constant per term
  T w_r11, w_r17, w_r18, w_t1a, w_x1, w_t1b, w_q1;  // row e:   -cR../36, -cT1a/36, -cX1/36, cT1b/36, q1/36
  T w_seps, w_q2, w_sq;                             // rows eps, q: s_eps/36, q2/36, s_q/12
  T w_r71, w_r77, w_t7, w_x7, w_t7b, w_q7;          // row p_xx: -cR../4, -cT7/4, -cX7/4, -cT7 2b/4, q7/4
  T w_r81, w_r88, w_x8, w_t8;                       // row p_xy: -cR../4, -cX8/4, -cT8/4
};

// Reciprocal: the one-instruction v_rcp_f32 (1 ulp) on the device, a
// division elsewhere.  Every kernel uses the same function, so forward steps
// and recomputations agree bit for bit.
template <typename T>
__host__ __device__ __forceinline__ T recip(T x) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(x);
#endif
  return T(1) / x;
}

// rho = sum_i f_i in one fixed order (the order forward_moments uses), so a
// node's density is the same number in every kernel that forms it.
template <typename T>
__host__ __device__ __forceinline__ T density(const T* f) {
  return f[0] + (((f[1] + f[3]) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8])));
}

// Stencil of main Eq. 12 (the weights 1/3 and 1/12, unit spacing):
// g = sum_i w_i rho(x + e_i) e_i.  Arguments are the eight neighbour
// densities named by direction.
template <typename T>
__host__ __device__ __forceinline__ void stencil(T rE, T rN, T rW, T rS, T rNE, T rNW, T rSW, T rSE, T& gx,
                                                 T& gy) {
  const T third = T(1) / T(3), twelfth = T(1) / T(12);
  const T dd1 = rNE - rSW, dd2 = rSE - rNW;  // the two diagonals
  gx = third * (rE - rW) + twelfth * (dd1 + dd2);
  gy = third * (rN - rS) + twelfth * (dd1 - dd2);
}

// Pressure of the lattice Boltzmann equation and its density slope:
// p_LBE = K'[rho R T Z - a rho^2] + G^2 rho^2/2 (main Eqs. 18, 20),
// Z = (1 + v + v^2 - v^3)/(1 - v)^3, d(rho Z)/d rho = (1 + 4v + 4v^2 - 4v^3 + v^4)/(1 - v)^4.
template <typename T>
__host__ __device__ __forceinline__ void eos(T rho, const Coef<T>& c, T& p_lbe, T& dp_lbe) {
  const T v = c.b4 * rho;
  const T iw = recip(T(1) - v);
  const T iw3 = iw * iw * iw;
  const T z = (T(1) + v * (T(1) + v * (T(1) - v))) * iw3;
  const T dz = (T(1) + v * (T(4) + v * (T(4) + v * (v - T(4))))) * (iw3 * iw);
  p_lbe = rho * (c.kprt * z + c.e_rho * rho);
  dp_lbe = c.kprt * dz + c.de_rho * rho;
}

// m = M f (supplement Eq. 4) as an add/subtract tree; m[0] is density(f).
template <typename T>
__host__ __device__ __forceinline__ void forward_moments(const T* f, T* m) {
  const T a13 = f[1] + f[3], a24 = f[2] + f[4], d57 = f[5] + f[7], d68 = f[6] + f[8];
  const T s13 = f[1] - f[3], s24 = f[2] - f[4], e57 = f[5] - f[7], e86 = f[8] - f[6];
  const T ax = a13 + a24, dg = d57 + d68;
  m[0] = f[0] + (ax + dg);  // = density(f)
  m[1] = T(2) * dg - ax - T(4) * f[0];
  m[2] = T(4) * f[0] - T(2) * ax + dg;
  m[3] = s13 + (e57 + e86);
  m[4] = (e57 + e86) - T(2) * s13;
  m[5] = s24 + (e57 - e86);
  m[6] = (e57 - e86) - T(2) * s24;
  m[7] = a13 - a24;
  m[8] = d57 - d68;
}

// f = M^-1 m = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m,
// with the rest population formed last as m_0 minus the eight moving ones
// (so the populations sum to m_0 up to one rounding).
template <typename T>
__host__ __device__ __forceinline__ void inverse_moments(const T* m, T* f) {
  const T w0 = m[0] * T(1.0 / 9.0), w1 = m[1] * T(1.0 / 36.0), w2 = m[2] * T(1.0 / 36.0);
  const T w3 = m[3] * T(1.0 / 6.0), w4 = m[4] * T(1.0 / 12.0);
  const T w5 = m[5] * T(1.0 / 6.0), w6 = m[6] * T(1.0 / 12.0);
  const T w7 = m[7] * T(0.25), w8 = m[8] * T(0.25);
  const T A = w0 - w1 - T(2) * w2, X = w3 - T(2) * w4, Y = w5 - T(2) * w6;
  f[1] = (A + w7) + X;
  f[3] = (A + w7) - X;
  f[2] = (A - w7) + Y;
  f[4] = (A - w7) - Y;
  const T D = w0 + T(2) * w1 + w2, P = w3 + w4, Q = w5 + w6;
  f[5] = (D + w8) + (P + Q);
  f[7] = (D + w8) - (P + Q);
  f[6] = (D - w8) + (Q - P);
  f[8] = (D - w8) - (Q - P);
  f[0] = m[0] - (((f[1] + f[3]) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8])));
}

// Node-local quantities at time t: velocity with the half-force correction
// (main Eq. 5), force F = G^2 rho g, and the pressure slope.
template <typename T>
struct NodeState {
  T rho, ux, uy, Fx, Fy, p_lbe, dp_lbe, eta;
};

template <typename T>
__host__ __device__ __forceinline__ NodeState<T> node_state(T rho, T jx, T jy, T gx, T gy, const Coef<T>& c) {
  NodeState<T> s;
  s.rho = rho;
  s.Fx = c.g2 * rho * gx;
  s.Fy = c.g2 * rho * gy;
  const T inv = recip(rho);
  s.ux = (jx + T(0.5) * s.Fx) * inv;
  s.uy = (jy + T(0.5) * s.Fy) * inv;
  eos(rho, c, s.p_lbe, s.dp_lbe);
  s.eta = T(3) * s.p_lbe - rho;  // p_LBE = (rho + eta)/3 (main Eq. 9, alpha1 = -1, beta1 = 1)
  return s;
}

// Moment-space collision (supplement Eq. 1) by the six-step sequence of
// supplement Sec. IV, returned as the change of the moments m-bar - m for
// the pre-collision moments m, already scaled by the diagonal of
// M^-1 = M^T D: w = D (m-bar - m), so that f-bar = f + M^T w.  Row 0 does
// not change (mass) and rows 3, 5 gain F (w = F/6); rows 1, 2, 4, 6, 7, 8
// follow the six steps below.  The scalings and the signs of the correction
// terms are folded into the w_* constants, and the cubic velocity monomials
// u_x^3, u_y^3, u_x u_y^2, u_x^2 u_y are formed once for the force moments
// and for the T and X terms (T . g + dp X . g is one coefficient per
// monomial and row).  g is the stencil gradient (= grad rho, supplement
// Eq. 61); grad p_LBE = dp_lbe g.
template <typename T>
__host__ __device__ __forceinline__ void collide_scaled(const T* m, const NodeState<T>& s, T gx, T gy,
                                                        const Coef<T>& c, T* w) {
  const T rho = s.rho, ux = s.ux, uy = s.uy, Fx = s.Fx, Fy = s.Fy, dp = s.dp_lbe;
  const T ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy, u2 = ux2 + uy2, dxy = ux2 - uy2;
  const T c3x = ux * ux2, c3y = uy * uy2, cxyy = uxy * uy, cxxy = uxy * ux;
  // equilibrium moments (main Eq. 3) and half force moments (main Eq. 4)
  const T meq1 = T(2) * (s.eta - rho) + T(3) * rho * u2;
  const T meq2 = c.alpha2 * rho + c.beta2 * s.eta + rho * (T(9) * ux2 * uy2 - T(3) * u2);
  const T meq4 = rho * (T(3) * cxyy - ux), meq6 = rho * (T(3) * cxxy - uy);
  const T meq7 = rho * dxy, meq8 = rho * uxy;
  const T Fxu = Fx * ux, Fyu = Fy * uy;
  const T Fu3 = T(3) * (Fxu + Fyu);
  const T hF2 = T(9) * (Fx * cxyy + Fy * cxxy) - Fu3;
  const T hF4 = T(1.5) * (Fx * uy2 + T(2) * Fy * uxy) - T(0.5) * Fx;
  const T hF6 = T(1.5) * (Fy * ux2 + T(2) * Fx * uxy) - T(0.5) * Fy;
  const T hF7 = Fxu - Fyu;
  const T hF8 = T(0.5) * (Fx * uy + Fy * ux);
  // (1) d = m - m^eq + F_m/2
  const T d1 = m[1] - meq1 + Fu3, d2 = m[2] - meq2 + hF2, d4 = m[4] - meq4 + hF4;
  const T d6 = m[6] - meq6 + hF6, d7 = m[7] - meq7 + hF7, d8 = m[8] - meq8 + hF8;
  // (2)-(3) D = (1 - s/2)(d + N d)
  const T D1 = c.om_e * (d1 + c.k_seps_h * d2 + c.h_sq_h * (ux * d4 + uy * d6));
  const T D7 = c.om_p * (d7 + c.b_sq * (ux * d4 - uy * d6));
  const T D8 = c.om_p * (d8 + c.b_sq_h * (uy * d4 + ux * d6));
  // (4) corrections with (5) m-bar - m = 2 (D - d + F_m/2) - corrections and
  // (6) S Q_m, each row times its factor of D
  const T gg = gx * gx + gy * gy;
  const T b1 = dp * c.w_x1 + c.w_t1b, b7 = dp * c.w_x7 + c.w_t7b, b8 = dp * c.w_x8 + c.w_t8;
  w[1] = T(2.0 / 36.0) * ((D1 - d1) + Fu3) + c.w_r11 * u2 * D1 + c.w_r17 * dxy * D7 + c.w_r18 * uxy * D8 +
         (c.w_t1a * c3x + b1 * cxyy) * gx + (c.w_t1a * c3y + b1 * cxxy) * gy + c.w_q1 * gg;
  w[2] = T(2.0 / 36.0) * hF2 - c.w_seps * d2 - c.w_q2 * gg;
  w[4] = T(1.0 / 6.0) * hF4 - c.w_sq * d4;
  w[6] = T(1.0 / 6.0) * hF6 - c.w_sq * d6;
  w[7] = T(0.5) * ((D7 - d7) + hF7) + c.w_r71 * dxy * D1 + c.w_r77 * u2 * D7 +
         (c.w_t7 * c3x + b7 * cxyy) * gx - (c.w_t7 * c3y + b7 * cxxy) * gy + c.w_q7 * (gx * gx - gy * gy);
  w[8] = T(0.5) * ((D8 - d8) + hF8) + c.w_r81 * uxy * D1 + c.w_r88 * u2 * D8 +
         b8 * ((c3y + T(2) * cxxy) * gx + (c3x + T(2) * cxyy) * gy) + c.w_q7 * (gx * gy);
  w[3] = Fx * T(1.0 / 6.0);
  w[5] = Fy * T(1.0 / 6.0);
}

// f += M^T w (w = D dm from collide_scaled, w_0 = 0).
template <typename T>
__host__ __device__ __forceinline__ void add_transpose_moments(const T* w, T* f) {
  const T A = -(w[1] + T(2) * w[2]), X = w[3] - T(2) * w[4], Y = w[5] - T(2) * w[6];
  f[0] += T(4) * (w[2] - w[1]);
  f[1] += (A + w[7]) + X;
  f[3] += (A + w[7]) - X;
  f[2] += (A - w[7]) + Y;
  f[4] += (A - w[7]) - Y;
  const T D = T(2) * w[1] + w[2], P = w[3] + w[4], Q = w[5] + w[6];
  f[5] += (D + w[8]) + (P + Q);
  f[7] += (D + w[8]) - (P + Q);
  f[6] += (D - w[8]) + (Q - P);
  f[8] += (D - w[8]) - (Q - P);
}

// f-bar from pre-collision f at one node of density rho (density(f)), given
// the stencil gradient g.
template <typename T>
__host__ __device__ __forceinline__ void collide_node(T* f, T rho, T gx, T gy, const Coef<T>& c) {
  T m[9], w[9];
  forward_moments(f, m);
  const NodeState<T> s = node_state(rho, m[3], m[5], gx, gy, c);
  collide_scaled(m, s, gx, gy, c, w);
  add_transpose_moments(w, f);
}

// Equilibrium populations f^eq = M^-1 m^eq(rho, u, eta(rho)).
template <typename T>
__host__ __device__ __forceinline__ void equilibrium_node(T rho, T ux, T uy, const Coef<T>& c, T* f) {
  T p, dp;
  eos(rho, c, p, dp);
  const T eta = T(3) * p - rho;
  const T ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2;
  T m[9];
  m[0] = rho;
  m[1] = T(2) * (eta - rho) + T(3) * rho * u2;
  m[2] = c.alpha2 * rho + c.beta2 * eta + rho * (T(9) * ux2 * uy2 - T(3) * u2);
  m[3] = rho * ux;
  m[4] = rho * ux * (T(3) * uy2 - T(1));
  m[5] = rho * uy;
  m[6] = rho * uy * (T(3) * ux2 - T(1));
  m[7] = rho * (ux2 - uy2);
  m[8] = rho * ux * uy;
  inverse_moments(m, f);
}

// Reference populations of the 2-byte storages: the rest equilibrium
// f^eq(rho~, eta_ref(rho~), u = 0) of a reference density rho~, per velocity
// class (0 rest, 1 axis, 2 diagonal), as cubic polynomials in rho~ whose
// coefficients the host fits once.  Stored values are S (f - f_ref).
template <typename T>
struct RefPoly {
  T c[3][4];   // class value = ((c3 r + c2) r + c1) r + c0
  T scale;     // S, a power of two
  T inv_scale; // 1/S
};

__host__ __device__ __forceinline__ constexpr int velocity_class(int i) { return i == 0 ? 0 : (i <= 4 ? 1 : 2); }

template <typename T>
__host__ __device__ __forceinline__ T ref_value(const RefPoly<T>& q, int cls, T r) {
  return ((q.c[cls][3] * r + q.c[cls][2]) * r + q.c[cls][1]) * r + q.c[cls][0];
}

// ---------------------------------------------------------------------------
// Adjoint of the per-node collision
// ---------------------------------------------------------------------------
// M^T a by the same add/subtract tree as inverse_moments (M^-1 = M^T D).
template <typename T>
__host__ __device__ __forceinline__ void transpose_moments(const T* a, T* f) {
  const T A = a[0] - a[1] - T(2) * a[2], X = a[3] - T(2) * a[4], Y = a[5] - T(2) * a[6];
  f[0] = a[0] + T(4) * (a[2] - a[1]);
  f[1] = (A + a[7]) + X;
  f[3] = (A + a[7]) - X;
  f[2] = (A - a[7]) + Y;
  f[4] = (A - a[7]) - Y;
  const T D = a[0] + T(2) * a[1] + a[2], P = a[3] + a[4], Q = a[5] + a[6];
  f[5] = (D + a[8]) + (P + Q);
  f[7] = (D + a[8]) - (P + Q);
  f[6] = (D - a[8]) + (Q - P);
  f[8] = (D - a[8]) - (Q - P);
}

// Reverse-mode derivative of collide_node.  Given the pre-collision
// populations f, the stencil gradient g and lam = dL/d f-bar, returns
// lam_f = dL/d f (at fixed g), a_g = dL/d g, and adds dL/d(G'^2, K', R T)
// to a_th.  The forward quantities are recomputed here; the sweep visits the
// assignments of collide_node / collide_scaled / node_state / eos in
// reverse order, written for the unscaled moments (m-bar = m + D^-1 w).
template <typename T>
__host__ __device__ __forceinline__ void collide_node_vjp(const T* f, T gx, T gy, const Coef<T>& c, const T* lam,
                                                          T* lam_f, T& a_gx, T& a_gy, T* a_th) {
  // ---- forward recomputation --------------------------------------------
  T m[9];
  forward_moments(f, m);
  const T rho = m[0];
  const T Fx = c.g2 * rho * gx, Fy = c.g2 * rho * gy;
  const T inv = recip(rho);
  const T ux = (m[3] + T(0.5) * Fx) * inv, uy = (m[5] + T(0.5) * Fy) * inv;
  const T v = c.b4 * rho;
  const T iw = recip(T(1) - v);
  const T iw3 = iw * iw * iw;
  const T z = (T(1) + v * (T(1) + v * (T(1) - v))) * iw3;
  const T dz = (T(1) + v * (T(4) + v * (T(4) + v * (v - T(4))))) * (iw3 * iw);
  const T p = rho * (c.kprt * z + c.e_rho * rho);
  const T dp = c.kprt * dz + c.de_rho * rho;
  const T eta = T(3) * p - rho;
  const T ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy, u2 = ux2 + uy2, dxy = ux2 - uy2;
  const T meq1 = T(2) * (eta - rho) + T(3) * rho * u2;
  const T meq2 = c.alpha2 * rho + c.beta2 * eta + rho * (T(9) * ux2 * uy2 - T(3) * u2);
  const T meq4 = rho * ux * (T(3) * uy2 - T(1));
  const T meq6 = rho * uy * (T(3) * ux2 - T(1));
  const T meq7 = rho * dxy, meq8 = rho * uxy;
  const T Fu3 = T(3) * (Fx * ux + Fy * uy);
  const T hF2 = T(9) * (Fx * ux * uy2 + Fy * uy * ux2) - Fu3;
  const T hF4 = T(1.5) * (Fx * uy2 + T(2) * Fy * uxy) - T(0.5) * Fx;
  const T hF6 = T(1.5) * (Fy * ux2 + T(2) * Fx * uxy) - T(0.5) * Fy;
  const T hF7 = Fx * ux - Fy * uy;
  const T hF8 = T(0.5) * (Fx * uy + Fy * ux);
  const T d1 = m[1] - meq1 + Fu3, d2 = m[2] - meq2 + hF2, d4 = m[4] - meq4 + hF4;
  const T d6 = m[6] - meq6 + hF6, d7 = m[7] - meq7 + hF7, d8 = m[8] - meq8 + hF8;
  const T D1 = c.om_e * (d1 + c.k_seps_h * d2 + c.h_sq_h * (ux * d4 + uy * d6));
  const T D7 = c.om_p * (d7 + c.b_sq * (ux * d4 - uy * d6));
  const T D8 = c.om_p * (d8 + c.b_sq_h * (uy * d4 + ux * d6));
  const T R11 = c.cR11 * u2, R17 = c.cR17 * dxy, R18 = c.cR18 * uxy;
  const T t1x = ux * (c.cT1a * ux2 - c.cT1b * uy2), t1y = uy * (c.cT1a * uy2 - c.cT1b * ux2);
  const T x1x = c.cX1 * uxy * uy, x1y = c.cX1 * uxy * ux;
  const T R71 = c.cR71 * dxy, R77 = c.cR77 * u2;
  const T t7x = c.cT7 * ux * (ux2 + c.two_b * uy2), t7y = -c.cT7 * uy * (uy2 + c.two_b * ux2);
  const T x7x = c.cX7 * uxy * uy, x7y = -c.cX7 * uxy * ux;
  const T R81 = c.cR81 * uxy, R88 = c.cR88 * u2;
  const T v8x = uy * (uy2 + T(2) * ux2), v8y = ux * (ux2 + T(2) * uy2);
  const T W8 = c.cT8 + dp * c.cX8, V8 = v8x * gx + v8y * gy;
  const T gg = gx * gx + gy * gy;

  // ---- lam of the post-collision moments: (M^-1)^T lam = D M lam ---------
  T l[9];
  forward_moments(lam, l);
  l[0] *= T(1.0 / 9.0), l[1] *= T(1.0 / 36.0), l[2] *= T(1.0 / 36.0), l[3] *= T(1.0 / 6.0);
  l[4] *= T(1.0 / 12.0), l[5] *= T(1.0 / 6.0), l[6] *= T(1.0 / 12.0), l[7] *= T(0.25), l[8] *= T(0.25);

  T a_rho = l[0], a_ux = 0, a_uy = 0, a_Fx = l[3], a_Fy = l[5], a_dp = 0, a_eta = 0, a_g2 = 0;
  T a_m[9] = {0, 0, 0, l[3], 0, l[5], 0, 0, 0};
  a_gx = 0, a_gy = 0;
  // post-collision rows (collide_scaled steps (5)-(6))
  T a_meq1 = l[1], a_hF1 = l[1], a_d1 = -l[1], a_D1 = T(2) * l[1], a_c1 = -l[1];
  T a_gg = c.q1 * l[1] - c.s_eps * T(0.5) * c.g2 * l[2];
  a_g2 += T(0.5) * (c.s_e - c.kq2) * gg * l[1] - c.s_eps * T(0.5) * gg * l[2];
  T a_meq2 = l[2], a_hF2 = l[2], a_d2 = c.one_m_seps * l[2];
  T a_meq4 = l[4], a_hF4 = l[4], a_d4 = c.one_m_sq * l[4];
  T a_meq6 = l[6], a_hF6 = l[6], a_d6 = c.one_m_sq * l[6];
  T a_meq7 = l[7], a_hF7 = l[7], a_d7 = -l[7], a_D7 = T(2) * l[7], a_c7 = -l[7];
  a_gx += T(2) * c.q7 * gx * l[7], a_gy -= T(2) * c.q7 * gy * l[7];
  a_g2 += c.s_p * T(1.0 / 12.0) * (gx * gx - gy * gy) * l[7];
  T a_meq8 = l[8], a_hF8 = l[8], a_d8 = -l[8], a_D8 = T(2) * l[8], a_c8 = -l[8];
  a_gx += c.q7 * gy * l[8], a_gy += c.q7 * gx * l[8];
  a_g2 += c.s_p * T(1.0 / 12.0) * gx * gy * l[8];
  a_gx += T(2) * gx * a_gg, a_gy += T(2) * gy * a_gg;

  T a_u2 = 0, a_dxy = 0, a_uxy = 0, a_ux2 = 0, a_uy2 = 0;
  // corr8 = R81 D1 + R88 D8 + W8 V8
  {
    a_uxy += c.cR81 * D1 * a_c8, a_D1 += R81 * a_c8;
    a_u2 += c.cR88 * D8 * a_c8, a_D8 += R88 * a_c8;
    a_dp += c.cX8 * V8 * a_c8;
    const T a_V = W8 * a_c8;
    const T a_v8x = gx * a_V, a_v8y = gy * a_V;
    a_gx += v8x * a_V, a_gy += v8y * a_V;
    a_ux += T(4) * uxy * a_v8x + (T(3) * ux2 + T(2) * uy2) * a_v8y;
    a_uy += (T(3) * uy2 + T(2) * ux2) * a_v8x + T(4) * uxy * a_v8y;
  }
  // corr7 = R71 D1 + R77 D7 + (t7x + dp x7x) gx + (t7y + dp x7y) gy
  {
    a_dxy += c.cR71 * D1 * a_c7, a_D1 += R71 * a_c7;
    a_u2 += c.cR77 * D7 * a_c7, a_D7 += R77 * a_c7;
    a_dp += (x7x * gx + x7y * gy) * a_c7;
    a_gx += (t7x + dp * x7x) * a_c7, a_gy += (t7y + dp * x7y) * a_c7;
    const T a_t7x = gx * a_c7, a_t7y = gy * a_c7, a_x7x = dp * gx * a_c7, a_x7y = dp * gy * a_c7;
    a_ux += c.cT7 * (T(3) * ux2 + c.two_b * uy2) * a_t7x - c.cT7 * T(2) * c.two_b * uxy * a_t7y;
    a_uy += c.cT7 * T(2) * c.two_b * uxy * a_t7x - c.cT7 * (T(3) * uy2 + c.two_b * ux2) * a_t7y;
    a_ux += c.cX7 * uy2 * a_x7x - T(2) * c.cX7 * uxy * a_x7y;
    a_uy += T(2) * c.cX7 * uxy * a_x7x - c.cX7 * ux2 * a_x7y;
  }
  // corr1 = R11 D1 + R17 D7 + R18 D8 + (t1x + dp x1x) gx + (t1y + dp x1y) gy
  {
    a_u2 += c.cR11 * D1 * a_c1, a_D1 += R11 * a_c1;
    a_dxy += c.cR17 * D7 * a_c1, a_D7 += R17 * a_c1;
    a_uxy += c.cR18 * D8 * a_c1, a_D8 += R18 * a_c1;
    a_dp += (x1x * gx + x1y * gy) * a_c1;
    a_gx += (t1x + dp * x1x) * a_c1, a_gy += (t1y + dp * x1y) * a_c1;
    const T a_t1x = gx * a_c1, a_t1y = gy * a_c1, a_x1x = dp * gx * a_c1, a_x1y = dp * gy * a_c1;
    a_ux += (T(3) * c.cT1a * ux2 - c.cT1b * uy2) * a_t1x - T(2) * c.cT1b * uxy * a_t1y;
    a_uy += -T(2) * c.cT1b * uxy * a_t1x + (T(3) * c.cT1a * uy2 - c.cT1b * ux2) * a_t1y;
    a_ux += c.cX1 * uy2 * a_x1x + T(2) * c.cX1 * uxy * a_x1y;
    a_uy += T(2) * c.cX1 * uxy * a_x1x + c.cX1 * ux2 * a_x1y;
  }
  // D8 = om_p (d8 + b_sq_h (uy d4 + ux d6))
  {
    a_d8 += c.om_p * a_D8;
    const T t = c.om_p * c.b_sq_h * a_D8;
    a_uy += d4 * t, a_d4 += uy * t, a_ux += d6 * t, a_d6 += ux * t;
  }
  // D7 = om_p (d7 + b_sq (ux d4 - uy d6))
  {
    a_d7 += c.om_p * a_D7;
    const T t = c.om_p * c.b_sq * a_D7;
    a_ux += d4 * t, a_d4 += ux * t, a_uy -= d6 * t, a_d6 -= uy * t;
  }
  // D1 = om_e (d1 + k_seps_h d2 + h_sq_h (ux d4 + uy d6))
  {
    a_d1 += c.om_e * a_D1;
    a_d2 += c.om_e * c.k_seps_h * a_D1;
    const T t = c.om_e * c.h_sq_h * a_D1;
    a_ux += d4 * t, a_d4 += ux * t, a_uy += d6 * t, a_d6 += uy * t;
  }
  // d_k = m_k - meq_k + hF_k
  a_m[1] += a_d1, a_meq1 -= a_d1, a_hF1 += a_d1;
  a_m[2] += a_d2, a_meq2 -= a_d2, a_hF2 += a_d2;
  a_m[4] += a_d4, a_meq4 -= a_d4, a_hF4 += a_d4;
  a_m[6] += a_d6, a_meq6 -= a_d6, a_hF6 += a_d6;
  a_m[7] += a_d7, a_meq7 -= a_d7, a_hF7 += a_d7;
  a_m[8] += a_d8, a_meq8 -= a_d8, a_hF8 += a_d8;
  // half force moments
  a_Fx += T(0.5) * uy * a_hF8, a_uy += T(0.5) * Fx * a_hF8, a_Fy += T(0.5) * ux * a_hF8, a_ux += T(0.5) * Fy * a_hF8;
  a_Fx += ux * a_hF7, a_ux += Fx * a_hF7, a_Fy -= uy * a_hF7, a_uy -= Fy * a_hF7;
  a_Fy += (T(1.5) * ux2 - T(0.5)) * a_hF6, a_ux2 += T(1.5) * Fy * a_hF6, a_Fx += T(3) * uxy * a_hF6,
      a_uxy += T(3) * Fx * a_hF6;
  a_Fx += (T(1.5) * uy2 - T(0.5)) * a_hF4, a_uy2 += T(1.5) * Fx * a_hF4, a_Fy += T(3) * uxy * a_hF4,
      a_uxy += T(3) * Fy * a_hF4;
  T a_Fu3 = a_hF1 - a_hF2;
  a_Fx += T(9) * ux * uy2 * a_hF2, a_ux += T(9) * Fx * uy2 * a_hF2, a_uy2 += T(9) * Fx * ux * a_hF2;
  a_Fy += T(9) * uy * ux2 * a_hF2, a_uy += T(9) * Fy * ux2 * a_hF2, a_ux2 += T(9) * Fy * uy * a_hF2;
  a_Fx += T(3) * ux * a_Fu3, a_ux += T(3) * Fx * a_Fu3, a_Fy += T(3) * uy * a_Fu3, a_uy += T(3) * Fy * a_Fu3;
  // equilibrium moments
  a_rho += uxy * a_meq8, a_uxy += rho * a_meq8;
  a_rho += dxy * a_meq7, a_dxy += rho * a_meq7;
  a_rho += uy * (T(3) * ux2 - T(1)) * a_meq6, a_uy += rho * (T(3) * ux2 - T(1)) * a_meq6,
      a_ux2 += T(3) * rho * uy * a_meq6;
  a_rho += ux * (T(3) * uy2 - T(1)) * a_meq4, a_ux += rho * (T(3) * uy2 - T(1)) * a_meq4,
      a_uy2 += T(3) * rho * ux * a_meq4;
  a_rho += (c.alpha2 + T(9) * ux2 * uy2 - T(3) * u2) * a_meq2, a_eta += c.beta2 * a_meq2;
  a_ux2 += T(9) * rho * uy2 * a_meq2, a_uy2 += T(9) * rho * ux2 * a_meq2, a_u2 -= T(3) * rho * a_meq2;
  a_eta += T(2) * a_meq1, a_rho += (T(3) * u2 - T(2)) * a_meq1, a_u2 += T(3) * rho * a_meq1;
  // velocity products
  a_ux2 += a_u2 + a_dxy, a_uy2 += a_u2 - a_dxy;
  a_ux += uy * a_uxy + T(2) * ux * a_ux2;
  a_uy += ux * a_uxy + T(2) * uy * a_uy2;
  // ---- node state ----------------------------------------------------------
  // eta = 3 p - rho;  dp = kprt dz + de_rho rho;  p = rho (kprt z + e_rho rho)
  const T a_p = T(3) * a_eta;
  a_rho -= a_eta;
  const T a_dz = c.kprt * a_dp;
  a_rho += c.de_rho * a_dp + (c.kprt * z + T(2) * c.e_rho * rho) * a_p;
  const T a_z = rho * c.kprt * a_p;
  const T a_kprt = dz * a_dp + rho * z * a_p;
  const T a_erho = rho * rho * a_p, a_derho = rho * a_dp;
  // z(rho) = Z(v) with d z / d rho = (dz - z)/rho (dz = d(rho Z)/d rho), and
  // d dz / d rho = (b/4) (8 + 20 v - 4 v^2) / (1 - v)^5
  a_rho += a_z * (dz - z) * inv + a_dz * c.b4 * (T(8) + v * (T(20) - T(4) * v)) * (iw3 * iw * iw);
  // u = (j + F/2) / rho
  a_m[3] += inv * a_ux, a_Fx += T(0.5) * inv * a_ux;
  a_m[5] += inv * a_uy, a_Fy += T(0.5) * inv * a_uy;
  a_rho -= (ux * a_ux + uy * a_uy) * inv;
  // F = G'^2 rho g
  a_rho += c.g2 * (gx * a_Fx + gy * a_Fy);
  a_gx += c.g2 * rho * a_Fx, a_gy += c.g2 * rho * a_Fy;
  a_g2 += rho * (gx * a_Fx + gy * a_Fy);
  // parameters: kprt = K' RT, e_rho = G'^2/2 - K' a, de_rho = G'^2 - 2 K' a
  a_th[0] += a_g2 + T(0.5) * a_erho + a_derho;
  a_th[1] += c.rt * a_kprt - c.a * a_erho - T(2) * c.a * a_derho;
  a_th[2] += c.kp * a_kprt;
  // ---- populations: m = M f and rho = sum f ------------------------------
  a_m[0] = a_rho;
  transpose_moments(a_m, lam_f);
}

// Adjoint of the equilibrium initial state f^eq(rho0, u0, eta(rho0)) with
// respect to rho0 (at fixed u0) and to (G'^2, K', R T), for lam = dL/d f^eq.
template <typename T>
__host__ __device__ __forceinline__ T equilibrium_vjp(T rho, T ux, T uy, const Coef<T>& c, const T* lam, T* a_th) {
  // lam of the equilibrium moments: (M^-1)^T lam = D M lam
  T l[9];
  forward_moments(lam, l);
  l[0] *= T(1.0 / 9.0), l[1] *= T(1.0 / 36.0), l[2] *= T(1.0 / 36.0), l[3] *= T(1.0 / 6.0);
  l[4] *= T(1.0 / 12.0), l[5] *= T(1.0 / 6.0), l[6] *= T(1.0 / 12.0), l[7] *= T(0.25), l[8] *= T(0.25);
  const T ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2;
  T p, dp;
  eos(rho, c, p, dp);
  const T v = c.b4 * rho;
  const T iw = recip(T(1) - v);
  const T z = (T(1) + v * (T(1) + v * (T(1) - v))) * (iw * iw * iw);
  // d m^eq / d rho at fixed u and eta, and d m^eq / d eta
  const T dm_rho = l[0] + (T(3) * u2 - T(2)) * l[1] + (c.alpha2 + T(9) * ux2 * uy2 - T(3) * u2) * l[2] +
                   ux * l[3] + ux * (T(3) * uy2 - T(1)) * l[4] + uy * l[5] + uy * (T(3) * ux2 - T(1)) * l[6] +
                   (ux2 - uy2) * l[7] + ux * uy * l[8];
  const T a_eta = T(2) * l[1] + c.beta2 * l[2];
  // eta = 3 p_LBE - rho:  d eta / d rho = 3 dp - 1;  p = K' rho (RT z - a rho) + G'^2 rho^2 / 2
  a_th[0] += a_eta * T(1.5) * rho * rho;
  a_th[1] += a_eta * T(3) * rho * (c.rt * z - c.a * rho);
  a_th[2] += a_eta * T(3) * c.kp * rho * z;
  return dm_rho + a_eta * (T(3) * dp - T(1));
}

}  // namespace lbm
