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

// a b + c with one rounding.  The functions of the forward step below
// disable contraction (fp contract off) and fuse where they say so, so
// that a node's update is the same sequence of roundings in every kernel
// that inlines them, whatever products the compiler would otherwise fuse.
template <typename T>
__host__ __device__ __forceinline__ T fma_(T a, T b, T c) {
  if constexpr (sizeof(T) == 4)
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
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
#pragma clang fp contract(off)
  const T third = T(1) / T(3), twelfth = T(1) / T(12);
  const T dd1 = rNE - rSW, dd2 = rSE - rNW;  // the two diagonals
  gx = fma_(twelfth, dd1 + dd2, third * (rE - rW));
  gy = fma_(twelfth, dd1 - dd2, third * (rN - rS));
}

// Pressure of the lattice Boltzmann equation and its density slope:
// p_LBE = K'[rho R T Z - a rho^2] + G^2 rho^2/2 (main Eqs. 18, 20),
// Z = (1 + v + v^2 - v^3)/(1 - v)^3, d(rho Z)/d rho = (1 + 4v + 4v^2 - 4v^3 + v^4)/(1 - v)^4.
template <typename T>
__host__ __device__ __forceinline__ void eos(T rho, const Coef<T>& c, T& p_lbe, T& dp_lbe) {
#pragma clang fp contract(off)
  const T v = c.b4 * rho;
  const T iw = recip(T(1) - v);
  const T iw3 = iw * iw * iw;
  const T z = fma_(v, fma_(v, T(1) - v, T(1)), T(1)) * iw3;
  const T dz = fma_(v, fma_(v, fma_(v, v - T(4), T(4)), T(4)), T(1)) * (iw3 * iw);
  p_lbe = rho * fma_(c.kprt, z, c.e_rho * rho);
  dp_lbe = fma_(c.kprt, dz, c.de_rho * rho);
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
#pragma clang fp contract(off)
  NodeState<T> s;
  s.rho = rho;
  s.Fx = c.g2 * rho * gx;
  s.Fy = c.g2 * rho * gy;
  const T inv = recip(rho);
  s.ux = fma_(T(0.5), s.Fx, jx) * inv;
  s.uy = fma_(T(0.5), s.Fy, jy) * inv;
  eos(rho, c, s.p_lbe, s.dp_lbe);
  s.eta = fma_(T(3), s.p_lbe, -rho);  // p_LBE = (rho + eta)/3 (main Eq. 9, alpha1 = -1, beta1 = 1)
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
//
// kFewerOps: three fewer instructions per node (F_m2 from hF8, 3 u_x u_y
// shared by F_m4, F_m6 and 9 u_x^2 u_y^2 = (3 u_x u_y)^2, the factor 3 of
// F . u folded into its fused multiply-adds), in longer chains of dependent
// instructions: faster where many waves hide them (the 2-byte steps), slower
// in the two-step FP32 kernel.  The FP32 kernels keep the other form, which
// both of them share bit for bit.
template <typename T, bool kFewerOps = false>
__host__ __device__ __forceinline__ void collide_scaled(const T* m, const NodeState<T>& s, T gx, T gy,
                                                        const Coef<T>& c, T* w) {
#pragma clang fp contract(off)
  const T rho = s.rho, ux = s.ux, uy = s.uy, Fx = s.Fx, Fy = s.Fy, dp = s.dp_lbe;
  const T ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy, u2 = ux2 + uy2, dxy = ux2 - uy2;
  const T c3x = ux * ux2, c3y = uy * uy2, cxyy = uxy * uy, cxxy = uxy * ux;
  // half force moments (main Eq. 4; hF8 = 2 F_m8 / 2; with kFewerOps
  // F_x u_x u_y^2 + F_y u_x^2 u_y = u_x u_y hF8, Fu = F_m1 / 6) and
  // (1) d = m - m^eq + F_m/2 with the equilibrium moments of main Eq. 3
  // (kFewerOps: 9 u_x^2 u_y^2 = (3 u_x u_y)^2)
  const T Fxu = Fx * ux, Fyu = Fy * uy;
  T Fu3 = T(0), Fu = T(0), hF2, hF4, hF6, hF7, hF8, meq2, d1;
  if constexpr (!kFewerOps) {
    Fu3 = T(3) * (Fxu + Fyu);
    hF2 = fma_(T(9), fma_(Fx, cxyy, Fy * cxxy), -Fu3);
    hF4 = fma_(Fx, fma_(T(1.5), uy2, T(-0.5)), T(3) * Fy * uxy);
    hF6 = fma_(Fy, fma_(T(1.5), ux2, T(-0.5)), T(3) * Fx * uxy);
    hF7 = Fxu - Fyu;
    hF8 = fma_(Fx, uy, Fy * ux);
    meq2 = fma_(rho, fma_(T(9) * ux2, uy2, T(-3) * u2), fma_(c.alpha2, rho, c.beta2 * s.eta));
    d1 = fma_(T(-3) * rho, u2, fma_(T(-2), s.eta - rho, m[1])) + Fu3;
  } else {
    Fu = Fxu + Fyu;
    const T uxy3 = T(3) * uxy;
    hF8 = fma_(Fx, uy, Fy * ux);
    hF2 = fma_(T(-3), Fu, (T(3) * uxy3) * hF8);
    hF4 = fma_(Fx, fma_(T(1.5), uy2, T(-0.5)), uxy3 * Fy);
    hF6 = fma_(Fy, fma_(T(1.5), ux2, T(-0.5)), uxy3 * Fx);
    hF7 = Fxu - Fyu;
    meq2 = fma_(rho, fma_(uxy3, uxy3, T(-3) * u2), fma_(c.alpha2, rho, c.beta2 * s.eta));
    d1 = fma_(T(3), Fu, fma_(T(-3) * rho, u2, fma_(T(-2), s.eta - rho, m[1])));
  }
  const T d2 = m[2] - meq2 + hF2;
  const T d4 = fma_(-rho, fma_(T(3), cxyy, -ux), m[4]) + hF4;
  const T d6 = fma_(-rho, fma_(T(3), cxxy, -uy), m[6]) + hF6;
  const T d7 = fma_(-rho, dxy, m[7]) + hF7;
  const T d8 = fma_(T(0.5), hF8, fma_(-rho, uxy, m[8]));
  // (2)-(3) D = (1 - s/2)(d + N d)
  const T D1 = c.om_e * fma_(c.h_sq_h, fma_(ux, d4, uy * d6), fma_(c.k_seps_h, d2, d1));
  const T D7 = c.om_p * fma_(c.b_sq, fma_(ux, d4, -(uy * d6)), d7);
  const T D8 = c.om_p * fma_(c.b_sq_h, fma_(uy, d4, ux * d6), d8);
  // (4) corrections with (5) m-bar - m = 2 (D - d + F_m/2) - corrections and
  // (6) S Q_m, each row times its factor of D
  const T gg = fma_(gx, gx, gy * gy);
  const T b1 = fma_(dp, c.w_x1, c.w_t1b), b7 = fma_(dp, c.w_x7, c.w_t7b), b8 = fma_(dp, c.w_x8, c.w_t8);
  T a;
  if constexpr (kFewerOps)
    a = T(2.0 / 36.0) * fma_(T(3), Fu, D1 - d1);
  else
    a = T(2.0 / 36.0) * ((D1 - d1) + Fu3);
  a = fma_(c.w_r11 * u2, D1, a);
  a = fma_(c.w_r17 * dxy, D7, a);
  a = fma_(c.w_r18 * uxy, D8, a);
  a = fma_(fma_(c.w_t1a, c3x, b1 * cxyy), gx, a);
  a = fma_(fma_(c.w_t1a, c3y, b1 * cxxy), gy, a);
  w[1] = fma_(c.w_q1, gg, a);
  w[2] = fma_(-c.w_q2, gg, fma_(-c.w_seps, d2, T(2.0 / 36.0) * hF2));
  w[4] = fma_(-c.w_sq, d4, T(1.0 / 6.0) * hF4);
  w[6] = fma_(-c.w_sq, d6, T(1.0 / 6.0) * hF6);
  a = T(0.5) * ((D7 - d7) + hF7);
  a = fma_(c.w_r71 * dxy, D1, a);
  a = fma_(c.w_r77 * u2, D7, a);
  a = fma_(fma_(c.w_t7, c3x, b7 * cxyy), gx, a);
  a = fma_(-fma_(c.w_t7, c3y, b7 * cxxy), gy, a);
  w[7] = fma_(c.w_q7, fma_(gx, gx, -(gy * gy)), a);
  a = T(0.5) * fma_(T(0.5), hF8, D8 - d8);
  a = fma_(c.w_r81 * uxy, D1, a);
  a = fma_(c.w_r88 * u2, D8, a);
  a = fma_(b8, fma_(fma_(T(2), cxxy, c3y), gx, fma_(T(2), cxyy, c3x) * gy), a);
  w[8] = fma_(c.w_q7, gx * gy, a);
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
template <typename T, bool kFewerOps = false>
__host__ __device__ __forceinline__ void collide_node(T* f, T rho, T gx, T gy, const Coef<T>& c) {
  T m[9], w[9];
  forward_moments(f, m);
  const NodeState<T> s = node_state(rho, m[3], m[5], gx, gy, c);
  collide_scaled<T, kFewerOps>(m, s, gx, gy, c, w);
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
// to a_th.  f-bar = f + M^T w with w from collide_scaled, so dL/dw = M lam;
// the sweep visits the assignments of collide_scaled, node_state and eos in
// reverse order, gathering the cotangents of the cubic velocity monomials
// (shared by the force moments and the T and X terms) before they are
// carried to u.
template <typename T>
__host__ __device__ __forceinline__ void collide_node_vjp(const T* f, T gx, T gy, const Coef<T>& c, const T* lam,
                                                          T* lam_f, T& a_gx, T& a_gy, T* a_th) {
  // ---- forward recomputation (collide_node) ------------------------------
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
  const T c3x = ux * ux2, c3y = uy * uy2, cxyy = uxy * uy, cxxy = uxy * ux;
  const T meq1 = T(2) * (eta - rho) + T(3) * rho * u2;
  const T meq2 = c.alpha2 * rho + c.beta2 * eta + rho * (T(9) * ux2 * uy2 - T(3) * u2);
  const T meq4 = rho * (T(3) * cxyy - ux), meq6 = rho * (T(3) * cxxy - uy);
  const T meq7 = rho * dxy, meq8 = rho * uxy;
  const T Fxu = Fx * ux, Fyu = Fy * uy;
  const T Fu3 = T(3) * (Fxu + Fyu);
  const T hF2 = T(9) * (Fx * cxyy + Fy * cxxy) - Fu3;
  const T hF4 = T(1.5) * (Fx * uy2 + T(2) * Fy * uxy) - T(0.5) * Fx;
  const T hF6 = T(1.5) * (Fy * ux2 + T(2) * Fx * uxy) - T(0.5) * Fy;
  const T hF7 = Fxu - Fyu;
  const T hF8 = T(0.5) * (Fx * uy + Fy * ux);
  const T d1 = m[1] - meq1 + Fu3, d2 = m[2] - meq2 + hF2, d4 = m[4] - meq4 + hF4;
  const T d6 = m[6] - meq6 + hF6, d7 = m[7] - meq7 + hF7, d8 = m[8] - meq8 + hF8;
  const T D1 = c.om_e * (d1 + c.k_seps_h * d2 + c.h_sq_h * (ux * d4 + uy * d6));
  const T D7 = c.om_p * (d7 + c.b_sq * (ux * d4 - uy * d6));
  const T D8 = c.om_p * (d8 + c.b_sq_h * (uy * d4 + ux * d6));
  const T gg = gx * gx + gy * gy;
  const T b1 = dp * c.w_x1 + c.w_t1b, b7 = dp * c.w_x7 + c.w_t7b, b8 = dp * c.w_x8 + c.w_t8;
  const T v8x = c3y + T(2) * cxxy, v8y = c3x + T(2) * cxyy;

  // ---- w: dL/dw = M lam ------------------------------------------------------
  T W[9];
  forward_moments(lam, W);
  const T A1 = W[1], A7 = W[7], A8 = W[8];
  T a_Fx = W[3] * T(1.0 / 6.0), a_Fy = W[5] * T(1.0 / 6.0);
  // w1
  T a_D1 = (T(2.0 / 36.0) + c.w_r11 * u2) * A1, a_d1 = -T(2.0 / 36.0) * A1, a_Fu3 = T(2.0 / 36.0) * A1;
  T a_u2 = c.w_r11 * D1 * A1, a_dxy = c.w_r17 * D7 * A1, a_uxy = c.w_r18 * D8 * A1;
  T a_D7 = c.w_r17 * dxy * A1, a_D8 = c.w_r18 * uxy * A1;
  const T gx1 = gx * A1, gy1 = gy * A1;
  T a_c3x = c.w_t1a * gx1, a_c3y = c.w_t1a * gy1, a_cxyy = b1 * gx1, a_cxxy = b1 * gy1;
  T a_dp = c.w_x1 * (cxyy * gx1 + cxxy * gy1);
  a_gx = (c.w_t1a * c3x + b1 * cxyy) * A1;
  a_gy = (c.w_t1a * c3y + b1 * cxxy) * A1;
  T a_gg = c.w_q1 * A1 - c.w_q2 * W[2];
  // w2, w4, w6
  T a_hF2 = T(2.0 / 36.0) * W[2], a_d2 = -c.w_seps * W[2];
  T a_hF4 = T(1.0 / 6.0) * W[4], a_d4 = -c.w_sq * W[4];
  T a_hF6 = T(1.0 / 6.0) * W[6], a_d6 = -c.w_sq * W[6];
  // w7
  a_D7 += (T(0.5) + c.w_r77 * u2) * A7;
  T a_d7 = -T(0.5) * A7, a_hF7 = T(0.5) * A7;
  a_dxy += c.w_r71 * D1 * A7, a_D1 += c.w_r71 * dxy * A7, a_u2 += c.w_r77 * D7 * A7;
  const T gx7 = gx * A7, gy7 = gy * A7;
  a_c3x += c.w_t7 * gx7, a_c3y -= c.w_t7 * gy7, a_cxyy += b7 * gx7, a_cxxy -= b7 * gy7;
  a_dp += c.w_x7 * (cxyy * gx7 - cxxy * gy7);
  a_gx += (c.w_t7 * c3x + b7 * cxyy) * A7 + T(2) * c.w_q7 * gx7;
  a_gy -= (c.w_t7 * c3y + b7 * cxxy) * A7 + T(2) * c.w_q7 * gy7;
  // w8
  a_D8 += (T(0.5) + c.w_r88 * u2) * A8;
  T a_d8 = -T(0.5) * A8, a_hF8 = T(0.5) * A8;
  a_uxy += c.w_r81 * D1 * A8, a_D1 += c.w_r81 * uxy * A8, a_u2 += c.w_r88 * D8 * A8;
  const T b8A = b8 * A8, gxb = gx * b8A, gyb = gy * b8A;
  a_c3y += gxb, a_cxxy += T(2) * gxb, a_c3x += gyb, a_cxyy += T(2) * gyb;
  a_dp += c.w_x8 * (v8x * gx + v8y * gy) * A8;
  a_gx += v8x * b8A + c.w_q7 * gy * A8;
  a_gy += v8y * b8A + c.w_q7 * gx * A8;
  a_gx += T(2) * gx * a_gg, a_gy += T(2) * gy * a_gg;
  // G'^2 through the Q_m terms: w_q1, w_q2, w_q7 are G'^2 (s_e - kq2)/72,
  // G'^2 s_eps/72 and G'^2 s_p/48
  T a_g2 = T(1.0 / 72.0) * gg * ((c.s_e - c.kq2) * A1 - c.s_eps * W[2]) +
           c.s_p * T(1.0 / 48.0) * ((gx * gx - gy * gy) * A7 + gx * gy * A8);
  // D1 = om_e (d1 + k_seps_h d2 + h_sq_h (ux d4 + uy d6))
  T a_ux, a_uy;
  {
    const T t = c.om_e * a_D1, th = c.h_sq_h * t;
    a_d1 += t, a_d2 += c.k_seps_h * t;
    a_ux = d4 * th, a_uy = d6 * th, a_d4 += ux * th, a_d6 += uy * th;
  }
  // D7 = om_p (d7 + b_sq (ux d4 - uy d6))
  {
    const T t = c.om_p * a_D7, tb = c.b_sq * t;
    a_d7 += t;
    a_ux += d4 * tb, a_d4 += ux * tb, a_uy -= d6 * tb, a_d6 -= uy * tb;
  }
  // D8 = om_p (d8 + b_sq_h (uy d4 + ux d6))
  {
    const T t = c.om_p * a_D8, tb = c.b_sq_h * t;
    a_d8 += t;
    a_uy += d4 * tb, a_d4 += uy * tb, a_ux += d6 * tb, a_d6 += ux * tb;
  }
  // d_k = m_k - meq_k + hF_k (hF_1 = Fu3)
  a_Fu3 += a_d1, a_hF2 += a_d2, a_hF4 += a_d4, a_hF6 += a_d6, a_hF7 += a_d7, a_hF8 += a_d8;
  // half force moments
  a_Fu3 -= a_hF2;
  a_Fx += T(9) * cxyy * a_hF2, a_cxyy += T(9) * Fx * a_hF2;
  a_Fy += T(9) * cxxy * a_hF2, a_cxxy += T(9) * Fy * a_hF2;
  a_Fx += (T(1.5) * uy2 - T(0.5)) * a_hF4, a_Fy += T(3) * uxy * a_hF4, a_uxy += T(3) * Fy * a_hF4;
  T a_uy2 = T(1.5) * Fx * a_hF4;
  a_Fy += (T(1.5) * ux2 - T(0.5)) * a_hF6, a_Fx += T(3) * uxy * a_hF6, a_uxy += T(3) * Fx * a_hF6;
  T a_ux2 = T(1.5) * Fy * a_hF6;
  a_Fx += T(0.5) * uy * a_hF8, a_uy += T(0.5) * Fx * a_hF8, a_Fy += T(0.5) * ux * a_hF8, a_ux += T(0.5) * Fy * a_hF8;
  const T a_Fxu = T(3) * a_Fu3 + a_hF7, a_Fyu = T(3) * a_Fu3 - a_hF7;
  a_Fx += ux * a_Fxu, a_ux += Fx * a_Fxu, a_Fy += uy * a_Fyu, a_uy += Fy * a_Fyu;
  // equilibrium moments (dL/d meq_k = -dL/d d_k)
  T a_eta = -(T(2) * a_d1 + c.beta2 * a_d2);
  T a_rho = -((T(3) * u2 - T(2)) * a_d1 + (c.alpha2 + T(9) * ux2 * uy2 - T(3) * u2) * a_d2 +
              (T(3) * cxyy - ux) * a_d4 + (T(3) * cxxy - uy) * a_d6 + dxy * a_d7 + uxy * a_d8);
  a_u2 -= T(3) * rho * (a_d1 - a_d2);
  const T r9 = -T(9) * rho * a_d2;
  a_ux2 += uy2 * r9, a_uy2 += ux2 * r9;
  a_cxyy -= T(3) * rho * a_d4, a_ux += rho * a_d4;
  a_cxxy -= T(3) * rho * a_d6, a_uy += rho * a_d6;
  a_dxy -= rho * a_d7, a_uxy -= rho * a_d8;
  // velocity monomials
  a_ux2 += a_u2 + a_dxy + ux * a_c3x, a_uy2 += a_u2 - a_dxy + uy * a_c3y;
  a_uxy += uy * a_cxyy + ux * a_cxxy;
  a_ux += ux2 * a_c3x + uxy * a_cxxy + uy * a_uxy + T(2) * ux * a_ux2;
  a_uy += uy2 * a_c3y + uxy * a_cxyy + ux * a_uxy + T(2) * uy * a_uy2;
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
  const T a_m3 = inv * a_ux, a_m5 = inv * a_uy;
  a_Fx += T(0.5) * a_m3, a_Fy += T(0.5) * a_m5;
  a_rho -= ux * a_m3 + uy * a_m5;
  // F = G'^2 rho g
  const T gF = gx * a_Fx + gy * a_Fy;
  a_rho += c.g2 * gF;
  a_gx += c.g2 * rho * a_Fx, a_gy += c.g2 * rho * a_Fy;
  a_g2 += rho * gF;
  // parameters: kprt = K' RT, e_rho = G'^2/2 - K' a, de_rho = G'^2 - 2 K' a
  a_th[0] += a_g2 + T(0.5) * a_erho + a_derho;
  a_th[1] += c.rt * a_kprt - c.a * a_erho - T(2) * c.a * a_derho;
  a_th[2] += c.kp * a_kprt;
  // ---- populations: lam_f = lam + M^T dL/dm ---------------------------------
  const T am[9] = {a_rho, a_d1, a_d2, a_m3, a_d4, a_m5, a_d6, a_d7, a_d8};
  transpose_moments(am, lam_f);
#pragma unroll
  for (int i = 0; i < 9; ++i) lam_f[i] += lam[i];
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
