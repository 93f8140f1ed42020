// Host parameter map of the self-tuning-EOS model (FP64, no GPU).
//
// Carnahan-Starling EOS (main Eq. 20), Maxwell construction (main Eq. 19),
// the flat-interface surface tension and thickness of the pressure tensor
// (main Eqs. 17-18) at K_EOS = K_INT = 1, the sigma/W -> K_EOS/K_INT map
// (main Eqs. 21, 23), the coefficient constraints (main Eq. 7) and the
// relaxation-rate constraint (main Eq. 16).  Lattice units, c = 1.
#include <cmath>
#include <cstdio>

#include "lbm_internal.h"

namespace lbm {
namespace {

// Printed constants of main Eq. 20: a = 0.496388 R^2 Tc^2/pc, b = 0.187295 R Tc/pc.
constexpr double kCsA = 0.496388;
constexpr double kCsB = 0.187295;

struct Cs {
  double rt, a, b;
  // compressibility factor Z = (1 + v + v^2 - v^3)/(1 - v)^3, v = b rho / 4
  double pressure(double r) const {
    const double v = 0.25 * b * r, w = 1.0 - v;
    return r * rt * (1.0 + v * (1.0 + v * (1.0 - v))) / (w * w * w) - a * r * r;
  }
  // d(rho Z)/d rho = (1 + 4v + 4v^2 - 4v^3 + v^4)/(1 - v)^4
  double repulsive_slope(double r) const {
    const double v = 0.25 * b * r, w = 1.0 - v;
    return rt * (1.0 + v * (4.0 + v * (4.0 + v * (-4.0 + v)))) / (w * w * w * w);
  }
  double slope(double r) const { return repulsive_slope(r) - 2.0 * a * r; }
  // chemical potential (psi_b' with psi_b the bulk free energy of Eq. 19)
  double chem(double r) const {
    const double v = 0.25 * b * r, w = 1.0 - v;
    return rt * (std::log(r) + v * (4.0 - 3.0 * v) / (w * w) + v * (4.0 - 2.0 * v) / (w * w * w)) -
           2.0 * a * r;
  }
  double free_energy(double r) const {
    const double v = 0.25 * b * r, w = 1.0 - v;
    return r * rt * (std::log(r) - 1.0 + v * (4.0 - 3.0 * v) / (w * w)) - a * r * r;
  }
};

// Root of a monotone bracketed function by bisection down to the last bit.
template <class F>
double bisect(F f, double lo, double hi) {
  double flo = f(lo);
  for (int it = 0; it < 400; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    const double fm = f(mid);
    if ((fm < 0) == (flo < 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton on P_n.
struct Gauss {
  static constexpr int n = 48;
  double x[n], w[n];
  Gauss() {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

template <class F>
double integrate(F f, double lo, double hi, int panels) {
  static const Gauss g;
  const double h = (hi - lo) / panels;
  double s = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double c = lo + (p + 0.5) * h;
    double ps = 0.0;
    for (int i = 0; i < Gauss::n; ++i) ps += g.w[i] * f(c + 0.5 * h * g.x[i]);
    s += 0.5 * h * ps;
  }
  return s;
}

}  // namespace

double critical_temperature(double a, double b, double r_gas) { return kCsB / kCsA * a / (b * r_gas); }

// Coexistence of the CS fluid at reduced temperature tr.  The two spinodal
// densities bracket the gas and liquid branches; the coexistence pressure
// equalises the chemical potentials of the two outer roots of p = P.
int maxwell(double tr, double a, double b, double r_gas, double* rho_g, double* rho_l, double* p0) {
  const Cs cs{r_gas * tr * critical_temperature(a, b, r_gas), a, b};
  const double top = 4.0 / b;
  // the slope is positive at small rho, negative between the spinodals and
  // positive again near the packing limit; locate its maximum-free dip
  const int n = 20000;
  double s1 = -1, s2 = -1, prev = cs.slope(top * 1e-7);
  for (int i = 1; i <= n; ++i) {
    const double r = top * i / (n + 1.0), s = cs.slope(r);
    if (prev > 0 && s <= 0 && s1 < 0) s1 = r;
    if (prev <= 0 && s > 0 && s1 > 0) {
      s2 = r;
      break;
    }
    prev = s;
  }
  if (s1 < 0 || s2 < 0) return LBM_ENOCOEX;
  const double dr = top / (n + 1.0);
  const double r1 = bisect([&](double r) { return -cs.slope(r); }, s1 - dr, s1);  // gas spinodal
  const double r2 = bisect([&](double r) { return cs.slope(r); }, s2 - dr, s2);   // liquid spinodal
  const double p_hi = cs.pressure(r1), p_lo = cs.pressure(r2);
  auto roots = [&](double P, double* g, double* l) {
    *g = bisect([&](double r) { return cs.pressure(r) - P; }, 1e-300, r1);
    *l = bisect([&](double r) { return cs.pressure(r) - P; }, r2, top * (1.0 - 1e-15));
  };
  const double lo = std::fmax(p_lo, 0.0) + 1e-14 * p_hi, hi = p_hi * (1.0 - 1e-13);
  double g, l;
  auto dmu = [&](double P) {
    roots(P, &g, &l);
    return cs.chem(l) - cs.chem(g);
  };
  if ((dmu(lo) > 0) == (dmu(hi) > 0)) return LBM_ENOCOEX;
  const double P = bisect(dmu, lo, hi);
  roots(P, &g, &l);
  // Newton polish on (rho_g, rho_l): equal pressure and chemical potential;
  // d mu / d rho = (d p / d rho) / rho.
  for (int it = 0; it < 4; ++it) {
    const double f1 = cs.pressure(l) - cs.pressure(g), f2 = cs.chem(l) - cs.chem(g);
    const double pg = cs.slope(g), pl = cs.slope(l);
    const double j11 = -pg, j12 = pl, j21 = -pg / g, j22 = pl / l;
    const double det = j11 * j22 - j12 * j21;
    if (!(std::fabs(det) > 0)) break;
    const double dg = (f1 * j22 - f2 * j12) / det, dl = (j11 * f2 - j21 * f1) / det;
    if (!(std::fabs(dg) < 0.1 * g && std::fabs(dl) < 0.1 * l)) break;
    g -= dg;
    l -= dl;
  }
  if (!(g > 0 && l > g && l < top)) return LBM_ENOCOEX;
  *rho_g = g;
  *rho_l = l;
  *p0 = 0.5 * (cs.pressure(g) + cs.pressure(l));
  return LBM_OK;
}

// Flat-interface constants at K_EOS = K_INT = 1 (kappa = a/2): the planar
// profile satisfies (kappa/2) rho'^2 = dOmega(rho) = psi_b - mu0 rho + p0, so
// sigma = int sqrt(2 kappa dOmega) d rho over [rho_g, rho_l] and the 5%-95%
// thickness is int sqrt(kappa/(2 dOmega)) d rho.  The thickness integrand
// grows like 1/(rho - rho_g) towards the ends; the logistic substitution
// rho = rho_g + (rho_l - rho_g)/(1 + exp(-z)) makes it smooth.
int interface_constants(double tr, double a, double b, double r_gas, double* c_sigma, double* c_w) {
  double g, l, p0;
  int st = maxwell(tr, a, b, r_gas, &g, &l, &p0);
  if (st) return st;
  const Cs cs{r_gas * tr * critical_temperature(a, b, r_gas), a, b};
  const double mu0 = 0.5 * (cs.chem(g) + cs.chem(l)), kappa = 0.5 * a, d = l - g;
  auto domega = [&](double r) { return cs.free_energy(r) - mu0 * r + p0; };
  *c_sigma = integrate([&](double r) { return std::sqrt(2.0 * kappa * std::fmax(domega(r), 0.0)); }, g, l,
                       64);
  const double z0 = std::log(0.05 / 0.95);
  *c_w = integrate(
      [&](double z) {
        const double s = 1.0 / (1.0 + std::exp(-z));
        const double r = g + d * s;
        return std::sqrt(kappa / (2.0 * domega(r))) * d * s * (1.0 - s);
      },
      z0, -z0, 32);
  return (std::isfinite(*c_sigma) && std::isfinite(*c_w)) ? LBM_OK : LBM_ENOCOEX;
}

int sigma_paper(double width, double tr, double a, double b, double r_gas, double* sigma) {
  double g, l, p0, cs_, cw;
  int st = maxwell(tr, a, b, r_gas, &g, &l, &p0);
  if (st) return st;
  st = interface_constants(tr, a, b, r_gas, &cs_, &cw);
  if (st) return st;
  const Cs cs{r_gas * tr * critical_temperature(a, b, r_gas), a, b};
  // c^2 = 3 K_INT^2 K_EOS RT (rho Z)'(rho_l) = 1  ->  sigma = C_sigma K_INT K_EOS
  const double k_int = width / cw;
  *sigma = cs_ / (3.0 * k_int * cs.repulsive_slope(l));
  return LBM_OK;
}

int validate(const lbm_params* p, char* msg, size_t len) {
  auto bad = [&](const char* what) {
    std::snprintf(msg, len, "invalid parameter: %s", what);
    return LBM_EINVAL;
  };
  if (!p) return bad("params is NULL");
  if (p->nx < 1 || p->ny < 1) return bad("nx and ny must be >= 1");
  if ((double)p->nx * (double)p->ny * 9.0 >= 2147483647.0) return bad("nx*ny*9 must be < 2^31");
  if (p->storage < LBM_FP32 || p->storage > LBM_BF16) return bad("storage must be LBM_FP32, LBM_FP16 or LBM_BF16");
  if (p->reserved != 0) return bad("reserved must be 0");
  if (!(p->s_p > 0.0 && p->s_p < 2.0)) return bad("s_p must lie in (0, 2)");
  if (!(p->s_eps <= 0.0 || p->s_eps < 2.0)) return bad("s_eps must lie in (0, 2) or be <= 0");
  if (!(p->varpi > 0.0 && p->varpi < 1.0)) return bad("varpi must lie in (0, 1)");
  if (std::fabs(p->varpi - 1.0 / 3.0) < 1e-6) return bad("varpi = 1/3 makes h and b singular");
  if (!(p->a > 0.0) || !(p->b > 0.0) || !(p->r_gas > 0.0)) return bad("a, b and r_gas must be > 0");
  if (!(p->tr > 0.0 && p->tr < 1.0)) return bad("tr must lie in (0, 1)");
  if (!(p->width > 0.0) || !std::isfinite(p->width)) return bad("width must be > 0");
  if (!std::isfinite(p->sigma)) return bad("sigma must be finite");
  return LBM_OK;
}

int derive(const lbm_params* p, lbm_derived* o, char* msg, size_t len) {
  int st = validate(p, msg, len);
  if (st) return st;
  lbm_derived d{};
  st = maxwell(p->tr, p->a, p->b, p->r_gas, &d.rho_g, &d.rho_l, &d.p0);
  if (!st) st = interface_constants(p->tr, p->a, p->b, p->r_gas, &d.c_sigma, &d.c_w);
  if (!st && p->sigma <= 0.0) st = sigma_paper(p->width, p->tr, p->a, p->b, p->r_gas, &d.sigma);
  if (st) {
    std::snprintf(msg, len, "no two-phase coexistence found at tr = %g", p->tr);
    return st;
  }
  if (p->sigma > 0.0) d.sigma = p->sigma;
  d.width = p->width;
  d.tc = critical_temperature(p->a, p->b, p->r_gas);
  d.rt = p->r_gas * p->tr * d.tc;
  d.k_int = p->width / d.c_w;
  d.k_eos = d.sigma / (d.c_sigma * d.k_int);
  d.g2 = 2.0 * d.k_int * d.k_int * d.k_eos * p->a;
  d.kp = d.k_eos;
  const double vp = p->varpi;
  d.alpha2 = -(2.0 * (-1.0) + vp + 1.0) / (1.0 - vp);
  d.beta2 = -2.0 / (1.0 - vp);
  d.k = 1.0 - vp;
  d.h = 6.0 * vp * (1.0 - vp) / (1.0 - 3.0 * vp);
  d.bs = (1.0 - vp) / (1.0 - 3.0 * vp);
  // tau_p tau_q = (k + 1) tau_e tau_q = 1/12, tau = 1/s - 1/2
  const double tau_p = 1.0 / p->s_p - 0.5, tau_q = 1.0 / (12.0 * tau_p), tau_e = tau_p / (d.k + 1.0);
  d.s_p = p->s_p;
  d.s_q = 1.0 / (tau_q + 0.5);
  d.s_e = 1.0 / (tau_e + 0.5);
  d.s_eps = p->s_eps > 0.0 ? p->s_eps : d.s_e;
  *o = d;
  return LBM_OK;
}

// d(G'^2, K', R T) / d(sigma, W, T_r), row-major 3 x 3.  With
// K_INT = W / C_W and K_EOS = sigma / (C_sigma K_INT) (main Eqs. 21, 23):
//   G'^2 = 2 a sigma W / (C_sigma C_W),  K' = sigma C_W / (C_sigma W),  R T = R T_r T_c,
// so only d C_sigma / d T_r and d C_W / d T_r are not closed forms; they are
// taken by the fourth-order central difference of interface_constants (a
// smooth function: fixed Gauss-Legendre panels and roots to the last bit).
// sigma is the value the context uses (prescribed or the default rule) and
// is held independent of W and T_r.
int param_jacobian(const lbm_params* p, double* jac, char* msg, size_t len) {
  lbm_derived d;
  int st = derive(p, &d, msg, len);
  if (st) return st;
  const double tr = p->tr, h = 1e-3 * std::fmin(tr, 1.0 - tr);
  double cs[4], cw[4];
  const double off[4] = {-2.0, -1.0, 1.0, 2.0};
  for (int k = 0; k < 4; ++k) {
    st = interface_constants(tr + off[k] * h, p->a, p->b, p->r_gas, &cs[k], &cw[k]);
    if (st) {
      std::snprintf(msg, len, "no two-phase coexistence near tr = %g", tr);
      return st;
    }
  }
  const double dcs = (cs[0] - 8.0 * cs[1] + 8.0 * cs[2] - cs[3]) / (12.0 * h);
  const double dcw = (cw[0] - 8.0 * cw[1] + 8.0 * cw[2] - cw[3]) / (12.0 * h);
  const double ls = dcs / d.c_sigma, lw = dcw / d.c_w;
  const double J[9] = {d.g2 / d.sigma, d.g2 / d.width, -d.g2 * (ls + lw),
                       d.kp / d.sigma, -d.kp / d.width, d.kp * (lw - ls),
                       0.0,            0.0,             p->r_gas * d.tc};
  for (int k = 0; k < 9; ++k) jac[k] = J[k];
  return LBM_OK;
}

}  // namespace lbm
