// Parameter defaults, validation and the mapping of the problem statement
// (the dimensionless groups of Sec. 2) to lattice units.  Host code only.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "lbm_ltne.h"
#include "params.hpp"

namespace ltne {

namespace {
thread_local std::string g_last_error;
}

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

const char* last_error() { return g_last_error.c_str(); }

void clear_error() { g_last_error.clear(); }

static bool walled(const lbm_ltne_params* p, int w) { return w < 2 ? !p->periodic_x : !p->periodic_y; }

static bool finite_all(const lbm_ltne_params* p) {
  const double v[] = {p->T_wall[0], p->T_wall[1], p->T_wall[2], p->T_wall[3], p->T0, p->T_init_f,
                      p->T_init_s, p->L, p->dT, p->phi, p->Da, p->F_phi, p->Ra, p->Pr, p->Je,
                      p->gamma_sf, p->sigma, p->Hv, p->Qf, p->Qs, p->Ma, p->nu_f,
                      p->body_force[0], p->body_force[1], p->varpi, p->s_e, p->s_eps, p->s_q,
                      p->zeta_e, p->zeta_nu, p->eta_e, p->eta_nu, p->rho0, p->fp16_scale_f,
                      p->fp16_scale_g, p->pore_size};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

static bool rate_ok(double s) { return s > 0.0 && s < 2.0; }

static bool pow2_or_zero(double s) {
  if (s == 0.0) return true;
  if (!(s > 0.0)) return false;
  int e;
  return std::frexp(s, &e) == 0.5;
}

int hot_wall(const lbm_ltne_params* p) {
  if (p->nu_wall >= 0) return p->nu_wall;
  int best = -1;
  for (int w = 0; w < 4; ++w) {
    if (!walled(p, w) || p->wall_thermal[w] != LBM_WALL_DIRICHLET) continue;
    if (best < 0 || p->T_wall[w] > p->T_wall[best]) best = w;
  }
  return best;
}

void temperature_range(const lbm_ltne_params* p, double* tmin, double* tmax) {
  double lo = std::fmin(p->T_init_f, p->T_init_s), hi = std::fmax(p->T_init_f, p->T_init_s);
  for (int w = 0; w < 4; ++w)
    if (walled(p, w) && p->wall_thermal[w] == LBM_WALL_DIRICHLET) {
      lo = std::fmin(lo, p->T_wall[w]);
      hi = std::fmax(hi, p->T_wall[w]);
    }
  *tmin = lo;
  *tmax = hi;
}

static double pow2_floor(double v) {
  int e;
  std::frexp(v, &e);  // v = m 2^e, m in [0.5, 1)
  return std::ldexp(1.0, e - 1);
}

int derive(const lbm_ltne_params* p, double tmin, double tmax, lbm_ltne_derived* d) {
  std::memset(d, 0, sizeof(*d));
  if (!p) return set_error(LBM_EINVAL, "params is NULL");
  if (!finite_all(p)) return set_error(LBM_EINVAL, "a parameter is not finite");
  if (p->precision < LBM_FP64 || p->precision > LBM_FP32SR)
    return set_error(LBM_EINVAL, "precision %d is not LBM_FP64, LBM_FP32, LBM_FP16S or LBM_FP32SR", p->precision);
  if ((p->periodic_x != 0 && p->periodic_x != 1) || (p->periodic_y != 0 && p->periodic_y != 1))
    return set_error(LBM_EINVAL, "periodic_x / periodic_y must be 0 or 1");
  const int minx = p->periodic_x ? 3 : 4, miny = p->periodic_y ? 3 : 4;
  if (p->nx < minx || p->ny < miny)
    return set_error(LBM_EINVAL, "lattice %d x %d too small (walled axis needs >= 4 nodes, periodic >= 3)",
                     p->nx, p->ny);
  if (static_cast<long long>(p->nx) * p->ny > (1LL << 30))
    return set_error(LBM_EINVAL, "lattice %d x %d exceeds 2^30 nodes", p->nx, p->ny);
  for (int w = 0; w < 4; ++w)
    if (walled(p, w) && p->wall_thermal[w] != LBM_WALL_DIRICHLET &&
        p->wall_thermal[w] != LBM_WALL_ADIABATIC)
      return set_error(LBM_EINVAL, "wall_thermal[%d] = %d is not a wall condition", w, p->wall_thermal[w]);
  if (p->nu_wall < -1 || p->nu_wall > 3 || (p->nu_wall >= 0 && !walled(p, p->nu_wall)))
    return set_error(LBM_EINVAL, "nu_wall = %d does not name a wall of this lattice", p->nu_wall);
  if (!(p->phi > 0.0 && p->phi < 1.0)) return set_error(LBM_EINVAL, "phi = %g not in (0, 1)", p->phi);
  if (!(p->Da > 0.0)) return set_error(LBM_EINVAL, "Da = %g must be > 0", p->Da);
  if (!(p->Pr > 0.0)) return set_error(LBM_EINVAL, "Pr = %g must be > 0", p->Pr);
  if (!(p->Je > 0.0)) return set_error(LBM_EINVAL, "Je = %g must be > 0", p->Je);
  if (!(p->sigma > 0.0)) return set_error(LBM_EINVAL, "sigma = %g must be > 0", p->sigma);
  if (!(p->gamma_sf > 0.0)) return set_error(LBM_EINVAL, "gamma_sf = %g must be > 0", p->gamma_sf);
  if (!(p->Hv >= 0.0)) return set_error(LBM_EINVAL, "Hv = %g must be >= 0", p->Hv);
  if (!(p->Ra >= 0.0)) return set_error(LBM_EINVAL, "Ra = %g must be >= 0", p->Ra);
  if (!(p->varpi > 0.0 && p->varpi < 1.0)) return set_error(LBM_EINVAL, "varpi = %g not in (0, 1)", p->varpi);
  if (!(p->rho0 > 0.0)) return set_error(LBM_EINVAL, "rho0 = %g must be > 0", p->rho0);
  const double rates[] = {p->s_e, p->s_eps, p->s_q, p->zeta_e, p->zeta_nu, p->eta_e, p->eta_nu};
  const char* names[] = {"s_e", "s_eps", "s_q", "zeta_e", "zeta_nu", "eta_e", "eta_nu"};
  for (int i = 0; i < 7; ++i)
    if (!rate_ok(rates[i])) return set_error(LBM_EINVAL, "%s = %g not in (0, 2)", names[i], rates[i]);
  if (!pow2_or_zero(p->fp16_scale_f) || !pow2_or_zero(p->fp16_scale_g))
    return set_error(LBM_EINVAL, "fp16 storage scales must be 0 or a power of two");
  if (p->thermal_correction != 0 && p->thermal_correction != 1)
    return set_error(LBM_EINVAL, "thermal_correction must be 0 or 1");
  if (!(p->pore_size >= 0.0)) return set_error(LBM_EINVAL, "pore_size = %g must be >= 0", p->pore_size);
  if (p->diag_every < 0) return set_error(LBM_EINVAL, "diag_every = %d must be >= 0", p->diag_every);

  d->cs2 = 1.0 / 3.0;
  d->csT2 = 0.5 * p->varpi;
  d->L = p->L > 0.0 ? p->L : (p->periodic_x ? p->ny - 1.0 : p->nx - 1.0);
  double dT = p->dT;
  if (!(dT > 0.0)) {
    double lo = INFINITY, hi = -INFINITY;
    for (int w = 0; w < 4; ++w)
      if (walled(p, w) && p->wall_thermal[w] == LBM_WALL_DIRICHLET) {
        lo = std::fmin(lo, p->T_wall[w]);
        hi = std::fmax(hi, p->T_wall[w]);
      }
    dT = hi > lo ? hi - lo : 1.0;
  }
  d->dT = dT;
  const double L = d->L;
  if (p->nu_f > 0.0) {
    d->nu_f = p->nu_f;
    d->gbeta = p->Ra * p->nu_f * p->nu_f / (p->Pr * dT * L * L * L);
    d->u_c = std::sqrt(d->gbeta * dT * L);
  } else if (p->Ma > 0.0 && p->Ra > 0.0) {
    d->u_c = p->Ma * std::sqrt(d->cs2);
    d->gbeta = d->u_c * d->u_c / (dT * L);
    d->nu_f = d->u_c * L * std::sqrt(p->Pr / p->Ra);
  } else {
    return set_error(LBM_EINVAL, "no lattice scale: give nu_f > 0, or Ma > 0 with Ra > 0");
  }
  d->nu_e = p->Je * d->nu_f;
  d->tau_nu = d->nu_e / d->cs2 + 0.5;  // Eq. 23
  d->s_nu = 1.0 / d->tau_nu;
  d->alpha_f = d->nu_f / p->Pr;
  d->alpha_s = p->gamma_sf / p->sigma * d->alpha_f;
  d->tau_Tf = d->alpha_f / d->csT2 + 0.5;  // Eq. 49
  d->tau_Ts = d->alpha_s / d->csT2 + 0.5;
  d->zeta_a = 1.0 / d->tau_Tf;
  d->eta_a = 1.0 / d->tau_Ts;
  if (!(d->tau_nu > 0.5) || !(d->tau_Tf > 0.5) || !(d->tau_Ts > 0.5))
    return set_error(LBM_EINVAL, "a derived relaxation time is <= 1/2 (tau_nu %g, tau_Tf %g, tau_Ts %g)",
                     d->tau_nu, d->tau_Tf, d->tau_Ts);
  d->K = p->Da * L * L;
  const double phi = p->phi;
  d->F_phi = p->F_phi >= 0.0 ? p->F_phi : 1.75 / std::sqrt(150.0 * phi * phi * phi);  // Eq. 7
  d->l0 = 0.5 * (1.0 + 0.5 * phi * d->nu_f / d->K);                                   // Eq. 22
  d->l1 = 0.5 * phi * d->F_phi / std::sqrt(d->K);
  const double hv = p->Hv * d->alpha_f / (L * L);  // h_v / (rho c_p)_f, from H_v = h_v L^2 / k_f
  d->d0 = 0.5 * hv / phi;                          // Eq. 46
  d->d1 = 0.5 * hv / ((1.0 - phi) * p->sigma);

  // Shift reference and binary16 storage scales.
  d->T_ref = std::isnan(p->T_ref) ? 0.5 * (tmin + tmax) : p->T_ref;
  if (!std::isfinite(d->T_ref)) return set_error(LBM_EINVAL, "T_ref is not finite");
  d->scale_f = d->scale_g = 1.0;
  if (p->precision == LBM_FP16S) {
    // Magnitude estimates of the shifted populations: w_i rho 3 e.u for the
    // flow, w~ (T - T_ref) + (e.u) T / (2 phi) for the temperatures, with the
    // buoyancy velocity or the Darcy velocity of the body force as the
    // velocity scale; the scale maps them near 2^11 (binary16 max 65504).
    const double gb = std::hypot(p->body_force[0], p->body_force[1]);
    const double umax = std::fmax(std::fmax(d->u_c, gb * d->K / d->nu_f), 1e-4);
    const double est_f = std::fmax(umax / 3.0, 1e-5);
    const double spread = std::fmax(std::fabs(tmax - d->T_ref), std::fabs(tmin - d->T_ref));
    const double est_g =
        std::fmax(spread + (std::fabs(d->T_ref) + spread) * umax / phi, 1e-5);
    d->scale_f = p->fp16_scale_f > 0.0 ? p->fp16_scale_f : pow2_floor(2048.0 / est_f);
    d->scale_g = p->fp16_scale_g > 0.0 ? p->fp16_scale_g : pow2_floor(2048.0 / est_g);
  }
  return LBM_OK;
}

}  // namespace ltne

extern "C" {

int lbm_ltne_default_params(lbm_ltne_params* p) {
  if (!p) return ltne::set_error(LBM_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->nx = p->ny = 64;
  p->precision = LBM_FP64;
  p->periodic_x = p->periodic_y = 0;
  p->wall_thermal[0] = p->wall_thermal[1] = LBM_WALL_DIRICHLET;
  p->wall_thermal[2] = p->wall_thermal[3] = LBM_WALL_ADIABATIC;
  p->nu_wall = -1;
  p->T_wall[0] = 11.0;  // T_h
  p->T_wall[1] = 1.0;   // T_c
  p->T0 = 1.0;          // T_0 = T_c
  p->T_init_f = p->T_init_s = 1.0;
  p->L = 0.0;
  p->dT = 0.0;
  p->phi = 0.8;
  p->Da = 1e-4;
  p->F_phi = 0.068;
  p->Ra = 1e6;
  p->Pr = 1.0;
  p->Je = 1.0;
  p->gamma_sf = 1000.0;
  p->sigma = 1.0;
  p->Hv = 0.0;
  p->Qf = p->Qs = 0.0;
  p->Ma = 0.1;
  p->nu_f = 0.0;
  p->varpi = 0.4;
  p->s_e = 1.1;
  p->s_eps = 1.1;
  p->s_q = 1.2;
  p->zeta_e = p->zeta_nu = 1.1;
  p->eta_e = p->eta_nu = 1.1;
  p->rho0 = 1.0;
  p->T_ref = NAN;
  p->fp16_scale_f = p->fp16_scale_g = 0.0;
  p->pore_size = 0.0;
  p->diag_every = 0;
  return LBM_OK;
}

int lbm_ltne_derive(const lbm_ltne_params* p, lbm_ltne_derived* d) {
  lbm_ltne_derived tmp;
  if (!p) return ltne::set_error(LBM_EINVAL, "params is NULL");
  double lo = 0.0, hi = 0.0;
  ltne::temperature_range(p, &lo, &hi);
  return ltne::derive(p, lo, hi, d ? d : &tmp);
}

const char* lbm_ltne_strerror(int code) {
  switch (code) {
    case LBM_OK: return "success";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of device memory";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_EDIVERGED: return "simulation diverged (non-finite mass or energy)";
    case LBM_EUNSUPPORTED: return "unsupported request";
    case LBM_ENODEV: return "no gfx950 device";
    default: return "unknown error code";
  }
}

const char* lbm_ltne_last_error(void) { return ltne::last_error(); }

int lbm_ltne_abi_version(void) { return LBM_LTNE_ABI_VERSION; }

}  // extern "C"
