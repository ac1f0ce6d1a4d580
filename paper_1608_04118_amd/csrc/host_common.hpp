// Host-side helpers shared by the single-lattice and the batched runtime.
// Not part of the public ABI.
#pragma once

#include <cmath>
#include <cstring>

#include "common.hpp"
#include "lbm_ltne.h"
#include "params.hpp"
#include "reduce_kernels.hpp"

namespace ltne {

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return set_error(LBM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kSumBlocks = 1024;
constexpr uint32_t kStateMagic = 0x524e544cu;  // "LTNR": f, g_f and h = g_s - g_f, row-interleaved

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline size_t storage_bytes(int precision) {
  return precision == LBM_FP64 ? 8 : ((precision == LBM_FP32 || precision == LBM_FP32SR) ? 4 : 2);
}
inline size_t compute_bytes(int precision) { return (precision == LBM_FP64 || precision == LBM_FP32SR) ? 8 : 4; }

// Population layout: lattice row y holds the 19 population rows of that
// row one after another, population q of node (x, y) at y rs + q qs + x.
// qs is nx rounded up to 64 elements (every population row starts on a
// 128-byte or wider boundary) and rs = 19 qs.  A workgroup then reads and
// writes a few dozen kilobytes of contiguous memory per lattice row instead
// of 38 streams far apart, which HBM serves faster (measured on the 8192^2
// layer: 6.2 TB/s for the bare 19-population pull copy against 5.6 TB/s
// with one plane per population).
inline long long pop_row_elems(int nx) { return static_cast<long long>(align_up(static_cast<size_t>(nx), 64)); }
inline long long pop_elems(int nx, int ny) { return kPlanes * pop_row_elems(nx) * ny; }
// The two-step kernel addresses a lattice row (its kPlanes population rows)
// through one buffer resource with 32-bit byte offsets: the row must span
// less than 2^31 bytes of populations (elem_bytes each).
inline bool step2_addressable(int nx, size_t elem_bytes) {
  return kPlanes * pop_row_elems(nx) * static_cast<long long>(elem_bytes) < (1LL << 31);
}

struct Layout {
  size_t pop_bytes, field_bytes, mac_bytes;
  size_t off_pop[2], off_phi, off_hv, off_mac[2], off_partial, off_result;
  size_t total;
};

inline Layout make_layout(const lbm_ltne_params* p, bool has_phi, bool has_hv) {
  Layout L{};
  const long long n = static_cast<long long>(p->nx) * p->ny;
  L.pop_bytes = align_up(pop_elems(p->nx, p->ny) * storage_bytes(p->precision), kAlign);
  L.field_bytes = align_up(n * compute_bytes(p->precision), kAlign);
  L.mac_bytes = align_up(5 * n * compute_bytes(p->precision), kAlign);
  size_t o = 0;
  L.off_pop[0] = o; o += L.pop_bytes;
  L.off_pop[1] = o; o += L.pop_bytes;
  L.off_phi = o; o += has_phi ? L.field_bytes : 0;
  L.off_hv = o; o += has_hv ? L.field_bytes : 0;
  L.off_mac[0] = o; o += L.mac_bytes;
  L.off_mac[1] = o; o += L.mac_bytes;
  L.off_partial = o; o += align_up(kSumBlocks * kSums * sizeof(double), kAlign);
  L.off_result = o; o += kAlign;
  L.total = o;
  return L;
}

// Tiles of 2^shift x (256 / 2^shift) kRows nodes.  Default widths: 256 for
// the step kernel in every form (measured on the 8192^2 layer), never wider
// than the lattice needs; pref_shift names another preferred width (the
// adjoint's), shift_override > 0 forces a width.
inline TileMap make_tiles(int nx, int ny, int precision, int shift_override = 0, int pref_shift = 8) {
  TileMap t{};
  (void)precision;
  const int pref = pref_shift;
  t.tw_shift = nx >= 256 ? 8 : (nx >= 128 ? 7 : 6);
  if (t.tw_shift > pref) t.tw_shift = pref;
  if (t.tw_shift > kTwShiftMax) t.tw_shift = kTwShiftMax;
  if (shift_override >= 6 && shift_override <= 8) t.tw_shift = shift_override;
  const int tw = 1 << t.tw_shift, th = (kBlock / tw) * kRows;
  t.ntx = (nx + tw - 1) / tw;
  const int nty = (ny + th - 1) / th;
  t.ntiles = t.ntx * nty;
  t.per_xcd = (t.ntiles + kXcds - 1) / kXcds;
  return t;
}

inline int grid_blocks(const TileMap& t) { return kXcdRemap ? kXcds * t.per_xcd : t.ntiles; }

template <typename T>
inline void fill_thermal_k(const lbm_ltne_params& p, const lbm_ltne_derived& d, ThermalK<T>* t) {
  const double c1 = 5.0 * p.varpi - 4.0;
  t->Qf = static_cast<T>(p.Qf);
  t->Qs = static_cast<T>(p.Qs);
  t->hQf = static_cast<T>(0.5 * p.Qf);
  t->hdQ = static_cast<T>(0.5 * (p.Qs - p.Qf));
  t->T_ref = static_cast<T>(d.T_ref);
  t->w0 = static_cast<T>(1.0 - p.varpi);
  t->w1 = static_cast<T>(0.25 * p.varpi);
  for (int w = 0; w < 4; ++w) t->theta_wall[w] = static_cast<T>(p.T_wall[w] - d.T_ref);
  t->theta_init_f = static_cast<T>(p.T_init_f - d.T_ref);
  t->theta_init_s = static_cast<T>(p.T_init_s - d.T_ref);
  t->c1 = static_cast<T>(c1);
  t->z_a = static_cast<T>(d.zeta_a);
  t->z_e = static_cast<T>(p.zeta_e);
  t->z_nu = static_cast<T>(p.zeta_nu);
  t->e_a = static_cast<T>(d.eta_a);
  t->e_e = static_cast<T>(p.eta_e);
  t->e_nu = static_cast<T>(p.eta_nu);
  t->k3 = static_cast<T>((1.0 - 0.5 * p.zeta_e) * c1);
  t->k4 = static_cast<T>((1.0 - 0.5 * p.eta_e) * c1);
  t->tc = static_cast<T>(p.thermal_correction ? 1.0 - 0.5 * d.zeta_a : 0.0);
  t->sg = static_cast<T>(d.scale_g);
}

template <typename C>
inline void fill_step_consts(const lbm_ltne_params& p, const lbm_ltne_derived& d, StepConsts<C>* k) {
  k->nx = p.nx;
  k->ny = p.ny;
  k->px = p.periodic_x;
  k->py = p.periodic_y;
  k->qs = pop_row_elems(p.nx);
  k->rs = kPlanes * k->qs;
  k->mplane = static_cast<long long>(p.nx) * p.ny;
  k->tm = make_tiles(p.nx, p.ny, p.precision);
  k->rho0 = static_cast<C>(p.rho0);
  k->phi_u = static_cast<C>(p.phi);
  k->hv_u = static_cast<C>(p.Hv);
  k->gbeta = static_cast<C>(d.gbeta);
  k->dT0 = static_cast<C>(d.T_ref - p.T0);
  k->Gbx = static_cast<C>(p.body_force[0]);
  k->Gby = static_cast<C>(p.body_force[1]);
  k->nu_over_K = static_cast<C>(d.nu_f / d.K);
  k->inv_sqrtK = static_cast<C>(1.0 / std::sqrt(d.K));
  k->Fphi = static_cast<C>(p.F_phi >= 0.0 ? p.F_phi : -1.0);
  k->hvf = static_cast<C>(d.alpha_f / (d.L * d.L));
  k->inv_sigma = static_cast<C>(1.0 / p.sigma);
  k->Qf = static_cast<C>(p.Qf);
  k->Qs = static_cast<C>(p.Qs);
  k->s_e = static_cast<C>(p.s_e);
  k->s_eps = static_cast<C>(p.s_eps);
  k->s_q = static_cast<C>(p.s_q);
  k->s_nu = static_cast<C>(d.s_nu);
  k->z_a = static_cast<C>(d.zeta_a);
  k->z_e = static_cast<C>(p.zeta_e);
  k->z_nu = static_cast<C>(p.zeta_nu);
  k->e_a = static_cast<C>(d.eta_a);
  k->e_e = static_cast<C>(p.eta_e);
  k->e_nu = static_cast<C>(p.eta_nu);
  k->varpi = static_cast<C>(p.varpi);
  k->T_ref = static_cast<C>(d.T_ref);
  for (int w = 0; w < 4; ++w) {
    k->wall_kind[w] = p.wall_thermal[w];
    k->theta_wall[w] = static_cast<C>(p.T_wall[w] - d.T_ref);
  }
  k->sf = static_cast<C>(d.scale_f);
  k->inv_sf = static_cast<C>(1.0 / d.scale_f);
  k->sg = static_cast<C>(d.scale_g);
  k->inv_sg = static_cast<C>(1.0 / d.scale_g);
  k->theta_init_f = static_cast<C>(p.T_init_f - d.T_ref);
  k->theta_init_s = static_cast<C>(p.T_init_s - d.T_ref);
  // Eq. 52: H_p = h_v D_p^2 / k_f = 0.376 Re^0.644 Pr^0.37, Re = u_m D_p / nu_f,
  // D_p = pore_size L, so h_v / (rho c_p)_f = H_p alpha_f / D_p^2
  k->hv_corr = p.pore_size > 0.0 ? 1 : 0;
  const double Dp = p.pore_size * d.L;
  k->corr_a = static_cast<C>(k->hv_corr ? 0.376 * std::pow(p.Pr, 0.37) * d.alpha_f / (Dp * Dp) : 0.0);
  k->corr_b = static_cast<C>(k->hv_corr ? Dp / d.nu_f : 0.0);
  k->tc = static_cast<C>(p.thermal_correction ? 1.0 - 0.5 * d.zeta_a : 0.0);
  fill_thermal_k(p, d, &k->td);
  fill_thermal_k(p, d, &k->tf);
}

inline int check_device(int* dev) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
    return set_error(LBM_ENODEV, "no HIP device is visible");
  HIP_TRY(hipGetDevice(dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, *dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(LBM_ENODEV, "device %d is %s; this library is built for gfx950", *dev,
                     prop.gcnArchName);
  return LBM_OK;
}

}  // namespace ltne
