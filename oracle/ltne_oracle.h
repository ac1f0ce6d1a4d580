/*
 * ltne_oracle.h -- interface of the FP64 CPU oracle (test infrastructure
 * only; see ltne_oracle.c).  Node index c = y * nx + x.  Populations are
 * node-major: f[c*9 + i], g[c*5 + i], with the velocity order of Eq. 8.
 */
#ifndef LTNE_ORACLE_H
#define LTNE_ORACLE_H

#include <stddef.h>
#include <stdint.h>

typedef struct {
  int32_t nx, ny;
  int32_t periodic_x, periodic_y;
  int32_t wall_thermal[4]; /* left, right, bottom, top: 0 Dirichlet, 1 adiabatic */
  int32_t nu_wall;         /* wall for the Nusselt number, -1: hottest Dirichlet wall */
  int32_t thermal_correction; /* 1: add the correction term of Sec. 3.2 to the fluid D2Q5 equation */
  double T_wall[4];
  double T0;               /* Boussinesq reference temperature (Eq. 6) */
  double T_init_f, T_init_s;
  double L, dT;            /* <= 0: derived */
  double phi, Da, F_phi;   /* F_phi < 0: Ergun (Eq. 7) at the local porosity */
  double Ra, Pr, Je;
  double gamma_sf, sigma, Hv;
  double Qf, Qs;           /* q'''/(rho c_p) of each phase (Eq. 45) */
  double Ma, nu_f;         /* nu_f > 0 wins; otherwise Ma */
  double body_force[2];
  double varpi, s_e, s_eps, s_q, zeta_e, zeta_nu, eta_e, eta_nu;
  double rho0;
  double pore_size;        /* D_p / L; > 0: h_v of every node from the correlation of Eq. 52 */
} orc_params;

typedef struct {
  double L, dT, cs2, csT2, gbeta, u_c, nu_f, nu_e, s_nu, alpha_f, alpha_s, zeta_a, eta_a, K;
} orc_derived;

typedef struct orc orc;

int orc_derive(const orc_params *p, orc_derived *d);
orc *orc_create(const orc_params *p, const double *phi, const double *Hv, const double *Tf0,
                const double *Ts0);
void orc_free(orc *o);
void orc_step(orc *o, int64_t nsteps);
int64_t orc_steps_done(const orc *o);
void orc_macros(const orc *o, double *rho, double *ux, double *uy, double *Tf, double *Ts);
void orc_get_populations(const orc *o, double *f, double *gf, double *gs);
void orc_set_populations(orc *o, const double *f, const double *gf, const double *gs);
int orc_nusselt(const orc *o, double *Nu_f, double *Nu_s);
int orc_nusselt_field(const orc_params *p, const double *T, int w, double *Nu);
void orc_diagnostics(const orc *o, double *mass, double *energy, double *residual);

void orc_feq(double rho, double ux, double uy, double phi, double feq[9]);
void orc_geq_fluid(double T, double ux, double uy, double phi, double varpi, double geq[5]);
void orc_geq_solid(double T, double varpi, double geq[5]);
void orc_forcing(double rho, double ux, double uy, double Fx, double Fy, double phi, double S[9]);
void orc_matrices(double M[81], double Minv[81], double N[25], double Ninv[25]);
void orc_velocity(double rho, double jx, double jy, double Gx, double Gy, double phi, double nu_f,
                  double K, double Fphi, double *ux, double *uy, double *Fx, double *Fy);
void orc_temperatures(double sum_gf, double sum_gs, double Qf, double Qs, double d0, double d1,
                      double *Tf, double *Ts);
int orc_threads(void);
size_t orc_params_size(void);

#endif
