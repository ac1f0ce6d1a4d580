/*
 * ltne_oracle.c -- plain FP64 CPU oracle for one time step of the REV-scale
 * MRT lattice Boltzmann model for porous-media convection under local thermal
 * non-equilibrium (Liu & He, arXiv:1608.04118).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU library never links, includes or calls it, and it shares no code with
 * the GPU library (no headers, helpers, tables or constants).
 *
 * Arithmetic: IEEE binary64, compiled with -ffp-contract=off so every run is
 * reproducible.  The moment transforms are the literal matrices of the paper
 * (M of Eq. 13, N of Eq. 36) applied as matrix-vector products; the inverses
 * are obtained by Gauss-Jordan elimination, i.e. straight from the definition
 * M^{-1} M = I.  Equilibrium moments are computed as M f^eq and N g^eq from the
 * velocity-space equilibria (Eqs. 24, 50, 51) following Eq. 12 and Eq. 27; the
 * tests check that this reproduces Eqs. 15, 37, 38.
 *
 * Readings of passages where the paper is silent or garbled (each one is also
 * listed with its justification in the design notes of the repository):
 *  - Forcing in moment space (Eq. 16 is garbled in the available text): the
 *    moment-space forcing is S~ = M S with the velocity-space porous forcing
 *    S_i = w_i rho [ e_i.F/cs^2 + (e_i.u)(e_i.F)/(phi cs^4) - u.F/(phi cs^2) ],
 *    the form whose zeroth, first and second moments are 0, rho F and
 *    rho (uF + Fu)/phi (the conditions the Chapman-Enskog analysis of
 *    Sec. 3.1 needs).
 *  - Order inside a node: T_f, T_s first (Eqs. 43-46 need no velocity), then
 *    the buoyancy G(T_f) (Eq. 6), the velocity (Eqs. 20-22) and F(u) (Eq. 5).
 *  - Gravity points along -y, so G = (0, g beta (T_f - T_0)); an optional
 *    constant body acceleration G_b is added to G.
 *  - Walls sit on the outermost nodes (L = n - 1).  Boundaries use the
 *    non-equilibrium extrapolation scheme cited in Sec. 4: after streaming,
 *    every population of a wall node x_b is rebuilt from the post-streaming
 *    populations of its inward neighbour x_f (diagonal neighbour at corners):
 *    f(x_b) = f^eq(rho_f, 0) + f(x_f) - f^eq(rho_f, u_f), and likewise for
 *    g_f, g_s with the wall temperature.  The wall node then collides with
 *    the prescribed macroscopic values rho_b = rho(x_f), u_b = 0, T_b, and
 *    F_b = phi_b G(T_fb).  Dirichlet walls give both phases the wall
 *    temperature; adiabatic walls take T_b = T(x_f); a corner takes the value
 *    of its vertical (x) wall when that wall is Dirichlet.
 *  - Initial state (paper silent): f = w_i rho0 (fluid at rest) and
 *    g = g^eq(T_init, 0) - w~_i Sr(T_init)/2, so that Eqs. 43-44 return
 *    T_init exactly.  These are the pre-collision populations of t = 0;
 *    creating a lattice performs the boundary treatment and collision of
 *    t = 0, so the stored state is always post-collision and the macros
 *    belong to the same time as the state.
 *  - Per-cell porosity and interphase coefficient (an extension: the paper
 *    treats a homogeneous medium) enter every coefficient at the node.
 *  - Interphase coefficient from the correlation of Eq. 52 (Sec. 4), when
 *    pore_size = D_p / L > 0: H_p = h_v D_p^2 / k_f = 0.376 Re^0.644 Pr^0.37
 *    with the local Reynolds number Re = u_m D_p / nu_f, i.e.
 *    H_v = h_v L^2 / k_f = H_p / pore_size^2 at every node.  The paper calls
 *    u_m the local average velocity; it is taken as |j| / rho with
 *    j = sum_i e_i f_i the momentum the node's populations carry after
 *    streaming (Eq. 18's companion first moment), because the velocity u of
 *    Eq. 20 depends on T_f through the buoyancy, and T_f (Eqs. 43-46) in turn
 *    on h_v: |j| / rho is the velocity of the same node and time that does
 *    not close that loop (it differs from |u| by the half-step force
 *    correction of Eq. 19, which is small where the buoyancy balances the
 *    drag).  Wall nodes have u_b = 0 and hence h_v = 0; so has the fluid at
 *    rest of the initial state.
 *  - Correction term of Sec. 3.2 (flag thermal_correction): the fluid D2Q5
 *    equation gains N^-1 (I - Q/2) C with C = N C~,
 *    C~_i = w~_i T_f (e_i . F) / (phi cs_T^2), F the force of Eq. 5 of the
 *    node (F_b at a wall node), added in moment space to the post-collision
 *    moments.
 *  - Nusselt number (not defined in the paper): Nu = (L/dT) <-dT/dn> along the
 *    chosen wall, dT/dn from the one-sided second-order difference
 *    (-3T_0 + 4T_1 - T_2)/2, averaged with the trapezoid rule along a walled
 *    tangent axis or the plain mean along a periodic one.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "ltne_oracle.h"

/* ---------------------------------------------------------------------------
 * Lattice constants.
 * ------------------------------------------------------------------------- */

/* D2Q9 velocities, Eq. 8 with c = 1: rest, four axis directions at angles
 * (i-1) pi/2, four diagonals at angles (2i-9) pi/4. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* D2Q9 weights, stated after Eq. 24. */
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Transformation matrix M, Eq. 13. */
static const double M9[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},      {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},  {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},   {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},   {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* Transformation matrix N, Eq. 36. */
static const double N5[5][5] = {{1, 1, 1, 1, 1},
                                {0, 1, 0, -1, 0},
                                {0, 0, 1, 0, -1},
                                {-4, 1, 1, 1, 1},
                                {0, 1, -1, 1, -1}};

static double M9inv[9][9];
static double N5inv[5][5];
static int inverses_ready = 0;

/* Gauss-Jordan inverse with partial pivoting of an n x n matrix (n <= 9). */
static void invert(int n, const double *a, double *ainv) {
  double w[9][18];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c)
      w[r][c] = (c < n) ? a[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(w[r][col]) > fabs(w[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) {
        double t = w[col][c];
        w[col][c] = w[piv][c];
        w[piv][c] = t;
      }
    double d = w[col][col];
    for (int c = 0; c < 2 * n; ++c) w[col][c] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double m = w[r][col];
      if (m != 0.0)
        for (int c = 0; c < 2 * n; ++c) w[r][c] -= m * w[col][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) ainv[r * n + c] = w[r][n + c];
}

static void ensure_inverses(void) {
  if (inverses_ready) return;
  invert(9, &M9[0][0], &M9inv[0][0]);
  invert(5, &N5[0][0], &N5inv[0][0]);
  inverses_ready = 1;
}

static void matvec9(const double a[9][9], const double *x, double *y) {
  for (int r = 0; r < 9; ++r) {
    double s = 0.0;
    for (int c = 0; c < 9; ++c) s += a[r][c] * x[c];
    y[r] = s;
  }
}

static void matvec5(const double a[5][5], const double *x, double *y) {
  for (int r = 0; r < 5; ++r) {
    double s = 0.0;
    for (int c = 0; c < 5; ++c) s += a[r][c] * x[c];
    y[r] = s;
  }
}

/* D2Q5 weights w~ stated after Eq. 31. */
static void wtilde(double varpi, double wt[5]) {
  wt[0] = 1.0 - varpi;
  for (int i = 1; i < 5; ++i) wt[i] = varpi / 4.0;
}

/* ---------------------------------------------------------------------------
 * Velocity-space building blocks.
 * ------------------------------------------------------------------------- */

/* Eq. 24, cs^2 = 1/3. */
void orc_feq(double rho, double ux, double uy, double phi, double feq[9]) {
  const double cs2 = 1.0 / 3.0;
  const double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    feq[i] = W9[i] * rho *
             (1.0 + eu / cs2 + eu * eu / (2.0 * phi * cs2 * cs2) - uu / (2.0 * phi * cs2));
  }
}

/* Eq. 50 (fluid phase). */
void orc_geq_fluid(double T, double ux, double uy, double phi, double varpi, double geq[5]) {
  geq[0] = (1.0 - varpi) * T;
  for (int i = 1; i < 5; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    geq[i] = 0.25 * varpi * T + 0.5 * eu * T / phi;
  }
}

/* Eq. 51 (solid phase). */
void orc_geq_solid(double T, double varpi, double geq[5]) {
  double wt[5];
  wtilde(varpi, wt);
  for (int i = 0; i < 5; ++i) geq[i] = wt[i] * T;
}

/* Velocity-space porous forcing S_i whose moments are 0, rho F and
 * rho (uF + Fu)/phi; the moment-space forcing is M S (Eq. 12). */
void orc_forcing(double rho, double ux, double uy, double Fx, double Fy, double phi,
                 double S[9]) {
  const double cs2 = 1.0 / 3.0;
  const double uF = ux * Fx + uy * Fy;
  for (int i = 0; i < 9; ++i) {
    double eF = EX[i] * Fx + EY[i] * Fy;
    double eu = EX[i] * ux + EY[i] * uy;
    S[i] = W9[i] * rho * (eF / cs2 + eu * eF / (phi * cs2 * cs2) - uF / (phi * cs2));
  }
}

void orc_matrices(double M[81], double Minv[81], double N[25], double Ninv[25]) {
  ensure_inverses();
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) {
      M[r * 9 + c] = M9[r][c];
      Minv[r * 9 + c] = M9inv[r][c];
    }
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) {
      N[r * 5 + c] = N5[r][c];
      Ninv[r * 5 + c] = N5inv[r][c];
    }
}

/* ---------------------------------------------------------------------------
 * Parameter mapping to lattice units (delta_x = delta_t = 1).
 *   Ra = g beta dT L^3 / (nu_f alpha_f), Pr = nu_f / alpha_f, Da = K / L^2,
 *   J_e = nu_e / nu_f, Gamma_sf = alpha_s / alpha_f = gamma_sf / sigma,
 *   H_v = h_v L^2 / k_f                                   (Sec. 2 groups)
 *   nu_e = cs^2 (1/s_nu - 1/2)                            (Eq. 23)
 *   alpha_f = csT^2 (1/zeta_a - 1/2), alpha_s likewise    (Eq. 49)
 * Scale: nu_f given directly, or a Mach number Ma = u_c / cs with the
 * buoyancy velocity u_c = sqrt(g beta dT L).
 * ------------------------------------------------------------------------- */

static int is_wall_x(const orc_params *p) { return !p->periodic_x; }
static int is_wall_y(const orc_params *p) { return !p->periodic_y; }

int orc_derive(const orc_params *p, orc_derived *d) {
  memset(d, 0, sizeof(*d));
  if (p->nx < 3 || p->ny < 3) return -1;
  d->cs2 = 1.0 / 3.0;
  d->csT2 = p->varpi / 2.0;
  double L = p->L;
  if (!(L > 0.0)) L = is_wall_x(p) ? (double)(p->nx - 1) : (double)(p->ny - 1);
  d->L = L;
  double dT = p->dT;
  if (!(dT > 0.0)) {
    double tmin = INFINITY, tmax = -INFINITY;
    for (int w = 0; w < 4; ++w) {
      int walled = (w < 2) ? is_wall_x(p) : is_wall_y(p);
      if (walled && p->wall_thermal[w] == 0) {
        if (p->T_wall[w] < tmin) tmin = p->T_wall[w];
        if (p->T_wall[w] > tmax) tmax = p->T_wall[w];
      }
    }
    dT = (tmax > tmin) ? (tmax - tmin) : 1.0;
  }
  d->dT = dT;
  if (p->nu_f > 0.0) {
    d->nu_f = p->nu_f;
    d->gbeta = p->Ra * p->nu_f * p->nu_f / (p->Pr * dT * L * L * L);
    d->u_c = sqrt(d->gbeta * dT * L);
  } else if (p->Ma > 0.0 && p->Ra > 0.0) {
    d->u_c = p->Ma * sqrt(d->cs2);
    d->gbeta = d->u_c * d->u_c / (dT * L);
    d->nu_f = d->u_c * L * sqrt(p->Pr / p->Ra);
  } else {
    return -1;
  }
  d->nu_e = p->Je * d->nu_f;
  d->s_nu = 1.0 / (d->nu_e / d->cs2 + 0.5);
  d->alpha_f = d->nu_f / p->Pr;
  d->alpha_s = (p->gamma_sf / p->sigma) * d->alpha_f;
  d->zeta_a = 1.0 / (d->alpha_f / d->csT2 + 0.5);
  d->eta_a = 1.0 / (d->alpha_s / d->csT2 + 0.5);
  d->K = p->Da * L * L;
  return 0;
}

/* ---------------------------------------------------------------------------
 * State.
 * ------------------------------------------------------------------------- */

struct orc {
  orc_params p;
  orc_derived d;
  int nx, ny;
  double *phi, *Hv;          /* per node */
  double *f, *gf, *gs;       /* post-collision populations, node-major */
  double *fp, *gfp, *gsp;    /* post-streaming populations, node-major */
  double *rho, *ux, *uy, *Tf, *Ts;       /* macros of the latest step */
  double *prho, *pux, *puy, *pTf, *pTs;  /* macros at the end of the previous step call */
  int64_t steps;
};

typedef struct {
  double rho, ux, uy, Tf, Ts, Fx, Fy, Srf, Srs;
} node_macros;

static double cell_Fphi(const orc *o, double phi) {
  if (o->p.F_phi >= 0.0) return o->p.F_phi;
  return 1.75 / sqrt(150.0 * phi * phi * phi); /* Ergun, Eq. 7 */
}

/* H_v = h_v L^2 / k_f of node c, whose local velocity is um: the given
 * value, or the correlation of Eq. 52 with Re = um D_p / nu_f when a pore
 * size is set (see the header). */
static double node_Hv(const orc *o, int c, double um) {
  if (!(o->p.pore_size > 0.0)) return o->Hv[c];
  const double Dp = o->p.pore_size * o->d.L;  /* D_p in lattice units */
  const double Re = um * Dp / o->d.nu_f;
  const double Hp = 0.376 * pow(Re, 0.644) * pow(o->p.Pr, 0.37); /* Eq. 52 */
  return Hp / (o->p.pore_size * o->p.pore_size);
}

/* d_0, d_1 of Eq. 46 with h_v/(rho c_p)_f = H_v alpha_f / L^2 (definition
 * of H_v, Sec. 2) and (rho c_p)_s = sigma (rho c_p)_f. */
static void cell_d(const orc *o, double phi, double Hv, double *d0, double *d1) {
  double hv_f = Hv * o->d.alpha_f / (o->d.L * o->d.L); /* h_v / (rho c_p)_f */
  *d0 = 0.5 * hv_f / phi;
  *d1 = 0.5 * hv_f / ((1.0 - phi) * o->p.sigma);
}

/* Buoyancy plus constant body acceleration: Eq. 6 with gravity along -y. */
static void buoyancy(const orc *o, double Tf, double *Gx, double *Gy) {
  *Gx = o->p.body_force[0];
  *Gy = o->p.body_force[1] + o->d.gbeta * (Tf - o->p.T0);
}

/* Macroscopic values of an interior node from its post-streaming populations
 * (Eqs. 18, 20-22, 43-46, 42, 6, 5). */
static void compute_macros(const orc *o, int c, const double *f, const double *gf,
                           const double *gs, node_macros *m) {
  const double phi = o->phi[c];
  /* Eq. 18 and the first moment */
  double rho = 0.0;
  for (int i = 0; i < 9; ++i) rho += f[i];
  double jx = 0.0, jy = 0.0;
  for (int i = 0; i < 9; ++i) {
    jx += EX[i] * f[i];
    jy += EY[i] * f[i];
  }
  double d0, d1;
  cell_d(o, phi, node_Hv(o, c, sqrt(jx * jx + jy * jy) / rho), &d0, &d1);
  /* Eqs. 43-46 */
  double sgf = 0.0, sgs = 0.0;
  for (int i = 0; i < 5; ++i) {
    sgf += gf[i];
    sgs += gs[i];
  }
  double A = sgf + 0.5 * o->p.Qf;
  double B = sgs + 0.5 * o->p.Qs;
  double Tf = ((1.0 + d1) * A + d0 * B) / (1.0 + d0 + d1);
  double Ts = (d1 * A + (1.0 + d0) * B) / (1.0 + d0 + d1);
  /* Eq. 42 */
  double Srf = 2.0 * d0 * (Ts - Tf) + o->p.Qf;
  double Srs = 2.0 * d1 * (Tf - Ts) + o->p.Qs;
  /* Eq. 6 */
  double Gx, Gy;
  buoyancy(o, Tf, &Gx, &Gy);
  /* Eq. 21 */
  double vx = jx / rho + 0.5 * phi * Gx;
  double vy = jy / rho + 0.5 * phi * Gy;
  /* Eq. 22 */
  const double K = o->d.K;
  const double Fphi = cell_Fphi(o, phi);
  double l0 = 0.5 * (1.0 + phi * 0.5 * o->d.nu_f / K);
  double l1 = phi * 0.5 * Fphi / sqrt(K);
  /* Eq. 20 */
  double vmag = sqrt(vx * vx + vy * vy);
  double den = l0 + sqrt(l0 * l0 + l1 * vmag);
  double ux = vx / den, uy = vy / den;
  /* Eq. 5 */
  double umag = sqrt(ux * ux + uy * uy);
  double Fx = -phi * o->d.nu_f / K * ux - phi * Fphi / sqrt(K) * umag * ux + phi * Gx;
  double Fy = -phi * o->d.nu_f / K * uy - phi * Fphi / sqrt(K) * umag * uy + phi * Gy;
  m->rho = rho;
  m->ux = ux;
  m->uy = uy;
  m->Tf = Tf;
  m->Ts = Ts;
  m->Fx = Fx;
  m->Fy = Fy;
  m->Srf = Srf;
  m->Srs = Srs;
}

/* Collision of one node: Eq. 10 with Eqs. 12, 15, 17 for the flow lattice,
 * Eqs. 32-33 with Eqs. 29-31, 37-40 for the two temperature lattices. */
static void collide(const orc *o, int c, const node_macros *m, const double *f,
                    const double *gf, const double *gs, double *fo, double *gfo,
                    double *gso) {
  const double phi = o->phi[c];
  const orc_params *p = &o->p;
  /* flow */
  double feq[9], S[9], mom[9], meq[9], St[9], ms[9];
  orc_feq(m->rho, m->ux, m->uy, phi, feq);
  orc_forcing(m->rho, m->ux, m->uy, m->Fx, m->Fy, phi, S);
  matvec9(M9, f, mom);
  matvec9(M9, feq, meq);
  matvec9(M9, S, St);
  const double lam[9] = {1.0, p->s_e, p->s_eps, 1.0, p->s_q, 1.0, p->s_q, o->d.s_nu, o->d.s_nu};
  for (int k = 0; k < 9; ++k)
    ms[k] = mom[k] - lam[k] * (mom[k] - meq[k]) + (1.0 - 0.5 * lam[k]) * St[k];
  matvec9((const double(*)[9])M9inv, ms, fo);
  /* temperatures */
  double wt[5], geq[5], n[5], neq[5], psi_v[5], psi[5], ns[5];
  wtilde(p->varpi, wt);
  const double qf[5] = {1.0, o->d.zeta_a, o->d.zeta_a, p->zeta_e, p->zeta_nu};
  const double qs[5] = {1.0, o->d.eta_a, o->d.eta_a, p->eta_e, p->eta_nu};
  /* fluid phase */
  orc_geq_fluid(m->Tf, m->ux, m->uy, phi, p->varpi, geq);
  matvec5(N5, gf, n);
  matvec5(N5, geq, neq);
  for (int i = 0; i < 5; ++i) psi_v[i] = wt[i] * m->Srf; /* Eq. 30 */
  matvec5(N5, psi_v, psi);                              /* Eq. 29 */
  for (int k = 0; k < 5; ++k)
    ns[k] = n[k] - qf[k] * (n[k] - neq[k]) + (1.0 - 0.5 * qf[k]) * psi[k];
  if (p->thermal_correction) {
    /* correction term of Sec. 3.2: (I - Q/2) N C~ added to the moments */
    double ct[5], cm[5];
    for (int i = 0; i < 5; ++i)
      ct[i] = wt[i] * m->Tf * (EX[i] * m->Fx + EY[i] * m->Fy) / (phi * o->d.csT2);
    matvec5(N5, ct, cm);
    for (int k = 0; k < 5; ++k) ns[k] += (1.0 - 0.5 * qf[k]) * cm[k];
  }
  matvec5((const double(*)[5])N5inv, ns, gfo);
  /* solid phase */
  orc_geq_solid(m->Ts, p->varpi, geq);
  matvec5(N5, gs, n);
  matvec5(N5, geq, neq);
  for (int i = 0; i < 5; ++i) psi_v[i] = wt[i] * m->Srs; /* Eq. 31 */
  matvec5(N5, psi_v, psi);
  for (int k = 0; k < 5; ++k)
    ns[k] = n[k] - qs[k] * (n[k] - neq[k]) + (1.0 - 0.5 * qs[k]) * psi[k];
  matvec5((const double(*)[5])N5inv, ns, gso);
}

static int wrap(int i, int n) { return (i < 0) ? i + n : (i >= n ? i - n : i); }

/* Wall classification of node (x, y). Returns 1 for a wall node and sets the
 * inward neighbour. */
static int wall_node(const orc *o, int x, int y, int *xf, int *yf) {
  int wx = is_wall_x(&o->p) && (x == 0 || x == o->nx - 1);
  int wy = is_wall_y(&o->p) && (y == 0 || y == o->ny - 1);
  *xf = x;
  *yf = y;
  if (wx) *xf = (x == 0) ? 1 : o->nx - 2;
  if (wy) *yf = (y == 0) ? 1 : o->ny - 2;
  return wx || wy;
}

/* Thermal condition of wall node (x, y): returns 1 and the wall temperature
 * for a Dirichlet condition, 0 for an adiabatic one. */
static int wall_temperature(const orc *o, int x, int y, double *Tb) {
  const orc_params *p = &o->p;
  if (is_wall_x(p) && (x == 0 || x == o->nx - 1)) {
    int w = (x == 0) ? 0 : 1;
    if (p->wall_thermal[w] == 0) {
      *Tb = p->T_wall[w];
      return 1;
    }
  }
  if (is_wall_y(p) && (y == 0 || y == o->ny - 1)) {
    int w = (y == 0) ? 2 : 3;
    if (p->wall_thermal[w] == 0) {
      *Tb = p->T_wall[w];
      return 1;
    }
  }
  return 0;
}

/* Initial state (paper silent; see header): the pre-collision populations
 * of time t = 0, written to the post-streaming arrays. */
static void initialize(orc *o, const double *Tf0, const double *Ts0) {
  const int n = o->nx * o->ny;
  double wt[5];
  wtilde(o->p.varpi, wt);
  for (int c = 0; c < n; ++c) {
    double Tf = Tf0 ? Tf0[c] : o->p.T_init_f;
    double Ts = Ts0 ? Ts0[c] : o->p.T_init_s;
    double d0, d1;
    cell_d(o, o->phi[c], node_Hv(o, c, 0.0), &d0, &d1); /* fluid at rest */
    double Srf = 2.0 * d0 * (Ts - Tf) + o->p.Qf;
    double Srs = 2.0 * d1 * (Tf - Ts) + o->p.Qs;
    double geq[5];
    for (int i = 0; i < 9; ++i) o->fp[c * 9 + i] = W9[i] * o->p.rho0;
    orc_geq_fluid(Tf, 0.0, 0.0, o->phi[c], o->p.varpi, geq);
    for (int i = 0; i < 5; ++i) o->gfp[c * 5 + i] = geq[i] - 0.5 * wt[i] * Srf;
    orc_geq_solid(Ts, o->p.varpi, geq);
    for (int i = 0; i < 5; ++i) o->gsp[c * 5 + i] = geq[i] - 0.5 * wt[i] * Srs;
  }
}

static void boundaries_macros_collide(orc *o);

orc *orc_create(const orc_params *p, const double *phi, const double *Hv, const double *Tf0,
                const double *Ts0) {
  ensure_inverses();
  orc *o = (orc *)calloc(1, sizeof(orc));
  if (!o) return NULL;
  o->p = *p;
  if (orc_derive(p, &o->d) != 0) {
    free(o);
    return NULL;
  }
  o->nx = p->nx;
  o->ny = p->ny;
  const size_t n = (size_t)o->nx * (size_t)o->ny;
  o->phi = (double *)malloc(n * sizeof(double));
  o->Hv = (double *)malloc(n * sizeof(double));
  o->f = (double *)malloc(9 * n * sizeof(double));
  o->gf = (double *)malloc(5 * n * sizeof(double));
  o->gs = (double *)malloc(5 * n * sizeof(double));
  o->fp = (double *)malloc(9 * n * sizeof(double));
  o->gfp = (double *)malloc(5 * n * sizeof(double));
  o->gsp = (double *)malloc(5 * n * sizeof(double));
  double **mac[10] = {&o->rho, &o->ux, &o->uy, &o->Tf, &o->Ts,
                      &o->prho, &o->pux, &o->puy, &o->pTf, &o->pTs};
  for (int k = 0; k < 10; ++k) *mac[k] = (double *)calloc(n, sizeof(double));
  for (size_t c = 0; c < n; ++c) {
    o->phi[c] = phi ? phi[c] : p->phi;
    o->Hv[c] = Hv ? Hv[c] : p->Hv;
  }
  initialize(o, Tf0, Ts0);
  boundaries_macros_collide(o); /* the collision of time t = 0 */
  memcpy(o->prho, o->rho, n * sizeof(double));
  memcpy(o->pux, o->ux, n * sizeof(double));
  memcpy(o->puy, o->uy, n * sizeof(double));
  memcpy(o->pTf, o->Tf, n * sizeof(double));
  memcpy(o->pTs, o->Ts, n * sizeof(double));
  return o;
}

void orc_free(orc *o) {
  if (!o) return;
  double *bufs[] = {o->phi, o->Hv,  o->f,   o->gf,  o->gs,  o->fp,  o->gfp, o->gsp,
                    o->rho, o->ux,  o->uy,  o->Tf,  o->Ts,  o->prho, o->pux, o->puy,
                    o->pTf, o->pTs};
  for (size_t k = 0; k < sizeof(bufs) / sizeof(bufs[0]); ++k) free(bufs[k]);
  free(o);
}

/* Streaming (Eqs. 11, 34, 35) in pull form, f_i(x, t+1) = f_i*(x - e_i, t),
 * for every non-wall node. */
static void stream_all(orc *o) {
  const int nx = o->nx, ny = o->ny;
  const int px = o->p.periodic_x, py = o->p.periodic_y;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int xf, yf;
      if (wall_node(o, x, y, &xf, &yf)) continue;
      const int c = y * nx + x;
      for (int i = 0; i < 9; ++i) {
        int sx = x - EX[i], sy = y - EY[i];
        if (px) sx = wrap(sx, nx);
        if (py) sy = wrap(sy, ny);
        o->fp[c * 9 + i] = o->f[(sy * nx + sx) * 9 + i];
      }
      for (int i = 0; i < 5; ++i) {
        int sx = x - EX[i], sy = y - EY[i];
        if (px) sx = wrap(sx, nx);
        if (py) sy = wrap(sy, ny);
        o->gfp[c * 5 + i] = o->gf[(sy * nx + sx) * 5 + i];
        o->gsp[c * 5 + i] = o->gs[(sy * nx + sx) * 5 + i];
      }
    }
}

/* Boundaries, macros and collision of every node, from the post-streaming
 * arrays into the state arrays.  Wall nodes read only the post-streaming
 * populations of interior nodes, which streaming completed. */
static void boundaries_macros_collide(orc *o) {
  const int nx = o->nx, ny = o->ny;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int c = y * nx + x;
      int xf, yf;
      node_macros m;
      double fb[9], gfb[5], gsb[5];
      const double *f, *gf, *gs;
      if (wall_node(o, x, y, &xf, &yf)) {
        const int cf = yf * nx + xf;
        node_macros mf;
        compute_macros(o, cf, &o->fp[cf * 9], &o->gfp[cf * 5], &o->gsp[cf * 5], &mf);
        double Tfb = mf.Tf, Tsb = mf.Ts, Tw;
        if (wall_temperature(o, x, y, &Tw)) Tfb = Tsb = Tw;
        const double phib = o->phi[c];
        const double phif = o->phi[cf];
        /* non-equilibrium extrapolation */
        double e0[9], e1[9], h0[5], h1[5];
        orc_feq(mf.rho, 0.0, 0.0, phib, e0);
        orc_feq(mf.rho, mf.ux, mf.uy, phif, e1);
        for (int i = 0; i < 9; ++i) fb[i] = e0[i] + (o->fp[cf * 9 + i] - e1[i]);
        orc_geq_fluid(Tfb, 0.0, 0.0, phib, o->p.varpi, h0);
        orc_geq_fluid(mf.Tf, mf.ux, mf.uy, phif, o->p.varpi, h1);
        for (int i = 0; i < 5; ++i) gfb[i] = h0[i] + (o->gfp[cf * 5 + i] - h1[i]);
        orc_geq_solid(Tsb, o->p.varpi, h0);
        orc_geq_solid(mf.Ts, o->p.varpi, h1);
        for (int i = 0; i < 5; ++i) gsb[i] = h0[i] + (o->gsp[cf * 5 + i] - h1[i]);
        /* prescribed macroscopic values of the wall node */
        double d0, d1, Gx, Gy;
        cell_d(o, phib, node_Hv(o, c, 0.0), &d0, &d1); /* u_b = 0 */
        buoyancy(o, Tfb, &Gx, &Gy);
        m.rho = mf.rho;
        m.ux = 0.0;
        m.uy = 0.0;
        m.Tf = Tfb;
        m.Ts = Tsb;
        m.Fx = phib * Gx;
        m.Fy = phib * Gy;
        m.Srf = 2.0 * d0 * (Tsb - Tfb) + o->p.Qf;
        m.Srs = 2.0 * d1 * (Tfb - Tsb) + o->p.Qs;
        f = fb;
        gf = gfb;
        gs = gsb;
      } else {
        f = &o->fp[c * 9];
        gf = &o->gfp[c * 5];
        gs = &o->gsp[c * 5];
        compute_macros(o, c, f, gf, gs, &m);
      }
      o->rho[c] = m.rho;
      o->ux[c] = m.ux;
      o->uy[c] = m.uy;
      o->Tf[c] = m.Tf;
      o->Ts[c] = m.Ts;
      /* The post-collision populations of the previous time are dead once
       * streaming has finished, so the new state overwrites them; the
       * post-streaming arrays stay intact for the wall nodes that read them. */
      collide(o, c, &m, f, gf, gs, &o->f[c * 9], &o->gf[c * 5], &o->gs[c * 5]);
    }
}

/* One time step t -> t+1. */
static void one_step(orc *o) {
  stream_all(o);
  boundaries_macros_collide(o);
  o->steps += 1;
}

/* ---------------------------------------------------------------------------
 * Public entry points.
 * ------------------------------------------------------------------------- */

void orc_step(orc *o, int64_t nsteps) {
  const size_t n = (size_t)o->nx * (size_t)o->ny;
  if (nsteps <= 0) return; /* a call that advances nothing keeps the residual's reference */
  memcpy(o->prho, o->rho, n * sizeof(double));
  memcpy(o->pux, o->ux, n * sizeof(double));
  memcpy(o->puy, o->uy, n * sizeof(double));
  memcpy(o->pTf, o->Tf, n * sizeof(double));
  memcpy(o->pTs, o->Ts, n * sizeof(double));
  for (int64_t s = 0; s < nsteps; ++s) one_step(o);
}

int64_t orc_steps_done(const orc *o) { return o->steps; }

void orc_macros(const orc *o, double *rho, double *ux, double *uy, double *Tf, double *Ts) {
  const size_t n = (size_t)o->nx * (size_t)o->ny;
  if (rho) memcpy(rho, o->rho, n * sizeof(double));
  if (ux) memcpy(ux, o->ux, n * sizeof(double));
  if (uy) memcpy(uy, o->uy, n * sizeof(double));
  if (Tf) memcpy(Tf, o->Tf, n * sizeof(double));
  if (Ts) memcpy(Ts, o->Ts, n * sizeof(double));
}

/* Post-collision populations (node-major: f[c*9+i], g[c*5+i]). */
void orc_get_populations(const orc *o, double *f, double *gf, double *gs) {
  const size_t n = (size_t)o->nx * (size_t)o->ny;
  if (f) memcpy(f, o->f, 9 * n * sizeof(double));
  if (gf) memcpy(gf, o->gf, 5 * n * sizeof(double));
  if (gs) memcpy(gs, o->gs, 5 * n * sizeof(double));
}

void orc_set_populations(orc *o, const double *f, const double *gf, const double *gs) {
  const size_t n = (size_t)o->nx * (size_t)o->ny;
  if (f) memcpy(o->f, f, 9 * n * sizeof(double));
  if (gf) memcpy(o->gf, gf, 5 * n * sizeof(double));
  if (gs) memcpy(o->gs, gs, 5 * n * sizeof(double));
}

/* Wall index: 0 left (x = 0), 1 right, 2 bottom (y = 0), 3 top. */
static int hot_wall(const orc *o) {
  const orc_params *p = &o->p;
  if (p->nu_wall >= 0) return p->nu_wall;
  int best = -1;
  for (int w = 0; w < 4; ++w) {
    int walled = (w < 2) ? is_wall_x(p) : is_wall_y(p);
    if (!walled || p->wall_thermal[w] != 0) continue;
    if (best < 0 || p->T_wall[w] > p->T_wall[best]) best = w;
  }
  return best;
}

/* Mean Nusselt number over wall w of a temperature field T (ny x nx). */
static double wall_nusselt(const orc_params *p, const orc_derived *d, const double *T, int w) {
  const int nx = p->nx, ny = p->ny;
  const int along_y = (w < 2); /* left/right walls run along y */
  const int len = along_y ? ny : nx;
  const int periodic_t = along_y ? p->periodic_y : p->periodic_x;
  double sum = 0.0, wsum = 0.0;
  for (int k = 0; k < len; ++k) {
    double t0, t1, t2;
    if (w == 0) { t0 = T[k * nx + 0]; t1 = T[k * nx + 1]; t2 = T[k * nx + 2]; }
    else if (w == 1) { t0 = T[k * nx + nx - 1]; t1 = T[k * nx + nx - 2]; t2 = T[k * nx + nx - 3]; }
    else if (w == 2) { t0 = T[0 * nx + k]; t1 = T[1 * nx + k]; t2 = T[2 * nx + k]; }
    else { t0 = T[(ny - 1) * nx + k]; t1 = T[(ny - 2) * nx + k]; t2 = T[(ny - 3) * nx + k]; }
    /* derivative along the inward normal, second-order one-sided */
    double dTdn = (-3.0 * t0 + 4.0 * t1 - t2) / 2.0;
    double weight = (!periodic_t && (k == 0 || k == len - 1)) ? 0.5 : 1.0;
    sum += weight * (-dTdn);
    wsum += weight;
  }
  return d->L / d->dT * (sum / wsum);
}

/* Nusselt number of an arbitrary temperature field over wall w (exposed for
 * the closed-form check of the definition). */
int orc_nusselt_field(const orc_params *p, const double *T, int w, double *Nu) {
  orc_derived d;
  if (orc_derive(p, &d) != 0 || w < 0 || w > 3) return -1;
  *Nu = wall_nusselt(p, &d, T, w);
  return 0;
}

int orc_nusselt(const orc *o, double *Nu_f, double *Nu_s) {
  int w = hot_wall(o);
  if (w < 0) return -1;
  if (Nu_f) *Nu_f = wall_nusselt(&o->p, &o->d, o->Tf, w);
  if (Nu_s) *Nu_s = wall_nusselt(&o->p, &o->d, o->Ts, w);
  return 0;
}

/* Total mass sum(rho); thermal energy sum(phi T_f + (1-phi) sigma T_s);
 * residual = max over u, T_f, T_s of sum|a - a_prev| / sum|a| between the
 * macros of this and of the previous step call. */
void orc_diagnostics(const orc *o, double *mass, double *energy, double *residual) {
  const size_t n = (size_t)o->nx * (size_t)o->ny;
  double m = 0.0, e = 0.0;
  double du = 0.0, nu = 0.0, dtf = 0.0, ntf = 0.0, dts = 0.0, nts = 0.0;
  for (size_t c = 0; c < n; ++c) {
    m += o->rho[c];
    e += o->phi[c] * o->Tf[c] + (1.0 - o->phi[c]) * o->p.sigma * o->Ts[c];
    du += fabs(o->ux[c] - o->pux[c]) + fabs(o->uy[c] - o->puy[c]);
    nu += fabs(o->ux[c]) + fabs(o->uy[c]);
    dtf += fabs(o->Tf[c] - o->pTf[c]);
    ntf += fabs(o->Tf[c]);
    dts += fabs(o->Ts[c] - o->pTs[c]);
    nts += fabs(o->Ts[c]);
  }
  double r = 0.0, q;
  q = nu > 0.0 ? du / nu : du;
  if (q > r) r = q;
  q = ntf > 0.0 ? dtf / ntf : dtf;
  if (q > r) r = q;
  q = nts > 0.0 ? dts / nts : dts;
  if (q > r) r = q;
  if (mass) *mass = m;
  if (energy) *energy = e;
  if (residual) *residual = r;
}

/* Node-level pieces exposed for identity checks. */

/* Eqs. 20-22 and Eq. 5 for given sums: returns u and F. */
void orc_velocity(double rho, double jx, double jy, double Gx, double Gy, double phi, double nu_f,
                  double K, double Fphi, double *ux, double *uy, double *Fx, double *Fy) {
  double vx = jx / rho + 0.5 * phi * Gx;
  double vy = jy / rho + 0.5 * phi * Gy;
  double l0 = 0.5 * (1.0 + phi * 0.5 * nu_f / K);
  double l1 = phi * 0.5 * Fphi / sqrt(K);
  double vmag = sqrt(vx * vx + vy * vy);
  double den = l0 + sqrt(l0 * l0 + l1 * vmag);
  *ux = vx / den;
  *uy = vy / den;
  double umag = sqrt((*ux) * (*ux) + (*uy) * (*uy));
  *Fx = -phi * nu_f / K * (*ux) - phi * Fphi / sqrt(K) * umag * (*ux) + phi * Gx;
  *Fy = -phi * nu_f / K * (*uy) - phi * Fphi / sqrt(K) * umag * (*uy) + phi * Gy;
}

/* Eqs. 43-46: temperatures from the population sums. */
void orc_temperatures(double sum_gf, double sum_gs, double Qf, double Qs, double d0, double d1,
                      double *Tf, double *Ts) {
  double A = sum_gf + 0.5 * Qf, B = sum_gs + 0.5 * Qs;
  *Tf = ((1.0 + d1) * A + d0 * B) / (1.0 + d0 + d1);
  *Ts = (d1 * A + (1.0 + d0) * B) / (1.0 + d0 + d1);
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

size_t orc_params_size(void) { return sizeof(orc_params); }
