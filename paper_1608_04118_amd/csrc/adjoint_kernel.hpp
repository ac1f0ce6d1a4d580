// Discrete adjoint of the fused LTNE MRT step (reverse-time sweep).
//
// Structure used.  The state is (f, g_f, h) with h = g_s - g_f, the form
// the step kernel carries.  At a node z the post-collision populations are
//     s*(z) = L p(z) + g(q(z); phi, H)
// where p(z) are the 19 pulled populations and L is the constant relaxation
// of the non-conserved moments (Eqs. 10, 32, 33): M^-1 (I - Lambda) M on f,
// N^-1 (I - Q) N on g_f, and on h, in moments,
//     n_h,k -> (1 - eta_k) n_h,k + (zeta_k - eta_k) n_f,k   (k = 1..4).
// g collects everything that depends on the macroscopic state: equilibria
// (Eqs. 15, 37, 38), forcing (Eq. 12), sources (Eqs. 29-31) and the
// conserved moments.  g depends on p only through the five sums
// q = (rho - rho0, j_x, j_y, sum g_f, sum h) = P p: temperatures (Eqs. 43-46),
// velocity (Eqs. 20-22) and force (Eq. 5) are functions of q.  A wall node b
// rebuilt from its inward neighbour z has the same form,
// s*(b) = L p(z) + g_b(q(z); phi_z, H_z, phi_b, H_b), the reconstruction
// contributing L applied to the equilibrium difference.  Hence, with lambda
// the adjoint of s*,
//     d<lambda, s*>/dp = L^T lambda + P^T grad_q Phi,   Phi = <lambda, g>,
// and the parameter gradients are dPhi/dphi, dPhi/dH.  L^T is applied in
// moment space (M^-T = D M, D = diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12,
// 1/4, 1/4); N^-T = diag(1/5, 1/2, 1/2, 1/20, 1/4) N).  The gradient of the
// scalar Phi over (q, phi, H) is taken in reverse mode, written out by hand:
// Phi is first differentiated with respect to the node's macroscopic
// quantities (it is a polynomial in them), then that adjoint is carried
// back through the force, the velocity solve and the temperature solve.
//
// Streaming is a permutation whose adjoint is the push: the adjoint of the
// pulled population p_i(z) belongs to population i of node z - e_i.  Each
// sweep stores mu_i(z) = d<lambda, s*>/dp_i(z) at z itself (aligned stores)
// and the next sweep gathers lambda_i(y) = mu_i(y + e_i), which is zero where
// y + e_i is a wall node (wall nodes discard what streams in) or lies
// outside the lattice: the same shifted-load pattern as the forward pull.
#pragma once

#include "common.hpp"
#include "step_kernel.hpp"

namespace ltne {

// ---- macroscopic state of a node as a function of q ---------------------

// Forward values kept for the reverse pass.
template <typename C>
struct NodeMacros {
  C q[5], phi, H;
  C ip, iq, hv, d0, d1, iE, D, thf, Tf, srf, srs, dsr;
  C rho, ir, Gy, Fphi, vx, vy, l0, l1, vm, S, idn, ux, uy, um, dr, rFx, rFy;
};

// Temperatures (Eqs. 43-46), density (Eq. 18), buoyancy (Eq. 6), velocity
// (Eqs. 20-22) and force (Eq. 5) from q = (drho, jx, jy, sum g_f, sum h)
// at porosity phi and interphase coefficient H, as in the step kernel.
template <typename C>
__device__ __forceinline__ void node_macros(NodeMacros<C>& m, const StepConsts<C>& k) {
  m.ip = C(1) / m.phi;
  m.iq = C(1) / (C(1) - m.phi);
  m.hv = k.hvf * m.H;
  m.d0 = C(0.5) * m.hv * m.ip;
  m.d1 = C(0.5) * k.inv_sigma * m.hv * m.iq;
  m.iE = C(1) / (C(1) + m.d0 + m.d1);
  m.D = (m.q[4] + C(0.5) * (k.Qs - k.Qf)) * m.iE;
  m.thf = (m.q[3] + C(0.5) * k.Qf) + m.d0 * m.D;
  m.Tf = m.thf + k.T_ref;
  m.srf = C(2) * m.d0 * m.D + k.Qf;
  m.srs = C(-2) * m.d1 * m.D + k.Qs;
  m.dsr = C(-2) * (m.d0 + m.d1) * m.D + (k.Qs - k.Qf);
  m.rho = m.q[0] + k.rho0;
  m.ir = C(1) / m.rho;
  m.Gy = k.gbeta * (m.thf + k.dT0) + k.Gby;
  m.Fphi = (k.Fphi >= C(0)) ? k.Fphi : C(1.75) / sqrt(C(150) * m.phi * m.phi * m.phi);
  m.vx = m.q[1] * m.ir + C(0.5) * m.phi * k.Gbx;
  m.vy = m.q[2] * m.ir + C(0.5) * m.phi * m.Gy;
  m.l0 = C(0.25) * k.nu_over_K * m.phi + C(0.5);
  m.l1 = C(0.5) * k.inv_sqrtK * m.phi * m.Fphi;
  m.vm = sqrt(m.vx * m.vx + m.vy * m.vy);
  m.S = sqrt(m.l0 * m.l0 + m.l1 * m.vm);
  m.idn = C(1) / (m.l0 + m.S);
  m.ux = m.vx * m.idn;
  m.uy = m.vy * m.idn;
  m.um = sqrt(m.ux * m.ux + m.uy * m.uy);
  m.dr = -m.phi * (k.inv_sqrtK * m.Fphi * m.um + k.nu_over_K);
  m.rFx = m.rho * (m.dr * m.ux + m.phi * k.Gbx);
  m.rFy = m.rho * (m.dr * m.uy + m.phi * m.Gy);
}

// Adjoints of the node's macroscopic quantities, accumulated over the node's
// own collision and those of the walls rebuilt from it.  The coefficients
// e3, m7, m8, jx, jy, advx, advy multiply the shared expressions
//   e3 = 3 rho |u|^2 / phi, m7 = rho (u_x^2 - u_y^2) / phi, m8 = rho u_x u_y / phi,
//   jx = rho u_x, jy = rho u_y, advx = u_x T_f / phi, advy = u_y T_f / phi.
template <typename C>
struct MacroAdj {
  C q[5];
  C rho, ip, ux, uy, rFx, rFy, thf, D, srf, srs, dsr;
  C e3, m7, m8, jx, jy, advx, advy;
};

template <typename C>
__device__ __forceinline__ void clear(MacroAdj<C>& b) {
  for (int j = 0; j < 5; ++j) b.q[j] = C(0);
  b.rho = b.ip = b.ux = b.uy = b.rFx = b.rFy = b.thf = b.D = b.srf = b.srs = b.dsr = C(0);
  b.e3 = b.m7 = b.m8 = b.jx = b.jy = b.advx = b.advy = C(0);
}

// Moment-space adjoints of one node's outputs: f = M^-T lambda_f,
// a = N^-T lambda_gf, s = N^-T lambda_h.
template <typename C>
struct MomAdj {
  C f[9], a[5], s[5];
};

#ifndef LTNE_ADJ_DIV
#define LTNE_ADJ_DIV 1
#endif

// Normalisation of a conserved row.  These rows carry the adjoint of the
// conserved moments from step to step with no damping, so a rounded
// reciprocal (fl(1/9), fl(1/6), fl(0.2) all err upwards in binary32) would
// grow them by a fixed factor per step; a correctly rounded division has no
// such bias.
template <typename C>
__device__ __forceinline__ C cons_div(C v, int d) {
#if LTNE_ADJ_DIV
  return v / C(d);
#else
  return v * (C(1) / C(d));
#endif
}

template <typename C>
__device__ __forceinline__ void mom_adjoint(const C (&l)[19], MomAdj<C>& m) {
  const C* f = l;
  const C s14 = (f[1] + f[2]) + (f[3] + f[4]);
  const C s58 = (f[5] + f[6]) + (f[7] + f[8]);
  m.f[0] = cons_div(f[0] + s14 + s58, 9);
  m.f[1] = (C(-4) * f[0] - s14 + C(2) * s58) * (C(1) / C(36));
  m.f[2] = (C(4) * f[0] - C(2) * s14 + s58) * (C(1) / C(36));
  m.f[3] = cons_div((f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]), 6);
  m.f[4] = (C(2) * (f[3] - f[1]) + (f[5] - f[6]) + (f[8] - f[7])) * (C(1) / C(12));
  m.f[5] = cons_div((f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]), 6);
  m.f[6] = (C(2) * (f[4] - f[2]) + (f[5] + f[6]) - (f[7] + f[8])) * (C(1) / C(12));
  m.f[7] = ((f[1] - f[2]) + (f[3] - f[4])) * C(0.25);
  m.f[8] = ((f[5] - f[6]) + (f[7] - f[8])) * C(0.25);
  for (int ph = 0; ph < 2; ++ph) {
    const C* g = l + 9 + 5 * ph;
    C* o = ph == 0 ? m.a : m.s;
    o[0] = cons_div(((g[0] + g[1]) + (g[2] + g[3])) + g[4], 5);
    o[1] = (g[1] - g[3]) * C(0.5);
    o[2] = (g[2] - g[4]) * C(0.5);
    o[3] = (C(-4) * g[0] + ((g[1] + g[2]) + (g[3] + g[4]))) * C(0.05);
    o[4] = ((g[1] - g[2]) + (g[3] - g[4])) * C(0.25);
  }
}

// d Phi / d(macros) of an interior node's own collision, Phi = <L, g>:
//   f:   L0 drho + L1 (s_e meq1 + (1 - s_e/2) S1) + L2 (s_eps meq2 - (1 - s_eps/2) S1)
//        + L3 (jx + rFx) + L4 (-s_q rho ux - (1 - s_q/2) rFx) + (y likewise)
//        + L7 (s_nu meq7 + (1 - s_nu/2) S7) + L8 (s_nu meq8 + (1 - s_nu/2) S8),
//   g_f: a0 (sum g_f + Sr_f) + zeta_a (a1 ux + a2 uy) T_f / phi
//        + a3 (zeta_e c1 theta_f + (1 - zeta_e/2) c1 Sr_f),
//   h:   s0 (sum h + Sr_s - Sr_f) - zeta_a (s1 ux + s2 uy) T_f / phi
//        + s3 c1 (eta_e D - (zeta_e - eta_e) theta_f + (1 - eta_e/2) Sr_s - (1 - zeta_e/2) Sr_f),
// with meq1 = -2 drho + e3, meq2 = drho - e3, S1 = 6 u.rF / phi,
// S7 = 2 (ux rFx - uy rFy) / phi, S8 = (ux rFy + uy rFx) / phi, c1 = 5 varpi - 4.
template <typename C, typename A>
__device__ __forceinline__ void adj_interior(const NodeMacros<C>& m, const MomAdj<A>& La, MacroAdj<C>& b,
                                             const StepConsts<C>& k) {
  MomAdj<C> L;
  for (int i = 0; i < 9; ++i) L.f[i] = static_cast<C>(La.f[i]);
  for (int i = 0; i < 5; ++i) {
    L.a[i] = static_cast<C>(La.a[i]);
    L.s[i] = static_cast<C>(La.s[i]);
  }
  const C c1 = C(5) * k.varpi - C(4);
  const C ce = C(1) - C(0.5) * k.s_e, ceps = C(1) - C(0.5) * k.s_eps;
  const C cq = C(1) - C(0.5) * k.s_q, cnu = C(1) - C(0.5) * k.s_nu;
  const C cze = C(1) - C(0.5) * k.z_e, cee = C(1) - C(0.5) * k.e_e;
  b.q[0] += L.f[0] - C(2) * k.s_e * L.f[1] + k.s_eps * L.f[2];
  b.q[1] += L.f[3];
  b.q[2] += L.f[5];
  b.q[3] += L.a[0];
  b.q[4] += L.s[0];
  b.e3 += k.s_e * L.f[1] - k.s_eps * L.f[2];
  b.m7 += k.s_nu * L.f[7];
  b.m8 += k.s_nu * L.f[8];
  // forcing moments
  {
    const C cs1 = ce * L.f[1] - ceps * L.f[2];
    const C cs7 = cnu * L.f[7], cs8 = cnu * L.f[8];
    const C ax = C(6) * cs1 + C(2) * cs7;  // coefficient of ux rFx / phi
    const C ay = C(6) * cs1 - C(2) * cs7;  // coefficient of uy rFy / phi
    b.ux += (ax * m.rFx + cs8 * m.rFy) * m.ip;
    b.uy += (ay * m.rFy + cs8 * m.rFx) * m.ip;
    b.rFx += (ax * m.ux + cs8 * m.uy) * m.ip;
    b.rFy += (ay * m.uy + cs8 * m.ux) * m.ip;
    b.ip += ax * m.ux * m.rFx + ay * m.uy * m.rFy + cs8 * (m.ux * m.rFy + m.uy * m.rFx);
  }
  b.rFx += L.f[3] - cq * L.f[4];
  b.rFy += L.f[5] - cq * L.f[6];
  b.jx -= k.s_q * L.f[4];
  b.jy -= k.s_q * L.f[6];
  b.advx += k.z_a * (L.a[1] - L.s[1]);
  b.advy += k.z_a * (L.a[2] - L.s[2]);
  // correction term of Sec. 3.2: tc T_f (rho F) / (phi rho) on the fluid heat
  // flux, minus that on the difference lattice (tc = 0 when it is off)
  {
    const C cxa = k.tc * (L.a[1] - L.s[1]), cya = k.tc * (L.a[2] - L.s[2]);
    const C w = m.Tf * m.ip * m.ir;
    const C cf = cxa * m.rFx + cya * m.rFy;
    b.rFx += cxa * w;
    b.rFy += cya * w;
    b.thf += cf * m.ip * m.ir;
    b.ip += cf * m.Tf * m.ir;
    b.rho -= cf * w * m.ir;
  }
  b.srf += L.a[0] + c1 * cze * (L.a[3] - L.s[3]);
  b.srs += c1 * cee * L.s[3];
  b.dsr += L.s[0];
  b.thf += c1 * (k.z_e * L.a[3] - (k.z_e - k.e_e) * L.s[3]);
  b.D += c1 * k.e_e * L.s[3];
}

// d Phi_b / d(macros of z) for a wall node b rebuilt from z, and Phi_b's own
// derivatives in (phi_b, H_b).  The rebuilt populations are z's plus the
// equilibrium differences f^eq(rho, 0) - f^eq(rho, u) and
// g^eq(T_b, 0) - g^eq(T(z), u); the wall then collides with rho_b = rho(z),
// u_b = 0, T_fb, T_sb = T_fb + D_b and F_b = phi_b (G_b + G(T_fb)).
// dirichlet: T_fb = T_sb = theta_w (D_b = 0); otherwise T_fb = T_f(z),
// D_b = D(z).
template <typename C, typename A>
__device__ __forceinline__ void adj_wall(const NodeMacros<C>& m, const MomAdj<A>& La, C phb, C Hb,
                                         bool dirichlet, C theta_w, MacroAdj<C>& b, C& gpb, C& ghb,
                                         const StepConsts<C>& k) {
  MomAdj<C> L;
  for (int i = 0; i < 9; ++i) L.f[i] = static_cast<C>(La.f[i]);
  for (int i = 0; i < 5; ++i) {
    L.a[i] = static_cast<C>(La.a[i]);
    L.s[i] = static_cast<C>(La.s[i]);
  }
  const C c1 = C(5) * k.varpi - C(4);
  const C cq = C(1) - C(0.5) * k.s_q;
  const C cze = C(1) - C(0.5) * k.z_e, cee = C(1) - C(0.5) * k.e_e;
  // relaxed non-equilibrium parts taken over from z (for the flow: minus the
  // u-dependent equilibrium moments of z)
  b.e3 += -(C(1) - k.s_e) * L.f[1] + (C(1) - k.s_eps) * L.f[2];
  b.m7 -= (C(1) - k.s_nu) * L.f[7];
  b.m8 -= (C(1) - k.s_nu) * L.f[8];
  b.jx += (C(1) - k.s_q) * L.f[4];
  b.jy += (C(1) - k.s_q) * L.f[6];
  b.advx += (C(1) - k.z_a) * (L.s[1] - L.a[1]);
  b.advy += (C(1) - k.z_a) * (L.s[2] - L.a[2]);
  b.thf -= (k.z_e - k.e_e) * c1 * L.s[3];
  if (dirichlet) {
    b.thf -= (C(1) - k.z_e) * c1 * L.a[3];
    b.D -= (C(1) - k.e_e) * c1 * L.s[3];
  }
  // collision with the prescribed wall values
  b.q[0] += L.f[0] - C(2) * k.s_e * L.f[1] + k.s_eps * L.f[2];
  const C thfb = dirichlet ? theta_w : m.thf;
  const C Db = dirichlet ? C(0) : m.D;
  const C Gyb = k.gbeta * (thfb + k.dT0) + k.Gby;
  const C cx = C(0.5) * L.f[3] - cq * L.f[4];  // coefficient of rho F_x at b
  const C cy = C(0.5) * L.f[5] - cq * L.f[6];
  b.rho += phb * (cx * k.Gbx + cy * Gyb);
  gpb += m.rho * (cx * k.Gbx + cy * Gyb);
  const C ipb = C(1) / phb, iqb = C(1) / (C(1) - phb);
  const C hvb = k.hvf * Hb;
  const C d0b = C(0.5) * hvb * ipb, d1b = C(0.5) * k.inv_sigma * hvb * iqb;
  const C bsrf = C(0.5) * L.a[0] + c1 * cze * (L.a[3] - L.s[3]);
  const C bsrs = c1 * cee * L.s[3];
  const C bdsr = C(0.5) * L.s[0];
  const C bd0b = C(2) * Db * (bsrf - bdsr);
  const C bd1b = C(-2) * Db * (bsrs + bdsr);
  gpb += -bd0b * d0b * ipb + bd1b * d1b * iqb;
  ghb += C(0.5) * k.hvf * (bd0b * ipb + k.inv_sigma * bd1b * iqb);
  if (!dirichlet) {
    // the correction term at the wall is tc T_fb (G_bx, G_y(T_fb)): phi_b and
    // rho cancel
    const C ctx = k.tc * (L.a[1] - L.s[1]), cty = k.tc * (L.a[2] - L.s[2]);
    b.thf += ctx * k.Gbx + cty * (Gyb + (thfb + k.T_ref) * k.gbeta);
    b.thf += L.a[0] + c1 * k.z_e * L.a[3] + cy * m.rho * phb * k.gbeta;
    b.D += L.s[0] + c1 * k.e_e * L.s[3] + C(2) * d0b * bsrf - C(2) * d1b * bsrs -
           C(2) * (d0b + d1b) * bdsr;
  }
}

// Carries b back to q, phi and H: nu = dPhi/dq, gp = dPhi/dphi,
// gh = dPhi/dH.
template <typename C>
__device__ __forceinline__ void adj_backprop(const NodeMacros<C>& m, MacroAdj<C>& b, C (&nu)[5], C& gp, C& gh,
                                             const StepConsts<C>& k) {
  const C ux2 = m.ux * m.ux, uy2 = m.uy * m.uy;
  // shared expressions
  {
    const C usq = ux2 + uy2;
    b.rho += C(3) * b.e3 * usq * m.ip + b.m7 * (ux2 - uy2) * m.ip + b.m8 * m.ux * m.uy * m.ip +
             b.jx * m.ux + b.jy * m.uy;
    b.ip += C(3) * b.e3 * m.rho * usq + b.m7 * m.rho * (ux2 - uy2) + b.m8 * m.rho * m.ux * m.uy +
            (b.advx * m.ux + b.advy * m.uy) * m.Tf;
    const C r = m.rho * m.ip;
    b.ux += C(6) * b.e3 * r * m.ux + C(2) * b.m7 * r * m.ux + b.m8 * r * m.uy + b.jx * m.rho +
            b.advx * m.Tf * m.ip;
    b.uy += C(6) * b.e3 * r * m.uy - C(2) * b.m7 * r * m.uy + b.m8 * r * m.ux + b.jy * m.rho +
            b.advy * m.Tf * m.ip;
    b.thf += (b.advx * m.ux + b.advy * m.uy) * m.ip;
  }
  // force, Eq. 5: rF = rho (dr u + phi G)
  C gphi = m.rho * (b.rFx * k.Gbx + b.rFy * m.Gy);
  C bGy = b.rFy * m.rho * m.phi;
  b.rho += b.rFx * (m.dr * m.ux + m.phi * k.Gbx) + b.rFy * (m.dr * m.uy + m.phi * m.Gy);
  const C bdr = m.rho * (b.rFx * m.ux + b.rFy * m.uy);
  b.ux += b.rFx * m.rho * m.dr;
  b.uy += b.rFy * m.rho * m.dr;
  // dr = -phi (Fphi |u| / sqrt(K) + nu / K)
  gphi -= bdr * (k.inv_sqrtK * m.Fphi * m.um + k.nu_over_K);
  C bF = -bdr * m.phi * k.inv_sqrtK * m.um;
  const C bum = -bdr * m.phi * k.inv_sqrtK * m.Fphi;
  if (m.um > C(0)) {  // C^1 limit at rest: |u| enters multiplied by u
    b.ux += bum * m.ux / m.um;
    b.uy += bum * m.uy / m.um;
  }
  // velocity, Eq. 20: u = v / (l0 + sqrt(l0^2 + l1 |v|))
  C bvx = b.ux * m.idn, bvy = b.uy * m.idn;
  const C bden = -(b.ux * m.ux + b.uy * m.uy) * m.idn;
  const C hS = C(0.5) / m.S;
  const C bl0 = bden * (C(1) + C(2) * m.l0 * hS);
  const C bl1 = bden * m.vm * hS;
  const C bvm = bden * m.l1 * hS;
  if (m.vm > C(0)) {
    bvx += bvm * m.vx / m.vm;
    bvy += bvm * m.vy / m.vm;
  }
  gphi += bl1 * C(0.5) * k.inv_sqrtK * m.Fphi + bl0 * C(0.25) * k.nu_over_K;
  bF += bl1 * C(0.5) * k.inv_sqrtK * m.phi;
  // Eq. 21: v = j / rho + phi G / 2
  nu[1] = b.q[1] + bvx * m.ir;
  nu[2] = b.q[2] + bvy * m.ir;
  const C bir = bvx * m.q[1] + bvy * m.q[2];
  gphi += C(0.5) * (bvx * k.Gbx + bvy * m.Gy);
  bGy += C(0.5) * m.phi * bvy;
  if (k.Fphi < C(0)) gphi += bF * C(-1.5) * m.Fphi * m.ip;  // Ergun, Eq. 7
  b.thf += bGy * k.gbeta;
  b.rho -= bir * m.ir * m.ir;
  nu[0] = b.q[0] + b.rho;
  // temperatures, Eqs. 42-46
  C bd0 = C(2) * m.D * (b.srf - b.dsr) + b.thf * m.D;
  C bd1 = C(-2) * m.D * (b.srs + b.dsr);
  const C bD = b.D + C(2) * m.d0 * b.srf - C(2) * m.d1 * b.srs - C(2) * (m.d0 + m.d1) * b.dsr + b.thf * m.d0;
  nu[3] = b.q[3] + b.thf;
  nu[4] = b.q[4] + bD * m.iE;
  const C bE = -bD * m.D * m.iE;
  bd0 += bE;
  bd1 += bE;
  b.ip += C(0.5) * bd0 * m.hv;
  const C biq = C(0.5) * k.inv_sigma * bd1 * m.hv;
  gh = C(0.5) * k.hvf * (bd0 * m.ip + k.inv_sigma * bd1 * m.iq);
  gp = gphi - b.ip * m.ip * m.ip + biq * m.iq * m.iq;
}

// Thermal-phase wall temperature rule of the forward kernel.
template <typename C>
__device__ __forceinline__ bool wall_dirichlet(const StepConsts<C>& k, int x, int y, C& theta_w) {
  const bool wx = !k.px && (x == 0 || x == k.nx - 1);
  const bool wy = !k.py && (y == 0 || y == k.ny - 1);
  if (wx) {
    const int w = (x == 0) ? 0 : 1;
    if (k.wall_kind[w] == 0) { theta_w = k.theta_wall[w]; return true; }
  }
  if (wy) {
    const int w = (y == 0) ? 2 : 3;
    if (k.wall_kind[w] == 0) { theta_w = k.theta_wall[w]; return true; }
  }
  theta_w = C(0);
  return false;
}

// Index one step outside [0, n) brought back by the periodic wrap.
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// lambda_i at node (x, y): mu_i of the previous sweep at (x, y) + e_i, or 0
// when that node is a wall node or outside the lattice.
template <typename Lm, typename C>
__device__ __forceinline__ void gather_lambda(const Lm* __restrict__ mu, int x, int y, const StepConsts<C>& k,
                                              const long long P, Lm (&lam)[19]) {
  const int nx = k.nx, ny = k.ny;
#pragma unroll
  for (int i = 0; i < kPlanes; ++i) {
    const int q = i < 9 ? i : (i < 14 ? i - 9 : i - 14);
    int sx = x + vel_x(q), sy = y + vel_y(q);
    if (k.px) sx = wrap1(sx, nx);
    if (k.py) sy = wrap1(sy, ny);
    const bool inside = sx >= 0 && sx < nx && sy >= 0 && sy < ny;
    const bool wall = (!k.px && (sx == 0 || sx == nx - 1)) || (!k.py && (sy == 0 || sy == ny - 1));
    lam[i] = (inside && !wall) ? mu[i * P + (sy * nx + sx)] : Lm(0);
  }
}

// The parts of the moment adjoints that the relaxation transpose needs:
// (1 - s_k) L_k of the non-conserved D2Q9 moments (e, eps, q_x, q_y, p_xx,
// p_xy) and the non-conserved moments 1..4 of the two thermal lattices.
template <typename C>
struct RelaxAdj {
  C e, eps, qx, qy, pxx, pxy, a[4], s[4];
};

template <typename A, typename C>
__device__ __forceinline__ void relax_add(RelaxAdj<A>& r, const MomAdj<A>& L, const StepConsts<C>& k) {
  r.e += static_cast<A>(C(1) - k.s_e) * L.f[1];
  r.eps += static_cast<A>(C(1) - k.s_eps) * L.f[2];
  r.qx += static_cast<A>(C(1) - k.s_q) * L.f[4];
  r.qy += static_cast<A>(C(1) - k.s_q) * L.f[6];
  r.pxx += static_cast<A>(C(1) - k.s_nu) * L.f[7];
  r.pxy += static_cast<A>(C(1) - k.s_nu) * L.f[8];
  for (int i = 0; i < 4; ++i) {
    r.a[i] += L.a[i + 1];
    r.s[i] += L.s[i + 1];
  }
}

// Adjoint sweep modes.
constexpr int kAdjStep = 0;  // lambda_t -> lambda_{t-1}, gradients of step t
constexpr int kAdjSeed = 1;  // loss weights on T_f of the last step -> lambda_{N-1}
constexpr int kAdjInit = 2;  // lambda_0 -> gradients of the initialisation (no push)

// Node enumeration of one adjoint sweep.  Interior nodes next to a wall
// (x in {1, nx-2} on a walled x axis, y in {1, ny-2} on a walled y axis) also
// carry the adjoint of the wall nodes rebuilt from them (up to three: two
// sides and their corner).  They are listed separately (rows first, then the
// columns without the rows' nodes) and each gets four lanes of one wavefront:
// lane 0 takes the node's own collision, lanes 1-3 one wall each, in
// parallel, and the four partial adjoints are summed across the lanes.  The
// bulk region [bx0, bx0 + bw) x [by0, by0 + bh) takes one lane per node and no
// wall code, in workgroups of its own placed first in the grid.
struct AdjGrid {
  TileMap tm;          // tiles of the bulk region
  int bx0, by0, bw, bh;
  int bulk_blocks;     // workgroups of the bulk region (XCD-remapped)
  int nrow, rowlen, rx0;  // edge rows: y = 1 and (if nrow == 2) y = ny - 2
  int ncol, collen, cy0;  // edge columns: x = 1 and (if ncol == 2) x = nx - 2
  int nedge;
  int edge_blocks;     // workgroups of the edge list, four lanes per node
  long long lplane;    // elements between the planes of the adjoint populations (one plane each)
};

__device__ __forceinline__ void edge_node(int e, const AdjGrid& g, int nx, int ny, int& x, int& y) {
  const int nr = g.nrow * g.rowlen;
  if (e < nr) {
    const int r = e / g.rowlen;
    y = (r == 0) ? 1 : ny - 2;
    x = g.rx0 + (e - r * g.rowlen);
  } else {
    e -= nr;
    const int c = e / g.collen;
    x = (c == 0) ? 1 : nx - 2;
    y = g.cy0 + (e - c * g.collen);
  }
}

// Sum of v over the four lanes 4j..4j+3 of the wavefront (all lanes take part).
template <typename T>
__device__ __forceinline__ T quad_sum(T v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  return v;
}

template <typename C, typename Lm>
__device__ __forceinline__ void quad_sum(MacroAdj<C>& b, RelaxAdj<Lm>& r) {
  for (int j = 0; j < 5; ++j) b.q[j] = quad_sum(b.q[j]);
  b.rho = quad_sum(b.rho); b.ip = quad_sum(b.ip); b.ux = quad_sum(b.ux); b.uy = quad_sum(b.uy);
  b.rFx = quad_sum(b.rFx); b.rFy = quad_sum(b.rFy); b.thf = quad_sum(b.thf); b.D = quad_sum(b.D);
  b.srf = quad_sum(b.srf); b.srs = quad_sum(b.srs); b.dsr = quad_sum(b.dsr);
  b.e3 = quad_sum(b.e3); b.m7 = quad_sum(b.m7); b.m8 = quad_sum(b.m8); b.jx = quad_sum(b.jx);
  b.jy = quad_sum(b.jy); b.advx = quad_sum(b.advx); b.advy = quad_sum(b.advy);
  r.e = quad_sum(r.e); r.eps = quad_sum(r.eps); r.qx = quad_sum(r.qx); r.qy = quad_sum(r.qy);
  r.pxx = quad_sum(r.pxx); r.pxy = quad_sum(r.pxy);
  for (int i = 0; i < 4; ++i) {
    r.a[i] = quad_sum(r.a[i]);
    r.s[i] = quad_sum(r.s[i]);
  }
}

// Lm: storage type of the adjoint populations, C: arithmetic type, R: type
// of the lattice's fields and recorded sums.
static_assert(kRows == 1, "the adjoint kernel takes one node (or one part of one) per lane");

template <typename Lm, typename C, typename R, int Mode>
__global__ __launch_bounds__(kBlock) void adjoint_kernel(
    const Lm* __restrict__ lam_in, Lm* __restrict__ lam_out, const R* __restrict__ rec,
    const R* __restrict__ phi_field, const R* __restrict__ hv_field, double* __restrict__ gphi,
    double* __restrict__ ghv, const R* __restrict__ wseed, const R* __restrict__ init_tf,
    const R* __restrict__ init_ts, const StepConsts<C> k, const AdjGrid g) {
  const int b = blockIdx.x;
  const int nx = k.nx, ny = k.ny;
  const long long P = g.lplane;
  // ---- which node, and which part of it, this lane takes ----
  int x, y, slot = 0;
  bool valid;
  if (b < g.bulk_blocks) {
    const int t = (b & (kXcds - 1)) * g.tm.per_xcd + (b >> 3);
    if (t >= g.tm.ntiles) return;
    const int tw = 1 << g.tm.tw_shift;
    const int xl = (t % g.tm.ntx) * tw + (static_cast<int>(threadIdx.x) & (tw - 1));
    const int yl = (t / g.tm.ntx) * (kBlock >> g.tm.tw_shift) + (static_cast<int>(threadIdx.x) >> g.tm.tw_shift);
    if (xl >= g.bw || yl >= g.bh) return;
    x = g.bx0 + xl;
    y = g.by0 + yl;
    valid = true;
  } else {
    // four lanes per edge node; every lane of the wavefront stays to the
    // cross-lane sums
    const int e4 = (b - g.bulk_blocks) * kBlock + static_cast<int>(threadIdx.x);
    const int e = e4 >> 2;
    slot = e4 & 3;
    valid = e < g.nedge;
    x = 1;
    y = 1;
    if (valid) edge_node(e, g, nx, ny, x, y);
  }
  const bool edge = b >= g.bulk_blocks;
  const int iz = y * nx + x;
  // the wall this lane takes (slots 1-3), if any
  const int cx = (!k.px && x == 1) ? 0 : ((!k.px && x == nx - 2) ? nx - 1 : -1);
  const int cy = (!k.py && y == 1) ? 0 : ((!k.py && y == ny - 2) ? ny - 1 : -1);
  const bool has_wall = edge && Mode != kAdjSeed &&
                        ((slot == 1 && cx >= 0) || (slot == 2 && cy >= 0) || (slot == 3 && cx >= 0 && cy >= 0));
  const bool active = valid && (slot == 0 || has_wall);
  const int ax = (slot == 2) ? x : cx, ay = (slot == 1) ? y : cy;  // wall node of slots 1-3
  // own (slot 0) or wall adjoint populations first, so the loads overlap the
  // arithmetic
  Lm lam[19];
  if (Mode != kAdjSeed && active) gather_lambda(lam_in, slot == 0 ? x : ax, slot == 0 ? y : ay, k, P, lam);
  NodeMacros<C> m;
  C D0 = C(0);
  MacroAdj<C> bar;
  clear(bar);
  RelaxAdj<Lm> rx;
  rx.e = rx.eps = rx.qx = rx.qy = rx.pxx = rx.pxy = Lm(0);
  for (int i = 0; i < 4; ++i) rx.a[i] = rx.s[i] = Lm(0);
  if (valid) {
    m.phi = phi_field ? static_cast<C>(phi_field[iz]) : k.phi_u;
    m.H = hv_field ? static_cast<C>(hv_field[iz]) : k.hv_u;
    if (Mode == kAdjInit) {
      // initial pre-collision populations: f = 0 (shifted), g_f = w~ (T_f0 - Sr_f / 2),
      // h = w~ (D0 - (Sr_s - Sr_f) / 2)
      const C thf0 = init_tf ? static_cast<C>(init_tf[iz]) : k.theta_init_f;
      const C ths0 = init_ts ? static_cast<C>(init_ts[iz]) : k.theta_init_s;
      const C hv = m.H * k.hvf;
      const C d0 = C(0.5) * hv / m.phi;
      const C d1 = C(0.5) * hv * k.inv_sigma / (C(1) - m.phi);
      D0 = ths0 - thf0;
      m.q[0] = m.q[1] = m.q[2] = C(0);
      m.q[3] = thf0 - (d0 * D0 + C(0.5) * k.Qf);
      m.q[4] = D0 - C(0.5) * ((k.Qs - k.Qf) - C(2) * (d0 + d1) * D0);
    } else {
      for (int j = 0; j < 5; ++j) m.q[j] = static_cast<C>(rec[j * k.mplane + iz]);
    }
    node_macros(m, k);
    if (Mode == kAdjSeed) {
      // the loss weights the reported T_f of the last step
      if (slot == 0) bar.thf = static_cast<C>(wseed[iz]);
    } else if (active) {
      MomAdj<Lm> L;
      mom_adjoint(lam, L);
      if (slot == 0) {
        adj_interior(m, L, bar, k);
      } else {
        const int ib = ay * nx + ax;
        const C phb = phi_field ? static_cast<C>(phi_field[ib]) : k.phi_u;
        const C hvb = hv_field ? static_cast<C>(hv_field[ib]) : k.hv_u;
        C thw;
        const bool dir_w = wall_dirichlet(k, ax, ay, thw);
        C gpb = C(0), ghb = C(0);
        adj_wall(m, L, phb, hvb, dir_w, thw, bar, gpb, ghb, k);
        gphi[ib] += static_cast<double>(gpb);
        ghv[ib] += static_cast<double>(ghb);
      }
      relax_add(rx, L, k);
    }
  }
  if (edge) quad_sum(bar, rx);
  if (!valid || slot != 0) return;
  C nu[5], gpz, ghz;
  adj_backprop(m, bar, nu, gpz, ghz, k);
  // mu = L^T lambda_sum + P^T nu, in population space
  Lm mu[19];
  {
    // D2Q9: M^T (I - Lambda) lf, rest of the moments vanish (conserved)
    const Lm bb = rx.e, c = rx.eps, e = rx.qx, h = rx.qy, p7 = rx.pxx, p8 = rx.pxy;
    const Lm n0 = static_cast<Lm>(nu[0]), n1 = static_cast<Lm>(nu[1]), n2 = static_cast<Lm>(nu[2]);
    // row i of M^T (I-Lambda) lf = sum_k M[k][i] w_k
    mu[0] = Lm(-4) * bb + Lm(4) * c;
    mu[1] = -bb - Lm(2) * c - Lm(2) * e + p7;
    mu[2] = -bb - Lm(2) * c - Lm(2) * h - p7;
    mu[3] = -bb - Lm(2) * c + Lm(2) * e + p7;
    mu[4] = -bb - Lm(2) * c + Lm(2) * h - p7;
    mu[5] = Lm(2) * bb + c + e + h + p8;
    mu[6] = Lm(2) * bb + c - e + h - p8;
    mu[7] = Lm(2) * bb + c - e - h + p8;
    mu[8] = Lm(2) * bb + c + e - h - p8;
    for (int i = 0; i < 9; ++i) mu[i] += n0 + Lm(vel_x(i)) * n1 + Lm(vel_y(i)) * n2;
    // moments of (L^T lambda): g_f rows take (1 - zeta_k) a_k + (zeta_k - eta_k) s_k,
    // h rows (1 - eta_k) s_k
    const Lm* la = rx.a;  // moments 1..4
    const Lm* lh = rx.s;
    auto cv = [](C v) { return static_cast<Lm>(v); };
    for (int ph = 0; ph < 2; ++ph) {
      Lm w1, w2, w3, w4;
      if (ph == 0) {
        w1 = cv(C(1) - k.z_a) * la[0] + cv(k.z_a - k.e_a) * lh[0];
        w2 = cv(C(1) - k.z_a) * la[1] + cv(k.z_a - k.e_a) * lh[1];
        w3 = cv(C(1) - k.z_e) * la[2] + cv(k.z_e - k.e_e) * lh[2];
        w4 = cv(C(1) - k.z_nu) * la[3] + cv(k.z_nu - k.e_nu) * lh[3];
      } else {
        w1 = cv(C(1) - k.e_a) * lh[0];
        w2 = cv(C(1) - k.e_a) * lh[1];
        w3 = cv(C(1) - k.e_e) * lh[2];
        w4 = cv(C(1) - k.e_nu) * lh[3];
      }
      const Lm ns = cv(nu[3 + ph]);
      Lm* o = mu + 9 + 5 * ph;
      o[0] = Lm(-4) * w3 + ns;
      o[1] = w1 + w3 + w4 + ns;
      o[2] = w2 + w3 - w4 + ns;
      o[3] = -w1 + w3 + w4 + ns;
      o[4] = -w2 + w3 - w4 + ns;
    }
  }
  double gpd = static_cast<double>(gpz), ghd = static_cast<double>(ghz);
  if (Mode == kAdjInit) {
    // the initial populations depend on phi, H through Sr(T_init):
    // d g_f / dp = -w~ D0 d(d0)/dp, d h / dp = w~ D0 d(d0 + d1)/dp
    const C w0 = C(1) - k.varpi, w1 = C(0.25) * k.varpi;
    const C sa = w0 * C(mu[9]) + w1 * ((C(mu[10]) + C(mu[11])) + (C(mu[12]) + C(mu[13])));
    const C sh = w0 * C(mu[14]) + w1 * ((C(mu[15]) + C(mu[16])) + (C(mu[17]) + C(mu[18])));
    const C dd0_dphi = -m.d0 * m.ip, dd1_dphi = m.d1 * m.iq;
    const C dd0_dh = C(0.5) * k.hvf * m.ip, dd1_dh = C(0.5) * k.hvf * k.inv_sigma * m.iq;
    gpd += static_cast<double>((-sa * dd0_dphi + sh * (dd0_dphi + dd1_dphi)) * D0);
    ghd += static_cast<double>((-sa * dd0_dh + sh * (dd0_dh + dd1_dh)) * D0);
  } else {
    for (int i = 0; i < kPlanes; ++i) lam_out[i * P + iz] = mu[i];
  }
  gphi[iz] += gpd;
  ghv[iz] += ghd;
}

}  // namespace ltne
