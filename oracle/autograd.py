"""Differentiable FP64 transcription of the oracle's time step (PyTorch, CPU).

TEST INFRASTRUCTURE ONLY.  Only the test suite may import this module.  It
restates, with whole-lattice tensor operations instead of per-node loops, the
algorithm of ``ltne_oracle.c`` (same readings of the paper, same order of
steps), so that reverse-mode automatic differentiation gives the exact
gradient of the discrete map, in binary64, with no hand-derived adjoint.  It
shares no code with the GPU library.  The constants it needs come from the
oracle itself: the derived lattice values (``oracle.derive``) and the literal
matrices M (Eq. 13) and N (Eq. 36) with their inverses (``oracle.matrices``).

The step, as in the oracle:
  1. pull streaming (Eqs. 11, 34, 35), periodic wrap on periodic axes;
  2. macroscopic values of every node from its pulled populations: rho
     (Eq. 18), T_f, T_s (Eqs. 43-46), Sr_f, Sr_s (Eq. 42), buoyancy (Eq. 6,
     gravity along -y), velocity (Eqs. 20-22), force (Eq. 5);
  3. wall nodes rebuilt by non-equilibrium extrapolation from the inward
     neighbour (diagonal at a corner) and given the prescribed values
     rho_b = rho(x_f), u_b = 0, T_b, F_b = phi_b G(T_fb);
  4. collisions in moment space: D2Q9 with the forcing M S (Eqs. 10, 12, 15,
     17), D2Q5 for both phases with the sources (Eqs. 29-33, 37-40), and the
     correction term of Sec. 3.2 in the fluid phase when it is switched on.
The initial state is f = w rho0, g = g^eq(T_init, 0) - w~ Sr(T_init)/2 taken as
the pre-collision populations of t = 0, followed by the walls and collision
of t = 0.  The loss is the mean Nusselt number of T_f over the chosen wall:
(L/dT) times the mean of -(-3 T_0 + 4 T_1 - T_2)/2, trapezoid weights along a
walled tangent axis.

Square roots of squared norms use the C^1 limit at zero (derivative 0 there):
|v| and |u| only enter multiplied by the vector itself, so that is the
derivative of the composite map at rest.
"""
from __future__ import annotations

import numpy as np
import torch

from . import derive, matrices

EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
W9 = (4.0 / 9.0,) + (1.0 / 9.0,) * 4 + (1.0 / 36.0,) * 4
DT = torch.float64


def _sqrt0(a):
    pos = a > 0
    s = torch.sqrt(torch.where(pos, a, torch.ones_like(a)))
    return torch.where(pos, s, torch.zeros_like(a))


def hot_wall(p: dict) -> int:
    """The wall whose Nusselt number is the loss (same rule as the oracle)."""
    if int(p.get("nu_wall", -1)) >= 0:
        return int(p["nu_wall"])
    best = -1
    for w in range(4):
        walled = not (p["periodic_x"] if w < 2 else p["periodic_y"])
        if not walled or int(p["wall_thermal"][w]) != 0:
            continue
        if best < 0 or p["T_wall"][w] > p["T_wall"][best]:
            best = w
    return best


class DiffLattice:
    """One lattice in binary64 torch tensors; phi and Hv may require grad."""

    def __init__(self, p: dict, phi, Hv, Tf0=None, Ts0=None):
        if float(p.get("pore_size", 0.0)) > 0.0:
            raise NotImplementedError("the transcription covers the model without the h_v correlation")
        self.p = dict(p)
        self.d = derive(p)
        self.nx, self.ny = int(p["nx"]), int(p["ny"])
        sh = (self.ny, self.nx)
        t = lambda a, v: (torch.full(sh, float(v), dtype=DT) if a is None
                          else torch.as_tensor(np.asarray(a, dtype=np.float64)).to(DT).expand(sh))
        self.phi = phi if isinstance(phi, torch.Tensor) else t(phi, p["phi"])
        self.Hv = Hv if isinstance(Hv, torch.Tensor) else t(Hv, p["Hv"])
        M, Mi, N, Ni = matrices()
        self.M, self.Mi = torch.as_tensor(M), torch.as_tensor(Mi)
        self.N, self.Ni = torch.as_tensor(N), torch.as_tensor(Ni)
        v = float(p["varpi"])
        self.wt = torch.tensor([1.0 - v] + [0.25 * v] * 4, dtype=DT)
        self.w9 = torch.tensor(W9, dtype=DT)
        self.ex = torch.tensor(EX, dtype=DT).view(9, 1, 1)
        self.ey = torch.tensor(EY, dtype=DT).view(9, 1, 1)
        self._walls()
        # t = 0: initial pre-collision populations, then walls and collision
        Tf = t(Tf0, p["T_init_f"])
        Ts = t(Ts0, p["T_init_s"])
        d0, d1 = self._d01(self.phi, self.Hv)
        Srf = 2.0 * d0 * (Ts - Tf) + p["Qf"]
        Srs = 2.0 * d1 * (Tf - Ts) + p["Qs"]
        zero = torch.zeros(sh, dtype=DT)
        f = self.w9.view(9, 1, 1) * float(p["rho0"]) * torch.ones((9,) + sh, dtype=DT)
        gf = self._geq_fluid(Tf, zero, zero, self.phi) - 0.5 * self.wt.view(5, 1, 1) * Srf
        gs = self._geq_solid(Ts) - 0.5 * self.wt.view(5, 1, 1) * Srs
        self.state = self._walls_macros_collide(f, gf, gs)
        self.steps = 0

    # ---- geometry of the walls ----
    def _walls(self):
        nx, ny, p = self.nx, self.ny, self.p
        y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        wx = (not p["periodic_x"]) & ((x == 0) | (x == nx - 1))
        wy = (not p["periodic_y"]) & ((y == 0) | (y == ny - 1))
        wall = wx | wy
        xf = np.where(wx, np.where(x == 0, 1, nx - 2), x)
        yf = np.where(wy, np.where(y == 0, 1, ny - 2), y)
        dirichlet = np.zeros((ny, nx), bool)
        Tw = np.zeros((ny, nx))
        for w in (3, 2, 1, 0):  # the x walls win at corners: written last
            if w < 2:
                on = wx & ((x == 0) if w == 0 else (x == nx - 1))
            else:
                on = wy & ((y == 0) if w == 2 else (y == ny - 1))
            if int(p["wall_thermal"][w]) == 0:
                dirichlet |= on
                Tw = np.where(on, p["T_wall"][w], Tw)
        # a corner with an adiabatic x wall takes the y wall's Dirichlet value
        self.wall = torch.as_tensor(wall)
        self.src = torch.as_tensor((yf * nx + xf).reshape(-1))
        self.dirichlet = torch.as_tensor(dirichlet)
        self.Tw = torch.as_tensor(Tw)

    # ---- building blocks (Eqs. 24, 50, 51, forcing of Eq. 12) ----
    def _d01(self, phi, Hv):
        hv_f = Hv * (self.d["alpha_f"] / (self.d["L"] * self.d["L"]))
        return 0.5 * hv_f / phi, 0.5 * hv_f / ((1.0 - phi) * self.p["sigma"])

    def _feq(self, rho, ux, uy, phi):
        cs2 = 1.0 / 3.0
        eu = self.ex * ux + self.ey * uy
        uu = ux * ux + uy * uy
        return self.w9.view(9, 1, 1) * rho * (1.0 + eu / cs2 + eu * eu / (2.0 * phi * cs2 * cs2)
                                              - uu / (2.0 * phi * cs2))

    def _geq_fluid(self, T, ux, uy, phi):
        v = float(self.p["varpi"])
        eu = self.ex[:5] * ux + self.ey[:5] * uy
        g = 0.25 * v * T + 0.5 * eu * T / phi
        return torch.cat([((1.0 - v) * T).unsqueeze(0), g[1:]], 0)

    def _geq_solid(self, T):
        return self.wt.view(5, 1, 1) * T

    def _forcing(self, rho, ux, uy, Fx, Fy, phi):
        cs2 = 1.0 / 3.0
        uF = ux * Fx + uy * Fy
        eF = self.ex * Fx + self.ey * Fy
        eu = self.ex * ux + self.ey * uy
        return self.w9.view(9, 1, 1) * rho * (eF / cs2 + eu * eF / (phi * cs2 * cs2) - uF / (phi * cs2))

    def _Fphi(self, phi):
        if self.p["F_phi"] >= 0.0:
            return torch.full_like(phi, float(self.p["F_phi"]))
        return 1.75 / torch.sqrt(150.0 * phi * phi * phi)  # Ergun, Eq. 7

    def _buoyancy(self, Tf):
        Gx = torch.full_like(Tf, float(self.p["body_force"][0]))
        Gy = self.p["body_force"][1] + self.d["gbeta"] * (Tf - self.p["T0"])
        return Gx, Gy

    def _macros(self, f, gf, gs, phi, Hv):
        """Eqs. 18, 43-46, 42, 6, 21, 22, 20, 5 at every node."""
        p, d = self.p, self.d
        d0, d1 = self._d01(phi, Hv)
        rho = f.sum(0)
        A = gf.sum(0) + 0.5 * p["Qf"]
        B = gs.sum(0) + 0.5 * p["Qs"]
        Tf = ((1.0 + d1) * A + d0 * B) / (1.0 + d0 + d1)
        Ts = (d1 * A + (1.0 + d0) * B) / (1.0 + d0 + d1)
        Srf = 2.0 * d0 * (Ts - Tf) + p["Qf"]
        Srs = 2.0 * d1 * (Tf - Ts) + p["Qs"]
        Gx, Gy = self._buoyancy(Tf)
        jx = (self.ex * f).sum(0)
        jy = (self.ey * f).sum(0)
        vx = jx / rho + 0.5 * phi * Gx
        vy = jy / rho + 0.5 * phi * Gy
        K = d["K"]
        Fphi = self._Fphi(phi)
        l0 = 0.5 * (1.0 + phi * 0.5 * d["nu_f"] / K)
        l1 = phi * 0.5 * Fphi / np.sqrt(K)
        vmag = _sqrt0(vx * vx + vy * vy)
        den = l0 + torch.sqrt(l0 * l0 + l1 * vmag)
        ux, uy = vx / den, vy / den
        umag = _sqrt0(ux * ux + uy * uy)
        Fx = -phi * d["nu_f"] / K * ux - phi * Fphi / np.sqrt(K) * umag * ux + phi * Gx
        Fy = -phi * d["nu_f"] / K * uy - phi * Fphi / np.sqrt(K) * umag * uy + phi * Gy
        return dict(rho=rho, ux=ux, uy=uy, Tf=Tf, Ts=Ts, Fx=Fx, Fy=Fy, Srf=Srf, Srs=Srs)

    def _at_src(self, a):
        """Value of a (..., ny, nx) at every node's inward neighbour."""
        lead = a.shape[:-2]
        return a.reshape(lead + (-1,))[..., self.src].reshape(a.shape)

    def _walls_macros_collide(self, f, gf, gs):
        p = self.p
        phi, Hv = self.phi, self.Hv
        m = self._macros(f, gf, gs, phi, Hv)
        # wall nodes: values of the inward neighbour x_f
        mf = {k: self._at_src(v) for k, v in m.items()}
        phif = self._at_src(phi)
        ff, gff, gsf = self._at_src(f), self._at_src(gf), self._at_src(gs)
        Tfb = torch.where(self.dirichlet, self.Tw, mf["Tf"])
        Tsb = torch.where(self.dirichlet, self.Tw, mf["Ts"])
        zero = torch.zeros_like(phi)
        fb = self._feq(mf["rho"], zero, zero, phi) + (ff - self._feq(mf["rho"], mf["ux"], mf["uy"], phif))
        gfb = self._geq_fluid(Tfb, zero, zero, phi) + (gff - self._geq_fluid(mf["Tf"], mf["ux"], mf["uy"], phif))
        gsb = self._geq_solid(Tsb) + (gsf - self._geq_solid(mf["Ts"]))
        d0, d1 = self._d01(phi, Hv)
        Gx, Gy = self._buoyancy(Tfb)
        mb = dict(rho=mf["rho"], ux=zero, uy=zero, Tf=Tfb, Ts=Tsb, Fx=phi * Gx, Fy=phi * Gy,
                  Srf=2.0 * d0 * (Tsb - Tfb) + p["Qf"], Srs=2.0 * d1 * (Tfb - Tsb) + p["Qs"])
        W = self.wall
        m = {k: torch.where(W, mb[k], m[k]) for k in m}
        f = torch.where(W, fb, f)
        gf = torch.where(W, gfb, gf)
        gs = torch.where(W, gsb, gs)
        self.macros = m
        return self._collide(m, f, gf, gs)

    def _collide(self, m, f, gf, gs):
        p, d, phi = self.p, self.d, self.phi
        mv = lambda A, x: torch.tensordot(A, x, dims=1)
        feq = self._feq(m["rho"], m["ux"], m["uy"], phi)
        S = self._forcing(m["rho"], m["ux"], m["uy"], m["Fx"], m["Fy"], phi)
        lam = torch.tensor([1.0, p["s_e"], p["s_eps"], 1.0, p["s_q"], 1.0, p["s_q"], d["s_nu"], d["s_nu"]],
                           dtype=DT).view(9, 1, 1)
        mom, meq, St = mv(self.M, f), mv(self.M, feq), mv(self.M, S)
        fo = mv(self.Mi, mom - lam * (mom - meq) + (1.0 - 0.5 * lam) * St)
        wt = self.wt.view(5, 1, 1)
        out = [fo]
        for g, geq, Sr, rates in (
                (gf, self._geq_fluid(m["Tf"], m["ux"], m["uy"], phi), m["Srf"],
                 (1.0, d["zeta_a"], d["zeta_a"], p["zeta_e"], p["zeta_nu"])),
                (gs, self._geq_solid(m["Ts"]), m["Srs"],
                 (1.0, d["eta_a"], d["eta_a"], p["eta_e"], p["eta_nu"]))):
            q = torch.tensor(rates, dtype=DT).view(5, 1, 1)
            n, neq, psi = mv(self.N, g), mv(self.N, geq), mv(self.N, wt * Sr)
            ns = n - q * (n - neq) + (1.0 - 0.5 * q) * psi
            if g is gf and int(p.get("thermal_correction", 0)):
                # correction term of Sec. 3.2: C~_i = w~_i T_f (e_i . F) / (phi cs_T^2)
                ex = torch.tensor(EX[:5], dtype=DT).view(5, 1, 1)
                ey = torch.tensor(EY[:5], dtype=DT).view(5, 1, 1)
                ct = wt * m["Tf"] * (ex * m["Fx"] + ey * m["Fy"]) / (phi * d["csT2"])
                ns = ns + (1.0 - 0.5 * q) * mv(self.N, ct)
            out.append(mv(self.Ni, ns))
        return tuple(out)

    def _stream(self, a, k):
        """Pull: a_i(x) = a*_i(x - e_i), periodic wrap (wall nodes are rebuilt)."""
        return torch.stack([torch.roll(a[i], shifts=(EY[i], EX[i]), dims=(0, 1)) for i in range(k)], 0)

    def step(self, n: int = 1) -> "DiffLattice":
        for _ in range(int(n)):
            f, gf, gs = self.state
            self.state = self._walls_macros_collide(self._stream(f, 9), self._stream(gf, 5), self._stream(gs, 5))
            self.steps += 1
        return self

    def detach(self) -> "DiffLattice":
        """Cut the graph: the current state becomes a constant input."""
        self.state = tuple(s.detach() for s in self.state)
        self.macros = {k: v.detach() for k, v in self.macros.items()}
        return self

    def nusselt(self, field: str = "Tf"):
        """Mean Nusselt number of T_f (or T_s) over the loss wall (a tensor)."""
        w = hot_wall(self.p)
        T = self.macros[field]
        if w == 0:
            t0, t1, t2 = T[:, 0], T[:, 1], T[:, 2]
        elif w == 1:
            t0, t1, t2 = T[:, -1], T[:, -2], T[:, -3]
        elif w == 2:
            t0, t1, t2 = T[0], T[1], T[2]
        else:
            t0, t1, t2 = T[-1], T[-2], T[-3]
        q = -(-3.0 * t0 + 4.0 * t1 - t2) / 2.0
        wt = torch.ones_like(q)
        if not (self.p["periodic_y"] if w < 2 else self.p["periodic_x"]):
            wt[0] = wt[-1] = 0.5
        return self.d["L"] / self.d["dT"] * (wt * q).sum() / wt.sum()


def gradients(p: dict, nsteps: int, phi, Hv, Tf0=None, Ts0=None, t0: int = 0):
    """Loss (mean hot-wall Nu_f after t0 + nsteps steps) and its gradients with
    respect to the per-node porosity and interphase coefficient.  With t0 > 0
    the state reached at t0 is taken as given (no gradient through it)."""
    phi_t = torch.as_tensor(np.asarray(phi, dtype=np.float64)).clone().requires_grad_(True)
    hv_t = torch.as_tensor(np.asarray(Hv, dtype=np.float64)).clone().requires_grad_(True)
    lat = DiffLattice(p, phi_t, hv_t, Tf0, Ts0)
    if t0 > 0:
        with torch.no_grad():
            lat.step(t0)
        lat.detach()
    lat.step(nsteps)
    loss = lat.nusselt()
    gp, gh = torch.autograd.grad(loss, (phi_t, hv_t))
    return float(loss.detach()), gp.numpy(), gh.numpy()
