// Fused time step of the LTNE MRT lattice Boltzmann model (Liu & He,
// arXiv:1608.04118, Sec. 3) for gfx950: one workgroup per tile, one node per
// thread.  Each thread
//   1. pulls its 19 post-collision populations of the previous time step
//      from its neighbours (streaming, Eqs. 11, 34, 35) -- a wall node pulls
//      those of its inward neighbour instead;
//   2. computes the temperatures (Eqs. 43-46), the buoyancy (Eq. 6), the
//      velocity (Eqs. 20-22) and the total force (Eq. 5);
//   3. on a wall node, rebuilds its populations by non-equilibrium
//      extrapolation from the inward neighbour and takes the prescribed
//      wall values (rho of the neighbour, u = 0, wall temperature);
//   4. collides the three lattices in moment space (Eqs. 10, 32, 33) with the
//      transforms of Eqs. 13 and 36 unrolled into adds and a few multiplies;
//   5. stores the 19 post-collision populations at its own node.
// All populations are stored shifted by their rest state (w_i rho0 and
// w~_i T_ref), which is exact in real arithmetic and keeps the stored values
// small enough for binary32 and binary16.
#pragma once

#include "common.hpp"

namespace ltne {

template <typename S>
__device__ __forceinline__ S load_raw(const S* __restrict__ p) {
  if constexpr (kNtLoad) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}

// Element i of a population row: a wave-uniform 64-bit row base plus the
// lane's 32-bit byte offset, which maps to the scalar-base + vector-offset
// form of the global memory instructions.
template <typename S>
__device__ __forceinline__ const S* at(const S* __restrict__ base, uint32_t i) {
  return reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + i * static_cast<uint32_t>(sizeof(S)));
}
template <typename S>
__device__ __forceinline__ S* at(S* __restrict__ base, uint32_t i) {
  return reinterpret_cast<S*>(reinterpret_cast<char*>(base) + i * static_cast<uint32_t>(sizeof(S)));
}

template <typename S, typename C>
__device__ __forceinline__ C load_pop(const S* __restrict__ p, C inv_scale) {
  if constexpr (std::is_same<S, _Float16>::value) {
    return static_cast<C>(static_cast<float>(load_raw(p))) * inv_scale;
  } else {
    (void)inv_scale;
    return static_cast<C>(load_raw(p));
  }
}

// NT: non-temporal store (the single-step kernels, whose rows are written
// whole by one wavefront); the two-step kernels store plainly, so the L2
// merges the partial cache lines that neighbouring strips write.
template <bool NT = kNtStore, typename S>
__device__ __forceinline__ void store_raw(S* __restrict__ p, S v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v, p);
  } else {
    *p = v;
  }
}

// Storage forms narrower than the arithmetic round stochastically: random
// bits are added below the kept significand bits, which are then truncated,
// so a value is rounded up with probability equal to its distance from the
// lower neighbour in units of the last place.  The expected stored value is
// the exact one: rounding errors no longer repeat themselves step after step
// on a slowly changing field (where round-to-nearest would add the same
// error at every step), they average out.  r carries the random bits in its
// top 16 bits (the low 16 bits are ignored).
template <typename S, typename V>
constexpr bool kStochastic = !std::is_same<S, V>::value;

// Arithmetic type of the two temperature lattices.  With binary32 storage and
// arithmetic the flow lattice is fine (its rounding errors are damped by the
// drag and viscosity within a few hundred steps), but the temperature
// lattices are not: their moment sums cancel (the non-equilibrium part of
// the D2Q5 energy moment is a small difference of populations of order
// T - T_ref), and a temperature that round-to-nearest stores shift by the
// same fraction of a unit in the last place at every step drifts over the
// field's diffusion time (1.3e-4 after 50000 steps of the 1024^2 cavity).
// The FP32 form therefore carries the temperature populations through
// binary64 arithmetic, from the binary32 loads to the binary32 stores; the
// moving populations are rounded to nearest and the rest population, which
// closes the zeroth moment (the temperature itself) exactly in binary64
// against the rounded moving ones, stochastically (kRestOnlySR): the stored
// temperature is then unbiased, and the errors of the other moments relax
// away.
template <typename S, typename C>
struct ThermalArith {
  using type = typename std::conditional<std::is_same<S, float>::value, double, C>::type;
};
template <typename S, typename C>
using thermal_t = typename ThermalArith<S, C>::type;
// Only the temperature lattices' rest populations round stochastically (the
// FP32 form); the narrow forms round every stored value stochastically.
template <typename S, typename C>
constexpr bool kRestOnlySR = std::is_same<S, float>::value && std::is_same<C, float>::value;

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// The storage value of v in a same-or-wider-than-storage form: binary64 ->
// binary32 rounds stochastically (29 discarded significand bits, 16 random
// ones added at their top, then truncated; the conversion is then exact),
// equal types pass through.
template <typename S, typename V>
__device__ __forceinline__ S to_storage(V v, uint32_t r) {
  if constexpr (std::is_same<S, float>::value && std::is_same<V, double>::value) {
    unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v)) +
                           (static_cast<unsigned long long>(r >> 16) << 13);
    u &= ~0x1fffffffull;
    return static_cast<float>(__longlong_as_double(static_cast<long long>(u)));  // exact
  } else {
    static_assert(std::is_same<S, V>::value, "storage narrower than the value needs a rounding rule");
    (void)r;
    return v;
  }
}

template <bool NT = kNtStore, typename S, typename V>
__device__ __forceinline__ void store_pop(S* __restrict__ p, V v, V scale, uint32_t r) {
  if constexpr (std::is_same<S, _Float16>::value) {
    // binary32 -> binary16: the gfx950 stochastic-rounding convert adds the
    // top 13 bits of r to the 13 discarded significand bits
    half2_t h = __builtin_nondeterministic_value(h);
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, static_cast<float>(v * scale), r, false);
    store_raw<NT>(p, h[0]);
  } else {
    (void)scale;
    store_raw<NT>(p, to_storage<S>(v, r));
  }
}

// Two stores that share one random word w: the first value takes its bottom
// half (moved to the top), the second its top half.  In binary16 both go
// through the gfx950 stochastic-rounding convert, which adds the top 13
// bits of its random operand to the 13 discarded significand bits, into the
// two halves of one register (h carries that register from pair to pair, so
// no register is cleared for it).  The two values may differ in type (a flow
// and a temperature population of the FP32 form).
template <bool NT = kNtStore, typename S, typename VA, typename VB>
__device__ __forceinline__ void store_pair(S* __restrict__ pa, VA va, VA sa, S* __restrict__ pb, VB vb, VB sb,
                                           uint32_t w, half2_t& h) {
  if constexpr (std::is_same<S, _Float16>::value) {
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, static_cast<float>(va * sa), w << 16, false);
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, static_cast<float>(vb * sb), w, true);
    store_raw<NT>(pa, h[0]);
    store_raw<NT>(pb, h[1]);
  } else {
    (void)h;
    store_pop<NT>(pa, va, sa, w << 16);
    store_pop<NT>(pb, vb, sb, w);
  }
}

// Reciprocal and reciprocal square root: the hardware approximations
// (v_rcp_f32 / v_rsq_f32, about 1 ulp) in binary32; in binary64 the hardware
// reciprocal refined by two Newton steps, r <- r + r (1 - v r) (each step
// squares the relative error, so the result is within about an ulp: five
// instructions against eleven for a correctly rounded division).  They only
// enter coefficients and small corrections, never a rounded factor applied
// to a conserved sum.
template <typename C>
__device__ __forceinline__ C dev_rcp(C v) {
  if constexpr (std::is_same<C, double>::value) {
    double r = __builtin_amdgcn_rcp(v);
    r = __builtin_fma(r, __builtin_fma(-v, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-v, r, 1.0), r);
  } else {
    return __builtin_amdgcn_rcpf(v);
  }
}

// Reciprocal in the temperature arithmetic: exact in binary64 forms; in
// the FP32 form (binary64 temperatures, binary32 elsewhere) the binary32
// hardware reciprocal refined by one Newton step (relative error ~1e-14,
// far below the binary32 storage of the result).
template <typename C, typename T>
__device__ __forceinline__ T thermal_rcp(T v) {
  if constexpr (std::is_same<T, double>::value && std::is_same<C, float>::value) {
    double r = static_cast<double>(__builtin_amdgcn_rcpf(static_cast<float>(v)));
    return r + r * (1.0 - v * r);
  } else {
    return dev_rcp(v);
  }
}

template <typename C>
__device__ __forceinline__ C dev_rsqrt(C v) {
  if constexpr (std::is_same<C, double>::value) {
    return dev_rcp(sqrt(v));
  } else {
    return __builtin_amdgcn_rsqf(v);
  }
}

template <typename C>
__device__ __forceinline__ C dev_sqrt(C v) {
  if constexpr (std::is_same<C, double>::value) {
    return sqrt(v);
  } else {
    return __builtin_sqrtf(v);
  }
}

// v^0.644 for v >= 0 (the Reynolds-number exponent of Eq. 52): exp2 of
// 0.644 log2 v with the hardware log2 / exp2 in binary32, pow in binary64.
template <typename C>
__device__ __forceinline__ C pow_0644(C v) {
  if constexpr (std::is_same<C, double>::value) {
    return v > 0.0 ? pow(v, 0.644) : 0.0;
  } else {
    return v > 1e-30f ? __builtin_amdgcn_exp2f(0.644f * __builtin_amdgcn_logf(v)) : 0.0f;
  }
}

// Where a node update takes its 19 pulled populations from and puts its 19
// post-collision ones.  The global forms read and write the population
// buffers in device memory; the two-step kernel substitutes register and
// cross-lane forms for its intermediate time level.

// Pull: population i arrives from node (xc, yc) - e_i.  A wave covers part
// of one lattice row, so the three source rows are wave-uniform: their bases
// are formed once in scalar registers (readfirstlane tells the compiler) and
// every load is a scalar base plus the lane's x.
template <typename S, typename C>
struct GlobalPull {
  const S* __restrict__ src;
  __device__ __forceinline__ void operator()(int xc, int yc, const StepConsts<C>& k, C (&v)[kPlanes]) const {
    const int nx = k.nx, ny = k.ny;
    const int yu = __builtin_amdgcn_readfirstlane(yc);
    int xm = xc - 1, xp = xc + 1, ym = yu - 1, yp = yu + 1;
    if (k.px) {
      xm = (xc == 0) ? nx - 1 : xm;
      xp = (xc == nx - 1) ? 0 : xp;
    }
    if (k.py) {
      ym = (yu == 0) ? ny - 1 : ym;
      yp = (yu == ny - 1) ? 0 : yp;
    }
    const long long Q = k.qs;
    const S* __restrict__ s0 = src + yu * k.rs;
    const S* __restrict__ sm = src + ym * k.rs;
    const S* __restrict__ sp = src + yp * k.rs;
    const C isf = k.inv_sf, isg = k.inv_sg;
    v[0] = load_pop(at(s0 + 0 * Q, xc), isf);
    v[1] = load_pop(at(s0 + 1 * Q, xm), isf);
    v[2] = load_pop(at(sm + 2 * Q, xc), isf);
    v[3] = load_pop(at(s0 + 3 * Q, xp), isf);
    v[4] = load_pop(at(sp + 4 * Q, xc), isf);
    v[5] = load_pop(at(sm + 5 * Q, xm), isf);
    v[6] = load_pop(at(sm + 6 * Q, xp), isf);
    v[7] = load_pop(at(sp + 7 * Q, xp), isf);
    v[8] = load_pop(at(sp + 8 * Q, xm), isf);
    v[9] = load_pop(at(s0 + 9 * Q, xc), isg);
    v[10] = load_pop(at(s0 + 10 * Q, xm), isg);
    v[11] = load_pop(at(sm + 11 * Q, xc), isg);
    v[12] = load_pop(at(s0 + 12 * Q, xp), isg);
    v[13] = load_pop(at(sp + 13 * Q, xc), isg);
    v[14] = load_pop(at(s0 + 14 * Q, xc), isg);
    v[15] = load_pop(at(s0 + 15 * Q, xm), isg);
    v[16] = load_pop(at(sm + 16 * Q, xc), isg);
    v[17] = load_pop(at(s0 + 17 * Q, xp), isg);
    v[18] = load_pop(at(sp + 18 * Q, xc), isg);
  }
};

// Put: the node's own 19 slots of the destination buffer, in pairs that
// share one random word (see store_pair); NT selects non-temporal stores.
template <typename S, typename C, bool NT = kNtStore>
struct GlobalPut {
  S* __restrict__ dst;
  S* __restrict__ drow = nullptr;
  long long P = 0;
  int x = 0;
  __device__ __forceinline__ void begin(int x_, int y, const StepConsts<C>& k) {
    drow = dst + static_cast<long long>(__builtin_amdgcn_readfirstlane(y)) * k.rs;
    P = k.qs;
    x = x_;
  }
  template <typename VA, typename VB>
  __device__ __forceinline__ void pair(int i, VA va, VA sa, int j, VB vb, VB sb, uint32_t w, half2_t& h) {
    store_pair<NT>(at(drow + i * P, x), va, sa, at(drow + j * P, x), vb, sb, w, h);
  }
  template <typename V>
  __device__ __forceinline__ void single(int i, V v, V s, uint32_t r) { store_pop<NT>(at(drow + i * P, x), v, s, r); }
};

// Porosity and H_v of the node whose populations a node update pulls (the
// node itself, or its inward neighbour at a wall).  A caller that reads them
// ahead, with the populations, passes them in; otherwise the update reads
// them where it needs them.
template <typename C>
struct CenterFields {
  C phi, hv;
};

template <typename C, int F>
__device__ __forceinline__ CenterFields<C> load_center(const C* __restrict__ phi_field,
                                                       const C* __restrict__ hv_field, const int ic,
                                                       const StepConsts<C>& k) {
  return {(F & kPhiField) ? phi_field[ic] : k.phi_u, (F & kHvField) ? hv_field[ic] : k.hv_u};
}

// kt: the temperature-lattice constants of k (thermal_k), passed apart so a
// caller can hand in a copy in LDS (the two-step kernel: vector operands that
// free the scalar registers of the binary64 constants).  pre: the fields at
// the pulled node, read ahead by the caller (nullptr: read here).
template <typename S, typename C, int F, class Pull, class Put>
__device__ __forceinline__ void node_update_with(
    const int x, const int y, const Pull& pull, Put& put,
    const C* __restrict__ phi_field, const C* __restrict__ hv_field, C* __restrict__ mac,
    const C* __restrict__ init_tf, const C* __restrict__ init_ts, const StepConsts<C>& k,
    const uint32_t step, C* __restrict__ rec, const ThermalK<thermal_t<S, C>>& kt,
    const CenterFields<C>* pre = nullptr);

// One node update: pull, macros, walls, collisions, store.  step numbers
// the time step being computed (0: initialisation); with a narrow storage
// form it seeds the stochastic rounding of the stores.
template <typename S, typename C, int F>
__device__ __forceinline__ void node_update(
    const int x, const int y, const S* __restrict__ src, S* __restrict__ dst,
    const C* __restrict__ phi_field, const C* __restrict__ hv_field, C* __restrict__ mac,
    const C* __restrict__ init_tf, const C* __restrict__ init_ts, const StepConsts<C>& k,
    const uint32_t step, C* __restrict__ rec = nullptr) {
  const GlobalPull<S, C> pull{src};
  GlobalPut<S, C> put{dst};
  node_update_with<S, C, F>(x, y, pull, put, phi_field, hv_field, mac, init_tf, init_ts, k, step, rec,
                            thermal_k<thermal_t<S, C>>(k));
}

template <typename S, typename C, int F, class Pull, class Put>
__device__ __forceinline__ void node_update_with(
    const int x, const int y, const Pull& pull, Put& put,
    const C* __restrict__ phi_field, const C* __restrict__ hv_field, C* __restrict__ mac,
    const C* __restrict__ init_tf, const C* __restrict__ init_ts, const StepConsts<C>& k,
    const uint32_t step, C* __restrict__ rec, const ThermalK<thermal_t<S, C>>& kt,
    const CenterFields<C>* pre) {
  const int nx = k.nx, ny = k.ny;

  // Wall classification and the node whose post-streaming populations this
  // thread reads: itself, or the inward neighbour (diagonal at a corner).
  const bool wx = !k.px && (x == 0 || x == nx - 1);
  const bool wy = !k.py && (y == 0 || y == ny - 1);
  const bool wall = wx || wy;
  const int xc = wx ? (x == 0 ? 1 : nx - 2) : x;
  const int yc = wy ? (y == 0 ? 1 : ny - 2) : y;
  const int ic = yc * nx + xc;

  const CenterFields<C> cf = pre ? *pre : load_center<C, F>(phi_field, hv_field, ic, k);
  const C phi_c = cf.phi;
  const C hv_c = cf.hv;

  // T: arithmetic type of the temperature lattices (see ThermalArith)
  using T = thermal_t<S, C>;
  C f0, f1, f2, f3, f4, f5, f6, f7, f8;
  T a0, a1, a2, a3, a4;  // fluid temperature populations
  T b0, b1, b2, b3, b4;  // solid minus fluid temperature populations
  if constexpr ((F & kInit) != 0) {
    // t = 0: fluid at rest at rho0 (all shifted D2Q9 populations vanish) and
    // g = w~ (T - Sr / 2), so that Eqs. 43-44 give back the initial T.
    const T thf = init_tf ? T(init_tf[ic]) : kt.theta_init_f;
    const T ths = init_ts ? T(init_ts[ic]) : kt.theta_init_s;
    const C hv = k.hv_corr ? C(0) : hv_c * k.hvf;  // the correlation gives 0 at rest
    const C rpp = dev_rcp(phi_c * (C(1) - phi_c));  // as in the step below
    const T d0 = T(C(0.5) * hv * ((C(1) - phi_c) * rpp));
    const T d1 = T(C(0.5) * hv * k.inv_sigma * (phi_c * rpp));
    const T srf = T(2) * d0 * (ths - thf) + kt.Qf;
    const T srs = T(2) * d1 * (thf - ths) + kt.Qs;
    const T w0 = kt.w0, w1 = kt.w1;
    f0 = f1 = f2 = f3 = f4 = f5 = f6 = f7 = f8 = C(0);
    const T gf = thf - T(0.5) * srf;
    const T gh = (ths - thf) - T(0.5) * (srs - srf);
    a0 = w0 * gf;
    a1 = a2 = a3 = a4 = w1 * gf;
    b0 = w0 * gh;
    b1 = b2 = b3 = b4 = w1 * gh;
  } else {
    C v[kPlanes];
    pull(xc, yc, k, v);
    f0 = v[0]; f1 = v[1]; f2 = v[2]; f3 = v[3]; f4 = v[4]; f5 = v[5]; f6 = v[6]; f7 = v[7]; f8 = v[8];
    a0 = v[9]; a1 = v[10]; a2 = v[11]; a3 = v[12]; a4 = v[13];
    b0 = v[14]; b1 = v[15]; b2 = v[16]; b3 = v[17]; b4 = v[18];
  }

  // ---- macros at (xc, yc) ----
  // Temperatures, Eqs. 43-46, relative to T_ref.  The solid lattice is
  // carried as its difference from the fluid one, so its zeroth moment is
  // sum g_s - sum g_f directly and
  //   D = T_s - T_f = (B - A) / (1 + d0 + d1),  T_f = A + d0 D,  T_s = T_f + D,
  // which equals Eqs. 43-44.  The interphase exchange of one step, 2 d0 D,
  // can be far below the rounding unit of the temperature populations
  // themselves; on the difference lattice it is resolved to full relative
  // precision, and no carried sum is ever scaled by a rounded factor close
  // to 1 (a systematic drift in binary32 otherwise).
  // Density (Eq. 18) and momentum sums.
  const C drho = ((f0 + f1) + (f2 + f3)) + ((f4 + f5) + (f6 + f7)) + f8;
  const C rho = k.rho0 + drho;
  const C jx = (f1 - f3) + (f5 - f6) + (f8 - f7);
  const C jy = (f2 - f4) + (f5 + f6) - (f7 + f8);
  const C inv_rho = dev_rcp(rho);

  C hv = hv_c * k.hvf;  // h_v / (rho c_p)_f
  if (k.hv_corr) {
    // Eq. 52 with the local velocity u_m = |j| / rho (u of Eq. 20 needs T_f,
    // which needs h_v): h_v / (rho c_p)_f = corr_a Re^0.644, Re = corr_b u_m
    hv = k.corr_a * pow_0644(k.corr_b * dev_sqrt(jx * jx + jy * jy) * inv_rho);
  }
  // 1 / phi and 1 / (1 - phi) from one reciprocal (transcendentals issue at a
  // fraction of the rate of multiplies)
  const C rpp = dev_rcp(phi_c * (C(1) - phi_c));
  const C rphi_c = (C(1) - phi_c) * rpp;
  T d0 = T(C(0.5) * hv * rphi_c);
  T d1 = T(C(0.5) * hv * k.inv_sigma * (phi_c * rpp));
  const T sgf = ((a0 + a1) + (a2 + a3)) + a4;
  const T sgh = ((b0 + b1) + (b2 + b3)) + b4;  // sum g_s - sum g_f
  const T A = sgf + kt.hQf;
  T D = (sgh + kt.hdQ) * thermal_rcp<C>(T(1) + d0 + d1);
  T thf = A + d0 * D;
  T ths = thf + D;

  if constexpr ((F & kRecord) != 0) {
    if (!wall) {
      const int ir = y * nx + x;
      rec[0 * k.mplane + ir] = drho;
      rec[1 * k.mplane + ir] = jx;
      rec[2 * k.mplane + ir] = jy;
      rec[3 * k.mplane + ir] = C(sgf);
      rec[4 * k.mplane + ir] = C(sgh);
    }
  }

  // Buoyancy (Eq. 6, gravity along -y) plus body acceleration.
  const C Gx = k.Gbx;
  C Gy = k.Gby + k.gbeta * (C(thf) + k.dT0);

  // Velocity, Eqs. 20-22, and total force, Eq. 5 (rFx = rho F_x).
  C ux, uy, rFx, rFy;
  {
    const C Fphi = (k.Fphi >= C(0)) ? k.Fphi : C(1.75) * dev_rsqrt(C(150) * phi_c * phi_c * phi_c);
    const C vx = jx * inv_rho + C(0.5) * phi_c * Gx;
    const C vy = jy * inv_rho + C(0.5) * phi_c * Gy;
    const C l0 = C(0.5) * (C(1) + C(0.5) * phi_c * k.nu_over_K);
    const C l1 = C(0.5) * phi_c * Fphi * k.inv_sqrtK;
    const C vm = dev_sqrt(vx * vx + vy * vy);
    const C den = l0 + dev_sqrt(l0 * l0 + l1 * vm);
    const C rden = dev_rcp(den);
    ux = vx * rden;
    uy = vy * rden;
    const C um = vm * rden;  // |u| = |v| / den (Eq. 20)
    const C drag = -phi_c * (k.nu_over_K + Fphi * k.inv_sqrtK * um);
    rFx = rho * (drag * ux + phi_c * Gx);
    rFy = rho * (drag * uy + phi_c * Gy);
  }
  // Post-collision conserved moments.  In the interior, Eq. 19 gives
  // rho u + rho F / 2 = j + rho F (momentum plus the force of one step) and
  // the zeroth thermal moments gain the source: n_0* = n_0 + Sr (for the
  // difference lattice: Sr_s - Sr_f = Q_s - Q_f - 2 (d0 + d1) D).
  C ms3 = jx + rFx, ms5 = jy + rFy;
  T srf = T(2) * d0 * D + kt.Qf;  // Eq. 42
  T srs = T(-2) * d1 * D + kt.Qs;
  T dsr = srs - srf;  // Sr_s - Sr_f
  T nf0 = sgf + srf, nh0 = sgh + dsr;

  C phi = phi_c;
  C rphi = rphi_c;
  if (wall) {
    // Non-equilibrium extrapolation from the inward neighbour:
    //   f(x_b) = f^eq(rho, 0) + f(x_f) - f^eq(rho, u),
    //   g_f(x_b) = g_f^eq(T_b, 0) + g_f(x_f) - g_f^eq(T_f, u), g_s likewise
    // (the difference lattice takes the difference of the two).
    T thfb = thf, thsb = ths;
    int kind = 1;
    {
      T tw = T(0);
      if (wx) {
        const int w = (x == 0) ? 0 : 1;
        if (k.wall_kind[w] == 0) { kind = 0; tw = kt.theta_wall[w]; }
      }
      if (kind != 0 && wy) {
        const int w = (y == 0) ? 2 : 3;
        if (k.wall_kind[w] == 0) { kind = 0; tw = kt.theta_wall[w]; }
      }
      if (kind == 0) thfb = thsb = tw;
    }
    // T_s - T_f at the wall: zero on a Dirichlet wall, D of x_f otherwise
    const T Db = (kind == 0) ? T(0) : D;
    const C ip = rphi_c;
    const C uu = (ux * ux + uy * uy) * ip;
    const C r9 = rho * (C(1) / C(9)), r36 = rho * (C(1) / C(36));
    // f^eq(rho,0) - f^eq(rho,u) = -w rho [3 e.u + 4.5 (e.u)^2 / phi - 1.5 u^2 / phi]
    const C q0 = C(1.5) * uu;
    f0 += C(4) * r9 * q0;
    f1 -= r9 * (C(3) * ux + C(4.5) * ux * ux * ip - q0);
    f3 -= r9 * (-C(3) * ux + C(4.5) * ux * ux * ip - q0);
    f2 -= r9 * (C(3) * uy + C(4.5) * uy * uy * ip - q0);
    f4 -= r9 * (-C(3) * uy + C(4.5) * uy * uy * ip - q0);
    const C sp = ux + uy, sm = ux - uy;
    f5 -= r36 * (C(3) * sp + C(4.5) * sp * sp * ip - q0);
    f7 -= r36 * (-C(3) * sp + C(4.5) * sp * sp * ip - q0);
    f8 -= r36 * (C(3) * sm + C(4.5) * sm * sm * ip - q0);
    f6 -= r36 * (-C(3) * sm + C(4.5) * sm * sm * ip - q0);
    const T w0 = kt.w0, w1 = kt.w1;
    const T dtf = thfb - thf, dD = Db - D;
    const T adv = T(0.5) * (thf + kt.T_ref) * T(ip);  // (e.u) T_f / (2 phi)
    const T tux = T(ux), tuy = T(uy);
    a0 += w0 * dtf;
    a1 += w1 * dtf - adv * tux;
    a3 += w1 * dtf + adv * tux;
    a2 += w1 * dtf - adv * tuy;
    a4 += w1 * dtf + adv * tuy;
    b0 += w0 * dD;
    b1 += w1 * dD + adv * tux;
    b3 += w1 * dD - adv * tux;
    b2 += w1 * dD + adv * tuy;
    b4 += w1 * dD - adv * tuy;
    // Prescribed wall values; coefficients at the wall node itself.
    const int ib = y * nx + x;
    phi = (F & kPhiField) ? phi_field[ib] : k.phi_u;
    const C rppb = dev_rcp(phi * (C(1) - phi));
    rphi = (C(1) - phi) * rppb;
    // (u = 0 at the wall: the correlation gives h_v = 0 there)
    const C hvb = k.hv_corr ? C(0) : ((F & kHvField) ? hv_field[ib] : k.hv_u) * k.hvf;
    d0 = T(C(0.5) * hvb * rphi);
    d1 = T(C(0.5) * hvb * k.inv_sigma * (phi * rppb));
    thf = thfb;
    ths = thsb;
    D = Db;
    Gy = k.Gby + k.gbeta * (C(thf) + k.dT0);
    ux = C(0);
    uy = C(0);
    rFx = rho * phi * Gx;
    rFy = rho * phi * Gy;
    ms3 = C(0.5) * rFx;  // rho u + rho F / 2 with u = 0
    ms5 = C(0.5) * rFy;
    srf = T(2) * d0 * D + kt.Qf;
    srs = T(-2) * d1 * D + kt.Qs;
    dsr = srs - srf;
    nf0 = thf + T(0.5) * srf;  // n_0* = T + Sr / 2 (Eq. 41 at the wall)
    nh0 = D + T(0.5) * dsr;
  }

  if constexpr ((F & kMacros) != 0) {
    const int ib = y * nx + x;
    mac[0 * k.mplane + ib] = rho;
    mac[1 * k.mplane + ib] = ux;
    mac[2 * k.mplane + ib] = uy;
    mac[3 * k.mplane + ib] = C(thf + kt.T_ref);
    mac[4 * k.mplane + ib] = C(ths + kt.T_ref);
  }

  const int io = y * nx + x;  // node index (hash input)
  put.begin(x, y, k);
  // 19 x 16 random bits for the stores, two stores per word (its top and
  // its bottom half moved to the top; population 8 takes the top half of
  // word 4 alone).  The FP32 form needs only the two rest populations'
  // 16 bits each: the halves of the node's hash itself (word 5).
  uint32_t rb[10];
  if constexpr (kRestOnlySR<S, C>) {
#pragma unroll
    for (int j = 0; j < 10; ++j) rb[j] = 0u;
    rb[5] = mix32(static_cast<uint32_t>(io) ^ mix32(step * 0x9e3779b9u + 0x632be5abu));
  } else if constexpr (kStochastic<S, C>) {
    const uint32_t base = mix32(static_cast<uint32_t>(io) ^ mix32(step * 0x9e3779b9u + 0x632be5abu));
    // word j: one xor-shift / multiply / xor-shift round of base + j K (the
    // full two-multiply mix is kept for base; a second multiply per word cost
    // 2% of the binary16 step and adds nothing the rounding can use)
#pragma unroll
    for (int j = 0; j < 10; ++j) {
      uint32_t w = base + static_cast<uint32_t>(j) * 0x85ebca77u;
      w ^= w >> 16;
      w *= 0x7feb352du;
      w ^= w >> 15;
      rb[j] = w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 10; ++j) rb[j] = 0u;
  }

  half2_t hs = __builtin_nondeterministic_value(hs);  // binary16 store register (see store_pair)
  // ---- D2Q9 collision in moment space (Eq. 10) ----
  {
    const C ip = rphi;
    const C s14 = (f1 + f2) + (f3 + f4);
    const C s58 = (f5 + f6) + (f7 + f8);
    const C m1 = C(-4) * f0 - s14 + C(2) * s58;
    const C m2 = C(4) * f0 - C(2) * s14 + s58;
    const C m4 = C(2) * (f3 - f1) + (f5 - f6) + (f8 - f7);
    const C m6 = C(2) * (f4 - f2) + (f5 + f6) - (f7 + f8);
    const C m7 = (f1 - f2) + (f3 - f4);
    const C m8 = (f5 - f6) + (f7 - f8);
    const C jxr = rho * ux, jyr = rho * uy;
    const C e3 = C(3) * rho * (ux * ux + uy * uy) * ip;
    // equilibria (Eq. 15) relative to the rest state
    const C meq1 = C(-2) * drho + e3;
    const C meq2 = drho - e3;
    const C meq7 = rho * (ux * ux - uy * uy) * ip;
    const C meq8 = rho * ux * uy * ip;
    // forcing moments S~ = M S
    const C uF = (ux * rFx + uy * rFy) * ip;
    const C S1 = C(6) * uF;
    const C S7 = C(2) * (ux * rFx - uy * rFy) * ip;
    const C S8 = (ux * rFy + uy * rFx) * ip;
    const C ms0 = drho;
    const C ms1 = m1 - k.s_e * (m1 - meq1) + (C(1) - C(0.5) * k.s_e) * S1;
    const C ms2 = m2 - k.s_eps * (m2 - meq2) - (C(1) - C(0.5) * k.s_eps) * S1;
    const C ms4 = m4 - k.s_q * (m4 + jxr) - (C(1) - C(0.5) * k.s_q) * rFx;
    const C ms6 = m6 - k.s_q * (m6 + jyr) - (C(1) - C(0.5) * k.s_q) * rFy;
    const C ms7 = m7 - k.s_nu * (m7 - meq7) + (C(1) - C(0.5) * k.s_nu) * S7;
    const C ms8 = m8 - k.s_nu * (m8 - meq8) + (C(1) - C(0.5) * k.s_nu) * S8;
    // f* = M^{-1} m*, M^{-1} = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const C a = ms0 * (C(1) / C(9));
    const C b = ms1 * (C(1) / C(36));
    const C c = ms2 * (C(1) / C(36));
    const C d = ms3 * (C(1) / C(6));
    const C e = ms4 * (C(1) / C(12));
    const C g = ms5 * (C(1) / C(6));
    const C h = ms6 * (C(1) / C(12));
    const C p = ms7 * C(0.25);
    const C q = ms8 * C(0.25);
    const C base1 = a - b - C(2) * c;
    const C base5 = a + C(2) * b + c;
    const C de = d + e, gh = g + h;
    const C o1 = base1 + (d - C(2) * e) + p;
    const C o2 = base1 + (g - C(2) * h) - p;
    const C o5 = base5 + de + gh + q;
    const C o6 = base5 - de + gh - q;
    const C o7 = base5 - de - gh + q;
    const C o8 = base5 + de - gh - q;
    // f3, f4 and f0 close the conserved moments (momentum ms3, ms5 and mass
    // ms0) up to one rounding each, so the inexact constants 1/6, 1/9, ...
    // cannot bias them from step to step.
    const C o3 = o1 + ((o5 - o6) + (o8 - o7)) - ms3;
    const C o4 = o2 + ((o5 + o6) - (o7 + o8)) - ms5;
    const C o0 = ms0 - (((o1 + o2) + (o3 + o4)) + ((o5 + o6) + (o7 + o8)));
    const C sf = k.sf;
    put.pair(0, o0, sf, 1, o1, sf, rb[0], hs);
    put.pair(2, o2, sf, 3, o3, sf, rb[1], hs);
    put.pair(4, o4, sf, 5, o5, sf, rb[2], hs);
    put.pair(6, o6, sf, 7, o7, sf, rb[3], hs);
    put.single(8, o8, sf, rb[4]);
  }

  // ---- D2Q5 collisions (Eqs. 32, 33) ----
  // g* = N^{-1} n* with N^{-1} = N^T diag(1/5, 1/2, 1/2, 1/20, 1/4): with
  // base = n0*/5 + n3*/20, the moving populations are base +- n1*/2 + n4*/4
  // (along x) and base +- n2*/2 - n4*/4 (along y), the rest population
  // (n0* - n3*)/5.
  {
    const T ip = T(rphi);
    const T Tf = thf + kt.T_ref;
    const T sg = kt.sg;
    const T Tfip = Tf * ip;
    const T qx = T(ux) * Tfip, qy = T(uy) * Tfip;  // equilibrium heat flux u T_f / phi (Eq. 37)
    // correction term of Sec. 3.2 in moments: (1 - zeta_a / 2) T_f F / phi
    // added to the post-collision heat flux of the fluid lattice (tc = 0
    // when the term is off); F = rho F / rho, the node's force of Eq. 5
    const T tcf = kt.tc * Tfip * T(inv_rho);
    // fluid phase, equilibria of Eq. 37, source moments (Sr, 0, 0, c1 Sr, 0):
    //   n1* = n1 - zeta_a (n1 - u_x T_f / phi) (+ correction),
    //   n3* = n3 - zeta_e (n3 - c1 T_f) + (1 - zeta_e / 2) c1 Sr_f,
    //   n4* = (1 - zeta_nu) n4;
    // tx = zeta_a (n1 - u_x T_f / phi) - correction and u3 = n3 - c1 T_f are
    // shared with the solid phase
    const T nf1 = a1 - a3, nf2 = a2 - a4;
    const T nf3 = T(-4) * a0 + ((a1 + a2) + (a3 + a4));
    const T nf4 = (a1 - a2) + (a3 - a4);
    const T tx = kt.z_a * (nf1 - qx) - tcf * T(rFx), ty = kt.z_a * (nf2 - qy) - tcf * T(rFy);
    const T u3 = nf3 - kt.c1 * thf;
    T f4o;  // its last population, stored with the solid lattice's first
    S f4;   // the same, rounded (FP32 form)
    {
      const T ns1 = nf1 - tx, ns2 = nf2 - ty;
      const T ns3 = (nf3 - kt.z_e * u3) + kt.k3 * srf;
      const T ns4 = nf4 - kt.z_nu * nf4;
      const T base = T(0.2) * nf0 + T(0.05) * ns3;
      const T px = base + T(0.25) * ns4, py = base - T(0.25) * ns4;
      if constexpr (kRestOnlySR<S, C>) {
        // moving populations rounded to nearest; the rest population closes
        // the zeroth moment against them in binary64, rounded stochastically
        const S q1 = S(px + T(0.5) * ns1), q2 = S(py + T(0.5) * ns2), q3 = S(px - T(0.5) * ns1);
        f4 = S(py - T(0.5) * ns2);
        const T rest = nf0 - ((T(q1) + T(q2)) + (T(q3) + T(f4)));
        put.pair(9, rest, sg, 10, q1, S(1), rb[5], hs);
        put.pair(11, q2, S(1), 12, q3, S(1), 0u, hs);
      } else {
        put.pair(9, T(0.2) * (nf0 - ns3), sg, 10, px + T(0.5) * ns1, sg, rb[5], hs);
        put.pair(11, py + T(0.5) * ns2, sg, 12, px - T(0.5) * ns1, sg, rb[6], hs);
        f4o = py - T(0.5) * ns2;
      }
    }
    // solid phase (Eq. 33, equilibria of Eq. 38), carried as the difference
    // h = g_s - g_f: in moments, n_h* = n_s* - n_f* with n_s = n_f + n_h,
    //   n_h1* = n_h1 - eta_a (n_h1 + n_f1) + zeta_a (n_f1 - u_x T_f / phi)
    //           (minus the fluid's correction term when it is on),
    //   n_h3* = n_h3 - eta_e (n_h3 + u3 - c1 D) + zeta_e u3
    //           + (1 - eta_e / 2) c1 Sr_s - (1 - zeta_e / 2) c1 Sr_f,
    //   n_h4* = n_h4 - eta_nu (n_h4 + n_f4) + zeta_nu n_f4,
    // every term small where the two phases are close.
    {
      const T n1 = b1 - b3, n2 = b2 - b4;
      const T n3 = T(-4) * b0 + ((b1 + b2) + (b3 + b4));
      const T n4 = (b1 - b2) + (b3 - b4);
      const T ns1 = (n1 - kt.e_a * (n1 + nf1)) + tx;
      const T ns2 = (n2 - kt.e_a * (n2 + nf2)) + ty;
      const T ns3 = ((n3 - kt.e_e * ((n3 + u3) - kt.c1 * D)) + kt.z_e * u3) + (kt.k4 * srs - kt.k3 * srf);
      const T ns4 = (n4 - kt.e_nu * (n4 + nf4)) + kt.z_nu * nf4;
      const T base = T(0.2) * nh0 + T(0.05) * ns3;
      const T px = base + T(0.25) * ns4, py = base - T(0.25) * ns4;
      if constexpr (kRestOnlySR<S, C>) {
        const S q1 = S(px + T(0.5) * ns1), q2 = S(py + T(0.5) * ns2), q3 = S(px - T(0.5) * ns1),
                q4 = S(py - T(0.5) * ns2);
        const T rest = nh0 - ((T(q1) + T(q2)) + (T(q3) + T(q4)));
        put.pair(13, f4, S(1), 14, rest, sg, rb[5], hs);  // the top half of the node's word
        put.pair(15, q1, S(1), 16, q2, S(1), 0u, hs);
        put.pair(17, q3, S(1), 18, q4, S(1), 0u, hs);
      } else {
        put.pair(13, f4o, sg, 14, T(0.2) * (nh0 - ns3), sg, rb[7], hs);
        put.pair(15, px + T(0.5) * ns1, sg, 16, py + T(0.5) * ns2, sg, rb[8], hs);
        put.pair(17, px - T(0.5) * ns1, sg, 18, py - T(0.5) * ns2, sg, rb[9], hs);
      }
    }
  }
}

// The nodes of the tile that workgroup b runs: tile (b % 8) * per_xcd + b / 8
// (see TileMap); each thread updates kRows nodes of one column of the tile,
// kRowStride rows apart.
template <typename S, typename C, int F>
__device__ __forceinline__ void step_tile(const S* __restrict__ src, S* __restrict__ dst,
                                          const C* __restrict__ phi_field, const C* __restrict__ hv_field,
                                          C* __restrict__ mac, const C* __restrict__ init_tf,
                                          const C* __restrict__ init_ts, const StepConsts<C>& k,
                                          const uint32_t step, C* __restrict__ rec) {
  const int b = blockIdx.x;
  const int t = kXcdRemap ? (b & (kXcds - 1)) * k.tm.per_xcd + (b >> 3) : b;
  if (t >= k.tm.ntiles) return;
  const int tx = t % k.tm.ntx;
  const int ty = t / k.tm.ntx;
  const int tw = 1 << k.tm.tw_shift;
  const int th = kBlock >> k.tm.tw_shift;
  const int x = tx * tw + (static_cast<int>(threadIdx.x) & (tw - 1));
  const int y0 = ty * th * kRows + (static_cast<int>(threadIdx.x) >> k.tm.tw_shift);
  if (x >= k.nx) return;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int y = y0 + r * th;
    if (y < k.ny) node_update<S, C, F>(x, y, src, dst, phi_field, hv_field, mac, init_tf, init_ts, k, step, rec);
  }
}

template <typename S, typename C, int F>
__global__ __launch_bounds__(kBlock) void step_kernel(
    const S* __restrict__ src, S* __restrict__ dst, const C* __restrict__ phi_field,
    const C* __restrict__ hv_field, C* __restrict__ mac, const C* __restrict__ init_tf,
    const C* __restrict__ init_ts, const StepConsts<C> k, const uint32_t step, C* __restrict__ rec = nullptr) {
  step_tile<S, C, F>(src, dst, phi_field, hv_field, mac, init_tf, init_ts, k, step, rec);
}

// The step as a node of a recorded sequence of steps (a HIP graph replayed
// many times): its step number, which seeds the stochastic rounding, is
// *step_base + offset, the base living in device memory and advanced by
// step_advance_kernel at the end of every replay.
template <typename S, typename C, int F>
__global__ __launch_bounds__(kBlock) void step_seq_kernel(const S* __restrict__ src, S* __restrict__ dst,
                                                          const C* __restrict__ phi_field,
                                                          const C* __restrict__ hv_field, const StepConsts<C> k,
                                                          const uint32_t* __restrict__ step_base,
                                                          const uint32_t offset) {
  step_tile<S, C, F>(src, dst, phi_field, hv_field, nullptr, nullptr, nullptr, k, *step_base + offset, nullptr);
}

// Sets (add = 0) or advances (add = 1) the device step base by n.
[[maybe_unused]] static __global__ void step_base_kernel(uint32_t* __restrict__ step_base, uint32_t n, int add) {
  if (threadIdx.x == 0) *step_base = add ? *step_base + n : n;
}

}  // namespace ltne
