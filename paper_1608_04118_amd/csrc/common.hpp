// Internal types shared by the host runtime and the kernels of the LTNE
// MRT lattice Boltzmann library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace ltne {

// Populations per node: 9 of the D2Q9 flow lattice (Eq. 8), 5 of the fluid
// and 5 of the solid D2Q5 temperature lattices: 0..8 f, 9..13 g_f,
// 14..18 g_s.  Population q of node (x, y) sits at y rs + q qs + x (see
// StepConsts): each lattice row stores its 19 population rows back to back.
constexpr int kPlanes = 19;
constexpr int kBlock = 256;  // threads per workgroup (4 wave64s)
constexpr int kXcds = 8;     // MI355X: workgroups are dealt round-robin to 8 XCDs

// Launch-shape and memory-path choices of the step kernel (compile time).
#ifndef LTNE_ROWS
#define LTNE_ROWS 1
#endif
#ifndef LTNE_TW_SHIFT_MAX
#define LTNE_TW_SHIFT_MAX 8
#endif
#ifndef LTNE_XCD_REMAP
#define LTNE_XCD_REMAP 1
#endif
#ifndef LTNE_NT_LOAD
#define LTNE_NT_LOAD 0
#endif
#ifndef LTNE_NT_STORE
#define LTNE_NT_STORE 1
#endif
constexpr int kRows = LTNE_ROWS;               // nodes per thread along y
constexpr int kTwShiftMax = LTNE_TW_SHIFT_MAX;  // widest tile: 2^k nodes
constexpr bool kXcdRemap = LTNE_XCD_REMAP != 0;
constexpr bool kNtLoad = LTNE_NT_LOAD != 0;
constexpr bool kNtStore = LTNE_NT_STORE != 0;
// Every wave of the step kernel covers one lattice row (tiles are at least
// 64 nodes wide), which its row addressing relies on.
static_assert(kTwShiftMax >= 6, "tiles narrower than a wave");

// Velocity components of Eq. 8 (D2Q9; the first five are the D2Q5 set).
__host__ __device__ constexpr int vel_x(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int vel_y(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}

// 32-bit integer mixer (xor-shift / multiply rounds of the kind used as the
// finalizer of MurmurHash3; constants from Wellons' low-bias search): every
// input bit affects every output bit.  Source of the stochastic-rounding bits,
// counter-based so a result depends only on (node, step), never on the
// launch shape or the order of execution.
__host__ __device__ constexpr uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// A device pointer read from memory (a batch's per-lattice buffers) is a
// generic pointer, and loads through it become flat-address instructions
// with 64-bit per-lane addresses.  Passing it through the global address
// space tells the compiler where it points, so it uses global loads and
// stores with a scalar base.
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
  return (T*)((__attribute__((address_space(1))) T*)p);
}

// Flags of the fused step kernel.
constexpr int kPhiField = 1;  // per-node porosity
constexpr int kHvField = 2;   // per-node interphase coefficient
constexpr int kMacros = 4;    // write rho, u, T_f, T_s of this step
constexpr int kInit = 8;      // build the t = 0 populations instead of streaming
constexpr int kRecord = 16;   // write q = (rho - rho0, j_x, j_y, sum g_f, sum h) at interior nodes

// Mapping of workgroups to lattice tiles.  A tile is tw x (kRows 256 / tw)
// nodes, tiles are numbered row-major, and workgroup b runs tile
// (b % 8) * per_xcd + b / 8 so that each XCD (and its L2) sweeps one
// contiguous band of rows.
struct TileMap {
  int tw_shift;  // log2 of the tile width (6, 7 or 8)
  int ntx;       // tiles per row of tiles
  int ntiles;    // tiles in the lattice
  int per_xcd;   // tiles per XCD; the grid has 8 * per_xcd workgroups
};

// Constants of the two temperature lattices in their arithmetic type T
// (binary64 for the forms with binary32 or binary64 storage, binary32 for
// binary16 storage), combined on the host.  Few on purpose: the node update
// keeps them in scalar registers, two per binary64 value.
template <typename T>
struct ThermalK {
  T Qf, Qs;               // heat sources (Eq. 45)
  T hQf, hdQ;             // Qf / 2, (Qs - Qf) / 2
  T T_ref;                // temperature shift
  T w0, w1;               // D2Q5 weights 1 - varpi and varpi / 4
  T theta_wall[4];        // Dirichlet wall temperatures relative to T_ref
  T theta_init_f, theta_init_s;
  T c1;                   // 5 varpi - 4
  T z_a, z_e, z_nu;       // fluid rates (Eq. 39)
  T e_a, e_e, e_nu;       // solid rates (Eq. 40)
  T k3, k4;               // (1 - zeta_e / 2) c1 and (1 - eta_e / 2) c1: source factors
  T tc;                   // 1 - zeta_a / 2 with the correction term of Sec. 3.2, else 0
  T sg;                   // storage scale of the D2Q5 populations (1 unless FP16)
};

// Constants of one lattice in the arithmetic type C.  Temperatures are
// carried relative to T_ref (theta = T - T_ref), populations relative to
// their rest state at rho0 and T_ref, in every precision form.
template <typename C>
struct StepConsts {
  int nx, ny;
  int px, py;            // periodic axes
  long long qs;          // elements between the rows of populations q and q + 1 of one lattice row
  long long rs;          // elements between lattice rows (19 qs)
  long long mplane;      // elements between macro planes
  TileMap tm;
  C rho0;
  C phi_u, hv_u;         // uniform porosity / interphase coefficient
  C gbeta, dT0;          // buoyancy: G_y = Gby + gbeta (theta_f + dT0), dT0 = T_ref - T0
  C Gbx, Gby;            // body acceleration
  C nu_over_K;           // nu_f / K
  C inv_sqrtK;           // 1 / sqrt(K)
  C Fphi;                // Forchheimer coefficient, < 0: Ergun (Eq. 7) at the local phi
  C hvf;                 // alpha_f / L^2, so h_v / (rho c_p)_f = H_v hvf
  C inv_sigma;           // (rho c_p)_f / (rho c_p)_s
  C Qf, Qs;              // heat sources (Eq. 45)
  C s_e, s_eps, s_q, s_nu;
  C z_a, z_e, z_nu;      // fluid D2Q5 rates (Eq. 39)
  C e_a, e_e, e_nu;      // solid D2Q5 rates (Eq. 40)
  C varpi;
  C T_ref;
  int wall_kind[4];      // 0 Dirichlet, 1 adiabatic, for walls left, right, bottom, top
  C theta_wall[4];       // Dirichlet wall temperatures relative to T_ref
  C sf, inv_sf;          // storage scale of the shifted D2Q9 populations (1 unless FP16)
  C sg, inv_sg;          // same for the D2Q5 populations
  C theta_init_f, theta_init_s;  // uniform initial temperatures relative to T_ref
  int hv_corr;           // 1: h_v of every node from the correlation of Eq. 52
  C corr_a, corr_b;      // h_v / (rho c_p)_f = corr_a Re^0.644 with Re = corr_b |j| / rho
  C tc;                  // 1 - zeta_alpha / 2 with the correction term of Sec. 3.2, else 0
  ThermalK<double> td;   // temperature-lattice constants, binary64
  ThermalK<float> tf;    // the same, binary32
};

// The temperature-lattice constants in the type T.
template <typename T, typename C>
__host__ __device__ __forceinline__ const ThermalK<T>& thermal_k(const StepConsts<C>& k) {
  if constexpr (std::is_same<T, double>::value) {
    return k.td;
  } else {
    return k.tf;
  }
}

}  // namespace ltne
