// Binary64 reductions over the macroscopic fields: mean wall Nusselt numbers
// and the mass / thermal-energy / residual sums.  Every sum runs in a fixed
// order (per-thread strided partials, a butterfly of cross-lane exchanges
// within each wavefront, the wavefront sums through LDS, then one final
// workgroup over the per-workgroup partials), so repeated calls give
// bit-identical results.
#pragma once

#include "common.hpp"

namespace ltne {

// Number of double sums produced by sums_kernel.
constexpr int kSums = 8;

// Sum of v over the workgroup, in every thread afterwards: a butterfly of
// cross-lane exchanges within each wavefront (lane distances 32, 16, ..., 1;
// lane 0's order is fixed), then the kBlock / 64 wavefront sums of lane 0
// through LDS in a fixed order, so repeated calls give bit-identical results.
constexpr int kWaves = kBlock / 64;
template <int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], double (*lds)[kWaves]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] += __shfl_xor(v[j], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
    for (int j = 0; j < N; ++j) lds[j][wave] = v[j];
  __syncthreads();
  for (int j = 0; j < N; ++j) {
    double t = lds[j][0];
    for (int w = 1; w < kWaves; ++w) t += lds[j][w];
    v[j] = t;
  }
}

// Per-workgroup partial sums over nodes [0, n): mass, energy, and for the
// residual sum|du|, sum|u|, sum|dTf|, sum|Tf|, sum|dTs|, sum|Ts|.
// mac / prev: 5 planes (rho, ux, uy, Tf, Ts) of stride mplane.
template <typename C>
__global__ __launch_bounds__(kBlock) void sums_kernel(const C* __restrict__ mac,
                                                      const C* __restrict__ prev,
                                                      const C* __restrict__ phi_field, double phi_u,
                                                      double sigma, long long n, long long mplane,
                                                      double* __restrict__ partial) {
  __shared__ double lds[kSums][kWaves];
  double v[kSums] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  for (long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
    const double rho = mac[i];
    const double ux = mac[mplane + i], uy = mac[2 * mplane + i];
    const double tf = mac[3 * mplane + i], ts = mac[4 * mplane + i];
    const double ph = phi_field ? static_cast<double>(phi_field[i]) : phi_u;
    v[0] += rho;
    v[1] += ph * tf + (1.0 - ph) * sigma * ts;
    v[2] += fabs(ux - static_cast<double>(prev[mplane + i])) +
            fabs(uy - static_cast<double>(prev[2 * mplane + i]));
    v[3] += fabs(ux) + fabs(uy);
    v[4] += fabs(tf - static_cast<double>(prev[3 * mplane + i]));
    v[5] += fabs(tf);
    v[6] += fabs(ts - static_cast<double>(prev[4 * mplane + i]));
    v[7] += fabs(ts);
  }
  block_reduce<kSums>(v, lds);
  if (threadIdx.x == 0)
    for (int j = 0; j < kSums; ++j) partial[blockIdx.x * kSums + j] = v[j];
}

// Sums nparts partial rows into out[0..kSums) (one workgroup).  Internal
// linkage: every translation unit that launches it has its own copy.
[[maybe_unused]] static __global__ __launch_bounds__(kBlock) void sums_final_kernel(const double* __restrict__ partial,
                                                            int nparts, double* __restrict__ out) {
  __shared__ double lds[kSums][kWaves];
  double v[kSums] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += kBlock)
    for (int j = 0; j < kSums; ++j) v[j] += partial[b * kSums + j];
  block_reduce<kSums>(v, lds);
  if (threadIdx.x == 0)
    for (int j = 0; j < kSums; ++j) out[j] = v[j];
}

// Divergence check of a step: sums the mass and energy partials of
// sums_kernel (one workgroup) and, if either is not finite, records the
// step number in *flag unless an earlier step is already recorded.
[[maybe_unused]] static __global__ __launch_bounds__(kBlock) void finite_check_kernel(const double* __restrict__ partial,
                                                              int nparts,
                                                              unsigned long long* __restrict__ flag,
                                                              unsigned long long step) {
  __shared__ double lds[2][kWaves];
  double v[2] = {0, 0};
  for (int b = threadIdx.x; b < nparts; b += kBlock) {
    v[0] += partial[b * kSums + 0];
    v[1] += partial[b * kSums + 1];
  }
  block_reduce<2>(v, lds);
  if (threadIdx.x == 0 && !(isfinite(v[0]) && isfinite(v[1])) && *flag == 0ull) *flag = step;
}

// Mean Nusselt numbers of T_f and T_s over wall w (one workgroup):
// out[0] = Nu_f, out[1] = Nu_s.
template <typename C>
__global__ __launch_bounds__(kBlock) void nusselt_kernel(const C* __restrict__ mac, int nx, int ny,
                                                         long long mplane, int w, int periodic_t,
                                                         double scale, double* __restrict__ out) {
  __shared__ double lds[3][kWaves];
  const int len = (w < 2) ? ny : nx;
  double v[3] = {0, 0, 0};
  const C* Tf = mac + 3 * mplane;
  const C* Ts = mac + 4 * mplane;
  for (int kk = threadIdx.x; kk < len; kk += kBlock) {
    int i0, i1, i2;
    if (w == 0) { i0 = kk * nx; i1 = i0 + 1; i2 = i0 + 2; }
    else if (w == 1) { i0 = kk * nx + nx - 1; i1 = i0 - 1; i2 = i0 - 2; }
    else if (w == 2) { i0 = kk; i1 = nx + kk; i2 = 2 * nx + kk; }
    else { i0 = (ny - 1) * nx + kk; i1 = i0 - nx; i2 = i0 - 2 * nx; }
    const double wt = (!periodic_t && (kk == 0 || kk == len - 1)) ? 0.5 : 1.0;
    const double qf = -(-3.0 * Tf[i0] + 4.0 * Tf[i1] - static_cast<double>(Tf[i2])) * 0.5;
    const double qs = -(-3.0 * Ts[i0] + 4.0 * Ts[i1] - static_cast<double>(Ts[i2])) * 0.5;
    v[0] += wt * qf;
    v[1] += wt * qs;
    v[2] += wt;
  }
  block_reduce<3>(v, lds);
  if (threadIdx.x == 0) {
    out[0] = scale * v[0] / v[2];
    out[1] = scale * v[1] / v[2];
  }
}

}  // namespace ltne
