// Batched execution: many independent lattices of uneven size and
// parameters advanced together, either by one launch per step over the
// combined tile list (the default), or by one persistent cooperative launch
// that loops over the time steps with a grid-wide barrier between steps.
// On MI355X the barrier's device-scope release and acquire (L2 write-back
// and invalidation on every XCD, once per resident workgroup) cost more than
// a kernel launch per step, so the per-step form is the default.  Every lattice keeps
// its own populations, parameter block and macro buffer; the per-node update
// is the same node_update as the single-lattice kernel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <new>
#include <vector>

#include "host_common.hpp"
#include "lbm_ltne.h"
#include "params.hpp"
#include "reduce_kernels.hpp"
#include "step2_kernel.hpp"
#include "step_kernel.hpp"

namespace ltne {

// Buffers of one lattice as byte offsets into the batch's single allocation,
// whose base the kernels take as an argument: addresses formed from a kernel
// argument are known to be global memory, so the loads and stores use a
// scalar base (pointers read from device memory would be generic and turn
// every access into a flat one with a 64-bit per-lane address).
template <typename C>
struct CavityDesc {
  long long pop[2];  // population buffers (storage type), ping-pong
  long long phi;     // per-node porosity, or -1
  long long hv;      // per-node interphase coefficient, or -1
  long long mac;     // macros of the last step (5 planes of nx*ny)
  int tile_begin;    // first entry of this lattice in the combined tile list
  int wave_begin;    // first entry of this lattice in the two-step wavefront list
  int rows2;         // chunk height of its two-step wavefronts
  int pad_;
};

template <typename T>
__device__ __forceinline__ T* at_offset(char* base, long long off) {
  return off < 0 ? nullptr : reinterpret_cast<T*>(base + off);
}

// Grid barrier state, zeroed by the host before each persistent launch.
struct BatchCtl {
  unsigned count;       // workgroups arrived at the current barrier
  unsigned generation;  // barriers completed
  int error;            // 1: a wait exceeded its spin limit (all workgroups then leave)
  int pad_;
  // work counters of the persistent two-step kernel: pair s of a launch
  // hands out the work items of XCD x from next[s % 2][x]
  unsigned next[2][kXcds];
};
static_assert(sizeof(BatchCtl) <= kAlign, "control block larger than its slot");

template <typename S, typename C, int F>
__device__ __forceinline__ void batch_tile(char* base, int t, const CavityDesc<C>* __restrict__ cav,
                                           const StepConsts<C>* __restrict__ ks,
                                           const int* __restrict__ tile_cav, int parity, bool macros,
                                           uint32_t step) {
  const int c = tile_cav[t];
  const StepConsts<C>& k = ks[c];
  const CavityDesc<C>& d = cav[c];
  const int lt = t - d.tile_begin;
  const int tx = lt % k.tm.ntx;
  const int ty = lt / k.tm.ntx;
  const int tw = 1 << k.tm.tw_shift;
  const int th = kBlock >> k.tm.tw_shift;
  const int x = tx * tw + (static_cast<int>(threadIdx.x) & (tw - 1));
  const int y0 = ty * th * kRows + (static_cast<int>(threadIdx.x) >> k.tm.tw_shift);
  if (x >= k.nx) return;
  const S* src = at_offset<const S>(base, d.pop[parity]);
  S* dst = at_offset<S>(base, d.pop[parity ^ 1]);
  const C* phi = at_offset<const C>(base, d.phi);
  const C* hv = at_offset<const C>(base, d.hv);
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int y = y0 + r * th;
    if (y >= k.ny) continue;
    if (macros)
      node_update<S, C, F | kMacros>(x, y, src, dst, phi, hv, at_offset<C>(base, d.mac), nullptr, nullptr, k,
                                     step);
    else
      node_update<S, C, F>(x, y, src, dst, phi, hv, nullptr, nullptr, nullptr, k, step);
  }
}

// Grid-wide barrier for a co-resident (cooperative) grid.  Every wave waits
// for its own stores; thread 0 of each workgroup releases them device-wide
// (one agent-scope release: the write-back of its XCD's L2) and arrives with
// a relaxed increment.  The last to arrive acquires (so it has seen every
// workgroup's release), releases again and publishes the new generation;
// the others poll the generation with relaxed loads (an acquiring load would
// invalidate the L2 at every poll) and acquire once when it moves on -- at
// most spin_limit polls, after which a waiter raises the error flag and
// reports failure so the whole grid leaves the step loop.
__device__ __forceinline__ bool grid_barrier(BatchCtl* ctl, unsigned nblocks, unsigned& gen,
                                             unsigned spin_limit) {
  __shared__ int ok;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    const unsigned target = gen + 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned arrived = __hip_atomic_fetch_add(&ctl->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
    if (arrived == nblocks) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&ctl->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&ctl->generation, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&ctl->generation, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > spin_limit ||
            __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    gen = target;
  }
  __syncthreads();
  return ok != 0;
}

// nsteps time steps of every lattice, the first numbered step0.  The tile
// list is split into 8 contiguous ranges, one per XCD (workgroup b runs on
// XCD b % 8); the grid has a multiple of 8 workgroups.  With persistent = 0
// the kernel does one step and needs no barrier.
template <typename S, typename C, int F>
__global__ __launch_bounds__(kBlock) void batch_kernel(
    char* base, const CavityDesc<C>* __restrict__ cav, const StepConsts<C>* __restrict__ ks,
    const int* __restrict__ tile_cav, int ntiles, int nsteps, int parity0, int macros_last,
    BatchCtl* ctl, unsigned spin_limit, uint32_t step0) {
  const int xcd = blockIdx.x & (kXcds - 1);
  const int slot = blockIdx.x >> 3;
  const int slots = gridDim.x >> 3;
  const int per = (ntiles + kXcds - 1) / kXcds;
  const int t0 = xcd * per;
  const int t1 = min(ntiles, t0 + per);
  unsigned gen = 0;
  for (int s = 0; s < nsteps; ++s) {
    const int parity = (parity0 + s) & 1;
    const bool macros = macros_last && (s == nsteps - 1);
    for (int t = t0 + slot; t < t1; t += slots)
      batch_tile<S, C, F>(base, t, cav, ks, tile_cav, parity, macros, step0 + static_cast<uint32_t>(s));
    if (s + 1 < nsteps && !grid_barrier(ctl, gridDim.x, gen, spin_limit)) return;
  }
}

// Two steps of every lattice (FP32 form) in one launch: wavefront w runs
// strip and chunk w - wave_begin of lattice wave_cav[w], as the
// single-lattice two-step kernel does; with kMacros in F the second step
// also writes each lattice's macros.
template <int F>
__global__ __launch_bounds__(kBatch2Block) void batch2_kernel(char* base, const CavityDesc<float>* __restrict__ cav,
                                                        const StepConsts<float>* __restrict__ ks,
                                                        const int* __restrict__ wave_cav, int nwaves, int per_xcd,
                                                        int parity, uint32_t step) {
  const int b = blockIdx.x;
  const int blk = (b & (kXcds - 1)) * per_xcd + (b >> 3);
  const int wl = static_cast<int>(threadIdx.x) >> 6;
  const int wave = blk * (kBatch2Block / 64) + wl;
  if (wave >= nwaves) return;  // whole wavefronts
  const int c = __builtin_amdgcn_readfirstlane(wave_cav[wave]);
  const StepConsts<float>& k = ks[c];
  // this wavefront's lattice's binary64 temperature constants in LDS (see
  // step2_kernel), copied by its own lanes into its own slot.  No workgroup
  // barrier: a wavefront's LDS operations execute in order, so its reads see
  // its own writes (and a barrier would make the compiler treat the
  // parameter table as possibly written, loading it into vector registers).
  __shared__ ThermalK<double> kts[kBatch2Block / 64];
  {
    constexpr int words = sizeof(ThermalK<double>) / 8;
    static_assert(sizeof(ThermalK<double>) % 8 == 0 && words <= 64, "constant block too large");
    const int lane = static_cast<int>(threadIdx.x) & 63;
    if (lane < words)
      reinterpret_cast<unsigned long long*>(&kts[wl])[lane] = reinterpret_cast<const unsigned long long*>(&k.td)[lane];
    __builtin_amdgcn_wave_barrier();
  }
  const CavityDesc<float>& d = cav[c];
  const int local = wave - d.wave_begin;
  const int nstrips = (k.nx + step2_out(k.px) - 1) / step2_out(k.px);
  float* mac = (F & kMacros) ? at_offset<float>(base, d.mac) : nullptr;
  step2_wave<F, float>(at_offset<const float>(base, d.pop[parity]), at_offset<float>(base, d.pop[parity ^ 1]),
                at_offset<const float>(base, d.phi), at_offset<const float>(base, d.hv), mac, k,
                kts[wl], local % nstrips, local / nstrips, d.rows2, step);
}

// Threads per workgroup of the persistent two-step kernel: one workgroup of
// eight wavefronts fills a CU at two wavefronts per SIMD, so the grid
// barrier has one participant per CU.
constexpr int kPersistBlock = 512;

// Every pair of steps of every lattice (FP32 form) in one persistent
// cooperative launch, with one grid barrier per pair: the wavefront work
// items of the two-step launches (lattice strips and chunks) are split into
// 8 contiguous ranges, one per XCD, and the wavefronts of that XCD's
// workgroups take the items of its range one at a time from a counter, so
// that they reach the barrier together however the items' lengths differ.
// The parameter table is read through the constant address space, so the
// barriers' fences do not make the compiler reload it into vector
// registers.
template <int F>
__global__ __launch_bounds__(kPersistBlock) void batch2p_kernel(
    char* base, const CavityDesc<float>* __restrict__ cav, const StepConsts<float>* __restrict__ ks_generic,
    const int* __restrict__ wave_cav, int nwaves, int npairs, int parity0, BatchCtl* ctl, unsigned spin_limit,
    uint32_t step0) {
  typedef __attribute__((address_space(4))) const StepConsts<float> ConstK;
  ConstK* ks = (ConstK*)ks_generic;
  const int xcd = blockIdx.x & (kXcds - 1);
  const int slot = blockIdx.x >> 3;
  constexpr int wpb = kPersistBlock / 64;
  const int wl = static_cast<int>(threadIdx.x) >> 6;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int per = (nwaves + kXcds - 1) / kXcds;
  const int w0 = xcd * per;
  const int w1 = min(nwaves, w0 + per);
  __shared__ ThermalK<double> kts[wpb];
  constexpr int words = sizeof(ThermalK<double>) / 8;
  static_assert(sizeof(ThermalK<double>) % 8 == 0 && words <= 64, "constant block too large");
  unsigned gen = 0;
  for (int s = 0; s < npairs; ++s) {
    const int parity = (parity0 + s) & 1;
    unsigned* next = &ctl->next[s & 1][xcd];
    // the counter of the next pair, last used by the pair before this one
    // (finished at the barrier before this pair); the barrier after this
    // pair publishes the reset
    if (slot == 0 && threadIdx.x == 0)
      __hip_atomic_store(&ctl->next[(s + 1) & 1][xcd], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
      unsigned item = 0;
      if (lane == 0) item = __hip_atomic_fetch_add(next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int w = w0 + static_cast<int>(__builtin_amdgcn_readfirstlane(item));
      if (w >= w1) break;
      const int c = __builtin_amdgcn_readfirstlane(wave_cav[w]);
      const StepConsts<float>& k = *(const StepConsts<float>*)&ks[c];
      // this item's lattice constants into the wavefront's own LDS slot (its
      // LDS operations execute in order; see batch2_kernel)
      if (lane < words)
        reinterpret_cast<unsigned long long*>(&kts[wl])[lane] =
            reinterpret_cast<const unsigned long long*>(&k.td)[lane];
      __builtin_amdgcn_wave_barrier();
      const CavityDesc<float>& d = cav[c];
      const int local = w - d.wave_begin;
      const int nstrips = (k.nx + step2_out(k.px) - 1) / step2_out(k.px);
      step2_wave<F, float>(at_offset<const float>(base, d.pop[parity]), at_offset<float>(base, d.pop[parity ^ 1]),
                    at_offset<const float>(base, d.phi), at_offset<const float>(base, d.hv), nullptr, k,
                    kts[wl], local % nstrips, local / nstrips, d.rows2, step0 + 2u * static_cast<uint32_t>(s));
      __builtin_amdgcn_wave_barrier();
    }
    if (s + 1 < npairs && !grid_barrier(ctl, gridDim.x, gen, spin_limit)) return;
  }
}

}  // namespace ltne

using namespace ltne;

struct lbm_ltne_batch {
  int n = 0;
  int precision = LBM_FP32;
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<lbm_ltne_params> p;
  std::vector<lbm_ltne_derived> d;
  std::vector<int> shift;  // tile width shift per lattice
  std::vector<int> rows2;  // chunk height of the two-step launches per lattice
  char* base = nullptr;    // all device memory of the batch
  size_t bytes = 0;
  std::vector<size_t> off_pop0, off_pop1, off_phi, off_hv, off_mac;
  size_t off_cav = 0, off_consts = 0, off_tiles = 0, off_waves = 0, off_ctl = 0, off_result = 0;
  int nwaves2 = 0;    // wavefronts of a two-step launch over every lattice (current chunk heights)
  int nwaves2_min = 0;  // the same at the smallest chunk height (decides whether to use it; table size)
  bool step2_addr = true;  // every lattice's rows addressable by the two-step kernel
  int ntiles = 0;
  int max_tiles = 0;
  int fields = 0;     // kPhiField / kHvField if any lattice has that field
  int parity = 0;     // buffer holding the current state
  int64_t steps = 0;
  int persistent = 0; // 1: cooperative persistent launch, 0: one launch per step (default, faster)
  int grid = 0;       // workgroups of the persistent launch
  int grid2 = 0;      // workgroups of the persistent two-step launch (FP32)
  size_t consts_bytes = 0, desc_bytes = 0;
  long long nodes = 0;

  long long n_of(int i) const { return static_cast<long long>(p[i].nx) * p[i].ny; }
};

namespace {

void batch_release(lbm_ltne_batch* b) {
  if (!b) return;
  if (b->base) (void)hipFree(b->base);
  delete b;
}

template <typename C>
int upload_tables_t(lbm_ltne_batch* b) {
  std::vector<StepConsts<C>> ks(b->n);
  std::vector<CavityDesc<C>> cav(b->n);
  std::vector<int> tile_cav, wave_cav;
  tile_cav.reserve(b->max_tiles);
  wave_cav.reserve(b->nwaves2_min);
  for (int i = 0; i < b->n; ++i) {
    fill_step_consts(b->p[i], b->d[i], &ks[i]);
    ks[i].tm = make_tiles(b->p[i].nx, b->p[i].ny, b->precision, b->shift[i]);
    cav[i].pop[0] = static_cast<long long>(b->off_pop0[i]);
    cav[i].pop[1] = static_cast<long long>(b->off_pop1[i]);
    cav[i].phi = b->off_phi[i] ? static_cast<long long>(b->off_phi[i]) : -1;
    cav[i].hv = b->off_hv[i] ? static_cast<long long>(b->off_hv[i]) : -1;
    cav[i].mac = static_cast<long long>(b->off_mac[i]);
    cav[i].tile_begin = static_cast<int>(tile_cav.size());
    for (int t = 0; t < ks[i].tm.ntiles; ++t) tile_cav.push_back(i);
    cav[i].wave_begin = static_cast<int>(wave_cav.size());
    cav[i].rows2 = b->rows2[i];
    cav[i].pad_ = 0;
    for (int w = 0; w < step2_waves(b->p[i].nx, b->p[i].ny, b->p[i].periodic_x, b->rows2[i]); ++w)
      wave_cav.push_back(i);
  }
  b->nwaves2 = static_cast<int>(wave_cav.size());
  b->ntiles = static_cast<int>(tile_cav.size());
  HIP_TRY(hipMemcpyAsync(b->base + b->off_consts, ks.data(), ks.size() * sizeof(ks[0]),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->base + b->off_cav, cav.data(), cav.size() * sizeof(cav[0]),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->base + b->off_tiles, tile_cav.data(), tile_cav.size() * sizeof(int),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->base + b->off_waves, wave_cav.data(), wave_cav.size() * sizeof(int),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int upload_tables(lbm_ltne_batch* b) {
  return compute_bytes(b->precision) == 8 ? upload_tables_t<double>(b) : upload_tables_t<float>(b);
}

template <typename S, typename C, int F>
const void* batch_fn() {
  return reinterpret_cast<const void*>(&batch_kernel<S, C, F>);
}

template <typename S, typename C>
const void* pick_fn(int fields) {
  switch (fields) {
    case kPhiField: return batch_fn<S, C, kPhiField>();
    case kHvField: return batch_fn<S, C, kHvField>();
    case kPhiField | kHvField: return batch_fn<S, C, kPhiField | kHvField>();
    default: return batch_fn<S, C, 0>();
  }
}

const void* batch_function(const lbm_ltne_batch* b) {
  if (b->precision == LBM_FP64) return pick_fn<double, double>(b->fields);
  if (b->precision == LBM_FP32) return pick_fn<float, float>(b->fields);
  if (b->precision == LBM_FP32SR) return pick_fn<float, double>(b->fields);
  return pick_fn<_Float16, float>(b->fields);
}

const void* batch2p_function(const lbm_ltne_batch* b) {
  switch (b->fields) {
    case kPhiField: return reinterpret_cast<const void*>(&batch2p_kernel<kPhiField>);
    case kHvField: return reinterpret_cast<const void*>(&batch2p_kernel<kHvField>);
    case kPhiField | kHvField: return reinterpret_cast<const void*>(&batch2p_kernel<kPhiField | kHvField>);
    default: return reinterpret_cast<const void*>(&batch2p_kernel<0>);
  }
}

// Workgroups that can be resident at once (multiple of 8), for the
// cooperative launch.
int resident_grid(const lbm_ltne_batch* b, int* out, const void* fn = nullptr, int block = kBlock) {
  int per_cu = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn ? fn : batch_function(b), block, 0));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, b->device));
  int g = per_cu * prop.multiProcessorCount;
  g -= g % kXcds;
  *out = g;
  return LBM_OK;
}

constexpr unsigned kSpinLimit = 1u << 24;

template <int F>
void launch_batch2_f(const lbm_ltne_batch* b, int parity, uint32_t step, bool macros) {
  const CavityDesc<float>* cav = reinterpret_cast<const CavityDesc<float>*>(b->base + b->off_cav);
  const StepConsts<float>* ks = reinterpret_cast<const StepConsts<float>*>(b->base + b->off_consts);
  const int* waves = reinterpret_cast<const int*>(b->base + b->off_waves);
  const int nblocks = (b->nwaves2 + kBatch2Block / 64 - 1) / (kBatch2Block / 64);
  const int per_xcd = (nblocks + kXcds - 1) / kXcds;
  const dim3 grid(kXcds * per_xcd), block(kBatch2Block);
  if (macros)
    hipLaunchKernelGGL(batch2_kernel<F | kMacros>, grid, block, 0, b->stream, b->base, cav, ks, waves, b->nwaves2,
                       per_xcd, parity, step);
  else
    hipLaunchKernelGGL(batch2_kernel<F>, grid, block, 0, b->stream, b->base, cav, ks, waves, b->nwaves2, per_xcd,
                       parity, step);
}

// A two-step launch over every lattice; macros: the second step also writes
// the macros.
hipError_t launch_batch2(const lbm_ltne_batch* b, int parity, uint32_t step, bool macros = false) {
  switch (b->fields) {
    case kPhiField: launch_batch2_f<kPhiField>(b, parity, step, macros); break;
    case kHvField: launch_batch2_f<kHvField>(b, parity, step, macros); break;
    case kPhiField | kHvField: launch_batch2_f<kPhiField | kHvField>(b, parity, step, macros); break;
    default: launch_batch2_f<0>(b, parity, step, macros);
  }
  return hipGetLastError();
}

// FP32 batches with enough wavefronts at the smallest chunk height, whose
// rows the two-step kernel can address, run pairs of steps per launch.
bool two_step_ok(const lbm_ltne_batch* b) {
  return b->precision == LBM_FP32 && b->step2_addr && b->nwaves2_min >= LTNE_STEP2_MIN_WAVES;
}

// nsteps steps of every lattice.  Per-step mode: the FP32 form runs pairs
// of steps in one two-step launch (two_step, and enough wavefronts), an odd
// last step alone; the last launch writes the macros (macros_last).  The
// autotuner's tile trials run single steps only (the tile widths it chooses
// apply to them).
int launch_batch(lbm_ltne_batch* b, int nsteps, int macros_last, bool two_step = true) {
  const void* fn = batch_function(b);
  char* base = b->base;
  const void* cav = b->base + b->off_cav;
  const void* ks = b->base + b->off_consts;
  const void* tiles = b->base + b->off_tiles;
  BatchCtl* ctl = reinterpret_cast<BatchCtl*>(b->base + b->off_ctl);
  int ntiles = b->ntiles;
  unsigned spin = kSpinLimit;
  const bool two_ok = two_step && two_step_ok(b);
  if (b->persistent && two_ok) {
    // the pairs of steps in one persistent launch, then the remaining single
    // step (the one that writes the macros) as an ordinary launch
    int npairs = (nsteps - (macros_last ? 1 : 0)) / 2;
    int parity = b->parity;
    if (npairs > 0) {
      HIP_TRY(hipMemsetAsync(ctl, 0, sizeof(BatchCtl), b->stream));
      const void* waves = b->base + b->off_waves;
      int nw = b->nwaves2;
      uint32_t step0 = static_cast<uint32_t>(b->steps + 1);
      void* args[] = {&base, &cav, &ks, &waves, &nw, &npairs, &parity, &ctl, &spin, &step0};
      HIP_TRY(hipLaunchCooperativeKernel(batch2p_function(b), dim3(b->grid2), dim3(kPersistBlock), args, 0,
                                         b->stream));
      parity = (parity + npairs) & 1;
    }
    const int per = (ntiles + kXcds - 1) / kXcds;
    for (int s = 2 * npairs; s < nsteps; ++s) {
      int one = 1;
      int mac = (macros_last && s == nsteps - 1) ? 1 : 0;
      uint32_t st = static_cast<uint32_t>(b->steps + 1 + s);
      void* args[] = {&base, &cav, &ks, &tiles, &ntiles, &one, &parity, &mac, &ctl, &spin, &st};
      HIP_TRY(hipLaunchKernel(fn, dim3(kXcds * per), dim3(kBlock), args, 0, b->stream));
      parity ^= 1;
    }
    b->parity = parity;
  } else if (b->persistent) {
    HIP_TRY(hipMemsetAsync(ctl, 0, sizeof(BatchCtl), b->stream));
    int parity = b->parity;
    uint32_t step0 = static_cast<uint32_t>(b->steps + 1);
    void* args[] = {&base, &cav, &ks, &tiles, &ntiles, &nsteps, &parity, &macros_last, &ctl, &spin, &step0};
    HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(b->grid), dim3(kBlock), args, 0, b->stream));
    b->parity = (b->parity + nsteps) & 1;
  } else {
    const int per = (ntiles + kXcds - 1) / kXcds;
    const int grid = kXcds * per;  // one tile per workgroup per step
    const bool two = two_ok;
    int parity = b->parity;
    for (int s = 0; s < nsteps;) {
      const uint32_t step0 = static_cast<uint32_t>(b->steps + 1 + s);
      if (two && s + 2 <= nsteps) {
        // the pair that ends the call writes the macros of its second step
        HIP_TRY(launch_batch2(b, parity, step0, macros_last && s + 2 == nsteps));
        s += 2;
      } else {
        int one = 1;
        int mac = (macros_last && s == nsteps - 1) ? 1 : 0;
        uint32_t st = step0;
        void* args[] = {&base, &cav, &ks, &tiles, &ntiles, &one, &parity, &mac, &ctl, &spin, &st};
        HIP_TRY(hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, 0, b->stream));
        s += 1;
      }
      parity ^= 1;
    }
    b->parity = parity;
  }
  return LBM_OK;
}

int check_ctl(lbm_ltne_batch* b) {
  BatchCtl c;
  HIP_TRY(hipMemcpyAsync(&c, b->base + b->off_ctl, sizeof(c), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (c.error) return set_error(LBM_EHIP, "a grid barrier of the persistent batch launch timed out");
  return LBM_OK;
}

template <typename S, typename C>
hipError_t init_one(const lbm_ltne_batch* b, int i) {
  StepConsts<C> k;
  fill_step_consts(b->p[i], b->d[i], &k);
  k.tm = make_tiles(b->p[i].nx, b->p[i].ny, b->precision, b->shift[i]);
  const C* phi = b->off_phi[i] ? reinterpret_cast<const C*>(b->base + b->off_phi[i]) : nullptr;
  const C* hv = b->off_hv[i] ? reinterpret_cast<const C*>(b->base + b->off_hv[i]) : nullptr;
  S* dst = reinterpret_cast<S*>(b->base + b->off_pop0[i]);
  C* mac = reinterpret_cast<C*>(b->base + b->off_mac[i]);
  const dim3 grid(grid_blocks(k.tm)), block(kBlock);
  const int fl = (phi ? kPhiField : 0) | (hv ? kHvField : 0);
  switch (fl) {
    case 0:
      hipLaunchKernelGGL((step_kernel<S, C, kMacros | kInit>), grid, block, 0, b->stream, nullptr,
                         dst, phi, hv, mac, nullptr, nullptr, k, 0u);
      break;
    case kPhiField:
      hipLaunchKernelGGL((step_kernel<S, C, kPhiField | kMacros | kInit>), grid, block, 0, b->stream,
                         nullptr, dst, phi, hv, mac, nullptr, nullptr, k, 0u);
      break;
    case kHvField:
      hipLaunchKernelGGL((step_kernel<S, C, kHvField | kMacros | kInit>), grid, block, 0, b->stream,
                         nullptr, dst, phi, hv, mac, nullptr, nullptr, k, 0u);
      break;
    default:
      hipLaunchKernelGGL((step_kernel<S, C, kPhiField | kHvField | kMacros | kInit>), grid, block, 0,
                         b->stream, nullptr, dst, phi, hv, mac, nullptr, nullptr, k, 0u);
  }
  return hipGetLastError();
}

hipError_t init_lattice(const lbm_ltne_batch* b, int i) {
  if (b->precision == LBM_FP64) return init_one<double, double>(b, i);
  if (b->precision == LBM_FP32) return init_one<float, float>(b, i);
  if (b->precision == LBM_FP32SR) return init_one<float, double>(b, i);
  return init_one<_Float16, float>(b, i);
}

int upload_batch_field(const lbm_ltne_batch* b, const double* src, size_t off, long long n) {
  if (compute_bytes(b->precision) == 8) {
    HIP_TRY(hipMemcpyAsync(b->base + off, src, n * sizeof(double), hipMemcpyHostToDevice, b->stream));
  } else {
    std::vector<float> tmp(n);
    for (long long j = 0; j < n; ++j) tmp[j] = static_cast<float>(src[j]);
    HIP_TRY(hipMemcpyAsync(b->base + off, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_ltne_batch_create(int32_t n, const lbm_ltne_params* ps, const double* const* phi_fields,
                          const double* const* Hv_fields, void* hip_stream, lbm_ltne_batch_t* out) {
  clear_error();
  if (!out) return set_error(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (n <= 0 || !ps) return set_error(LBM_EINVAL, "need n > 0 parameter sets");
  const int precision = ps[0].precision;
  std::vector<lbm_ltne_derived> ds(n);
  for (int i = 0; i < n; ++i) {
    if (ps[i].precision != precision)
      return set_error(LBM_EINVAL, "lattice %d: all lattices of a batch share one precision", i);
    double lo, hi;
    temperature_range(&ps[i], &lo, &hi);
    const int rc = derive(&ps[i], lo, hi, &ds[i]);
    if (rc != LBM_OK) {
      std::string msg = last_error();
      return set_error(rc, "lattice %d: %s", i, msg.c_str());
    }
    if (ps[i].diag_every != 0)
      return set_error(LBM_EUNSUPPORTED, "lattice %d: diag_every is for single lattices only", i);
    const long long nn = static_cast<long long>(ps[i].nx) * ps[i].ny;
    if (phi_fields && phi_fields[i])
      for (long long j = 0; j < nn; ++j)
        if (!(phi_fields[i][j] > 0.0 && phi_fields[i][j] < 1.0))
          return set_error(LBM_EINVAL, "lattice %d: phi_field[%lld] not in (0, 1)", i, j);
    if (Hv_fields && Hv_fields[i] && ps[i].pore_size > 0.0)
      return set_error(LBM_EINVAL, "lattice %d: an H_v field and the correlation of Eq. 52 exclude each other", i);
    if (Hv_fields && Hv_fields[i])
      for (long long j = 0; j < nn; ++j)
        if (!(Hv_fields[i][j] >= 0.0) || !std::isfinite(Hv_fields[i][j]))
          return set_error(LBM_EINVAL, "lattice %d: Hv_field[%lld] must be finite and >= 0", i, j);
  }
  int dev = 0;
  int rc = check_device(&dev);
  if (rc != LBM_OK) return rc;
  lbm_ltne_batch* b = new (std::nothrow) lbm_ltne_batch();
  if (!b) return set_error(LBM_ENOMEM, "host allocation failed");
  b->n = n;
  b->precision = precision;
  b->device = dev;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->p.assign(ps, ps + n);
  b->d = ds;
  b->shift.assign(n, 0);
  b->rows2.assign(n, kBatch2Rows);
  for (int i = 0; i < n; ++i) {
    if (phi_fields && phi_fields[i]) b->fields |= kPhiField;
    if (Hv_fields && Hv_fields[i]) b->fields |= kHvField;
  }
  // Layout: per lattice two population buffers, fields, macros; then the
  // tables.  A lattice without a field gets the uniform value materialised
  // when another lattice of the batch has one (one kernel variant per batch).
  size_t o = 0;
  b->off_pop0.resize(n);
  b->off_pop1.resize(n);
  b->off_phi.assign(n, 0);
  b->off_hv.assign(n, 0);
  b->off_mac.resize(n);
  const size_t sb = storage_bytes(precision), cb = compute_bytes(precision);
  for (int i = 0; i < n; ++i) {
    const long long nn = b->n_of(i);
    const size_t popb = align_up(pop_elems(ps[i].nx, ps[i].ny) * sb, kAlign);
    b->off_pop0[i] = o; o += popb;
    b->off_pop1[i] = o; o += popb;
    if (b->fields & kPhiField) { b->off_phi[i] = o; o += align_up(nn * cb, kAlign); }
    if (b->fields & kHvField) { b->off_hv[i] = o; o += align_up(nn * cb, kAlign); }
    b->off_mac[i] = o; o += align_up(5 * nn * cb, kAlign);
    b->nodes += nn;
    int most = 0;  // the tile table must hold the tiles of any width choice
    for (int sh = 6; sh <= 8; ++sh) most = std::max(most, make_tiles(ps[i].nx, ps[i].ny, precision, sh).ntiles);
    b->max_tiles += most;
    b->nwaves2_min += step2_waves(ps[i].nx, ps[i].ny, ps[i].periodic_x, kStep2MinRows);
    b->step2_addr = b->step2_addr && step2_addressable(ps[i].nx, sizeof(float));
  }
  const bool cdouble = compute_bytes(precision) == 8;
  b->consts_bytes = (cdouble ? sizeof(StepConsts<double>) : sizeof(StepConsts<float>));
  b->desc_bytes = (cdouble ? sizeof(CavityDesc<double>) : sizeof(CavityDesc<float>));
  b->off_consts = o; o += align_up(n * b->consts_bytes, kAlign);
  b->off_cav = o; o += align_up(n * b->desc_bytes, kAlign);
  b->off_tiles = o; o += align_up(static_cast<size_t>(b->max_tiles) * sizeof(int), kAlign);
  b->off_waves = o; o += align_up(static_cast<size_t>(b->nwaves2_min) * sizeof(int), kAlign);
  b->off_ctl = o; o += kAlign;
  b->off_result = o; o += kAlign;
  b->bytes = o;
  if (hipMalloc(&b->base, b->bytes) != hipSuccess) {
    (void)hipGetLastError();
    const size_t want = b->bytes;
    b->base = nullptr;
    batch_release(b);
    return set_error(LBM_ENOMEM, "hipMalloc of %zu bytes failed", want);
  }
  rc = LBM_OK;
  for (int i = 0; i < n && rc == LBM_OK; ++i) {
    const long long nn = b->n_of(i);
    std::vector<double> fill;
    if (b->fields & kPhiField) {
      const double* src = (phi_fields && phi_fields[i]) ? phi_fields[i] : nullptr;
      if (!src) { fill.assign(nn, ps[i].phi); src = fill.data(); }
      rc = upload_batch_field(b, src, b->off_phi[i], nn);
    }
    if (rc == LBM_OK && (b->fields & kHvField)) {
      const double* src = (Hv_fields && Hv_fields[i]) ? Hv_fields[i] : nullptr;
      if (!src) { fill.assign(nn, ps[i].Hv); src = fill.data(); }
      rc = upload_batch_field(b, src, b->off_hv[i], nn);
    }
    if (rc == LBM_OK) {
      hipError_t e = init_lattice(b, i);
      if (e != hipSuccess) rc = set_error(LBM_EHIP, "initialisation of lattice %d: %s", i, hipGetErrorString(e));
    }
  }
  if (rc == LBM_OK) rc = upload_tables(b);
  if (rc == LBM_OK) rc = resident_grid(b, &b->grid);
  if (rc == LBM_OK && precision == LBM_FP32) rc = resident_grid(b, &b->grid2, batch2p_function(b), kPersistBlock);

  if (rc == LBM_OK) {
    hipError_t e = hipMemsetAsync(b->base + b->off_ctl, 0, sizeof(BatchCtl), b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) rc = set_error(LBM_EHIP, "batch setup: %s", hipGetErrorString(e));
  }
  if (rc != LBM_OK) {
    batch_release(b);
    return rc;
  }
  *out = b;
  return LBM_OK;
}

int lbm_ltne_batch_step(lbm_ltne_batch_t b, int64_t nsteps) {
  if (!b) return set_error(LBM_EINVAL, "batch is NULL");
  if (nsteps < 0) return set_error(LBM_EINVAL, "nsteps < 0");
  if (nsteps == 0) return LBM_OK;
  // one persistent launch covers up to 2^20 steps; longer runs are split
  int64_t left = nsteps;
  while (left > 0) {
    const int chunk = static_cast<int>(std::min<int64_t>(left, 1 << 20));
    const int rc = launch_batch(b, chunk, left == chunk ? 1 : 0);
    if (rc != LBM_OK) return rc;
    left -= chunk;
  }
  b->steps += nsteps;
  return LBM_OK;
}

int lbm_ltne_batch_set_mode(lbm_ltne_batch_t b, int32_t persistent) {
  if (!b) return set_error(LBM_EINVAL, "batch is NULL");
  if (persistent && (b->grid < kXcds || (b->precision == LBM_FP32 && b->grid2 < kXcds)))
    return set_error(LBM_EUNSUPPORTED, "no resident grid for a persistent launch");
  b->persistent = persistent ? 1 : 0;
  return LBM_OK;
}

int lbm_ltne_batch_info(lbm_ltne_batch_t b, int64_t* nodes, int32_t* tiles, int32_t* grid,
                        int32_t* persistent) {
  if (!b) return set_error(LBM_EINVAL, "batch is NULL");
  if (nodes) *nodes = b->nodes;
  if (tiles) *tiles = b->ntiles;
  if (grid) *grid = two_step_ok(b) ? b->grid2 : b->grid;
  if (persistent) *persistent = b->persistent;
  return LBM_OK;
}

int lbm_ltne_batch_set_tiles(lbm_ltne_batch_t b, const int32_t* tile_shift) {
  if (!b || !tile_shift) return set_error(LBM_EINVAL, "batch or shifts NULL");
  for (int i = 0; i < b->n; ++i)
    if (tile_shift[i] != 0 && (tile_shift[i] < 6 || tile_shift[i] > 8))
      return set_error(LBM_EINVAL, "tile shift %d of lattice %d not in {0, 6, 7, 8}", tile_shift[i], i);
  for (int i = 0; i < b->n; ++i) b->shift[i] = tile_shift[i];
  return upload_tables(b);
}

int lbm_ltne_batch_get_tiles(lbm_ltne_batch_t b, int32_t* tile_shift) {
  if (!b || !tile_shift) return set_error(LBM_EINVAL, "batch or shifts NULL");
  for (int i = 0; i < b->n; ++i)
    tile_shift[i] = make_tiles(b->p[i].nx, b->p[i].ny, b->precision, b->shift[i]).tw_shift;
  return LBM_OK;
}

int lbm_ltne_batch_set_chunks(lbm_ltne_batch_t b, const int32_t* rows) {
  if (!b || !rows) return set_error(LBM_EINVAL, "batch or chunk heights NULL");
  for (int i = 0; i < b->n; ++i) {
    bool ok = rows[i] == 0;
    for (int r : kBatch2RowChoices) ok = ok || rows[i] == r;
    if (!ok) return set_error(LBM_EINVAL, "chunk height %d of lattice %d not in {0, 8, 12, 16, 24, 32}", rows[i], i);
  }
  for (int i = 0; i < b->n; ++i) b->rows2[i] = rows[i] ? rows[i] : kBatch2Rows;
  return upload_tables(b);
}

int lbm_ltne_batch_get_chunks(lbm_ltne_batch_t b, int32_t* rows) {
  if (!b || !rows) return set_error(LBM_EINVAL, "batch or chunk heights NULL");
  for (int i = 0; i < b->n; ++i) rows[i] = b->rows2[i];
  return LBM_OK;
}

int lbm_ltne_batch_autotune(lbm_ltne_batch_t b, int32_t reps, double* ms_per_step) {
  if (!b) return set_error(LBM_EINVAL, "batch is NULL");
  if (reps <= 0) reps = 4;
  // Snapshot the state: trial steps must not advance the simulation.
  size_t pop_total = 0;
  for (int i = 0; i < b->n; ++i) pop_total += b->off_pop1[i] - b->off_pop0[i];
  char* snap = nullptr;
  if (hipMalloc(&snap, pop_total) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(LBM_ENOMEM, "autotune snapshot of %zu bytes failed", pop_total);
  }
  auto copy_state = [&](bool save) -> int {
    size_t o = 0;
    for (int i = 0; i < b->n; ++i) {
      const size_t sz = b->off_pop1[i] - b->off_pop0[i];
      char* cur = b->base + (b->parity ? b->off_pop1[i] : b->off_pop0[i]);
      HIP_TRY(hipMemcpyAsync(save ? snap + o : cur, save ? cur : snap + o, sz, hipMemcpyDeviceToDevice,
                             b->stream));
      o += sz;
    }
    return LBM_OK;
  };
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipFree(snap);
    return set_error(LBM_EHIP, "event creation failed");
  }
  const int parity0 = b->parity;
  auto trial = [&](float* ms) -> int {
    int rc = copy_state(false);
    if (rc != LBM_OK) return rc;
    b->parity = parity0;
    rc = launch_batch(b, 1, 0, false);  // warm-up
    if (rc != LBM_OK) return rc;
    HIP_TRY(hipEventRecord(e0, b->stream));
    rc = launch_batch(b, reps, 0, false);
    if (rc != LBM_OK) return rc;
    HIP_TRY(hipEventRecord(e1, b->stream));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    rc = check_ctl(b);
    *ms /= static_cast<float>(reps);
    b->parity = parity0;
    return rc;
  };
  int rc = copy_state(true);
  if (rc == LBM_OK) rc = (hipStreamSynchronize(b->stream) == hipSuccess) ? LBM_OK : LBM_EHIP;
  // Coordinate descent over the size classes (lattices of equal width share
  // a choice), starting from the defaults.
  std::map<int, std::vector<int>> classes;
  for (int i = 0; i < b->n; ++i) classes[b->p[i].nx].push_back(i);
  float best = 0.0f;
  if (rc == LBM_OK) rc = upload_tables(b);
  if (rc == LBM_OK) rc = trial(&best);
  for (auto& kv : classes) {
    if (rc != LBM_OK) break;
    const int nx = kv.first;
    const int keep = b->shift[kv.second[0]];
    int best_shift = keep;
    for (int sh = 6; sh <= 8; ++sh) {
      if ((1 << sh) > std::max(64, nx)) break;
      for (int i : kv.second) b->shift[i] = sh;
      rc = upload_tables(b);
      float ms = 0.0f;
      if (rc == LBM_OK) rc = trial(&ms);
      if (rc != LBM_OK) break;
      if (ms < best) {
        best = ms;
        best_shift = sh;
      }
    }
    for (int i : kv.second) b->shift[i] = best_shift;
  }
  // The chunk heights of the two-step launches (FP32 form), timed on the
  // path that runs: pairs of steps per launch over every lattice.
  const bool two = two_step_ok(b);
  if (two && rc == LBM_OK) {
    auto trial2 = [&](float* ms) -> int {
      int r = copy_state(false);
      if (r != LBM_OK) return r;
      b->parity = parity0;
      r = launch_batch(b, 2, 0, true);  // warm-up
      if (r != LBM_OK) return r;
      HIP_TRY(hipEventRecord(e0, b->stream));
      r = launch_batch(b, 2 * reps, 0, true);
      if (r != LBM_OK) return r;
      HIP_TRY(hipEventRecord(e1, b->stream));
      HIP_TRY(hipEventSynchronize(e1));
      HIP_TRY(hipEventElapsedTime(ms, e0, e1));
      *ms /= static_cast<float>(2 * reps);
      b->parity = parity0;
      return LBM_OK;
    };
    rc = upload_tables(b);
    if (rc == LBM_OK) rc = trial2(&best);
    for (auto& kv : classes) {
      if (rc != LBM_OK) break;
      int best_rows = b->rows2[kv.second[0]];
      for (int r : kBatch2RowChoices) {
        if (r == best_rows) continue;
        for (int i : kv.second) b->rows2[i] = r;
        rc = upload_tables(b);
        float ms = 0.0f;
        if (rc == LBM_OK) rc = trial2(&ms);
        if (rc != LBM_OK) break;
        if (ms < best) {
          best = ms;
          best_rows = r;
        }
      }
      for (int i : kv.second) b->rows2[i] = best_rows;
    }
  }
  if (rc == LBM_OK) rc = upload_tables(b);
  // The launch mode, with the shapes chosen: both modes timed over 2 reps
  // steps of the path each runs (pairs of steps where they apply), from the
  // snapshot; the faster is kept.  Persistent launches pay off where
  // launches are a large part of a step (small batches).
  const bool can_persist = b->grid >= kXcds && !(b->precision == LBM_FP32 && b->grid2 < kXcds);
  if (rc == LBM_OK && can_persist) {
    const int mode0 = b->persistent;
    float ms_mode[2] = {0.0f, 0.0f};
    for (int m = 0; m < 2 && rc == LBM_OK; ++m) {
      b->persistent = m;
      rc = copy_state(false);
      b->parity = parity0;
      if (rc == LBM_OK) rc = launch_batch(b, 2, 0, true);  // warm-up
      if (rc == LBM_OK && hipEventRecord(e0, b->stream) != hipSuccess) rc = set_error(LBM_EHIP, "event record");
      if (rc == LBM_OK) rc = launch_batch(b, 2 * reps, 0, true);
      if (rc == LBM_OK && hipEventRecord(e1, b->stream) != hipSuccess) rc = set_error(LBM_EHIP, "event record");
      if (rc == LBM_OK && hipEventSynchronize(e1) != hipSuccess) rc = set_error(LBM_EHIP, "event sync");
      if (rc == LBM_OK && hipEventElapsedTime(&ms_mode[m], e0, e1) != hipSuccess)
        rc = set_error(LBM_EHIP, "event time");
      if (rc == LBM_OK) rc = check_ctl(b);
      ms_mode[m] /= static_cast<float>(2 * reps);
    }
    b->parity = parity0;
    if (rc == LBM_OK) {
      b->persistent = ms_mode[1] < ms_mode[0] ? 1 : 0;
      best = ms_mode[b->persistent];
    } else {
      b->persistent = mode0;
    }
  }
  const int rc2 = copy_state(false);
  if (rc == LBM_OK) rc = rc2;
  if (hipStreamSynchronize(b->stream) != hipSuccess && rc == LBM_OK) rc = set_error(LBM_EHIP, "autotune sync");
  b->parity = parity0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(snap);
  if (ms_per_step) *ms_per_step = best;
  return rc;
}

int lbm_ltne_batch_macros(lbm_ltne_batch_t b, int32_t i, double* rho, double* ux, double* uy,
                          double* Tf, double* Ts) {
  if (!b) return set_error(LBM_EINVAL, "batch is NULL");
  if (i < 0 || i >= b->n) return set_error(LBM_EINVAL, "lattice index %d out of range", i);
  int rc = check_ctl(b);
  if (rc != LBM_OK) return rc;
  const long long n = b->n_of(i);
  const size_t cb = compute_bytes(b->precision);
  double* outs[5] = {rho, ux, uy, Tf, Ts};
  std::vector<float> tmp;
  for (int f = 0; f < 5; ++f) {
    if (!outs[f]) continue;
    const char* src = b->base + b->off_mac[i] + static_cast<size_t>(f) * n * cb;
    if (cb == 8) {
      HIP_TRY(hipMemcpyAsync(outs[f], src, n * 8, hipMemcpyDeviceToHost, b->stream));
      HIP_TRY(hipStreamSynchronize(b->stream));
    } else {
      tmp.resize(n);
      HIP_TRY(hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, b->stream));
      HIP_TRY(hipStreamSynchronize(b->stream));
      for (long long j = 0; j < n; ++j) outs[f][j] = tmp[j];
    }
  }
  return LBM_OK;
}

int lbm_ltne_batch_nusselt(lbm_ltne_batch_t b, int32_t i, double* Nu_f, double* Nu_s) {
  if (!b) return set_error(LBM_EINVAL, "batch is NULL");
  if (i < 0 || i >= b->n) return set_error(LBM_EINVAL, "lattice index %d out of range", i);
  int rc = check_ctl(b);
  if (rc != LBM_OK) return rc;
  const lbm_ltne_params& p = b->p[i];
  const int w = hot_wall(&p);
  if (w < 0) return set_error(LBM_EINVAL, "lattice %d has no wall for the Nusselt number", i);
  const int periodic_t = (w < 2) ? p.periodic_y : p.periodic_x;
  const double scale = b->d[i].L / b->d[i].dT;
  double* res = reinterpret_cast<double*>(b->base + b->off_result);
  const long long n = b->n_of(i);
  if (compute_bytes(b->precision) == 8)
    hipLaunchKernelGGL((nusselt_kernel<double>), dim3(1), dim3(kBlock), 0, b->stream,
                       reinterpret_cast<const double*>(b->base + b->off_mac[i]), p.nx, p.ny, n, w,
                       periodic_t, scale, res);
  else
    hipLaunchKernelGGL((nusselt_kernel<float>), dim3(1), dim3(kBlock), 0, b->stream,
                       reinterpret_cast<const float*>(b->base + b->off_mac[i]), p.nx, p.ny, n, w,
                       periodic_t, scale, res);
  HIP_TRY(hipGetLastError());
  double r[2];
  HIP_TRY(hipMemcpyAsync(r, res, sizeof(r), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (Nu_f) *Nu_f = r[0];
  if (Nu_s) *Nu_s = r[1];
  return LBM_OK;
}

int64_t lbm_ltne_batch_steps_done(lbm_ltne_batch_t b) { return b ? b->steps : -1; }

int lbm_ltne_batch_destroy(lbm_ltne_batch_t b) {
  if (!b) return LBM_OK;
  (void)hipStreamSynchronize(b->stream);
  batch_release(b);
  return LBM_OK;
}

}  // extern "C"
