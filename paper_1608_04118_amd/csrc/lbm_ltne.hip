// Host runtime and C ABI of the LTNE MRT lattice Boltzmann library: device
// memory layout, launch configuration, time stepping, outputs, checkpoints.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "lbm_ltne.h"
#include "host_common.hpp"
#include "params.hpp"
#include "reduce_kernels.hpp"
#include "adjoint_kernel.hpp"
#include "step_kernel.hpp"
#include "step2_kernel.hpp"

using namespace ltne;

struct lbm_ltne {
  lbm_ltne_params p;
  lbm_ltne_derived d;
  int device = 0;
  hipStream_t stream = nullptr;
  char* base = nullptr;
  bool owns = false;
  Layout lay{};
  bool has_phi = false, has_hv = false;
  int cur = 0;   // population buffer holding the current state
  int mcur = 0;  // macro buffer of the current time
  int64_t steps = 0;
  StepConsts<double> kd{};
  StepConsts<float> kf{};
  std::vector<double> tf0, ts0;  // initial temperature fields (if given), for the adjoint
  hipGraphExec_t seq[2] = {nullptr, nullptr};  // recorded runs of kSeqSteps steps from buffer 0 / 1

  void* pop(int i) const { return base + lay.off_pop[i]; }
  void* mac(int i) const { return base + lay.off_mac[i]; }
  void* phi() const { return has_phi ? base + lay.off_phi : nullptr; }
  void* hv() const { return has_hv ? base + lay.off_hv : nullptr; }
  double* partial() const { return reinterpret_cast<double*>(base + lay.off_partial); }
  double* result() const { return reinterpret_cast<double*>(base + lay.off_result); }
  // step number of the first checked step with non-finite sums (0: none),
  // in the result block after the sums
  unsigned long long* diverged() const {
    return reinterpret_cast<unsigned long long*>(base + lay.off_result + 16 * sizeof(double));
  }
  // step number of the next step of a recorded run (see step_seq_kernel)
  uint32_t* step_base() const { return reinterpret_cast<uint32_t*>(base + lay.off_result + 24 * sizeof(double)); }
  long long n() const { return static_cast<long long>(p.nx) * p.ny; }
};

namespace {

template <typename C>
void fill_consts(const lbm_ltne* h, StepConsts<C>* k) {
  fill_step_consts(h->p, h->d, k);
}

template <typename S, typename C, int F>
hipError_t launch_one(const lbm_ltne* h, const StepConsts<C>& k, uint32_t step, const void* src, void* dst,
                      void* mac, const void* init_tf, const void* init_ts, void* rec = nullptr,
                      hipStream_t stream = nullptr) {
  const dim3 grid(grid_blocks(k.tm)), block(kBlock);
  hipLaunchKernelGGL((step_kernel<S, C, F>), grid, block, 0, stream ? stream : h->stream,
                     static_cast<const S*>(src), static_cast<S*>(dst),
                     static_cast<const C*>(h->phi()), static_cast<const C*>(h->hv()),
                     static_cast<C*>(mac), static_cast<const C*>(init_tf),
                     static_cast<const C*>(init_ts), k, step, static_cast<C*>(rec));
  return hipGetLastError();
}

// Dispatch over the field flags; mode: 0 plain step, 1 step writing macros,
// 2 initialisation (writes macros), 3 step recording q at interior nodes,
// 4 recording step that also writes macros (modes 3, 4: FP32 and FP64 only).
template <typename S, typename C>
hipError_t launch_step_t(const lbm_ltne* h, const StepConsts<C>& k, int mode, uint32_t step, const void* src,
                         void* dst, void* mac, const void* init_tf, const void* init_ts,
                         void* rec, hipStream_t stream) {
  const int fl = (h->has_phi ? kPhiField : 0) | (h->has_hv ? kHvField : 0);
  if constexpr (!std::is_same<S, _Float16>::value) {
    if (mode == 3 || mode == 4) {
      switch (fl) {
        case 0:
          return mode == 3 ? launch_one<S, C, kRecord>(h, k, step, src, dst, mac, init_tf, init_ts, rec, stream)
                           : launch_one<S, C, kRecord | kMacros>(h, k, step, src, dst, mac, init_tf, init_ts, rec, stream);
        case kPhiField:
          return mode == 3 ? launch_one<S, C, kPhiField | kRecord>(h, k, step, src, dst, mac, init_tf, init_ts, rec, stream)
                           : launch_one<S, C, kPhiField | kRecord | kMacros>(h, k, step, src, dst, mac, init_tf,
                                                                            init_ts, rec, stream);
        case kHvField:
          return mode == 3 ? launch_one<S, C, kHvField | kRecord>(h, k, step, src, dst, mac, init_tf, init_ts, rec, stream)
                           : launch_one<S, C, kHvField | kRecord | kMacros>(h, k, step, src, dst, mac, init_tf,
                                                                           init_ts, rec, stream);
        default:
          return mode == 3
                     ? launch_one<S, C, kPhiField | kHvField | kRecord>(h, k, step, src, dst, mac, init_tf, init_ts, rec, stream)
                     : launch_one<S, C, kPhiField | kHvField | kRecord | kMacros>(h, k, step, src, dst, mac, init_tf,
                                                                                 init_ts, rec, stream);
      }
    }
  } else {
    (void)rec;
    if (mode == 3 || mode == 4) return hipErrorInvalidValue;
  }
#define LTNE_CASE(FL)                                                                               \
  case FL:                                                                                          \
    if (mode == 0) return launch_one<S, C, FL>(h, k, step, src, dst, mac, init_tf, init_ts, nullptr, stream); \
    if (mode == 1)                                                                                  \
      return launch_one<S, C, FL | kMacros>(h, k, step, src, dst, mac, init_tf, init_ts, nullptr, stream);  \
    return launch_one<S, C, FL | kMacros | kInit>(h, k, step, src, dst, mac, init_tf, init_ts, nullptr, stream);
  switch (fl) {
    LTNE_CASE(0)
    LTNE_CASE(kPhiField)
    LTNE_CASE(kHvField)
    LTNE_CASE(kPhiField | kHvField)
  }
#undef LTNE_CASE
  return hipErrorInvalidValue;
}

// step: the number of the time step being computed (0 for the
// initialisation), the counter of the stochastic rounding.
hipError_t launch_step(const lbm_ltne* h, int mode, int64_t step, const void* src, void* dst, void* mac,
                       const void* init_tf, const void* init_ts, void* rec = nullptr,
                       hipStream_t stream = nullptr) {
  const uint32_t st = static_cast<uint32_t>(step);
  switch (h->p.precision) {
    case LBM_FP64:
      return launch_step_t<double, double>(h, h->kd, mode, st, src, dst, mac, init_tf, init_ts, rec, stream);
    case LBM_FP32:
      return launch_step_t<float, float>(h, h->kf, mode, st, src, dst, mac, init_tf, init_ts, rec, stream);
    case LBM_FP32SR:
      return launch_step_t<float, double>(h, h->kd, mode, st, src, dst, mac, init_tf, init_ts, rec, stream);
    default:
      return launch_step_t<_Float16, float>(h, h->kf, mode, st, src, dst, mac, init_tf, init_ts, rec, stream);
  }
}


// Geometry of the two-step kernel: strips of 64 lanes (63 - halo output
// columns), chunks of step2_rows() rows, kStep2Block / 64 wavefronts per workgroup,
// workgroups dealt to the XCDs in contiguous ranges.
Step2Map step2_map(const lbm_ltne_params& p) {
  Step2Map m{};
  m.halo = step2_halo(p.periodic_x);
  m.out = step2_out(p.periodic_x);
  m.nstrips = (p.nx + m.out - 1) / m.out;
  m.rows = step2_rows(p.nx, p.ny, p.periodic_x, storage_bytes(p.precision));
  m.nchunks = (p.ny + m.rows - 1) / m.rows;
  m.nwaves = m.nstrips * m.nchunks;
  const int nblocks = (m.nwaves + kStep2Block / 64 - 1) / (kStep2Block / 64);
  m.per_xcd = (nblocks + kXcds - 1) / kXcds;
  return m;
}

// Two steps in one launch (FP32 and FP64 forms); with mac, the second step
// also writes the macros (the last two steps of a call).
template <typename S, int F>
void launch_step2_t(const lbm_ltne* h, const StepConsts<S>& k, const Step2Map& m, const S* s, S* d, S* mac,
                    uint32_t st) {
  const dim3 grid(kXcds * m.per_xcd), block(kStep2Block);
  const S* phi = static_cast<const S*>(h->phi());
  const S* hv = static_cast<const S*>(h->hv());
  if (mac)
    hipLaunchKernelGGL((step2_kernel<S, F | kMacros>), grid, block, 0, h->stream, s, d, phi, hv, mac, k, m, st);
  else
    hipLaunchKernelGGL((step2_kernel<S, F>), grid, block, 0, h->stream, s, d, phi, hv, mac, k, m, st);
}

template <typename S>
void launch_step2_s(const lbm_ltne* h, const StepConsts<S>& k, uint32_t st, const void* src, void* dst, void* mac) {
  const Step2Map m = step2_map(h->p);
  const S* s = static_cast<const S*>(src);
  S* d = static_cast<S*>(dst);
  S* mc = static_cast<S*>(mac);
  switch ((h->has_phi ? kPhiField : 0) | (h->has_hv ? kHvField : 0)) {
    case 0: launch_step2_t<S, 0>(h, k, m, s, d, mc, st); break;
    case kPhiField: launch_step2_t<S, kPhiField>(h, k, m, s, d, mc, st); break;
    case kHvField: launch_step2_t<S, kHvField>(h, k, m, s, d, mc, st); break;
    default: launch_step2_t<S, kPhiField | kHvField>(h, k, m, s, d, mc, st);
  }
}

hipError_t launch_step2(const lbm_ltne* h, int64_t step, const void* src, void* dst, void* mac = nullptr) {
  const uint32_t st = static_cast<uint32_t>(step);
  if (h->p.precision == LBM_FP64)
    launch_step2_s<double>(h, h->kd, st, src, dst, mac);
  else
    launch_step2_s<float>(h, h->kf, st, src, dst, mac);
  return hipGetLastError();
}

// Copies a host double field to device memory in the compute type.
int upload_field(const lbm_ltne* h, const double* src, void* dst) {
  const long long n = h->n();
  if (compute_bytes(h->p.precision) == 8) {
    HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  } else {
    std::vector<float> tmp(n);
    for (long long i = 0; i < n; ++i) tmp[i] = static_cast<float>(src[i]);
    HIP_TRY(hipMemcpyAsync(dst, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));  // tmp goes out of scope
  }
  return LBM_OK;
}

void release(lbm_ltne* h) {
  if (!h) return;
  for (hipGraphExec_t& g : h->seq)
    if (g) (void)hipGraphExecDestroy(g);
  if (h->owns && h->base) (void)hipFree(h->base);
  delete h;
}

// Lattices whose single steps are short enough that launching them one by
// one costs a large part of their time run their steps in recorded runs of
// kSeqSteps launches (a HIP graph replayed as a whole), when they do not take
// two steps per launch and no step of the run is checked under diag_every.
constexpr int kSeqSteps = 32;  // even: a run starts and ends on the same buffer
constexpr long long kSeqMaxNodes = 1LL << 20;

template <typename S, typename C, int F>
int build_seq_t(lbm_ltne* h, const StepConsts<C>& k, int start) {
  hipGraph_t g = nullptr;
  HIP_TRY(hipGraphCreate(&g, 0));
  hipGraphNode_t prev = nullptr;
  int rc = LBM_OK;
  const dim3 grid(grid_blocks(k.tm)), block(kBlock);
  for (int j = 0; j < kSeqSteps && rc == LBM_OK; ++j) {
    const S* src = static_cast<const S*>(h->pop((start + j) & 1));
    S* dst = static_cast<S*>(h->pop((start + j + 1) & 1));
    const C* phi = static_cast<const C*>(h->phi());
    const C* hv = static_cast<const C*>(h->hv());
    StepConsts<C> kk = k;
    const uint32_t* base = h->step_base();
    uint32_t off = static_cast<uint32_t>(j);
    void* args[] = {&src, &dst, &phi, &hv, &kk, &base, &off};
    hipKernelNodeParams np{};
    np.func = reinterpret_cast<void*>(&step_seq_kernel<S, C, F>);
    np.gridDim = grid;
    np.blockDim = block;
    np.sharedMemBytes = 0;
    np.kernelParams = args;
    np.extra = nullptr;
    hipGraphNode_t node = nullptr;
    const hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &np);
    if (e != hipSuccess) rc = set_error(LBM_EHIP, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
    prev = node;
  }
  if (rc == LBM_OK) {
    uint32_t* base = h->step_base();
    uint32_t n = kSeqSteps;
    int add = 1;
    void* args[] = {&base, &n, &add};
    hipKernelNodeParams np{};
    np.func = reinterpret_cast<void*>(&step_base_kernel);
    np.gridDim = dim3(1);
    np.blockDim = dim3(64);
    np.sharedMemBytes = 0;
    np.kernelParams = args;
    np.extra = nullptr;
    hipGraphNode_t node = nullptr;
    const hipError_t e = hipGraphAddKernelNode(&node, g, &prev, 1, &np);
    if (e != hipSuccess) rc = set_error(LBM_EHIP, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
  }
  if (rc == LBM_OK) {
    const hipError_t e = hipGraphInstantiate(&h->seq[start], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      h->seq[start] = nullptr;
      rc = set_error(LBM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
  }
  (void)hipGraphDestroy(g);
  return rc;
}

template <typename S, typename C>
int build_seq_p(lbm_ltne* h, const StepConsts<C>& k, int start) {
  switch ((h->has_phi ? kPhiField : 0) | (h->has_hv ? kHvField : 0)) {
    case kPhiField: return build_seq_t<S, C, kPhiField>(h, k, start);
    case kHvField: return build_seq_t<S, C, kHvField>(h, k, start);
    case kPhiField | kHvField: return build_seq_t<S, C, kPhiField | kHvField>(h, k, start);
    default: return build_seq_t<S, C, 0>(h, k, start);
  }
}

// The recorded run starting from population buffer `start`, built on first use.
int seq_graph(lbm_ltne* h, int start) {
  if (h->seq[start]) return LBM_OK;
  switch (h->p.precision) {
    case LBM_FP64: return build_seq_p<double, double>(h, h->kd, start);
    case LBM_FP32: return build_seq_p<float, float>(h, h->kf, start);
    case LBM_FP32SR: return build_seq_p<float, double>(h, h->kd, start);
    default: return build_seq_p<_Float16, float>(h, h->kf, start);
  }
}

// Workgroups of the binary64 sums over the macros.
int sum_blocks(const lbm_ltne* h) {
  return static_cast<int>(std::min<long long>(kSumBlocks, (h->n() + kBlock - 1) / kBlock));
}

// Per-workgroup partial sums (mass, energy, residual terms) of the macro
// buffer mac against prev, into the partial-sum scratch.
void launch_sums(const lbm_ltne* h, const void* mac, const void* prev) {
  const long long n = h->n();
  if (compute_bytes(h->p.precision) == 8) {
    hipLaunchKernelGGL((sums_kernel<double>), dim3(sum_blocks(h)), dim3(kBlock), 0, h->stream,
                       static_cast<const double*>(mac), static_cast<const double*>(prev),
                       static_cast<const double*>(h->phi()), h->p.phi, h->p.sigma, n, n, h->partial());
  } else {
    hipLaunchKernelGGL((sums_kernel<float>), dim3(sum_blocks(h)), dim3(kBlock), 0, h->stream,
                       static_cast<const float*>(mac), static_cast<const float*>(prev),
                       static_cast<const float*>(h->phi()), h->p.phi, h->p.sigma, n, n, h->partial());
  }
}

// After a synchronizing call's work has completed: LBM_EDIVERGED if a step
// checked under diag_every had non-finite sums, else rc.
int check_diverged(lbm_ltne* h, int rc) {
  if (h->p.diag_every <= 0 || rc != LBM_OK) return rc;
  unsigned long long t = 0;
  HIP_TRY(hipMemcpyAsync(&t, h->diverged(), sizeof(t), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (t != 0)
    return set_error(LBM_EDIVERGED, "non-finite mass or energy at step %llu (checked every %d steps)", t,
                     h->p.diag_every);
  return rc;
}

// Clears the divergence record (creation, loading a state).
hipError_t clear_diverged(lbm_ltne* h) {
  static const unsigned long long zero = 0;
  hipError_t e = hipMemcpyAsync(h->diverged(), &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return e;
}

}  // namespace

extern "C" {

size_t lbm_ltne_pool_bytes(const lbm_ltne_params* p, int has_phi, int has_Hv) {
  if (lbm_ltne_derive(p, nullptr) != LBM_OK) return 0;
  return make_layout(p, has_phi != 0, has_Hv != 0).total;
}

int lbm_ltne_create(const lbm_ltne_params* p, const double* phi_field, const double* Hv_field,
                    const double* Tf_init, const double* Ts_init, void* hip_stream,
                    void* device_pool, size_t pool_bytes, lbm_ltne_t* out) {
  clear_error();
  if (!out) return set_error(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return set_error(LBM_EINVAL, "params is NULL");
  const long long n = static_cast<long long>(p->nx) * p->ny;
  // Temperature range of walls, uniform and field initial values.
  double tmin = 0.0, tmax = 0.0;
  temperature_range(p, &tmin, &tmax);
  if (p->nx > 0 && p->ny > 0 && n <= (1LL << 30)) {
    for (const double* fld : {Tf_init, Ts_init}) {
      if (!fld) continue;
      for (long long i = 0; i < n; ++i) {
        if (!std::isfinite(fld[i])) return set_error(LBM_EINVAL, "initial temperature %lld is not finite", i);
        tmin = std::fmin(tmin, fld[i]);
        tmax = std::fmax(tmax, fld[i]);
      }
    }
  }
  lbm_ltne_derived d;
  int rc = derive(p, tmin, tmax, &d);
  if (rc != LBM_OK) return rc;
  if (phi_field)
    for (long long i = 0; i < n; ++i)
      if (!(phi_field[i] > 0.0 && phi_field[i] < 1.0))
        return set_error(LBM_EINVAL, "phi_field[%lld] = %g not in (0, 1)", i, phi_field[i]);
  if (Hv_field && p->pore_size > 0.0)
    return set_error(LBM_EINVAL, "an H_v field and the correlation of Eq. 52 (pore_size > 0) exclude each other");
  if (Hv_field)
    for (long long i = 0; i < n; ++i)
      if (!(Hv_field[i] >= 0.0) || !std::isfinite(Hv_field[i]))
        return set_error(LBM_EINVAL, "Hv_field[%lld] = %g must be finite and >= 0", i, Hv_field[i]);
  int dev = 0;
  rc = check_device(&dev);
  if (rc != LBM_OK) return rc;

  lbm_ltne* h = new (std::nothrow) lbm_ltne();
  if (!h) return set_error(LBM_ENOMEM, "host allocation failed");
  h->p = *p;
  h->d = d;
  h->device = dev;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->has_phi = phi_field != nullptr;
  h->has_hv = Hv_field != nullptr;
  if (Tf_init) h->tf0.assign(Tf_init, Tf_init + n);
  if (Ts_init) h->ts0.assign(Ts_init, Ts_init + n);
  h->lay = make_layout(p, h->has_phi, h->has_hv);
  if (device_pool) {
    if (pool_bytes < h->lay.total) {
      release(h);
      return set_error(LBM_ENOMEM, "device pool of %zu bytes is smaller than the %zu needed",
                       pool_bytes, h->lay.total);
    }
    if (reinterpret_cast<uintptr_t>(device_pool) % kAlign != 0) {
      release(h);
      return set_error(LBM_EINVAL, "device pool must be %zu-byte aligned", kAlign);
    }
    h->base = static_cast<char*>(device_pool);
    h->owns = false;
  } else {
    if (hipMalloc(&h->base, h->lay.total) != hipSuccess) {
      (void)hipGetLastError();
      const size_t want = h->lay.total;
      h->base = nullptr;
      release(h);
      return set_error(LBM_ENOMEM, "hipMalloc of %zu bytes failed", want);
    }
    h->owns = true;
  }
  fill_consts(h, &h->kd);
  fill_consts(h, &h->kf);

  rc = LBM_OK;
  if (phi_field) rc = upload_field(h, phi_field, h->phi());
  if (rc == LBM_OK && Hv_field) rc = upload_field(h, Hv_field, h->hv());
  // Initial temperature fields (relative to T_ref) are staged in the second
  // population buffer, which the first step overwrites.
  void* tf_dev = nullptr;
  void* ts_dev = nullptr;
  const size_t cb = compute_bytes(p->precision);
  if (rc == LBM_OK && (Tf_init || Ts_init)) {
    char* stage = static_cast<char*>(h->pop(1));
    std::vector<double> rel(n);
    if (Tf_init) {
      for (long long i = 0; i < n; ++i) rel[i] = Tf_init[i] - d.T_ref;
      tf_dev = stage;
      rc = upload_field(h, rel.data(), tf_dev);
    }
    if (rc == LBM_OK && Ts_init) {
      for (long long i = 0; i < n; ++i) rel[i] = Ts_init[i] - d.T_ref;
      ts_dev = stage + align_up(n * cb, kAlign);
      rc = upload_field(h, rel.data(), ts_dev);
    }
    if (rc == LBM_OK) {
      hipError_t e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) rc = set_error(LBM_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
  }
  if (rc == LBM_OK) {
    hipError_t e = launch_step(h, 2, 0, nullptr, h->pop(0), h->mac(0), tf_dev, ts_dev);
    if (e != hipSuccess) rc = set_error(LBM_EHIP, "initialisation launch: %s", hipGetErrorString(e));
  }
  if (rc == LBM_OK) {
    // the residual of the first step call compares with the initial macros
    hipError_t e = hipMemcpyAsync(h->mac(1), h->mac(0), h->lay.mac_bytes, hipMemcpyDeviceToDevice,
                                  h->stream);
    if (e == hipSuccess) e = clear_diverged(h);
    if (e != hipSuccess) rc = set_error(LBM_EHIP, "initialisation: %s", hipGetErrorString(e));
  }
  if (rc != LBM_OK) {
    release(h);
    return rc;
  }
  h->cur = 0;
  h->mcur = 0;
  h->steps = 0;
  *out = h;
  return LBM_OK;
}

int lbm_ltne_step(lbm_ltne_t h, int64_t nsteps) {
  if (!h) return set_error(LBM_EINVAL, "handle is NULL");
  if (nsteps < 0) return set_error(LBM_EINVAL, "nsteps = %lld < 0", static_cast<long long>(nsteps));
  if (nsteps == 0) return LBM_OK;
  // two steps per launch where the lattice gives the two-step kernel enough
  // wavefronts to hide its latency (each wavefront runs a serial chain of
  // rows); small lattices run faster one step at a time
  const bool fp64 = h->p.precision == LBM_FP64;
  const bool pairs = (h->p.precision == LBM_FP32 || fp64) &&
                     step2_addressable(h->p.nx, storage_bytes(h->p.precision)) &&
                     step2_waves(h->p.nx, h->p.ny, h->p.periodic_x, kStep2MinRows) >=
                         (fp64 ? LTNE_STEP2_MIN_WAVES_64 : LTNE_STEP2_MIN_WAVES);
  const int64_t de = h->p.diag_every;
  auto checked = [de](int64_t t) { return de > 0 && t % de == 0; };
  void* scratch_mac = h->mac(1 - h->mcur);  // overwritten by the call's last step
  int64_t s = 0;
  // recorded runs of kSeqSteps single steps on small lattices
  if (!pairs && de == 0 && h->n() <= kSeqMaxNodes && nsteps - 1 >= kSeqSteps) {
    hipLaunchKernelGGL(step_base_kernel, dim3(1), dim3(64), 0, h->stream, h->step_base(),
                       static_cast<uint32_t>(h->steps + 1), 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LBM_EHIP, "step base: %s", hipGetErrorString(e));
    for (; s + kSeqSteps <= nsteps - 1; s += kSeqSteps) {
      const int rc = seq_graph(h, h->cur);
      if (rc != LBM_OK) return rc;
      e = hipGraphLaunch(h->seq[h->cur], h->stream);
      if (e != hipSuccess) return set_error(LBM_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
      h->steps += kSeqSteps;  // an even number of steps: the state stays in buffer cur
    }
  }
  while (s < nsteps) {
    const int64_t t = h->steps + 1;  // number of the next step
    // a pair of steps in one launch where neither step is checked; the
    // pair that ends the call also writes the macros of its second step
    if (pairs && s + 2 <= nsteps && !checked(t) && !checked(t + 1)) {
      const bool ends = s + 2 == nsteps;
      hipError_t e = launch_step2(h, t, h->pop(h->cur), h->pop(1 - h->cur), ends ? scratch_mac : nullptr);
      if (e != hipSuccess) return set_error(LBM_EHIP, "step launch: %s", hipGetErrorString(e));
      h->cur = 1 - h->cur;
      h->steps += 2;
      s += 2;
      continue;
    }
    const bool last = (s == nsteps - 1), check = checked(t);
    hipError_t e = launch_step(h, (last || check) ? 1 : 0, t, h->pop(h->cur), h->pop(1 - h->cur),
                               (last || check) ? scratch_mac : nullptr, nullptr, nullptr);
    if (e != hipSuccess) return set_error(LBM_EHIP, "step launch: %s", hipGetErrorString(e));
    h->cur = 1 - h->cur;
    h->steps += 1;
    s += 1;
    if (check) {
      // binary64 mass and energy of this step's macros; a non-finite sum
      // records the step on the device (read by the next synchronizing call)
      const int blocks = sum_blocks(h);
      launch_sums(h, scratch_mac, h->mac(h->mcur));
      hipLaunchKernelGGL(finite_check_kernel, dim3(1), dim3(kBlock), 0, h->stream, h->partial(), blocks,
                         h->diverged(), static_cast<unsigned long long>(t));
      e = hipGetLastError();
      if (e != hipSuccess) return set_error(LBM_EHIP, "divergence check: %s", hipGetErrorString(e));
    }
  }
  h->mcur = 1 - h->mcur;
  return LBM_OK;
}

int64_t lbm_ltne_steps_done(lbm_ltne_t h) { return h ? h->steps : -1; }

int lbm_ltne_macros(lbm_ltne_t h, double* rho, double* ux, double* uy, double* Tf, double* Ts) {
  if (!h) return set_error(LBM_EINVAL, "handle is NULL");
  const long long n = h->n();
  const size_t cb = compute_bytes(h->p.precision);
  double* outs[5] = {rho, ux, uy, Tf, Ts};
  std::vector<float> tmp;
  for (int f = 0; f < 5; ++f) {
    if (!outs[f]) continue;
    const char* src = static_cast<const char*>(h->mac(h->mcur)) + static_cast<size_t>(f) * n * cb;
    if (cb == 8) {
      HIP_TRY(hipMemcpyAsync(outs[f], src, n * 8, hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
    } else {
      tmp.resize(n);
      HIP_TRY(hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
      for (long long i = 0; i < n; ++i) outs[f][i] = tmp[i];
    }
  }
  return check_diverged(h, LBM_OK);
}

int lbm_ltne_nusselt(lbm_ltne_t h, double* Nu_f, double* Nu_s) {
  if (!h) return set_error(LBM_EINVAL, "handle is NULL");
  const int w = hot_wall(&h->p);
  if (w < 0) return set_error(LBM_EINVAL, "no wall selected for the Nusselt number");
  const int periodic_t = (w < 2) ? h->p.periodic_y : h->p.periodic_x;
  const double scale = h->d.L / h->d.dT;
  if (compute_bytes(h->p.precision) == 8) {
    hipLaunchKernelGGL((nusselt_kernel<double>), dim3(1), dim3(kBlock), 0, h->stream,
                       static_cast<const double*>(h->mac(h->mcur)), h->p.nx, h->p.ny, h->n(), w,
                       periodic_t, scale, h->result());
  } else {
    hipLaunchKernelGGL((nusselt_kernel<float>), dim3(1), dim3(kBlock), 0, h->stream,
                       static_cast<const float*>(h->mac(h->mcur)), h->p.nx, h->p.ny, h->n(), w,
                       periodic_t, scale, h->result());
  }
  HIP_TRY(hipGetLastError());
  double r[2];
  HIP_TRY(hipMemcpyAsync(r, h->result(), sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (Nu_f) *Nu_f = r[0];
  if (Nu_s) *Nu_s = r[1];
  return check_diverged(h, LBM_OK);
}

int lbm_ltne_diagnostics(lbm_ltne_t h, double* mass, double* energy, double* residual) {
  if (!h) return set_error(LBM_EINVAL, "handle is NULL");
  const int blocks = sum_blocks(h);
  launch_sums(h, h->mac(h->mcur), h->mac(1 - h->mcur));
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(kBlock), 0, h->stream, h->partial(), blocks,
                     h->result());
  HIP_TRY(hipGetLastError());
  double s[kSums];
  HIP_TRY(hipMemcpyAsync(s, h->result(), sizeof(s), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  auto rel = [](double num, double den) { return den > 0.0 ? num / den : num; };
  const double r = std::max(rel(s[2], s[3]), std::max(rel(s[4], s[5]), rel(s[6], s[7])));
  if (mass) *mass = s[0];
  if (energy) *energy = s[1];
  if (residual) *residual = r;
  if (!std::isfinite(s[0]) || !std::isfinite(s[1]))
    return set_error(LBM_EDIVERGED, "mass %g, energy %g after %lld steps", s[0], s[1],
                     static_cast<long long>(h->steps));
  return check_diverged(h, LBM_OK);
}

namespace {
struct StateHeader {
  uint32_t magic;
  int32_t abi;
  int32_t nx, ny, precision, mcur;
  int64_t steps;
  int64_t pop_bytes, mac_bytes;
};
}  // namespace

size_t lbm_ltne_state_bytes(lbm_ltne_t h) {
  if (!h) return 0;
  return sizeof(StateHeader) + h->lay.pop_bytes + 2 * h->lay.mac_bytes;
}

int lbm_ltne_save(lbm_ltne_t h, void* host_buf, size_t bytes) {
  if (!h || !host_buf) return set_error(LBM_EINVAL, "handle or buffer is NULL");
  if (bytes < lbm_ltne_state_bytes(h))
    return set_error(LBM_EINVAL, "buffer of %zu bytes < %zu needed", bytes, lbm_ltne_state_bytes(h));
  StateHeader hd{kStateMagic, LBM_LTNE_ABI_VERSION, h->p.nx, h->p.ny, h->p.precision, h->mcur,
                 h->steps, static_cast<int64_t>(h->lay.pop_bytes),
                 static_cast<int64_t>(h->lay.mac_bytes)};
  char* b = static_cast<char*>(host_buf);
  std::memcpy(b, &hd, sizeof(hd));
  b += sizeof(hd);
  HIP_TRY(hipMemcpyAsync(b, h->pop(h->cur), h->lay.pop_bytes, hipMemcpyDeviceToHost, h->stream));
  b += h->lay.pop_bytes;
  HIP_TRY(hipMemcpyAsync(b, h->mac(0), h->lay.mac_bytes, hipMemcpyDeviceToHost, h->stream));
  b += h->lay.mac_bytes;
  HIP_TRY(hipMemcpyAsync(b, h->mac(1), h->lay.mac_bytes, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return check_diverged(h, LBM_OK);
}

int lbm_ltne_load(lbm_ltne_t h, const void* host_buf, size_t bytes) {
  if (!h || !host_buf) return set_error(LBM_EINVAL, "handle or buffer is NULL");
  if (bytes < sizeof(StateHeader)) return set_error(LBM_EINVAL, "buffer too small for a state");
  StateHeader hd;
  std::memcpy(&hd, host_buf, sizeof(hd));
  if (hd.magic != kStateMagic || hd.abi != LBM_LTNE_ABI_VERSION)
    return set_error(LBM_EINVAL, "buffer does not hold a saved state of this library version");
  if (hd.nx != h->p.nx || hd.ny != h->p.ny || hd.precision != h->p.precision ||
      hd.pop_bytes != static_cast<int64_t>(h->lay.pop_bytes) ||
      hd.mac_bytes != static_cast<int64_t>(h->lay.mac_bytes) || (hd.mcur != 0 && hd.mcur != 1))
    return set_error(LBM_EINVAL, "saved state has a different shape or precision");
  if (bytes < lbm_ltne_state_bytes(h))
    return set_error(LBM_EINVAL, "buffer of %zu bytes < %zu needed", bytes, lbm_ltne_state_bytes(h));
  const char* b = static_cast<const char*>(host_buf) + sizeof(hd);
  HIP_TRY(hipMemcpyAsync(h->pop(0), b, h->lay.pop_bytes, hipMemcpyHostToDevice, h->stream));
  b += h->lay.pop_bytes;
  HIP_TRY(hipMemcpyAsync(h->mac(0), b, h->lay.mac_bytes, hipMemcpyHostToDevice, h->stream));
  b += h->lay.mac_bytes;
  HIP_TRY(hipMemcpyAsync(h->mac(1), b, h->lay.mac_bytes, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(clear_diverged(h));
  h->cur = 0;
  h->mcur = hd.mcur;
  h->steps = hd.steps;
  return LBM_OK;
}

int lbm_ltne_get_derived(lbm_ltne_t h, lbm_ltne_derived* d) {
  if (!h || !d) return set_error(LBM_EINVAL, "handle or output is NULL");
  *d = h->d;
  return LBM_OK;
}

}  // extern "C"

// Adjoint storage and arithmetic types of the FP32 form.  With the local
// gradient taken in reverse mode, binary32 arithmetic gives gradients within
// a few 1e-5 of central differences of the FP64 forward (512^2 cavity, 4000
// steps), the same as binary64 arithmetic, at lower register pressure.
#ifndef LTNE_ADJ32_LAM
#define LTNE_ADJ32_LAM float
#endif
#ifndef LTNE_ADJ32_MATH
#define LTNE_ADJ32_MATH float
#endif

namespace {

// dNu_f/dT_f at interior nodes.  Nu_f is the mean over the hot wall of
// -dT/dn with dT/dn = (-3 T_0 + 4 T_1 - T_2)/2 (see lbm_ltne_nusselt); the
// reported temperature of a wall node is its Dirichlet value (no
// dependence) or, on an adiabatic wall, T_f of its inward neighbour.
std::vector<double> nusselt_weights(const lbm_ltne* h, int w) {
  const int nx = h->p.nx, ny = h->p.ny;
  const long long n = h->n();
  std::vector<double> wT(n, 0.0), wI(n, 0.0);
  const int len = (w < 2) ? ny : nx;
  const int periodic_t = (w < 2) ? h->p.periodic_y : h->p.periodic_x;
  double W = 0.0;
  for (int kk = 0; kk < len; ++kk) W += (!periodic_t && (kk == 0 || kk == len - 1)) ? 0.5 : 1.0;
  const double scale = h->d.L / h->d.dT;
  for (int kk = 0; kk < len; ++kk) {
    long long i0, i1, i2;
    if (w == 0) { i0 = 1LL * kk * nx; i1 = i0 + 1; i2 = i0 + 2; }
    else if (w == 1) { i0 = 1LL * kk * nx + nx - 1; i1 = i0 - 1; i2 = i0 - 2; }
    else if (w == 2) { i0 = kk; i1 = nx + kk; i2 = 2LL * nx + kk; }
    else { i0 = 1LL * (ny - 1) * nx + kk; i1 = i0 - nx; i2 = i0 - 2LL * nx; }
    const double c = ((!periodic_t && (kk == 0 || kk == len - 1)) ? 0.5 : 1.0) * scale / W;
    wT[i0] += 1.5 * c;
    wT[i1] += -2.0 * c;
    wT[i2] += 0.5 * c;
  }
  for (long long i = 0; i < n; ++i) {
    if (wT[i] == 0.0) continue;
    const int x = static_cast<int>(i % nx), y = static_cast<int>(i / nx);
    const bool wx = !h->p.periodic_x && (x == 0 || x == nx - 1);
    const bool wy = !h->p.periodic_y && (y == 0 || y == ny - 1);
    if (!wx && !wy) {
      wI[i] += wT[i];
      continue;
    }
    bool dirichlet = false;
    if (wx && h->p.wall_thermal[x == 0 ? 0 : 1] == LBM_WALL_DIRICHLET) dirichlet = true;
    if (!dirichlet && wy && h->p.wall_thermal[y == 0 ? 2 : 3] == LBM_WALL_DIRICHLET) dirichlet = true;
    if (dirichlet) continue;
    const int xf = wx ? (x == 0 ? 1 : nx - 2) : x;
    const int yf = wy ? (y == 0 ? 1 : ny - 2) : y;
    wI[1LL * yf * nx + xf] += wT[i];
  }
  return wI;
}

// Bulk region and edge list of one adjoint sweep (see AdjGrid).
AdjGrid adjoint_grid(const lbm_ltne_params& p) {
  AdjGrid g{};
  const int nx = p.nx, ny = p.ny;
  const bool wxa = !p.periodic_x, wya = !p.periodic_y;
  g.bx0 = wxa ? 2 : 0;
  g.by0 = wya ? 2 : 0;
  g.bw = std::max(0, (wxa ? nx - 3 : nx - 1) - g.bx0 + 1);
  g.bh = std::max(0, (wya ? ny - 3 : ny - 1) - g.by0 + 1);
  if (g.bw > 0 && g.bh > 0) {
    g.tm = make_tiles(g.bw, g.bh, p.precision, 0, p.precision == LBM_FP32 ? 6 : 8);
    g.bulk_blocks = grid_blocks(g.tm);
  }
  g.rowlen = wxa ? nx - 2 : nx;
  g.rx0 = wxa ? 1 : 0;
  g.nrow = wya ? (ny - 2 > 1 ? 2 : 1) : 0;
  g.collen = wya ? std::max(0, ny - 4) : ny;
  g.cy0 = wya ? 2 : 0;
  g.ncol = wxa ? (nx - 2 > 1 ? 2 : 1) : 0;
  g.nedge = g.nrow * g.rowlen + g.ncol * g.collen;
  g.edge_blocks = static_cast<int>((4LL * g.nedge + kBlock - 1) / kBlock);
  // planes rounded up to 1024 elements plus 256, so that the 19 planes do
  // not all start on the same power-of-two boundary
  g.lplane = static_cast<long long>(align_up(static_cast<size_t>(nx) * ny, 1024)) + 256;
  return g;
}

template <typename C>
int upload_compute(const lbm_ltne* h, const std::vector<double>& src, void* dst) {
  std::vector<C> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = static_cast<C>(src[i]);
  HIP_TRY(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(C), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

// R: the lattice's compute type (fields, recorded sums); Lm: storage of the
// adjoint populations; C: arithmetic of the adjoint sweep.
template <typename R, typename Lm, typename C>
int adjoint_t(lbm_ltne* h, int64_t nsteps, int64_t K, double* loss, double* dphi, double* dhv) {
  const StepConsts<C>& k = *reinterpret_cast<const StepConsts<C>*>(
      std::is_same<C, double>::value ? static_cast<const void*>(&h->kd) : static_cast<const void*>(&h->kf));
  const long long n = h->n();
  const int w = hot_wall(&h->p);
  if (w < 0) return set_error(LBM_EINVAL, "no wall selected for the Nusselt number");
  const bool include_init = (h->steps == 0);
  const int64_t t0 = h->steps;
  const int64_t nseg = (nsteps + K - 1) / K;
  const size_t popb = h->lay.pop_bytes;
  const size_t recb = align_up(static_cast<size_t>(K) * 5 * n * sizeof(R), kAlign);
  const AdjGrid ag = adjoint_grid(h->p);
  const size_t lamb = align_up(static_cast<size_t>(kPlanes) * ag.lplane * sizeof(Lm), kAlign);
  const size_t gb = align_up(n * sizeof(double), kAlign);
  const size_t fb = align_up(n * sizeof(R), kAlign);
  auto total_for = [&](int nbuf) { return nseg * popb + 2 * popb + nbuf * recb + 2 * lamb + 2 * gb + 3 * fb; };

  // Work memory, a second stream and its events, released on every path out
  // (after both streams drained).
  struct Work {
    char* buf = nullptr;
    hipStream_t main = nullptr, side = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    ~Work() {
      if (side) (void)hipStreamSynchronize(side);
      if (main) (void)hipStreamSynchronize(main);
      for (hipEvent_t& x : ev)
        if (x) (void)hipEventDestroy(x);
      if (side) (void)hipStreamDestroy(side);
      if (buf) (void)hipFree(buf);
    }
  } wk;
  wk.main = h->stream;
  // Segments are recomputed on the second stream into one of two recording
  // buffers while the main stream sweeps the segment after them backwards
  // from the other, so the two latency-bound kernels share the machine; with
  // memory for one buffer only, recompute and sweep alternate.
  int nbuf = 2;
  if (hipMalloc(&wk.buf, total_for(2)) != hipSuccess) {
    wk.buf = nullptr;
    (void)hipGetLastError();
    nbuf = 1;
    if (hipMalloc(&wk.buf, total_for(1)) != hipSuccess) {
      wk.buf = nullptr;
      (void)hipGetLastError();
      return set_error(LBM_ENOMEM, "adjoint work memory of %zu bytes failed", total_for(1));
    }
  }
  hipError_t e;
  auto hip_fail = [&](hipError_t err, const char* what) {
    return set_error(LBM_EHIP, "adjoint %s: %s", what, hipGetErrorString(err));
  };
  if ((e = hipStreamCreateWithFlags(&wk.side, hipStreamNonBlocking)) != hipSuccess) {
    wk.side = nullptr;
    return hip_fail(e, "stream");
  }
  for (hipEvent_t& x : wk.ev)
    if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming)) != hipSuccess) {
      x = nullptr;
      return hip_fail(e, "event");
    }
  hipEvent_t ev_fwd = wk.ev[0];
  hipEvent_t ev_rec[2] = {wk.ev[1], wk.ev[2]};    // segment recorded into buffer i
  hipEvent_t ev_sweep[2] = {wk.ev[3], wk.ev[4]};  // sweep done reading buffer i

  char* ckpt = wk.buf;
  char* work[2] = {ckpt + nseg * popb, ckpt + nseg * popb + popb};
  R* rec[2] = {reinterpret_cast<R*>(work[1] + popb), reinterpret_cast<R*>(work[1] + popb + (nbuf - 1) * recb)};
  Lm* lam[2] = {reinterpret_cast<Lm*>(reinterpret_cast<char*>(rec[0]) + nbuf * recb),
                reinterpret_cast<Lm*>(reinterpret_cast<char*>(rec[0]) + nbuf * recb + lamb)};
  double* gphi = reinterpret_cast<double*>(reinterpret_cast<char*>(lam[1]) + lamb);
  double* ghv = reinterpret_cast<double*>(reinterpret_cast<char*>(gphi) + gb);
  R* wseed = reinterpret_cast<R*>(reinterpret_cast<char*>(ghv) + gb);
  R* itf = reinterpret_cast<R*>(reinterpret_cast<char*>(wseed) + fb);
  R* its = reinterpret_cast<R*>(reinterpret_cast<char*>(itf) + fb);

  // forward with checkpoints; the handle itself advances to t0 + nsteps.
  // A failure after this point puts the state of t0 (checkpoint 0) back.
  const int cur0 = h->cur;
  auto bail = [&](int code) {
    (void)hipStreamSynchronize(wk.side);
    (void)hipStreamSynchronize(h->stream);
    if (hipMemcpyAsync(h->pop(cur0), ckpt, popb, hipMemcpyDeviceToDevice, h->stream) == hipSuccess)
      (void)hipStreamSynchronize(h->stream);
    h->cur = cur0;
    return code;
  };
  for (int64_t sg = 0; sg < nseg; ++sg) {
    e = hipMemcpyAsync(ckpt + sg * popb, h->pop(h->cur), popb, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return sg == 0 ? hip_fail(e, "checkpoint") : bail(hip_fail(e, "checkpoint"));
    const int64_t steps_in = std::min<int64_t>(K, nsteps - sg * K);
    for (int64_t j = 0; j < steps_in; ++j) {
      e = launch_step(h, 0, t0 + sg * K + j + 1, h->pop(h->cur), h->pop(1 - h->cur), nullptr, nullptr, nullptr);
      if (e != hipSuccess) return bail(hip_fail(e, "forward launch"));
      h->cur = 1 - h->cur;
    }
  }
  int rc = upload_compute<R>(h, nusselt_weights(h, w), wseed);
  if (rc != LBM_OK) return bail(rc);
  if ((e = hipMemsetAsync(gphi, 0, 2 * gb, h->stream)) != hipSuccess) return bail(hip_fail(e, "zero"));
  const R* phi_f = static_cast<const R*>(h->phi());
  const R* hv_f = static_cast<const R*>(h->hv());
  const dim3 block(kBlock), grid(ag.bulk_blocks + ag.edge_blocks);
  auto sweep = [&](auto kernel, const Lm* lin, Lm* lout, const R* recp, const R* ws, const R* tf,
                   const R* ts) -> hipError_t {
    hipLaunchKernelGGL(kernel, grid, block, 0, h->stream, lin, lout, recp, phi_f, hv_f, gphi, ghv, ws, tf, ts, k,
                       ag);
    return hipGetLastError();
  };
  int la = 0;
  // the recomputes read the checkpoints of the forward
  if ((e = hipEventRecord(ev_fwd, h->stream)) != hipSuccess) return bail(hip_fail(e, "event record"));
  if ((e = hipStreamWaitEvent(wk.side, ev_fwd, 0)) != hipSuccess) return bail(hip_fail(e, "event wait"));
  for (int64_t sg = nseg - 1; sg >= 0; --sg) {
    const int b = static_cast<int>(sg % nbuf);
    R* rb = rec[b];
    // recompute the segment on the side stream, recording q of every step,
    // once the sweep that last read this buffer (segment sg + nbuf) is done
    if (sg + nbuf <= nseg - 1 && (e = hipStreamWaitEvent(wk.side, ev_sweep[b], 0)) != hipSuccess)
      return bail(hip_fail(e, "event wait"));
    e = hipMemcpyAsync(work[0], ckpt + sg * popb, popb, hipMemcpyDeviceToDevice, wk.side);
    if (e != hipSuccess) return bail(hip_fail(e, "restore"));
    const int64_t steps_in = std::min<int64_t>(K, nsteps - sg * K);
    int wc = 0;
    for (int64_t j = 1; j <= steps_in; ++j) {
      const bool last = (sg == nseg - 1 && j == steps_in);
      e = launch_step(h, last ? 4 : 3, t0 + sg * K + j, work[wc], work[1 - wc],
                      last ? h->mac(1 - h->mcur) : nullptr, nullptr, nullptr, rb + (j - 1) * 5 * n, wk.side);
      if (e != hipSuccess) return bail(hip_fail(e, "recompute launch"));
      wc = 1 - wc;
    }
    if ((e = hipEventRecord(ev_rec[b], wk.side)) != hipSuccess) return bail(hip_fail(e, "event record"));
    // sweep it backwards on the main stream
    if ((e = hipStreamWaitEvent(h->stream, ev_rec[b], 0)) != hipSuccess) return bail(hip_fail(e, "event wait"));
    int64_t jhi = steps_in;
    if (sg == nseg - 1) {
      e = sweep(adjoint_kernel<Lm, C, R, kAdjSeed>, nullptr, lam[la], rb + (steps_in - 1) * 5 * n, wseed,
                nullptr, nullptr);
      if (e != hipSuccess) return bail(hip_fail(e, "seed launch"));
      jhi = steps_in - 1;
    }
    for (int64_t j = jhi; j >= 1; --j) {
      e = sweep(adjoint_kernel<Lm, C, R, kAdjStep>, lam[la], lam[1 - la], rb + (j - 1) * 5 * n, nullptr, nullptr,
                nullptr);
      if (e != hipSuccess) return bail(hip_fail(e, "adjoint launch"));
      la = 1 - la;
    }
    if ((e = hipEventRecord(ev_sweep[b], h->stream)) != hipSuccess) return bail(hip_fail(e, "event record"));
  }
  if (include_init) {
    const R* tf = nullptr;
    const R* ts = nullptr;
    if (!h->tf0.empty()) {
      std::vector<double> rel(h->tf0);
      for (auto& v : rel) v -= h->d.T_ref;
      if ((rc = upload_compute<R>(h, rel, itf)) != LBM_OK) return bail(rc);
      tf = itf;
    }
    if (!h->ts0.empty()) {
      std::vector<double> rel(h->ts0);
      for (auto& v : rel) v -= h->d.T_ref;
      if ((rc = upload_compute<R>(h, rel, its)) != LBM_OK) return bail(rc);
      ts = its;
    }
    e = sweep(adjoint_kernel<Lm, C, R, kAdjInit>, lam[la], nullptr, nullptr, nullptr, tf, ts);
    if (e != hipSuccess) return bail(hip_fail(e, "init adjoint launch"));
  }
  if (dphi && (e = hipMemcpyAsync(dphi, gphi, n * sizeof(double), hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
    return bail(hip_fail(e, "gradient copy"));
  if (dhv && (e = hipMemcpyAsync(dhv, ghv, n * sizeof(double), hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
    return bail(hip_fail(e, "gradient copy"));
  if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return bail(hip_fail(e, "sync"));
  h->mcur = 1 - h->mcur;
  h->steps += nsteps;
  if (loss) {
    double nus = 0.0;
    rc = lbm_ltne_nusselt(h, loss, &nus);
    if (rc != LBM_OK) return rc;
  }
  return LBM_OK;
}

}  // namespace

extern "C" int lbm_ltne_adjoint(lbm_ltne_t h, int64_t nsteps, int64_t ckpt_every, double* loss,
                                double* dL_dphi, double* dL_dHv) {
  if (!h) return set_error(LBM_EINVAL, "handle is NULL");
  if (nsteps < 1) return set_error(LBM_EINVAL, "nsteps = %lld must be >= 1", static_cast<long long>(nsteps));
  if (ckpt_every < 1) ckpt_every = nsteps;
  if (ckpt_every > nsteps) ckpt_every = nsteps;
  if (h->p.precision == LBM_FP16S)
    return set_error(LBM_EUNSUPPORTED, "the adjoint is built for the FP64, FP32 and FP32SR forms");
  if (h->p.pore_size > 0.0)
    return set_error(LBM_EUNSUPPORTED, "the adjoint covers the model without the correlation of Eq. 52");
  if (h->p.precision == LBM_FP64)
    return adjoint_t<double, double, double>(h, nsteps, ckpt_every, loss, dL_dphi, dL_dHv);
  if (h->p.precision == LBM_FP32SR)
    return adjoint_t<double, LTNE_ADJ32_LAM, LTNE_ADJ32_MATH>(h, nsteps, ckpt_every, loss, dL_dphi, dL_dHv);
  return adjoint_t<float, LTNE_ADJ32_LAM, LTNE_ADJ32_MATH>(h, nsteps, ckpt_every, loss, dL_dphi, dL_dHv);
}

extern "C" {

int lbm_ltne_destroy(lbm_ltne_t h) {
  if (!h) return LBM_OK;
  (void)hipStreamSynchronize(h->stream);
  release(h);
  return LBM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Binary64 sums of caller-held macro fields without any allocation.
//
// The partial sums and the result live in a file-scope device array: each
// GPU the library runs on holds one copy (about 66 KB) until the process
// ends.  Host code never uses the array's name as an address: at the first
// call on a device, with that device current, hipGetSymbolAddress gives the
// device's own address, which is kept per device.
namespace {
constexpr int kNoAllocMaxDevices = 64;
constexpr size_t kNoAllocScratchDoubles = static_cast<size_t>(kSumBlocks) * kSums + 32;
__device__ __align__(256) double scratch[kNoAllocScratchDoubles];
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kNoAllocMaxDevices] = {};

int scratch_for_current_device(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return set_error(LBM_EUNSUPPORTED, "device %d beyond the %d devices this entry point supports", dev,
                     kNoAllocMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(LBM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}
}  // namespace

extern "C" int lbm_ltne_macro_sums_noalloc(const lbm_ltne_params* p, const void* mac, const void* prev,
                                           const void* phi_field, void* hip_stream, double* mass,
                                           double* energy, double* residual) {
  clear_error();
  if (!p || !mac || !prev) return set_error(LBM_EINVAL, "params, mac and prev must not be NULL");
  if (p->precision < LBM_FP64 || p->precision > LBM_FP32SR)
    return set_error(LBM_EINVAL, "precision %d is not a precision form", p->precision);
  if (p->nx < 1 || p->ny < 1) return set_error(LBM_EINVAL, "lattice %d x %d is empty", p->nx, p->ny);
  const long long n = static_cast<long long>(p->nx) * p->ny;
  if (n > (1LL << 30)) return set_error(LBM_EINVAL, "lattice %d x %d exceeds 2^30 nodes", p->nx, p->ny);
  if (!phi_field && !(p->phi > 0.0 && p->phi < 1.0))
    return set_error(LBM_EINVAL, "phi = %g not in (0, 1)", p->phi);
  if (!(p->sigma > 0.0)) return set_error(LBM_EINVAL, "sigma = %g must be > 0", p->sigma);
  double* scr = nullptr;
  int rc = scratch_for_current_device(&scr);
  if (rc != LBM_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double* partial = scr;
  double* result = scr + static_cast<size_t>(kSumBlocks) * kSums;
  const int blocks = static_cast<int>(std::min<long long>(kSumBlocks, (n + kBlock - 1) / kBlock));
  if (compute_bytes(p->precision) == 8) {
    hipLaunchKernelGGL((sums_kernel<double>), dim3(blocks), dim3(kBlock), 0, st, static_cast<const double*>(mac),
                       static_cast<const double*>(prev), static_cast<const double*>(phi_field), p->phi,
                       p->sigma, n, n, partial);
  } else {
    hipLaunchKernelGGL((sums_kernel<float>), dim3(blocks), dim3(kBlock), 0, st, static_cast<const float*>(mac),
                       static_cast<const float*>(prev), static_cast<const float*>(phi_field), p->phi,
                       p->sigma, n, n, partial);
  }
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(kBlock), 0, st, partial, blocks, result);
  HIP_TRY(hipGetLastError());
  double s[kSums];
  HIP_TRY(hipMemcpyAsync(s, result, sizeof(s), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  auto rel = [](double num, double den) { return den > 0.0 ? num / den : num; };
  if (mass) *mass = s[0];
  if (energy) *energy = s[1];
  if (residual) *residual = std::max(rel(s[2], s[3]), std::max(rel(s[4], s[5]), rel(s[6], s[7])));
  if (!std::isfinite(s[0]) || !std::isfinite(s[1]))
    return set_error(LBM_EDIVERGED, "mass %g, energy %g", s[0], s[1]);
  return LBM_OK;
}
