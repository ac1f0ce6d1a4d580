// Two fused time steps per launch for the FP32 form (binary32 storage,
// binary32 flow and binary64 temperature arithmetic) and the FP64 form (the
// same code over binary64 populations).  The single-step kernel is bound by
// memory traffic; computing two steps per pass over the populations halves
// the traffic per lattice-node update.
//
// Each wavefront owns a strip of columns and a chunk of rows and marches
// down the rows.  Lane l holds column x0 - H + l (H = 1 on a periodic x axis,
// 2 with x walls, whose nodes pull from two columns inward).  At row y it
//   1. updates its column at row y + 1 to time t + 1 from device memory (the
//      ordinary pull and node update), keeping the 19 results in registers:
//      a window of three rows, y - 1, y, y + 1;
//   2. gathers the pulls of its node at row y from the window, the column
//      offsets by cross-lane permutes;
//   3. updates the node at row y to time t + 2 and stores it.
// The lanes at the strip edges only feed their neighbours.  A wall row takes
// the pulls of its inward neighbour row (non-equilibrium extrapolation), so
// it is updated at that row's step.  The results equal two single steps bit
// for bit: the same node update, and values of the storage type in
// registers instead of a round trip through memory.
#pragma once

#include "step_kernel.hpp"

namespace ltne {

// Rows per chunk.  A chunk recomputes two halo rows at the intermediate time
// level, so taller chunks do less redundant work but leave fewer wavefronts
// in flight.  A single lattice takes the tallest of kStep2RowChoices that
// still yields kStep2TargetWaves wavefronts; a batch of lattices (many small
// ones) uses kBatch2Rows.  The binary64 kernel holds one wavefront per SIMD
// (it needs more than half the register file), so it fills the chip with
// half the wavefronts and may take chunks of 64 rows.  LTNE_STEP2_ROWS
// forces one height (experiments).
constexpr int kStep2RowChoices[] = {64, 32, 24, 16, 12, 8};
constexpr int kStep2MaxRows32 = 32;  // tallest chunk of the binary32 kernel
constexpr int kStep2MinRows = 8;
// chunk heights a batch may take (chosen per size class by the autotuner)
constexpr int kBatch2RowChoices[] = {32, 24, 16, 12, 8};
#ifndef LTNE_STEP2_TARGET_WAVES
#define LTNE_STEP2_TARGET_WAVES 16384
#endif
constexpr int kStep2TargetWaves = LTNE_STEP2_TARGET_WAVES;
#ifndef LTNE_BATCH2_ROWS
#define LTNE_BATCH2_ROWS 16
#endif
constexpr int kBatch2Rows = LTNE_BATCH2_ROWS;
// Threads per workgroup of the two-step kernels (whole wavefronts; each
// wavefront works on its own strip and chunk).
#ifndef LTNE_STEP2_BLOCK
#define LTNE_STEP2_BLOCK 256
#endif
constexpr int kStep2Block = LTNE_STEP2_BLOCK;
static_assert(kStep2Block % 64 == 0 && kStep2Block <= 1024, "whole wavefronts per workgroup");
// Threads per workgroup of the batched two-step kernel: one wavefront, so a
// compute unit starts a new strip as soon as any of its wavefronts ends (the
// strips of small lattices differ in length; on the 256-cavity batch one
// wavefront per workgroup was 5% faster than four, while a single large
// lattice runs faster with four neighbouring strips per workgroup).
#ifndef LTNE_BATCH2_BLOCK
#define LTNE_BATCH2_BLOCK 64
#endif
constexpr int kBatch2Block = LTNE_BATCH2_BLOCK;
static_assert(kBatch2Block % 64 == 0 && kBatch2Block <= 1024, "whole wavefronts per workgroup");
// Stores of the two-step kernels: plain, so the L2 merges the partial cache
// lines written by neighbouring strips (62 or 61 columns wide) before they go
// to HBM; non-temporal stores were 5% slower on the 8192^2 layer.
#ifndef LTNE_STEP2_NT_STORE
#define LTNE_STEP2_NT_STORE 0
#endif
constexpr bool kStep2NtStore = LTNE_STEP2_NT_STORE != 0;
// Two-step launches need this many wavefronts at the smallest chunk height
// to hide the serial chain of rows each one runs; with fewer, single steps
// are faster (the FP32 layer: 640^2 with 880 wavefronts 2% slower in pairs,
// 768^2 with 1248 2% faster).  The binary64 kernel runs one wavefront per
// SIMD and needs more (the FP64 layer: 1024^2 with 2176 wavefronts 2% slower
// in pairs, 1152^2 with 2736 13% faster).
#ifndef LTNE_STEP2_MIN_WAVES
#define LTNE_STEP2_MIN_WAVES 1024
#endif
#ifndef LTNE_STEP2_MIN_WAVES_64
#define LTNE_STEP2_MIN_WAVES_64 2560
#endif

// Lanes left of a strip's first output column: one on a periodic x axis,
// two with x walls (a wall node pulls from two columns inward).
__host__ __device__ constexpr int step2_halo(int periodic_x) { return periodic_x ? 1 : 2; }
__host__ __device__ constexpr int step2_out(int periodic_x) { return 63 - step2_halo(periodic_x); }
__host__ __device__ constexpr int step2_waves(int nx, int ny, int periodic_x, int rows) {
  return ((nx + step2_out(periodic_x) - 1) / step2_out(periodic_x)) * ((ny + rows - 1) / rows);
}
// Chunk height of a single lattice's two-step launches (elem_bytes: 4 or 8,
// the storage type).
inline int step2_rows(int nx, int ny, int periodic_x, size_t elem_bytes) {
#ifdef LTNE_STEP2_ROWS
  (void)nx, (void)ny, (void)periodic_x, (void)elem_bytes;
  return LTNE_STEP2_ROWS;
#else
  const bool wide = elem_bytes == 8;
  const int target = wide ? kStep2TargetWaves / 2 : kStep2TargetWaves;
  for (int r : kStep2RowChoices)
    if ((wide || r <= kStep2MaxRows32) && step2_waves(nx, ny, periodic_x, r) >= target) return r;
  return kStep2MinRows;
#endif
}

// Launch geometry of the two-step kernel.
struct Step2Map {
  int halo;     // lanes left of the first output column (1 or 2)
  int out;      // output columns per strip (63 - halo)
  int nstrips;  // strips across the lattice
  int rows;     // rows per chunk
  int nchunks;  // chunks down the lattice
  int nwaves;   // nstrips * nchunks
  int per_xcd;  // workgroups per XCD
};

// Loads and stores of the two-step kernel through buffer resources: one
// resource per lattice row (its 19 population rows), the population's offset
// in the scalar offset operand and the lane's column in the vector offset,
// so no vector instruction is spent forming 64-bit addresses.
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const S* row, long long rs) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(row), static_cast<short>(0),
                                           static_cast<int>(rs * static_cast<long long>(sizeof(S))), 0x00020000);
}

// One element (binary32 or binary64) through a buffer resource.
template <typename S>
__device__ __forceinline__ S buf_load(__amdgpu_buffer_rsrc_t r, int vo, int so) {
  if constexpr (sizeof(S) == 8)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  else
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
template <int Aux, typename S>
__device__ __forceinline__ void buf_store(S v, __amdgpu_buffer_rsrc_t r, int vo, int so) {
  if constexpr (sizeof(S) == 8) {
    using W = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(W, v), r, vo, so, Aux);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, vo, so, Aux);
  }
}

template <typename S>
struct BufPull {
  const S* __restrict__ src;
  __device__ __forceinline__ void operator()(int xc, int yc, const StepConsts<S>& k, S (&v)[kPlanes]) const {
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
    const __amdgpu_buffer_rsrc_t r0 = row_rsrc(src + yu * k.rs, k.rs);
    const __amdgpu_buffer_rsrc_t rm = row_rsrc(src + ym * k.rs, k.rs);
    const __amdgpu_buffer_rsrc_t rp = row_rsrc(src + yp * k.rs, k.rs);
    constexpr int E = sizeof(S);
    const int Q = static_cast<int>(k.qs) * E;
    const int oc = xc * E, om = xm * E, op = xp * E;
    auto ld = [&](__amdgpu_buffer_rsrc_t r, int vo, int q) { return buf_load<S>(r, vo, q * Q); };
    v[0] = ld(r0, oc, 0);
    v[1] = ld(r0, om, 1);
    v[2] = ld(rm, oc, 2);
    v[3] = ld(r0, op, 3);
    v[4] = ld(rp, oc, 4);
    v[5] = ld(rm, om, 5);
    v[6] = ld(rm, op, 6);
    v[7] = ld(rp, op, 7);
    v[8] = ld(rp, om, 8);
    v[9] = ld(r0, oc, 9);
    v[10] = ld(r0, om, 10);
    v[11] = ld(rm, oc, 11);
    v[12] = ld(r0, op, 12);
    v[13] = ld(rp, oc, 13);
    v[14] = ld(r0, oc, 14);
    v[15] = ld(r0, om, 15);
    v[16] = ld(rm, oc, 16);
    v[17] = ld(r0, op, 17);
    v[18] = ld(rp, oc, 18);
  }
};

// One field value (porosity or H_v) of node (xc, yc) through a buffer
// resource over the field's row, so a wavefront's loads are all of one kind.
template <typename S>
__device__ __forceinline__ S buf_field(const S* __restrict__ f, int xc, int yc, int nx) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<S*>(f + static_cast<long long>(__builtin_amdgcn_readfirstlane(yc)) * nx), static_cast<short>(0),
      nx * static_cast<int>(sizeof(S)), 0x00020000);
  return buf_load<S>(r, xc * static_cast<int>(sizeof(S)), 0);
}

template <int F, typename S>
__device__ __forceinline__ CenterFields<S> buf_center(const S* __restrict__ phi_field, const S* __restrict__ hv_field,
                                                      int xc, int yc, const StepConsts<S>& k) {
  return {(F & kPhiField) ? buf_field(phi_field, xc, yc, k.nx) : k.phi_u,
          (F & kHvField) ? buf_field(hv_field, xc, yc, k.nx) : k.hv_u};
}

template <typename S>
struct BufPut {
  // cache policy of the stores: the non-temporal bit when kStep2NtStore
  static constexpr int kNtAux = kStep2NtStore ? 2 : 0;
  S* __restrict__ dst;
  __amdgpu_buffer_rsrc_t r;
  int vo = 0, Q = 0;
  __device__ __forceinline__ void begin(int x, int y, const StepConsts<S>& k) {
    r = row_rsrc(dst + static_cast<long long>(__builtin_amdgcn_readfirstlane(y)) * k.rs, k.rs);
    vo = x * static_cast<int>(sizeof(S));
    Q = static_cast<int>(k.qs) * static_cast<int>(sizeof(S));
  }
  __device__ __forceinline__ void st(int i, S v) { buf_store<kNtAux>(v, r, vo, i * Q); }
  template <typename VA, typename VB>
  __device__ __forceinline__ void pair(int i, VA va, VA, int j, VB vb, VB, uint32_t w, half2_t&) {
    st(i, to_storage<S>(va, w << 16));
    st(j, to_storage<S>(vb, w));
  }
  template <typename V>
  __device__ __forceinline__ void single(int i, V v, V, uint32_t w) { st(i, to_storage<S>(v, w)); }
};

// Copies a constant block into LDS, one 8-byte word per thread.
template <typename K>
__device__ __forceinline__ void copy_to_lds(const K& src, K& dst) {
  static_assert(sizeof(K) % 8 == 0 && sizeof(K) / 8 <= 64, "constant block too large");
  const int t = static_cast<int>(threadIdx.x);
  if (t < static_cast<int>(sizeof(K) / 8))
    reinterpret_cast<unsigned long long*>(&dst)[t] = reinterpret_cast<const unsigned long long*>(&src)[t];
}

// Put into registers: the 19 post-collision populations of one node, rounded
// to the storage type exactly as a store to memory would round them (the
// binary64 temperature values of the FP32 form stochastically, with the
// same random words), so the intermediate time level equals a single step's.
template <typename C>
struct RegPut {
  C* v;
  __device__ __forceinline__ void begin(int, int, const StepConsts<C>&) {}
  template <typename VA, typename VB>
  __device__ __forceinline__ void pair(int i, VA va, VA, int j, VB vb, VB, uint32_t w, half2_t&) {
    v[i] = to_storage<C>(va, w << 16);
    v[j] = to_storage<C>(vb, w);
  }
  template <typename V>
  __device__ __forceinline__ void single(int i, V val, V, uint32_t r) { v[i] = to_storage<C>(val, r); }
};

// Pull from registers: populations already gathered for the node.
template <typename C>
struct RegPull {
  const C* g;
  __device__ __forceinline__ void operator()(int, int, const StepConsts<C>&, C (&v)[kPlanes]) const {
#pragma unroll
    for (int i = 0; i < kPlanes; ++i) v[i] = g[i];
  }
};

// A copy of fields already used (so loaded) that the compiler must keep in
// registers of its own.  Carrying loaded values from row to row otherwise
// lets it load the next row's values into other registers and copy them back
// at the end of the row, and that copy waits for every memory access issued
// before it, stores included.  Uniform fields (not loaded) are left as they
// are, so that what derives from them stays hoisted out of the row loop.
template <int F, typename S>
__device__ __forceinline__ CenterFields<S> detach(CenterFields<S> f) {
  if constexpr ((F & kPhiField) != 0) asm volatile("" : "+v"(f.phi));
  if constexpr ((F & kHvField) != 0) asm volatile("" : "+v"(f.hv));
  return f;
}

// The work of one lane of a strip and chunk: its columns, the chunk's rows,
// and the three parts of the update (fetch, intermediate level, output).
template <typename S, int F>
struct Step2Lane {
  const S* __restrict__ src;
  S* __restrict__ dst;
  const S* __restrict__ phi_field;
  const S* __restrict__ hv_field;
  S* __restrict__ mac;  // macros of the second step (F & kMacros)
  const StepConsts<S>& k;
  const ThermalK<double>& kt;
  uint32_t step;
  int lane, col, xo, dx, y_lo, y_hi;
  bool colok, outlane;
  // the intermediate level writes no macros
  static constexpr int FA = F & ~kMacros;

  __device__ __forceinline__ Step2Lane(const S* __restrict__ src_, S* __restrict__ dst_,
                                       const S* __restrict__ phi_, const S* __restrict__ hv_,
                                       S* __restrict__ mac_, const StepConsts<S>& k_,
                                       const ThermalK<double>& kt_, const int strip, const int chunk, const int rows,
                                       const uint32_t step_)
      : src(src_), dst(dst_), phi_field(phi_), hv_field(hv_), mac(mac_), k(k_), kt(kt_), step(step_) {
    lane = static_cast<int>(threadIdx.x) & 63;
    const int nx = k.nx, ny = k.ny;
    const int halo = step2_halo(k.px), out = step2_out(k.px);
    const int x0 = strip * out;
    // column of this lane at time t + 1
    col = x0 - halo + lane;
    colok = true;
    if (k.px) {
      col %= nx;
      if (col < 0) col += nx;
    } else {
      colok = col >= 0 && col < nx;
    }
    // output column and the column offset of its pulls (x walls pull inward)
    xo = x0 - halo + lane;
    outlane = lane >= halo && lane < halo + out && xo < nx;
    dx = (!k.px && xo == 0) ? 1 : ((!k.px && xo == nx - 1) ? -1 : 0);
    // rows of this chunk; a wall row is updated with its inward neighbour row
    y_lo = chunk * rows;
    y_hi = y_lo + rows < ny ? y_lo + rows : ny;
    if (!k.py) {
      y_lo = y_lo > 1 ? y_lo : 1;
      y_hi = y_hi < ny - 1 ? y_hi : ny - 1;
    }
  }

  // row r at this lane's column, wrapped on a periodic axis; ok: a node exists
  __device__ __forceinline__ int row_of(int r, bool& ok) const {
    ok = colok;
    if (k.py) return r < 0 ? r + k.ny : (r >= k.ny ? r - k.ny : r);
    ok = ok && r >= 0 && r < k.ny;
    return r;
  }

  // the pulls of node (col, r) at time t (a wall node pulls those of its
  // inward neighbour) and the porosity and H_v there, issued ahead of their
  // use so the loads overlap arithmetic
  __device__ __forceinline__ void fetch(int r, S (&v)[kPlanes], CenterFields<S>& cf) const {
    bool ok;
    r = row_of(r, ok);
    if (ok) {
      const int nx = k.nx, ny = k.ny;
      const int xc = (!k.px && col == 0) ? 1 : ((!k.px && col == nx - 1) ? nx - 2 : col);
      const int yc = (!k.py && r == 0) ? 1 : ((!k.py && r == ny - 1) ? ny - 2 : r);
      const BufPull<S> gpull{src};
      gpull(xc, yc, k, v);
      cf = buf_center<F>(phi_field, hv_field, xc, yc, k);
    }
  }

  // node (col, r) at time t + 1 from its fetched pulls and fields into w;
  // zeros where there is no node
  __device__ __forceinline__ void advance(int r, const S (&v)[kPlanes], const CenterFields<S>& cf,
                                          S (&w)[kPlanes]) const {
    bool ok;
    r = row_of(r, ok);
    if (ok) {
      const RegPull<S> rp{v};
      RegPut<S> put{w};
      node_update_with<S, S, FA>(col, r, rp, put, phi_field, hv_field, nullptr, nullptr, nullptr, k, step,
                                        nullptr, kt, &cf);
    } else {
#pragma unroll
      for (int i = 0; i < kPlanes; ++i) w[i] = S(0);
    }
  }

  // node (xo, y) at time t + 2 from its gathered pulls g (time t + 1) and the
  // fields fy of its pulled node, stored; then the wall row it feeds (one
  // call site)
  __device__ __forceinline__ void output(int y, const S (&g)[kPlanes], const CenterFields<S>& fy) const {
    const RegPull<S> rpull{g};
    BufPut<S> put{dst};
    const int ny = k.ny;
    const int nrep = (!k.py && (y == 1 || y == ny - 2)) ? 2 : 1;
#pragma nounroll
    for (int rep = 0; rep < nrep; ++rep) {
      const int yy = rep == 0 ? y : (y == 1 ? 0 : ny - 1);
      node_update_with<S, S, F>(xo, yy, rpull, put, phi_field, hv_field, mac, nullptr, nullptr, k,
                                        step + 1u, nullptr, kt, &fy);
    }
  }
};

// One wavefront's strip and chunk of a lattice.  At row y it
//   1. updates its column at row y + 1 to time t + 1 from device memory,
//      keeping the 19 results in registers: a window of rows y - 1, y, y + 1;
//   2. gathers the pulls of its node at row y from the window, the column
//      offsets by cross-lane permutes;
//   3. updates the node at row y to time t + 2 and stores it.
// kt: the lattice's temperature constants, a copy in LDS (see the kernels).
// mac: the macros of the second step (F & kMacros), else unused.
template <int F, typename S>
__device__ __forceinline__ void step2_wave(const S* __restrict__ src, S* __restrict__ dst,
                                           const S* __restrict__ phi_field, const S* __restrict__ hv_field,
                                           S* __restrict__ mac, const StepConsts<S>& k,
                                           const ThermalK<double>& kt, const int strip, const int chunk,
                                           const int rows, const uint32_t step) {
  const Step2Lane<S, F> L(src, dst, phi_field, hv_field, mac, k, kt, strip, chunk, rows, step);
  const int y_lo = L.y_lo, y_hi = L.y_hi, lane = L.lane, dx = L.dx;
  if (y_lo >= y_hi) return;

  S wa[kPlanes], wb[kPlanes], wc[kPlanes];  // time t + 1 at rows y - 1, y, y + 1
  S pa[kPlanes], pb[kPlanes];               // fetched pulls of two rows
  CenterFields<S> fa{}, fb{};               // and the fields fetched with them
  L.fetch(y_lo - 1, pa, fa);
  L.fetch(y_lo, pb, fb);
  L.advance(y_lo - 1, pa, fa, wa);
  L.fetch(y_lo + 1, pa, fa);
  L.advance(y_lo, pb, fb, wb);
  // fields of node (col, y), the pulled node of the output update at row y
  // (on an output lane col = xo, and a wall row pulls from row y as well)
  CenterFields<S> fy = detach<F>(fb);
#pragma nounroll
  for (int y = y_lo; y < y_hi; ++y) {
    L.advance(y + 1, pa, fa, wc);
    const CenterFields<S> fn = detach<F>(fa);
    if (y + 1 < y_hi) L.fetch(y + 2, pa, fa);
    // pulls of node (xo + dx, y) at time t + 1: population i from column
    // xo + dx - e_ix (lane offset) and row y - e_iy (window row)
    S g[kPlanes];
#pragma unroll
    for (int i = 0; i < kPlanes; ++i) {
      const int q = i < 9 ? i : (i < 14 ? i - 9 : i - 14);
      const S v = vel_y(q) == 1 ? wa[i] : (vel_y(q) == -1 ? wc[i] : wb[i]);
      const int sl = (lane + dx - vel_x(q)) & 63;
      g[i] = __shfl(v, sl, 64);
    }
    if (L.outlane) L.output(y, g, fy);
#pragma unroll
    for (int i = 0; i < kPlanes; ++i) {
      wa[i] = wb[i];
      wb[i] = wc[i];
    }
    fy = fn;
  }
}

template <typename S, int F>
__global__ __launch_bounds__(kStep2Block) void step2_kernel(const S* __restrict__ src, S* __restrict__ dst,
                                                       const S* __restrict__ phi_field,
                                                       const S* __restrict__ hv_field,
                                                       S* __restrict__ mac, const StepConsts<S> k,
                                                       const Step2Map m, const uint32_t step) {
  const int b = blockIdx.x;
  const int blk = (b & (kXcds - 1)) * m.per_xcd + (b >> 3);
  const int wave = blk * (kStep2Block / 64) + (static_cast<int>(threadIdx.x) >> 6);
  // the binary64 temperature constants as vector operands from LDS rather
  // than scalar registers (which the kernel runs short of)
  __shared__ ThermalK<double> kt;
  copy_to_lds(k.td, kt);
  __syncthreads();
  if (wave >= m.nwaves) return;  // whole wavefronts
  step2_wave<F>(src, dst, phi_field, hv_field, mac, k, kt, wave % m.nstrips, wave / m.nstrips, m.rows, step);
}

}  // namespace ltne
