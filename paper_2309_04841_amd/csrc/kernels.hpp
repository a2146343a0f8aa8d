// kernels.hpp -- HIP kernels of the QAOA hot path for gfx950 (CDNA4, wave64).
//
//   qaoa_sweep_kernel   fused tile sweep: [|+> init | load] -> per layer
//                       {phase exp(-i g c) (Section 3.1), mixer gates
//                       cos(b) I - i sin(b) X on the tile's active qubits
//                       (Section 3.2, Algorithms 1-2)} -> [E partials] -> store
//   fwht_sweep_kernel   same tiling, butterfly (u, v) -> (u + v, u - v): the
//                       unnormalised Walsh-Hadamard transform that turns the
//                       sparse term weights into the cost vector (Eq. (1))
//   expectation_kernel  E = sum |psi|^2 c and sum |psi|^2 (Section 3.1), FP64
//   finalize_kernel     fixed-order sum of per-block partials
//   helpers             fill, scatter, integer range check, narrowing
//
// All reductions have a fixed order (no atomics), so results are bitwise
// reproducible run to run.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "tile.hpp"

namespace qk {

constexpr int kMaxLayersPerLaunch = 32;
// rows prepared per chunk of host angles: the chunk's layers and the next one
// (a fused sweep at the end of a chunk reads the following layer's row)
constexpr int kPrepRows = kMaxLayersPerLaunch + 1;
constexpr int kScatterChunk = 240;

enum : int { F_INIT = 1, F_PHASE = 2, F_EXPV = 4, F_FUSE = 8 };

// ----------------------------------------------------------------------------
// element policies
// ----------------------------------------------------------------------------
// The state is streamed once per sweep: its loads and stores carry the
// non-temporal hint so they do not displace the cost vector and tables, which
// are re-read every layer (except in 2^14-element complex128 tiles, below).
// LDS accesses by byte address.  The tile kernels declare no static LDS, so
// their dynamic LDS (smem_raw) starts at address 0 and a tile position's byte
// offset is its LDS address; addressing it directly saves the per-access add of
// the smem_raw symbol, which the compiler cannot fold.  (A CPU test checks that
// these kernels have no static LDS.)
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) dvec2 lds_f64x2;
typedef __attribute__((address_space(3))) fvec2 lds_f32x2;
__device__ __forceinline__ lds_f64* lds_d(uint32_t addr) { return (lds_f64*)(uintptr_t)addr; }

struct C128 {  // complex128: (double re, double im)
  using L = double2;
  using R = double;    // arithmetic type of the forward sweeps
  using Tab = double2; // their LDS phase-table entries
  static constexpr bool kDualPrecision = false;
  static constexpr int kBytes = 16;
  static constexpr int kLdsBytes = 16;   // LDS bytes per tile element
  static constexpr bool kSplit = false;  // exchanges move whole elements
  static constexpr int kAdjMinWavesPerSimd = 2;  // reverse sweeps
  static constexpr int kMaxThreads = 512;
  // 64 KiB tiles + tables: two workgroups per CU by LDS, up to 256 VGPRs.
  // (Measured: four waves per SIMD at 128 VGPRs, with split exchanges to fit
  // four workgroups, was slower: the fused kernels spill there.)
  static constexpr int kMinWavesPerSimd = 2;
  __device__ static __forceinline__ void load(const void* p, uint64_t x, double& r, double& i) {
    const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p) + x);
    r = v.x; i = v.y;
  }
  __device__ static __forceinline__ void store(void* p, uint64_t x, double r, double i) {
    const dvec2 v = {r, i};
    __builtin_nontemporal_store(v, reinterpret_cast<dvec2*>(p) + x);
  }
  // LDS accessors take byte offsets (the swizzled position times the entry size)
  __device__ static __forceinline__ void lput(L*, uint32_t off, double r, double i) {
    const dvec2 v = {r, i};
    *(lds_f64x2*)(uintptr_t)off = v;
  }
  __device__ static __forceinline__ void lget(const L*, uint32_t off, double& r, double& i) {
    const dvec2 v = *(lds_f64x2*)(uintptr_t)off;
    r = v.x; i = v.y;
  }
};

// complex64 storage.  The forward sweeps compute in FP32 (R, Tab), which leaves
// out the conversions at every load, store and window change (LABS n=31
// p=10: 5.86 -> 6.54 evaluations/s), except for layers with |tan beta| above
// kTanMaxF32; the reverse (gradient) sweeps and the XY kernels keep FP64
// registers (the double overloads below).
struct C64 {
  using L = float2;
  using R = float;
  using Tab = float2;
  static constexpr bool kDualPrecision = true;  // FP64 sweeps for large |tan beta|
  static constexpr int kBytes = 8;
  static constexpr int kLdsBytes = 8;
  static constexpr bool kSplit = false;
  static constexpr int kMaxThreads = 512;
  // 512-thread tiles: four waves per SIMD keep two workgroups resident per CU
  static constexpr int kMinWavesPerSimd = 4;
  static constexpr int kAdjMinWavesPerSimd = 4;  // reverse sweeps
  __device__ static __forceinline__ void load(const void* p, uint64_t x, double& r, double& i) {
    const fvec2 v = __builtin_nontemporal_load(reinterpret_cast<const fvec2*>(p) + x);
    r = (double)v.x; i = (double)v.y;
  }
  __device__ static __forceinline__ void store(void* p, uint64_t x, double r, double i) {
    const fvec2 v = {(float)r, (float)i};
    __builtin_nontemporal_store(v, reinterpret_cast<fvec2*>(p) + x);
  }
  __device__ static __forceinline__ void lput(L*, uint32_t off, double r, double i) {
    const fvec2 v = {(float)r, (float)i};
    *(lds_f32x2*)(uintptr_t)off = v;
  }
  __device__ static __forceinline__ void lget(const L*, uint32_t off, double& r, double& i) {
    const fvec2 v = *(lds_f32x2*)(uintptr_t)off;
    r = (double)v.x; i = (double)v.y;
  }
  __device__ static __forceinline__ void load(const void* p, uint64_t x, float& r, float& i) {
    const fvec2 v = __builtin_nontemporal_load(reinterpret_cast<const fvec2*>(p) + x);
    r = v.x; i = v.y;
  }
  __device__ static __forceinline__ void store(void* p, uint64_t x, float r, float i) {
    const fvec2 v = {r, i};
    __builtin_nontemporal_store(v, reinterpret_cast<fvec2*>(p) + x);
  }
  __device__ static __forceinline__ void lput(L*, uint32_t off, float r, float i) {
    const fvec2 v = {r, i};
    *(lds_f32x2*)(uintptr_t)off = v;
  }
  __device__ static __forceinline__ void lget(const L*, uint32_t off, float& r, float& i) {
    const fvec2 v = *(lds_f32x2*)(uintptr_t)off;
    r = v.x; i = v.y;
  }
};

// complex128 in tiles of up to 2^14 elements (256 KiB, more than the LDS):
// 1024 threads of 16 elements; a window change moves the real parts, then the
// imaginary parts, through one 128 KiB buffer of doubles.  Used when the larger
// tile saves a sweep per layer.
struct C128W : C128 {
  // Ordinary (temporal) loads and stores: the sweep with 64-byte runs reads and
  // writes each 128-byte line in halves from two workgroups, and a line kept in
  // L2 from its load takes both halves of the store before it is written back
  // (measured, n=26 complex128: 160.8 -> 167.0 evaluations/s; temporal loads
  // or stores alone gained nothing)
  __device__ static __forceinline__ void load(const void* p, uint64_t x, double& r, double& i) {
    const dvec2 v = *(reinterpret_cast<const dvec2*>(p) + x);
    r = v.x; i = v.y;
  }
  __device__ static __forceinline__ void store(void* p, uint64_t x, double r, double i) {
    const dvec2 v = {r, i};
    *(reinterpret_cast<dvec2*>(p) + x) = v;
  }
  static constexpr int kLdsBytes = 8;
  static constexpr bool kSplit = true;
  static constexpr int kMaxThreads = 1024;
  static constexpr int kMinWavesPerSimd = 4;  // one 16-wave workgroup per CU
};

// Cost-vector policies.  `get` returns the stored value as a double (the
// cost is get() + offset).  For integer storage, `tab_index` maps the stored
// value to an index u in [0, 2^16) of the per-layer phase table, or returns a
// negative value when the table does not cover it (then sincos is used).
struct DI32 {
  static constexpr bool kTable = true;
  __device__ static __forceinline__ int32_t load_raw(const void* p, uint64_t x) { return reinterpret_cast<const int32_t*>(p)[x]; }
  static constexpr bool kAlwaysInTable = false;
  __device__ static __forceinline__ double get(const void* p, uint64_t x) {
    return (double)reinterpret_cast<const int32_t*>(p)[x];
  }
  __device__ static __forceinline__ int32_t raw(const void* p, uint64_t x) {
    return reinterpret_cast<const int32_t*>(p)[x];
  }
  // table covers stored values in [-2^15, 2^15)
  __device__ static __forceinline__ int32_t tab_index(int32_t v) {
    const uint32_t u = (uint32_t)v + 32768u;
    return u < 65536u ? (int32_t)u : -1;
  }
  static constexpr double kTableBase = -32768.0;
  static constexpr int kTabLds = 288;  // LDS entries: HI|MID|LO, F1|MID|LO or F3|F2M|F2L
  static constexpr bool kPack16 = false;
  using RawT = int32_t;
  __device__ static __forceinline__ double value(RawT r) { return (double)r; }
};
struct DU16 {
  static constexpr bool kTable = true;
  __device__ static __forceinline__ int32_t load_raw(const void* p, uint64_t x) { return (int32_t)reinterpret_cast<const uint16_t*>(p)[x]; }
  static constexpr bool kAlwaysInTable = true;
  __device__ static __forceinline__ double get(const void* p, uint64_t x) {
    return (double)reinterpret_cast<const uint16_t*>(p)[x];
  }
  __device__ static __forceinline__ int32_t raw(const void* p, uint64_t x) {
    return (int32_t)reinterpret_cast<const uint16_t*>(p)[x];
  }
  __device__ static __forceinline__ int32_t tab_index(int32_t v) { return v; }
  static constexpr double kTableBase = 0.0;
  static constexpr int kTabLds = 288;
  static constexpr bool kPack16 = true;  // two stored values fit one 32-bit register
  using RawT = int32_t;
  __device__ static __forceinline__ double value(RawT r) { return (double)r; }
};
struct DF64 {
  static constexpr bool kTable = false;
  __device__ static __forceinline__ double load_raw(const void* p, uint64_t x) { return reinterpret_cast<const double*>(p)[x]; }
  static constexpr bool kAlwaysInTable = false;
  __device__ static __forceinline__ double get(const void* p, uint64_t x) {
    return reinterpret_cast<const double*>(p)[x];
  }
  __device__ static __forceinline__ int32_t raw(const void*, uint64_t) { return 0; }
  __device__ static __forceinline__ int32_t tab_index(int32_t) { return -1; }
  static constexpr double kTableBase = 0.0;
  static constexpr int kTabLds = 0;
  static constexpr bool kPack16 = false;
  using RawT = double;
  __device__ static __forceinline__ double value(RawT r) { return r; }
};

// Phase tables for integer cost vectors.  With u = stored - base in [0, 2^16)
// the cost is c = u + base + offset, and
//   exp(-i g c) = HI[u >> 8] * MID[(u >> 4) & 15] * LO[u & 15],
//   HI[m] = exp(-i g (256 m + base + offset)),  MID[j] = exp(-i g 16 j),
//   LO[j] = exp(-i g j),
// each entry from one sincos of an exactly representable integer times g.
// MID and LO are 16 entries of 16 bytes: each occupies every LDS bank exactly
// once, so their gathers never conflict (a 256-entry low table did, at
// random indices); HI sees few distinct indices for costs of small range.
// int32 values outside that range use the bytes b0..b3 of the stored value v
// (two's complement, b3 signed), in two passes of the same three-table product:
//   exp(-i g (v + offset)) = (F1[b1] * MID[b0 >> 4] * LO[b0 & 15])
//                          * (F3[b3] * F2M[b2 >> 4] * F2L[b2 & 15]),
//   F1[m] = exp(-i g 256 m),  F2M[j] = exp(-i g 2^20 j),  F2L[j] = exp(-i g 2^16 j),
//   F3[m] = exp(-i g (2^24 s(m) + offset)),  s(m) = m - 256 [m >= 128].
// A layer's row holds HI, MID, LO, F1, F3, F2M, F2L (double2 (cos, -sin)).
constexpr int kTabEntries = 288;  // HI, MID, LO: the part staged for in-range values
constexpr int kTabRow = 832;      // row stride: HI 256, MID 16, LO 16, F1 256, F3 256, F2M 16, F2L 16
constexpr int kParamRow = 4;      // doubles per parameter row: gamma, cos beta, sin beta, tan beta

// Per-layer parameters, computed on the device for every path so that batched
// and single evaluations use bit-identical values: row r gets
// pset[4r..4r+3] = (gamma, cos beta, sin beta, tan beta) and, when tab != nullptr, the
// phase tables tab[kTabRow r ..].  Angles come from device arrays (gamma_d, beta_d)
// or, when those are null, from the kernel arguments (at most kPrepRows rows).
struct PrepArgs {
  const double* gamma_d;
  const double* beta_d;
  double* pset;
  double2* tab;
  double base;   // table base + cost offset
  double off;    // cost offset
  int rows;
  double gamma[kPrepRows];
  double beta[kPrepRows];
};

__global__ void __launch_bounds__(256) layer_prep_kernel(const PrepArgs a) {
  const int r = blockIdx.x;
  if (r >= a.rows) return;
  const double g = a.gamma_d ? a.gamma_d[r] : a.gamma[r];
  if (threadIdx.x == 0) {
    const double b = a.beta_d ? a.beta_d[r] : a.beta[r];
    double sb, cb;
    sincos(b, &sb, &cb);
    a.pset[kParamRow * r] = g;
    a.pset[kParamRow * r + 1] = cb;
    a.pset[kParamRow * r + 2] = sb;
    a.pset[kParamRow * r + 3] = sb / cb;
  }
  if (a.tab != nullptr) {
    for (int e = threadIdx.x; e < kTabRow; e += blockDim.x) {
      double v;
      if (e < 256) {
        v = 256.0 * (double)e + a.base;  // HI
      } else if (e < 288) {
        const int j = (e - 256) & 15;
        v = e < 272 ? 16.0 * (double)j : (double)j;  // MID, LO
      } else if (e < 544) {
        v = 256.0 * (double)(e - 288);  // F1
      } else if (e < 800) {
        const int m = e - 544;
        v = 16777216.0 * (double)(m < 128 ? m : m - 256) + a.off;  // F3
      } else {
        const int j = (e - 800) & 15;
        v = e < 816 ? 1048576.0 * (double)j : 65536.0 * (double)j;  // F2M, F2L
      }
      double sn, cs;
      sincos(g * v, &sn, &cs);
      a.tab[(size_t)r * kTabRow + e] = make_double2(cs, -sn);
    }
  }
}

// ----------------------------------------------------------------------------
// reductions
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums (x, y) over the workgroup in a fixed order; result valid in thread 0.
// `scratch` holds 2 doubles per wave (2 per thread when the workgroup is a
// single partial wave).  Ends with all threads past a barrier.
// nthr: threads of the workgroup, passed in by each kernel (blockDim.x read
// in the kernel body, or the tile geometry): blockDim.x inside an inlined
// helper becomes a per-lane load that allows for a partial last workgroup and
// waits for all vector memory (vmcnt(0)), stalling on loads in flight.
__device__ __forceinline__ void block_sum2(double& x, double& y, double* scratch, uint32_t nthr) {
  if (nthr < 64) {
    // partial wave: no cross-lane shuffles over inactive lanes
    scratch[2 * threadIdx.x] = x;
    scratch[2 * threadIdx.x + 1] = y;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sx = 0.0, sy = 0.0;
      for (uint32_t i = 0; i < nthr; ++i) { sx += scratch[2 * i]; sy += scratch[2 * i + 1]; }
      x = sx; y = sy;
    }
    __syncthreads();
    return;
  }
  x = wave_sum(x);
  y = wave_sum(y);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  if (lane == 0) { scratch[2 * wv] = x; scratch[2 * wv + 1] = y; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nw = (nthr + 63u) >> 6;
    double sx = 0.0, sy = 0.0;
    for (uint32_t i = 0; i < nw; ++i) { sx += scratch[2 * i]; sy += scratch[2 * i + 1]; }
    x = sx; y = sy;
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// fused QAOA sweep
// ----------------------------------------------------------------------------
struct SweepArgs {
  void* psi;
  const void* diag;
  const double2* ptab; // phase tables (integer cost vectors), kTabRow per layer
  double* partials;   // 2 doubles per block (E, norm) when F_EXPV
  double diag_offset;
  double amp0;        // 2^{-n/2} for F_INIT
  int flags;
  int nlayers;        // layers applied by this launch
  TileGeom g;
  // Parameters: layer l of state s (set = blockIdx.y for sweeps, blockIdx.x
  // for whole-state tiles) uses row r = (set0 + s) * p_total + layer0 + l of
  // pset (gamma, cos beta, sin beta) and of ptab.  State s starts at
  // psi + s * set_stride_bytes and its partials at partials + s * partials_stride.
  const double* pset;
  int set0;
  int p_total;
  int layer0;
  uint64_t set_stride_bytes;
  uint64_t partials_stride;
};

// Largest |tan beta| for which complex64 sweeps compute in FP32.
constexpr double kTanMaxF32 = 64.0;

struct LayerParams {
  double g, ca, sb, tn;  // gamma, cos beta, sin beta, tan beta
  const double2* tab;
};

__device__ __forceinline__ LayerParams layer_params(const SweepArgs& a, uint32_t set, int l) {
  const size_t r = (size_t)(a.set0 + set) * a.p_total + a.layer0 + l;
  const double* row = a.pset + kParamRow * r;
  return LayerParams{row[0], row[1], row[2], row[3], a.ptab + r * kTabRow};
}

// gate cos(b) I - i sin(b) X on the pair (y0, y1):
//   y0' = a y0 - i s y1,  y1' = -i s y0 + a y1
__device__ __forceinline__ void rx_pair(double& r0, double& i0, double& r1, double& i1, double a, double s) {
  const double nr0 = fma(a, r0, s * i1);
  const double ni0 = fma(a, i0, -s * r1);
  const double nr1 = fma(a, r1, s * i0);
  const double ni1 = fma(a, i1, -s * r0);
  r0 = nr0; i0 = ni0; r1 = nr1; i1 = ni1;
}

// The same gate divided by cos(b): (y0, y1) -> (y0 - i t y1, y1 - i t y0) with
// t = tan(b), four FMAs per pair instead of eight operations.  A sweep applies
// it to each of its k qubits and multiplies the tile by cos(b)^k afterwards.
// Every element carries the same factor, so relative precision is unchanged;
// in double the growth 1/|cos b|^k stays finite for every representable b and
// k <= 14 (|cos b| >= ~1e-19), and tiles are rescaled before the next layer.
template <class T>
__device__ __forceinline__ void rx_pair_t(T& r0, T& i0, T& r1, T& i1, T t) {
  const T nr0 = fma(t, i1, r0);
  const T ni0 = fma(-t, r1, i0);
  const T nr1 = fma(t, i0, r1);
  const T ni1 = fma(-t, r0, i1);
  r0 = nr0; i0 = ni0; r1 = nr1; i1 = ni1;
}

// x^k for small k by repeated multiplication.
__device__ __forceinline__ double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

template <int E, class T>
__device__ __forceinline__ void scale_tile(T (&vr)[E], T (&vi)[E], double f) {
  const T ft = (T)f;
#pragma unroll
  for (int k = 0; k < E; ++k) { vr[k] *= ft; vi[k] *= ft; }
}


// Synchronisation between the write and read halves of a window change.  A
// change between two windows <= kLocalWin keeps every element in its wave:
// each wave reads back only what it wrote, so the wave's own LDS writes must
// complete (lgkmcnt(0)) but no other wave is waited for.  Otherwise the whole
// workgroup meets at a barrier.
__device__ __forceinline__ void exchange_sync(bool local) {
  if (local) {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt not waited for
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Per-thread part of the swizzled LDS byte address in window w.
template <class S, int EB>
__device__ __forceinline__ uint32_t lds_tpart(uint32_t tid, int w) {
  return swz<S::kLdsBytes>(thr_part<EB>(tid, w), EB) * S::kLdsBytes;
}

// Window change wf -> wt through LDS.  Linear swizzle in bytes: per-thread
// parts pf, pt (lds_tpart of the two windows), per-register part (g.loff,
// already in bytes) from the host, so each access costs one XOR.
template <class S, int EB, class T>
__device__ __forceinline__ void exchange_p(T (&vr)[1 << EB], T (&vi)[1 << EB], typename S::L* lds,
                                           const TileGeom& g, int wf, int wt, uint32_t pf, uint32_t pt) {
  // a wave-local change writes and reads only the wave's own positions; the
  // positions it writes were last read by the same wave, so no barrier is
  // needed after the reads either
  const bool local = (wf > wt ? wf : wt) <= kLocalWin;
  if constexpr (S::kSplit) {
    // real parts, then imaginary parts, as 8-byte entries
#pragma unroll
    for (int k = 0; k < (1 << EB); ++k) *lds_d(pf ^ g.loff[wf][k]) = vr[k];
    exchange_sync(local);
#pragma unroll
    for (int k = 0; k < (1 << EB); ++k) vr[k] = *lds_d(pt ^ g.loff[wt][k]);
    exchange_sync(local);
#pragma unroll
    for (int k = 0; k < (1 << EB); ++k) *lds_d(pf ^ g.loff[wf][k]) = vi[k];
    exchange_sync(local);
#pragma unroll
    for (int k = 0; k < (1 << EB); ++k) vi[k] = *lds_d(pt ^ g.loff[wt][k]);
    if (!local) __syncthreads();
    (void)lds;
  } else {
#pragma unroll
    for (int k = 0; k < (1 << EB); ++k) S::lput(lds, pf ^ g.loff[wf][k], vr[k], vi[k]);
    exchange_sync(local);
#pragma unroll
    for (int k = 0; k < (1 << EB); ++k) S::lget(lds, pt ^ g.loff[wt][k], vr[k], vi[k]);
    if (!local) __syncthreads();
  }
}

template <class S, int EB, class T>
__device__ __forceinline__ void exchange_c(T (&vr)[1 << EB], T (&vi)[1 << EB], typename S::L* lds,
                                           const TileGeom& g, uint32_t tid, int wf, int wt) {
  exchange_p<S, EB>(vr, vi, lds, g, wf, wt, lds_tpart<S, EB>(tid, wf), lds_tpart<S, EB>(tid, wt));
}

// exp(-i g c) evaluated directly from the double-precision angle g * c.  Kept
// out of line: it is the rare path for integer cost vectors and the only path
// for F64 ones, and inlining sixteen copies of sincos into the unrolled tile
// loop would cost registers and instruction cache in the common path.
__device__ __noinline__ double2 phase_direct(double g, double c) {
  double sn, cs;
  sincos(g * c, &sn, &cs);
  return make_double2(cs, -sn);
}

template <class T>
__device__ __forceinline__ void cmul_inplace(T& r, T& i, T fr, T fi) {
  const T nr = fma(fr, r, -fi * i);
  const T ni = fma(fr, i, fi * r);
  r = nr; i = ni;
}

// Table passes of the integer phase.  Every pass multiplies each element by
// T[(x >> 8) & 255] * T[256 + ((x >> 4) & 15)] * T[272 + (x & 15)] with
// x = (v + add) >> shift, where v is the stored value and T the 288 entries
// staged in LDS:
//   in range (one pass):  T = HI|MID|LO, add = -base, shift 0;
//   out of range (int32): T = F1|MID|LO, then T = F3|F2M|F2L with shift 16 (the
//   byte decomposition).
// One code path serves both cases, so the rare case costs no registers in the
// common one; prepare_pass stages pass `pass`.
// LDS table entry from a double2 table row (FP32 sweeps round it once here).
__device__ __forceinline__ void tab_set(double2& d, const double2& s) { d = s; }
__device__ __forceinline__ void tab_set(float2& d, const double2& s) { d = make_float2((float)s.x, (float)s.y); }

template <class V>
__device__ __forceinline__ void prepare_pass(V* tab, const double2* row, uint32_t tid, int pass, uint32_t nthr) {
  __syncthreads();  // readers of the previous tables are done
  for (uint32_t e = tid; e < 288u; e += nthr) {
    if (pass == 0) {
      if (e < 256u) tab_set(tab[e], row[288 + e]);  // F1 (MID, LO stay)
    } else {
      tab_set(tab[e], row[544 + e]);  // F3, F2M, F2L
    }
  }
  __syncthreads();
}

// The phase factor of table index x (both cases above).
template <class V>
__device__ __forceinline__ V table_phase(const V* tab, uint32_t x) {
  const V h = tab[(x >> 8) & 255u], m = tab[256u + ((x >> 4) & 15u)], l = tab[272u + (x & 15u)];
  const V hm(fma(h.x, m.x, -h.y * m.y), fma(h.x, m.y, h.y * m.x));
  return V(fma(hm.x, l.x, -hm.y * l.y), fma(hm.x, l.y, hm.y * l.x));
}

// Stage HI|LO and decide (workgroup-uniform) whether every value of the tile is
// covered by it.
// Workgroup-wide OR of a flag: one word per wave after the tables (flags),
// written by each wave's first active lane, read by everyone after a barrier.
__device__ __forceinline__ bool block_any(bool v, uint32_t* flags, uint32_t nthr) {
  const uint64_t m = __ballot(v);
  const uint32_t wv = threadIdx.x >> 6, nw = (nthr + 63u) >> 6;
  if (__lane_id() == (uint32_t)__ffsll((unsigned long long)__ballot(1)) - 1u) flags[wv] = m != 0;
  __syncthreads();
  uint32_t any = 0;
  for (uint32_t i = 0; i < nw; ++i) any |= flags[i];
  return any != 0;
}

template <class D, int E, bool PRESTAGED = false, class V>
__device__ __forceinline__ bool stage_phase_tables(const typename D::RawT (&cv)[E], V* tab, const double2* row,
                                                   uint32_t tid, uint32_t nthr) {
  int ok = 1;
  if constexpr (!D::kAlwaysInTable) {
#pragma unroll
    for (int k = 0; k < E; ++k) ok &= (D::tab_index(cv[k]) >= 0);
  }
  if constexpr (!PRESTAGED)  // else written at kernel start, overlapping the state loads
    for (uint32_t e = tid; e < (uint32_t)kTabEntries; e += nthr) tab_set(tab[e], row[e]);
  if constexpr (D::kAlwaysInTable) {
    __syncthreads();
    return true;
  } else {
    return !block_any(!ok, reinterpret_cast<uint32_t*>(tab + kTabEntries), nthr);
  }
}

// Phase operator of one layer on the thread's register elements, from the
// stored cost values `cv` of those elements.  Integer cost vectors use the
// LDS-staged tables (one pass, or two byte-table passes when some int32 value
// of the workgroup is outside the two-level table; a workgroup-uniform choice);
// float64 ones evaluate sincos of the angle.
template <class S, class D, int EB, bool PRESTAGED = false, class T, class V>
__device__ __forceinline__ void phase_from_raw(T (&vr)[1 << EB], T (&vi)[1 << EB],
                                               const typename D::RawT (&cv)[1 << EB], const SweepArgs& a,
                                               const LayerParams& lp, uint32_t tid, V* tab, uint32_t nthr) {
  constexpr int E = 1 << EB;
  if constexpr (D::kTable) {
    const bool fast = stage_phase_tables<D, E, PRESTAGED>(cv, tab, lp.tab, tid, nthr);
    const int npass = fast ? 1 : 2;
    const uint32_t add = fast ? (uint32_t)(-(int32_t)D::kTableBase) : 0u;
#pragma clang loop unroll(disable)
    for (int pass = 0; pass < npass; ++pass) {
      if (!fast) prepare_pass(tab, lp.tab, tid, pass, nthr);
      const int shift = pass ? 16 : 0;
      // groups of four elements: bounds how many table entries the scheduler
      // keeps in flight (register pressure decides occupancy here)
#pragma unroll
      for (int k0 = 0; k0 < E; k0 += 4) {
#pragma unroll
        for (int k = k0; k < k0 + 4 && k < E; ++k) {
          const V f = table_phase(tab, ((uint32_t)cv[k] + add) >> shift);
          cmul_inplace(vr[k], vi[k], f.x, f.y);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const double2 f = phase_direct(lp.g, D::value(cv[k]) + a.diag_offset);
      cmul_inplace(vr[k], vi[k], (T)f.x, (T)f.y);
    }
  }
}

// Stored cost values of the thread's register elements in window w.
template <class D, int EB>
__device__ __forceinline__ void load_cost_g(typename D::RawT (&cv)[1 << EB], const void* diag, uint64_t base,
                                            uint32_t tid, int w, const TileGeom& g) {
  const uint64_t xb = base + tile_off(thr_part<EB>(tid, w), g);
#pragma unroll
  for (int k = 0; k < (1 << EB); ++k) cv[k] = D::load_raw(diag, xb + g.goff[w][k]);
}
template <class D, int EB>
__device__ __forceinline__ void load_cost(typename D::RawT (&cv)[1 << EB], const SweepArgs& a, uint64_t base,
                                          uint32_t tid, int w) {
  load_cost_g<D, EB>(cv, a.diag, base, tid, w, a.g);
}

// Tangent-form butterflies on register bits [LO, HI) of the window.
template <int EB, int LO, int HI, class T>
__device__ __forceinline__ void butterflies(T (&vr)[1 << EB], T (&vi)[1 << EB], T t) {
#pragma unroll
  for (int j = LO; j < HI && j < EB; ++j) {
#pragma unroll
    for (int k = 0; k < (1 << EB); ++k) {
      if (!(k & (1 << j))) rx_pair_t(vr[k], vi[k], vr[k | (1 << j)], vi[k | (1 << j)], t);
    }
  }
}

// Mixer gates of one layer on the tile's active qubits, window by window, in
// chunk order or (REV) in reverse chunk order; the gates commute, so both
// orders give the same layer.  Each gate is applied divided by cos(beta)
// (rx_pair_t with tn = tan beta): the caller multiplies the tile by
// cos(beta)^(tb - act_lo), or (CS) each chunk is multiplied by cos(beta)^(its
// gates) here, which keeps every window change's values at the scale of the
// state: FP64 tiles whose exchanges go through FP32 LDS need that when
// |tan beta| is large.  Returns the final window; pcur holds lds_tpart of
// the current window on entry and on return (each change computes only the
// new window's part).
//
// Every register bit of a chunk takes a butterfly; bits outside [jlo, jhi)
// take the identity (t = 0 gives exactly (y0, y1)).  Straight-line code: a
// branch per bit made the compiler copy all 16 elements after each butterfly.
// When PHI > PLO the caller guarantees that chunk g.part has jlo = PLO,
// jhi = PHI; that chunk is then applied outside the loops with only its own
// butterflies (plans have at most one such chunk of one to three bits).
template <class S, int EB, bool REV = false, int PLO = 0, int PHI = 0, bool CS = false, class T>
__device__ __forceinline__ int apply_mixer(T (&vr)[1 << EB], T (&vi)[1 << EB], typename S::L* lds,
                                           const TileGeom& g, uint32_t tid, int w, double tn_d, double ca,
                                           uint32_t& pcur) {
  constexpr int E = 1 << EB;
  const T tn = (T)tn_d;
  constexpr bool kPart = PHI > PLO;
  auto to_window = [&](int wt) __attribute__((always_inline)) {
    if (wt != w) {
      const uint32_t pt = lds_tpart<S, EB>(tid, wt);
      exchange_p<S, EB>(vr, vi, lds, g, w, wt, pcur, pt);
      w = wt;
      pcur = pt;
    }
  };
  auto chunk = [&](const Chunk ch) __attribute__((always_inline)) {
    to_window(ch.w);
#pragma unroll
    for (int j = 0; j < EB; ++j) {
      const T tj = (j >= ch.jlo && j < ch.jhi) ? tn : T(0);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        if (!(k & (1 << j))) rx_pair_t(vr[k], vi[k], vr[k | (1 << j)], vi[k | (1 << j)], tj);
      }
    }
    if constexpr (CS) scale_tile(vr, vi, ipow(ca, ch.jhi - ch.jlo));
  };
  const int nc = g.nchunks;
  if constexpr (!kPart) {
    for (int i = 0; i < nc; ++i) chunk(g.chunk[REV ? nc - 1 - i : i]);
  } else {
    // the short chunk g.part (bits [PLO, PHI) of its window) between two loops
    // of ordinary chunks, so neither loop branches on the chunk kind
    const int pi = g.part;
    if constexpr (!REV) {
      for (int i = 0; i < pi; ++i) chunk(g.chunk[i]);
      to_window(g.chunk[pi].w);
      butterflies<EB, PLO, PHI>(vr, vi, tn);
      if constexpr (CS) scale_tile(vr, vi, ipow(ca, PHI - PLO));
      for (int i = pi + 1; i < nc; ++i) chunk(g.chunk[i]);
    } else {
      for (int i = nc - 1; i > pi; --i) chunk(g.chunk[i]);
      to_window(g.chunk[pi].w);
      butterflies<EB, PLO, PHI>(vr, vi, tn);
      if constexpr (CS) scale_tile(vr, vi, ipow(ca, PHI - PLO));
      for (int i = pi - 1; i >= 0; --i) chunk(g.chunk[i]);
    }
  }
  return w;
}

// (E, norm) partial sums of the thread's elements.
template <class D, int EB, class T>
__device__ __forceinline__ void expv_partials(const T (&vr)[1 << EB], const T (&vi)[1 << EB],
                                              const SweepArgs& a, uint64_t base, uint32_t tid, int w,
                                              double& e_part, double& n_part) {
  const uint64_t xb = base + tile_off(thr_part<EB>(tid, w), a.g);
#pragma unroll
  for (int k = 0; k < (1 << EB); ++k) {
    const double c = D::get(a.diag, xb + a.g.goff[w][k]) + a.diag_offset;
    const double r = vr[k], i = vi[k];
    const double pr = r * r + i * i;
    e_part += pr * c;
    n_part += pr;
  }
}

// Workgroups are handed to the eight XCDs round robin.  Renumbered this way,
// each XCD walks one contiguous range of tiles, so tiles that share cache
// lines or pages run on the same XCD (and its L2) at about the same time.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  if (nb & 7u) return b;
  return (b & 7u) * (nb >> 3) + (b >> 3);
}

// The tile work of one sweep in arithmetic type R (table entries V).
template <class S, class D, int EB, bool INIT, bool PHASE, bool EXPV, bool FUSE, int PLO, int PHI, class R, class V>
__device__ __forceinline__ void sweep_tile(const SweepArgs& a) {
  constexpr int E = 1 << EB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  typename S::L* lds = reinterpret_cast<typename S::L*>(smem_raw);
  V* tab = reinterpret_cast<V*>(smem_raw + (1u << a.g.tb) * S::kLdsBytes);
  const uint32_t tid = threadIdx.x;
  const uint32_t nthr = 1u << (a.g.tb - EB);  // the launch's threads per workgroup
  const uint64_t base = block_base(xcd_block(blockIdx.x, gridDim.x), a.g);
  const uint32_t set = blockIdx.y;
  void* psi = reinterpret_cast<char*>(a.psi) + (uint64_t)set * a.set_stride_bytes;
  const LayerParams lp = layer_params(a, set, 0);
  // Narrow tiles (two workgroups per CU) read the next layer's parameters here,
  // with the state loads, instead of stalling on them between the two layers
  // (n=31 complex64 +2.6 %); the wide complex128 kernel reads them where they
  // are used (holding them from the start cost it 2.4 %).
  constexpr bool kEarlyNext = FUSE && !S::kSplit;
  const LayerParams lq_early = kEarlyNext ? layer_params(a, set, 1) : lp;

  R vr[E], vi[E];
  const int w_load = a.g.chunk[0].w;  // the load mapping: the first chunk's window
  int w = w_load;
  // EXPV: the cost values are read with the state, in the coalesced load
  // mapping, and the tile returns to that mapping for the reduction.  FUSE:
  // they are read up front in the mapping the phase is applied in (the last
  // window of the chunk order).
  typename D::RawT cv[(EXPV || FUSE) ? E : 1];
  {
    const uint64_t xb = base + tile_off(thr_part<EB>(tid, w), a.g);
    if constexpr (INIT) {
#pragma unroll
      for (int k = 0; k < E; ++k) { vr[k] = (R)a.amp0; vi[k] = R(0); }
    } else {
#pragma unroll
      for (int k = 0; k < E; ++k) S::load(psi, xb + a.g.goff[w][k], vr[k], vi[k]);
    }
  }
  if constexpr (EXPV) load_cost<D, EB>(cv, a, base, tid, w_load);
  // complex64 tiles hold the cost values from the start (their loads overlap
  // the state loads); complex128 ones hold uint16 values packed two per
  // register, and read wider ones when needed (holding them through the first
  // gates would spill registers)
  constexpr bool kEarlyCost = !S::kSplit;
  constexpr bool kPackedCost = FUSE && !kEarlyCost && D::kPack16;
  uint32_t cpk[kPackedCost ? E / 2 : 1];
  if constexpr (FUSE && kEarlyCost) load_cost<D, EB>(cv, a, base, tid, a.g.chunk[a.g.nchunks - 1].w);
  if constexpr (kPackedCost) {
    const int wp = a.g.chunk[a.g.nchunks - 1].w;
    const uint64_t xb = base + tile_off(thr_part<EB>(tid, wp), a.g);
    const uint16_t* c16 = reinterpret_cast<const uint16_t*>(a.diag);
#pragma unroll
    for (int k = 0; k < E; k += 2)
      cpk[k / 2] = (uint32_t)c16[xb + a.g.goff[wp][k]] | ((uint32_t)c16[xb + a.g.goff[wp][k + 1]] << 16);
  }
  if constexpr ((FUSE || PHASE) && D::kTable) {
    // the tables of the phase this launch applies go to LDS now, overlapping
    // the state loads (FUSE: the next layer's; PHASE: this layer's)
    const LayerParams lq0 = FUSE ? (kEarlyNext ? lq_early : layer_params(a, set, 1)) : lp;
    for (uint32_t e = tid; e < (uint32_t)kTabEntries; e += nthr) tab_set(tab[e], lq0.tab[e]);
  }
  if constexpr (PHASE) {
    typename D::RawT pc[E];
    load_cost<D, EB>(pc, a, base, tid, w);
    phase_from_raw<S, D, EB, D::kTable>(vr, vi, pc, a, lp, tid, tab, nthr);
  }
  const int nq = a.g.tb - a.g.act_lo;  // gates per layer in this tile
  // FP64 tiles of complex64 states (large |tan beta|) rescale chunk by chunk
  constexpr bool kCS = S::kDualPrecision && std::is_same<R, double>::value;
  uint32_t pcur = lds_tpart<S, EB>(tid, w);
  w = apply_mixer<S, EB, false, PLO, PHI, kCS>(vr, vi, lds, a.g, tid, w, lp.tn, lp.ca, pcur);
  if constexpr (!kCS) scale_tile(vr, vi, ipow(lp.ca, nq));
  if constexpr (FUSE) {
    const LayerParams lq = kEarlyNext ? lq_early : layer_params(a, set, 1);
    if constexpr (kPackedCost) {
#pragma unroll
      for (int k = 0; k < E; ++k) cv[k] = (int32_t)((k & 1) ? (cpk[k / 2] >> 16) : (cpk[k / 2] & 0xFFFFu));
    } else if constexpr (!kEarlyCost) {
      load_cost<D, EB>(cv, a, base, tid, w);
    }
    phase_from_raw<S, D, EB, D::kTable>(vr, vi, cv, a, lq, tid, tab, nthr);
    w = apply_mixer<S, EB, true, PLO, PHI, kCS>(vr, vi, lds, a.g, tid, w, lq.tn, lq.ca, pcur);  // ends in the load mapping
    if constexpr (!kCS) scale_tile(vr, vi, ipow(lq.ca, nq));
  }

  double e_part = 0.0, n_part = 0.0;
  // wide tiles store from the window their chunk order ends in (the top
  // window, coalesced, in their plans): no final change of window, whose code
  // alone made the register allocator spill in these 16-wave kernels
  const int w_out = EXPV ? w_load : ((FUSE || S::kSplit) ? w : a.g.w_store);
  if (w != w_out) {
    exchange_p<S, EB>(vr, vi, lds, a.g, w, w_out, pcur, lds_tpart<S, EB>(tid, w_out));
    w = w_out;
  }
  if constexpr (EXPV) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const double r = vr[k], i = vi[k];
      const double pr = r * r + i * i;
      e_part += pr * (D::value(cv[k]) + a.diag_offset);
      n_part += pr;
    }
  }
  {
    const uint64_t xb = base + tile_off(thr_part<EB>(tid, w), a.g);
#pragma unroll
    for (int k = 0; k < E; ++k) S::store(psi, xb + a.g.goff[w][k], vr[k], vi[k]);
  }
  if constexpr (EXPV) {
    __syncthreads();  // the tile buffer becomes reduction scratch (the last window change may have been wave-local)
    block_sum2(e_part, n_part, reinterpret_cast<double*>(smem_raw), nthr);
    if (tid == 0) {
      double* part = a.partials + (uint64_t)set * a.partials_stride;
      part[2 * (uint64_t)blockIdx.x] = e_part;
      part[2 * (uint64_t)blockIdx.x + 1] = n_part;
    }
  }
}

// One HBM sweep (multi-tile states).  The flags are compile-time so each
// launch carries only the code it runs:
//   INIT   generate |+> in registers instead of loading the state
//   PHASE  apply the layer's phase before the mixer gates
//   EXPV   emit per-workgroup (E, norm) partials of the result
//   FUSE   the tile's mixer gates of layer l, the phase of layer l+1, then the
//          tile's mixer gates of layer l+1 (valid when this sweep is the last
//          of layer l: every other gate of layer l is already applied)
// complex64 tiles compute in FP32 when every layer the launch applies has
// |tan beta| <= kTanMaxF32, and in FP64 otherwise (a workgroup-uniform
// choice): the tangent-form gates let the tile grow by 1/|cos beta| per gate
// until the rescale after the layer's gates, at most 64.01^13 < 2^79 here,
// far inside FP32's range, while beta near pi/2 would overflow it.
template <class S, class D, int EB, bool INIT, bool PHASE, bool EXPV, bool FUSE, int PLO = 0, int PHI = 0>
__global__ void __launch_bounds__(S::kMaxThreads, S::kMinWavesPerSimd) qaoa_sweep_kernel(const SweepArgs a_param) {
  if constexpr (S::kDualPrecision) {
    // Two inlined tile bodies read the arguments where they lie, in the
    // kernarg segment (the only explicit argument sits at its start): a
    // reference to the by-value parameter made the compiler copy its 2.2 KiB
    // into scratch memory per lane for them.
    typedef __attribute__((address_space(4))) const SweepArgs KernArgs;
    const SweepArgs& a = *(const SweepArgs*)(KernArgs*)__builtin_amdgcn_kernarg_segment_ptr();
    const uint32_t set = blockIdx.y;
    bool f32 = fabs(layer_params(a, set, 0).tn) <= kTanMaxF32;
    if constexpr (FUSE) f32 = f32 && fabs(layer_params(a, set, 1).tn) <= kTanMaxF32;
    if (f32) sweep_tile<S, D, EB, INIT, PHASE, EXPV, FUSE, PLO, PHI, float, float2>(a);
    else sweep_tile<S, D, EB, INIT, PHASE, EXPV, FUSE, PLO, PHI, double, double2>(a);
  } else {
    sweep_tile<S, D, EB, INIT, PHASE, EXPV, FUSE, PLO, PHI, typename S::R, typename S::Tab>(a_param);
  }
}

// Whole state in one tile (n <= tile bits): up to kMaxLayersPerLaunch layers
// in one launch, one workgroup.  Latency-bound; runtime flags.
template <class S, class D, int EB>
__global__ void __launch_bounds__(512) qaoa_tile_kernel(const SweepArgs a) {
  const uint32_t nthr = blockDim.x;
  constexpr int E = 1 << EB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  typename S::L* lds = reinterpret_cast<typename S::L*>(smem_raw);
  double2* tab = reinterpret_cast<double2*>(smem_raw + (1u << a.g.tb) * S::kLdsBytes);
  const uint32_t tid = threadIdx.x;
  const uint32_t set = blockIdx.x;
  void* psi = reinterpret_cast<char*>(a.psi) + (uint64_t)set * a.set_stride_bytes;
  double vr[E], vi[E];
  int w = a.g.tb - EB;
  if (a.flags & F_INIT) {
#pragma unroll
    for (int k = 0; k < E; ++k) { vr[k] = a.amp0; vi[k] = 0.0; }
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k) S::load(psi, tmap<EB>(tid, k, w), vr[k], vi[k]);
  }
  for (int l = 0; l < a.nlayers; ++l) {
    // the previous layer's table reads must finish before the table is restaged
    if (l > 0) __syncthreads();
    const LayerParams lp = layer_params(a, set, l);
    typename D::RawT pc[E];
    load_cost<D, EB>(pc, a, 0, tid, w);
    phase_from_raw<S, D, EB>(vr, vi, pc, a, lp, tid, tab, nthr);
    // alternate the chunk order: each layer starts in the window the last one ended in
    uint32_t pcur = lds_tpart<S, EB>(tid, w);
    // complex64 tiles exchange through FP32 LDS: rescale chunk by chunk
    constexpr bool kCS = S::kDualPrecision;
    if (l & 1) w = apply_mixer<S, EB, true, 0, 0, kCS>(vr, vi, lds, a.g, tid, w, lp.tn, lp.ca, pcur);
    else w = apply_mixer<S, EB, false, 0, 0, kCS>(vr, vi, lds, a.g, tid, w, lp.tn, lp.ca, pcur);
    if constexpr (!kCS) scale_tile(vr, vi, ipow(lp.ca, a.g.tb));
  }
  double e_part = 0.0, n_part = 0.0;
  if (a.flags & F_EXPV) expv_partials<D, EB>(vr, vi, a, 0, tid, w, e_part, n_part);
  if (w != a.g.w_store) {
    exchange_c<S, EB>(vr, vi, lds, a.g, tid, w, a.g.w_store);
    w = a.g.w_store;
  }
#pragma unroll
  for (int k = 0; k < E; ++k) S::store(psi, tmap<EB>(tid, k, w), vr[k], vi[k]);
  if (a.flags & F_EXPV) {
    __syncthreads();  // the tile buffer becomes reduction scratch
    block_sum2(e_part, n_part, reinterpret_cast<double*>(smem_raw), nthr);
    if (tid == 0) {
      double* part = a.partials + (uint64_t)set * a.partials_stride;
      part[0] = e_part;
      part[1] = n_part;
    }
  }
}

// ----------------------------------------------------------------------------
// reverse (adjoint) sweeps for the gradient
// ----------------------------------------------------------------------------
enum : int { A_FIRST = 1, A_PHASE = 2, A_FUSE = 8 };

struct AdjArgs {
  void* psi;           // forward state, uncomputed in place
  void* lam;           // adjoint state
  const void* diag;
  const double2* ptab; // phase tables, kTabRow per layer row
  const double* pset;  // rows (gamma, cos beta, sin beta)
  double* partials;    // this launch's (beta term, gamma term) per block
  double* partials2;   // A_FUSE: the beta term of layer - 1 per block (gamma term 0)
  double diag_offset;
  int layer;           // row of pset / ptab (the layer undone first)
  int nlayers;         // whole-state tile kernel: layers [0, nlayers) in reverse
  uint64_t layer_partials_stride;  // tile kernel: doubles between layers' partials
  TileGeom g;
};

// Im(conj(l0) p1 + conj(l1) p0): the pair's contribution to Im<lambda|X_q|psi>.
__device__ __forceinline__ double xterm(double pr0, double pi0, double pr1, double pi1, double lr0, double li0,
                                        double lr1, double li1) {
  return (lr0 * pi1 - li0 * pr1) + (lr1 * pi0 - li1 * pr0);
}

// Undo the layer's mixer gates on the tile's active qubits for psi and lambda
// (gate with -beta), accumulating Im<lambda|X_q|psi> per undone qubit (X_q
// commutes with every mixer gate, so any point of the undo gives the same value).
// Each undo gate cos(b) I + i sin(b) X is applied divided by cos(b), as
// (y0, y1) -> (y0 + i t y1, y1 + i t y0) with t = tan(b): four FMAs per pair
// and state instead of eight operations.  Within a chunk both states then
// carry 1/cos(b) per gate already undone, so the X term of a later qubit is
// scaled back by cos(b)^2 per such gate, and the tile is rescaled by
// cos(b)^(gates) at the end of each chunk (so the growth stays below
// |cos b|^-(2 EB) even for b near pi/2).  Bits outside [jlo, jhi) take the
// identity (t = 0) and add nothing to the X term.
template <class S, int EB, bool REV = false, int PLO = 0, int PHI = 0>
__device__ __forceinline__ int undo_mixer(double (&vr)[1 << EB], double (&vi)[1 << EB], double (&lr)[1 << EB],
                                          double (&li)[1 << EB], typename S::L* lds, const TileGeom& g,
                                          uint32_t tid, int w, double ca, double tn, double& xacc) {
  constexpr int E = 1 << EB;
  constexpr bool kPart = PHI > PLO;
  const double c2 = ca * ca;
  // one chunk: register bits [lo, hi) of its window (compile-time bounds for
  // the specialised short chunk, so its other bits take no identity butterflies)
  auto chunk = [&](const Chunk ch, auto lo_c, auto hi_c) __attribute__((always_inline)) {
    constexpr int LO = decltype(lo_c)::value, HI = decltype(hi_c)::value;
    if (ch.w != w) {
      exchange_c<S, EB>(vr, vi, lds, g, tid, w, ch.w);
      exchange_c<S, EB>(lr, li, lds, g, tid, w, ch.w);
      w = ch.w;
    }
    double s2 = 1.0;  // cos(b)^2 per gate undone so far in this chunk
    double cs = 1.0;  // cos(b) per gate undone so far in this chunk
#pragma unroll
    for (int j = 0; j < EB; ++j) {
      if (HI > LO && (j < LO || j >= HI)) continue;
      const bool on = HI > LO || (j >= ch.jlo && j < ch.jhi);
      const double tj = on ? -tn : 0.0, mj = on ? s2 : 0.0;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        if (!(k & (1 << j))) {
          const int k1 = k | (1 << j);
          xacc = fma(mj, xterm(vr[k], vi[k], vr[k1], vi[k1], lr[k], li[k], lr[k1], li[k1]), xacc);
          rx_pair_t(vr[k], vi[k], vr[k1], vi[k1], tj);
          rx_pair_t(lr[k], li[k], lr[k1], li[k1], tj);
        }
      }
      s2 = on ? s2 * c2 : s2;
      cs = on ? cs * ca : cs;
    }
    scale_tile(vr, vi, cs);
    scale_tile(lr, li, cs);
  };
  using Z = std::integral_constant<int, 0>;
  using PL = std::integral_constant<int, PLO>;
  using PH = std::integral_constant<int, PHI>;
  const int nc = g.nchunks;
  if constexpr (!kPart) {
    for (int i = 0; i < nc; ++i) chunk(g.chunk[REV ? nc - 1 - i : i], Z{}, Z{});
  } else {
    // the short chunk g.part between two loops of ordinary chunks
    const int pi = g.part;
    if constexpr (!REV) {
      for (int i = 0; i < pi; ++i) chunk(g.chunk[i], Z{}, Z{});
      chunk(g.chunk[pi], PL{}, PH{});
      for (int i = pi + 1; i < nc; ++i) chunk(g.chunk[i], Z{}, Z{});
    } else {
      for (int i = nc - 1; i > pi; --i) chunk(g.chunk[i], Z{}, Z{});
      chunk(g.chunk[pi], PL{}, PH{});
      for (int i = pi - 1; i >= 0; --i) chunk(g.chunk[i], Z{}, Z{});
    }
  }
  return w;
}

// Gamma term Im<lambda|C|psi> of the tile and the phase undo exp(+i g c) on both
// states; cv holds the stored cost values of the thread's elements.
template <class D, int EB>
__device__ __forceinline__ void undo_phase(double (&vr)[1 << EB], double (&vi)[1 << EB], double (&lr)[1 << EB],
                                           double (&li)[1 << EB], const typename D::RawT (&cv)[1 << EB],
                                           const AdjArgs& a, const LayerParams& lp, double2* tab, uint32_t tid,
                                           double& gacc, uint32_t nthr) {
  constexpr int E = 1 << EB;
#pragma unroll
  for (int k = 0; k < E; ++k) gacc += (D::value(cv[k]) + a.diag_offset) * (lr[k] * vi[k] - li[k] * vr[k]);
  if constexpr (D::kTable) {
    const bool fast = stage_phase_tables<D, E>(cv, tab, lp.tab, tid, nthr);
    const int npass = fast ? 1 : 2;
    const uint32_t add = fast ? (uint32_t)(-(int32_t)D::kTableBase) : 0u;
#pragma clang loop unroll(disable)
    for (int pass = 0; pass < npass; ++pass) {
      if (!fast) prepare_pass(tab, lp.tab, tid, pass, nthr);
      const int shift = pass ? 16 : 0;
#pragma unroll
      for (int k0 = 0; k0 < E; k0 += 4) {
#pragma unroll
        for (int k = k0; k < k0 + 4 && k < E; ++k) {
          const double2 f = table_phase(tab, ((uint32_t)cv[k] + add) >> shift);
          cmul_inplace(vr[k], vi[k], f.x, -f.y);  // conjugate
          cmul_inplace(lr[k], li[k], f.x, -f.y);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const double2 f = phase_direct(lp.g, D::value(cv[k]) + a.diag_offset);
      cmul_inplace(vr[k], vi[k], f.x, -f.y);
      cmul_inplace(lr[k], li[k], f.x, -f.y);
    }
  }
}

// One reverse sweep (multi-tile states):
//   FIRST  lambda = c * psi from the loaded psi (lambda is only written)
//   PHASE  after the mixer undo: gamma term and phase undo (last sweep of the layer)
//   FUSE   the tile's gates of layer l undone, then layer l's gamma term and
//          phase undo (every other gate of layer l is undone by then), then
//          the tile's gates of layer l-1 undone
// complex64: four waves per SIMD (two 512-thread workgroups per CU, which the
// LDS allows) double the resident waves of the fused variant, which then
// spills 160 bytes per lane and is still faster (n=26 complex64 gradient -9 %
// time).  complex128 keeps its registers: capped, its fused variant spilled
// 168 bytes per lane, the spill traffic raised the measured HBM bytes per
// launch by a third, and the gradient gained only 2.6 %.
template <class S, class D, int EB, bool FIRST, bool PHASE, bool FUSE, int PLO = 0, int PHI = 0>
__global__ void __launch_bounds__(512, S::kAdjMinWavesPerSimd) qaoa_adjoint_kernel(const AdjArgs a) {
  const uint32_t nthr = blockDim.x;
  constexpr int E = 1 << EB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  typename S::L* lds = reinterpret_cast<typename S::L*>(smem_raw);
  double2* tab = reinterpret_cast<double2*>(smem_raw + (1u << a.g.tb) * S::kLdsBytes);
  const uint32_t tid = threadIdx.x;
  const uint64_t base = block_base(xcd_block(blockIdx.x, gridDim.x), a.g);
  const size_t r = (size_t)a.layer;
  const double* prow = a.pset + kParamRow * r;
  const LayerParams lp{prow[0], prow[1], prow[2], prow[3], a.ptab + r * kTabRow};
  const int w_load = a.g.tb - EB;
  int w = w_load;
  double vr[E], vi[E], lr[E], li[E];
  typename D::RawT cv[(FIRST || PHASE || FUSE) ? E : 1];
  {
    const uint64_t xb = base + tile_off(thr_part<EB>(tid, w), a.g);
#pragma unroll
    for (int k = 0; k < E; ++k) S::load(a.psi, xb + a.g.goff[w][k], vr[k], vi[k]);
    if constexpr (FIRST || PHASE) load_cost_g<D, EB>(cv, a.diag, base, tid, w, a.g);
    if constexpr (FIRST) {
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const double c = D::value(cv[k]) + a.diag_offset;
        lr[k] = c * vr[k];
        li[k] = c * vi[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < E; ++k) S::load(a.lam, xb + a.g.goff[w][k], lr[k], li[k]);
    }
    // FUSE: cost values in the mapping of the last chunk's window, where the
    // phase is undone
    if constexpr (FUSE) load_cost_g<D, EB>(cv, a.diag, base, tid, a.g.chunk[a.g.nchunks - 1].w, a.g);
  }
  double xacc = 0.0, gacc = 0.0, xacc2 = 0.0;
  w = undo_mixer<S, EB, false, PLO, PHI>(vr, vi, lr, li, lds, a.g, tid, w, lp.ca, lp.tn, xacc);
  if constexpr (FUSE) {
    undo_phase<D, EB>(vr, vi, lr, li, cv, a, lp, tab, tid, gacc, nthr);
    const size_t r1 = r - 1;
    w = undo_mixer<S, EB, true, PLO, PHI>(vr, vi, lr, li, lds, a.g, tid, w, a.pset[kParamRow * r1 + 1],
                                          a.pset[kParamRow * r1 + 3], xacc2);
  }
  const int w_out = PHASE ? w_load : (FUSE ? w : a.g.w_store);
  if (w != w_out) {
    exchange_c<S, EB>(vr, vi, lds, a.g, tid, w, w_out);
    exchange_c<S, EB>(lr, li, lds, a.g, tid, w, w_out);
    w = w_out;
  }
  if constexpr (PHASE) undo_phase<D, EB>(vr, vi, lr, li, cv, a, lp, tab, tid, gacc, nthr);
  {
    const uint64_t xb = base + tile_off(thr_part<EB>(tid, w), a.g);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const uint64_t x = xb + a.g.goff[w][k];
      S::store(a.psi, x, vr[k], vi[k]);
      S::store(a.lam, x, lr[k], li[k]);
    }
  }
  __syncthreads();  // the tables and tile buffer are reused as reduction scratch
  block_sum2(xacc, gacc, reinterpret_cast<double*>(smem_raw), nthr);
  if (tid == 0) {
    a.partials[2 * (uint64_t)blockIdx.x] = xacc;
    a.partials[2 * (uint64_t)blockIdx.x + 1] = gacc;
  }
  if constexpr (FUSE) {
    double zero = 0.0;
    block_sum2(xacc2, zero, reinterpret_cast<double*>(smem_raw), nthr);
    if (tid == 0) {
      a.partials2[2 * (uint64_t)blockIdx.x] = xacc2;
      a.partials2[2 * (uint64_t)blockIdx.x + 1] = 0.0;
    }
  }
}

// ----------------------------------------------------------------------------
// XY mixers (Section 3.2): M = sum over edges <i,j> of (X_i X_j + Y_i Y_j)/2.
// exp(-i beta (X_i X_j + Y_i Y_j)/2) leaves |00>, |11> of the pair unchanged and
// rotates the amplitude pair (bit i = 0, bit j = 1) / (bit i = 1, bit j = 0)
// by [[cos b, -i sin b], [-i sin b, cos b]], the same 2x2 as the X gate.  The
// gates of an edge sequence do not commute, so a sweep applies a contiguous
// run of the sequence, in order, to a tile that holds all their qubits; the
// tile lives in LDS (complex128 entries) while the gates run.
// ----------------------------------------------------------------------------
constexpr int kMaxXyGates = 128;

// x with zero bits inserted at positions lo < hi.
__device__ __forceinline__ uint32_t insert_two_zeros(uint32_t q, int lo, int hi) {
  q = ((q >> lo) << (lo + 1)) | (q & ((1u << lo) - 1u));
  return ((q >> hi) << (hi + 1)) | (q & ((1u << hi) - 1u));
}

struct XyArgs {
  SweepArgs s;       // state, cost vector, tables, geometry, parameter rows, partials, flags
  int ngates;        // gates per layer in this launch, applied in order
  int dicke_k;       // F_INIT: -1 = |+>^n (amp0 everywhere); k >= 0 = amp0 on Hamming weight k
  int ngroups;       // > 0: the gates in ngroups groups of consecutive gates (below), else one pass per gate
  int8_t gate[kMaxXyGates][2];  // tile-bit pairs (i, j)
  // Group g is one LDS pass over the next gates of the list, of kind
  //   XG_ONE   one gate, on its two amplitudes per pair (gate[e])
  //   XG_PAIR  two gates on disjoint qubits: local bits (0,1), (2,3)
  //   XG_STAR2 two gates sharing local bit 0: (0,1) then (0,2)
  //   XG_STAR3 three gates sharing local bit 0: (0,1), (0,2), (0,3)
  // over tile bits grp_bits[g] (local bit order; a fourth bit pads STAR2)
  // and the same bits ascending in grp_sorted[g].
  int8_t grp_kind[kMaxXyGates];
  int8_t grp_bits[kMaxXyGates][4];
  int8_t grp_sorted[kMaxXyGates][4];
};
enum : int { XG_ONE = 1, XG_PAIR = 2, XG_STAR2 = 3, XG_STAR3 = 4 };

// LDS position of XY tile entry t (16-byte entries): the low four bits are
// XORed with bits 4-7 and 8-11, so 16 consecutive lanes reach 16 different
// 16-byte slots of a 256-byte bank row for the usual access patterns (whole
// tile in order, gate pairs, four-bit groups at any bits).
__device__ __forceinline__ uint32_t xy_pos(uint32_t t) { return t ^ (((t >> 4) ^ (t >> 8)) & 15u); }

// One XY gate on local bits (I, J) of a 16-amplitude group in registers:
// amplitudes with (bit I, bit J) = (0, 1) and (1, 0) are rotated together.
template <int I, int J>
__device__ __forceinline__ void xy_gate16(double (&r)[16], double (&m)[16], double ca, double sb) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (((k >> I) & 1) == 0 && ((k >> J) & 1) == 1) {
      const int k1 = k ^ (1 << I) ^ (1 << J);
      rx_pair(r[k], m[k], r[k1], m[k1], ca, sb);
    }
  }
}

// One grouped LDS pass of kind KIND (XG_PAIR / XG_STAR2 / XG_STAR3): each
// work item loads the 16 amplitudes of one value of the other tile bits,
// applies the kind's gates in order and writes them back.  Tile position of
// local index k: the item's part xor the uniform part of k's bits (xy_pos is
// linear over GF(2)).
template <int KIND>
__device__ __forceinline__ void xy_group_pass(double2* tile, const int8_t (&lb)[4], const int8_t (&sb4)[4],
                                              uint32_t tid, uint32_t nitems, double ca, double sb, uint32_t nthr) {
  const int b0 = lb[0], b1 = lb[1], b2 = lb[2], b3 = lb[3];
  for (uint32_t q = tid; q < nitems; q += nthr) {
    const uint32_t px = xy_pos(insert_two_zeros(insert_two_zeros(q, sb4[0], sb4[1]), sb4[2], sb4[3]));
    double r[16], m[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double2 v = tile[px ^ xy_pos(((uint32_t)(k & 1) << b0) | ((uint32_t)((k >> 1) & 1) << b1) |
                                         ((uint32_t)((k >> 2) & 1) << b2) | ((uint32_t)((k >> 3) & 1) << b3))];
      r[k] = v.x; m[k] = v.y;
    }
    if constexpr (KIND == XG_PAIR) {
      xy_gate16<0, 1>(r, m, ca, sb);
      xy_gate16<2, 3>(r, m, ca, sb);
    } else {
      xy_gate16<0, 1>(r, m, ca, sb);
      xy_gate16<0, 2>(r, m, ca, sb);
      if constexpr (KIND == XG_STAR3) xy_gate16<0, 3>(r, m, ca, sb);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k)
      tile[px ^ xy_pos(((uint32_t)(k & 1) << b0) | ((uint32_t)((k >> 1) & 1) << b1) |
                       ((uint32_t)((k >> 2) & 1) << b2) | ((uint32_t)((k >> 3) & 1) << b3))] = make_double2(r[k], m[k]);
  }
}


// One launch: for each of nlayers layers (several only when the tile is the
// whole state): [phase] then the gate list; flags F_INIT / F_PHASE / F_EXPV as
// in the X mixer sweeps.  Tile in LDS as double2, 2^tb entries, natural order.
template <class S, class D, int EB>
__global__ void __launch_bounds__(512) qaoa_xy_kernel(const XyArgs a) {
  const uint32_t nthr = blockDim.x;
  constexpr int E = 1 << EB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const SweepArgs& sa = a.s;
  const TileGeom& g = sa.g;
  double2* tile = reinterpret_cast<double2*>(smem_raw);
  double2* tab = reinterpret_cast<double2*>(smem_raw + ((size_t)1 << g.tb) * sizeof(double2));
  const uint32_t tid = threadIdx.x;
  const uint64_t base = block_base(xcd_block(blockIdx.x, gridDim.x), g);
  const uint32_t set = blockIdx.y;
  void* psi = reinterpret_cast<char*>(sa.psi) + (uint64_t)set * sa.set_stride_bytes;
  const int w = g.tb - EB;  // the coalesced load mapping
  const uint64_t xb = base + tile_off(thr_part<EB>(tid, w), g);
  double vr[E], vi[E];
  if (sa.flags & F_INIT) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const uint64_t x = xb + g.goff[w][k];
      const bool on = a.dicke_k < 0 || __popcll(x) == a.dicke_k;
      vr[k] = on ? sa.amp0 : 0.0;
      vi[k] = 0.0;
    }
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k) S::load(psi, xb + g.goff[w][k], vr[k], vi[k]);
  }
  typename D::RawT cv[E];
  if (sa.flags & (F_PHASE | F_EXPV)) load_cost<D, EB>(cv, sa, base, tid, w);
  const uint32_t npairs = 1u << (g.tb - 2);
  // xy_pos is linear over GF(2): the position of thr | k << w (disjoint bits)
  // is xy_pos(thr) ^ xy_pos(k << w), a per-thread part and a uniform part
  const uint32_t pthr = xy_pos(thr_part<EB>(tid, w));
  for (int l = 0; l < sa.nlayers; ++l) {
    const LayerParams lp = layer_params(sa, set, l);
    if (l > 0) {
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const double2 v = tile[pthr ^ xy_pos((uint32_t)k << w)];
        vr[k] = v.x; vi[k] = v.y;
      }
      __syncthreads();  // table reads of the previous layer are done before restaging
    }
    if (sa.flags & F_PHASE) phase_from_raw<S, D, EB>(vr, vi, cv, sa, lp, tid, tab, nthr);
#pragma unroll
    for (int k = 0; k < E; ++k) tile[pthr ^ xy_pos((uint32_t)k << w)] = make_double2(vr[k], vi[k]);
    __syncthreads();
    if (a.ngroups > 0) {
      // gates in groups: one LDS pass and one barrier per group
      const uint32_t nitems = 1u << (g.tb - 4);
      int e = 0;
      for (int gi = 0; gi < a.ngroups; ++gi) {
        const int kind = a.grp_kind[gi];
        if (kind == XG_ONE) {
          const int ti = a.gate[e][0], tj = a.gate[e][1];
          const int lo = ti < tj ? ti : tj, hi = ti < tj ? tj : ti;
          for (uint32_t q = tid; q < npairs; q += blockDim.x) {
            const uint32_t x = insert_two_zeros(q, lo, hi);
            const uint32_t x0 = xy_pos(x | (1u << tj)), x1 = xy_pos(x | (1u << ti));
            double2 u = tile[x0], v = tile[x1];
            rx_pair(u.x, u.y, v.x, v.y, lp.ca, lp.sb);
            tile[x0] = u;
            tile[x1] = v;
          }
          e += 1;
        } else if (kind == XG_PAIR) {
          xy_group_pass<XG_PAIR>(tile, a.grp_bits[gi], a.grp_sorted[gi], tid, nitems, lp.ca, lp.sb, nthr);
          e += 2;
        } else if (kind == XG_STAR2) {
          xy_group_pass<XG_STAR2>(tile, a.grp_bits[gi], a.grp_sorted[gi], tid, nitems, lp.ca, lp.sb, nthr);
          e += 2;
        } else {
          xy_group_pass<XG_STAR3>(tile, a.grp_bits[gi], a.grp_sorted[gi], tid, nitems, lp.ca, lp.sb, nthr);
          e += 3;
        }
        __syncthreads();
      }
    } else {
      for (int e = 0; e < a.ngates; ++e) {
        const int ti = a.gate[e][0], tj = a.gate[e][1];
        const int lo = ti < tj ? ti : tj, hi = ti < tj ? tj : ti;
        for (uint32_t q = tid; q < npairs; q += blockDim.x) {
          const uint32_t x = insert_two_zeros(q, lo, hi);
          const uint32_t x0 = xy_pos(x | (1u << tj)), x1 = xy_pos(x | (1u << ti));
          double2 u = tile[x0], v = tile[x1];
          rx_pair(u.x, u.y, v.x, v.y, lp.ca, lp.sb);
          tile[x0] = u;
          tile[x1] = v;
        }
        __syncthreads();
      }
    }
  }
  if (sa.nlayers > 0) {  // else the registers still hold the loaded (or generated) state
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const double2 v = tile[pthr ^ xy_pos((uint32_t)k << w)];
      vr[k] = v.x; vi[k] = v.y;
    }
  }
  double e_part = 0.0, n_part = 0.0;
  if (sa.flags & F_EXPV) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const double pr = vr[k] * vr[k] + vi[k] * vi[k];
      e_part += pr * (D::value(cv[k]) + sa.diag_offset);
      n_part += pr;
    }
  }
#pragma unroll
  for (int k = 0; k < E; ++k) S::store(psi, xb + g.goff[w][k], vr[k], vi[k]);
  if (sa.flags & F_EXPV) {
    __syncthreads();  // the tile buffer becomes reduction scratch
    block_sum2(e_part, n_part, reinterpret_cast<double*>(smem_raw), nthr);
    if (tid == 0) {
      double* part = sa.partials + (uint64_t)set * sa.partials_stride;
      part[2 * (uint64_t)blockIdx.x] = e_part;
      part[2 * (uint64_t)blockIdx.x + 1] = n_part;
    }
  }
}

// Whole state in one tile: lambda = c psi, then layers nlayers-1 .. 0 in reverse;
// layer l's (beta term, gamma term) go to partials + l * layer_partials_stride.
template <class S, class D, int EB>
__global__ void __launch_bounds__(512) qaoa_adjoint_tile_kernel(const AdjArgs a) {
  const uint32_t nthr = blockDim.x;
  constexpr int E = 1 << EB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  typename S::L* lds = reinterpret_cast<typename S::L*>(smem_raw);
  double2* tab = reinterpret_cast<double2*>(smem_raw + (1u << a.g.tb) * S::kLdsBytes);
  double* scratch = reinterpret_cast<double*>(smem_raw + (1u << a.g.tb) * S::kLdsBytes + D::kTabLds * sizeof(double2) +
                                              16 * sizeof(uint32_t));
  const uint32_t tid = threadIdx.x;
  const int w_load = a.g.tb - EB;
  int w = w_load;
  double vr[E], vi[E], lr[E], li[E];
  typename D::RawT cv[E];
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const uint32_t x = tmap<EB>(tid, k, w);
    S::load(a.psi, x, vr[k], vi[k]);
    cv[k] = D::load_raw(a.diag, x);
    const double c = D::value(cv[k]) + a.diag_offset;
    lr[k] = c * vr[k];
    li[k] = c * vi[k];
  }
  for (int l = a.nlayers - 1; l >= 0; --l) {
    const double* prow = a.pset + kParamRow * (size_t)l;
    const LayerParams lp{prow[0], prow[1], prow[2], prow[3], a.ptab + (size_t)l * kTabRow};
    double xacc = 0.0, gacc = 0.0;
    w = undo_mixer<S, EB>(vr, vi, lr, li, lds, a.g, tid, w, lp.ca, lp.tn, xacc);
    if (w != w_load) {
      exchange_c<S, EB>(vr, vi, lds, a.g, tid, w, w_load);
      exchange_c<S, EB>(lr, li, lds, a.g, tid, w, w_load);
      w = w_load;
    }
    __syncthreads();  // previous layer's table reads are done
    undo_phase<D, EB>(vr, vi, lr, li, cv, a, lp, tab, tid, gacc, nthr);
    block_sum2(xacc, gacc, scratch, nthr);
    if (tid == 0) {
      a.partials[(uint64_t)l * a.layer_partials_stride] = xacc;
      a.partials[(uint64_t)l * a.layer_partials_stride + 1] = gacc;
    }
  }
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const uint32_t x = tmap<EB>(tid, k, w);
    S::store(a.psi, x, vr[k], vi[k]);
    S::store(a.lam, x, lr[k], li[k]);
  }
}

// out[1 + l] = 2 * sum of layer l's gamma terms, out[1 + p + l] = 2 * sum of its
// beta terms; layer l's partials: nsw runs of `blocks` pairs at
// partials + l * layer_stride + s * blocks * 2 (the gamma term only in run 0).
__global__ void __launch_bounds__(256) grad_finalize_kernel(const double* partials, int p, int nsw, uint64_t blocks,
                                                            uint64_t layer_stride, double* out) {
  const uint32_t nthr = blockDim.x;
  __shared__ double scratch[16];
  const int l = blockIdx.x;
  const double* part = partials + (uint64_t)l * layer_stride;
  double xb = 0.0, gg = 0.0;
  // the gamma term is nonzero only in the sweep that undid the layer's phase
  for (int s = 0; s < nsw; ++s)
    for (uint64_t i = threadIdx.x; i < blocks; i += blockDim.x) {
      xb += part[2 * (s * blocks + i)];
      gg += part[2 * (s * blocks + i) + 1];
    }
  block_sum2(xb, gg, scratch, nthr);
  if (threadIdx.x == 0) {
    out[1 + l] = 2.0 * gg;
    out[1 + p + l] = 2.0 * xb;
  }
}

// ----------------------------------------------------------------------------
// batched evaluation helpers
// ----------------------------------------------------------------------------

// Stage 1 of the two-stage reduction of per-workgroup partials: block b of
// state s (blockIdx.y) sums pairs [b * per, min((b + 1) * per, count)) of that
// state's partials and writes tmp[s * tstride + 2 b + {0,1}].  Fixed order.
__global__ void __launch_bounds__(256) reduce_chunks_kernel(const double* partials, uint64_t count, uint64_t stride,
                                                            uint64_t per, double* tmp, uint64_t tstride) {
  const uint32_t nthr = blockDim.x;
  __shared__ double scratch[16];
  const double* part = partials + (uint64_t)blockIdx.y * stride;
  const uint64_t lo = (uint64_t)blockIdx.x * per;
  const uint64_t hi = lo + per < count ? lo + per : count;
  double e = 0.0, q = 0.0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) { e += part[2 * i]; q += part[2 * i + 1]; }
  block_sum2(e, q, scratch, nthr);
  if (threadIdx.x == 0) {
    tmp[(uint64_t)blockIdx.y * tstride + 2 * blockIdx.x] = e;
    tmp[(uint64_t)blockIdx.y * tstride + 2 * blockIdx.x + 1] = q;
  }
}

// out[2 s + {0,1}] = fixed-order sum of set s's `count` partial pairs.
__global__ void __launch_bounds__(256) finalize_batch_kernel(const double* partials, uint64_t count,
                                                             uint64_t stride, double* out) {
  const uint32_t nthr = blockDim.x;
  __shared__ double scratch[16];
  const double* part = partials + (uint64_t)blockIdx.x * stride;
  double e = 0.0, q = 0.0;
  for (uint64_t i = threadIdx.x; i < count; i += blockDim.x) { e += part[2 * i]; q += part[2 * i + 1]; }
  block_sum2(e, q, scratch, nthr);
  if (threadIdx.x == 0) { out[2 * blockIdx.x] = e; out[2 * blockIdx.x + 1] = q; }
}

// ----------------------------------------------------------------------------
// Walsh-Hadamard sweep for the cost-vector precompute
// ----------------------------------------------------------------------------
struct FwhtArgs {
  void* data;
  TileGeom g;
};

template <typename T> struct FwhtReg { using R = T; };
template <> struct FwhtReg<int32_t> { using R = uint32_t; };   // wrap-around arithmetic
template <> struct FwhtReg<uint16_t> { using R = uint32_t; };  // exact mod 2^16 after truncation

template <typename T, int EB>
__global__ void __launch_bounds__(512) fwht_sweep_kernel(const FwhtArgs a) {
  using R = typename FwhtReg<T>::R;
  constexpr int E = 1 << EB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* data = reinterpret_cast<T*>(a.data);
  const uint32_t tid = threadIdx.x;
  const uint64_t base = block_base(xcd_block(blockIdx.x, gridDim.x), a.g);
  R v[E];
  int w = a.g.tb - EB;
#pragma unroll
  for (int k = 0; k < E; ++k) v[k] = (R)data[base + tile_off(tmap<EB>(tid, k, w), a.g)];
  for (int ci = 0; ci < a.g.nchunks; ++ci) {
    const Chunk ch = a.g.chunk[ci];
    if (ch.w != w) {
#pragma unroll
      for (int k = 0; k < E; ++k) lds[swz<sizeof(T)>(tmap<EB>(tid, k, w), EB)] = (T)v[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = (R)lds[swz<sizeof(T)>(tmap<EB>(tid, k, ch.w), EB)];
      __syncthreads();
      w = ch.w;
    }
#pragma unroll
    for (int j = 0; j < EB; ++j) {
      if (j >= ch.jlo && j < ch.jhi) {
#pragma unroll
        for (int k = 0; k < E; ++k) {
          if (!(k & (1 << j))) {
            const R u = v[k], x = v[k | (1 << j)];
            v[k] = u + x;
            v[k | (1 << j)] = u - x;
          }
        }
      }
    }
  }
  if (w != a.g.w_store) {
#pragma unroll
    for (int k = 0; k < E; ++k) lds[swz<sizeof(T)>(tmap<EB>(tid, k, w), EB)] = (T)v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = (R)lds[swz<sizeof(T)>(tmap<EB>(tid, k, a.g.w_store), EB)];
    w = a.g.w_store;
  }
#pragma unroll
  for (int k = 0; k < E; ++k) data[base + tile_off(tmap<EB>(tid, k, w), a.g)] = (T)v[k];
}

// ----------------------------------------------------------------------------
// standalone expectation and finalisation
// ----------------------------------------------------------------------------
template <class S, class D>
__global__ void __launch_bounds__(256) expectation_kernel(const void* psi, const void* diag, double offset,
                                                          uint64_t N, double* partials) {
  const uint32_t nthr = blockDim.x;
  __shared__ double scratch[16];
  double e = 0.0, q = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) {
    double r, i;
    S::load(psi, x, r, i);
    const double pr = r * r + i * i;
    e += pr * (D::get(diag, x) + offset);
    q += pr;
  }
  block_sum2(e, q, scratch, nthr);
  if (threadIdx.x == 0) { partials[2 * blockIdx.x] = e; partials[2 * blockIdx.x + 1] = q; }
}

__global__ void __launch_bounds__(256) finalize_kernel(const double* partials, uint64_t count, double* out) {
  const uint32_t nthr = blockDim.x;
  __shared__ double scratch[16];
  double e = 0.0, q = 0.0;
  for (uint64_t i = threadIdx.x; i < count; i += blockDim.x) { e += partials[2 * i]; q += partials[2 * i + 1]; }
  block_sum2(e, q, scratch, nthr);
  if (threadIdx.x == 0) { out[0] = e; out[1] = q; }
}

template <class S>
__global__ void __launch_bounds__(256) fill_state_kernel(void* psi, uint64_t N, double amp) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) S::store(psi, x, amp, 0.0);
}

// ----------------------------------------------------------------------------
// precompute helpers
// ----------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) zero_kernel(T* p, uint64_t N) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) p[x] = (T)0;
}

template <typename T>
struct ScatterArgs {
  T* data;
  int count;
  uint64_t mask[kScatterChunk];
  T val[kScatterChunk];
};

template <typename T>
__global__ void __launch_bounds__(256) scatter_kernel(const ScatterArgs<T> a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.count) a.data[a.mask[i]] = a.val[i];
}

// per-block (min, max, OR of low bits) of an int32 vector
__global__ void __launch_bounds__(256) int_stats_kernel(const int32_t* p, uint64_t N, int32_t lowmask, int64_t* partials) {
  __shared__ int64_t smin[256], smax[256], sor[256];
  int64_t mn = INT64_MAX, mx = INT64_MIN, orr = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) {
    const int64_t v = p[x];
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
    orr |= (v & lowmask);
  }
  smin[threadIdx.x] = mn; smax[threadIdx.x] = mx; sor[threadIdx.x] = orr;
  __syncthreads();
  for (uint32_t s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smin[threadIdx.x] = smin[threadIdx.x + s] < smin[threadIdx.x] ? smin[threadIdx.x + s] : smin[threadIdx.x];
      smax[threadIdx.x] = smax[threadIdx.x + s] > smax[threadIdx.x] ? smax[threadIdx.x + s] : smax[threadIdx.x];
      sor[threadIdx.x] |= sor[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x] = smin[0];
    partials[3 * blockIdx.x + 1] = smax[0];
    partials[3 * blockIdx.x + 2] = sor[0];
  }
}

__global__ void __launch_bounds__(64) int_stats_finalize(const int64_t* partials, int count, int64_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int64_t mn = INT64_MAX, mx = INT64_MIN, orr = 0;
    for (int i = 0; i < count; ++i) {
      mn = partials[3 * i] < mn ? partials[3 * i] : mn;
      mx = partials[3 * i + 1] > mx ? partials[3 * i + 1] : mx;
      orr |= partials[3 * i + 2];
    }
    out[0] = mn; out[1] = mx; out[2] = orr;
  }
}

// dst[x] = (src[x] >> k) - sub   (src holds 2^k * c, exactly divisible)
template <typename TD>
__global__ void __launch_bounds__(256) narrow_kernel(const int32_t* src, TD* dst, uint64_t N, int k, int64_t sub) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride)
    dst[x] = (TD)((int64_t)(src[x] >> k) - sub);
}

}  // namespace qk
