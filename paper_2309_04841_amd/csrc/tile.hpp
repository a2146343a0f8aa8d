// tile.hpp -- tiled in-place butterfly sweeps over a 2^n vector (gfx950).
//
// A "sweep" is one read + one write of the whole vector.  Each workgroup owns
// one tile of 2^tb elements.  The tile's index bits map to global index bits as
//   tile bits [0, P)   -> global bits [0, P)          (passengers: contiguous,
//                                                      never butterflied in a
//                                                      high sweep)
//   tile bits [P, tb)  -> global bits [q0, q0+tb-P)   (active qubits)
// and the workgroup index fills the remaining global bits (first [P, q0), then
// [q0+tb-P, n)).  A "low" sweep has P = 0, q0 = 0: a contiguous tile whose bits
// are all active.
//
// Every thread holds 2^EB elements in registers.  For a register "window" w the
// thread's k-th element is tile element
//   t(tid, k, w) = (tid mod 2^w) | k << w | (tid >> w) << (w + EB),
// so the EB tile bits [w, w+EB) are register bits and butterflies on them need
// no communication.  Moving to another window goes through LDS (write under the
// old mapping, barrier, read under the new).  Window tb-EB is the coalesced
// load mapping (t = k * threads + tid).
//
// Because the single-qubit gates of the mixer (and the 2x2 Hadamard factors of
// the Walsh-Hadamard transform) act on distinct qubits and commute, the active
// bits can be processed in any order; the host picks an order of windows that
// minimises LDS round trips and ends on a store-friendly window.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qk {

constexpr int kMaxChunks = 8;

struct Chunk {
  int8_t w;    // register window: tile bits [w, w+EB)
  int8_t jlo;  // butterflies on register bits [jlo, jhi) of that window
  int8_t jhi;
  int8_t pad;
};

struct TileGeom {
  int tb;       // tile bits
  int P;        // passenger bits
  int q0;       // global bit of tile bit P
  int nchunks;  // chunks per layer
  int w_store;  // window the tile is stored from
  Chunk chunk[kMaxChunks];
};

template <int EB>
__device__ __forceinline__ uint32_t tmap(uint32_t tid, uint32_t k, int w) {
  const uint32_t lo = tid & ((1u << w) - 1u);
  return lo | (k << w) | ((tid >> w) << (w + EB));
}

// Thread part of the window-w mapping: t(tid, k, w) = thr(tid, w) | k << w.
template <int EB>
__device__ __forceinline__ uint32_t thr_part(uint32_t tid, int w) {
  return (tid & ((1u << w) - 1u)) | ((tid >> w) << (w + EB));
}

// Global offset of tile element t relative to the block base.  tile_off maps
// tile bits to disjoint global bits, so tile_off(a | b) = tile_off(a) +
// tile_off(b) for disjoint a, b: addresses split into a per-thread part and a
// per-register part that is uniform across the workgroup.
__device__ __forceinline__ uint64_t tile_off(uint32_t t, int P, int q0) {
  const uint32_t pm = (1u << P) - 1u;
  return (uint64_t)(t & pm) | ((uint64_t)(t >> P) << q0);
}

// Global index of element 0 of block b.
__device__ __forceinline__ uint64_t block_base(uint64_t b, int tb, int P, int q0) {
  const int nlow = q0 - P;
  const uint64_t blo = b & ((1ull << nlow) - 1ull);
  const uint64_t bhi = b >> nlow;
  return (blo << P) | (bhi << (q0 + tb - P));
}

// LDS position of tile element t: pos = t ^ L(t >> S), L linear over GF(2)
// into the low S bits (so pos is a permutation of the tile).  The maps are
// chosen so that every register window's access pattern is free of bank
// conflicts (64 banks x 4 B): for 16-byte elements each group of 16 lanes, for
// 8-byte elements each group of 32 lanes, hits distinct banks.  Linearity also
// splits pos(thr | k << w) = pos(thr) ^ pos(k << w) into a per-thread part and
// a workgroup-uniform part.
template <int ELEM_BYTES>
struct Swz;
template <>
struct Swz<16> {
  static constexpr int kShift = 4;
  static constexpr int kCols = 4;
  __host__ __device__ static constexpr uint32_t col(int j) { return 1u << j; }
};
template <>
struct Swz<8> {
  static constexpr int kShift = 5;
  static constexpr int kCols = 9;
  __host__ __device__ static constexpr uint32_t col(int j) {
    constexpr uint32_t c[9] = {2, 28, 8, 25, 28, 1, 17, 5, 16};
    return c[j];
  }
};
template <>
struct Swz<4> {
  static constexpr int kShift = 5;
  static constexpr int kCols = 5;
  __host__ __device__ static constexpr uint32_t col(int j) { return 1u << j; }
};
template <>
struct Swz<2> : Swz<4> {};

template <int ELEM_BYTES>
__device__ __forceinline__ uint32_t swz(uint32_t t) {
  using Z = Swz<ELEM_BYTES>;
  uint32_t x = 0;
#pragma unroll
  for (int j = 0; j < Z::kCols; ++j) x ^= ((t >> (Z::kShift + j)) & 1u) ? Z::col(j) : 0u;
  return t ^ x;
}

}  // namespace qk
