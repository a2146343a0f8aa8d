// tile.hpp -- tiled in-place butterfly sweeps over a 2^n vector (gfx950).
//
// A "sweep" is one read + one write of the whole vector.  Each workgroup owns
// one tile of 2^tb elements.  Tile bits map to global index bits as
//   tile bits [0, R)              -> global bits [0, R)       (the contiguous run)
//   tile bits [R, R + hA)         -> global bits [qA, qA + hA)  (segment A)
//   tile bits [R + hA, tb)        -> global bits [qB, qB + hB)  (segment B)
// with R <= qA, qA + hA <= qB, qB + hB <= n, and the workgroup index fills the
// remaining global bits in increasing order.  Tile bits [act_lo, tb) are the
// active qubits of the sweep: act_lo = 0 in the first sweep of a layer (the
// run is active too), act_lo = R in the others (the run's qubits are only
// passengers that make each row a contiguous burst).  Two segments let the
// planner spread the qubits above the 2 MiB page boundary over all sweeps, so
// no sweep touches hundreds of pages per workgroup.
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
constexpr int kMaxWin = 11;  // register windows w in [0, 10] (tiles of up to 2^14, >= 8 elements per thread)
// Windows w <= kLocalWin place every thread bit >= 6 (the wave index within the
// workgroup) above the register bits, at the same tile bits: a change between
// two such windows keeps each element in its wave.
constexpr int kLocalWin = 6;

struct Chunk {
  int8_t w;    // register window: tile bits [w, w+EB)
  int8_t jlo;  // butterflies on register bits [jlo, jhi) of that window
  int8_t jhi;
  int8_t pad;
};

struct TileGeom {
  int tb;       // tile bits
  int R;        // contiguous run: tile bits [0, R) = global bits [0, R)
  int hA, qA;   // segment A: tile bits [R, R + hA) = global bits [qA, qA + hA)
  int qB;       // segment B: tile bits [R + hA, tb) = global bits [qB, qB + tb - R - hA)
  int act_lo;   // active tile bits [act_lo, tb)
  int nchunks;  // chunks per layer
  int w_store;  // window the tile is stored from
  int part;     // index of the short chunk the fused sweeps specialise (bits [jlo, EB) of its window), or -1
  Chunk chunk[kMaxChunks];
  // Per-register parts of the addresses for register window w, filled on the
  // host (uniform across the workgroup, so the kernels read them with scalar
  // loads instead of recomputing them at every window change):
  //   goff[w][k] = tile_off(k << w): global element offset of register k
  //   loff[w][k] = swz(k << w, eb) * LDS entry bytes: LDS byte offset part of register k
  uint64_t goff[kMaxWin][16];
  uint32_t loff[kMaxWin][16];
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
__host__ __device__ __forceinline__ uint64_t tile_off(uint32_t t, const TileGeom& g) {
  const uint32_t rm = (1u << g.R) - 1u, am = (1u << g.hA) - 1u;
  return (uint64_t)(t & rm) | ((uint64_t)((t >> g.R) & am) << g.qA) | ((uint64_t)(t >> (g.R + g.hA)) << g.qB);
}

// Global index of element 0 of block b: b's bits fill the gaps [R, qA),
// [qA + hA, qB) and [qB + hB, n) in that order.
__device__ __forceinline__ uint64_t block_base(uint64_t b, const TileGeom& g) {
  const int g1 = g.qA - g.R;
  const int g2 = g.qB - (g.qA + g.hA);
  const int topB = g.qB + (g.tb - g.R - g.hA);
  const uint64_t lo = b & ((1ull << g1) - 1ull);
  b >>= g1;
  const uint64_t mid = b & ((1ull << g2) - 1ull);
  b >>= g2;
  return (lo << g.R) | (mid << (g.qA + g.hA)) | (b << topB);
}

// LDS position of tile element t for tiles held as 2^eb elements per thread:
// pos = t ^ ((t >> eb) & m), m = 31 for 8-byte entries (complex64, and the
// split complex128 exchanges), 15 for 16-byte ones: the low bits are XORed with
// the bits just above the register bits (a unitriangular map over GF(2), so pos
// is a permutation of the tile).  It keeps every register window's accesses free
// of bank conflicts on gfx950, whose LDS serves the two directions differently
// (measured with the SQ_LDS_BANK_CONFLICT counter): ds_read_b64 serves 32 lanes
// per cycle from 64 banks of 4 bytes, ds_write_b64 16 lanes from 32 banks,
// ds_write_b128 8 lanes from 32 banks; the read and write counters are zero for
// this map in every window, for 8 and 16 elements per thread.  (A map chosen
// against the read pattern alone left 4 extra cycles on every 8-byte write in
// windows 0, 2 and 3, and 8 on 16-byte writes in windows 1 and 2.)  Linearity
// splits pos(thr | k << w) = pos(thr) ^ pos(k << w) into a per-thread part and a
// workgroup-uniform part.  Cost-vector tiles (4- and 2-byte entries) use
// pos = t ^ ((t >> 5) & 31).
template <int ELEM_BYTES>
__host__ __device__ __forceinline__ uint32_t swz(uint32_t t, int eb) {
  if constexpr (ELEM_BYTES == 16) return t ^ ((t >> eb) & 15u);
  else if constexpr (ELEM_BYTES == 8) return t ^ ((t >> eb) & 31u);
  else return t ^ ((t >> 5) & 31u);
}

// Fill goff / loff for `eb` register bits and LDS entries of LDS_BYTES.
template <int LDS_BYTES>
inline void fill_reg_offsets(TileGeom& g, int eb) {
  for (int w = 0; w < kMaxWin; ++w)
    for (int k = 0; k < 16; ++k) {
      const bool used = k < (1 << eb) && w + eb <= g.tb;
      g.goff[w][k] = used ? tile_off((uint32_t)k << w, g) : 0;
      g.loff[w][k] = used ? swz<LDS_BYTES>((uint32_t)k << w, eb) * LDS_BYTES : 0;
    }
}
}  // namespace qk
