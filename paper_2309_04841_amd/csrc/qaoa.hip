// qaoa.hip -- host side of libqaoa.so: argument validation, sweep planning,
// kernel launches and the C ABI declared in include/qaoa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "qaoa.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(QAOA_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK(what)                                                                \
  do {                                                                                    \
    hipError_t e_ = hipGetLastError();                                                    \
    if (e_ != hipSuccess) return fail(QAOA_ERR_DEVICE, "launch of %s failed: %s", what, hipGetErrorString(e_)); \
  } while (0)

constexpr int kEB = 4;                 // 16 elements per thread
constexpr int kExpectBlocks = 2048;    // fixed grid of the standalone expectation
constexpr int kStatBlocks = 1024;      // fixed grid of the integer range check

size_t state_elem_bytes(int dt) { return dt == QAOA_C128 ? 16 : 8; }
size_t diag_elem_bytes(int dt) { return dt == QAOA_DIAG_F64 ? 8 : dt == QAOA_DIAG_I32 ? 4 : 2; }
bool valid_state_dtype(int dt) { return dt == QAOA_C64 || dt == QAOA_C128; }
bool valid_diag_dtype(int dt) { return dt == QAOA_DIAG_F64 || dt == QAOA_DIAG_I32 || dt == QAOA_DIAG_U16; }

// Largest tile (log2 elements) per dtype: 64 KiB of LDS per workgroup, so two
// workgroups fit in a CU's 160 KiB and overlap memory with exchanges.
// Capped so a tile never needs more than 512 threads (2^(cap - eb)).
int tile_bits_for_bytes(size_t elem_bytes, int cap) {
  int tb = 0;
  while (tb < cap && ((size_t)1 << (tb + 1)) * elem_bytes <= 65536) ++tb;
  return tb;
}
// Minimum passenger bits so that a high sweep touches >= run_bytes contiguous bytes.
int min_passenger_bits(size_t elem_bytes, size_t run_bytes = 128) {
  int p = 0;
  while (((size_t)1 << p) * elem_bytes < run_bytes) ++p;
  return p;
}

// Chunk order for one tile: first the top EB bits (the coalesced load window),
// then the remaining active bits bottom-up; the tile is stored from the last
// window if that window keeps >= 2^store_min_bits contiguous elements per run,
// else it is exchanged back to the load window first.  The lower chunks use
// windows w <= qk::kLocalWin where they can: in all such windows the thread
// bits >= 6 (a thread's wave) map to the same tile bits, so changing between
// them moves data only within each wave and needs no workgroup barrier.
//
// local_load (tiles of 1024 threads, whose top window is not wave-local): the
// lower active bits are split around window kLocalWin instead, whose chunk
// comes first and is the load (and fused store) window, then the other lower
// chunks (a short one last among them), then the top chunk.  Each wave then
// loads, applies the local chunks and, at the end, stores without waiting for
// the others; only the changes into and out of the top window meet at
// barriers.  In window kLocalWin the lanes are tile bits [0, 6), so loads stay
// coalesced as in the top window.
qk::TileGeom make_geom(int tb, int R, int hA, int qA, int qB, int act_lo, int eb, int store_min_bits,
                       bool local_load = false) {
  qk::TileGeom g{};
  g.tb = tb; g.R = R; g.hA = hA; g.qA = qA; g.qB = qB; g.act_lo = act_lo; g.nchunks = 0; g.part = -1;
  const int top_w = tb - eb;
  const int lo0 = std::max(act_lo, top_w);
  const qk::Chunk top{(int8_t)top_w, (int8_t)(lo0 - top_w), (int8_t)eb, 0};
  // chunks over [lo, hi), bottom-up; a short last one sits at the top of its window
  // (jhi = eb), the form the fused kernels specialise
  auto split = [&](int lo, int hi, std::vector<qk::Chunk>& out) {
    while (lo < hi) {
      const int chi = std::min(lo + eb, hi);
      const int w = (chi - lo < eb && chi >= eb) ? chi - eb : std::max(chi - eb, std::min(lo, qk::kLocalWin));
      out.push_back(qk::Chunk{(int8_t)w, (int8_t)(lo - w), (int8_t)(chi - w), 0});
      lo = chi;
    }
  };
  auto is_short = [&](const qk::Chunk& c) { return c.jlo > 0 && c.jhi == eb; };
  const int wl = qk::kLocalWin;
  if (local_load && top_w > wl + eb - 1 && top.jlo == 0 && act_lo <= wl && lo0 == wl + eb) {
    std::vector<qk::Chunk> low;
    split(act_lo, wl, low);
    int nshort = 0;
    bool ok = true;
    for (size_t i = 0; i < low.size(); ++i) {
      if (is_short(low[i])) { ++nshort; ok = ok && i + 1 == low.size(); }
      else ok = ok && low[i].jlo == 0 && low[i].jhi == eb;
    }
    if (ok && nshort <= 1) {
      g.chunk[g.nchunks++] = qk::Chunk{(int8_t)wl, 0, (int8_t)eb, 0};
      for (const auto& c : low) {
        if (is_short(c)) g.part = g.nchunks;
        g.chunk[g.nchunks++] = c;
      }
      g.chunk[g.nchunks++] = top;
      g.w_store = top_w;  // coalesced like window kLocalWin; plain sweeps end there
      return g;
    }
  }
  g.chunk[g.nchunks++] = top;
  std::vector<qk::Chunk> low;
  split(act_lo, lo0, low);
  for (const auto& c : low) g.chunk[g.nchunks++] = c;
  if (is_short(g.chunk[g.nchunks - 1])) g.part = g.nchunks - 1;
  const int last_w = g.chunk[g.nchunks - 1].w;
  g.w_store = (std::min(last_w, R) >= store_min_bits || last_w == top_w) ? last_w : top_w;
  return g;
}

// Sweep plan covering all n qubits with tiles of at most tbmax bits.
struct Plan {
  bool single;          // whole vector in one tile
  bool wide;            // complex128 tiles of up to 2^14 elements (qk::C128W)
  int eb;               // register bits per thread
  std::vector<qk::TileGeom> sweeps;
};

// Qubits at or above this bit select the 2 MiB page of an element.
int page_bit(size_t elem_bytes) {
  int b = 0;
  while (((size_t)1 << (b + 1)) * elem_bytes <= ((size_t)2 << 20)) ++b;
  return b;
}

// The first sweep of a layer takes the contiguous low qubits [0, R0) plus m0
// qubits at the top; the other sweeps take P passengers [0, P) plus a segment
// of the remaining low qubits and a segment of the remaining page-selecting
// qubits.  m0 and the split are chosen to minimise the largest number of
// page-selecting qubits in any sweep (2^that = pages a workgroup touches),
// keeping the sweep count of the plain split.
Plan make_plan(int n, size_t elem_bytes, int eb = kEB, int tb_cap = 0, size_t run_bytes = 128,
               bool local_load = false) {
  Plan pl;
  pl.wide = false;
  const int tbmax = tb_cap ? tb_cap : tile_bits_for_bytes(elem_bytes, 9 + eb);
  const int pmin = min_passenger_bits(elem_bytes, run_bytes);
  const int smin = pmin;  // store runs of >= 128 B
  if (n <= tbmax) {
    pl.single = true;
    pl.eb = std::min(eb, n);
    pl.sweeps.push_back(make_geom(n, n, 0, n, n, 0, pl.eb, 0));
    return pl;
  }
  pl.single = false;
  pl.eb = eb;
  const int hmax = tbmax - pmin;
  const int k = 1 + (n - tbmax + hmax - 1) / hmax;  // sweeps per layer
  const int pb = std::max(page_bit(elem_bytes), tbmax);
  const int npage = std::max(0, n - pb);
  const int r0_min = std::max(pmin + 4, tbmax - 6);
  int best_m0 = 0, best_cost = 1 << 30;
  std::vector<int> best_h, best_b;
  for (int m0 = 0; tbmax - m0 >= r0_min && m0 <= npage; ++m0) {
    const int R0 = tbmax - m0;
    const int T = n - m0 - R0;  // qubits left for the other sweeps
    if (T > (k - 1) * hmax) continue;
    std::vector<int> h(k - 1), b(k - 1);
    for (int i = 0; i < k - 1; ++i) h[i] = T / (k - 1) + (i < T % (k - 1) ? 1 : 0);
    int rem = npage - m0;
    bool ok = true;
    for (int i = 0; i < k - 1; ++i) {
      const int share = rem / (k - 1 - i) + (rem % (k - 1 - i) ? 1 : 0);
      b[i] = std::min(share, h[i]);
      rem -= b[i];
      if (h[i] < m0 && m0 > 0) ok = false;  // passengers [0, tbmax - h) must stay inside [0, R0)
    }
    if (rem != 0 || !ok) continue;
    int cost = m0;
    for (int i = 0; i < k - 1; ++i) cost = std::max(cost, b[i]);
    if (cost < best_cost) { best_cost = cost; best_m0 = m0; best_h = h; best_b = b; }
  }
  const int m0 = best_m0, R0 = tbmax - m0;
  // first sweep: run [0, R0) + segment [n - m0, n), all active
  pl.sweeps.push_back(make_geom(tbmax, R0, m0, n - m0, n, 0, eb, smin, local_load));
  int xa = R0, xb = std::max(pb, R0);
  for (int i = 0; i < k - 1; ++i) {
    const int h = best_h[i], bpage = best_b[i], a = h - bpage, P = tbmax - h;
    const int qA = a ? xa : xb;         // an empty segment A sits where B starts
    const int qB = bpage ? xb : qA + a;  // an empty segment B sits where A ends
    pl.sweeps.push_back(make_geom(tbmax, P, a, qA, qB, P, eb, smin, local_load));
    xa += a;
    xb += bpage;
  }
  return pl;
}

uint64_t plan_blocks(int n, const qk::TileGeom& g) { return (uint64_t)1 << (n - g.tb); }

// Forward plan of a state.  complex128 states above 2^14 elements also try
// 2^14-element tiles (qk::C128W), first with 128-byte passenger runs, then
// with 64-byte runs, and take them when they need fewer sweeps per layer.
constexpr int kWideTileBits = 14;
std::atomic<int> g_wide_tiles{1};   // QAOA_TUNE_WIDE_TILES
std::atomic<int> g_fuse_layers{1};  // QAOA_TUNE_FUSE_LAYERS

// The knobs as one entry point sees them: read once per call and passed to
// every step that plans, sizes or launches, so a concurrent qaoa_set_tuning
// cannot give one call two different plans.
struct Tuning {
  bool wide, fuse;
};
Tuning tuning_now() { return Tuning{g_wide_tiles.load() != 0, g_fuse_layers.load() != 0}; }

Plan state_plan(int n, int state_dtype, bool wide) {
  const size_t S = state_elem_bytes(state_dtype);
  Plan best = make_plan(n, S);
  if (state_dtype != QAOA_C128 || n <= kWideTileBits || !wide) return best;
  for (size_t run : {(size_t)128, (size_t)64}) {
    Plan w = make_plan(n, S, kEB, kWideTileBits, run, true);
    if (w.sweeps.size() < best.sweeps.size()) {
      w.wide = true;
      best = w;
    }
  }
  return best;
}

// Launch order of a multi-tile evaluation.  The mixer gates of a layer commute
// (one gate per qubit), so layer l runs its sweeps in plan order when l is
// even and in reverse order when l is odd.  The last sweep of layer l and the
// first of layer l+1 then cover the same qubits and merge into one fused
// launch: mixer gates of layer l, phase of layer l+1 (all of layer l is done
// by then), mixer gates of layer l+1.  p layers of s sweeps take
// 1 + (s-1) p launches instead of s p.
struct SweepStep {
  int sweep;  // index into Plan::sweeps
  int layer;  // first layer this launch applies
  int flags;  // qk::F_*
};
// Reverse pass of the gradient: layers p-1 .. 0, each run with alternating
// sweep order; the last sweep of layer l > 0 also undoes layer l's phase (all
// of layer l's gates are undone by then) and layer l-1's gates on the same
// qubits.  `layer` is the layer undone first; flags are qk::A_*.
std::vector<SweepStep> adjoint_schedule(int nsw, int p, bool fuse) {
  std::vector<SweepStep> out;
  if (!fuse) {  // layers p-1..0, sweeps nsw-1..0, phase undone in sweep 0
    for (int l = p - 1; l >= 0; --l)
      for (int sw = nsw - 1; sw >= 0; --sw)
        out.push_back(SweepStep{sw, l, (l == p - 1 && sw == nsw - 1 ? qk::A_FIRST : 0) | (sw == 0 ? qk::A_PHASE : 0)});
    return out;
  }
  for (int l = p - 1; l >= 0; --l) {
    const int r = p - 1 - l;
    for (int i = (l == p - 1 ? 0 : 1); i < nsw; ++i) {  // position 0 of layer l < p-1 ran fused
      const int sw = (r & 1) ? i : nsw - 1 - i;
      int flags = 0;
      if (l == p - 1 && i == 0) flags |= qk::A_FIRST;
      if (i == nsw - 1) flags |= (l > 0) ? qk::A_FUSE : qk::A_PHASE;
      out.push_back(SweepStep{sw, l, flags});
    }
  }
  return out;
}

std::vector<SweepStep> sweep_schedule(int nsw, int p, bool init, bool expv, bool fuse) {
  std::vector<SweepStep> out;
  if (!fuse) {  // every layer in plan order, phase in its first sweep
    for (int l = 0; l < p; ++l)
      for (int sw = 0; sw < nsw; ++sw) {
        int flags = sw == 0 ? qk::F_PHASE | ((l == 0 && init) ? qk::F_INIT : 0) : 0;
        if (l == p - 1 && sw == nsw - 1 && expv) flags |= qk::F_EXPV;
        out.push_back(SweepStep{sw, l, flags});
      }
    return out;
  }
  for (int l = 0; l < p; ++l) {
    for (int i = (l == 0 ? 0 : 1); i < nsw; ++i) {  // position 0 of layer l > 0 ran fused
      const int sw = (l & 1) ? nsw - 1 - i : i;
      int flags = 0;
      if (l == 0 && i == 0) flags |= qk::F_PHASE | (init ? qk::F_INIT : 0);
      if (i == nsw - 1) flags |= (l + 1 < p) ? qk::F_FUSE : (expv ? qk::F_EXPV : 0);
      out.push_back(SweepStep{sw, l, flags});
    }
  }
  return out;
}

// Reverse (adjoint) sweeps hold two states per thread: 8 elements of each.
constexpr int kEBAdj = 3;
// complex128 reverse sweeps use 2^11-element tiles when that costs no sweep:
// their fused variant needs ~235 registers per lane, so a 2^12-element tile's
// 512 threads fill a compute unit alone, while two 256-thread workgroups of
// 2^11 elements share it and overlap one's memory phase with the other's
// arithmetic (LABS n=24 p=20 gradient: 13.2 -> 12.4 ms).
Plan adjoint_plan(int n, size_t state_bytes) {
  Plan a = make_plan(n, state_bytes, kEBAdj);
  if (state_bytes == 16 && !a.single) {
    Plan b = make_plan(n, state_bytes, kEBAdj, 11);
    if (!b.single && b.sweeps.size() <= a.sweeps.size()) return b;
  }
  return a;
}

// ---------------------------------------------------------------------------
// XY mixer plans (Section 3.2).  One layer is an ordered edge sequence
// (ring: (i, i+1) for even i, then odd i, then the wrap edge (n-1, 0) when
// n > 2; complete graph: (i, j), i < j, lexicographic).  A sweep applies a
// subset of the pending gates, in an order that keeps every pair of gates
// sharing a qubit in sequence, to tiles that hold all its qubits plus the
// passenger bits [0, pmin) for coalescing; the tile's bits must form the run
// [0, R) and at most two more contiguous segments (the tile geometry).
// ---------------------------------------------------------------------------
constexpr int kXyTileBits = 12;  // 2^12 complex128 LDS entries = 64 KiB

std::vector<std::pair<int, int>> xy_edges(int n, int mixer) {
  std::vector<std::pair<int, int>> e;
  if (mixer == QAOA_MIXER_XY_RING) {
    for (int par = 0; par < 2; ++par)
      for (int i = par; i + 1 < n; i += 2) e.emplace_back(i, i + 1);
    if (n > 2) e.emplace_back(n - 1, 0);
  } else {
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) e.emplace_back(i, j);
  }
  return e;
}

struct XySweep {
  qk::TileGeom g;
  std::vector<std::pair<int, int>> gates;  // tile bits
};
struct XyPlan {
  bool single;
  int eb;
  std::vector<XySweep> sweeps;
};

// Runs of consecutive set bits in `bits` (sorted): (start, length).
std::vector<std::pair<int, int>> bit_runs(const std::vector<int>& bits) {
  std::vector<std::pair<int, int>> r;
  for (int b : bits) {
    if (!r.empty() && r.back().first + r.back().second == b) ++r.back().second;
    else r.emplace_back(b, 1);
  }
  return r;
}

// Tile bits of a qubit set (bit mask q): the set plus [0, pmin); fits if at
// most tbmax bits forming the run from 0 and at most two more runs.
bool xy_fits(uint64_t q, int pmin, int tbmax) {
  const uint64_t b = q | ((1ull << pmin) - 1ull);
  if (__builtin_popcountll(b) > tbmax) return false;
  const int runs = __builtin_popcountll(b & ~(b << 1));
  return runs - (int)(b & 1ull) <= 2;
}

// One pass over the pending gates in order with qubit set q: a gate is taken
// when both qubits are in q and neither is blocked; any other gate blocks its
// qubits (every later gate on them must follow it).  Returns the count taken
// and, if `taken` is given, their indices in order.
int xy_pass(const std::vector<std::pair<int, int>>& pend, uint64_t q, std::vector<size_t>* taken) {
  uint64_t blocked = 0;
  int cnt = 0;
  for (size_t e = 0; e < pend.size(); ++e) {
    const uint64_t m = (1ull << pend[e].first) | (1ull << pend[e].second);
    if (!(blocked & m) && (q & m) == m) {
      ++cnt;
      if (taken) taken->push_back(e);
    } else {
      blocked |= m;
    }
  }
  return cnt;
}

XySweep xy_sweep(int n, const std::set<int>& q, const std::vector<std::pair<int, int>>& edges, int pmin, int tbmax) {
  std::set<int> b(q);
  for (int i = 0; i < pmin; ++i) b.insert(i);
  for (int x = 0; (int)b.size() < tbmax && x < n; ++x) b.insert(x);  // pad: extend the run from 0
  const std::vector<int> bits(b.begin(), b.end());
  auto runs = bit_runs(bits);
  XySweep sw{};
  qk::TileGeom& g = sw.g;
  g.tb = (int)bits.size();
  g.R = runs.front().first == 0 ? runs.front().second : 0;
  if (g.R > 0) runs.erase(runs.begin());
  if (runs.empty()) { g.hA = 0; g.qA = g.qB = n; }
  else if (runs.size() == 1) { g.hA = runs[0].second; g.qA = runs[0].first; g.qB = g.qA + g.hA; }
  else { g.hA = runs[0].second; g.qA = runs[0].first; g.qB = runs[1].first; }
  g.act_lo = 0;
  g.nchunks = 0;
  g.w_store = 0;
  auto tbit = [&](int x) {
    return (int)(std::lower_bound(bits.begin(), bits.end(), x) - bits.begin());  // bits sorted = tile bit order
  };
  for (const auto& e : edges) sw.gates.emplace_back(tbit(e.first), tbit(e.second));
  return sw;
}

XyPlan build_xy_plan(int n, int mixer, size_t elem_bytes) {
  XyPlan pl;
  const auto edges = xy_edges(n, mixer);
  if (n <= kXyTileBits) {
    pl.single = true;
    pl.eb = std::min(kEB, n);
    std::set<int> all;
    for (int i = 0; i < n; ++i) all.insert(i);
    pl.sweeps.push_back(xy_sweep(n, all, edges, 0, n));
    return pl;
  }
  pl.single = false;
  pl.eb = kEB;
  const int pmin = min_passenger_bits(elem_bytes);
  // Gates on disjoint qubits commute, so a sweep may take any gate whose
  // earlier neighbours (earlier gates sharing a qubit) are all applied: the
  // gates one xy_pass takes.  Each sweep grows its qubit set from the
  // passengers, adding the qubit (or, when no single qubit helps, the pair of
  // one of the first pending gates) that lets the pass take the most gates,
  // while the set fits a tile.  The first pending gate always fits with the
  // passengers, so every sweep makes progress.
  std::vector<std::pair<int, int>> pend = edges;
  while (!pend.empty()) {
    uint64_t q = (1ull << pmin) - 1ull;
    for (;;) {
      int best = xy_pass(pend, q, nullptr);
      uint64_t add = 0, cand = 0;
      for (const auto& e : pend) cand |= (1ull << e.first) | (1ull << e.second);
      cand &= ~q;
      for (int c = 0; c < n; ++c) {
        if (!((cand >> c) & 1ull) || !xy_fits(q | (1ull << c), pmin, kXyTileBits)) continue;
        const int cnt = xy_pass(pend, q | (1ull << c), nullptr);
        if (cnt > best) { best = cnt; add = 1ull << c; }
      }
      if (!add) {
        for (size_t e = 0; e < pend.size() && e < 40; ++e) {
          const uint64_t m = (1ull << pend[e].first) | (1ull << pend[e].second);
          if ((q | m) == q || !xy_fits(q | m, pmin, kXyTileBits)) continue;
          const int cnt = xy_pass(pend, q | m, nullptr);
          if (cnt > best) { best = cnt; add = m & ~q; }
        }
      }
      if (!add) break;
      q |= add;
    }
    std::vector<size_t> taken;
    xy_pass(pend, q, &taken);
    std::vector<std::pair<int, int>> run;
    std::vector<char> used(pend.size(), 0);
    for (size_t e : taken) { run.push_back(pend[e]); used[e] = 1; }
    std::vector<std::pair<int, int>> rest;
    for (size_t e = 0; e < pend.size(); ++e)
      if (!used[e]) rest.push_back(pend[e]);
    pend.swap(rest);
    std::set<int> qs;
    for (int b = 0; b < n; ++b)
      if ((q >> b) & 1ull) qs.insert(b);
    pl.sweeps.push_back(xy_sweep(n, qs, run, pmin, kXyTileBits));
  }
  return pl;
}

// Plans are built once per (n, mixer, element size) and kept for the process.
XyPlan make_xy_plan(int n, int mixer, size_t elem_bytes) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, size_t>, XyPlan> cache;
  const auto key = std::make_tuple(n, mixer, elem_bytes);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it == cache.end()) it = cache.emplace(key, build_xy_plan(n, mixer, elem_bytes)).first;
  return it->second;
}

// ---------------------------------------------------------------------------
// typed launchers
// ---------------------------------------------------------------------------
// LDS bytes of a tile kernel: the tile, the phase tables when the launch
// applies a phase with an integer cost vector, and at least the reduction
// scratch (16 doubles, or 2 per thread for a partial wave), which is only
// used after the tile and the tables are done with.
template <class S, class D>
size_t tile_lds_bytes(const qk::TileGeom& g, uint32_t threads, bool phase) {
  const size_t tile = ((size_t)1 << g.tb) * S::kLdsBytes;
  // tables, then one flag word per wave (16) for the range check
  const size_t tab = (D::kTable && phase) ? D::kTabLds * sizeof(double2) + 16 * sizeof(uint32_t) : 0;
  return std::max<size_t>(tile + tab, std::max<size_t>(16, 2 * threads) * sizeof(double));
}

// A copy of the launch arguments with the per-register offset tables of the
// geometry filled for state policy S and `eb` register bits.
template <class S, class Args>
Args with_offsets(const Args& a, int eb) {
  Args b = a;
  qk::fill_reg_offsets<S::kLdsBytes>(b.g, eb);
  return b;
}

template <class S, class D, bool INIT, bool PHASE, bool EXPV, bool FUSE = false, int PLO = 0, int PHI = 0>
void launch_sweep_f(const qk::SweepArgs& a, uint64_t blocks, uint32_t sets, hipStream_t st) {
  const uint32_t threads = 1u << (a.g.tb - kEB);
  const size_t lds = tile_lds_bytes<S, D>(a.g, threads, PHASE || FUSE);
  hipLaunchKernelGGL((qk::qaoa_sweep_kernel<S, D, kEB, INIT, PHASE, EXPV, FUSE, PLO, PHI>),
                     dim3((uint32_t)blocks, sets), dim3(threads), lds, st, with_offsets<S>(a, kEB));
}

// Sweeps specialise a plan's short chunk g.part (register bits [1, 4), [2, 4)
// or [3, 4) of its window: plans put short chunks at the top of their window),
// so its other bits take no identity butterflies.
template <class S, class D, bool INIT, bool PHASE, bool EXPV, bool FUSE>
void launch_sweep_p(const qk::SweepArgs& a, uint64_t blocks, uint32_t sets, hipStream_t st) {
  const qk::Chunk last = a.g.part >= 0 ? a.g.chunk[a.g.part] : qk::Chunk{0, 0, 0, 0};
  if (last.jhi == kEB && last.jlo == 1) launch_sweep_f<S, D, INIT, PHASE, EXPV, FUSE, 1, 4>(a, blocks, sets, st);
  else if (last.jhi == kEB && last.jlo == 2) launch_sweep_f<S, D, INIT, PHASE, EXPV, FUSE, 2, 4>(a, blocks, sets, st);
  else if (last.jhi == kEB && last.jlo == 3) launch_sweep_f<S, D, INIT, PHASE, EXPV, FUSE, 3, 4>(a, blocks, sets, st);
  else launch_sweep_f<S, D, INIT, PHASE, EXPV, FUSE>(a, blocks, sets, st);
}

// One sweep launch.  The schedules only produce these flag combinations: the
// phase sweep that opens the first layer (|+> generated in registers when
// init), plain mixer sweeps, fused sweeps (layer l's last sweep + layer l+1's
// phase + the same qubits of layer l+1) and the reducing last sweep.
template <class S, class D>
int launch_sweep_d(const qk::SweepArgs& a, uint64_t blocks, uint32_t sets, hipStream_t st) {
  const bool init = a.flags & qk::F_INIT, phase = a.flags & qk::F_PHASE, expv = a.flags & qk::F_EXPV;
  const bool fuse = a.flags & qk::F_FUSE;
  if (fuse) {
    if (init || phase || expv)
      return fail(QAOA_ERR_UNSUPPORTED, "internal: sweep flag combination %d not instantiated", a.flags);
    launch_sweep_p<S, D, false, false, false, true>(a, blocks, sets, st);
  } else if (phase && !expv) {
    if (init) launch_sweep_p<S, D, true, true, false, false>(a, blocks, sets, st);
    else launch_sweep_p<S, D, false, true, false, false>(a, blocks, sets, st);
  } else if (!init && !phase) {
    if (expv) launch_sweep_p<S, D, false, false, true, false>(a, blocks, sets, st);
    else launch_sweep_p<S, qk::DF64, false, false, false, false>(a, blocks, sets, st);  // does not read the cost vector
  } else {
    return fail(QAOA_ERR_UNSUPPORTED, "internal: sweep flag combination %d not instantiated", a.flags);
  }
  return QAOA_OK;
}

template <class S>
int launch_sweep_s(const qk::SweepArgs& a, int diag_dtype, uint64_t blocks, uint32_t sets, hipStream_t st) {
  switch (diag_dtype) {
    case QAOA_DIAG_I32: return launch_sweep_d<S, qk::DI32>(a, blocks, sets, st);
    case QAOA_DIAG_U16: return launch_sweep_d<S, qk::DU16>(a, blocks, sets, st);
    default: return launch_sweep_d<S, qk::DF64>(a, blocks, sets, st);
  }
}

// One sweep over `blocks` tiles of each of `sets` states.
int launch_sweep(const qk::SweepArgs& a, int state_dtype, int diag_dtype, bool wide, uint64_t blocks, uint32_t sets,
                 hipStream_t st) {
  if (state_dtype == QAOA_C128 && wide) return launch_sweep_s<qk::C128W>(a, diag_dtype, blocks, sets, st);
  if (state_dtype == QAOA_C128) return launch_sweep_s<qk::C128>(a, diag_dtype, blocks, sets, st);
  return launch_sweep_s<qk::C64>(a, diag_dtype, blocks, sets, st);
}

template <class S, class D, int EB>
void launch_tile_t(const qk::SweepArgs& a, uint32_t sets, hipStream_t st) {
  const uint32_t threads = 1u << (a.g.tb - EB);
  const size_t lds = tile_lds_bytes<S, D>(a.g, threads, true);
  hipLaunchKernelGGL((qk::qaoa_tile_kernel<S, D, EB>), dim3(sets), dim3(threads), lds, st, with_offsets<S>(a, EB));
}

template <class S, class D>
void launch_tile_d(const qk::SweepArgs& a, int eb, uint32_t sets, hipStream_t st) {
  switch (eb) {
    case 1: launch_tile_t<S, D, 1>(a, sets, st); break;
    case 2: launch_tile_t<S, D, 2>(a, sets, st); break;
    case 3: launch_tile_t<S, D, 3>(a, sets, st); break;
    default: launch_tile_t<S, D, 4>(a, sets, st); break;
  }
}

template <class S>
void launch_tile_s(const qk::SweepArgs& a, int diag_dtype, int eb, uint32_t sets, hipStream_t st) {
  switch (diag_dtype) {
    case QAOA_DIAG_I32: launch_tile_d<S, qk::DI32>(a, eb, sets, st); break;
    case QAOA_DIAG_U16: launch_tile_d<S, qk::DU16>(a, eb, sets, st); break;
    default: launch_tile_d<S, qk::DF64>(a, eb, sets, st); break;
  }
}

// Whole-state tiles: one workgroup per state, `sets` states.
void launch_tile(const qk::SweepArgs& a, int state_dtype, int diag_dtype, int eb, uint32_t sets, hipStream_t st) {
  if (state_dtype == QAOA_C128) launch_tile_s<qk::C128>(a, diag_dtype, eb, sets, st);
  else launch_tile_s<qk::C64>(a, diag_dtype, eb, sets, st);
}

// Consecutive gates of a sweep share one LDS pass when they form one of the
// kernel's group kinds: two gates on disjoint qubits (XG_PAIR), or two or
// three gates with one common qubit and distinct others (XG_STAR2, XG_STAR3,
// applied in list order); any other gate is a pass of its own (XG_ONE).  A
// group's tile bits are listed in the kind's local order (the common qubit
// first), STAR2 padded with the lowest tile bit it does not use.  Kernels with
// fewer than four register bits per thread (the smallest states) keep one pass
// per gate (ngroups = 0).
void set_xy_groups(qk::XyArgs& a, int tb, int eb) {
  a.ngroups = 0;
  if (eb != 4 || tb < 4 || a.ngates == 0) return;
  auto g0 = [&](int e) { return (int)a.gate[e][0]; };
  auto g1 = [&](int e) { return (int)a.gate[e][1]; };
  int e = 0;
  while (e < a.ngates) {
    const int gi = a.ngroups++;
    int bits[4] = {g0(e), g1(e), -1, -1};
    int kind = qk::XG_ONE, used = 1;
    if (e + 1 < a.ngates) {
      const int c = g0(e + 1), d = g1(e + 1);
      const bool sc = c == bits[0] || c == bits[1], sd = d == bits[0] || d == bits[1];
      if (!sc && !sd) {
        kind = qk::XG_PAIR; used = 2;
        bits[2] = c; bits[3] = d;
      } else if (sc != sd) {
        const int center = sc ? c : d, other = sc ? d : c;
        const int first = bits[0] == center ? bits[1] : bits[0];
        bits[0] = center; bits[1] = first; bits[2] = other;
        kind = qk::XG_STAR2; used = 2;
        if (e + 2 < a.ngates) {
          const int x = g0(e + 2), y = g1(e + 2);
          const int nx = x == center ? y : (y == center ? x : -1);
          if (nx >= 0 && nx != first && nx != other) {
            bits[3] = nx;
            kind = qk::XG_STAR3; used = 3;
          }
        }
        if (kind == qk::XG_STAR2)
          for (int b = 0; b < tb; ++b)
            if (b != bits[0] && b != bits[1] && b != bits[2]) { bits[3] = b; break; }
      }
    }
    a.grp_kind[gi] = (int8_t)kind;
    if (kind != qk::XG_ONE) {
      int srt[4] = {bits[0], bits[1], bits[2], bits[3]};
      std::sort(srt, srt + 4);
      for (int i = 0; i < 4; ++i) {
        a.grp_bits[gi][i] = (int8_t)bits[i];
        a.grp_sorted[gi][i] = (int8_t)srt[i];
      }
    }
    e += used;
  }
}

static_assert(sizeof(qk::XyArgs) <= 4096, "XY launch arguments exceed the kernarg limit");

// XY mixer launches: tile of 2^tb complex128 LDS entries + phase tables + flags.
template <class S, class D, int EB>
void launch_xy_t(const qk::XyArgs& a, uint64_t blocks, uint32_t sets, hipStream_t st) {
  const uint32_t threads = 1u << (a.s.g.tb - EB);
  const size_t tile = ((size_t)1 << a.s.g.tb) * sizeof(double2);
  const size_t lds = std::max<size_t>(tile + qk::kTabEntries * sizeof(double2) + 16 * sizeof(uint32_t),
                                      std::max<size_t>(16, 2 * threads) * sizeof(double));
  qk::XyArgs b = a;
  qk::fill_reg_offsets<16>(b.s.g, EB);
  hipLaunchKernelGGL((qk::qaoa_xy_kernel<S, D, EB>), dim3((uint32_t)blocks, sets), dim3(threads), lds, st, b);
}

template <class S, class D>
void launch_xy_d(const qk::XyArgs& a, int eb, uint64_t blocks, uint32_t sets, hipStream_t st) {
  switch (eb) {
    case 1: launch_xy_t<S, D, 1>(a, blocks, sets, st); break;
    case 2: launch_xy_t<S, D, 2>(a, blocks, sets, st); break;
    case 3: launch_xy_t<S, D, 3>(a, blocks, sets, st); break;
    default: launch_xy_t<S, D, 4>(a, blocks, sets, st); break;
  }
}

void launch_xy(const qk::XyArgs& a, int sdt, int ddt, int eb, uint64_t blocks, uint32_t sets, hipStream_t st) {
  if (sdt == QAOA_C128) {
    if (ddt == QAOA_DIAG_I32) launch_xy_d<qk::C128, qk::DI32>(a, eb, blocks, sets, st);
    else if (ddt == QAOA_DIAG_U16) launch_xy_d<qk::C128, qk::DU16>(a, eb, blocks, sets, st);
    else launch_xy_d<qk::C128, qk::DF64>(a, eb, blocks, sets, st);
  } else {
    if (ddt == QAOA_DIAG_I32) launch_xy_d<qk::C64, qk::DI32>(a, eb, blocks, sets, st);
    else if (ddt == QAOA_DIAG_U16) launch_xy_d<qk::C64, qk::DU16>(a, eb, blocks, sets, st);
    else launch_xy_d<qk::C64, qk::DF64>(a, eb, blocks, sets, st);
  }
}

template <class S, class D, bool FIRST, bool PHASE, bool FUSE, int PLO = 0, int PHI = 0>
void launch_adj_ff(const qk::AdjArgs& a, uint64_t blocks, hipStream_t st) {
  const uint32_t threads = 1u << (a.g.tb - kEBAdj);
  const size_t tile = ((size_t)1 << a.g.tb) * S::kLdsBytes;
  const size_t lds = std::max<size_t>(tile + D::kTabLds * sizeof(double2) + 16 * sizeof(uint32_t),
                                      std::max<size_t>(16, 2 * threads) * sizeof(double));
  hipLaunchKernelGGL((qk::qaoa_adjoint_kernel<S, D, kEBAdj, FIRST, PHASE, FUSE, PLO, PHI>), dim3((uint32_t)blocks),
                     dim3(threads), lds, st, with_offsets<S>(a, kEBAdj));
}

// Reverse sweeps specialise a plan's short chunk (register bits [1, 3) or [2, 3)).
template <class S, class D, bool FIRST, bool PHASE, bool FUSE>
void launch_adj_f(const qk::AdjArgs& a, uint64_t blocks, hipStream_t st) {
  const qk::Chunk c = a.g.part >= 0 ? a.g.chunk[a.g.part] : qk::Chunk{0, 0, 0, 0};
  if (c.jhi == kEBAdj && c.jlo == 1) launch_adj_ff<S, D, FIRST, PHASE, FUSE, 1, kEBAdj>(a, blocks, st);
  else if (c.jhi == kEBAdj && c.jlo == 2) launch_adj_ff<S, D, FIRST, PHASE, FUSE, 2, kEBAdj>(a, blocks, st);
  else launch_adj_ff<S, D, FIRST, PHASE, FUSE>(a, blocks, st);
}

template <class S, class D>
int launch_adj_d(const qk::AdjArgs& a, int flags, uint64_t blocks, hipStream_t st) {
  switch (flags) {
    case qk::A_FIRST: launch_adj_f<S, D, true, false, false>(a, blocks, st); break;
    case qk::A_PHASE: launch_adj_f<S, D, false, true, false>(a, blocks, st); break;
    case qk::A_FUSE: launch_adj_f<S, D, false, false, true>(a, blocks, st); break;
    case 0: launch_adj_f<S, D, false, false, false>(a, blocks, st); break;
    default: return fail(QAOA_ERR_UNSUPPORTED, "internal: adjoint flag combination %d not instantiated", flags);
  }
  return QAOA_OK;
}

template <class S, class D, int EB>
void launch_adj_tile_t(const qk::AdjArgs& a, hipStream_t st) {
  const uint32_t threads = 1u << (a.g.tb - EB);
  const size_t lds = ((size_t)1 << a.g.tb) * S::kLdsBytes + D::kTabLds * sizeof(double2) + 16 * sizeof(uint32_t) +
                     std::max<size_t>(16, 2 * threads) * sizeof(double);
  hipLaunchKernelGGL((qk::qaoa_adjoint_tile_kernel<S, D, EB>), dim3(1), dim3(threads), lds, st, with_offsets<S>(a, EB));
}

template <class S, class D>
void launch_adj_tile_d(const qk::AdjArgs& a, int eb, hipStream_t st) {
  switch (eb) {
    case 1: launch_adj_tile_t<S, D, 1>(a, st); break;
    case 2: launch_adj_tile_t<S, D, 2>(a, st); break;
    default: launch_adj_tile_t<S, D, 3>(a, st); break;
  }
}

// Reverse sweep (tile == false) or whole-state reverse pass (tile == true).
template <class S>
int launch_adj_s(const qk::AdjArgs& a, int ddt, bool tile, int eb, int flags, uint64_t blocks, hipStream_t st) {
  switch (ddt) {
    case QAOA_DIAG_I32:
      if (tile) { launch_adj_tile_d<S, qk::DI32>(a, eb, st); return QAOA_OK; }
      return launch_adj_d<S, qk::DI32>(a, flags, blocks, st);
    case QAOA_DIAG_U16:
      if (tile) { launch_adj_tile_d<S, qk::DU16>(a, eb, st); return QAOA_OK; }
      return launch_adj_d<S, qk::DU16>(a, flags, blocks, st);
    default:
      if (tile) { launch_adj_tile_d<S, qk::DF64>(a, eb, st); return QAOA_OK; }
      return launch_adj_d<S, qk::DF64>(a, flags, blocks, st);
  }
}

// Reverse sweep with qk::A_* flags (tile == false) or whole-state reverse pass (tile == true).
int launch_adj(const qk::AdjArgs& a, int sdt, int ddt, bool tile, int eb, int flags, uint64_t blocks, hipStream_t st) {
  if (sdt == QAOA_C128) return launch_adj_s<qk::C128>(a, ddt, tile, eb, flags, blocks, st);
  return launch_adj_s<qk::C64>(a, ddt, tile, eb, flags, blocks, st);
}

template <class S, class D>
void launch_expect_t(const void* psi, const void* diag, double off, uint64_t N, double* partials, uint32_t blocks,
                     hipStream_t st) {
  hipLaunchKernelGGL((qk::expectation_kernel<S, D>), dim3(blocks), dim3(256), 0, st, psi, diag, off, N, partials);
}

void launch_expect(int sdt, int ddt, const void* psi, const void* diag, double off, uint64_t N, double* partials,
                   uint32_t blocks, hipStream_t st) {
  if (sdt == QAOA_C128) {
    if (ddt == QAOA_DIAG_I32) launch_expect_t<qk::C128, qk::DI32>(psi, diag, off, N, partials, blocks, st);
    else if (ddt == QAOA_DIAG_U16) launch_expect_t<qk::C128, qk::DU16>(psi, diag, off, N, partials, blocks, st);
    else launch_expect_t<qk::C128, qk::DF64>(psi, diag, off, N, partials, blocks, st);
  } else {
    if (ddt == QAOA_DIAG_I32) launch_expect_t<qk::C64, qk::DI32>(psi, diag, off, N, partials, blocks, st);
    else if (ddt == QAOA_DIAG_U16) launch_expect_t<qk::C64, qk::DU16>(psi, diag, off, N, partials, blocks, st);
    else launch_expect_t<qk::C64, qk::DF64>(psi, diag, off, N, partials, blocks, st);
  }
}

uint32_t expect_blocks(uint64_t N) {
  const uint64_t b = (N + 256 * 16 - 1) / (256 * 16);
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kExpectBlocks, b));
}

template <typename T, int EB>
void launch_fwht_t(const qk::FwhtArgs& a, uint64_t blocks, hipStream_t st) {
  const uint32_t threads = 1u << (a.g.tb - EB);
  const size_t lds = ((size_t)1 << a.g.tb) * sizeof(T);
  hipLaunchKernelGGL((qk::fwht_sweep_kernel<T, EB>), dim3((uint32_t)blocks), dim3(threads), lds, st, a);
}

template <typename T>
void launch_fwht(const qk::FwhtArgs& a, int eb, uint64_t blocks, hipStream_t st) {
  switch (eb) {
    case 1: launch_fwht_t<T, 1>(a, blocks, st); break;
    case 2: launch_fwht_t<T, 2>(a, blocks, st); break;
    case 3: launch_fwht_t<T, 3>(a, blocks, st); break;
    default: launch_fwht_t<T, 4>(a, blocks, st); break;
  }
}

uint32_t grid_for(uint64_t N, uint32_t threads, uint32_t cap) {
  const uint64_t b = (N + threads - 1) / threads;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cap, b));
}

// ---------------------------------------------------------------------------
// precompute
// ---------------------------------------------------------------------------

// Unnormalised Walsh-Hadamard transform in place over all n bits.
template <typename T>
int fwht_all(int n, T* data, hipStream_t st) {
  const Plan pl = make_plan(n, sizeof(T));
  for (const auto& g : pl.sweeps) {
    qk::FwhtArgs a{};
    a.data = data;
    a.g = g;
    launch_fwht<T>(a, pl.eb, plan_blocks(n, g), st);
    LAUNCH_CHECK("fwht_sweep_kernel");
  }
  return QAOA_OK;
}

template <typename T>
int zero_and_scatter(int n, T* data, const std::vector<uint64_t>& masks, const std::vector<T>& vals, hipStream_t st) {
  const uint64_t N = (uint64_t)1 << n;
  hipLaunchKernelGGL((qk::zero_kernel<T>), dim3(grid_for(N, 256, 8192)), dim3(256), 0, st, data, N);
  LAUNCH_CHECK("zero_kernel");
  for (size_t s = 0; s < masks.size(); s += qk::kScatterChunk) {
    qk::ScatterArgs<T> a{};
    a.data = data;
    a.count = (int)std::min<size_t>(qk::kScatterChunk, masks.size() - s);
    for (int i = 0; i < a.count; ++i) { a.mask[i] = masks[s + i]; a.val[i] = vals[s + i]; }
    hipLaunchKernelGGL((qk::scatter_kernel<T>), dim3((a.count + 255) / 256), dim3(256), 0, st, a);
    LAUNCH_CHECK("scatter_kernel");
  }
  return QAOA_OK;
}

// (min, max, OR of low bits) of an int32 vector, read back to the host (syncs).
int int_stats(int n, const int32_t* data, int32_t lowmask, void* work, int64_t out[3], hipStream_t st) {
  const uint64_t N = (uint64_t)1 << n;
  const uint32_t blocks = grid_for(N, 256 * 16, kStatBlocks);
  int64_t* partials = reinterpret_cast<int64_t*>(work);
  int64_t* res = partials + 3 * kStatBlocks;
  hipLaunchKernelGGL(qk::int_stats_kernel, dim3(blocks), dim3(256), 0, st, data, N, lowmask, partials);
  LAUNCH_CHECK("int_stats_kernel");
  hipLaunchKernelGGL(qk::int_stats_finalize, dim3(1), dim3(64), 0, st, partials, (int)blocks, res);
  LAUNCH_CHECK("int_stats_finalize");
  HIP_TRY(hipMemcpyAsync(out, res, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return QAOA_OK;
}

constexpr size_t kStatWork = (3 * kStatBlocks + 4) * sizeof(int64_t);

// Evolve workspace layout: [per-state (E, norm) partials of the last sweep]
// [parameter rows: 3 doubles each][phase tables: kTabRow double2 per row].
// A single evaluation with host angles uses kPrepRows rows (one chunk of
// layers at a time, plus the next layer); a batch with device angles uses
// batch * p rows.
constexpr uint64_t kReduceChunks = 1024;  // stage-1 chunks of the two-stage reduction

struct EvolveWork {
  size_t partials_stride;  // doubles per state
  size_t partials_bytes, pset_bytes, tab_bytes, tmp_bytes, total;
};
EvolveWork evolve_work(int n, size_t states, size_t rows, int state_dtype) {
  EvolveWork b{};
  // most workgroups of any sweep of either plan (the last sweep depends on p,
  // the plan on the wide-tile knob), so the size does not depend on the knobs
  uint64_t last = 0;
  for (bool wide : {false, true})
    for (const auto& g : state_plan(n, state_dtype, wide).sweeps) last = std::max(last, plan_blocks(n, g));
  b.partials_stride = 2 * std::max<uint64_t>(last, kExpectBlocks);
  b.partials_bytes = sizeof(double) * b.partials_stride * states;
  b.pset_bytes = ((qk::kParamRow * sizeof(double) * rows + 255) / 256) * 256;
  b.tab_bytes = rows * qk::kTabRow * sizeof(double2);
  b.tmp_bytes = sizeof(double) * 2 * kReduceChunks * states;
  b.total = b.partials_bytes + b.pset_bytes + b.tab_bytes + b.tmp_bytes;
  return b;
}

// (E, norm) of `sets` states from `count` partial pairs each (stride doubles
// apart) into out[2 s + {0,1}]: two fixed-order stages through tmp.
int enqueue_reduce(const double* partials, uint64_t count, uint64_t stride, uint32_t sets, double* tmp, double* out,
                   hipStream_t st) {
  if (count <= 256) {
    hipLaunchKernelGGL(qk::finalize_batch_kernel, dim3(sets), dim3(256), 0, st, partials, count, stride, out);
    LAUNCH_CHECK("finalize_batch_kernel");
    return QAOA_OK;
  }
  const uint64_t chunks = std::min<uint64_t>(kReduceChunks, (count + 255) / 256);
  const uint64_t per = (count + chunks - 1) / chunks;
  const uint64_t nchunks = (count + per - 1) / per;
  hipLaunchKernelGGL(qk::reduce_chunks_kernel, dim3((uint32_t)nchunks, sets), dim3(256), 0, st, partials, count,
                     stride, per, tmp, (uint64_t)(2 * kReduceChunks));
  LAUNCH_CHECK("reduce_chunks_kernel");
  hipLaunchKernelGGL(qk::finalize_batch_kernel, dim3(sets), dim3(256), 0, st, (const double*)tmp, nchunks,
                     (uint64_t)(2 * kReduceChunks), out);
  LAUNCH_CHECK("finalize_batch_kernel");
  return QAOA_OK;
}
size_t evolve_work_bytes(int n, int state_dtype) { return evolve_work(n, 1, qk::kPrepRows, state_dtype).total; }
size_t partials_bytes(int n, int state_dtype) { return evolve_work(n, 1, 0, state_dtype).partials_bytes; }

// Gradient workspace: [forward evolve workspace][p parameter rows][p table rows]
// [reverse partials: p layers x sweeps x blocks x 2 doubles].
struct GradWork {
  size_t fwd, pset_off, tab_off, rev_off, layer_stride /* doubles */, total;
};
GradWork grad_work(int n, int p, int state_dtype) {
  GradWork g{};
  const Plan pl = adjoint_plan(n, state_elem_bytes(state_dtype));
  const uint64_t blocks = pl.single ? 1 : plan_blocks(n, pl.sweeps[0]);
  g.fwd = evolve_work_bytes(n, state_dtype);
  g.pset_off = g.fwd;
  g.tab_off = g.pset_off + ((qk::kParamRow * sizeof(double) * (size_t)p + 255) / 256) * 256;
  g.rev_off = g.tab_off + (size_t)p * qk::kTabRow * sizeof(double2);
  g.layer_stride = 2 * pl.sweeps.size() * blocks;
  g.total = g.rev_off + sizeof(double) * g.layer_stride * (size_t)p;
  return g;
}

double table_base(int diag_dtype, double diag_offset) {
  return (diag_dtype == QAOA_DIAG_I32 ? qk::DI32::kTableBase : qk::DU16::kTableBase) + diag_offset;
}

}  // namespace

// Used by the request loop (server.hip) to report errors through qaoa_last_error().
__attribute__((visibility("hidden"))) int qaoa_internal_set_error(int code, const char* msg) {
  g_err = msg;
  return code;
}

extern "C" {

const char* qaoa_version(void) { return "0.3.0"; }

int qaoa_set_tuning(int knob, int value) {
  if (value != 0 && value != 1) return fail(QAOA_ERR_INVALID, "tuning value must be 0 or 1, got %d", value);
  switch (knob) {
    case QAOA_TUNE_WIDE_TILES: g_wide_tiles.store(value); return QAOA_OK;
    case QAOA_TUNE_FUSE_LAYERS: g_fuse_layers.store(value); return QAOA_OK;
    default: return fail(QAOA_ERR_INVALID, "unknown tuning knob %d", knob);
  }
}

int qaoa_get_tuning(int knob, int* value) {
  if (!value) return fail(QAOA_ERR_INVALID, "value is NULL");
  switch (knob) {
    case QAOA_TUNE_WIDE_TILES: *value = g_wide_tiles.load(); return QAOA_OK;
    case QAOA_TUNE_FUSE_LAYERS: *value = g_fuse_layers.load(); return QAOA_OK;
    default: return fail(QAOA_ERR_INVALID, "unknown tuning knob %d", knob);
  }
}

const char* qaoa_last_error(void) { return g_err.c_str(); }

int qaoa_workspace_bytes(int op, int n, int state_dtype, int diag_dtype, size_t* bytes) {
  if (!bytes) return fail(QAOA_ERR_INVALID, "bytes is NULL");
  if (n < 1 || n > QAOA_MAX_QUBITS) return fail(QAOA_ERR_INVALID, "n=%d out of range [1, %d]", n, QAOA_MAX_QUBITS);
  const uint64_t N = (uint64_t)1 << n;
  switch (op) {
    case QAOA_OP_PRECOMPUTE:
      if (!valid_diag_dtype(diag_dtype)) return fail(QAOA_ERR_INVALID, "bad diag dtype %d", diag_dtype);
      *bytes = diag_dtype == QAOA_DIAG_F64 ? 0 : diag_dtype == QAOA_DIAG_I32 ? kStatWork : 4 * N + kStatWork;
      return QAOA_OK;
    case QAOA_OP_EVOLVE:
    case QAOA_OP_EXPECTATION:
    case QAOA_OP_GRAD: {
      if (!valid_state_dtype(state_dtype)) return fail(QAOA_ERR_INVALID, "bad state dtype %d", state_dtype);
      *bytes = evolve_work_bytes(n, state_dtype);
      return QAOA_OK;
    }
    default:
      return fail(QAOA_ERR_INVALID, "bad op %d", op);
  }
}

int qaoa_precompute_diag(int n, int64_t num_terms, const double* w, const int64_t* term_ptr,
                         const int32_t* term_idx, int diag_dtype, void* d_diag, size_t diag_bytes,
                         double* out_offset, void* d_work, size_t work_bytes, void* stream) {
  // ---- validation (nothing enqueued before this block ends) ----
  if (n < 1 || n > QAOA_MAX_QUBITS) return fail(QAOA_ERR_INVALID, "n=%d out of range [1, %d]", n, QAOA_MAX_QUBITS);
  if (num_terms < 0) return fail(QAOA_ERR_INVALID, "num_terms < 0");
  if (num_terms > 0 && (!w || !term_ptr)) return fail(QAOA_ERR_INVALID, "w/term_ptr is NULL");
  if (!valid_diag_dtype(diag_dtype)) return fail(QAOA_ERR_INVALID, "bad diag dtype %d", diag_dtype);
  if (!d_diag) return fail(QAOA_ERR_INVALID, "d_diag is NULL");
  if (!out_offset) return fail(QAOA_ERR_INVALID, "out_offset is NULL");
  const uint64_t N = (uint64_t)1 << n;
  if (diag_bytes < N * diag_elem_bytes(diag_dtype))
    return fail(QAOA_ERR_NOMEM, "diag buffer has %zu bytes, needs %llu", diag_bytes,
                (unsigned long long)(N * diag_elem_bytes(diag_dtype)));
  if (work_bytes > 0 && !d_work) return fail(QAOA_ERR_INVALID, "d_work is NULL but work_bytes > 0");
  if (num_terms > 0 && term_ptr[0] != 0) return fail(QAOA_ERR_INVALID, "term_ptr[0] != 0");
  for (int64_t k = 0; k < num_terms; ++k) {
    if (term_ptr[k + 1] < term_ptr[k]) return fail(QAOA_ERR_INVALID, "term_ptr decreases at %lld", (long long)k);
    if (!std::isfinite(w[k])) return fail(QAOA_ERR_INVALID, "weight %lld is not finite", (long long)k);
  }
  const int64_t nnz = num_terms > 0 ? term_ptr[num_terms] : 0;
  if (nnz > 0 && !term_idx) return fail(QAOA_ERR_INVALID, "term_idx is NULL");
  for (int64_t j = 0; j < nnz; ++j)
    if (term_idx[j] < 0 || term_idx[j] >= n)
      return fail(QAOA_ERR_INVALID, "term index %d out of range for n=%d", term_idx[j], n);

  // ---- encode: mask = XOR of 1 << i (s_i^2 = 1), merge equal masks ----
  std::unordered_map<uint64_t, double> acc;
  std::vector<uint64_t> order;
  for (int64_t k = 0; k < num_terms; ++k) {
    uint64_t m = 0;
    for (int64_t j = term_ptr[k]; j < term_ptr[k + 1]; ++j) m ^= (uint64_t)1 << term_idx[j];
    auto it = acc.find(m);
    if (it == acc.end()) { acc.emplace(m, w[k]); order.push_back(m); }
    else it->second += w[k];
  }
  double cst = 0.0, sabs = 0.0;
  for (uint64_t m : order) {
    if (m == 0) cst = acc[m];
    else sabs += std::fabs(acc[m]);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  if (diag_dtype == QAOA_DIAG_F64) {
    std::vector<uint64_t> masks;
    std::vector<double> vals;
    for (uint64_t m : order) { masks.push_back(m); vals.push_back(acc[m]); }
    int rc = zero_and_scatter<double>(n, reinterpret_cast<double*>(d_diag), masks, vals, st);
    if (rc) return rc;
    rc = fwht_all<double>(n, reinterpret_cast<double*>(d_diag), st);
    if (rc) return rc;
    *out_offset = 0.0;
    return QAOA_OK;
  }

  // integer dtypes: smallest k with every weight * 2^k integral
  int k = -1;
  for (int kk = 0; kk <= 20 && k < 0; ++kk) {
    bool ok = true;
    const double sc = std::ldexp(1.0, kk);
    for (uint64_t m : order) {
      const double v = acc[m] * sc;
      if (v != std::nearbyint(v)) { ok = false; break; }
    }
    if (ok) k = kk;
  }
  if (k < 0) return fail(QAOA_ERR_RANGE, "weights are not dyadic rationals: cost values are not integers");
  const double bound = std::ldexp(std::fabs(cst) + sabs, k);
  if (bound >= 2147483647.0) return fail(QAOA_ERR_RANGE, "|c| bound %.17g exceeds the int32 range", bound);

  if (diag_dtype == QAOA_DIAG_U16 && k == 0 && 2.0 * sabs < 65536.0) {
    // c - offset lies in [0, 2 sum|w|] < 2^16, so the transform in arithmetic
    // mod 2^16 is exact.
    const double offset = cst - sabs;
    std::vector<uint64_t> masks;
    std::vector<uint16_t> vals;
    for (uint64_t m : order) {
      const double v = (m == 0) ? cst - offset : acc[m];
      masks.push_back(m);
      vals.push_back((uint16_t)((int64_t)v & 0xFFFF));
    }
    if (acc.find(0) == acc.end()) { masks.push_back(0); vals.push_back((uint16_t)((int64_t)(-offset) & 0xFFFF)); }
    int rc = zero_and_scatter<uint16_t>(n, reinterpret_cast<uint16_t*>(d_diag), masks, vals, st);
    if (rc) return rc;
    rc = fwht_all<uint16_t>(n, reinterpret_cast<uint16_t*>(d_diag), st);
    if (rc) return rc;
    *out_offset = offset;
    return QAOA_OK;
  }

  // scaled int32 transform, in d_diag (I32) or in the workspace (U16)
  int32_t* buf = nullptr;
  void* stat_work = nullptr;
  if (diag_dtype == QAOA_DIAG_I32) {
    buf = reinterpret_cast<int32_t*>(d_diag);
    if (k > 0) {
      if (work_bytes < kStatWork) return fail(QAOA_ERR_NOMEM, "workspace too small: need %zu bytes", kStatWork);
      stat_work = d_work;
    }
  } else {
    if (work_bytes < 4 * N + kStatWork)
      return fail(QAOA_ERR_NOMEM, "workspace too small for the U16 path: need %llu bytes",
                  (unsigned long long)(4 * N + kStatWork));
    buf = reinterpret_cast<int32_t*>(d_work);
    stat_work = reinterpret_cast<char*>(d_work) + 4 * N;
  }
  {
    std::vector<uint64_t> masks;
    std::vector<int32_t> vals;
    const double sc = std::ldexp(1.0, k);
    for (uint64_t m : order) { masks.push_back(m); vals.push_back((int32_t)(acc[m] * sc)); }
    int rc = zero_and_scatter<int32_t>(n, buf, masks, vals, st);
    if (rc) return rc;
    rc = fwht_all<int32_t>(n, buf, st);
    if (rc) return rc;
  }
  if (diag_dtype == QAOA_DIAG_I32 && k == 0) { *out_offset = 0.0; return QAOA_OK; }

  int64_t stats[3];
  int rc = int_stats(n, buf, (int32_t)((1u << k) - 1u), stat_work, stats, st);
  if (rc) return rc;
  if (stats[2] != 0) return fail(QAOA_ERR_RANGE, "cost values are not all integers");
  const int64_t cmin = stats[0] >> k, cmax = stats[1] >> k;
  const uint64_t grid = grid_for(N, 256, 8192);
  if (diag_dtype == QAOA_DIAG_I32) {
    hipLaunchKernelGGL((qk::narrow_kernel<int32_t>), dim3((uint32_t)grid), dim3(256), 0, st, buf,
                       reinterpret_cast<int32_t*>(d_diag), N, k, (int64_t)0);
    LAUNCH_CHECK("narrow_kernel");
    *out_offset = 0.0;
    return QAOA_OK;
  }
  if (cmax - cmin >= 65536) return fail(QAOA_ERR_RANGE, "cost range [%lld, %lld] does not fit uint16",
                                        (long long)cmin, (long long)cmax);
  hipLaunchKernelGGL((qk::narrow_kernel<uint16_t>), dim3((uint32_t)grid), dim3(256), 0, st, buf,
                     reinterpret_cast<uint16_t*>(d_diag), N, k, cmin);
  LAUNCH_CHECK("narrow_kernel");
  *out_offset = (double)cmin;
  return QAOA_OK;
}

static int validate_common(int n, const void* d_diag, int diag_dtype, double diag_offset, size_t diag_bytes,
                           const void* d_state, int state_dtype, size_t state_bytes) {
  if (n < 1 || n > QAOA_MAX_QUBITS) return fail(QAOA_ERR_INVALID, "n=%d out of range [1, %d]", n, QAOA_MAX_QUBITS);
  if (!valid_state_dtype(state_dtype)) return fail(QAOA_ERR_INVALID, "bad state dtype %d", state_dtype);
  if (!valid_diag_dtype(diag_dtype)) return fail(QAOA_ERR_INVALID, "bad diag dtype %d", diag_dtype);
  if (!d_state) return fail(QAOA_ERR_INVALID, "d_state is NULL");
  if (!d_diag) return fail(QAOA_ERR_INVALID, "d_diag is NULL");
  if (!std::isfinite(diag_offset)) return fail(QAOA_ERR_INVALID, "diag_offset is not finite");
  if (diag_dtype != QAOA_DIAG_F64 && diag_offset != std::nearbyint(diag_offset))
    return fail(QAOA_ERR_INVALID, "diag_offset must be integral for integer cost vectors");
  const uint64_t N = (uint64_t)1 << n;
  if (state_bytes < N * state_elem_bytes(state_dtype))
    return fail(QAOA_ERR_NOMEM, "state buffer has %zu bytes, needs %llu", state_bytes,
                (unsigned long long)(N * state_elem_bytes(state_dtype)));
  if (diag_bytes < N * diag_elem_bytes(diag_dtype))
    return fail(QAOA_ERR_NOMEM, "diag buffer has %zu bytes, needs %llu", diag_bytes,
                (unsigned long long)(N * diag_elem_bytes(diag_dtype)));
  return QAOA_OK;
}

static int validate_angles(int p, const double* gamma, const double* beta) {
  if (p < 0) return fail(QAOA_ERR_INVALID, "p < 0");
  if (p > 0 && (!gamma || !beta)) return fail(QAOA_ERR_INVALID, "gamma/beta is NULL");
  for (int l = 0; l < p; ++l)
    if (!std::isfinite(gamma[l]) || !std::isfinite(beta[l]))
      return fail(QAOA_ERR_INVALID, "angle of layer %d is not finite", l);
  return QAOA_OK;
}

static int enqueue_expectation(int n, const void* d_state, int sdt, const void* d_diag, int ddt, double off,
                               double* d_out, void* d_work, hipStream_t st) {
  const uint64_t N = (uint64_t)1 << n;
  const uint32_t blocks = expect_blocks(N);
  double* partials = reinterpret_cast<double*>(d_work);
  launch_expect(sdt, ddt, d_state, d_diag, off, N, partials, blocks, st);
  LAUNCH_CHECK("expectation_kernel");
  hipLaunchKernelGGL(qk::finalize_kernel, dim3(1), dim3(256), 0, st, (const double*)partials, (uint64_t)blocks, d_out);
  LAUNCH_CHECK("finalize_kernel");
  return QAOA_OK;
}

// Enqueue p layers for `batch` states (stride 2^n elements) starting at d_states.
// Angles come from the host arrays (batch == 1; prepared on the device in
// chunks of kMaxLayersPerLaunch layers) or from device arrays [batch][p]
// (prepared once).  Both use layer_prep_kernel, so a state's result does not
// depend on which entry point or grouping produced it.
static int enqueue_evolve(int n, int p, int batch, const double* h_gamma, const double* h_beta, const double* d_gamma,
                          const double* d_beta, const void* d_diag, int diag_dtype, double diag_offset,
                          void* d_states, int state_dtype, int init, double* d_out, int G, void* d_work,
                          Tuning tn, hipStream_t st) {
  const uint64_t N = (uint64_t)1 << n;
  const size_t S = state_elem_bytes(state_dtype);
  const bool host_angles = (h_gamma != nullptr);
  const size_t rows = host_angles ? (size_t)qk::kPrepRows : (size_t)batch * (size_t)p;
  const EvolveWork ew = evolve_work(n, (size_t)batch, rows, state_dtype);
  char* wk = reinterpret_cast<char*>(d_work);
  double* partials = reinterpret_cast<double*>(wk);
  double* pset = reinterpret_cast<double*>(wk + ew.partials_bytes);
  double2* tab = reinterpret_cast<double2*>(wk + ew.partials_bytes + ew.pset_bytes);
  const bool use_tab = diag_dtype != QAOA_DIAG_F64;

  qk::PrepArgs pa{};
  pa.pset = pset;
  pa.tab = use_tab ? tab : nullptr;
  pa.base = use_tab ? table_base(diag_dtype, diag_offset) : 0.0;
  pa.off = diag_offset;
  auto prep = [&](int l0, int nl) -> int {  // host angles, layers [l0, l0 + nl), nl <= kPrepRows
    pa.rows = nl;
    for (int i = 0; i < nl; ++i) { pa.gamma[i] = h_gamma[l0 + i]; pa.beta[i] = h_beta[l0 + i]; }
    hipLaunchKernelGGL(qk::layer_prep_kernel, dim3(nl), dim3(256), 0, st, pa);
    LAUNCH_CHECK("layer_prep_kernel");
    return QAOA_OK;
  };
  if (!host_angles) {
    pa.gamma_d = d_gamma;
    pa.beta_d = d_beta;
    pa.rows = batch * p;
    hipLaunchKernelGGL(qk::layer_prep_kernel, dim3((uint32_t)(batch * p)), dim3(256), 0, st, pa);
    LAUNCH_CHECK("layer_prep_kernel");
  }

  const Plan pl = state_plan(n, state_dtype, tn.wide);
  qk::SweepArgs a{};
  a.diag = d_diag;
  a.diag_offset = diag_offset;
  a.amp0 = std::pow(2.0, -0.5 * n);
  a.ptab = tab;
  a.pset = pset;
  a.p_total = host_angles ? qk::kPrepRows : p;
  a.set_stride_bytes = N * S;
  a.partials_stride = ew.partials_stride;
  const std::vector<SweepStep> sched =
      pl.single ? std::vector<SweepStep>()
                : sweep_schedule((int)pl.sweeps.size(), p, init != 0, d_out != nullptr, tn.fuse);
  int rc = QAOA_OK;
  for (int s0 = 0; s0 < batch; s0 += G) {
    const uint32_t sets = (uint32_t)std::min(G, batch - s0);
    a.set0 = host_angles ? 0 : s0;
    a.psi = reinterpret_cast<char*>(d_states) + (size_t)s0 * N * S;
    a.partials = partials + (size_t)s0 * ew.partials_stride;
    uint64_t last_blocks = 1;
    size_t next = 0;  // next schedule step
    for (int l0 = 0; l0 < p; l0 += qk::kMaxLayersPerLaunch) {
      const int nl = std::min(qk::kMaxLayersPerLaunch, p - l0);
      if (host_angles) {
        rc = prep(l0, std::min(nl + 1, p - l0));  // + the next layer, read by a fused sweep
        if (rc) return rc;
      }
      if (pl.single) {
        a.g = pl.sweeps[0];
        a.layer0 = host_angles ? 0 : l0;
        a.nlayers = nl;
        a.flags = qk::F_PHASE | ((l0 == 0 && init) ? qk::F_INIT : 0) | ((l0 + nl == p && d_out) ? qk::F_EXPV : 0);
        launch_tile(a, state_dtype, diag_dtype, pl.eb, sets, st);
        LAUNCH_CHECK("qaoa_tile_kernel");
        continue;
      }
      a.nlayers = 1;
      for (; next < sched.size() && sched[next].layer < l0 + nl; ++next) {
        const SweepStep& stp = sched[next];
        a.g = pl.sweeps[stp.sweep];
        a.layer0 = host_angles ? stp.layer - l0 : stp.layer;
        a.flags = stp.flags;
        last_blocks = plan_blocks(n, a.g);
        rc = launch_sweep(a, state_dtype, diag_dtype, pl.wide, last_blocks, sets, st);
        if (rc) return rc;
        LAUNCH_CHECK("qaoa_sweep_kernel");
      }
    }
    if (d_out) {
      double* tmp = reinterpret_cast<double*>(wk + ew.partials_bytes + ew.pset_bytes + ew.tab_bytes) +
                    2 * kReduceChunks * (size_t)s0;
      rc = enqueue_reduce(a.partials, last_blocks, ew.partials_stride, sets, tmp, d_out + 2 * (size_t)s0, st);
      if (rc) return rc;
    }
  }
  return QAOA_OK;
}

int qaoa_evolve(int n, int p, const double* gamma, const double* beta, const void* d_diag, int diag_dtype,
                double diag_offset, size_t diag_bytes, void* d_state, int state_dtype, size_t state_bytes, int init,
                double* d_out, void* d_work, size_t work_bytes, void* stream) {
  int rc = validate_common(n, d_diag, diag_dtype, diag_offset, diag_bytes, d_state, state_dtype, state_bytes);
  if (rc) return rc;
  rc = validate_angles(p, gamma, beta);
  if (rc) return rc;
  if (init != 0 && init != 1) return fail(QAOA_ERR_INVALID, "init must be 0 or 1");
  if (p > 0 || d_out) {
    const size_t need = evolve_work_bytes(n, state_dtype);
    if (!d_work || work_bytes < need) return fail(QAOA_ERR_NOMEM, "workspace too small: need %zu bytes", need);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint64_t N = (uint64_t)1 << n;
  const double amp0 = std::pow(2.0, -0.5 * n);

  if (p == 0) {
    if (init) {
      if (state_dtype == QAOA_C128)
        hipLaunchKernelGGL((qk::fill_state_kernel<qk::C128>), dim3(grid_for(N, 256, 8192)), dim3(256), 0, st, d_state, N, amp0);
      else
        hipLaunchKernelGGL((qk::fill_state_kernel<qk::C64>), dim3(grid_for(N, 256, 8192)), dim3(256), 0, st, d_state, N, amp0);
      LAUNCH_CHECK("fill_state_kernel");
    }
    if (d_out) return enqueue_expectation(n, d_state, state_dtype, d_diag, diag_dtype, diag_offset, d_out, d_work, st);
    return QAOA_OK;
  }

  return enqueue_evolve(n, p, 1, gamma, beta, nullptr, nullptr, d_diag, diag_dtype, diag_offset, d_state, state_dtype,
                        init, d_out, 1, d_work, tuning_now(), st);
}

}  // extern "C"

// Scratch of qaoa_evolve_noalloc: the evolve workspace (per-workgroup (E, norm)
// partials, parameter rows, phase tables) in a static device array, so that
// callers that cannot allocate need no workspace.  Each GPU holds its own copy
// for the life of the process.  In host code this name is only a handle for
// hipGetSymbolAddress: kernels receive the device address looked up per device.
static __device__ __align__(256) unsigned char noalloc_scratch[QAOA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of noalloc_scratch, per device (null until looked up)

// Device address of noalloc_scratch on device `dev`, looked up on first use
// with that device current and kept for later calls.
int noalloc_scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(QAOA_ERR_DEVICE, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != dev) HIP_TRY(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch));
    if (cur != dev) HIP_TRY(hipSetDevice(cur));
    if (e != hipSuccess || ptr == nullptr)
      return fail(QAOA_ERR_DEVICE, "hipGetSymbolAddress(noalloc_scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return QAOA_OK;
}

}  // namespace

extern "C" {

int qaoa_evolve_noalloc(int n, int p, const double* gamma, const double* beta, const void* d_diag, int diag_dtype,
                        double diag_offset, size_t diag_bytes, void* d_state, int state_dtype, size_t state_bytes,
                        int init, double* d_out, void* stream) {
  int rc = validate_common(n, d_diag, diag_dtype, diag_offset, diag_bytes, d_state, state_dtype, state_bytes);
  if (rc) return rc;
  rc = validate_angles(p, gamma, beta);
  if (rc) return rc;
  if (init != 0 && init != 1) return fail(QAOA_ERR_INVALID, "init must be 0 or 1");
  const size_t need = (p > 0 || d_out) ? evolve_work_bytes(n, state_dtype) : 0;
  if (need > (size_t)QAOA_NOALLOC_SCRATCH_BYTES)
    return fail(QAOA_ERR_NOMEM,
                "qaoa_evolve_noalloc: n=%d %s needs %zu bytes of scratch, more than its static %zu bytes "
                "(use qaoa_evolve with a workspace)",
                n, state_dtype == QAOA_C128 ? "complex128" : "complex64", need, (size_t)QAOA_NOALLOC_SCRATCH_BYTES);
  void* work = nullptr;
  if (need) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int dev = -1;
    if (st) {
      HIP_TRY(hipStreamGetDevice(st, &dev));
    } else {
      HIP_TRY(hipGetDevice(&dev));
    }
    rc = noalloc_scratch_address(dev, &work);
    if (rc) return rc;
  }
  return qaoa_evolve(n, p, gamma, beta, d_diag, diag_dtype, diag_offset, diag_bytes, d_state, state_dtype,
                     state_bytes, init, d_out, work, need ? (size_t)QAOA_NOALLOC_SCRATCH_BYTES : 0, stream);
}

int qaoa_expectation(int n, const void* d_state, int state_dtype, size_t state_bytes, const void* d_diag,
                     int diag_dtype, double diag_offset, size_t diag_bytes, double* d_out, void* d_work,
                     size_t work_bytes, void* stream) {
  int rc = validate_common(n, d_diag, diag_dtype, diag_offset, diag_bytes, d_state, state_dtype, state_bytes);
  if (rc) return rc;
  if (!d_out) return fail(QAOA_ERR_INVALID, "d_out is NULL");
  size_t need = 0;
  qaoa_workspace_bytes(QAOA_OP_EXPECTATION, n, state_dtype, diag_dtype, &need);
  if (!d_work || work_bytes < need) return fail(QAOA_ERR_NOMEM, "workspace too small: need %zu bytes", need);
  return enqueue_expectation(n, d_state, state_dtype, d_diag, diag_dtype, diag_offset, d_out, d_work,
                             reinterpret_cast<hipStream_t>(stream));
}

int qaoa_batch_workspace_bytes(int n, int p, int batch, int state_dtype, int diag_dtype, size_t* bytes) {
  if (!bytes) return fail(QAOA_ERR_INVALID, "bytes is NULL");
  if (n < 1 || n > QAOA_MAX_QUBITS) return fail(QAOA_ERR_INVALID, "n=%d out of range [1, %d]", n, QAOA_MAX_QUBITS);
  if (p < 0 || batch < 1) return fail(QAOA_ERR_INVALID, "need p >= 0 and batch >= 1");
  if (!valid_state_dtype(state_dtype)) return fail(QAOA_ERR_INVALID, "bad state dtype %d", state_dtype);
  if (!valid_diag_dtype(diag_dtype)) return fail(QAOA_ERR_INVALID, "bad diag dtype %d", diag_dtype);
  *bytes = evolve_work(n, (size_t)batch, (size_t)batch * (size_t)p, state_dtype).total;
  return QAOA_OK;
}

int qaoa_evolve_batch(int n, int p, int batch, const double* d_gamma, const double* d_beta, const void* d_diag,
                      int diag_dtype, double diag_offset, size_t diag_bytes, void* d_states, int state_dtype,
                      size_t states_bytes, int init, double* d_out, int sets_per_pass, void* d_work,
                      size_t work_bytes, void* stream) {
  if (n < 1 || n > QAOA_MAX_QUBITS) return fail(QAOA_ERR_INVALID, "n=%d out of range [1, %d]", n, QAOA_MAX_QUBITS);
  if (batch < 1) return fail(QAOA_ERR_INVALID, "batch must be >= 1");
  if (p < 0) return fail(QAOA_ERR_INVALID, "p < 0");
  if (p > 0 && (!d_gamma || !d_beta)) return fail(QAOA_ERR_INVALID, "d_gamma/d_beta is NULL");
  if (sets_per_pass < 0) return fail(QAOA_ERR_INVALID, "sets_per_pass < 0");
  if (init != 0 && init != 1) return fail(QAOA_ERR_INVALID, "init must be 0 or 1");
  const uint64_t N = (uint64_t)1 << n;
  int rc = validate_common(n, d_diag, diag_dtype, diag_offset, diag_bytes, d_states, state_dtype,
                           states_bytes / (size_t)batch);
  if (rc) return rc;
  const size_t S = state_elem_bytes(state_dtype);
  if (states_bytes < (size_t)batch * N * S)
    return fail(QAOA_ERR_NOMEM, "states buffer has %zu bytes, needs %llu", states_bytes,
                (unsigned long long)((size_t)batch * N * S));
  const size_t need = evolve_work(n, (size_t)batch, (size_t)batch * (size_t)std::max(p, 0), state_dtype).total;
  if (!d_work || work_bytes < need) return fail(QAOA_ERR_NOMEM, "workspace too small: need %zu bytes", need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int G = (sets_per_pass == 0 || sets_per_pass > batch) ? std::min(batch, 65535) : std::min(sets_per_pass, 65535);
  if (p == 0) {
    const double amp0 = std::pow(2.0, -0.5 * n);
    for (int s = 0; s < batch; ++s) {
      void* psi = reinterpret_cast<char*>(d_states) + (size_t)s * N * S;
      if (init) {
        if (state_dtype == QAOA_C128)
          hipLaunchKernelGGL((qk::fill_state_kernel<qk::C128>), dim3(grid_for(N, 256, 8192)), dim3(256), 0, st, psi, N, amp0);
        else
          hipLaunchKernelGGL((qk::fill_state_kernel<qk::C64>), dim3(grid_for(N, 256, 8192)), dim3(256), 0, st, psi, N, amp0);
        LAUNCH_CHECK("fill_state_kernel");
      }
      if (d_out) {
        rc = enqueue_expectation(n, psi, state_dtype, d_diag, diag_dtype, diag_offset, d_out + 2 * s, d_work, st);
        if (rc) return rc;
      }
    }
    return QAOA_OK;
  }
  return enqueue_evolve(n, p, batch, nullptr, nullptr, d_gamma, d_beta, d_diag, diag_dtype, diag_offset, d_states,
                        state_dtype, init, d_out, G, d_work, tuning_now(), st);
}

int qaoa_plan_describe(int kind, int n, int state_dtype, int elem_bytes, int* out, int cap) {
  if (n < 1 || n > QAOA_MAX_QUBITS) return -fail(QAOA_ERR_INVALID, "n=%d out of range", n);
  Plan pl;
  if (kind == 0 || kind == 1) {
    if (!valid_state_dtype(state_dtype)) return -fail(QAOA_ERR_INVALID, "bad state dtype %d", state_dtype);
    pl = kind == 0 ? state_plan(n, state_dtype, tuning_now().wide) : adjoint_plan(n, state_elem_bytes(state_dtype));
  } else if (kind == 2) {
    if (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) return -fail(QAOA_ERR_INVALID, "bad elem_bytes");
    pl = make_plan(n, (size_t)elem_bytes);
  } else {
    return -fail(QAOA_ERR_INVALID, "bad plan kind %d", kind);
  }
  std::vector<int> v;
  v.push_back((int)pl.sweeps.size());
  v.push_back(pl.eb);
  v.push_back(pl.single ? 1 : 0);
  v.push_back(pl.wide ? 1 : 0);
  for (const auto& g : pl.sweeps) {
    v.push_back(g.tb); v.push_back(g.R); v.push_back(g.hA); v.push_back(g.qA); v.push_back(g.qB);
    v.push_back(g.act_lo); v.push_back(g.w_store); v.push_back(g.nchunks);
    for (int c = 0; c < g.nchunks; ++c) { v.push_back(g.chunk[c].w); v.push_back(g.chunk[c].jlo); v.push_back(g.chunk[c].jhi); }
  }
  if (out) for (int i = 0; i < (int)v.size() && i < cap; ++i) out[i] = v[i];
  return (int)v.size();
}

int qaoa_schedule_describe(int kind, int n, int p, int state_dtype, int init, int reduce, int* out, int cap) {
  if (kind != 0 && kind != 1) return -fail(QAOA_ERR_INVALID, "bad schedule kind %d", kind);
  if (n < 1 || n > QAOA_MAX_QUBITS) return -fail(QAOA_ERR_INVALID, "n=%d out of range", n);
  if (p < 0) return -fail(QAOA_ERR_INVALID, "p < 0");
  if (!valid_state_dtype(state_dtype)) return -fail(QAOA_ERR_INVALID, "bad state dtype %d", state_dtype);
  const size_t S = state_elem_bytes(state_dtype);
  const Tuning tn = tuning_now();
  const Plan pl = kind == 0 ? state_plan(n, state_dtype, tn.wide) : adjoint_plan(n, S);
  if (pl.single) return 0;
  const std::vector<SweepStep> sched = kind == 0
                                           ? sweep_schedule((int)pl.sweeps.size(), p, init != 0, reduce != 0, tn.fuse)
                                           : adjoint_schedule((int)pl.sweeps.size(), p, tn.fuse);
  int i = 0;
  for (const auto& s : sched) {
    const int v[3] = {s.sweep, s.layer, s.flags};
    for (int j = 0; j < 3; ++j, ++i)
      if (out && i < cap) out[i] = v[j];
  }
  return i;
}

static size_t xy_work_bytes(int n, int mixer, int sdt) {
  const XyPlan pl = make_xy_plan(n, mixer, state_elem_bytes(sdt));
  uint64_t blocks = 1;
  for (const auto& sw : pl.sweeps) blocks = std::max(blocks, plan_blocks(n, sw.g));
  const size_t stride = 2 * std::max<uint64_t>(blocks, kExpectBlocks);
  const size_t rows = qk::kPrepRows;
  return sizeof(double) * stride + ((qk::kParamRow * sizeof(double) * rows + 255) / 256) * 256 +
         rows * qk::kTabRow * sizeof(double2) + sizeof(double) * 2 * kReduceChunks;
}

static int validate_xy(int n, int mixer, int state_dtype) {
  if (mixer != QAOA_MIXER_XY_RING && mixer != QAOA_MIXER_XY_COMPLETE)
    return fail(QAOA_ERR_INVALID, "mixer must be QAOA_MIXER_XY_RING or QAOA_MIXER_XY_COMPLETE, got %d", mixer);
  if (n < 2 || n > 30) return fail(QAOA_ERR_INVALID, "n=%d out of range [2, 30] for XY mixers", n);
  if (!valid_state_dtype(state_dtype)) return fail(QAOA_ERR_INVALID, "bad state dtype %d", state_dtype);
  return QAOA_OK;
}

int qaoa_xy_workspace_bytes(int n, int mixer, int state_dtype, size_t* bytes) {
  if (!bytes) return fail(QAOA_ERR_INVALID, "bytes is NULL");
  int rc = validate_xy(n, mixer, state_dtype);
  if (rc) return rc;
  *bytes = xy_work_bytes(n, mixer, state_dtype);
  return QAOA_OK;
}

int qaoa_xy_plan_describe(int n, int mixer, int state_dtype, int* out, int cap) {
  if (validate_xy(n, mixer, state_dtype)) return -QAOA_ERR_INVALID;
  const XyPlan pl = make_xy_plan(n, mixer, state_elem_bytes(state_dtype));
  std::vector<int> v{(int)pl.sweeps.size(), pl.eb, pl.single ? 1 : 0};
  for (const auto& sw : pl.sweeps) {
    v.insert(v.end(), {sw.g.tb, sw.g.R, sw.g.hA, sw.g.qA, sw.g.qB, (int)sw.gates.size()});
    for (const auto& e : sw.gates) { v.push_back(e.first); v.push_back(e.second); }
  }
  if (out) for (int i = 0; i < (int)v.size() && i < cap; ++i) out[i] = v[i];
  return (int)v.size();
}

int qaoa_evolve_xy(int n, int p, const double* gamma, const double* beta, int mixer, const void* d_diag,
                   int diag_dtype, double diag_offset, size_t diag_bytes, void* d_state, int state_dtype,
                   size_t state_bytes, int init, int k, double* d_out, void* d_work, size_t work_bytes,
                   void* stream) {
  int rc = validate_xy(n, mixer, state_dtype);
  if (rc) return rc;
  rc = validate_common(n, d_diag, diag_dtype, diag_offset, diag_bytes, d_state, state_dtype, state_bytes);
  if (rc) return rc;
  rc = validate_angles(p, gamma, beta);
  if (rc) return rc;
  if (init != QAOA_INIT_GIVEN && init != QAOA_INIT_PLUS && init != QAOA_INIT_DICKE)
    return fail(QAOA_ERR_INVALID, "init must be QAOA_INIT_GIVEN, _PLUS or _DICKE");
  if (init == QAOA_INIT_DICKE && (k < 0 || k > n)) return fail(QAOA_ERR_INVALID, "Dicke weight k=%d not in [0, n]", k);
  const size_t need = xy_work_bytes(n, mixer, state_dtype);
  if (!d_work || work_bytes < need) return fail(QAOA_ERR_NOMEM, "workspace too small: need %zu bytes", need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint64_t N = (uint64_t)1 << n;
  if (p == 0 && init == QAOA_INIT_GIVEN) {
    if (d_out) return enqueue_expectation(n, d_state, state_dtype, d_diag, diag_dtype, diag_offset, d_out, d_work, st);
    return QAOA_OK;
  }
  const XyPlan pl = make_xy_plan(n, mixer, state_elem_bytes(state_dtype));
  for (const auto& sw : pl.sweeps)
    if ((int)sw.gates.size() > qk::kMaxXyGates)
      return fail(QAOA_ERR_UNSUPPORTED, "internal: %zu gates in one XY sweep (max %d)", sw.gates.size(), qk::kMaxXyGates);
  uint64_t blocks_max = 1;
  for (const auto& sw : pl.sweeps) blocks_max = std::max(blocks_max, plan_blocks(n, sw.g));
  const size_t stride = 2 * std::max<uint64_t>(blocks_max, kExpectBlocks);
  char* wk = reinterpret_cast<char*>(d_work);
  double* partials = reinterpret_cast<double*>(wk);
  double* pset = reinterpret_cast<double*>(wk + sizeof(double) * stride);
  const size_t pset_bytes = ((qk::kParamRow * sizeof(double) * qk::kPrepRows + 255) / 256) * 256;
  double2* tab = reinterpret_cast<double2*>(wk + sizeof(double) * stride + pset_bytes);
  double* tmp = reinterpret_cast<double*>(wk + sizeof(double) * stride + pset_bytes +
                                          qk::kPrepRows * qk::kTabRow * sizeof(double2));
  const bool use_tab = diag_dtype != QAOA_DIAG_F64;

  qk::XyArgs a{};
  a.s.psi = d_state;
  a.s.diag = d_diag;
  a.s.diag_offset = diag_offset;
  a.s.ptab = tab;
  a.s.pset = pset;
  a.s.partials = partials;
  a.s.partials_stride = stride;
  a.s.p_total = qk::kPrepRows;
  a.s.set_stride_bytes = N * state_elem_bytes(state_dtype);
  if (init == QAOA_INIT_DICKE) {
    double cnk = 1.0;
    for (int t = 1; t <= k; ++t) cnk = cnk * (double)(n - k + t) / (double)t;
    a.s.amp0 = 1.0 / std::sqrt(cnk);
    a.dicke_k = k;
  } else {
    a.s.amp0 = std::pow(2.0, -0.5 * n);
    a.dicke_k = -1;
  }
  const bool gen = init != QAOA_INIT_GIVEN;
  uint64_t last_blocks = 1;
  auto set_gates = [&](const XySweep& sw, int count) {
    a.ngates = count;
    for (int e = 0; e < count; ++e) {
      a.gate[e][0] = (int8_t)sw.gates[e].first;
      a.gate[e][1] = (int8_t)sw.gates[e].second;
    }
    set_xy_groups(a, sw.g.tb, pl.eb);
  };
  if (p == 0) {  // the initial state only (and its objective)
    a.s.g = pl.sweeps[0].g;
    a.s.nlayers = 0;
    a.s.layer0 = 0;
    set_gates(pl.sweeps[0], 0);
    a.s.flags = qk::F_INIT | (d_out ? qk::F_EXPV : 0);
    last_blocks = plan_blocks(n, a.s.g);
    launch_xy(a, state_dtype, diag_dtype, pl.eb, last_blocks, 1, st);
    LAUNCH_CHECK("qaoa_xy_kernel");
  }
  for (int l0 = 0; l0 < p; l0 += qk::kMaxLayersPerLaunch) {
    const int nl = std::min(qk::kMaxLayersPerLaunch, p - l0);
    qk::PrepArgs pa{};
    pa.pset = pset;
    pa.tab = use_tab ? tab : nullptr;
    pa.base = use_tab ? table_base(diag_dtype, diag_offset) : 0.0;
    pa.off = diag_offset;
    pa.rows = nl;
    for (int i = 0; i < nl; ++i) { pa.gamma[i] = gamma[l0 + i]; pa.beta[i] = beta[l0 + i]; }
    hipLaunchKernelGGL(qk::layer_prep_kernel, dim3(nl), dim3(256), 0, st, pa);
    LAUNCH_CHECK("layer_prep_kernel");
    if (pl.single) {
      a.s.g = pl.sweeps[0].g;
      a.s.nlayers = nl;
      a.s.layer0 = 0;
      set_gates(pl.sweeps[0], (int)pl.sweeps[0].gates.size());
      a.s.flags = qk::F_PHASE | ((l0 == 0 && gen) ? qk::F_INIT : 0) | ((l0 + nl == p && d_out) ? qk::F_EXPV : 0);
      launch_xy(a, state_dtype, diag_dtype, pl.eb, 1, 1, st);
      LAUNCH_CHECK("qaoa_xy_kernel");
      continue;
    }
    a.s.nlayers = 1;
    for (int l = l0; l < l0 + nl; ++l) {
      a.s.layer0 = l - l0;
      for (size_t sw = 0; sw < pl.sweeps.size(); ++sw) {
        a.s.g = pl.sweeps[sw].g;
        set_gates(pl.sweeps[sw], (int)pl.sweeps[sw].gates.size());
        const bool last = (l == p - 1) && (sw + 1 == pl.sweeps.size());
        a.s.flags = (sw == 0 ? qk::F_PHASE : 0) | ((sw == 0 && l == 0 && gen) ? qk::F_INIT : 0) |
                    ((last && d_out) ? qk::F_EXPV : 0);
        last_blocks = plan_blocks(n, a.s.g);
        launch_xy(a, state_dtype, diag_dtype, pl.eb, last_blocks, 1, st);
        LAUNCH_CHECK("qaoa_xy_kernel");
      }
    }
  }
  if (d_out) return enqueue_reduce(partials, last_blocks, stride, 1, tmp, d_out, st);
  (void)work_bytes;
  return QAOA_OK;
}

int qaoa_grad_workspace_bytes(int n, int p, int state_dtype, int diag_dtype, size_t* bytes) {
  if (!bytes) return fail(QAOA_ERR_INVALID, "bytes is NULL");
  if (n < 1 || n > QAOA_MAX_QUBITS) return fail(QAOA_ERR_INVALID, "n=%d out of range [1, %d]", n, QAOA_MAX_QUBITS);
  if (p < 1) return fail(QAOA_ERR_INVALID, "p must be >= 1");
  if (!valid_state_dtype(state_dtype)) return fail(QAOA_ERR_INVALID, "bad state dtype %d", state_dtype);
  if (!valid_diag_dtype(diag_dtype)) return fail(QAOA_ERR_INVALID, "bad diag dtype %d", diag_dtype);
  *bytes = grad_work(n, p, state_dtype).total;
  return QAOA_OK;
}

int qaoa_grad(int n, int p, const double* gamma, const double* beta, const void* d_diag, int diag_dtype,
              double diag_offset, size_t diag_bytes, void* d_state, void* d_adj, int state_dtype,
              size_t state_bytes, double* d_out, void* d_work, size_t work_bytes, void* stream) {
  int rc = validate_common(n, d_diag, diag_dtype, diag_offset, diag_bytes, d_state, state_dtype, state_bytes);
  if (rc) return rc;
  rc = validate_angles(p, gamma, beta);
  if (rc) return rc;
  if (p < 1) return fail(QAOA_ERR_INVALID, "p must be >= 1 for a gradient");
  if (!d_adj || !d_out) return fail(QAOA_ERR_INVALID, "d_adj/d_out is NULL");
  if (d_adj == d_state) return fail(QAOA_ERR_INVALID, "d_adj must not alias d_state");
  const GradWork gw = grad_work(n, p, state_dtype);
  if (!d_work || work_bytes < gw.total) return fail(QAOA_ERR_NOMEM, "workspace too small: need %zu bytes", gw.total);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* wk = reinterpret_cast<char*>(d_work);
  const Tuning tn = tuning_now();

  // forward pass: psi_p in d_state, (E, norm) in d_out[0..1] (d_out[1] is
  // overwritten by the gradient below)
  rc = enqueue_evolve(n, p, 1, gamma, beta, nullptr, nullptr, d_diag, diag_dtype, diag_offset, d_state, state_dtype, 1,
                      d_out, 1, d_work, tn, st);
  if (rc) return rc;

  // parameter rows and tables of all p layers
  double* pset = reinterpret_cast<double*>(wk + gw.pset_off);
  double2* tab = reinterpret_cast<double2*>(wk + gw.tab_off);
  double* rev = reinterpret_cast<double*>(wk + gw.rev_off);
  const bool use_tab = diag_dtype != QAOA_DIAG_F64;
  for (int l0 = 0; l0 < p; l0 += 32) {
    qk::PrepArgs pa{};
    pa.pset = pset + qk::kParamRow * (size_t)l0;
    pa.tab = use_tab ? tab + (size_t)l0 * qk::kTabRow : nullptr;
    pa.base = use_tab ? table_base(diag_dtype, diag_offset) : 0.0;
    pa.off = diag_offset;
    pa.rows = std::min(32, p - l0);
    for (int i = 0; i < pa.rows; ++i) { pa.gamma[i] = gamma[l0 + i]; pa.beta[i] = beta[l0 + i]; }
    hipLaunchKernelGGL(qk::layer_prep_kernel, dim3(pa.rows), dim3(256), 0, st, pa);
    LAUNCH_CHECK("layer_prep_kernel");
  }

  const Plan pl = adjoint_plan(n, state_elem_bytes(state_dtype));
  qk::AdjArgs a{};
  a.psi = d_state;
  a.lam = d_adj;
  a.diag = d_diag;
  a.diag_offset = diag_offset;
  a.pset = pset;
  a.ptab = tab;
  const int nsw = (int)pl.sweeps.size();
  uint64_t blocks = 1;
  if (pl.single) {
    a.g = pl.sweeps[0];
    a.nlayers = p;
    a.partials = rev;
    a.layer_partials_stride = gw.layer_stride;
    rc = launch_adj(a, state_dtype, diag_dtype, true, pl.eb, 0, 1, st);
    if (rc) return rc;
    LAUNCH_CHECK("qaoa_adjoint_tile_kernel");
  } else {
    blocks = plan_blocks(n, pl.sweeps[0]);
    auto slot = [&](int l, int sw) { return rev + (size_t)l * gw.layer_stride + (size_t)sw * blocks * 2; };
    for (const SweepStep& stp : adjoint_schedule(nsw, p, tn.fuse)) {
      a.layer = stp.layer;
      a.g = pl.sweeps[stp.sweep];
      a.partials = slot(stp.layer, stp.sweep);
      a.partials2 = (stp.flags & qk::A_FUSE) ? slot(stp.layer - 1, stp.sweep) : nullptr;
      rc = launch_adj(a, state_dtype, diag_dtype, false, kEBAdj, stp.flags, blocks, st);
      if (rc) return rc;
      LAUNCH_CHECK("qaoa_adjoint_kernel");
    }
  }
  hipLaunchKernelGGL(qk::grad_finalize_kernel, dim3(p), dim3(256), 0, st, (const double*)rev, p, nsw, blocks,
                     (uint64_t)gw.layer_stride, d_out);
  LAUNCH_CHECK("grad_finalize_kernel");
  (void)work_bytes;
  return QAOA_OK;
}

}  // extern "C"
