// Host-only checks of the request loop's arena bookkeeping (arena.hpp),
// compiled with g++ by test_server_arena_cpu.py.  Prints "name value" lines.
#include <cstdio>

#include "arena.hpp"

using qaoa_arena::ArenaMap;
using qaoa_arena::kNone;

int main() {
  const size_t U = 1 << 20;  // one unit
  // The fragmentation a mid-arena cost vector causes: request A (4 units) at
  // the bottom, then a cost vector (2 units) placed first fit right after it;
  // once A finishes, 8 units are free but no block holds 6.
  {
    ArenaMap m(10 * U);
    const size_t a = m.alloc_low(4 * U);
    const size_t c = m.alloc_low(2 * U);
    m.release(a, 4 * U);
    std::printf("firstfit_cost_at %zu\n", c / U);
    std::printf("firstfit_free_total %zu\n", (m.size() - m.used()) / U);
    std::printf("firstfit_largest %zu\n", m.largest_free() / U);
    std::printf("firstfit_six_fits %d\n", m.alloc_low(6 * U) != kNone);
    std::printf("head_blocked_idle_rejects %d\n",
                qaoa_arena::head_blocked(0) == qaoa_arena::HeadAction::kReject);
    std::printf("head_blocked_busy_waits %d\n", qaoa_arena::head_blocked(1) == qaoa_arena::HeadAction::kWait);
  }
  // The same sequence with the cost vector placed from the top.
  {
    ArenaMap m(10 * U);
    const size_t a = m.alloc_low(4 * U);
    const size_t c = m.alloc_high(2 * U);
    m.release(a, 4 * U);
    std::printf("top_cost_at %zu\n", c / U);
    std::printf("top_largest %zu\n", m.largest_free() / U);
    std::printf("top_six_fits %d\n", m.alloc_low(6 * U) != kNone);
  }
  // Exact bookkeeping: granule rounding, coalescing in any release order,
  // a full arena, high and low placement meeting in the middle.
  {
    ArenaMap m(1000 * 256 + 100);  // rounded down to 1000 granules
    std::printf("size_granules %zu\n", m.size() / 256);
    const size_t x = m.alloc_low(1);      // 1 granule at 0
    const size_t y = m.alloc_high(257);   // 2 granules at the top
    const size_t z = m.alloc_low(256 * 997);
    std::printf("x %zu y %zu z %zu\n", x / 256, y / 256, z / 256);
    std::printf("full_low_fails %d full_high_fails %d\n", m.alloc_low(1) == kNone, m.alloc_high(1) == kNone);
    std::printf("used_granules %zu\n", m.used() / 256);
    m.release(z, 256 * 997);
    m.release(x, 1);
    std::printf("after_release_ranges %zu after_release_largest %zu\n", m.free_ranges(), m.largest_free() / 256);
    m.release(y, 257);
    std::printf("all_free_ranges %zu all_free_largest %zu used %zu peak %zu\n", m.free_ranges(), m.largest_free() / 256,
                m.used(), m.peak() / 256);
  }
  return 0;
}
