// qaoa.hip -- host side of libqaoa.so: argument validation, sweep planning,
// kernel launches and the C ABI declared in include/qaoa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
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
// Capped at 13 bits so a tile never needs more than 512 threads (2^(13-kEB)).
int tile_bits_for_bytes(size_t elem_bytes) {
  int tb = 0;
  while (tb < 13 && ((size_t)1 << (tb + 1)) * elem_bytes <= 65536) ++tb;
  return tb;
}
// Minimum passenger bits so that a high sweep touches >= 128 contiguous bytes.
int min_passenger_bits(size_t elem_bytes) {
  int p = 0;
  while (((size_t)1 << p) * elem_bytes < 128) ++p;
  return p;
}

// Chunk order for one tile: first the top EB bits (the coalesced load window),
// then the remaining active bits bottom-up; the tile is stored from the last
// window if that window keeps >= 2^store_min_bits contiguous elements per run,
// else it is exchanged back to the load window first.
qk::TileGeom make_geom(int tb, int P, int q0, int eb, bool low, int store_min_bits) {
  qk::TileGeom g{};
  g.tb = tb; g.P = P; g.q0 = q0; g.nchunks = 0;
  const int top_w = tb - eb;
  const int lo0 = std::max(P, top_w);
  g.chunk[g.nchunks++] = qk::Chunk{(int8_t)top_w, (int8_t)(lo0 - top_w), (int8_t)eb, 0};
  int rlo = P;
  const int rhi = lo0;
  while (rlo < rhi) {
    const int chi = std::min(rlo + eb, rhi);
    const int w = std::min(rlo, top_w);
    g.chunk[g.nchunks++] = qk::Chunk{(int8_t)w, (int8_t)(rlo - w), (int8_t)(chi - w), 0};
    rlo = chi;
  }
  const int last_w = g.chunk[g.nchunks - 1].w;
  const int contig = low ? tb : P;
  g.w_store = (std::min(last_w, contig) >= store_min_bits || last_w == top_w) ? last_w : top_w;
  return g;
}

// Sweep plan covering all n qubits with tiles of at most tbmax bits.
struct Plan {
  bool single;          // whole vector in one tile
  int eb;               // register bits per thread
  std::vector<qk::TileGeom> sweeps;
};

Plan make_plan(int n, size_t elem_bytes) {
  Plan pl;
  const int tbmax = tile_bits_for_bytes(elem_bytes);
  const int pmin = min_passenger_bits(elem_bytes);
  const int smin = pmin;  // store runs of >= 128 B
  if (n <= tbmax) {
    pl.single = true;
    pl.eb = std::min(kEB, n);
    pl.sweeps.push_back(make_geom(n, 0, 0, pl.eb, true, 0));
    return pl;
  }
  pl.single = false;
  pl.eb = kEB;
  pl.sweeps.push_back(make_geom(tbmax, 0, 0, kEB, true, smin));
  const int r = n - tbmax;
  const int hmax = tbmax - pmin;
  const int ns = (r + hmax - 1) / hmax;
  int q = tbmax;
  for (int i = 0; i < ns; ++i) {
    const int h = r / ns + (i < r % ns ? 1 : 0);
    pl.sweeps.push_back(make_geom(tbmax, tbmax - h, q, kEB, false, smin));
    q += h;
  }
  return pl;
}

uint64_t plan_blocks(int n, const qk::TileGeom& g) { return (uint64_t)1 << (n - g.tb); }

// ---------------------------------------------------------------------------
// typed launchers
// ---------------------------------------------------------------------------
template <class S, class D, int EB>
void launch_sweep_t(const qk::SweepArgs& a, uint64_t blocks, hipStream_t st) {
  const uint32_t threads = 1u << (a.g.tb - EB);
  // tile buffer + phase tables; also the reduction scratch (16 doubles, or 2 per
  // thread for a partial wave), which is used after the tables are done with
  const size_t tile = ((size_t)1 << a.g.tb) * S::kBytes;
  const size_t tab = (D::kTable && (a.flags & qk::F_PHASE)) ? qk::kTabEntries * sizeof(double2) : 0;
  const size_t lds = std::max<size_t>(tile + tab, std::max<size_t>(16, 2 * threads) * sizeof(double));
  hipLaunchKernelGGL((qk::qaoa_sweep_kernel<S, D, EB>), dim3((uint32_t)blocks), dim3(threads), lds, st, a);
}

template <class S, class D>
void launch_sweep_d(const qk::SweepArgs& a, int eb, uint64_t blocks, hipStream_t st) {
  switch (eb) {
    case 1: launch_sweep_t<S, D, 1>(a, blocks, st); break;
    case 2: launch_sweep_t<S, D, 2>(a, blocks, st); break;
    case 3: launch_sweep_t<S, D, 3>(a, blocks, st); break;
    default: launch_sweep_t<S, D, 4>(a, blocks, st); break;
  }
}

template <class S>
void launch_sweep_s(const qk::SweepArgs& a, int diag_dtype, int eb, uint64_t blocks, hipStream_t st) {
  switch (diag_dtype) {
    case QAOA_DIAG_I32: launch_sweep_d<S, qk::DI32>(a, eb, blocks, st); break;
    case QAOA_DIAG_U16: launch_sweep_d<S, qk::DU16>(a, eb, blocks, st); break;
    default: launch_sweep_d<S, qk::DF64>(a, eb, blocks, st); break;
  }
}

void launch_sweep(const qk::SweepArgs& a, int state_dtype, int diag_dtype, int eb, uint64_t blocks, hipStream_t st) {
  if (state_dtype == QAOA_C128) launch_sweep_s<qk::C128>(a, diag_dtype, eb, blocks, st);
  else launch_sweep_s<qk::C64>(a, diag_dtype, eb, blocks, st);
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

// Evolve workspace: [per-block (E, norm) partials][phase tables of up to
// kMaxLayersPerLaunch layers].
size_t partials_bytes(int n, int state_dtype) {
  const Plan pl = make_plan(n, state_elem_bytes(state_dtype));
  const uint64_t last = plan_blocks(n, pl.sweeps.back());
  return 2 * sizeof(double) * std::max<uint64_t>(last, kExpectBlocks);
}
constexpr size_t kTableBytes = (size_t)qk::kMaxLayersPerLaunch * qk::kTabEntries * sizeof(double2);
size_t evolve_work_bytes(int n, int state_dtype) { return partials_bytes(n, state_dtype) + kTableBytes; }

// Phase tables for layers [l0, l0 + nl) into `tab` (integer cost vectors only).
int enqueue_phase_tables(double2* tab, const double* gamma, int l0, int nl, double base, hipStream_t st) {
  qk::PhaseTableArgs t{};
  t.out = tab;
  t.base = base;
  t.nlayers = nl;
  for (int i = 0; i < nl; ++i) t.gamma[i] = gamma[l0 + i];
  hipLaunchKernelGGL(qk::phase_table_kernel, dim3(nl), dim3(256), 0, st, t);
  LAUNCH_CHECK("phase_table_kernel");
  return QAOA_OK;
}

double table_base(int diag_dtype, double diag_offset) {
  return (diag_dtype == QAOA_DIAG_I32 ? qk::DI32::kTableBase : qk::DU16::kTableBase) + diag_offset;
}

}  // namespace

extern "C" {

const char* qaoa_version(void) { return "0.1.0"; }

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

  const Plan pl = make_plan(n, state_elem_bytes(state_dtype));
  qk::SweepArgs a{};
  a.psi = d_state;
  a.diag = d_diag;
  a.diag_offset = diag_offset;
  a.amp0 = amp0;
  double* partials = reinterpret_cast<double*>(d_work);
  double2* tab = reinterpret_cast<double2*>(reinterpret_cast<char*>(d_work) + partials_bytes(n, state_dtype));
  const bool use_tab = diag_dtype != QAOA_DIAG_F64;
  const double tbase = use_tab ? table_base(diag_dtype, diag_offset) : 0.0;
  a.ptab = tab;

  if (pl.single) {
    // whole state in one tile: up to kMaxLayersPerLaunch layers per launch
    a.g = pl.sweeps[0];
    for (int l0 = 0; l0 < p; l0 += qk::kMaxLayersPerLaunch) {
      const int nl = std::min(qk::kMaxLayersPerLaunch, p - l0);
      const bool last = (l0 + nl == p);
      if (use_tab) {
        const int rc2 = enqueue_phase_tables(tab, gamma, l0, nl, tbase, st);
        if (rc2) return rc2;
      }
      a.flags = qk::F_PHASE | ((l0 == 0 && init) ? qk::F_INIT : 0) | ((last && d_out) ? qk::F_EXPV : 0);
      a.nlayers = nl;
      for (int i = 0; i < nl; ++i) {
        a.gamma[i] = gamma[l0 + i];
        a.ca[i] = std::cos(beta[l0 + i]);
        a.sb[i] = std::sin(beta[l0 + i]);
      }
      a.partials = d_out;  // one block: its sum is the result
      launch_sweep(a, state_dtype, diag_dtype, pl.eb, 1, st);
      LAUNCH_CHECK("qaoa_sweep_kernel");
    }
    return QAOA_OK;
  }

  const size_t nsw = pl.sweeps.size();
  for (int l = 0; l < p; ++l) {
    if (use_tab && l % qk::kMaxLayersPerLaunch == 0) {
      const int rc2 = enqueue_phase_tables(tab, gamma, l, std::min(qk::kMaxLayersPerLaunch, p - l), tbase, st);
      if (rc2) return rc2;
    }
    a.ptab = tab + (size_t)(l % qk::kMaxLayersPerLaunch) * qk::kTabEntries;
    for (size_t s = 0; s < nsw; ++s) {
      a.g = pl.sweeps[s];
      a.nlayers = 1;
      a.gamma[0] = gamma[l];
      a.ca[0] = std::cos(beta[l]);
      a.sb[0] = std::sin(beta[l]);
      const bool last = (l == p - 1) && (s == nsw - 1);
      a.flags = (s == 0 ? qk::F_PHASE : 0) | ((s == 0 && l == 0 && init) ? qk::F_INIT : 0) |
                ((last && d_out) ? qk::F_EXPV : 0);
      a.partials = partials;
      const uint64_t blocks = plan_blocks(n, a.g);
      launch_sweep(a, state_dtype, diag_dtype, pl.eb, blocks, st);
      LAUNCH_CHECK("qaoa_sweep_kernel");
      if (last && d_out) {
        hipLaunchKernelGGL(qk::finalize_kernel, dim3(1), dim3(256), 0, st, (const double*)partials, blocks, d_out);
        LAUNCH_CHECK("finalize_kernel");
      }
    }
  }
  return QAOA_OK;
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

int qaoa_plan_describe(int n, int state_dtype, int elem_bytes, int* out, int cap) {
  if (n < 1 || n > QAOA_MAX_QUBITS) return -fail(QAOA_ERR_INVALID, "n=%d out of range", n);
  size_t eb_bytes;
  if (state_dtype >= 0) {
    if (!valid_state_dtype(state_dtype)) return -fail(QAOA_ERR_INVALID, "bad state dtype %d", state_dtype);
    eb_bytes = state_elem_bytes(state_dtype);
  } else {
    if (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) return -fail(QAOA_ERR_INVALID, "bad elem_bytes");
    eb_bytes = (size_t)elem_bytes;
  }
  const Plan pl = make_plan(n, eb_bytes);
  std::vector<int> v;
  v.push_back((int)pl.sweeps.size());
  v.push_back(pl.eb);
  v.push_back(pl.single ? 1 : 0);
  for (const auto& g : pl.sweeps) {
    v.push_back(g.tb); v.push_back(g.P); v.push_back(g.q0); v.push_back(g.w_store); v.push_back(g.nchunks);
    for (int c = 0; c < g.nchunks; ++c) { v.push_back(g.chunk[c].w); v.push_back(g.chunk[c].jlo); v.push_back(g.chunk[c].jhi); }
  }
  if (out) for (int i = 0; i < (int)v.size() && i < cap; ++i) out[i] = v[i];
  return (int)v.size();
}

int qaoa_grad(int n, int p, const double* gamma, const double* beta, const void* d_diag, int diag_dtype,
              double diag_offset, size_t diag_bytes, void* d_state, void* d_adj, int state_dtype,
              size_t state_bytes, double* d_out, void* d_work, size_t work_bytes, void* stream) {
  int rc = validate_common(n, d_diag, diag_dtype, diag_offset, diag_bytes, d_state, state_dtype, state_bytes);
  if (rc) return rc;
  rc = validate_angles(p, gamma, beta);
  if (rc) return rc;
  if (!d_adj || !d_out) return fail(QAOA_ERR_INVALID, "d_adj/d_out is NULL");
  (void)d_work; (void)work_bytes; (void)stream;
  return fail(QAOA_ERR_UNSUPPORTED, "qaoa_grad is not implemented in this build");
}

}  // extern "C"
