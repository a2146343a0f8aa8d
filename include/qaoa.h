/*
 * qaoa.h -- C ABI of libqaoa.so, a QAOA state-vector simulator for AMD MI355X
 * (gfx950).  It implements the hot path of "Fast Simulation of High-Depth QAOA
 * Circuits" (arXiv:2309.04841):
 *
 *   1. precompute the diagonal cost vector c[x] for all 2^n basis states from
 *      weighted spin terms (Eq. (1); Section 3.1);
 *   2. evolve the state through p layers of the phase exp(-i gamma_l c) and the
 *      transverse-field mixer prod_i exp(-i beta_l X_i) (Algorithm 3; the gate is
 *      cos(beta) I - i sin(beta) X as written in Section 3.2);
 *   3. evaluate E = sum_x |psi_x|^2 c_x (Section 3.1).
 *
 * Conventions.
 *   - Variable i (0-based) is bit i of the basis index x; spin s_i = 1 - 2*bit_i(x).
 *   - States are interleaved complex numbers (re, im): complex128 = 2 x double,
 *     complex64 = 2 x float.  2^n elements, index x at element x.
 *   - Cost vectors have 2^n elements of one of the diag dtypes below.  The value
 *     used by the simulator is  c[x] = stored[x] + diag_offset  (the offset is
 *     0 for F64 and I32 as produced by qaoa_precompute_diag; U16 needs one).
 *   - Layer order follows Algorithm 3: layer 1 first, phase before mixer.
 *
 * Memory and streams.
 *   - Every device buffer (state, cost vector, workspace, outputs) is allocated
 *     and owned by the caller; the library allocates nothing.  Sizes are passed
 *     in and checked.  qaoa_workspace_bytes() gives workspace sizes.
 *   - `stream` is a hipStream_t (NULL = the null stream).  qaoa_evolve and
 *     qaoa_expectation only enqueue work and never synchronise; results land in
 *     device memory.  qaoa_precompute_diag may synchronise `stream` once, to read
 *     back a range check (documented below).
 *   - Calls on different streams that touch the same buffers race; so do calls
 *     that share one workspace buffer concurrently.
 *
 * Errors.  Every entry point validates all arguments before enqueuing anything
 * and returns a qaoa_status; on failure nothing has been enqueued (except where
 * noted for device errors), and qaoa_last_error() returns a message for the
 * calling thread.  The library never aborts and is safe to call from several
 * host threads.
 */
#ifndef QAOA_H
#define QAOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    QAOA_OK = 0,
    QAOA_ERR_INVALID = 1,     /* bad argument: size, pointer, index, non-finite value */
    QAOA_ERR_RANGE = 2,       /* cost values not representable in the requested dtype */
    QAOA_ERR_NOMEM = 3,       /* a caller-provided buffer is too small */
    QAOA_ERR_DEVICE = 4,      /* HIP runtime or launch failure (message has the HIP error) */
    QAOA_ERR_UNSUPPORTED = 5  /* valid request the library does not implement */
};

/* State dtypes (interleaved complex). */
enum { QAOA_C64 = 0, QAOA_C128 = 1 };

/* Cost-vector dtypes. */
enum { QAOA_DIAG_F64 = 0, QAOA_DIAG_I32 = 1, QAOA_DIAG_U16 = 2 };

/* Mixers (Section 3.2) and initial states for qaoa_evolve_xy. */
enum { QAOA_MIXER_X = 0, QAOA_MIXER_XY_RING = 1, QAOA_MIXER_XY_COMPLETE = 2 };
enum { QAOA_INIT_GIVEN = 0, QAOA_INIT_PLUS = 1, QAOA_INIT_DICKE = 2 };

/* Operations for qaoa_workspace_bytes. */
enum { QAOA_OP_PRECOMPUTE = 0, QAOA_OP_EVOLVE = 1, QAOA_OP_EXPECTATION = 2, QAOA_OP_GRAD = 3 };

/* Largest qubit count accepted (2^34 complex64 amplitudes = 128 GiB). */
#define QAOA_MAX_QUBITS 34

/* Library version string, e.g. "0.1.0". Never NULL. */
const char *qaoa_version(void);

/* Message describing the last failing call made by this host thread ("" if none). */
const char *qaoa_last_error(void);

/* Process-wide tuning knobs.  They select sweep plans and the launch order
 * only: results change at most in rounding order.  Workspace sizes follow the
 * current setting, so set knobs before sizing workspaces; a call made with a
 * workspace sized under another setting fails with QAOA_ERR_NOMEM rather than
 * overrun it.
 *   QAOA_TUNE_WIDE_TILES  1 (default): complex128 states use 2^14-element tiles
 *                         when that saves a sweep per layer; 0: never.
 *   QAOA_TUNE_FUSE_LAYERS 1 (default): the sweep ending a layer also starts the
 *                         next one (evaluation and gradient); 0: one launch per
 *                         sweep and layer.
 * qaoa_set_tuning returns QAOA_ERR_INVALID for an unknown knob or value. */
enum { QAOA_TUNE_WIDE_TILES = 0, QAOA_TUNE_FUSE_LAYERS = 1 };
int qaoa_set_tuning(int knob, int value);
int qaoa_get_tuning(int knob, int *value);

/* Workspace size in bytes that `op` needs for n qubits with the given dtypes
 * (for QAOA_OP_PRECOMPUTE: the worst case over all term sets).  Writes *bytes.
 * Returns QAOA_ERR_INVALID for bad arguments. */
int qaoa_workspace_bytes(int op, int n, int state_dtype, int diag_dtype, size_t *bytes);

/*
 * qaoa_precompute_diag -- cost vector from weighted spin terms (Eq. (1),
 * Section 3.1): c[x] = sum_k w_k prod_{i in t_k} s_i(x).
 *
 *   n           number of variables, 1 <= n <= QAOA_MAX_QUBITS
 *   num_terms   L >= 0
 *   w           host, L weights (finite)
 *   term_ptr    host, L+1 offsets (CSR): term k owns term_idx[term_ptr[k] .. term_ptr[k+1]);
 *               term_ptr[0] = 0, non-decreasing.  An empty term is a constant.
 *   term_idx    host, term_ptr[L] variable indices, each 0 <= i < n (may be NULL if
 *               term_ptr[L] == 0).  A repeated index cancels (s_i^2 = 1).
 *   diag_dtype  QAOA_DIAG_F64 | QAOA_DIAG_I32 | QAOA_DIAG_U16
 *   d_diag      device, 2^n elements of diag_dtype (diag_bytes >= 2^n * size)
 *   out_offset  host, receives the offset such that c[x] = d_diag[x] + *out_offset
 *               (0 for F64 and I32)
 *   d_work      device workspace of work_bytes (may be NULL if work_bytes == 0).
 *               Only U16 with non-integer weights or 2*sum|w| >= 2^16 uses the
 *               2^n * 4-byte scratch; I32 with non-integer (dyadic) weights uses a
 *               few KiB.
 *   stream      hipStream_t
 *
 * Host arrays are only read during the call.  F64: exact for dyadic weights (else
 * rounding differs from a term-by-term sum by O(eps * sum|w|)).  I32/U16: weights
 * must be dyadic rationals (w * 2^k integral for some k <= 20) and every c[x] an
 * integer that fits the dtype (U16: max - min < 2^16); otherwise QAOA_ERR_RANGE.
 * Paths that need that check synchronise `stream` once; on QAOA_ERR_RANGE the
 * contents of d_diag are unspecified.
 */
int qaoa_precompute_diag(int n, int64_t num_terms, const double *w, const int64_t *term_ptr,
                         const int32_t *term_idx, int diag_dtype, void *d_diag, size_t diag_bytes,
                         double *out_offset, void *d_work, size_t work_bytes, void *stream);

/*
 * qaoa_evolve -- Algorithm 3: for l = 1..p, psi <- exp(-i gamma_l c) psi, then
 * psi <- prod_{i<n} exp(-i beta_l X_i) psi.  In place on d_state.
 *
 *   n, p        1 <= n <= QAOA_MAX_QUBITS, p >= 0
 *   gamma, beta host, p finite angles each (may be NULL if p == 0)
 *   d_diag      device cost vector (2^n of diag_dtype, diag_bytes), c = stored + diag_offset;
 *               diag_offset must be integral for U16 and I32 so c stays an integer
 *   d_state     device state, 2^n elements of state_dtype (state_bytes)
 *   init        1: start from |+>^n (d_state is only written);
 *               0: start from the contents of d_state
 *   d_out       device, nullable: receives d_out[0] = E = sum |psi|^2 c and
 *               d_out[1] = sum |psi|^2 of the final state (FP64, no renormalisation)
 *   d_work      device workspace, >= qaoa_workspace_bytes(QAOA_OP_EVOLVE, ...) bytes
 *               (may be NULL only when p == 0 and d_out == NULL)
 *
 * Phase factors: for F64 cost vectors exp(-i gamma_l c) is evaluated from the
 * double-precision angle gamma_l * c[x].  For integer cost vectors (I32 values in
 * [-2^15, 2^15), all U16 values) it is the product of three table entries
 * exp(-i gamma_l (256 m + base)) * exp(-i gamma_l 16 j) * exp(-i gamma_l k) with
 * c = 256 m + 16 j + k + base, each evaluated in double precision from an
 * exactly representable angle (agreeing with the direct evaluation to a few
 * units in the last place of the angle); a workgroup holding other I32 values
 * takes the same three-entry product twice, over the value's bytes.  complex64
 * states are updated in single precision (phase-table entries rounded once from
 * their double values), except in launches where a layer has |tan beta| > 64,
 * which use double precision; E and sum |psi|^2 are accumulated in FP64.
 * complex128 states are updated in double precision.
 * Results are deterministic (fixed reduction order).
 */
int qaoa_evolve(int n, int p, const double *gamma, const double *beta,
                const void *d_diag, int diag_dtype, double diag_offset, size_t diag_bytes,
                void *d_state, int state_dtype, size_t state_bytes, int init,
                double *d_out, void *d_work, size_t work_bytes, void *stream);

/*
 * qaoa_evolve_noalloc -- qaoa_evolve for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments without the workspace, the same kernels
 * and results (bitwise equal to qaoa_evolve with a workspace).  Its scratch is
 * a static device array of QAOA_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends; it covers complex64 states up to n = 32 and complex128 states
 * up to n = 31 (any p).  Larger requests return QAOA_ERR_NOMEM without
 * enqueuing anything.  The call itself allocates nothing: the array's device
 * address is looked up once per device (the stream's device, or the current
 * device for the null stream) and reused.  All calls on one GPU share that
 * array and it keeps the last call's contents: calls that overlap on one GPU
 * (different streams or host threads without ordering) race and give wrong
 * results; calls ordered on one stream are safe.
 */
#define QAOA_NOALLOC_SCRATCH_BYTES ((size_t)9 << 20)
int qaoa_evolve_noalloc(int n, int p, const double *gamma, const double *beta,
                        const void *d_diag, int diag_dtype, double diag_offset, size_t diag_bytes,
                        void *d_state, int state_dtype, size_t state_bytes, int init,
                        double *d_out, void *stream);

/*
 * qaoa_expectation -- E = sum_x |psi_x|^2 c_x and sum_x |psi_x|^2 (Section 3.1),
 * accumulated in FP64 with a fixed reduction order.  Any cost vector of the
 * right length may be passed (it need not be the one used for evolution).
 * The state is not modified.  d_out: device, 2 doubles.
 */
int qaoa_expectation(int n, const void *d_state, int state_dtype, size_t state_bytes,
                     const void *d_diag, int diag_dtype, double diag_offset, size_t diag_bytes,
                     double *d_out, void *d_work, size_t work_bytes, void *stream);

/*
 * qaoa_evolve_batch -- `batch` independent QAOA evaluations against one cost
 * vector (the repeated objective evaluations of an outer optimiser, Section 2
 * and Fig. 1): state s evolves through Algorithm 3 with its own angles.
 *
 *   d_gamma, d_beta  device, row-major [batch][p] doubles; read when the
 *               enqueued work runs (not at call time), so a caller may capture
 *               the call in a HIP graph and replay it after writing new angles
 *               into the same buffers.  Non-finite angles give non-finite results.
 *   d_states    device, [batch][2^n] states of state_dtype (states_bytes);
 *               init = 1 starts every state from |+>^n, init = 0 from its contents
 *   d_out       device, nullable, [batch][2] doubles: (E, sum |psi|^2) per state
 *   sets_per_pass  states advanced together through all layers before the next
 *               group starts (0 = all).  Smaller groups keep their states resident
 *               in the memory-side cache; the result does not depend on it.
 *   d_work      device workspace of qaoa_batch_workspace_bytes(n, p, batch, ...)
 *
 * The same kernels and reduction order as qaoa_evolve are used, so each state's
 * result is bitwise equal to a qaoa_evolve call with its angles.  Enqueues only
 * kernels (no memset, copy or synchronisation), so it can be graph-captured.
 */
int qaoa_evolve_batch(int n, int p, int batch, const double *d_gamma, const double *d_beta,
                      const void *d_diag, int diag_dtype, double diag_offset, size_t diag_bytes,
                      void *d_states, int state_dtype, size_t states_bytes, int init,
                      double *d_out, int sets_per_pass, void *d_work, size_t work_bytes, void *stream);

/* Workspace bytes qaoa_evolve_batch needs for these sizes and dtypes. */
int qaoa_batch_workspace_bytes(int n, int p, int batch, int state_dtype, int diag_dtype, size_t *bytes);

/*
 * qaoa_grad -- E and its gradient with respect to the layer angles, the
 * quantities an outer optimiser needs (Section 2: the angles are chosen to
 * minimise <gamma beta|C|gamma beta>).  Reverse-mode (adjoint) evaluation:
 * one forward pass (Algorithm 3), then the layers are undone in reverse order
 * on the state and on lambda = C psi_p together, accumulating
 *   dE/dbeta_l  = 2 Im <lambda| sum_i X_i |psi>   (at layer l's output)
 *   dE/dgamma_l = 2 Im <lambda| C |psi>           (after undoing layer l's mixer).
 *
 *   n, p        1 <= n <= QAOA_MAX_QUBITS, p >= 1; gamma, beta host arrays of p
 *   d_state     device, 2^n of state_dtype: overwritten (on return it holds the
 *               uncomputed state, |+>^n up to rounding)
 *   d_adj       device, 2^n of state_dtype, a second state buffer (scratch, must
 *               not alias d_state)
 *   d_out       device, 1 + 2p doubles: E, dE/dgamma[0..p), dE/dbeta[0..p)
 *   d_work      device, qaoa_grad_workspace_bytes(n, p, ...) bytes
 * Deterministic (fixed reduction order).  Memory traffic is about three times
 * that of qaoa_evolve.
 */
int qaoa_grad(int n, int p, const double *gamma, const double *beta,
              const void *d_diag, int diag_dtype, double diag_offset, size_t diag_bytes,
              void *d_state, void *d_adj, int state_dtype, size_t state_bytes,
              double *d_out, void *d_work, size_t work_bytes, void *stream);

/* Workspace bytes qaoa_grad needs. */
int qaoa_grad_workspace_bytes(int n, int p, int state_dtype, int diag_dtype, size_t *bytes);

/*
 * Request loop (continuous batching) for an outer optimiser's objective and
 * gradient queries (Section 2 / Fig. 1: the angles are tuned by repeated
 * evaluations).  Cost vectors are precomputed once per problem and stay
 * resident.  A scheduler thread admits queued requests in arrival order as soon
 * as their device footprint (state, second state for gradients, workspace,
 * output) fits the arena and an in-flight slot is free, runs them on a pool of
 * streams so that independent requests overlap on the GPU, and retires them
 * when their completion events fire, freeing memory for later admissions.
 * Results do not depend on the mix: each request owns its buffers and every
 * reduction has a fixed order.  The server allocates its arena (one device
 * allocation), its streams and pinned result slots at creation only.
 */
typedef struct qaoa_server qaoa_server;

typedef struct {
    uint64_t submitted, completed, failed, queued, in_flight;
    uint64_t arena_bytes, peak_bytes;  /* arena size, peak bytes in use */
    double p50_s, p99_s, mean_s, max_s; /* latency submit -> result on the host */
    double busy_s;                      /* first submit -> last completion */
    double requests_per_s;              /* completed / busy_s */
} qaoa_server_stats;

/* arena_bytes >= 1 MiB of device memory for cost vectors and request buffers;
 * 1 <= num_streams <= 64 (default priority); 1 <= max_in_flight <= 4096. */
int qaoa_server_create(size_t arena_bytes, int num_streams, int max_in_flight, qaoa_server **out);
/* Waits for the requests already running on the GPU, fails the ones still
 * queued (never admitted) with QAOA_ERR_INVALID, then releases everything.  No
 * qaoa_server_* call on s may overlap with or follow this one. */
int qaoa_server_destroy(qaoa_server *s);
/* Precompute a problem's cost vector into the arena (synchronous); terms as in
 * qaoa_precompute_diag.  Returns its id in *problem_id. */
int qaoa_server_add_problem(qaoa_server *s, int n, int64_t num_terms, const double *w,
                            const int64_t *term_ptr, const int32_t *term_idx, int diag_dtype,
                            int *problem_id);
/* Queue one request: kind 0 = objective (result E, sum |psi|^2), kind 1 =
 * gradient (result E, dE/dgamma[p], dE/dbeta[p]); 1 <= p <= 256; host angles are
 * copied.  QAOA_ERR_NOMEM if the request could never fit the arena.  Requests
 * take arena space from the bottom and cost vectors from the top; a queued
 * request that finds no contiguous block while no other request is in flight
 * finishes with QAOA_ERR_NOMEM (reported by qaoa_server_wait) instead of
 * blocking the queue. */
int qaoa_server_submit(qaoa_server *s, int problem_id, int kind, int state_dtype, int p,
                       const double *gamma, const double *beta, int64_t *ticket);
/* Block until the request finishes; copies its result (2 or 1 + 2p doubles)
 * into out (out_len doubles) and its latency in seconds.  A ticket can be
 * waited on once. */
int qaoa_server_wait(qaoa_server *s, int64_t ticket, double *out, int out_len, double *latency_s);
int qaoa_server_stats_get(qaoa_server *s, qaoa_server_stats *out);
int qaoa_server_reset_stats(qaoa_server *s);

/*
 * qaoa_evolve_xy -- QAOA with a Hamming-weight-preserving XY mixer (Section 3.2):
 * M = sum over the edges <i,j> of a ring or of the complete graph on the qubits
 * of (X_i X_j + Y_i Y_j)/2.  Each layer applies exp(-i gamma_l C) (Section 3.1),
 * then the product of the exact two-qubit gates exp(-i beta_l (X_i X_j +
 * Y_i Y_j)/2) in a fixed edge order: ring (i, i+1) for even i, then odd i, then
 * (n-1, 0) when n > 2; complete graph (i, j), i < j, lexicographic.  (The paper
 * fixes neither the order of these non-commuting terms nor an initial state.)
 *   mixer      QAOA_MIXER_XY_RING or QAOA_MIXER_XY_COMPLETE; 2 <= n <= 30.
 *   init       QAOA_INIT_GIVEN (d_state holds the start), QAOA_INIT_PLUS (|+>^n),
 *              QAOA_INIT_DICKE (the Dicke state of Hamming weight k, 0 <= k <= n).
 *   other arguments as in qaoa_evolve; d_out (E, sum |psi|^2) may be NULL.
 * Workspace: qaoa_xy_workspace_bytes.  Same stream semantics as qaoa_evolve.
 */
int qaoa_evolve_xy(int n, int p, const double *gamma, const double *beta, int mixer, const void *d_diag,
                   int diag_dtype, double diag_offset, size_t diag_bytes, void *d_state, int state_dtype,
                   size_t state_bytes, int init, int k, double *d_out, void *d_work, size_t work_bytes,
                   void *stream);
int qaoa_xy_workspace_bytes(int n, int mixer, int state_dtype, size_t *bytes);
/* Diagnostic: the XY sweep plan.  Writes [S, EB, single] then per sweep
 * tb, R, hA, qA, qB, ngates and ngates (i, j) tile-bit pairs (the tile-bit
 * mapping as in qaoa_plan_describe).  Returns the count or -QAOA_ERR_INVALID. */
int qaoa_xy_plan_describe(int n, int mixer, int state_dtype, int *out, int cap);

/*
 * qaoa_plan_describe -- diagnostic: the HBM sweep plan used for n qubits.
 * kind 0: qaoa_evolve / qaoa_evolve_batch sweeps for state_dtype;
 * kind 1: the reverse sweeps of qaoa_grad for state_dtype;
 * kind 2: the cost-vector transform for elements of elem_bytes (2, 4 or 8).
 * Writes up to `cap` ints:
 *   [0] number of sweeps S, [1] register bits per thread EB, [2] 1 if the whole
 *   vector is one tile (all layers in one launch), [3] 1 if complex128 tiles
 *   exceed the LDS (up to 2^14 elements, 1024 threads; window changes move real
 *   and imaginary parts separately as 8-byte entries), then per sweep:
 *   tb, R, hA, qA, qB, act_lo, w_store, nchunks, and nchunks triples (w, jlo, jhi).
 * Tile bits [0,R) are global bits [0,R); tile bits [R,R+hA) are global bits
 * [qA,qA+hA); tile bits [R+hA,tb) are global bits [qB,qB+tb-R-hA); tile bits
 * [act_lo,tb) are the sweep's qubits; a chunk butterflies tile bits [w+jlo, w+jhi).
 * Returns the number of ints needed (may exceed cap), or -QAOA_ERR_INVALID.
 */
int qaoa_plan_describe(int kind, int n, int state_dtype, int elem_bytes, int *out, int cap);

/*
 * qaoa_schedule_describe -- diagnostic: the launch order of one evaluation of
 * p layers (Sections 3.1-3.2: each layer is the phase, then one mixer gate per
 * qubit).  The gates of a layer commute, so the sweeps of alternate layers run
 * in reverse order and the sweep that ends a layer also starts the next one on
 * the same qubits.
 * kind 0: qaoa_evolve / qaoa_evolve_batch over the kind-0 plan; `init` and
 *   `reduce` as in qaoa_evolve (reduce = d_out given).  Flags: 1 generate |+>,
 *   2 phase of that layer before its gates, 4 emit (E, norm) partials,
 *   8 fused: then layer+1's phase and its gates on the same qubits.
 * kind 1: the reverse pass of qaoa_grad over the kind-1 plan, layers p-1..0
 *   (init, reduce ignored).  Flags: 1 lambda = c psi formed first, 2 undo of
 *   that layer's phase after its gates, 8 fused: that phase undone, then
 *   layer-1's gates on the same qubits.
 * Writes up to `cap` ints, three per launch: sweep index in the plan, first
 * layer applied, flags.  Returns the number of ints needed (0 when the state is
 * one tile and a single launch runs the layers), or -QAOA_ERR_INVALID.
 */
int qaoa_schedule_describe(int kind, int n, int p, int state_dtype, int init, int reduce, int *out, int cap);

#ifdef __cplusplus
}
#endif

#endif /* QAOA_H */
