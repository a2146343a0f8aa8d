/*
 * oracle.c -- plain FP64 CPU reference for the QAOA hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the GPU path.
 *
 * Everything is computed in IEEE double precision, straight from the
 * definitions in the paper:
 *   - cost vector          Eq. (1) (spin polynomial), Section 2 (MaxCut, LABS)
 *   - QAOA state           Section 2: prod_l exp(-i beta_l M) exp(-i gamma_l C) |+>^n,
 *                          applied as in Algorithm 3 (phase, then mixer, layer 1 first)
 *   - mixer                Section 3.2: exp(-i beta sum_i X_i) = prod_i (cos b I - i sin b X_i)
 *   - objective            Section 3.1: E = sum_x |psi_x|^2 c_x
 *   - XY mixers            Section 3.2: M = sum_<ij> (X_i X_j + Y_i Y_j)/2 over the edges
 *                          of a ring or a complete graph; one mixer layer is the
 *                          product of the exact two-qubit exponentials
 *                          exp(-i beta (X_i X_j + Y_i Y_j)/2) in a fixed edge order
 *   - gradient             dE/dgamma_l, dE/dbeta_l of that objective (the parameters
 *                          an outer optimiser varies, Section 2), by reverse-mode
 *                          (adjoint) differentiation of Algorithm 3
 *
 * Conventions (readings of the paper, see the design notes):
 *   - variable i <-> bit i of the basis index x (0-based), spin s_i = 1 - 2*bit_i(x);
 *   - the mixer gate on qubit i is cos(beta) I - i sin(beta) X_i (Section 3.2),
 *     i.e. off-diagonal entry b = -i sin(beta) in Algorithm 1's matrix form;
 *   - E is not renormalised; the squared norm is returned beside it.
 *
 * OpenMP is used on outer loops over basis states only; each output element is
 * produced by exactly the same arithmetic as in a serial run.  Sums over basis
 * states are either serial (the compensated objective) or split into a fixed
 * number of index ranges whose partial sums are added in range order (the
 * gradient's inner products), so no result depends on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline double spin(uint64_t x, int i) { return ((x >> i) & 1u) ? -1.0 : 1.0; }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Eq. (1): f(s) = sum_k w_k prod_{i in t_k} s_i, evaluated term by term with
 * explicit spin products (no parity tricks).  Term k owns idx[ptr[k]..ptr[k+1]). */
void oracle_diag_terms(int n, int64_t L, const double *w, const int64_t *ptr,
                       const int32_t *idx, double *c)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double f = 0.0;
        for (int64_t k = 0; k < L; ++k) {
            double term = w[k];
            for (int64_t j = ptr[k]; j < ptr[k + 1]; ++j)
                term *= spin((uint64_t)x, idx[j]);
            f += term;
        }
        c[x] = f;
    }
}

/* LABS, direct definition, at one basis state x:
 * c(s) = sum_{k=1}^{n-1} C_k^2, C_k = sum_{i=0}^{n-k-1} s_i s_{i+k}.
 * s_i s_{i+k} is +1 where bits i and i+k agree and -1 where they differ, so
 * C_k = (n - k) - 2 * #{i < n-k : bit_i(x) != bit_{i+k}(x)}, the count being the
 * population count of (x XOR x >> k) restricted to its low n - k bits (the
 * XOR / population-count evaluation of spin products of Section 3.1).
 * Integer arithmetic, exact. */
static int64_t labs_energy(int n, int64_t x)
{
    int64_t e = 0;
    for (int k = 1; k < n; ++k) {
        const uint64_t low = ((uint64_t)1 << (n - k)) - 1;
        const uint64_t differ = ((uint64_t)x ^ ((uint64_t)x >> k)) & low;
        const int64_t ck = (int64_t)(n - k) - 2 * (int64_t)__builtin_popcountll(differ);
        e += ck * ck;
    }
    return e;
}

/* LABS for every basis state. */
void oracle_diag_labs(int n, int64_t *c)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) c[x] = labs_energy(n, x);
}

/* LABS at selected basis states only, for sampled checks at sizes where the
 * full vector is too large to enumerate. */
void oracle_diag_labs_at(int n, int64_t m, const int64_t *xs, int64_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) out[j] = labs_energy(n, xs[j]);
}

/* Weighted MaxCut, direct definition in minimisation form (Section 2):
 * c(x) = - sum_{(u,v) in E} w_uv [bit_u(x) != bit_v(x)]. */
void oracle_diag_maxcut(int n, int64_t m, const int32_t *edges, const double *w, double *c)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double cut = 0.0;
        for (int64_t e = 0; e < m; ++e) {
            int u = edges[2 * e], v = edges[2 * e + 1];
            if (((x >> u) & 1) != ((x >> v) & 1)) cut += w[e];
        }
        c[x] = -cut;
    }
}

/* |+>^n: every amplitude 2^{-n/2}. psi is interleaved (re, im). */
void oracle_plus_state(int n, double *psi)
{
    const int64_t N = (int64_t)1 << n;
    const double a = pow(2.0, -0.5 * n);
    for (int64_t x = 0; x < N; ++x) { psi[2 * x] = a; psi[2 * x + 1] = 0.0; }
}

/* Phase operator (Section 3.1): psi_x <- exp(-i gamma c_x) psi_x, angle = gamma * c_x. */
void oracle_apply_phase(int n, const double *c, double gamma, double *psi)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double th = gamma * c[x];
        double cr = cos(th), ci = -sin(th);
        double r = psi[2 * x], i = psi[2 * x + 1];
        psi[2 * x] = cr * r - ci * i;
        psi[2 * x + 1] = cr * i + ci * r;
    }
}

/* One mixer gate exp(-i beta X_q) = cos(beta) I - i sin(beta) X_q (Section 3.2) on
 * qubit q: every basis state x with bit q clear is paired with x | 2^q and the
 * 2x2 matrix [[cos b, -i sin b], [-i sin b, cos b]] acts on the pair
 * (the single-qubit update of Algorithm 1). */
void oracle_apply_rx(int n, int q, double beta, double *psi)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t bit = (int64_t)1 << q;
    const double a = cos(beta), s = sin(beta);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        if (x & bit) continue;
        int64_t y = x | bit;
        double r0 = psi[2 * x], i0 = psi[2 * x + 1];
        double r1 = psi[2 * y], i1 = psi[2 * y + 1];
        /* u0 = a*y0 - i s*y1 ; u1 = -i s*y0 + a*y1 */
        psi[2 * x] = a * r0 + s * i1;
        psi[2 * x + 1] = a * i0 - s * r1;
        psi[2 * y] = a * r1 + s * i0;
        psi[2 * y + 1] = a * i1 - s * r0;
    }
}

/* Full transverse-field mixer: the gate above on every qubit (Algorithm 2). */
void oracle_apply_mixer(int n, double beta, double *psi)
{
    for (int q = 0; q < n; ++q) oracle_apply_rx(n, q, beta, psi);
}

/* Algorithm 3: optional |+>^n start, then for l = 1..p the phase with gamma_l
 * followed by the mixer with beta_l. */
void oracle_qaoa_evolve(int n, int p, const double *c, const double *gamma,
                        const double *beta, int init, double *psi)
{
    if (init) oracle_plus_state(n, psi);
    for (int l = 0; l < p; ++l) {
        oracle_apply_phase(n, c, gamma[l], psi);
        oracle_apply_mixer(n, beta[l], psi);
    }
}

/* ---------------------------------------------------------------------------
 * XY mixers (Section 3.2).  (X_i X_j + Y_i Y_j)/2 maps |01> <-> |10> on the
 * qubit pair (i, j) and annihilates |00> and |11>, so exp(-i beta (XX+YY)/2)
 * is the identity on |00>, |11> and the matrix [[cos b, -i sin b],
 * [-i sin b, cos b]] on the pair of amplitudes (x with bit i = 0, bit j = 1;
 * the same x with the two bits exchanged).
 * Edge orders (the paper does not fix them; these are the readings used):
 *   ring:     (i, i+1) for even i, then for odd i (i + 1 < n), then the wrap
 *             edge (n-1, 0) when n > 2;
 *   complete: (i, j), i < j, in lexicographic order.
 * ------------------------------------------------------------------------- */
void oracle_apply_xy(int n, int i, int j, double beta, double *psi)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t bi = (int64_t)1 << i, bj = (int64_t)1 << j;
    const double a = cos(beta), s = sin(beta);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        if ((x & bi) || !(x & bj)) continue;      /* x: bit i = 0, bit j = 1 */
        int64_t y = (x | bi) & ~bj;               /* y: bit i = 1, bit j = 0 */
        double r0 = psi[2 * x], i0 = psi[2 * x + 1];
        double r1 = psi[2 * y], i1 = psi[2 * y + 1];
        psi[2 * x] = a * r0 + s * i1;
        psi[2 * x + 1] = a * i0 - s * r1;
        psi[2 * y] = a * r1 + s * i0;
        psi[2 * y + 1] = a * i1 - s * r0;
    }
}

/* Edge list of one XY mixer layer in application order: kind 1 = ring,
 * kind 2 = complete.  Writes pairs into edges[2 * m], returns the count. */
int oracle_xy_edges(int n, int kind, int32_t *edges)
{
    int m = 0;
    if (kind == 1) {
        for (int par = 0; par < 2; ++par)
            for (int i = par; i + 1 < n; i += 2) { edges[2 * m] = i; edges[2 * m + 1] = i + 1; ++m; }
        if (n > 2) { edges[2 * m] = n - 1; edges[2 * m + 1] = 0; ++m; }
    } else if (kind == 2) {
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) { edges[2 * m] = i; edges[2 * m + 1] = j; ++m; }
    }
    return m;
}

void oracle_apply_xy_mixer(int n, int kind, double beta, double *psi)
{
    int32_t *edges = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)n + 8);
    const int m = oracle_xy_edges(n, kind, edges);
    for (int e = 0; e < m; ++e) oracle_apply_xy(n, edges[2 * e], edges[2 * e + 1], beta, psi);
    free(edges);
}

/* Dicke state |D^n_k>: equal amplitude C(n,k)^{-1/2} on every x of Hamming
 * weight k, zero elsewhere. */
void oracle_dicke_state(int n, int k, double *psi)
{
    const int64_t N = (int64_t)1 << n;
    double cnk = 1.0;
    for (int t = 1; t <= k; ++t) cnk = cnk * (double)(n - k + t) / (double)t;
    const double a = 1.0 / sqrt(cnk);
    for (int64_t x = 0; x < N; ++x) {
        psi[2 * x] = (__builtin_popcountll((unsigned long long)x) == k) ? a : 0.0;
        psi[2 * x + 1] = 0.0;
    }
}

/* QAOA with an XY mixer: start (init 0: given psi; 1: |+>^n; 2: Dicke |D^n_k>),
 * then for each layer the phase and the XY mixer layer. */
void oracle_qaoa_evolve_xy(int n, int p, const double *c, const double *gamma, const double *beta, int kind,
                           int init, int k, double *psi)
{
    if (init == 1) oracle_plus_state(n, psi);
    if (init == 2) oracle_dicke_state(n, k, psi);
    for (int l = 0; l < p; ++l) {
        oracle_apply_phase(n, c, gamma[l], psi);
        oracle_apply_xy_mixer(n, kind, beta[l], psi);
    }
}

/* Neumaier-compensated summation step. */
static inline void neumaier_add(double *sum, double *comp, double v)
{
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v)) *comp += (*sum - t) + v;
    else *comp += (v - t) + *sum;
    *sum = t;
}

/* Objective (Section 3.1): out[0] = sum_x |psi_x|^2 c_x, out[1] = sum_x |psi_x|^2,
 * both with compensated summation in index order. */
void oracle_expectation(int n, const double *psi, const double *c, double *out)
{
    const int64_t N = (int64_t)1 << n;
    double e = 0.0, ec = 0.0, q = 0.0, qc = 0.0;
    for (int64_t x = 0; x < N; ++x) {
        double pr = psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
        neumaier_add(&e, &ec, pr * c[x]);
        neumaier_add(&q, &qc, pr);
    }
    out[0] = e + ec;
    out[1] = q + qc;
}

/* Index ranges of the gradient's inner products: the sum over x is split into
 * GRAD_RANGES equal ranges, each summed in index order, and the range sums are
 * added in range order, whatever the number of threads. */
#define GRAD_RANGES 256

/* sum_x Im(conj(lam_x) psi_{x ^ flip}) * (c ? c_x : 1) */
static double im_inner(int64_t N, const double *lam, const double *psi, int64_t flip, const double *c)
{
    double part[GRAD_RANGES];
    const int64_t len = (N + GRAD_RANGES - 1) / GRAD_RANGES;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < GRAD_RANGES; ++r) {
        const int64_t lo = (int64_t)r * len;
        const int64_t hi = lo + len < N ? lo + len : N;
        double s = 0.0;
        for (int64_t x = lo; x < hi; ++x) {
            const int64_t y = x ^ flip;
            const double v = lam[2 * x] * psi[2 * y + 1] - lam[2 * x + 1] * psi[2 * y];
            s += c ? c[x] * v : v;
        }
        part[r] = s;
    }
    double total = 0.0;
    for (int r = 0; r < GRAD_RANGES; ++r) total += part[r];
    return total;
}

/* Gradient of E = <psi_p|C|psi_p> with respect to gamma[0..p) and beta[0..p),
 * by the adjoint method (exact up to rounding):
 *   lambda = C psi_p; for l = p..1:
 *     dE/dbeta_l  = 2 Im <lambda| sum_i X_i |psi>        (psi, lambda after layer l)
 *     undo the mixer of layer l on psi and lambda (gate with -beta_l)
 *     dE/dgamma_l = 2 Im <lambda| C |psi>
 *     undo the phase of layer l on psi and lambda (angle -gamma_l)
 * out[0] = E, out[1 + l] = dE/dgamma_l, out[1 + p + l] = dE/dbeta_l.
 * work: 4 * 2^n doubles (two states). */
void oracle_qaoa_grad(int n, int p, const double *c, const double *gamma, const double *beta,
                      double *out, double *work)
{
    const int64_t N = (int64_t)1 << n;
    double *psi = work, *lam = work + 2 * N;
    double eo[2];
    oracle_qaoa_evolve(n, p, c, gamma, beta, 1, psi);
    oracle_expectation(n, psi, c, eo);
    out[0] = eo[0];
    for (int64_t x = 0; x < N; ++x) {
        lam[2 * x] = c[x] * psi[2 * x];
        lam[2 * x + 1] = c[x] * psi[2 * x + 1];
    }
    for (int l = p - 1; l >= 0; --l) {
        double sb = 0.0;
        for (int q = 0; q < n; ++q) sb += im_inner(N, lam, psi, (int64_t)1 << q, NULL);
        out[1 + p + l] = 2.0 * sb;
        oracle_apply_mixer(n, -beta[l], psi);
        oracle_apply_mixer(n, -beta[l], lam);
        out[1 + l] = 2.0 * im_inner(N, lam, psi, 0, c);
        oracle_apply_phase(n, c, -gamma[l], psi);
        oracle_apply_phase(n, c, -gamma[l], lam);
    }
}
