"""Planted mistakes: each mutant of oracle.c must fail at least one pin.

A mutated copy of the oracle source is compiled into a temporary library,
swapped in for the real one, and the pin tests are run against it.  This shows
that the pins can tell a plausible slip (a sign, a dropped term, a wrong index,
a transposed convention) from the correct oracle.
"""
import os
import subprocess

import pytest

import oracle
import test_oracle_diag as D
import test_oracle_evolve as V
import test_oracle_grad as G
import test_oracle_xy as XY

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    # Algorithm 3 read literally (b = sin beta): a Y rotation instead of exp(-i beta X)
    "mixer_is_y_rotation": (
        "psi[2 * x] = a * r0 + s * i1;\n        psi[2 * x + 1] = a * i0 - s * r1;\n"
        "        psi[2 * y] = a * r1 + s * i0;\n        psi[2 * y + 1] = a * i1 - s * r0;",
        "psi[2 * x] = a * r0 - s * r1;\n        psi[2 * x + 1] = a * i0 - s * i1;\n"
        "        psi[2 * y] = a * r1 + s * r0;\n        psi[2 * y + 1] = a * i1 + s * i0;"),
    "phase_sign": ("double cr = cos(th), ci = -sin(th);", "double cr = cos(th), ci = sin(th);"),
    "mixer_skips_top_qubit": ("for (int q = 0; q < n; ++q) oracle_apply_rx",
                              "for (int q = 0; q + 1 < n; ++q) oracle_apply_rx"),
    "labs_drops_last_product": ("const uint64_t low = ((uint64_t)1 << (n - k)) - 1;",
                                "const uint64_t low = ((uint64_t)1 << (n - k - 1)) - 1;"),
    "labs_lag_count_off_by_one": ("const int64_t ck = (int64_t)(n - k) - 2", "const int64_t ck = (int64_t)(n - k + 1) - 2"),
    "spin_wrong_bit": ("return ((x >> i) & 1u) ? -1.0 : 1.0;", "return ((x >> (i ^ 1)) & 1u) ? -1.0 : 1.0;"),
    "maxcut_sign": ("c[x] = -cut;", "c[x] = cut;"),
    "phase_before_is_after": (
        "oracle_apply_phase(n, c, gamma[l], psi);\n        oracle_apply_mixer(n, beta[l], psi);",
        "oracle_apply_mixer(n, beta[l], psi);\n        oracle_apply_phase(n, c, gamma[l], psi);"),
    "plus_state_unnormalised": ("const double a = pow(2.0, -0.5 * n);", "const double a = pow(2.0, -0.5 * (n - 1));"),
    # adjoint: gamma term taken before the mixer is undone
    "grad_gamma_before_mixer_undo": (
        "        oracle_apply_mixer(n, -beta[l], psi);\n        oracle_apply_mixer(n, -beta[l], lam);\n"
        "        out[1 + l] = 2.0 * im_inner(N, lam, psi, 0, c);",
        "        out[1 + l] = 2.0 * im_inner(N, lam, psi, 0, c);\n"
        "        oracle_apply_mixer(n, -beta[l], psi);\n        oracle_apply_mixer(n, -beta[l], lam);"),
    # XY gate pairs x with bit j set but forgets to clear it in the partner
    "xy_partner_keeps_bit_j": ("int64_t y = (x | bi) & ~bj;               /* y: bit i = 1, bit j = 0 */",
                               "int64_t y = (x | bi);                     /* y: bit i = 1, bit j = 0 */"),
    # ring order: odd edges before even edges
    "xy_ring_parity_order": ("for (int par = 0; par < 2; ++par)", "for (int par = 1; par >= 0; --par)"),
    "xy_complete_reverse_order": ("for (int j = i + 1; j < n; ++j) { edges[2 * m] = i;",
                                  "for (int j = n - 1; j > i; --j) { edges[2 * m] = i;"),
    "dicke_wrong_weight": ("psi[2 * x] = (__builtin_popcountll((unsigned long long)x) == k) ? a : 0.0;",
                           "psi[2 * x] = (__builtin_popcountll((unsigned long long)x) == k + 1) ? a : 0.0;"),
    # adjoint: conjugation on the wrong factor (sign of the beta term)
    "grad_beta_conjugate": ("sb += im_inner(N, lam, psi, (int64_t)1 << q, NULL);",
                            "sb -= im_inner(N, lam, psi, (int64_t)1 << q, NULL);"),
    # adjoint: inner product pairs x with itself instead of its partner x ^ 2^q
    "grad_beta_no_flip": ("const int64_t y = x ^ flip;", "const int64_t y = x;"),
    # sampled LABS entry point off by one lag
    "labs_at_wrong_lag": ("for (int64_t j = 0; j < m; ++j) out[j] = labs_energy(n, xs[j]);",
                          "for (int64_t j = 0; j < m; ++j) out[j] = labs_energy(n - 1, xs[j]);"),
}

PINS = [
    lambda: [D.test_labs_direct_equals_term_expansion(n) for n in (5, 8)],
    lambda: D.test_labs_closed_forms(9),
    D.test_labs_barker_golden,
    D.test_maxcut_golden_graphs,
    D.test_spin_convention_odd_term,
    lambda: V.test_evolve_matches_dense_expm("random", 5, 3),
    lambda: V.test_evolve_matches_dense_expm("labs", 6, 2),
    lambda: V.test_p1_maxcut_closed_form(V._k4),
    lambda: V.test_norm_preserved_and_beta_zero_mean(4),
    lambda: G.test_grad_matches_central_differences(5, 3, 1),
    G.test_p1_maxcut_gradient_closed_form,
    lambda: XY.test_xy_layer_matches_dense_expm(5, oracle.XY_RING, XY.ring_order),
    lambda: XY.test_xy_layer_matches_dense_expm(4, oracle.XY_COMPLETE, XY.complete_order),
    lambda: XY.test_dicke_state(6, 3),
    lambda: D.test_labs_at_equals_full_vector(9),
    lambda: D.test_labs_at_against_numpy_autocorrelation(26),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found for {name}"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", str(mut), "-o", str(so), "-lm"])
    monkeypatch.setattr(oracle, "_lib", None)
    monkeypatch.setattr(oracle, "_LIB", str(so))
    oracle._load()
    failures = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failures += 1
    monkeypatch.setattr(oracle, "_lib", None)
    assert failures > 0, f"no pin caught mutant {name}"


def test_unmutated_oracle_passes_all_pins():
    for pin in PINS:
        pin()
