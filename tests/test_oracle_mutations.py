"""The oracle's pins reject plausible mistakes.

Each case plants one mistake in a private copy of the oracle's C source
(a flipped sign, a dropped neighbour or bond, a transposed index, a wrong RNG
word or constant), builds it on the CPU, and checks that the fast pins of
test_oracle_rng / test_oracle_updates / test_oracle_physics / test_oracle_chain
fail against it.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC_PATH = os.path.join(ROOT, "oracle", "xy_oracle.c")

MUTATIONS = {
    "metropolis_dE_sign": ("dE += cos(th_old - thj) - cos(th_new - thj);",
                           "dE += cos(th_new - thj) - cos(th_old - thj);"),
    "metropolis_drops_a_neighbour": ("for (int n = 0; n < 6; ++n) {\n        double thj",
                                     "for (int n = 0; n < 5; ++n) {\n        double thj"),
    "metropolis_half_beta": ("if (u < exp(-beta * dE)) {", "if (u < exp(-0.5 * beta * dE)) {"),
    "or_factor_one": ("double f = 2.0 * (Sx * Hx + Sy * Hy) / H2;",
                      "double f = 1.0 * (Sx * Hx + Sy * Hy) / H2;"),
    "or_sign": ("double Sx_new = -Sx + f * Hx;", "double Sx_new = Sx + f * Hx;"),
    "or_field_drops_a_term": ("Hy -= sin(theta[nb[n]]);", "Hy -= sin(theta[nb[n]]) * (n < 5);"),
    "energy_drops_z_bonds": ("nsum_add(&E, -cos(th - theta[nb[5]]));", ""),
    "magnetisation_uses_sin": ("nsum_add(&Mx, cos(th));", "nsum_add(&Mx, sin(th));"),
    "exchange_sign": ("double w = exp((beta[k] - beta[k + 1]) * (E[k] - E[k + 1]));",
                      "double w = exp((beta[k] - beta[k + 1]) * (E[k + 1] - E[k]));"),
    "exchange_parity": ("for (int k = (int)(tau & 1u); k + 1 < R; k += 2) {",
                        "for (int k = 0; k + 1 < R; k += 2) {"),
    "neighbour_z_plus": ("int zm = (z + L - 1) % L, zp = (z + 1) % L;",
                         "int zm = (z + L - 1) % L, zp = z;"),
    "neighbour_transposed": ("nb[2] = x + (int64_t)L * ym + LL * z;",
                             "nb[2] = xm + (int64_t)L * y + LL * z;"),
    "philox_hi_lo": ("uint32_t n1 = (uint32_t)p1;", "uint32_t n1 = (uint32_t)(p1 >> 32);"),
    "philox_key_bump": ("k1 += W1;", "k1 += W0;"),
    "uniform_shift": ("return (double)(r >> 8) * (1.0 / 16777216.0);",
                      "return (double)(r >> 9) * (1.0 / 16777216.0);"),
    "metro_odd_plane_takes_words_0_1": ("uint32_t wa = r[2 * odd], wb = r[2 * odd + 1];",
                                        "uint32_t wa = r[0], wb = r[1];"),
    "metro_pair_partner_keeps_x": ("int64_t i0 = odd ? (int64_t)(x ^ 1) + ",
                                   "int64_t i0 = odd ? (int64_t)x + "),
    "init_uses_word_1": ("theta[(int64_t)k * N + i] = TWO_PI * orc_uniform(r[0]);",
                         "theta[(int64_t)k * N + i] = TWO_PI * orc_uniform(r[1]);"),
    "margin_half_beta": ("margin[i] = u - exp(-beta * dE);", "margin[i] = u - exp(-0.5 * beta * dE);"),
    "margin_wrong_colour": ("if (((x + y + z) & 1) != colour) {\n                    margin[i] = NAN;",
                            "if (((x + y + z) & 1) == colour) {\n                    margin[i] = NAN;"),
    # the multi-replica chain (Sec. II, Monte Carlo step; Eq. (3))
    "sweep_uses_beta_0_for_every_position": (
        "acc += orc_metro_half(th, L, beta[k], seed, t, lat, k, s, window, c);",
        "acc += orc_metro_half(th, L, beta[0], seed, t, lat, k, s, window, c);"),
    "run_exchanges_before_measuring": (
        """        for (int k = 0; k < R; ++k) {
            double o[5];
            orc_measure(theta + (int64_t)k * N, L, o);
            E[k] = o[0];
            if (obs) memcpy(obs + ((int64_t)s * R + k) * 5, o, sizeof(o));
        }
        if (exchange_every > 0 && (s + 1) % exchange_every == 0) {
            orc_exchange(theta, E, L, R, beta, seed, tau, lat, n_swap_acc);
            ++tau;
        }""",
        """        for (int k = 0; k < R; ++k) {
            double o[5];
            orc_measure(theta + (int64_t)k * N, L, o);
            E[k] = o[0];
        }
        if (exchange_every > 0 && (s + 1) % exchange_every == 0) {
            orc_exchange(theta, E, L, R, beta, seed, tau, lat, n_swap_acc);
            ++tau;
        }
        for (int k = 0; k < R; ++k) {
            double o[5];
            orc_measure(theta + (int64_t)k * N, L, o);
            if (obs) memcpy(obs + ((int64_t)s * R + k) * 5, o, sizeof(o));
        }"""),
    "run_exchange_cadence_off_by_one": ("if (exchange_every > 0 && (s + 1) % exchange_every == 0) {",
                                        "if (exchange_every > 0 && s % exchange_every == 0) {"),
    "exchange_counts_the_next_pair": ("if (n_acc) n_acc[k] += 1;", "if (n_acc) n_acc[k + 1] += 1;"),
    "run_sweep_counter_frozen": ("uint32_t t = t0 + (uint32_t)s;", "uint32_t t = t0;"),
    "run_exchange_counter_frozen": ("            orc_exchange(theta, E, L, R, beta, seed, tau, lat, n_swap_acc);\n            ++tau;",
                                    "            orc_exchange(theta, E, L, R, beta, seed, tau, lat, n_swap_acc);"),
    "exchange_swaps_energies_only": ("                    a[i] = b[i];\n                    b[i] = tmp;",
                                     "                    (void)tmp;"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_mutation(name, tmp_path):
    src = open(SRC_PATH).read()
    a, b = MUTATIONS[name]
    assert a in src, "mutation anchor no longer present in the oracle source"
    (tmp_path / "xy_oracle.c").write_text(src.replace(a, b))
    (tmp_path / "xy_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "xy_oracle.h")).read())
    lib = str(tmp_path / "libmut.so")
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", lib,
                           str(tmp_path / "xy_oracle.c"), "-lm"])
    env = dict(os.environ, XY_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not slow", "tests/test_oracle_rng.py",
                        "tests/test_oracle_updates.py", "tests/test_oracle_physics.py",
                        "tests/test_oracle_chain.py"],
                       env=env, capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 1, r.stdout[-2000:]
