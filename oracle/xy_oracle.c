/*
 * Plain CPU FP64 oracle for the 3D XY model Monte Carlo hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library: every step below is written out again
 * from the paper (Lan, Hsieh, Kao, "High-precision Monte Carlo study of the
 * three-dimensional XY model on GPU", arXiv:1211.0780) and from the published
 * definition of Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
 *
 * It is deliberately slow and literal: double precision everywhere, libm for
 * every transcendental, site loops in plain lexicographic order, energies
 * evaluated as sums of cos(theta_i - theta_j) exactly as the Hamiltonian of
 * Eq. (1) is written, and the over-relaxation move evaluated in the vector
 * form of Eq. (2).
 *
 * Conventions (the readings where the paper is silent are listed with the
 * design notes of the repository):
 *   site index    i = x + L*(y + L*z), 0 <= x,y,z < L, periodic (Sec. II)
 *   colour        (x + y + z) mod 2; colour 0 ("black") is updated first
 *   angles        radians in [0, 2*pi), one array of N = L^3 per configuration
 *   configuration k of a lattice is the one at beta-position k (ladder index)
 *   RNG           Philox4x32-10, key = (seed mod 2^32, seed >> 32),
 *                 counter = (c0, c1, c2, c3) as documented per call below
 *   uniform       U(r) = (r >> 8) * 2^-24, in [0, 1 - 2^-24]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "xy_oracle.h"

static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------------
 * Philox4x32-10, from its published definition.  One round maps the counter
 * (c0, c1, c2, c3) with key (k0, k1) to
 *     (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
 * where hi/lo are the halves of the exact 64-bit product; between rounds the
 * key is advanced by the Weyl constants (W0, W1).  Ten rounds.
 * ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_uniform(uint32_t r)
{
    return (double)(r >> 8) * (1.0 / 16777216.0);
}

/* Draw the four words for one (site/pair, sweep, lattice/position, phase). */
static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t lat, uint32_t pos,
                 uint32_t phase, uint32_t substep, uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {c0, c1, (lat << 16) | pos, (phase << 24) | substep};
    orc_philox4x32_10(ctr, key, out);
}

/* Wrap an angle into [0, 2*pi). */
static double wrap_angle(double a)
{
    double r = fmod(a, TWO_PI);
    if (r < 0.0) r += TWO_PI;
    if (r >= TWO_PI) r = 0.0;
    return r;
}

/* The six nearest neighbours of site (x, y, z) under periodic boundaries. */
static void neighbours(int L, int x, int y, int z, int64_t nb[6])
{
    int xm = (x + L - 1) % L, xp = (x + 1) % L;
    int ym = (y + L - 1) % L, yp = (y + 1) % L;
    int zm = (z + L - 1) % L, zp = (z + 1) % L;
    int64_t LL = (int64_t)L * L;
    nb[0] = xm + (int64_t)L * y + LL * z;
    nb[1] = xp + (int64_t)L * y + LL * z;
    nb[2] = x + (int64_t)L * ym + LL * z;
    nb[3] = x + (int64_t)L * yp + LL * z;
    nb[4] = x + (int64_t)L * y + LL * zm;
    nb[5] = x + (int64_t)L * y + LL * zp;
}

/* ------------------------------------------------------------------------
 * Random start: theta = 2*pi*U(r0) with counter
 * (i, 0, (lat << 16) | k, INIT << 24).
 * ------------------------------------------------------------------------ */
void orc_init(double *theta, int L, int R, int lat, uint64_t seed)
{
    int64_t N = (int64_t)L * L * L;
    for (int k = 0; k < R; ++k)
        for (int64_t i = 0; i < N; ++i) {
            uint32_t r[4];
            draw(seed, (uint32_t)i, 0u, (uint32_t)lat, (uint32_t)k, ORC_PHASE_INIT, 0u, r);
            theta[(int64_t)k * N + i] = TWO_PI * orc_uniform(r[0]);
        }
}

/* ------------------------------------------------------------------------
 * Metropolis update of one site i, and the half-sweep over the sites of one
 * colour (Sec. II: checkerboard decomposition, all black sites, then all
 * white sites), which applies it to every site of that colour in increasing
 * i.  Random words: the same-colour sites (x, y, 2m) and (x xor 1, y, 2m+1)
 * share one Philox block
 *     r = Philox(i0, t, (lat << 16) | k, (METRO << 24) | substep),
 * i0 the natural index of the even-plane site; the even-plane site takes
 * (a, b) = (r0, r1), the odd-plane site (a, b) = (r2, r3).  Then
 *     proposal   theta' = 2*pi*U(a)         (uniform on the circle), or, with a
 *                window w > 0, theta' = wrap(theta + w (U(a) - 1/2)) (symmetric)
 *     dE         = H(theta') - H(theta), evaluated from Eq. (1) over the six
 *                  bonds of site i:  sum_j [cos(theta - theta_j) - cos(theta' - theta_j)]
 *     accept iff U(b) < exp(-beta * dE)
 * The site update returns 1 if accepted; the half-sweep returns the count.
 * ------------------------------------------------------------------------ */
/* Proposal theta', acceptance uniform u and dE of the move of site i. */
static void metro_eval(const double *theta, int L, uint64_t seed, uint32_t t, int lat, int k,
                       int substep, double window, int64_t i, double *th_prop, double *u_acc,
                       double *dE_out)
{
    int x = (int)(i % L), y = (int)((i / L) % L), z = (int)(i / ((int64_t)L * L));
    int64_t nb[6];
    neighbours(L, x, y, z, nb);
    int odd = z & 1;
    int64_t i0 = odd ? (int64_t)(x ^ 1) + (int64_t)L * (y + (int64_t)L * (z - 1)) : i;
    uint32_t r[4];
    draw(seed, (uint32_t)i0, t, (uint32_t)lat, (uint32_t)k, ORC_PHASE_METRO, (uint32_t)substep, r);
    uint32_t wa = r[2 * odd], wb = r[2 * odd + 1];
    double th_old = theta[i];
    double th_new = window > 0.0 ? wrap_angle(th_old + window * (orc_uniform(wa) - 0.5))
                                 : TWO_PI * orc_uniform(wa);
    double dE = 0.0;
    for (int n = 0; n < 6; ++n) {
        double thj = theta[nb[n]];
        dE += cos(th_old - thj) - cos(th_new - thj);
    }
    *th_prop = th_new;
    *u_acc = orc_uniform(wb);
    *dE_out = dE;
}

int orc_metro_site(double *theta, int L, double beta, uint64_t seed, uint32_t t, int lat,
                   int k, int substep, double window, int64_t i)
{
    double th_new, u, dE;
    metro_eval(theta, L, seed, t, lat, k, substep, window, i, &th_new, &u, &dE);
    if (u < exp(-beta * dE)) {
        theta[i] = th_new;
        return 1;
    }
    return 0;
}

int64_t orc_metro_half(double *theta, int L, double beta, uint64_t seed, uint32_t t,
                       int lat, int k, int substep, double window, int colour)
{
    int64_t accepted = 0;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                if (((x + y + z) & 1) != colour) continue;
                int64_t i = x + (int64_t)L * (y + (int64_t)L * z);
                accepted += orc_metro_site(theta, L, beta, seed, t, lat, k, substep, window, i);
            }
    return accepted;
}

/* ------------------------------------------------------------------------
 * Decision margins of one Metropolis half-sweep: for every site i of the
 * given colour, margin[i] = U(b) - exp(-beta * dE) with the draws and the dE
 * of orc_metro_site, evaluated on theta as given (sites of one colour do not
 * interact, so every decision of the half-sweep sees exactly this
 * configuration; Sec. II, checkerboard decomposition).  The move is taken
 * iff margin < 0.  Sites of the other colour get NaN.  theta is unchanged.
 * Used to tell a decision that two correct evaluations may take differently
 * (|margin| near rounding) from a wrong one.
 * ------------------------------------------------------------------------ */
void orc_metro_margin(const double *theta, int L, double beta, uint64_t seed, uint32_t t,
                      int lat, int k, int substep, double window, int colour, double *margin)
{
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int64_t i = x + (int64_t)L * (y + (int64_t)L * z);
                if (((x + y + z) & 1) != colour) {
                    margin[i] = NAN;
                    continue;
                }
                double th_new, u, dE;
                metro_eval(theta, L, seed, t, lat, k, substep, window, i, &th_new, &u, &dE);
                margin[i] = u - exp(-beta * dE);
            }
}

/* ------------------------------------------------------------------------
 * Over-relaxation of one site i, and the half-sweep applying it to every
 * site of one colour, Eq. (2):
 *     H_i  = - sum_j S_j                      (local molecular field)
 *     S_i' = - S_i + 2 (S_i . H_i / H_i^2) H_i
 * with S = (cos theta, sin theta); the new angle is the polar angle of S_i'.
 * Where H_i is exactly zero the reflection is undefined and the spin is left
 * unchanged.
 * ------------------------------------------------------------------------ */
void orc_or_site(double *theta, int L, int64_t i)
{
    int x = (int)(i % L), y = (int)((i / L) % L), z = (int)(i / ((int64_t)L * L));
    int64_t nb[6];
    neighbours(L, x, y, z, nb);
    double Hx = 0.0, Hy = 0.0;
    for (int n = 0; n < 6; ++n) {
        Hx -= cos(theta[nb[n]]);
        Hy -= sin(theta[nb[n]]);
    }
    double H2 = Hx * Hx + Hy * Hy;
    if (H2 == 0.0) return;
    double Sx = cos(theta[i]), Sy = sin(theta[i]);
    double f = 2.0 * (Sx * Hx + Sy * Hy) / H2;
    double Sx_new = -Sx + f * Hx;
    double Sy_new = -Sy + f * Hy;
    theta[i] = wrap_angle(atan2(Sy_new, Sx_new));
}

void orc_or_half(double *theta, int L, int colour)
{
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                if (((x + y + z) & 1) != colour) continue;
                orc_or_site(theta, L, x + (int64_t)L * (y + (int64_t)L * z));
            }
}

/* ------------------------------------------------------------------------
 * One sweep of every configuration of one lattice (Sec. II, definition of
 * the Monte Carlo step, generalised to n_metro Metropolis and n_or
 * over-relaxation sweeps): for each beta-position k,
 *   n_metro Metropolis substeps (colour 0 then colour 1 each), then
 *   n_or over-relaxation substeps (colour 0 then colour 1 each).
 * theta holds R configurations of N sites, configuration k at beta[k].
 * n_acc (may be NULL) receives the accepted Metropolis moves per position.
 * ------------------------------------------------------------------------ */
void orc_sweep(double *theta, int L, int R, const double *beta, uint64_t seed, uint32_t t,
               int lat, int n_metro, int n_or, double window, int64_t *n_acc)
{
    int64_t N = (int64_t)L * L * L;
    for (int k = 0; k < R; ++k) {
        double *th = theta + (int64_t)k * N;
        int64_t acc = 0;
        for (int s = 0; s < n_metro; ++s)
            for (int c = 0; c < 2; ++c)
                acc += orc_metro_half(th, L, beta[k], seed, t, lat, k, s, window, c);
        for (int s = 0; s < n_or; ++s)
            for (int c = 0; c < 2; ++c)
                orc_or_half(th, L, c);
        if (n_acc) n_acc[k] = acc;
    }
}

/* Neumaier-compensated accumulator. */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------
 * Observables of one configuration.
 *   E   = - sum over bonds cos(theta_i - theta_j)          Eq. (1), J = 1
 *   Mx  = sum_j cos theta_j,  My = sum_j sin theta_j
 *   |m| = sqrt(Mx^2 + My^2) / N                            Eq. (4), one sample
 *   out = {E, E/N, |m|, |m|^2, |m|^4}
 * Every bond is counted once as (i, i + mu) for mu = x, y, z.
 * ------------------------------------------------------------------------ */
void orc_measure(const double *theta, int L, double out[5])
{
    int64_t N = (int64_t)L * L * L;
    nsum E = {0, 0}, Mx = {0, 0}, My = {0, 0};
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int64_t i = x + (int64_t)L * (y + (int64_t)L * z);
                int64_t nb[6];
                neighbours(L, x, y, z, nb);
                double th = theta[i];
                nsum_add(&E, -cos(th - theta[nb[1]]));
                nsum_add(&E, -cos(th - theta[nb[3]]));
                nsum_add(&E, -cos(th - theta[nb[5]]));
                nsum_add(&Mx, cos(th));
                nsum_add(&My, sin(th));
            }
    double e = nsum_get(&E), mx = nsum_get(&Mx), my = nsum_get(&My);
    double m = sqrt(mx * mx + my * my) / (double)N;
    out[0] = e;
    out[1] = e / (double)N;
    out[2] = m;
    out[3] = m * m;
    out[4] = m * m * m * m;
}

/* ------------------------------------------------------------------------
 * Bond sums entering the spin stiffness of Eq. (6), one configuration:
 *   C_mu = sum_i cos(theta_i - theta_{i+mu}),  I_mu = sum_i sin(theta_i - theta_{i+mu})
 * for mu = x, y, z (each bond once, oriented from i to i + mu).
 * out = {C_x, C_y, C_z, I_x, I_y, I_z}.
 * ------------------------------------------------------------------------ */
void orc_bond_sums(const double *theta, int L, double out[6])
{
    nsum C[3] = {{0, 0}, {0, 0}, {0, 0}}, I[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int64_t i = x + (int64_t)L * (y + (int64_t)L * z);
                int64_t nb[6];
                neighbours(L, x, y, z, nb);
                for (int mu = 0; mu < 3; ++mu) {
                    double d = theta[i] - theta[nb[2 * mu + 1]];
                    nsum_add(&C[mu], cos(d));
                    nsum_add(&I[mu], sin(d));
                }
            }
    for (int mu = 0; mu < 3; ++mu) {
        out[mu] = nsum_get(&C[mu]);
        out[3 + mu] = nsum_get(&I[mu]);
    }
}

/* ------------------------------------------------------------------------
 * One parallel-tempering exchange step over one lattice's ladder, Eq. (3).
 * Pairs (k, k+1) with k = tau mod 2, tau mod 2 + 2, ... are attempted; for
 * each, with beta = 1/T,
 *     W = min[1, exp((beta_k - beta_{k+1}) (E_k - E_{k+1}))]
 * and the swap is taken iff U(r0) < W, r = Philox(k, tau, lat << 16, EXCH << 24).
 * On acceptance the two configurations and their energies trade places.
 * theta: R configurations of N sites; E: R total energies; n_acc (may be
 * NULL): per-pair acceptance counters, incremented in place.  Returns the
 * number of swaps taken.
 * ------------------------------------------------------------------------ */
int orc_exchange(double *theta, double *E, int L, int R, const double *beta, uint64_t seed,
                 uint32_t tau, int lat, int64_t *n_acc)
{
    int64_t N = (int64_t)L * L * L;
    int swaps = 0;
    for (int k = (int)(tau & 1u); k + 1 < R; k += 2) {
        double w = exp((beta[k] - beta[k + 1]) * (E[k] - E[k + 1]));
        uint32_t r[4];
        draw(seed, (uint32_t)k, tau, (uint32_t)lat, 0u, ORC_PHASE_EXCH, 0u, r);
        if (orc_uniform(r[0]) < w) {
            if (theta) {
                double *a = theta + (int64_t)k * N, *b = theta + (int64_t)(k + 1) * N;
                for (int64_t i = 0; i < N; ++i) {
                    double tmp = a[i];
                    a[i] = b[i];
                    b[i] = tmp;
                }
            }
            double te = E[k];
            E[k] = E[k + 1];
            E[k + 1] = te;
            if (n_acc) n_acc[k] += 1;
            ++swaps;
        }
    }
    return swaps;
}

/* ------------------------------------------------------------------------
 * A whole run of one lattice: init (random or ordered), then n_sweeps of
 * [sweep; measure every configuration; exchange if due].  obs receives
 * n_sweeps * R * 5 values (measure layout above, by beta-position, taken
 * before the exchange of that sweep).  exchange_every = 0 disables exchange.
 * t starts at t0 and advances by one per sweep; tau starts at tau0 and
 * advances by one per exchange step.
 * ------------------------------------------------------------------------ */
void orc_run(double *theta, int L, int R, const double *beta, uint64_t seed, int lat,
             int ordered_start, uint32_t t0, uint32_t tau0, int n_sweeps, int n_metro,
             int n_or, double window, int exchange_every, double *obs, int64_t *n_metro_acc,
             int64_t *n_swap_acc)
{
    int64_t N = (int64_t)L * L * L;
    if (ordered_start)
        memset(theta, 0, sizeof(double) * (size_t)(N * R));
    else
        orc_init(theta, L, R, lat, seed);
    double *E = (double *)malloc(sizeof(double) * (size_t)R);
    int64_t *acc = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    uint32_t tau = tau0;
    for (int s = 0; s < n_sweeps; ++s) {
        uint32_t t = t0 + (uint32_t)s;
        orc_sweep(theta, L, R, beta, seed, t, lat, n_metro, n_or, window, acc);
        if (n_metro_acc)
            for (int k = 0; k < R; ++k) n_metro_acc[k] += acc[k];
        for (int k = 0; k < R; ++k) {
            double o[5];
            orc_measure(theta + (int64_t)k * N, L, o);
            E[k] = o[0];
            if (obs) memcpy(obs + ((int64_t)s * R + k) * 5, o, sizeof(o));
        }
        if (exchange_every > 0 && (s + 1) % exchange_every == 0) {
            orc_exchange(theta, E, L, R, beta, seed, tau, lat, n_swap_acc);
            ++tau;
        }
    }
    free(E);
    free(acc);
}
