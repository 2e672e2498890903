/* Declarations of the CPU FP64 oracle (test infrastructure only; see
 * xy_oracle.c for the definitions and their citations). */
#ifndef XY_ORACLE_H
#define XY_ORACLE_H
#include <stdint.h>

#define ORC_PHASE_INIT 1u
#define ORC_PHASE_METRO 2u
#define ORC_PHASE_EXCH 3u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint32_t r);
void orc_init(double *theta, int L, int R, int lat, uint64_t seed);
int orc_metro_site(double *theta, int L, double beta, uint64_t seed, uint32_t t, int lat,
                   int k, int substep, double window, int64_t i);
void orc_or_site(double *theta, int L, int64_t i);
int64_t orc_metro_half(double *theta, int L, double beta, uint64_t seed, uint32_t t, int lat,
                       int k, int substep, double window, int colour);
void orc_metro_margin(const double *theta, int L, double beta, uint64_t seed, uint32_t t,
                      int lat, int k, int substep, double window, int colour, double *margin);
void orc_or_half(double *theta, int L, int colour);
void orc_sweep(double *theta, int L, int R, const double *beta, uint64_t seed, uint32_t t,
               int lat, int n_metro, int n_or, double window, int64_t *n_acc);
void orc_measure(const double *theta, int L, double out[5]);
void orc_bond_sums(const double *theta, int L, double out[6]);
int orc_exchange(double *theta, double *E, int L, int R, const double *beta, uint64_t seed,
                 uint32_t tau, int lat, int64_t *n_acc);
void orc_run(double *theta, int L, int R, const double *beta, uint64_t seed, int lat,
             int ordered_start, uint32_t t0, uint32_t tau0, int n_sweeps, int n_metro,
             int n_or, double window, int exchange_every, double *obs, int64_t *n_metro_acc,
             int64_t *n_swap_acc);
#endif
