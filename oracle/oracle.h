/*
 * oracle.h -- plain single-threaded CPU reference for Metropolis-Hastings with
 * Parallel Tempering on lattice spin models.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source with the GPU library.
 *
 * What it computes (paper: "Acceleration of Parallel Tempering for Markov Chain
 * Monte Carlo methods", arXiv 2512.03825):
 *   - the Metropolis-Hastings scheme of Sec. 2.1 with the acceptance of Eq. (1),
 *     specialised to single-spin flips of a lattice spin model whose target is
 *     the Boltzmann distribution of Eq. (2) (k = 1, beta = 1/T);
 *   - the Ising energy of Eq. (3) on a periodic square lattice, and a 3D +-J
 *     Edwards-Anderson variant on a periodic cubic lattice;
 *   - Parallel Tempering (Sec. 2.1): R replicas at their own temperatures that
 *     periodically try to swap their *states* with a neighbouring temperature,
 *     pairs alternating as described in Sec. 3, accepted with the logistic
 *     probability quoted in Sec. 3.
 * Site order is a checkerboard (colour 0 sites, then colour 1 sites); random
 * numbers come from a counter-based Philox4x32-10 stream keyed per draw, so
 * the result of a run is a pure function of its configuration.
 */
#ifndef PT_ORACLE_H
#define PT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ISING2D = 0, ORC_EA3D = 1 };

typedef struct {
  int32_t model;              /* ORC_ISING2D or ORC_EA3D */
  int32_t L;                  /* linear size, even, >= 2 */
  int32_t R;                  /* number of replicas (temperature slots), >= 1 */
  const double *beta;         /* [R] inverse temperatures, slot order */
  double J;                   /* 2D coupling (ignored for EA) */
  double h;                   /* 2D field: E = -J sum s_i s_j - h sum s_i (ignored for EA) */
  uint32_t seed;              /* Philox key word 0 for spin and flip/swap draws */
  uint32_t stream_id;         /* Philox key word 1 (instance id) */
  uint32_t coupling_seed;     /* Philox key word 0 for EA couplings */
  const int8_t *init_spins;   /* NULL, or [R][N] values +-1 (replica r starts at slot r) */
  const int8_t *couplings;    /* NULL, or EA [3][N] values +-1: bond (i, i+e_d) */
  uint32_t record_every;      /* record E, M every n sweeps (0 = never) */
  uint32_t max_records;       /* capacity of the record series */
} orc_config;

typedef struct orc_state orc_state;

/* Returns NULL if the configuration is invalid. */
orc_state *orc_create(const orc_config *cfg);
void orc_destroy(orc_state *st);

/* n checkerboard sweeps (each: all colour-0 sites, then all colour-1 sites). */
void orc_sweep(orc_state *st, uint64_t n);
/* One replica-exchange step with pair parity e & 1, then e += 1. */
void orc_exchange(orc_state *st);
/* n sweeps; after sweep s an exchange step runs when every > 0 and (s+1) % every == 0. */
void orc_run(orc_state *st, uint64_t n, uint32_t every);

int64_t orc_num_sites(const orc_state *st);
uint64_t orc_sweeps_done(const orc_state *st);
uint64_t orc_exchanges_done(const orc_state *st);
uint32_t orc_n_records(const orc_state *st);

void orc_get_spins(const orc_state *st, int8_t *out);          /* [R][N] +-1, slot order */
void orc_get_couplings(const orc_state *st, int8_t *out);      /* EA [3][N] +-1 */
void orc_get_labels(const orc_state *st, uint32_t *out);       /* [R] replica index held by each slot */
void orc_get_energy(const orc_state *st, int64_t *E, int64_t *M); /* [R] integer bond energy, magnetisation */
void orc_get_series(const orc_state *st, int32_t *E, int32_t *M); /* [n_records][R] */
void orc_get_swaps(const orc_state *st, uint64_t *att, uint64_t *acc); /* [R-1] per adjacent pair */
/* Full recount of the integer bond energy and the magnetisation of every slot. */
void orc_recount(const orc_state *st, int64_t *E, int64_t *M);

/* Building blocks exposed for tests. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Metropolis decision for a flip with energy change dE at inverse temperature beta. */
int orc_flip_accept(double beta, double dE, uint32_t r);
/* Replica-exchange decision for slots (k, k+1): x = (beta_k - beta_k1) * dE, dE = E_a - E_b. */
int orc_swap_accept(double beta_k, double beta_k1, double dE, uint32_t r);
/* Field factor of a swap for binary digit j of |dM|/2 (2D with h != 0). */
int orc_field_digit_accept(double dbeta_h_abs, int j, uint32_t r);

#ifdef __cplusplus
}
#endif
#endif
