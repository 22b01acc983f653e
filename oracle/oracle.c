/*
 * oracle.c -- plain single-threaded CPU reference for Metropolis-Hastings with
 * Parallel Tempering (arXiv 2512.03825).  TEST INFRASTRUCTURE ONLY: used by the
 * test suite, the smoke check and the benchmark's CPU baseline, never by the
 * product path.  Written for obviousness, not speed: every flip evaluates its
 * acceptance probability in FP64 with the C library's exp(), every draw runs a
 * whole Philox4x32-10 block, and replica exchange swaps the spin arrays
 * themselves ("swapping the state", Sec. 2.1).
 *
 * Conventions (the readings of the paper that this file commits to):
 *   - Energy, Eq. (3): E = -J sum_<ij> s_i s_j - h sum_i s_i, every bond counted
 *     once (the field is written with the opposite sign to the paper's B, i.e.
 *     h = -B; all workloads here have h = 0).  The 3D Edwards-Anderson variant is
 *     E = -sum_<ij> J_ij s_i s_j with J_ij = +-1 per bond.  The stored integer
 *     energy is E_int = -sum_<ij> J_b s_i s_j (J_b = 1 in 2D), so E = J*E_int - h*M.
 *   - Target, Eq. (2): P(sigma) ~ exp(-beta E), k = 1.
 *   - Flip acceptance, Eq. (1): A = min(1, exp(-beta dE)); a flip with draw r
 *     (a uniform 32-bit word) is accepted iff r < A * 2^32, evaluated in FP64.
 *   - Swap acceptance (Sec. 3): P = e^x / (1 + e^x) with x = dBeta * dE, where
 *     dBeta = beta_k - beta_{k+1} and dE = E_a - E_b for the states a, b held by
 *     slots k, k+1; evaluated as 1/(1+exp(-x)), saturated beyond |x| >= 32 ln 2;
 *     accepted iff r < P * 2^32.  The paper's model has no field; with a field
 *     (2D, h != 0) dE = J dE_int - h dM splits into x = x1 + y with
 *     x1 = dBeta J dE_int and y = -dBeta h dM, and the swap is accepted iff the
 *     logistic test on x1 passes and a Metropolis test min(1, e^y) passes.  The
 *     latter is a product of independent tests, one per set binary digit j of
 *     |dM|/2, each accepted with probability exp(-2^(j+1) |dBeta h|).  The ratio
 *     of forward to reverse acceptance stays e^(x1 + y) (detailed balance), and
 *     for h = 0 the rule is the logistic test alone.
 *   - Pairing (Sec. 3): exchange step e pairs slots (k, k+1) with k = e mod 2,
 *     e mod 2 + 2, ...; each slot takes part in at most one pair per step.
 *   - Checkerboard order: colour c = (x + y [+ z]) mod 2; a sweep updates every
 *     colour-0 site, then every colour-1 site.
 *   - Random words: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key
 *     (k0, k1) and counter (c0, c1, c2, c3); the purpose tag sits in c3 bits 8+.
 *       flip   at site i (j = i/2), sweep s, slot k, colour c:
 *              key (seed, stream_id), ctr (j/4, s, k, c),        word j mod 4
 *       swap   for pair (k, k+1) at exchange step e:
 *              key (seed, stream_id), ctr (k, e, 0, 1<<8),        word 0
 *              field digit j: ctr (k, e, 1 + j/4, 1<<8),          word j mod 4
 *       spin   initial value of site i in slot k:
 *              key (seed, stream_id), ctr (i/4, k, 0, 2<<8),      word i mod 4
 *       bond   EA coupling b = 3 i + d (d = 0,1,2 for +x,+y,+z):
 *              key (coupling_seed, stream_id), ctr (b/4, 0, 0, 3<<8), word b mod 4
 *     A spin or a coupling is -1 when the top bit of its word is set, else +1.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { PURPOSE_FLIP = 0, PURPOSE_SWAP = 1, PURPOSE_SPIN = 2, PURPOSE_BOND = 3 };

struct orc_state {
  orc_config cfg;
  double *beta;      /* [R] */
  int dim;           /* 2 or 3 */
  int64_t N;         /* sites per replica */
  int8_t *spins;     /* [R][N] +-1, indexed by temperature slot */
  int8_t *bond;      /* [3][N] +-1 couplings J_(i, i+e_d) (EA only) */
  int64_t *E;        /* [R] integer bond energy of the state held by each slot */
  int64_t *M;        /* [R] magnetisation */
  uint32_t *label;   /* [R] replica index of the state held by each slot */
  uint64_t sweeps;
  uint64_t exchanges;
  uint32_t n_records;
  int32_t *E_series; /* [max_records][R] */
  int32_t *M_series;
  uint64_t *att;     /* [R] attempts of pair (k, k+1) */
  uint64_t *acc;     /* [R] accepted swaps of pair (k, k+1) */
};

/* ---- Philox4x32-10, from its published definition (SC'11) ------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)prod1;
    uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)prod0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u; /* Weyl key schedule */
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t draw(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                     uint32_t c3, unsigned word) {
  uint32_t ctr[4] = {c0, c1, c2, c3}, key[2] = {k0, k1}, out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[word];
}

/* ---- acceptance rules ------------------------------------------------------ */
/* Eq. (1) with the Boltzmann target of Eq. (2): A = min(1, exp(-beta dE)). */
int orc_flip_accept(double beta, double dE, uint32_t r) {
  double p = (dE <= 0.0) ? 1.0 : exp(-(beta * dE));
  return (double)r < ldexp(p, 32);
}

/* Field factor of a swap, one binary digit j of |dM|/2: accept with
 * probability exp(-2^(j+1) |dBeta h|). */
int orc_field_digit_accept(double dbeta_h_abs, int j, uint32_t r) {
  double p = exp(-(dbeta_h_abs * ldexp(2.0, j)));
  return (double)r < ldexp(p, 32);
}

/* Swap probability of Sec. 3, e^x/(1+e^x) written as 1/(1+e^-x). */
int orc_swap_accept(double beta_k, double beta_k1, double dE, uint32_t r) {
  const double X = 0x1.62e42fefa39efp+4; /* 32 ln 2 */
  double x = (beta_k - beta_k1) * dE;
  if (x >= X) return 1;
  if (x <= -X) return 0;
  double p = 1.0 / (1.0 + exp(-x));
  return (double)r < ldexp(p, 32);
}

/* ---- lattice geometry ------------------------------------------------------ */
static void coords(const orc_state *st, int64_t i, int c[3]) {
  int L = st->cfg.L;
  c[0] = (int)(i % L);
  c[1] = (int)((i / L) % L);
  c[2] = (st->dim == 3) ? (int)(i / ((int64_t)L * L)) : 0;
}

static int64_t site(const orc_state *st, const int c[3]) {
  int64_t L = st->cfg.L;
  return (st->dim == 3) ? ((int64_t)c[2] * L + c[1]) * L + c[0] : (int64_t)c[1] * L + c[0];
}

/* Neighbour of site i one step along axis d, direction +1 or -1 (periodic). */
static int64_t neighbour(const orc_state *st, int64_t i, int d, int dir) {
  int c[3];
  coords(st, i, c);
  c[d] = (c[d] + dir + st->cfg.L) % st->cfg.L;
  return site(st, c);
}

/* J of the bond between site i and its neighbour along axis d, direction dir. */
static int bond_between(const orc_state *st, int64_t i, int d, int dir) {
  if (st->dim == 2) return 1;
  int64_t owner = (dir > 0) ? i : neighbour(st, i, d, -1);
  return st->bond[(int64_t)d * st->N + owner];
}

/* ---- energy ---------------------------------------------------------------- */
void orc_recount(const orc_state *st, int64_t *E, int64_t *M) {
  for (int k = 0; k < st->cfg.R; ++k) {
    const int8_t *s = st->spins + (int64_t)k * st->N;
    int64_t e = 0, m = 0;
    for (int64_t i = 0; i < st->N; ++i) {
      m += s[i];
      for (int d = 0; d < st->dim; ++d) /* each bond once: (i, i + e_d) */
        e -= (int64_t)bond_between(st, i, d, +1) * s[i] * s[neighbour(st, i, d, +1)];
    }
    E[k] = e;
    M[k] = m;
  }
}

/* ---- lifecycle ------------------------------------------------------------- */
orc_state *orc_create(const orc_config *cfg) {
  if (!cfg || !cfg->beta) return NULL;
  if (cfg->model != ORC_ISING2D && cfg->model != ORC_EA3D) return NULL;
  if (cfg->L < 2 || (cfg->L & 1) || cfg->R < 1) return NULL;
  for (int k = 0; k < cfg->R; ++k)
    if (!isfinite(cfg->beta[k]) || cfg->beta[k] < 0.0) return NULL;

  orc_state *st = (orc_state *)calloc(1, sizeof(orc_state));
  if (!st) return NULL;
  st->cfg = *cfg;
  st->dim = (cfg->model == ORC_EA3D) ? 3 : 2;
  st->N = (int64_t)cfg->L * cfg->L * (st->dim == 3 ? cfg->L : 1);
  int R = cfg->R;
  st->beta = (double *)malloc(sizeof(double) * R);
  st->spins = (int8_t *)malloc((size_t)(R * st->N));
  st->bond = (int8_t *)malloc((size_t)(3 * st->N));
  st->E = (int64_t *)calloc(R, sizeof(int64_t));
  st->M = (int64_t *)calloc(R, sizeof(int64_t));
  st->label = (uint32_t *)malloc(sizeof(uint32_t) * R);
  st->att = (uint64_t *)calloc(R, sizeof(uint64_t));
  st->acc = (uint64_t *)calloc(R, sizeof(uint64_t));
  size_t nrec = (size_t)cfg->max_records * R;
  st->E_series = (int32_t *)calloc(nrec ? nrec : 1, sizeof(int32_t));
  st->M_series = (int32_t *)calloc(nrec ? nrec : 1, sizeof(int32_t));
  st->cfg.beta = st->beta;
  st->cfg.init_spins = NULL;
  st->cfg.couplings = NULL;
  if (!st->beta || !st->spins || !st->bond || !st->E || !st->M || !st->label || !st->att ||
      !st->acc || !st->E_series || !st->M_series) {
    orc_destroy(st);
    return NULL;
  }
  memcpy(st->beta, cfg->beta, sizeof(double) * R);

  /* Initialisation phase (Sec. 3): every replica gets its own random state. */
  for (int k = 0; k < R; ++k) {
    st->label[k] = (uint32_t)k;
    for (int64_t i = 0; i < st->N; ++i) {
      int8_t v;
      if (cfg->init_spins) {
        v = cfg->init_spins[(int64_t)k * st->N + i];
        if (v != 1 && v != -1) { orc_destroy(st); return NULL; }
      } else {
        uint32_t w = draw(cfg->seed, cfg->stream_id, (uint32_t)(i >> 2), (uint32_t)k, 0u,
                          PURPOSE_SPIN << 8, (unsigned)(i & 3));
        v = (w >> 31) ? -1 : 1;
      }
      st->spins[(int64_t)k * st->N + i] = v;
    }
  }
  for (int d = 0; d < 3; ++d)
    for (int64_t i = 0; i < st->N; ++i) {
      int8_t v = 1;
      if (st->dim == 3) {
        if (cfg->couplings) {
          v = cfg->couplings[(int64_t)d * st->N + i];
          if (v != 1 && v != -1) { orc_destroy(st); return NULL; }
        } else {
          int64_t b = 3 * i + d;
          uint32_t w = draw(cfg->coupling_seed, cfg->stream_id, (uint32_t)(b >> 2), 0u, 0u,
                            PURPOSE_BOND << 8, (unsigned)(b & 3));
          v = (w >> 31) ? -1 : 1;
        }
      }
      st->bond[(int64_t)d * st->N + i] = v;
    }
  /* The "first iteration" of the initialisation phase: the initial E and M. */
  orc_recount(st, st->E, st->M);
  return st;
}

void orc_destroy(orc_state *st) {
  if (!st) return;
  free(st->beta); free(st->spins); free(st->bond); free(st->E); free(st->M);
  free(st->label); free(st->att); free(st->acc); free(st->E_series); free(st->M_series);
  free(st);
}

/* ---- Metropolis sweep (Sec. 2.1 scheme, Eq. 1) ----------------------------- */
static void sweep_once(orc_state *st) {
  const orc_config *cfg = &st->cfg;
  uint32_t s = (uint32_t)st->sweeps;
  for (int k = 0; k < cfg->R; ++k) {
    int8_t *sp = st->spins + (int64_t)k * st->N;
    for (int c = 0; c < 2; ++c) {
      for (int64_t i = 0; i < st->N; ++i) {
        int xyz[3];
        coords(st, i, xyz);
        if (((xyz[0] + xyz[1] + xyz[2]) & 1) != c) continue;
        int si = sp[i];
        /* local field: sum over neighbours of J_ij s_j */
        int F = 0;
        for (int d = 0; d < st->dim; ++d)
          for (int dir = -1; dir <= 1; dir += 2)
            F += bond_between(st, i, d, dir) * sp[neighbour(st, i, d, dir)];
        double dE = (st->dim == 2) ? (2.0 * (double)si) * (cfg->J * (double)F + cfg->h)
                                   : (2.0 * (double)si) * (double)F;
        uint32_t j = (uint32_t)(i >> 1);
        uint32_t r = draw(cfg->seed, cfg->stream_id, j >> 2, s, (uint32_t)k,
                          (uint32_t)c | (PURPOSE_FLIP << 8), j & 3u);
        if (orc_flip_accept(st->beta[k], dE, r)) {
          sp[i] = (int8_t)-si;
          st->E[k] += 2 * si * F;
          st->M[k] -= 2 * si;
        }
      }
    }
  }
  st->sweeps++;
  if (cfg->record_every && st->sweeps % cfg->record_every == 0 &&
      st->n_records < cfg->max_records) {
    for (int k = 0; k < cfg->R; ++k) {
      st->E_series[(size_t)st->n_records * cfg->R + k] = (int32_t)st->E[k];
      st->M_series[(size_t)st->n_records * cfg->R + k] = (int32_t)st->M[k];
    }
    st->n_records++;
  }
}

void orc_sweep(orc_state *st, uint64_t n) {
  for (uint64_t t = 0; t < n; ++t) sweep_once(st);
}

/* ---- replica exchange (Sec. 3): literal state swaps ------------------------ */
void orc_exchange(orc_state *st) {
  const orc_config *cfg = &st->cfg;
  uint32_t e = (uint32_t)st->exchanges;
  int R = cfg->R;
  int8_t *tmp = (int8_t *)malloc((size_t)st->N);
  for (int k = (int)(e & 1u); k + 1 < R; k += 2) {
    uint32_t r = draw(cfg->seed, cfg->stream_id, (uint32_t)k, e, 0u, PURPOSE_SWAP << 8, 0);
    int64_t dEint = st->E[k] - st->E[k + 1];
    double dE = (st->dim == 2) ? cfg->J * (double)dEint : (double)dEint;
    int accept = orc_swap_accept(st->beta[k], st->beta[k + 1], dE, r);
    if (accept && st->dim == 2 && cfg->h != 0.0) {
      /* field part y = -dBeta h dM; Metropolis min(1, e^y) as a product over digits */
      double dbeta = st->beta[k] - st->beta[k + 1];
      int64_t dM = st->M[k] - st->M[k + 1];
      double y = (dbeta * -cfg->h) * (double)dM;
      if (y < 0.0) {
        double a = fabs(dbeta * cfg->h);
        uint64_t n = (uint64_t)(dM < 0 ? -dM : dM) / 2u;
        for (int j = 0; n >> j; ++j)
          if ((n >> j) & 1u) {
            uint32_t rj = draw(cfg->seed, cfg->stream_id, (uint32_t)k, e, 1u + (uint32_t)(j >> 2),
                               PURPOSE_SWAP << 8, (unsigned)(j & 3));
            if (!orc_field_digit_accept(a, j, rj)) { accept = 0; break; }
          }
      }
    }
    st->att[k]++;
    if (accept) {
      int8_t *a = st->spins + (int64_t)k * st->N, *b = a + st->N;
      memcpy(tmp, a, (size_t)st->N);
      memcpy(a, b, (size_t)st->N);
      memcpy(b, tmp, (size_t)st->N);
      int64_t t64 = st->E[k]; st->E[k] = st->E[k + 1]; st->E[k + 1] = t64;
      t64 = st->M[k]; st->M[k] = st->M[k + 1]; st->M[k + 1] = t64;
      uint32_t t32 = st->label[k]; st->label[k] = st->label[k + 1]; st->label[k + 1] = t32;
      st->acc[k]++;
    }
  }
  free(tmp);
  st->exchanges++;
}

/* Intervals of sweeps separated by swap steps (Sec. 3, Fig. 2). */
void orc_run(orc_state *st, uint64_t n, uint32_t every) {
  for (uint64_t t = 0; t < n; ++t) {
    sweep_once(st);
    if (every && st->sweeps % every == 0) orc_exchange(st);
  }
}

/* ---- accessors ------------------------------------------------------------- */
int64_t orc_num_sites(const orc_state *st) { return st->N; }
uint64_t orc_sweeps_done(const orc_state *st) { return st->sweeps; }
uint64_t orc_exchanges_done(const orc_state *st) { return st->exchanges; }
uint32_t orc_n_records(const orc_state *st) { return st->n_records; }

void orc_get_spins(const orc_state *st, int8_t *out) {
  memcpy(out, st->spins, (size_t)(st->cfg.R * st->N));
}
void orc_get_couplings(const orc_state *st, int8_t *out) {
  memcpy(out, st->bond, (size_t)(3 * st->N));
}
void orc_get_labels(const orc_state *st, uint32_t *out) {
  memcpy(out, st->label, sizeof(uint32_t) * st->cfg.R);
}
void orc_get_energy(const orc_state *st, int64_t *E, int64_t *M) {
  memcpy(E, st->E, sizeof(int64_t) * st->cfg.R);
  memcpy(M, st->M, sizeof(int64_t) * st->cfg.R);
}
void orc_get_series(const orc_state *st, int32_t *E, int32_t *M) {
  memcpy(E, st->E_series, sizeof(int32_t) * (size_t)st->n_records * st->cfg.R);
  memcpy(M, st->M_series, sizeof(int32_t) * (size_t)st->n_records * st->cfg.R);
}
void orc_get_swaps(const orc_state *st, uint64_t *att, uint64_t *acc) {
  int n = st->cfg.R > 1 ? st->cfg.R - 1 : 0;
  memcpy(att, st->att, sizeof(uint64_t) * n);
  memcpy(acc, st->acc, sizeof(uint64_t) * n);
}
