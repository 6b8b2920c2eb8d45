/*
 * akmc_oracle.c -- plain, slow CPU reference of the classical AKMC
 * vacancy-jump path (rates, selection, time, swap) for BCC alloys.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The HIP library never
 * calls it, links it or shares a line of code, a header or a table with it.
 *
 * What is computed, following the paper:
 *   - Classical AKMC (Sec. III-B1): before every event, every migration
 *     direction of every vacancy is enumerated and its rate evaluated.
 *     This oracle does exactly that: a full recompute of all rates at every
 *     event, with no incremental bookkeeping.  A second entry point
 *     refreshes after each jump only the vacancies within reach of the two
 *     exchanged sites (the locality that lets classical codes scale); it
 *     gives the same trajectory and serves as the classical CPU baseline.
 *   - Rate of a candidate: the Arrhenius law of Eq. 8, r = nu exp(-Ea/kB T).
 *   - Feasibility mask (Eq. 1): a jump whose target site holds a vacancy is
 *     inadmissible and gets rate zero.
 *   - Selection: one event out of all candidates of the whole system, with
 *     probability proportional to its rate (the system-wide competition of
 *     Eq. 2, here with logits ln r).
 *   - Physical time: the increment is inversely proportional to the total
 *     rate (Sec. II); its mean 1/Gamma_tot follows from the first-passage
 *     relation of Eq. 5.
 * The paper does not state the energy model, the lattice, the random
 * stream or the summation order.  The readings used here are:
 *   - BCC, lx*ly*lz cubic cells, periodic, 2 sites per cell, each edge >= 3.
 *     Site index = b*lx*ly*lz + (z*ly + y)*lx + x, b = 0 cube corner,
 *     b = 1 body centre.
 *   - 1NN direction k = 4*[sx>0] + 2*[sy>0] + [sz>0] for the half-diagonal
 *     displacement (sx, sy, sz)*a/2; 2NN index m walks (+x,-x,+y,-y,+z,-z).
 *   - Energy: sum over 1NN and 2NN bonds of symmetric pair energies
 *     eps1[a][b], eps2[a][b], vacancy rows included.
 *   - Energy change of the jump "vacancy at i <- atom A at j" from the bonds
 *     it changes, as integer species counts times
 *     D_k[A][s] = eps_k[A][s] - eps_k[V][s], accumulated as one
 *     fused-multiply-add chain over s, shell 1 first.
 *   - Kang-Weinberg barrier Ea = E0[A] + dE/2 (no clamp).
 *   - Random stream: Philox4x64-10 (Salmon et al., SC'11), key
 *     (seed, stream_id), counter (n, 0, 0, 0) for global event index n;
 *     u1 = (x0 >> 11) 2^-53, u2 = ((x1 >> 11) + 1) 2^-53.
 *   - Selection: candidates c = 8*slot + k in slot order, slots ordered by
 *     ascending site at creation and following their vacancy; the chosen
 *     c is the first whose running sum exceeds u1*Gamma_tot (plain
 *     left-to-right sums), falling back to the last positive rate.
 *   - dt = -ln(u2)/Gamma_tot (or 1/Gamma_tot in mean-time mode).
 *   - Event digest: per event, one FNV-1a step (h ^= w; h *= 0x100000001b3,
 *     modulo 2^64) on the word w = from | to << 32, starting from the FNV
 *     offset basis.
 *
 * Precision: fp64 throughout by default.  A second mode computes energy
 * change, barrier and rate in binary32 (fmaf chain on the binary32 tables,
 * Ea = E0 + dE/2, x = -(Ea / kT) by one binary32 division, rate
 * nu * expf(x): the Arrhenius law of Eq. 8 written out in binary32) and
 * widens the rate to binary64 before any sum, so that the oracle takes
 * selection decisions in the same precision as a binary32 rate kernel.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t lx, ly, lz;
    int32_t n_species;           /* S; the vacancy code is S-1 */
    double eps1[64];             /* S*S row-major, eV */
    double eps2[64];
    double e0[8];                /* per migrating species, eV */
    double nu;                   /* Hz */
    double temperature;          /* K */
    double kb;                   /* eV/K */
    uint64_t seed;
    uint64_t stream_id;
    int32_t precision;           /* 0 = binary64, 1 = binary32 energies/rates */
    int32_t time_mode;           /* 0 = -ln(u2)/G, 1 = 1/G */
    int32_t n_shells;            /* 2 (1NN, 2NN) or 6 (every pair within 6.0 A) */
    int32_t pad_;
    double epsx[4][64];          /* shells 3..6 when n_shells = 6, S*S row-major, eV */
} orc_params;

typedef struct {
    int64_t n;                   /* global event index */
    int32_t slot;
    int32_t from_site;           /* vacancy site before the jump */
    int32_t to_site;             /* vacancy site after the jump */
    uint8_t dir;
    uint8_t species;             /* species of the atom that moved */
    uint8_t pad[2];
    double gamma_tot;            /* total rate of the state before the jump */
    double dt;
} orc_event;

typedef struct {
    int64_t n;                   /* next global event index */
    double t;                    /* physical time, s */
    uint64_t digest;
    double gamma_tot;            /* total rate of the current state */
    int64_t n_neg_evaluated;     /* evaluations (every event's, in full-recompute mode) with Ea < 0 */
} orc_state;

/* ---------------------------------------------------------------- lattice */

static int64_t n_cells(const orc_params *p) {
    return (int64_t)p->lx * p->ly * p->lz;
}

static int wrap(int a, int L) {
    int r = a % L;
    return r < 0 ? r + L : r;
}

int32_t orc_site(const orc_params *p, int b, int x, int y, int z) {
    x = wrap(x, p->lx);
    y = wrap(y, p->ly);
    z = wrap(z, p->lz);
    return (int32_t)(b * n_cells(p) + ((int64_t)z * p->ly + y) * p->lx + x);
}

void orc_decode(const orc_params *p, int32_t s, int *b, int *x, int *y, int *z) {
    int64_t nc = n_cells(p);
    *b = (int)(s / nc);
    int64_t r = s % nc;
    *x = (int)(r % p->lx);
    r /= p->lx;
    *y = (int)(r % p->ly);
    *z = (int)(r / p->ly);
}

int32_t orc_nbr1(const orc_params *p, int32_t s, int k) {
    int b, x, y, z;
    orc_decode(p, s, &b, &x, &y, &z);
    int px = (k >> 2) & 1, py = (k >> 1) & 1, pz = k & 1;
    if (b == 0) /* corner: +1/2 lands in this cell's centre, -1/2 in the previous cell's */
        return orc_site(p, 1, x - !px, y - !py, z - !pz);
    /* centre: +1/2 lands on the next cell's corner, -1/2 on this cell's */
    return orc_site(p, 0, x + px, y + py, z + pz);
}

int32_t orc_nbr2(const orc_params *p, int32_t s, int m) {
    int b, x, y, z;
    orc_decode(p, s, &b, &x, &y, &z);
    int step = (m & 1) ? -1 : 1;
    int axis = m >> 1;
    if (axis == 0) x += step;
    else if (axis == 1) y += step;
    else z += step;
    return orc_site(p, b, x, y, z);
}

/* --------------------------------------------------------------- energies */

static double dtab(const double *eps, int S, int a, int s) {
    int v = S - 1;
    return eps[a * S + s] - eps[v * S + s];
}

/* Species-count differences of the bonds the jump changes.  The vacancy
 * sits at i (whatever occ[i] holds), the atom at j = nbr1(i, k) moves to i.
 *   dn1[s] = #{n in N1(i)\{j}: s} - #{n in N1(j)\{i}: s}
 *   dn2[s] = #{n in N2(i):     s} - #{n in N2(j):     s}            */
static int counts(const orc_params *p, const uint8_t *occ, int32_t i, int k,
                  int dn1[8], int dn2[8]) {
    int32_t j = orc_nbr1(p, i, k);
    for (int s = 0; s < 8; s++) { dn1[s] = 0; dn2[s] = 0; }
    for (int q = 0; q < 8; q++) {
        int32_t n = orc_nbr1(p, i, q);
        if (n != j) dn1[occ[n]] += 1;
    }
    for (int q = 0; q < 8; q++) {
        int32_t n = orc_nbr1(p, j, q);
        if (n != i) dn1[occ[n]] -= 1;
    }
    for (int m = 0; m < 6; m++) dn2[occ[orc_nbr2(p, i, m)]] += 1;
    for (int m = 0; m < 6; m++) dn2[occ[orc_nbr2(p, j, m)]] -= 1;
    return occ[j];
}

/* The pair model out to 6.0 A (n_shells = 6): the bonds of shells 1-6 (the
 * 64 neighbours of the observation, 8, 6, 12, 24, 8, 6 per shell).  The
 * jump changes the bonds of i and j in every shell, so
 *   dn[m][s] = #{n in N_m(i)\{j}: s} - #{n in N_m(j)\{i}: s}
 * (j lies only in the first shell of i, and i in the first shell of j).
 * Defined after the observation offsets below. */
static int counts6(const orc_params *p, const uint8_t *occ, int32_t i, int k, int dn[6][8]);

static const double *shell_eps(const orc_params *p, int m) {
    return m == 0 ? p->eps1 : m == 1 ? p->eps2 : p->epsx[m - 2];
}

/* Energy change of the jump, binary64.  Returns NaN for a masked jump. */
double orc_delta_e(const orc_params *p, const uint8_t *occ, int32_t i, int k) {
    int S = p->n_species, dn1[8], dn2[8];
    if (p->n_shells == 6) {
        int dn[6][8];
        int A = counts6(p, occ, i, k, dn);
        if (A == S - 1) return NAN;
        double acc = 0.0;
        for (int m = 0; m < 6; m++)
            for (int s = 0; s < S; s++) acc = fma((double)dn[m][s], dtab(shell_eps(p, m), S, A, s), acc);
        return acc;
    }
    int A = counts(p, occ, i, k, dn1, dn2);
    if (A == S - 1) return NAN;
    double acc = 0.0;
    for (int s = 0; s < S; s++) acc = fma((double)dn1[s], dtab(p->eps1, S, A, s), acc);
    for (int s = 0; s < S; s++) acc = fma((double)dn2[s], dtab(p->eps2, S, A, s), acc);
    return acc;
}

/* Barrier, energy change and rate of one candidate, in the precision of
 * p->precision (widened to binary64).  Masked: Ea = +inf, dE = NaN,
 * rate = +0. */
static void candidate(const orc_params *p, const uint8_t *occ, int32_t i, int k,
                      double *ea_out, double *de_out, double *rate_out) {
    int S = p->n_species, dn1[8], dn2[8], dn[6][8];
    int A = p->n_shells == 6 ? counts6(p, occ, i, k, dn) : counts(p, occ, i, k, dn1, dn2);
    if (A == S - 1) {
        *ea_out = INFINITY;
        *de_out = NAN;
        *rate_out = 0.0;
        return;
    }
    if (p->n_shells == 6) {
        /* shells 1-6 in order, species in order: one fma chain */
        double acc = 0.0;
        float accf = 0.0f;
        for (int m = 0; m < 6; m++)
            for (int s = 0; s < S; s++) {
                acc = fma((double)dn[m][s], dtab(shell_eps(p, m), S, A, s), acc);
                accf = fmaf((float)dn[m][s], (float)dtab(shell_eps(p, m), S, A, s), accf);
            }
        if (p->precision == 0) {
            double ea = p->e0[A] + 0.5 * acc;
            double kt = p->kb * p->temperature;
            *ea_out = ea;
            *de_out = acc;
            *rate_out = p->nu * exp(-(ea / kt));
        } else {
            float ea = (float)p->e0[A] + 0.5f * accf;
            float kt = (float)(p->kb * p->temperature);
            *ea_out = (double)ea;
            *de_out = (double)accf;
            *rate_out = (double)((float)p->nu * expf(-(ea / kt)));
        }
        return;
    }
    if (p->precision == 0) {
        double acc = 0.0;
        for (int s = 0; s < S; s++) acc = fma((double)dn1[s], dtab(p->eps1, S, A, s), acc);
        for (int s = 0; s < S; s++) acc = fma((double)dn2[s], dtab(p->eps2, S, A, s), acc);
        double ea = p->e0[A] + 0.5 * acc;
        double kt = p->kb * p->temperature;
        double x = -(ea / kt);
        *ea_out = ea;
        *de_out = acc;
        *rate_out = p->nu * exp(x);
    } else {
        float acc = 0.0f;
        for (int s = 0; s < S; s++) acc = fmaf((float)dn1[s], (float)dtab(p->eps1, S, A, s), acc);
        for (int s = 0; s < S; s++) acc = fmaf((float)dn2[s], (float)dtab(p->eps2, S, A, s), acc);
        float ea = (float)p->e0[A] + 0.5f * acc;
        float kt = (float)(p->kb * p->temperature);
        float x = -(ea / kt);
        float r = (float)p->nu * expf(x);
        *ea_out = (double)ea;
        *de_out = (double)acc;
        *rate_out = (double)r;
    }
}

/* Barrier and rate of one candidate.  Masked: Ea = +inf, rate = +0. */
void orc_candidate(const orc_params *p, const uint8_t *occ, int32_t i, int k,
                   double *ea_out, double *rate_out) {
    double de;
    candidate(p, occ, i, k, ea_out, &de, rate_out);
}

/* Counts over the current candidates of the slots (admissible jumps only):
 * out[0] those with Ea < 0, out[1] those with Ea < dE, i.e. whose reverse
 * jump would have a negative barrier Ea - dE (both compared in the
 * precision of p->precision). */
void orc_barrier_counts(const orc_params *p, const uint8_t *occ, const int32_t *slots,
                        int32_t nv, int64_t out[2]) {
    out[0] = out[1] = 0;
    for (int32_t v = 0; v < nv; v++)
        for (int k = 0; k < 8; k++) {
            double ea, de, r;
            candidate(p, occ, slots[v], k, &ea, &de, &r);
            if (!(r > 0.0) && isinf(ea)) continue;
            if (ea < 0.0) out[0] += 1;
            if (ea < de) out[1] += 1;
        }
}

/* rates[n][8], ea[n][8] for a vacancy placed at each listed site. */
void orc_rates_sites(const orc_params *p, const uint8_t *occ, const int32_t *sites,
                     int64_t n, double *rates, double *ea) {
    for (int64_t a = 0; a < n; a++)
        for (int k = 0; k < 8; k++) {
            double e, r;
            orc_candidate(p, occ, sites[a], k, &e, &r);
            rates[a * 8 + k] = r;
            if (ea) ea[a * 8 + k] = e;
        }
}

/* ------------------------------------------------------------------ Philox */

static uint64_t mulhilo64(uint64_t a, uint64_t b, uint64_t *hi) {
    __uint128_t prod = (__uint128_t)a * (__uint128_t)b;
    *hi = (uint64_t)(prod >> 64);
    return (uint64_t)prod;
}

/* Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        uint64_t hi0, hi1;
        uint64_t lo0 = mulhilo64(M0, x0, &hi0);
        uint64_t lo1 = mulhilo64(M1, x2, &hi1);
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_uniforms(uint64_t seed, uint64_t stream_id, int64_t n, double *u1, double *u2) {
    uint64_t ctr[4] = {(uint64_t)n, 0, 0, 0}, key[2] = {seed, stream_id}, x[4];
    orc_philox4x64_10(ctr, key, x);
    const double two_m53 = 1.0 / 9007199254740992.0;
    *u1 = (double)(x[0] >> 11) * two_m53;
    *u2 = (double)((x[1] >> 11) + 1) * two_m53;
}

/* ---------------------------------------------------------------- digest */

uint64_t orc_fnv1a(uint64_t h, const uint8_t *bytes, int64_t n) {
    for (int64_t a = 0; a < n; a++) {
        h ^= bytes[a];
        h *= 0x100000001b3ULL;
    }
    return h;
}

/* One event of the trajectory digest: the FNV-1a step (xor, then multiply
 * by the 64-bit FNV prime, modulo 2^64) applied once to the 64-bit word
 * from | to << 32 (sites as unsigned 32-bit values).  For a word below 256
 * this is FNV-1a over that one byte. */
uint64_t orc_digest_event(uint64_t h, int32_t from, int32_t to) {
    const uint64_t w = (uint64_t)(uint32_t)from | ((uint64_t)(uint32_t)to << 32);
    return (h ^ w) * 0x100000001b3ULL;
}

/* -------------------------------------------------------------- selection */

/* First candidate whose left-to-right running sum exceeds u1*Gamma_tot;
 * falls back to the last positive rate.  Returns -1 when Gamma_tot is not
 * positive (frozen state). */
int64_t orc_select(const double *rates, int64_t n, double u1, double *gamma_tot) {
    double g = 0.0;
    for (int64_t c = 0; c < n; c++) g += rates[c];
    if (gamma_tot) *gamma_tot = g;
    if (!(g > 0.0)) return -1;
    double target = u1 * g, run = 0.0;
    int64_t last = -1;
    for (int64_t c = 0; c < n; c++) {
        run += rates[c];
        if (rates[c] > 0.0) last = c;
        if (run > target) return c;
    }
    return last;
}

static void all_rates(const orc_params *p, const uint8_t *occ, const int32_t *slots,
                      int32_t nv, double *rates, int64_t *n_neg) {
    for (int32_t v = 0; v < nv; v++)
        for (int k = 0; k < 8; k++) {
            double e, r;
            orc_candidate(p, occ, slots[v], k, &e, &r);
            rates[v * 8 + k] = r;
            if (n_neg && e < 0.0) *n_neg += 1;
        }
}

/* Total rate of the current state (plain sum of all candidates). */
double orc_gamma_tot(const orc_params *p, const uint8_t *occ, const int32_t *slots,
                     int32_t nv) {
    double *rates = (double *)malloc(sizeof(double) * 8 * (size_t)(nv > 0 ? nv : 1));
    all_rates(p, occ, slots, nv, rates, NULL);
    double g = 0.0;
    for (int64_t c = 0; c < 8 * (int64_t)nv; c++) g += rates[c];
    free(rates);
    return g;
}

/* Chebyshev distance between two sites in units of a/2 under the minimum
 * image: with site (b, x, y, z) at 2x+b, 2y+b, 2z+b half-cells, each axis
 * difference is taken modulo 2L and folded to at most L. */
static int half_dist(const orc_params *p, int32_t s, int32_t t) {
    int b1, x1, y1, z1, b2, x2, y2, z2;
    orc_decode(p, s, &b1, &x1, &y1, &z1);
    orc_decode(p, t, &b2, &x2, &y2, &z2);
    const int d[3][3] = {{2 * x1 + b1, 2 * x2 + b2, 2 * p->lx},
                         {2 * y1 + b1, 2 * y2 + b2, 2 * p->ly},
                         {2 * z1 + b1, 2 * z2 + b2, 2 * p->lz}};
    int m = 0;
    for (int a = 0; a < 3; a++) {
        int q = abs(d[a][0] - d[a][1]) % d[a][2];
        if (d[a][2] - q < q) q = d[a][2] - q;
        if (q > m) m = q;
    }
    return m;
}

/* The event loop of orc_run.  local = 0: every rate is recomputed before
 * every event (the classical enumeration).  local = 1: all rates once, then
 * after each jump only the slots whose vacancy lies within 3 half-cells of
 * the two exchanged sites, the reach of a vacancy's 8 candidates (a rate
 * reads sites up to 3 half-cells from its vacancy); every other rate is
 * unchanged by the jump, so both modes give the same trajectory.  n_neg
 * counts the candidates each mode evaluates. */
static int64_t run_events(const orc_params *p, uint8_t *occ, int32_t *slots, int32_t nv,
                          orc_state *st, int64_t n_events, orc_event *events, int local,
                          double t_end) {
    int V = p->n_species - 1;
    double *rates = (double *)malloc(sizeof(double) * 8 * (size_t)(nv > 0 ? nv : 1));
    int64_t done = 0;
    if (local) all_rates(p, occ, slots, nv, rates, &st->n_neg_evaluated);
    for (int64_t e = 0; e < n_events; e++) {
        /* Time horizon: an event starts only while t < t_end, so the event
         * that reaches or crosses t_end is the last one. */
        if (!(st->t < t_end)) break;
        if (!local) all_rates(p, occ, slots, nv, rates, &st->n_neg_evaluated);
        double u1, u2, g;
        orc_uniforms(p->seed, p->stream_id, st->n, &u1, &u2);
        int64_t c = orc_select(rates, 8 * (int64_t)nv, u1, &g);
        if (c < 0) {
            st->gamma_tot = g;
            free(rates);
            return done > 0 ? done : -4;
        }
        int32_t v = (int32_t)(c / 8);
        int k = (int)(c % 8);
        int32_t i = slots[v], j = orc_nbr1(p, i, k);
        double dt = (p->time_mode == 1) ? 1.0 / g : -log(u2) / g;
        if (events) {
            orc_event *ev = &events[e];
            memset(ev, 0, sizeof(*ev));
            ev->n = st->n;
            ev->slot = v;
            ev->from_site = i;
            ev->to_site = j;
            ev->dir = (uint8_t)k;
            ev->species = occ[j];
            ev->gamma_tot = g;
            ev->dt = dt;
        }
        occ[i] = occ[j];
        occ[j] = (uint8_t)V;
        slots[v] = j;
        st->digest = orc_digest_event(st->digest, i, j);
        st->t += dt;
        st->n += 1;
        done += 1;
        if (local)
            for (int32_t u = 0; u < nv; u++) {
                /* a candidate's bonds lie within 3 half-cells of its vacancy
                 * (5 for the pair model out to 6.0 A) */
                int reach = p->n_shells == 6 ? 5 : 3;
                if (half_dist(p, slots[u], i) > reach && half_dist(p, slots[u], j) > reach) continue;
                for (int kk = 0; kk < 8; kk++) {
                    double ea, r;
                    orc_candidate(p, occ, slots[u], kk, &ea, &r);
                    rates[u * 8 + kk] = r;
                    if (ea < 0.0) st->n_neg_evaluated += 1;
                }
            }
    }
    st->gamma_tot = orc_gamma_tot(p, occ, slots, nv);
    free(rates);
    return done;
}

/* Runs n_events events from (occ, slots, st).  Returns the number of events
 * done; -4 if the state is frozen before any event could be done (then
 * nothing changes).  log may be NULL. */
int64_t orc_run(const orc_params *p, uint8_t *occ, int32_t *slots, int32_t nv,
                orc_state *st, int64_t n_events, orc_event *events) {
    return run_events(p, occ, slots, nv, st, n_events, events, 0, INFINITY);
}

/* orc_run with the local refresh described at run_events. */
int64_t orc_run_local(const orc_params *p, uint8_t *occ, int32_t *slots, int32_t nv,
                      orc_state *st, int64_t n_events, orc_event *events) {
    return run_events(p, occ, slots, nv, st, n_events, events, 1, INFINITY);
}

/* Advances the lattice to the physical time t_end: events run while
 * t < t_end, at most max_events of them (a voxel evolved over a stretch of
 * service time, Sec. III-C1).  Returns the number done (0 if t >= t_end
 * already), or -4 if the state is frozen before the first event. */
int64_t orc_run_until(const orc_params *p, uint8_t *occ, int32_t *slots, int32_t nv,
                      orc_state *st, double t_end, int64_t max_events, orc_event *events) {
    return run_events(p, occ, slots, nv, st, max_events, events, 0, t_end);
}

/* Replays a given event log on (occ, slots, st) in binary64 and reports how
 * well every recorded choice agrees with the binary64 rates of the state it
 * was taken from:
 *   out[0] = max over events of the selection-interval violation, relative
 *            to Gamma_tot: max(0, C_{c-1} - u1 G, u1 G - C_c) / G
 *   out[1] = max relative difference of the recorded Gamma_tot
 *   out[2] = max relative difference of the recorded dt
 *   out[3] = number of structural mismatches (wrong index, site, species,
 *            a masked candidate chosen)
 *   out[4] = number of events whose recorded choice lies outside its
 *            binary64 interval (a binary64 run with the same uniform would
 *            have chosen another candidate)
 * The swaps recorded in the log are applied, so occ/slots end where the
 * logged trajectory ends. */
void orc_follow(const orc_params *p, uint8_t *occ, int32_t *slots, int32_t nv,
                orc_state *st, int64_t n_events, const orc_event *events, double out[5]) {
    int V = p->n_species - 1;
    double *rates = (double *)malloc(sizeof(double) * 8 * (size_t)(nv > 0 ? nv : 1));
    out[0] = out[1] = out[2] = out[3] = out[4] = 0.0;
    for (int64_t e = 0; e < n_events; e++) {
        const orc_event *ev = &events[e];
        all_rates(p, occ, slots, nv, rates, &st->n_neg_evaluated);
        double u1, u2;
        orc_uniforms(p->seed, p->stream_id, st->n, &u1, &u2);
        double g = 0.0;
        for (int64_t c = 0; c < 8 * (int64_t)nv; c++) g += rates[c];
        int64_t c = (int64_t)ev->slot * 8 + ev->dir;
        int bad = 0;
        if (ev->n != st->n || ev->slot < 0 || ev->slot >= nv || ev->dir > 7) bad = 1;
        if (!bad) {
            double before = 0.0;
            for (int64_t q = 0; q < c; q++) before += rates[q];
            double after = before + rates[c];
            double target = u1 * g;
            double viol = 0.0;
            if (before - target > viol) viol = before - target;
            if (target - after > viol) viol = target - after;
            if (viol / g > out[0]) out[0] = viol / g;
            if (viol > 0.0) out[4] += 1.0;
            if (!(rates[c] > 0.0)) bad = 1;
            double dg = fabs(ev->gamma_tot - g) / g;
            if (dg > out[1]) out[1] = dg;
            double dt = (p->time_mode == 1) ? 1.0 / g : -log(u2) / g;
            double ddt = fabs(ev->dt - dt) / dt;
            if (ddt > out[2]) out[2] = ddt;
            int32_t i = slots[ev->slot], j = orc_nbr1(p, i, ev->dir);
            if (ev->from_site != i || ev->to_site != j || ev->species != occ[j]) bad = 1;
            if (!bad) {
                occ[i] = occ[j];
                occ[j] = (uint8_t)V;
                slots[ev->slot] = j;
                st->digest = orc_digest_event(st->digest, i, j);
                st->t += dt;
            }
        }
        if (bad) {
            out[3] += 1.0;
            break;
        }
        st->n += 1;
    }
    free(rates);
}

/* ------------------------------------------------------------ observables */

/* Sizes of connected clusters of `species` under 1NN adjacency (plain
 * breadth-first search).  hist[s] counts clusters of size s for
 * 1 <= s <= max_size; larger clusters are counted in hist[max_size].
 * Returns the number of clusters. */
int64_t orc_cluster_hist(const orc_params *p, const uint8_t *occ, int species,
                         int64_t *hist, int64_t max_size) {
    int64_t n = 2 * n_cells(p);
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t clusters = 0;
    for (int64_t s = 0; s <= max_size; s++) hist[s] = 0;
    for (int64_t s = 0; s < n; s++) {
        if (occ[s] != species || seen[s]) continue;
        int64_t head = 0, tail = 0;
        queue[tail++] = (int32_t)s;
        seen[s] = 1;
        while (head < tail) {
            int32_t a = queue[head++];
            for (int k = 0; k < 8; k++) {
                int32_t b = orc_nbr1(p, a, k);
                if (occ[b] == species && !seen[b]) {
                    seen[b] = 1;
                    queue[tail++] = b;
                }
            }
        }
        hist[tail < max_size ? tail : max_size] += 1;
        clusters += 1;
    }
    free(seen);
    free(queue);
    return clusters;
}

/* ------------------------------------------------------------ surrogate input */

/* Species of the 27 footprint slots of a candidate, in a frame reflected so
 * that the jump direction becomes (+,+,+):
 *   slot 0        species A of the jumping atom (site j)
 *   slots 1..7    N1(i) without j, by reflected direction 0..6
 *   slots 8..13   N2(i), by reflected 2NN index (+x,-x,+y,-y,+z,-z)
 *   slots 14..20  N1(j) without i, by reflected direction 1..7
 *   slots 21..26  N2(j), by reflected 2NN index
 * Reflecting axis a (where the jump's sign is negative) flips bit (2-a) of
 * a 1NN direction and swaps the +/- entries of that axis' 2NN pair. */
void orc_encode_env(const orc_params *p, const uint8_t *occ, int32_t i, int k,
                    uint8_t out[27]) {
    int flip = (~k) & 7;
    int32_t j = orc_nbr1(p, i, k);
    out[0] = occ[j];
    for (int d = 0; d < 7; d++) out[1 + d] = occ[orc_nbr1(p, i, d ^ flip)];
    for (int m = 0; m < 6; m++) {
        int axis = m >> 1;
        int flipped = (flip >> (2 - axis)) & 1;
        out[8 + m] = occ[orc_nbr2(p, i, flipped ? (m ^ 1) : m)];
        out[21 + m] = occ[orc_nbr2(p, j, flipped ? (m ^ 1) : m)];
    }
    for (int d = 1; d < 8; d++) out[13 + d] = occ[orc_nbr1(p, j, d ^ flip)];
}

/* The 27 slot codes of all 8 candidates of every listed site:
 * out[n][8][27]. */
void orc_encode_env_sites(const orc_params *p, const uint8_t *occ, const int32_t *sites,
                          int64_t n, uint8_t *out) {
    for (int64_t a = 0; a < n; a++)
        for (int k = 0; k < 8; k++) orc_encode_env(p, occ, sites[a], k, out + (a * 8 + k) * 27);
}

/* ------------------------------------------- learned selection and time */

/* AtomWorld's runtime forms (Sec. III-A1, III-A3), written out plainly:
 *   - observation of a vacancy: the species of its 64 neighbours within
 *     6.0 A (the cutoff and neighbour cap of Sec. IV-C; on the BCC lattice
 *     these are shells 1-6 with 8, 6, 12, 24, 8, 6 sites);
 *   - local policy (Eq. 1-2): a network maps the observation to 8 logits,
 *     one per jump direction; an inadmissible jump's logit is -inf, the
 *     others are scaled by 1/tau; the event is drawn from the softmax over
 *     all candidates of the system, i.e. with weight exp(z_hat);
 *   - Poisson time (Eq. 5-7): u(s) is a sum of per-vacancy network values
 *     (the patch approximation of the dimensionless potential
 *     u = Gamma_tot tau), and an event advances time by
 *     dtau = (u(s) - Gamma_tot(s)/Gamma_tot(s') u(s')) / Gamma_tot(s),
 *     with Gamma_tot the physical total rate of the pair model.
 * Readings (the paper gives no sizes, order or activation):
 *   - neighbour m of the observation is the m-th offset (dx, dy, dz), in
 *     half-cell units, ordered by squared length, then dx, dy, dz
 *     ascending;
 *   - network: h1 = relu(b1 + sum_m W1[m][code_m]) (the one-hot first layer
 *     as a sum of the rows the codes select, m = 0..63 in order, binary32
 *     adds), h2 = relu(b2 + sum_i h1[i] W2[i][:]) and
 *     out = b3 + sum_i h2[i] W3[i][:] (i ascending, each term one binary32
 *     fused multiply-add); weights are bfloat16 values;
 *   - logits scaled by inv_tau = 1/tau rounded to binary32 once; weights
 *     exp(z_hat) in binary64;
 *   - u(s) = sum of the per-vacancy values in slot order in binary64;
 *   - a state s' with Gamma_tot(s') = 0 is frozen: its term is dropped
 *     (dtau = u(s)/Gamma_tot(s)). */

typedef struct {
    int32_t n_species;   /* S */
    int32_t hidden;      /* H <= 64 */
    int32_t n_out;       /* 8 (policy) or 1 (Poisson network) */
    int32_t pad_;
    const float *w1;     /* [64][S][H] */
    const float *b1;     /* [H] */
    const float *w2;     /* [H][H], input-major */
    const float *b2;     /* [H] */
    const float *w3;     /* [H][n_out], input-major */
    const float *b3;     /* [n_out] */
} orc_patchnet;

static int obs_off[64][3];
static int obs_ready = 0;

static void obs_build(void) {
    if (obs_ready) return;
    int n = 0;
    const int shells[6] = {3, 4, 8, 11, 12, 16};
    for (int sh = 0; sh < 6; sh++)
        for (int dx = -4; dx <= 4; dx++)
            for (int dy = -4; dy <= 4; dy++)
                for (int dz = -4; dz <= 4; dz++) {
                    int par = abs(dx) & 1;
                    if ((abs(dy) & 1) != par || (abs(dz) & 1) != par) continue;
                    if (dx * dx + dy * dy + dz * dz != shells[sh]) continue;
                    obs_off[n][0] = dx;
                    obs_off[n][1] = dy;
                    obs_off[n][2] = dz;
                    n++;
                }
    obs_ready = (n == 64);
}

/* Offset m of the observation, in half-cell units. */
void orc_obs_offset(int m, int out[3]) {
    obs_build();
    out[0] = obs_off[m][0];
    out[1] = obs_off[m][1];
    out[2] = obs_off[m][2];
}

/* Site at half-cell offset (dx, dy, dz) from site s (all three of the same
 * parity). */
static int32_t offset_site(const orc_params *p, int32_t s, int dx, int dy, int dz) {
    int b, x, y, z;
    orc_decode(p, s, &b, &x, &y, &z);
    int hx = wrap(2 * x + b + dx, 2 * p->lx);
    int hy = wrap(2 * y + b + dy, 2 * p->ly);
    int hz = wrap(2 * z + b + dz, 2 * p->lz);
    int bb = hx & 1;
    return orc_site(p, bb, (hx - bb) / 2, (hy - bb) / 2, (hz - bb) / 2);
}

/* Species codes of the 64-neighbour observation of a vacancy at site i. */
void orc_observation(const orc_params *p, const uint8_t *occ, int32_t i, uint8_t out[64]) {
    obs_build();
    for (int m = 0; m < 64; m++)
        out[m] = occ[offset_site(p, i, obs_off[m][0], obs_off[m][1], obs_off[m][2])];
}

/* Network outputs (n_out of them) for one observation. */
void orc_patchnet_forward(const orc_patchnet *net, const uint8_t codes[64], float *out) {
    int S = net->n_species, H = net->hidden;
    float h1[64], h2[64];
    for (int j = 0; j < H; j++) {
        float acc = net->b1[j];
        for (int m = 0; m < 64; m++) acc = acc + net->w1[((size_t)m * S + codes[m]) * H + j];
        h1[j] = acc > 0.0f ? acc : 0.0f;
    }
    for (int j = 0; j < H; j++) {
        float acc = net->b2[j];
        for (int i = 0; i < H; i++) acc = fmaf(h1[i], net->w2[i * H + j], acc);
        h2[j] = acc > 0.0f ? acc : 0.0f;
    }
    for (int k = 0; k < net->n_out; k++) {
        float acc = net->b3[k];
        for (int i = 0; i < H; i++) acc = fmaf(h2[i], net->w3[i * net->n_out + k], acc);
        out[k] = acc;
    }
}

/* Selection weights exp(z_hat) of the 8 candidates of a vacancy at site i
 * (0 for an inadmissible jump), and the logits themselves. */
void orc_policy_weights(const orc_params *p, const uint8_t *occ, int32_t i,
                        const orc_patchnet *pol, float inv_tau, double w[8], float z[8]) {
    uint8_t codes[64];
    orc_observation(p, occ, i, codes);
    orc_patchnet_forward(pol, codes, z);
    for (int k = 0; k < 8; k++) {
        int32_t j = orc_nbr1(p, i, k);
        w[k] = occ[j] == (uint8_t)(p->n_species - 1) ? 0.0 : exp((double)(z[k] * inv_tau));
    }
}

/* u(s): the Poisson network's values of every vacancy, summed in slot
 * order. */
double orc_poisson_u(const orc_params *p, const uint8_t *occ, const int32_t *slots, int32_t nv,
                     const orc_patchnet *pn) {
    double u = 0.0;
    for (int32_t v = 0; v < nv; v++) {
        uint8_t codes[64];
        float g;
        orc_observation(p, occ, slots[v], codes);
        orc_patchnet_forward(pn, codes, &g);
        u += (double)g;
    }
    return u;
}

/* Eq. 7: the time increment of an event from s to s'. */
double orc_poisson_dt(double u_s, double g_s, double u_s1, double g_s1) {
    if (!(g_s1 > 0.0)) return u_s / g_s;
    return (u_s - (g_s / g_s1) * u_s1) / g_s;
}

/* The event loop with a learned policy choosing the events (pol != NULL;
 * else the rates do) and, with pn != NULL, Poisson time (Eq. 7); without
 * pn, time follows p->time_mode with the physical total rate.  Every rate,
 * weight and network value is recomputed before every event.  Returns the
 * number of events done, or -4 if nothing can be chosen before the first. */
int64_t orc_run_learned(const orc_params *p, uint8_t *occ, int32_t *slots, int32_t nv,
                        orc_state *st, int64_t n_events, orc_event *events,
                        const orc_patchnet *pol, float inv_tau, const orc_patchnet *pn) {
    int V = p->n_species - 1;
    size_t nc = 8 * (size_t)(nv > 0 ? nv : 1);
    double *rates = (double *)malloc(sizeof(double) * nc);
    double *w = (double *)malloc(sizeof(double) * nc);
    int64_t done = 0;
    double g = 0.0;
    all_rates(p, occ, slots, nv, rates, NULL);
    for (int64_t c = 0; c < 8 * (int64_t)nv; c++) g += rates[c];
    double u = pn ? orc_poisson_u(p, occ, slots, nv, pn) : 0.0;
    for (int64_t e = 0; e < n_events; e++) {
        const double *sel = rates;
        if (pol) {
            for (int32_t v = 0; v < nv; v++) {
                float z[8];
                orc_policy_weights(p, occ, slots[v], pol, inv_tau, w + 8 * v, z);
            }
            sel = w;
        }
        double u1, u2, wsum;
        orc_uniforms(p->seed, p->stream_id, st->n, &u1, &u2);
        int64_t c = orc_select(sel, 8 * (int64_t)nv, u1, &wsum);
        if (c < 0 || !(g > 0.0)) {
            st->gamma_tot = g;
            free(rates);
            free(w);
            return done > 0 ? done : -4;
        }
        int32_t v = (int32_t)(c / 8);
        int k = (int)(c % 8);
        int32_t i = slots[v], j = orc_nbr1(p, i, k);
        uint8_t a = occ[j];
        occ[i] = a;
        occ[j] = (uint8_t)V;
        slots[v] = j;
        double g1 = 0.0;
        all_rates(p, occ, slots, nv, rates, NULL);
        for (int64_t q = 0; q < 8 * (int64_t)nv; q++) g1 += rates[q];
        double dt, u1s = 0.0;
        if (pn) {
            u1s = orc_poisson_u(p, occ, slots, nv, pn);
            dt = orc_poisson_dt(u, g, u1s, g1);
        } else {
            dt = (p->time_mode == 1) ? 1.0 / g : -log(u2) / g;
        }
        if (events) {
            orc_event *ev = &events[e];
            memset(ev, 0, sizeof(*ev));
            ev->n = st->n;
            ev->slot = v;
            ev->from_site = i;
            ev->to_site = j;
            ev->dir = (uint8_t)k;
            ev->species = a;
            ev->gamma_tot = g;
            ev->dt = dt;
        }
        st->digest = orc_digest_event(st->digest, i, j);
        st->t += dt;
        st->n += 1;
        done += 1;
        g = g1;
        u = u1s;
    }
    st->gamma_tot = g;
    free(rates);
    free(w);
    return done;
}

/* Replays a given event log under the learned forms (as orc_run_learned)
 * and reports how every recorded event agrees with the oracle's weights,
 * total rate and time increment of the state it was taken from:
 *   out[0] = max selection-interval violation relative to the weight total
 *   out[1] = max relative difference of the recorded (physical) Gamma_tot
 *   out[2] = max difference of the recorded dt relative to
 *            max(|dt|, u(s)/Gamma(s) + |u(s')|/Gamma(s')) (the scale of the
 *            two terms of Eq. 7; plain |dt| without a Poisson network)
 *   out[3] = structural mismatches (index, sites, species, a weight-0 pick)
 *   out[4] = events whose choice lies outside its exact interval
 * The logged swaps are applied. */
void orc_follow_learned(const orc_params *p, uint8_t *occ, int32_t *slots, int32_t nv,
                        orc_state *st, int64_t n_events, const orc_event *events,
                        const orc_patchnet *pol, float inv_tau, const orc_patchnet *pn,
                        double out[5]) {
    int V = p->n_species - 1;
    size_t nc = 8 * (size_t)(nv > 0 ? nv : 1);
    double *rates = (double *)malloc(sizeof(double) * nc);
    double *w = (double *)malloc(sizeof(double) * nc);
    for (int q = 0; q < 5; q++) out[q] = 0.0;
    for (int64_t e = 0; e < n_events; e++) {
        const orc_event *ev = &events[e];
        all_rates(p, occ, slots, nv, rates, NULL);
        double g = 0.0;
        for (int64_t c = 0; c < 8 * (int64_t)nv; c++) g += rates[c];
        const double *sel = rates;
        if (pol) {
            for (int32_t v = 0; v < nv; v++) {
                float z[8];
                orc_policy_weights(p, occ, slots[v], pol, inv_tau, w + 8 * v, z);
            }
            sel = w;
        }
        double wsum = 0.0;
        for (int64_t c = 0; c < 8 * (int64_t)nv; c++) wsum += sel[c];
        double u1, u2;
        orc_uniforms(p->seed, p->stream_id, st->n, &u1, &u2);
        int64_t c = (int64_t)ev->slot * 8 + ev->dir;
        int bad = (ev->n != st->n || ev->slot < 0 || ev->slot >= nv || ev->dir > 7);
        if (!bad) {
            double before = 0.0;
            for (int64_t q = 0; q < c; q++) before += sel[q];
            double after = before + sel[c];
            double target = u1 * wsum, viol = 0.0;
            if (before - target > viol) viol = before - target;
            if (target - after > viol) viol = target - after;
            if (viol / wsum > out[0]) out[0] = viol / wsum;
            if (viol > 0.0) out[4] += 1.0;
            if (!(sel[c] > 0.0)) bad = 1;
            double dg = fabs(ev->gamma_tot - g) / g;
            if (dg > out[1]) out[1] = dg;
            int32_t i = slots[ev->slot], j = orc_nbr1(p, i, ev->dir);
            if (ev->from_site != i || ev->to_site != j || ev->species != occ[j]) bad = 1;
            if (!bad) {
                double u_s = pn ? orc_poisson_u(p, occ, slots, nv, pn) : 0.0;
                occ[i] = occ[j];
                occ[j] = (uint8_t)V;
                slots[ev->slot] = j;
                double dt, scale;
                if (pn) {
                    double g1 = orc_gamma_tot(p, occ, slots, nv);
                    double u_s1 = orc_poisson_u(p, occ, slots, nv, pn);
                    dt = orc_poisson_dt(u_s, g, u_s1, g1);
                    scale = fabs(u_s) / g + (g1 > 0.0 ? fabs(u_s1) / g1 : 0.0);
                } else {
                    dt = (p->time_mode == 1) ? 1.0 / g : -log(u2) / g;
                    scale = fabs(dt);
                }
                if (fabs(dt) > scale) scale = fabs(dt);
                double ddt = fabs(ev->dt - dt) / scale;
                if (ddt > out[2]) out[2] = ddt;
                st->digest = orc_digest_event(st->digest, i, j);
                st->t += dt;
            }
        }
        if (bad) {
            out[3] += 1.0;
            break;
        }
        st->n += 1;
    }
    free(rates);
    free(w);
}

/* ------------------------------------------------ pair model out to 6.0 A */

static int shell_of_offset(const int d[3]) {
    int r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    return r2 == 3 ? 0 : r2 == 4 ? 1 : r2 == 8 ? 2 : r2 == 11 ? 3 : r2 == 12 ? 4 : r2 == 16 ? 5 : -1;
}

static int counts6(const orc_params *p, const uint8_t *occ, int32_t i, int k, int dn[6][8]) {
    int32_t j = orc_nbr1(p, i, k);
    obs_build();
    for (int m = 0; m < 6; m++)
        for (int s = 0; s < 8; s++) dn[m][s] = 0;
    for (int q = 0; q < 64; q++) {
        int sh = shell_of_offset(obs_off[q]);
        int32_t a = offset_site(p, i, obs_off[q][0], obs_off[q][1], obs_off[q][2]);
        int32_t b = offset_site(p, j, obs_off[q][0], obs_off[q][1], obs_off[q][2]);
        if (a != j) dn[sh][occ[a]] += 1;
        if (b != i) dn[sh][occ[b]] -= 1;
    }
    return occ[j];
}
