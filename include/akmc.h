/*
 * akmc.h -- C interface of the MI355X (gfx950) vacancy-jump AKMC library.
 *
 * The library runs the classical atomistic kinetic Monte Carlo step that
 * the paper (Sec. III-B1) describes as the memory-bound baseline of its
 * method: before every event, every migration direction of every vacancy
 * is evaluated (pair-bond energy change, Kang-Weinberg barrier, Arrhenius
 * rate of Eq. 8, feasibility mask of Eq. 1), one event is drawn with
 * probability proportional to its rate (the system-wide competition of
 * Eq. 2), physical time advances by an increment inversely proportional to
 * the total rate (Sec. II; mean 1/Gamma_tot by Eq. 5), the atom and the
 * vacancy swap, and the rates near the jump are refreshed.
 *
 * Conventions shared by every call (they are readings of the paper, which
 * does not state a lattice or an energy model):
 *   - BCC lattice of lx*ly*lz cubic cells, periodic, two sites per cell,
 *     each edge >= 3 cells.  Site index
 *         site = b*lx*ly*lz + (z*ly + y)*lx + x,
 *     b = 0 for the cube corner, b = 1 for the body centre.
 *   - Occupancy: one uint8 species code per site, codes 0..S-1, the last
 *     code S-1 is the vacancy.
 *   - First-neighbour direction k = 4*[sx>0] + 2*[sy>0] + [sz>0] for the
 *     displacement (sx, sy, sz)*a/2; candidate c = 8*slot + k.
 *   - Energy: symmetric 1NN and 2NN pair energies eps1, eps2 (S x S, eV,
 *     vacancy rows included).  The energy change of "vacancy at i <- atom
 *     of species A at j" is built from integer species counts of the bonds
 *     it changes times D_k[A][s] = eps_k[A][s] - eps_k[S-1][s].
 *   - Barrier Ea = e0[A] + dE/2 (no clamp); rate = nu * exp(-Ea/(kb*T)).
 *     A jump onto another vacancy is inadmissible: rate +0, Ea = +inf.
 *   - Random stream: Philox4x64-10, key (seed, stream_id), counter
 *     (n, 0, 0, 0) for global event index n; u1 = (x0 >> 11) * 2^-53,
 *     u2 = ((x1 >> 11) + 1) * 2^-53.  dt = -ln(u2)/Gamma_tot.
 *   - Vacancy slots are numbered by ascending site at creation; a slot
 *     follows its vacancy.
 *   - Digest: starting from digest0 (default the FNV-1a offset basis), every
 *     event applies one FNV-1a step, h = (h ^ w) * 0x100000001b3 modulo
 *     2^64, to the word w = from_site | to_site << 32 (unsigned 32-bit
 *     sites).
 *
 * Memory: the library allocates no device memory.  The caller owns a
 * device workspace (sized by the *_workspace_bytes calls) and every device
 * output buffer; host pointers are only read or written during the call.
 * Work is enqueued on the caller's HIP stream (hipStream_t passed as
 * void*); calls return before the GPU finishes unless stated otherwise.
 *
 * Errors: every call returns an akmc_status.  Nothing throws or aborts
 * across this interface.  akmc_last_error() describes the last failure of
 * the calling thread.  Calls on one handle are not thread-safe.
 */
#ifndef AKMC_H
#define AKMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t akmc_status;
#define AKMC_OK                 0
#define AKMC_ERR_INVALID       -1   /* bad argument (message says which) */
#define AKMC_ERR_WORKSPACE     -2   /* workspace smaller than required */
#define AKMC_ERR_HIP           -3   /* a HIP runtime call failed */
#define AKMC_ERR_FROZEN        -4   /* total rate is zero: no event possible */
#define AKMC_ERR_UNSUPPORTED   -5   /* valid but outside the built limits */

#define AKMC_MAX_SPECIES        8
#define AKMC_MAX_VACANCIES    512   /* per lattice */

/* precision */
#define AKMC_FP64 0     /* energies, barriers, rates, sums and time in binary64 */
#define AKMC_FP32 1     /* energies, barriers, rates in binary32; sums, time binary64 */
/* refresh */
#define AKMC_REFRESH_LOCAL 0  /* after a jump, refresh the slots near it */
#define AKMC_REFRESH_FULL  1  /* recompute every slot (same results, slower) */
/* time_mode */
#define AKMC_TIME_STOCHASTIC 0  /* dt = -ln(u2) / Gamma_tot */
#define AKMC_TIME_MEAN       1  /* dt = 1 / Gamma_tot */
/* barrier_model */
#define AKMC_BARRIER_PAIR 0
#define AKMC_BARRIER_MLP  1   /* needs akmc_mlp_attach */
/* rates_eval mode */
#define AKMC_RATES_VACANCIES 0  /* current slots      -> [n_vac][8]   */
#define AKMC_RATES_SITES     1  /* listed sites       -> [n_sites][8] */
#define AKMC_RATES_ALL_SITES 2  /* every lattice site -> [N][8]       */

/* Lattice and model parameters.  All host values are copied at create. */
typedef struct akmc_params {
    int32_t lx, ly, lz;        /* cubic cells per axis, each >= 3 */
    int32_t n_species;         /* S, 2..8; code S-1 is the vacancy */
    double eps1[64];           /* 1NN pair energies, S*S row-major, symmetric, eV */
    double eps2[64];           /* 2NN pair energies, same layout */
    double e0[8];              /* barrier offset per migrating species 0..S-2, eV */
    double nu;                 /* attempt frequency, Hz, > 0 */
    double temperature;        /* K, > 0 */
    double kb;                 /* Boltzmann constant, eV/K (8.617333262e-5) */
    uint64_t seed;             /* Philox key word 0 */
    uint64_t stream_id;        /* Philox key word 1 */
    int64_t event_counter0;    /* global index of the next event (resume) */
    double time0;              /* physical time at create, s (resume) */
    uint64_t digest0;          /* digest at create; 0 selects the FNV offset basis */
    int32_t precision;         /* AKMC_FP64 or AKMC_FP32 */
    int32_t refresh;           /* AKMC_REFRESH_LOCAL or AKMC_REFRESH_FULL */
    int32_t time_mode;         /* AKMC_TIME_STOCHASTIC or AKMC_TIME_MEAN */
    int32_t barrier_model;     /* AKMC_BARRIER_PAIR or AKMC_BARRIER_MLP */
    /* Range of the pair model: 2 (first and second neighbours, eps1, eps2)
     * or 6 (every pair within 6.0 A: shells 1-6 with 8, 6, 12, 24, 8, 6
     * neighbours, the 64-neighbour range of Sec. IV-C; shells 3-6 in
     * eps_far[0..3], same layout as eps1).  With 6 shells the energy change
     * is the integer species counts of the changed bonds of every shell
     * times D_m[A][s] = eps_m[A][s] - eps_m[S-1][s], one fused multiply-add
     * chain over shells 1..6 then species; edges must be >= 5 cells; the
     * learned barrier, the learned runtime forms and batches are not
     * available for it (UNSUPPORTED). */
    int32_t n_shells;
    int32_t pad_;
    double eps_far[4][64];
} akmc_params;

/* One executed event (40 bytes). */
typedef struct akmc_event {
    int64_t n;                 /* global event index */
    int32_t slot;              /* vacancy slot that moved */
    int32_t from_site;         /* vacancy site before the jump */
    int32_t to_site;           /* vacancy site after the jump */
    uint8_t dir;               /* first-neighbour direction 0..7 */
    uint8_t species;           /* species of the atom that moved */
    uint8_t pad[2];
    double gamma_tot;          /* total rate of the state before the jump, Hz */
    double dt;                 /* time increment, s */
} akmc_event;

typedef struct akmc_summary {
    double t;                  /* physical time, s */
    int64_t n_events;          /* global index of the next event */
    double gamma_tot;          /* total rate of the current state, Hz */
    uint64_t digest;
    int64_t species_count[8];  /* sites per species code */
    int64_t n_neg_barrier;     /* current candidates (pair model) with Ea < 0 */
    int64_t n_neg_reverse;     /* current candidates (pair model) with Ea < dE: the reverse
                                  jump's barrier Ea - dE is negative */
    int64_t n_ood;             /* surrogate evaluations that fell back to the pair model */
    int32_t n_vacancies;
    int32_t frozen;            /* 1 if the last kmc_step stopped on Gamma_tot = 0 */
    double loop_seconds;       /* device wall time the event loop has spent on this lattice
                                  since create, summed over launches */
} akmc_summary;

typedef struct akmc_lattice *akmc_handle;

/* Device bytes the workspace of one lattice with these parameters and
 * n_vac vacancies needs.  Defined for: the state that lattice_create
 * fills.  Errors: AKMC_ERR_INVALID for bad parameters. */
akmc_status akmc_workspace_bytes(const akmc_params *p, int32_t n_vac, size_t *bytes);

/* Creates a lattice.  occ_host: uint8[2*lx*ly*lz] host occupancy (copied).
 * slot_sites_host: int32[n_vac] site of every vacancy slot, in slot order
 * (copied), or NULL for ascending site order; a snapshot taken with
 * state_read and passed back here with its event counter, time and digest
 * continues exactly like the uninterrupted run.  d_ws: device workspace of
 * ws_bytes (borrowed; must outlive the handle, 256-byte aligned).
 * hip_stream: hipStream_t or NULL for the default stream.  Errors:
 * INVALID (bad parameters, species code >= S, a slot list that is not the
 * set of vacancy sites), UNSUPPORTED (more than AKMC_MAX_VACANCIES),
 * WORKSPACE, HIP. */
akmc_status akmc_lattice_create(const akmc_params *p, const uint8_t *occ_host,
                                const int32_t *slot_sites_host, void *d_ws,
                                size_t ws_bytes, void *hip_stream, akmc_handle *out);

/* Rates of the Eq. 8 law for a vacancy placed at each site of the mode's
 * site set (that site counts as a vacancy whatever it holds), in the
 * 8 directions: d_rates_out[site_index][k].  Element type is double for
 * AKMC_FP64 and float for AKMC_FP32.  d_ea_out (same type and shape, may
 * be NULL) receives the barriers.  d_sites: device int32 site list for
 * AKMC_RATES_SITES (ignored otherwise); a listed site outside [0, N) gets
 * NaN rates and barriers.  AKMC_RATES_ALL_SITES writes 16-byte vectors:
 * its outputs must be 16-byte aligned (hipMalloc and torch allocations
 * are).  Asynchronous.  Errors: INVALID (mode, NULL output or site list,
 * misaligned ALL_SITES output). */
akmc_status akmc_rates_eval(akmc_handle h, int32_t mode, const int32_t *d_sites,
                            int64_t n_sites, void *d_rates_out, void *d_ea_out);

/* Kernel timing of the bulk evaluation, for benchmarks and profilers (the
 * roofline of the AKMC_RATES_ALL_SITES kernel, Sec. III-B1's memory-bound
 * rate enumeration): every later AKMC_RATES_ALL_SITES launch on h records
 * start_event and stop_event (hipEvent_t, created by the caller, borrowed;
 * either may be NULL) at the start and the end of its kernel's execution
 * (hipExtLaunchKernel), so that hipEventElapsedTime gives the kernel's own
 * duration without the stream's dispatch gaps.  NULL, NULL stops it.
 * Errors: INVALID (NULL handle). */
akmc_status akmc_rates_timing(akmc_handle h, void *start_event, void *stop_event);

/* Performs exactly n_events residence-time events on the device with no
 * host round trip.  d_log: device array of n_events records, or NULL.
 * kmc_step(a) followed by kmc_step(b) gives the same state, bit for bit,
 * as kmc_step(a + b).  If the total rate becomes zero the lattice stops
 * where it is and state_read reports frozen = 1; further steps do nothing.
 * A lattice without vacancies returns AKMC_ERR_FROZEN.  Asynchronous. */
akmc_status akmc_kmc_step(akmc_handle h, int64_t n_events, akmc_event *d_log);

/* Advances the lattice toward the physical time t_end (a voxel evolved
 * over a stretch of service time, Sec. III-C1): an event starts only while
 * t < t_end, so the event that reaches or passes t_end is the last one; at
 * most max_events events in this call.  d_log: device array of max_events
 * records or NULL (only the first n_done are written; n_done is the change
 * of summary.n_events).  Chunked calls continue exactly like one call.
 * Asynchronous.  Errors: INVALID (NaN t_end, max_events < 0), FROZEN (no
 * vacancies), UNSUPPORTED (as kmc_step). */
akmc_status akmc_kmc_run_until(akmc_handle h, double t_end, int64_t max_events, akmc_event *d_log);

/* Barriers of the current candidates as the event loop last evaluated them
 * (the pair model of Eq. 8's barrier, or the learned barrier with its
 * pair-model fallback for a lattice with an attached network; the
 * candidates in slot order, c = 8*slot + k; +inf for an inadmissible jump):
 * d_ea_out receives n_vac*8 elements, double for AKMC_FP64 and float for
 * AKMC_FP32.  The loop refreshes a candidate whenever its bonds change, so
 * after every kmc_step these are the barriers of the current state.
 * Asynchronous (a device copy on the handle's stream).  Errors: INVALID
 * (NULL argument, no kmc_step has run on the handle yet), HIP. */
akmc_status akmc_loop_barriers(akmc_handle h, void *d_ea_out);

/* Synchronises the handle's stream and copies the state out.  occ_host
 * (uint8[N]) and slot_sites_host (int32[n_vac]) may be NULL; out may be
 * NULL. */
akmc_status akmc_state_read(akmc_handle h, uint8_t *occ_host, int32_t *slot_sites_host,
                            akmc_summary *out);

/* Cluster-size histogram of one species: connected components under
 * first-neighbour adjacency on the periodic lattice (clustering descriptor
 * of Sec. III-A2; Cu-rich precipitates of Sec. III-C1).  Off the event
 * path: it reads the lattice as the last enqueued step leaves it.
 *   species   code in [0, n_species)
 *   max_size  >= 1; d_hist (device int64[max_size + 1]) receives in
 *             hist[s] the number of clusters of size s for 1 <= s <
 *             max_size and in hist[max_size] those of size >= max_size;
 *             hist[0] = 0
 *   d_scratch device memory of at least akmc_cluster_scratch_bytes bytes,
 *             borrowed for the call (two int32 per site)
 * Errors: INVALID, WORKSPACE.  Asynchronous on the handle's stream. */
akmc_status akmc_cluster_scratch_bytes(akmc_handle h, size_t *bytes);
akmc_status akmc_cluster_hist(akmc_handle h, int32_t species, int64_t max_size,
                              int64_t *d_hist, void *d_scratch, size_t scratch_bytes);

/* Allocation-free variant of akmc_cluster_hist, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same histogram, with the
 * parent and size arrays taken from a scratch array the library holds in
 * its own device code object (32 MiB per device, kept until the process
 * ends) instead of from a caller buffer.  The caller still passes d_hist
 * (device int64[max_size + 1]).  The call allocates nothing and needs no
 * clearing: the first kernel overwrites every scratch element it uses.
 * All calls on one device share that one scratch array, so calls that
 * overlap on one device (different streams, or several host threads) race
 * and give wrong histograms; the caller serialises them.  Runs on the
 * device the handle was created on and on the handle's stream.
 * Errors: INVALID (as akmc_cluster_hist), UNSUPPORTED (more than
 * AKMC_CLUSTER_STATIC_MAX_SITES sites), HIP. */
#define AKMC_CLUSTER_STATIC_MAX_SITES 4194304
akmc_status akmc_cluster_hist_noalloc(akmc_handle h, int32_t species, int64_t max_size,
                                      int64_t *d_hist);

/* Releases the host-side handle.  Does not free d_ws. */
akmc_status akmc_lattice_destroy(akmc_handle h);

/* -------------------------------------------------------------- batches */

/* Independent replicas in one persistent launch: the paper's voxel
 * ensemble (Sec. III-C1), each replica a periodic lattice evolved with no
 * communication, scheduled heaviest first from a device work queue
 * (Sec. III-C2, priority of Eq. 10).  Replica r gives bit for bit the
 * same state as a standalone handle with the same parameters. */
typedef struct akmc_batch_s *akmc_batch;

typedef struct akmc_schedule {
    int32_t group_lanes;       /* lanes serving one replica: 8, 16, 32 or 64 */
    int32_t waves_per_block;   /* 1, 2 or 4 */
    int32_t blocks;            /* persistent blocks; 0 = one per 256 CUs worth */
    int32_t use_graph;         /* replay the chunk launches from a hipGraph */
    int64_t chunk_events;      /* events per replica per launch, > 0 */
} akmc_schedule;

/* n_vac[r] vacancies in replica r.  Errors: INVALID. */
akmc_status akmc_batch_workspace_bytes(int32_t n_rep, const akmc_params *p,
                                       const int32_t *n_vac, size_t *bytes);

/* p[n_rep] parameters (each replica's own lattice, temperature and Philox
 * key); occ_host[r] its occupancy; slot_sites_host NULL, or per replica a
 * slot list or NULL (as in lattice_create).  Same ownership rules as
 * lattice_create.  The initial schedule serves each replica with 8 lanes,
 * or with the fewest lanes whose groups fit in a workgroup's LDS. */
akmc_status akmc_batch_create(int32_t n_rep, const akmc_params *p,
                              const uint8_t *const *occ_host,
                              const int32_t *const *slot_sites_host, void *d_ws,
                              size_t ws_bytes, void *hip_stream, akmc_batch *out);

/* Sets the launch schedule (see akmc_batch_autotune).  Results do not
 * depend on the schedule.  Errors: INVALID (field out of range),
 * UNSUPPORTED (the (64 / group_lanes) * waves_per_block groups of a block,
 * each holding the largest replica's rate tree, slot lists and footprint
 * boxes, need more than the 160 KiB of LDS of a workgroup). */
akmc_status akmc_batch_set_schedule(akmc_batch b, const akmc_schedule *s);

/* Runs n_events events in every replica.  Asynchronous. */
akmc_status akmc_batch_step(akmc_batch b, int64_t n_events_per_replica);

/* Times candidate schedules on the live batch (each trial advances every
 * replica by trial_events events; results do not depend on the schedule),
 * keeps the fastest and returns it; schedules that do not fit in LDS (see
 * akmc_batch_set_schedule) are skipped.  Synchronises the stream. */
akmc_status akmc_batch_autotune(akmc_batch b, int64_t trial_events, akmc_schedule *chosen);

/* State of replica r (synchronises the stream). */
akmc_status akmc_batch_state_read(akmc_batch b, int32_t r, uint8_t *occ_host,
                                  int32_t *slot_sites_host, akmc_summary *out);

akmc_status akmc_batch_destroy(akmc_batch b);

/* ------------------------------------------------------ voxel ensemble */

/* Temperature-guided discretisation (Sec. III-C1): a reactor-vessel wall
 * section is split into a uniform n_x by n_z grid of voxels so that inside
 * every voxel the relative rate variation of Eq. 9, E dT/(kB T^2), stays
 * within tol, with dT the spread (max - min) of the field's samples in the
 * voxel and T their mean.  The grid with the fewest voxels is chosen; among
 * equal counts, the one with the fewest columns.
 *   T        host double[nz][nx] samples, x (through the wall) fastest, K
 *   e_eff    effective barrier E of Eq. 9, eV (> 0); kb eV/K; tol > 0
 *   t_vox    host double[nx*nz] capacity; receives the n_z*n_x voxel
 *            temperatures (means of their samples, summed row by row),
 *            voxel (b, a) at b*n_x + a; voxel a spans the sample columns
 *            floor(a*nx/n_x) .. floor((a+1)*nx/n_x) - 1, rows likewise
 *   worst    largest Eq. 9 variation of the chosen voxels (may be NULL)
 * Host only.  Errors: INVALID (NULL pointers, sizes < 1, non-finite or
 * non-positive samples or parameters). */
akmc_status akmc_voxel_grid(const double *T, int32_t nx, int32_t nz, double e_eff, double kb,
                            double tol, int32_t *n_x, int32_t *n_z, double *t_vox, double *worst);

/* Dispatch orders of akmc_batch_run_until. */
#define AKMC_ORDER_PRIORITY 0  /* workload proxy of Eq. 10, heaviest first */
#define AKMC_ORDER_INDEX    1  /* replica index */
#define AKMC_ORDER_CREATE   2  /* the order fixed at create */

/* Dynamic voxel scheduling (Sec. III-C2): the workload proxy of Eq. 10,
 * W_r = M_r exp(-E_r / kB T_r), of every replica from its current state
 * (M_r: admissible candidates; E_r: their mean barrier, summed in candidate
 * order in binary64; T_r: the replica's temperature), computed on the
 * device, and the queue order of the next launch set to decreasing W_r
 * (equal weights by index).  d_w_out: device double[n_rep] or NULL;
 * d_order_out: device int32[n_rep] receiving the order (replica indices,
 * first dispatched first) or NULL.  Before the first launch on the batch a
 * launch with no events evaluates the barriers.  Asynchronous.  Errors:
 * INVALID, HIP. */
akmc_status akmc_batch_priority(akmc_batch b, double *d_w_out, int32_t *d_order_out);

/* Advances every replica toward t_end (as akmc_kmc_run_until, at most
 * max_events_per_replica events each), the persistent groups pulling
 * replicas in the given order (AKMC_ORDER_*); AKMC_ORDER_PRIORITY first
 * recomputes the Eq. 10 order from the current states.  The order changes
 * only which replica runs when, never a replica's events.  Asynchronous.
 * Errors: INVALID (NaN t_end, negative count, unknown order), HIP. */
akmc_status akmc_batch_run_until(akmc_batch b, double t_end, int64_t max_events_per_replica,
                                 int32_t order);

/* ------------------------------------------------ learned runtime forms */

/* AtomWorld's runtime at simulation time (Sec. III-A): a local policy
 * network chooses the events and a Poisson time network advances physical
 * time, both on each vacancy's 64-neighbour observation (the species of the
 * sites within 6.0 A, the neighbour cap of Sec. IV-C; BCC shells 1-6, the
 * m-th neighbour being the m-th offset ordered by length, then x, y, z).
 * Network (the paper gives no architecture; this is the library's): hidden
 * width H a multiple of 8 up to 64, n_out outputs,
 *   h1 = relu(b1 + sum_m W1[m][code_m])          (m = 0..63, binary32 adds)
 *   h2 = relu(b2 + sum_i h1[i] W2[i][:])          (binary32 fma, i ascending)
 *   out = b3 + sum_i h2[i] W3[i][:]                (binary32 fma, i ascending)
 * with bfloat16 weights (W1, W2, W3) and binary32 biases.
 *   Policy (n_out = 8, Eq. 1-2): logit z_k of jump direction k; an
 *     inadmissible jump (onto a vacancy) is masked, the others scaled by
 *     1/tau (rounded to binary32 once); the event is drawn from the softmax
 *     over all candidates, i.e. with weight exp(z_k/tau) in binary64 in the
 *     same tree and residence-time selection as the rates.
 *   Poisson network (n_out = 1, Eq. 5-7): u(s) = sum over vacancies of the
 *     network's value; an event s -> s' advances time by
 *     (u(s) - Gamma(s)/Gamma(s') u(s'))/Gamma(s), Gamma the pair model's
 *     total rate (a frozen s' drops its term).
 * Without a policy the rates choose; without a Poisson network time
 * follows time_mode with the pair model's total rate.
 *
 * Blob: device memory of akmc_patchnet_blob_bytes, 256-byte aligned, owned
 * by the caller. */
akmc_status akmc_patchnet_blob_bytes(int32_t n_species, int32_t hidden, int32_t n_out, size_t *bytes);

/* Writes a network into the blob (synchronous copy on the default stream):
 * host_params binary32 [W1 (64*S*H, [m][s][j]), b1 (H), W2 (H*H, [i][j]),
 * b2 (H), W3 (H*n_out, [i][k]), b3 (n_out)]; the weights are rounded to
 * bfloat16 (to nearest, ties to even), the biases kept.  Errors: INVALID
 * (S not in [2, 8], H not a multiple of 8 in [8, 64], n_out not 1 or 8,
 * NULL, non-finite values), HIP. */
akmc_status akmc_patchnet_set(void *d_blob, int32_t n_species, int32_t hidden, int32_t n_out,
                              const float *host_params);

/* Reads the stored parameters back (the rounded weights), same layout;
 * host_params may be NULL to read only the sizes.  Synchronous. */
akmc_status akmc_patchnet_get(const void *d_blob, int32_t *n_species, int32_t *hidden, int32_t *n_out,
                              float *host_params);

/* The network's outputs for a vacancy placed at each listed site (its 64
 * neighbours as the lattice holds them): d_out float[n_sites][n_out]
 * (NaN for a site outside the lattice).  The same device forward the
 * event loop runs.  Asynchronous.  Errors: INVALID (species count differs
 * from the lattice's, NULL), HIP. */
akmc_status akmc_patchnet_eval(akmc_handle h, const void *d_blob, const int32_t *d_sites,
                               int64_t n_sites, float *d_out);

/* Lets the policy in d_blob (n_out = 8) choose this lattice's events from
 * the next kmc_step on, with temperature tau > 0; NULL restores selection
 * by the rates.  The blob is borrowed until detached.  Errors: INVALID
 * (not a policy blob, species count, tau, lattice edges below 5 cells: the
 * observation must hold 64 distinct sites), UNSUPPORTED (learned barrier
 * model lattice; the networks and the rate tree need more than 160 KiB of
 * LDS), HIP. */
akmc_status akmc_policy_attach(akmc_handle h, const void *d_blob, float tau);

/* Lets the Poisson network in d_blob (n_out = 1) advance this lattice's
 * time (Eq. 7) from the next kmc_step on; NULL restores time_mode.  Errors
 * as akmc_policy_attach. */
akmc_status akmc_poisson_attach(akmc_handle h, const void *d_blob);

/* ----------------------------------------------------- learned barrier */

/* A small network predicts the barrier Ea of a candidate from the species in
 * the bonds the jump changes; the pair model stays as the fallback and as
 * the reference for its error.  It applies the paper's reformulation of per-atom
 * network evaluation as batched matrix products on matrix units with
 * reduced precision and fused layers (Sec. III-B1), trained with AdamW at
 * batch 256 (Sec. IV-C).
 *   input   27 footprint slots of the candidate in the frame where the jump
 *           points along (+,+,+): slot 0 the moving species, 1..7 N1(i)
 *           without j, 8..13 N2(i), 14..20 N1(j) without i, 21..26 N2(j),
 *           each one-hot over S codes, zero-padded to 32*ceil(27*S/32);
 *   network 128 and 128 GELU(tanh) units, one output y; Ea = mu + sigma*y;
 *           bfloat16 weights and activations on the matrix cores with
 *           binary32 accumulation, binary32 biases and optimiser state.
 * The weights live in a caller-owned device blob. */

typedef struct akmc_train_cfg {
    int32_t batch;          /* rows per step, multiple of 16 (256) */
    int32_t epochs;         /* passes over the data set */
    float lr;               /* initial learning rate */
    float lr_final;         /* learning rate of the last step (cosine decay) */
    float beta1, beta2, eps;
    float weight_decay;     /* decoupled (AdamW) */
    int32_t shuffle;        /* 1: a fresh keyed permutation of the rows per epoch; 0: data order */
    int32_t pad_;
    uint64_t seed;          /* key of the row permutations */
} akmc_train_cfg;

/* Device bytes of the weight blob for n_species codes (2..8). */
akmc_status akmc_mlp_blob_bytes(int32_t n_species, size_t *bytes);

/* Initialises a blob: uniform random weights from the Philox stream of
 * seed, zero biases and optimiser moments, output scale Ea = mu + sigma*y.
 * Asynchronous on hip_stream. */
akmc_status akmc_mlp_init(void *d_blob, int32_t n_species, uint64_t seed, float mu,
                          float sigma, void *hip_stream);

/* Copies binary32 parameters in (host_params: the vector W1[K1][128],
 * b1[128], W2[128][128], b2[128], w3[128], b3[1], row-major input x output)
 * and clears the optimiser state, or out (get).  Synchronous. */
akmc_status akmc_mlp_set_params(void *d_blob, int32_t n_species, const float *host_params,
                                float mu, float sigma, void *hip_stream);
akmc_status akmc_mlp_get_params(const void *d_blob, int32_t n_species, float *host_params,
                                float *mu, float *sigma, void *hip_stream);
akmc_status akmc_mlp_param_count(int32_t n_species, int32_t *count);

/* Species codes of the 27 slots (d_env: uint8 [n][8][27]) and the pair-model
 * barrier (d_ea: float [n][8], +inf for an inadmissible jump; may be NULL)
 * of every candidate of the mode's site set (as in rates_eval). */
akmc_status akmc_env_encode(akmc_handle h, int32_t mode, const int32_t *d_sites, int64_t n_sites,
                            uint8_t *d_env, float *d_ea);

/* Records in the blob the largest per-species count of each of the four bond
 * groups over a data set, and which moving species occur; a candidate beyond
 * any of them is out of distribution and falls back to the pair model in the
 * event loop. */
akmc_status akmc_mlp_fit_ood(void *d_blob, int32_t n_species, const uint8_t *d_env, int64_t n,
                             void *hip_stream);

/* Barriers of n encoded candidates (d_ea: float [n]).  Asynchronous. */
akmc_status akmc_mlp_forward(const void *d_blob, int32_t n_species, const uint8_t *d_env,
                             int64_t n, float *d_ea, void *hip_stream);

/* Uses the blob's network for the barriers of a lattice created with
 * barrier_model AKMC_BARRIER_MLP (precision AKMC_FP32): inside the event
 * loop every refreshed candidate's 27 slot codes are staged in LDS and
 * evaluated on the matrix cores; candidates out of distribution (see
 * akmc_mlp_fit_ood) use the pair barrier and are counted in
 * akmc_summary.n_ood.  The blob is borrowed and must outlive the handle.
 * Synchronises the handle's stream.  Errors: INVALID (pair-model handle,
 * blob for another species count), UNSUPPORTED (the vacancies' rate tree
 * and the staged weights need more than the 160 KiB of LDS of a workgroup,
 * which happens only with 8 species and more than 504 vacancies). */
akmc_status akmc_mlp_attach(akmc_handle h, const void *d_blob);

/* Scratch bytes of training with this batch. */
akmc_status akmc_mlp_train_workspace_bytes(int32_t n_species, int32_t batch, size_t *bytes);

/* Trains on n rows (d_env [n][27] codes, d_ea [n] targets; rows whose slot 0
 * is the vacancy code are ignored) with mean-squared error on the
 * standardised barrier and AdamW.  d_loss: float per step or NULL.
 * Asynchronous. */
akmc_status akmc_mlp_train(void *d_blob, int32_t n_species, const uint8_t *d_env,
                           const float *d_ea, int64_t n, const akmc_train_cfg *cfg, float *d_loss,
                           void *d_work, size_t work_bytes, void *hip_stream);

/* Gradient of the mean loss over rows 0..n-1 (n <= batch of the workspace)
 * at the current weights, without an update: d_grad float [param_count]. */
akmc_status akmc_mlp_grad(const void *d_blob, int32_t n_species, const uint8_t *d_env,
                          const float *d_ea, int32_t n, float *d_grad, float *d_loss,
                          void *d_work, size_t work_bytes, void *hip_stream);

/* ------------------------------------------------------------ messages */

const char *akmc_status_string(akmc_status s);
const char *akmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AKMC_H */
