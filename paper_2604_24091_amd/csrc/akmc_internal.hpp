// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "akmc.h"

namespace akmc {

// Read-only description of one lattice (one replica), resident in device
// memory.  Tables hold D_k[A][s] = eps_k[A][s] - eps_k[V][s], rounded once
// from the binary64 difference.
struct LatDesc {
  int32_t lx, ly, lz, S;
  int32_t nv;                 // vacancy slots
  int32_t time_mode;
  int64_t ncell;              // lx*ly*lz
  int64_t occ_off;            // byte offset of the occupancy in the occupancy arena
  int64_t slot_off;           // element offset in the slot arena
  uint64_t seed, stream;
  double D1[64], D2[64];      // row A at 8*A: D_k[A][0..S-1], zero for s >= S
  double e0[8];
  double nu, kT;              // kT = kb*T in binary64
  float D1f[64], D2f[64];
  float e0f[8];
  float nuf, kTf;
  // Tables of the bulk sweep (relative to the all-Fe environment), scaled by
  // the exponent's factor h (beta/2 in binary64, (beta/2) log2(e) in
  // binary32), rows of 8 at 8*A for every code A (zero for s >= S):
  //   Hs_k[A][s] = h (D_k[A][s] - D_k[A][0]);  K[A][s] = D1[A][s] - D1[A][A].
  double Hs1[64], Hs2[64], K[64];
  alignas(64) float Hs1f[64];
  alignas(64) float Hs2f[64];
  float Kf[64];
  double beta;                // 1/kT
  float betaf;
  int32_t pad_[1];
  // Log-rate tables of the sweep:  ln r = Cn[A][s_p] + (beta/2)(G'_A(j) - G'_A(p))
  // with Cn[A][s] = ln(nu) - beta*e0[A] - (beta/2)*K[A][s];  C2f is Cn*log2(e)
  // in binary32 and h2f = (beta/2)*log2(e), for a base-2 exponential.
  double Cn[64];
  double half_beta, inv_half_beta;
  float C2f[64];
  float h2f, inv_h2f;
  // binary64 sweep: every factor exp(Cn - hG) and exp(hG) is bounded by
  // exp(700) either way for these tables (else the sweep is not used)
  int32_t sweep_factor_ok;
  int32_t pad2_;
  // Pair model out to 6.0 A (n_shells = 6): rows A at 8*A of
  // D_m[A][s] = eps_m[A][s] - eps_m[V][s] for shells m = 3..6.
  int32_t n_shells;
  int32_t pad3_;
  double Dx[4][64];
  float Dxf[4][64];
};

// Mutable per-lattice state.
struct LatState {
  double t;
  int64_t n;                  // next global event index
  uint64_t digest;
  double gamma_tot;
  int64_t n_ood;
  int32_t frozen;
  int32_t pad_;
  int64_t busy_ticks;         // device wall-clock ticks the event loop has spent on this lattice
};

// Event-loop launch description.
struct LoopArgs {
  const LatDesc *descs;
  LatState *states;
  uint8_t *occ;               // occupancy arena
  int32_t *slots;             // slot arena (site of each slot)
  akmc_event *log;            // NULL or [n_lat][log_stride]
  int64_t log_stride;
  const int32_t *order;       // processing order of lattices (heaviest first)
  int32_t *queue;             // work-queue counter (reset by the launcher)
  int32_t n_lat;
  int32_t nv_max;             // LDS sizing
  int32_t refresh_full;       // 1: refresh every slot after every event
  int64_t n_events;           // per lattice
  const unsigned char *mlp_blob;  // surrogate weights (barrier model MLP) or NULL
  // NULL, or the barrier of every candidate as the loop last evaluated it,
  // [slot][8] at element offset 8*slot_off of each lattice, in the rate
  // precision (double, or float for binary32): after every event it holds
  // the barriers of the current state (+inf for an inadmissible jump).
  void *ea_trace;
  // Time horizon: an event starts only while the lattice's t < t_end
  // (+inf for a fixed number of events).
  double t_end;
  // Learned runtime forms (launch_event_loop_lrn only): local policy
  // network choosing the events (NULL: the rates choose) with logits scaled
  // by inv_tau, Poisson time network (NULL: time_mode).
  const unsigned char *pol_blob, *pt_blob;
  float inv_tau;
  // LDS words of each group's coarse vacancy grid (0: none); every lattice
  // of the launch takes vac_grid(its edges, its slots, reach, grid_words).
  int32_t grid_words;
};

// LDS carve-up of one lattice group in the event loop.  Every array is
// sized for nv_max slots; the tree levels hold partial sums of groups of 8
// children: level 1 over slot totals, level l+1 over the last partial of
// each level-l group, until one group of at most 8 nodes remains.
constexpr int kBoxBytes = 352;   // 7x7x7 footprint box, padded to 16
constexpr int kBoxBytesFar = 1344;  // 11x11x11 box of the pair model out to 6.0 A
constexpr int kMaxLevels = 3;
static_assert(AKMC_MAX_VACANCIES <= 8 * 8 * 8, "three levels of groups of 8 cover every slot");

struct GroupLayout {
  int nv_max, G, fp32, nlev_max;
  int qlen[kMaxLevels + 1];       // elements of level l (1-based)
  int qoff[kMaxLevels + 1];       // element offset of level l in the Q region
  int off_part, off_q, off_pos, off_aff, off_la, off_lb, off_spec, off_box, off_tab, off_rng, off_tmp;
  int off_grid, grid_words;
  int bytes;
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

// Coarse grid of vacancy counts of one lattice, used to rule out other
// vacancies near a jump without scanning every slot.  Cells are 2^lc
// half-lattice units per axis (the last cell of an axis also takes the
// remainder of the edge), so every cell spans at least 2^lc units; counts
// sit in fields of 2^fb bits (wide enough for nv) packed into 32-bit words.
// With 2^lc >= 2R a window of 2R + 1 units along an axis touches at most
// two cells, the cells of its two ends: the 8 cells of (X +- R, Y +- R,
// Z +- R) hold every vacancy within Chebyshev distance R of (X, Y, Z).
// Cells grow by powers of two until the grid fits cap_words (words = 0:
// no grid fits).
struct VacGrid {
  int lc, fb, nx, ny, nz, words;
};

__host__ __device__ inline VacGrid vac_grid(int lx, int ly, int lz, int nv, int reach, int cap_words) {
  VacGrid g;
  g.lc = 1;
  while ((1 << g.lc) < 2 * reach) ++g.lc;
  g.fb = nv <= 15 ? 2 : (nv <= 255 ? 3 : 4);
  for (;;) {
    g.nx = (2 * lx) >> g.lc;
    g.ny = (2 * ly) >> g.lc;
    g.nz = (2 * lz) >> g.lc;
    g.nx = g.nx < 1 ? 1 : g.nx;
    g.ny = g.ny < 1 ? 1 : g.ny;
    g.nz = g.nz < 1 ? 1 : g.nz;
    const long long cells = (long long)g.nx * g.ny * g.nz;
    const long long words = ((cells << g.fb) + 31) >> 5;
    if (words <= cap_words) {
      g.words = (int)words;
      return g;
    }
    if (cells == 1) {
      g.words = 0;
      return g;
    }
    ++g.lc;
  }
}

// far: the pair model out to 6.0 A (11x11x11 boxes, tables of 6 shells);
// grid_words: LDS words of the vacancy grid.
__host__ __device__ inline GroupLayout make_layout(int nv_max, int G, int fp32, int far = 0,
                                                   int grid_words = 0) {
  GroupLayout L{};
  L.nv_max = nv_max;
  L.G = G;
  L.fp32 = fp32;
  int n = nv_max, lev = 1, qtot = 0;
  for (;;) {
    L.qlen[lev] = n;
    L.qoff[lev] = qtot;
    qtot += n;
    if (n <= 8 || lev == kMaxLevels) break;
    n = (n + 7) / 8;
    ++lev;
  }
  L.nlev_max = lev;
  const int real = fp32 ? 4 : 8;
  int o = 0;
  L.off_part = o; o = align16(o + nv_max * 8 * 8);
  L.off_q = o;    o = align16(o + qtot * 8);
  L.off_pos = o;  o = align16(o + nv_max * 4);
  L.off_aff = o;  o = align16(o + nv_max * 4);
  L.off_la = o;   o = align16(o + nv_max * 4);
  L.off_lb = o;   o = align16(o + nv_max * 4);
  L.off_spec = o; o = align16(o + nv_max * 8);
  L.off_box = o;  o = align16(o + (G / 8) * (far ? kBoxBytesFar : kBoxBytes));
  L.off_tab = o;  o = align16(o + (64 + 64 + 8 + (far ? 4 * 64 : 0)) * real);
  L.off_rng = o;  o = align16(o + 2 * G * 8);
  L.off_tmp = o;  o = align16(o + G * 8);
  L.off_grid = o; o = align16(o + grid_words * 4);
  L.grid_words = grid_words;
  L.bytes = o;
  return L;
}

struct Schedule {
  int group_lanes;
  int waves_per_block;
  int blocks;
};

// Launchers (return hipError_t).
hipError_t launch_event_loop(const LoopArgs &a, int precision, int refresh_full,
                             const Schedule &s, hipStream_t stream);
// Event loop with the learned barrier (one 64-lane group, binary32 rates).
hipError_t launch_event_loop_mlp(const LoopArgs &a, int refresh_full, int n_species,
                                 hipStream_t stream);
size_t event_loop_lds_bytes(int nv_max, int group_lanes, int waves_per_block, int precision,
                            int grid_words = 0);
// Event loop with the learned runtime forms (one 64-lane group); lds from
// event_loop_lrn_lds_bytes with each attached network's (S, H, n_out).
// Event loop of the pair model out to 6.0 A (one 64-lane group).
hipError_t launch_event_loop_far(const LoopArgs &a, int precision, int refresh_full, hipStream_t stream);
size_t event_loop_far_lds_bytes(int nv_max, int precision, int grid_words = 0);
hipError_t launch_event_loop_lrn(const LoopArgs &a, int precision, int refresh_full, size_t lds,
                                 hipStream_t stream);
size_t event_loop_lrn_lds_bytes(int nv_max, int precision, const int pol_dims[3],
                                const int pt_dims[3], int grid_words = 0);
// Local patch networks on listed sites: out[n][n_out] (NaN for a site
// outside the lattice).
hipError_t launch_patch_eval(const LatDesc *d_desc, const uint8_t *d_occ, const unsigned char *d_blob,
                             int S, int H, int n_out, const int32_t *d_sites, int64_t n, float *d_out,
                             hipStream_t st);
size_t patch_eval_lds_bytes(int S, int H, int n_out);
// Voxel ensembles: the discretisation of a thermal field (host), and the
// workload proxy of every replica with the heaviest-first order (device).
int voxel_grid(const double *T, int nx, int nz, double e_eff, double kb, double tol, int *n_x,
               int *n_z, double *t_vox, double *worst);
hipError_t launch_priority(const LatDesc *d_descs, const void *d_trace, int fp32, int n_rep,
                           double *d_w, int32_t *d_order, hipStream_t st);
hipError_t launch_order_index(int32_t *d_order, int n_rep, hipStream_t st);
// LDS of the event loop with the learned barrier (one 64-lane group).
size_t event_loop_mlp_lds_bytes(int nv_max, int n_species, int grid_words = 0);
// LDS a workgroup may hold on gfx950.
constexpr size_t kLdsBytes = 160 * 1024;
// Largest vacancy grid of a single-lattice loop and of a batch group (words).
constexpr int kLoopGridWords = 8192;
constexpr int kBatchGridWords = 512;
hipError_t launch_queue_reset(int32_t *queue, hipStream_t stream);
hipError_t launch_cluster_hist(const uint8_t *d_occ, int lx, int ly, int lz, int species,
                               int64_t max_size, int64_t *d_hist, int *d_parent, int *d_size,
                               hipStream_t st);
// Device address, on the current device, of the library's own cluster
// scratch (parent and size arrays of AKMC_CLUSTER_STATIC_MAX_SITES each),
// resolved once per device.
hipError_t cluster_static_scratch(int32_t **parent, int32_t **size);

// Events that a launch records at the start and the end of its kernel's
// execution (hipExtLaunchKernel), for callers that time kernels; either
// may be null.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};

hipError_t launch_rates_sites(const LatDesc *d_desc, const LatDesc &h_desc, const uint8_t *occ,
                              const int32_t *sites, int64_t n_sites, int precision,
                              void *rates, void *ea, hipStream_t stream,
                              const LaunchTiming *tm = nullptr, void *de = nullptr);
hipError_t launch_rates_all(const LatDesc *d_desc, const LatDesc &h_desc, const uint8_t *occ,
                            int precision, void *rates, void *ea, hipStream_t stream,
                            const LaunchTiming *tm = nullptr);

// Surrogate (akmc_mlp.hip).
hipError_t launch_env_encode(const LatDesc *d_desc, const uint8_t *occ, const int32_t *sites,
                             int64_t n_sites, uint8_t *env, float *ea, hipStream_t stream);
hipError_t launch_ood_fit(unsigned char *blob, const uint8_t *env, int64_t n, int S, hipStream_t stream);
hipError_t launch_mlp_forward(const unsigned char *blob, int S, const uint8_t *env, int64_t n,
                              float *ea, hipStream_t stream);
hipError_t launch_mlp_init(unsigned char *blob, int S, uint64_t seed, hipStream_t stream);
hipError_t launch_mlp_sync(unsigned char *blob, int S, hipStream_t stream);
hipError_t launch_mlp_step(unsigned char *blob, int S, const uint8_t *env, const float *ea,
                           int64_t n, int batch, int rows, int64_t start, uint64_t perm_key,
                           int perm_bits, float *partial, int apply, float lr, float beta1,
                           float beta2, float eps, float wd, int step, float *grad_out,
                           float *loss_out, hipStream_t stream);
size_t mlp_partial_bytes(int S, int batch);

}  // namespace akmc
