// C interface of the library (declared in include/akmc.h): argument
// checks, workspace carving, launches, state read-back and replica
// batches.  The library allocates no device memory; every device byte it
// touches belongs to the caller's workspace or output buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "akmc_internal.hpp"
#include "akmc_mlp.hpp"
#include "akmc_patch.hpp"

using namespace akmc;

namespace {

thread_local std::string g_last_error;

akmc_status fail(akmc_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

akmc_status hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return AKMC_ERR_HIP;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e__ = (expr);                            \
    if (e__ != hipSuccess) return hip_fail(e__, #expr); \
  } while (0)

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;
constexpr int64_t kChunkEvents = int64_t(1) << 22;

akmc_status check_params(const akmc_params *p) {
  if (!p) return fail(AKMC_ERR_INVALID, "params is NULL");
  if (p->lx < 3 || p->ly < 3 || p->lz < 3 || p->lx > 1000 || p->ly > 1000 || p->lz > 1000)
    return fail(AKMC_ERR_INVALID, "lattice edges must lie in [3, 1000] cells");
  if (2.0 * p->lx * (double)p->ly * p->lz >= 2147483647.0)
    return fail(AKMC_ERR_INVALID, "2*lx*ly*lz must stay below 2^31 sites");
  const int S = p->n_species;
  if (S < 2 || S > AKMC_MAX_SPECIES) return fail(AKMC_ERR_INVALID, "n_species must lie in [2, 8]");
  for (int a = 0; a < S; ++a)
    for (int b = 0; b < S; ++b) {
      const double e1 = p->eps1[a * S + b], e2 = p->eps2[a * S + b];
      if (!std::isfinite(e1) || !std::isfinite(e2))
        return fail(AKMC_ERR_INVALID, "pair energies must be finite");
      if (e1 != p->eps1[b * S + a] || e2 != p->eps2[b * S + a])
        return fail(AKMC_ERR_INVALID, "pair energy tables must be symmetric");
    }
  for (int a = 0; a < S - 1; ++a)
    if (!std::isfinite(p->e0[a])) return fail(AKMC_ERR_INVALID, "e0 must be finite");
  if (!(p->nu > 0.0) || !std::isfinite(p->nu)) return fail(AKMC_ERR_INVALID, "nu must be > 0");
  if (!(p->temperature > 0.0) || !std::isfinite(p->temperature))
    return fail(AKMC_ERR_INVALID, "temperature must be > 0");
  if (!(p->kb > 0.0) || !std::isfinite(p->kb)) return fail(AKMC_ERR_INVALID, "kb must be > 0");
  if (p->precision != AKMC_FP64 && p->precision != AKMC_FP32)
    return fail(AKMC_ERR_INVALID, "precision must be AKMC_FP64 or AKMC_FP32");
  if (p->refresh != AKMC_REFRESH_LOCAL && p->refresh != AKMC_REFRESH_FULL)
    return fail(AKMC_ERR_INVALID, "refresh must be LOCAL or FULL");
  if (p->time_mode != AKMC_TIME_STOCHASTIC && p->time_mode != AKMC_TIME_MEAN)
    return fail(AKMC_ERR_INVALID, "time_mode must be STOCHASTIC or MEAN");
  if (p->barrier_model != AKMC_BARRIER_PAIR && p->barrier_model != AKMC_BARRIER_MLP)
    return fail(AKMC_ERR_INVALID, "barrier_model must be PAIR or MLP");
  if (p->event_counter0 < 0) return fail(AKMC_ERR_INVALID, "event_counter0 must be >= 0");
  if (p->n_shells != 2 && p->n_shells != 6) return fail(AKMC_ERR_INVALID, "n_shells must be 2 or 6");
  if (p->n_shells == 6) {
    if (p->lx < 5 || p->ly < 5 || p->lz < 5)
      return fail(AKMC_ERR_INVALID, "the pair model out to 6.0 A needs lattice edges of at least 5 cells");
    for (int m = 0; m < 4; ++m)
      for (int a = 0; a < S; ++a)
        for (int b = 0; b < S; ++b) {
          const double e = p->eps_far[m][a * S + b];
          if (!std::isfinite(e)) return fail(AKMC_ERR_INVALID, "pair energies must be finite");
          if (e != p->eps_far[m][b * S + a]) return fail(AKMC_ERR_INVALID, "pair energy tables must be symmetric");
        }
  }
  if (!std::isfinite(p->time0)) return fail(AKMC_ERR_INVALID, "time0 must be finite");
  return AKMC_OK;
}

int64_t n_sites_of(const akmc_params *p) { return 2ll * p->lx * p->ly * p->lz; }

// Device description of one lattice, computed on the host in binary64.
LatDesc make_desc(const akmc_params *p, int nv) {
  LatDesc d;
  std::memset(&d, 0, sizeof(d));
  d.lx = p->lx; d.ly = p->ly; d.lz = p->lz;
  d.S = p->n_species;
  d.nv = nv;
  d.time_mode = p->time_mode;
  d.ncell = (int64_t)p->lx * p->ly * p->lz;
  d.seed = p->seed;
  d.stream = p->stream_id;
  const int S = p->n_species, V = S - 1;
  for (int A = 0; A < S; ++A)
    for (int s = 0; s < S; ++s) {
      const double d1 = p->eps1[A * S + s] - p->eps1[V * S + s];
      const double d2 = p->eps2[A * S + s] - p->eps2[V * S + s];
      d.D1[A * 8 + s] = d1;
      d.D2[A * 8 + s] = d2;
      d.D1f[A * 8 + s] = (float)d1;
      d.D2f[A * 8 + s] = (float)d2;
    }
  for (int A = 0; A < S; ++A)
    for (int s = 0; s < S; ++s) {
      const double kk = d.D1[A * 8 + s] - d.D1[A * 8 + A];
      d.K[A * S + s] = kk;
      d.Kf[A * S + s] = (float)kk;
    }
  for (int a = 0; a < S - 1; ++a) {
    d.e0[a] = p->e0[a];
    d.e0f[a] = (float)p->e0[a];
  }
  d.nu = p->nu;
  d.kT = p->kb * p->temperature;
  d.nuf = (float)d.nu;
  d.kTf = (float)d.kT;
  d.beta = 1.0 / d.kT;
  d.betaf = (float)d.beta;
  d.half_beta = 0.5 * d.beta;
  const double log2e = 1.4426950408889634074;
  const double lnnu = std::log(d.nu);
  for (int A = 0; A < S; ++A)
    for (int s = 0; s < S; ++s) {
      const double e0 = A < S - 1 ? d.e0[A] : 0.0;
      const double c = lnnu - d.beta * e0 - d.half_beta * d.K[A * S + s];
      d.Cn[A * S + s] = c;
      d.C2f[A * S + s] = (float)(c * log2e);
    }
  d.h2f = (float)(d.half_beta * log2e);
  d.inv_half_beta = 1.0 / d.half_beta;
  d.inv_h2f = 1.0f / d.h2f;
  for (int A = 0; A < S; ++A)
    for (int s = 0; s < S; ++s) {
      const double s1 = d.D1[A * 8 + s] - d.D1[A * 8 + 0];
      const double s2 = d.D2[A * 8 + s] - d.D2[A * 8 + 0];
      d.Hs1[A * 8 + s] = d.half_beta * s1;
      d.Hs2[A * 8 + s] = d.half_beta * s2;
      d.Hs1f[A * 8 + s] = (float)(d.half_beta * log2e * s1);
      d.Hs2f[A * 8 + s] = (float)(d.half_beta * log2e * s2);
    }
  // |hG_A| <= 8 max_s |Hs1[A][s]| + 6 max_s |Hs2[A][s]| (8 first and 6
  // second neighbours); the site exponent adds at most max |Cn|.
  double field = 0.0, cmax = 0.0;
  for (int A = 0; A < S; ++A) {
    double m1 = 0.0, m2 = 0.0;
    for (int s = 0; s < S; ++s) {
      m1 = std::max(m1, std::fabs(d.Hs1[A * 8 + s]));
      m2 = std::max(m2, std::fabs(d.Hs2[A * 8 + s]));
      cmax = std::max(cmax, std::fabs(d.Cn[A * S + s]));
    }
    field = std::max(field, 8.0 * m1 + 6.0 * m2);
  }
  d.sweep_factor_ok = cmax + field <= 700.0 ? 1 : 0;
  d.n_shells = p->n_shells;
  if (p->n_shells == 6)
    for (int m = 0; m < 4; ++m)
      for (int A = 0; A < S; ++A)
        for (int s = 0; s < S; ++s) {
          const double dx = p->eps_far[m][A * S + s] - p->eps_far[m][V * S + s];
          d.Dx[m][A * 8 + s] = dx;
          d.Dxf[m][A * 8 + s] = (float)dx;
        }
  return d;
}

struct WsLayout {
  size_t desc, state, order, queue, slots, scratch, trace, occ, total;
};

WsLayout ws_layout(int64_t nsites, int nv) {
  WsLayout w;
  size_t o = 0;
  w.desc = o;    o += up(sizeof(LatDesc));
  w.state = o;   o += up(sizeof(LatState));
  w.order = o;   o += up(sizeof(int32_t));
  w.queue = o;   o += up(sizeof(int32_t));
  w.slots = o;   o += up(sizeof(int32_t) * (size_t)std::max(nv, 1));
  w.scratch = o; o += up(sizeof(double) * 24 * (size_t)std::max(nv, 1));
  w.trace = o;   o += up(sizeof(double) * 8 * (size_t)std::max(nv, 1));
  w.occ = o;     o += up((size_t)nsites);
  w.total = o;
  return w;
}

bool aligned(const void *p) { return ((uintptr_t)p & (kAlign - 1)) == 0; }

// Vacancy slots of a host occupancy: the given slot list (checked to be
// exactly the set of vacancy sites) or all vacancy sites in ascending order.
akmc_status build_slots(const akmc_params *p, const uint8_t *occ, const int32_t *given,
                        std::vector<int32_t> &slots) {
  const int64_t N = n_sites_of(p);
  const int S = p->n_species;
  slots.clear();
  for (int64_t i = 0; i < N; ++i) {
    if (occ[i] >= S) return fail(AKMC_ERR_INVALID, "occupancy holds a code >= n_species");
    if (occ[i] == S - 1) slots.push_back((int32_t)i);
  }
  if ((int)slots.size() > AKMC_MAX_VACANCIES)
    return fail(AKMC_ERR_UNSUPPORTED, "more than AKMC_MAX_VACANCIES vacancies");
  if (given) {
    std::vector<int32_t> a(given, given + slots.size());
    std::vector<int32_t> b = a;
    std::sort(b.begin(), b.end());
    if (b != slots) return fail(AKMC_ERR_INVALID, "slot list is not the set of vacancy sites");
    slots = a;
  }
  return AKMC_OK;
}

}  // namespace

struct akmc_lattice {
  akmc_params p;
  int nv;
  int64_t nsites;
  hipStream_t stream;
  unsigned char *ws;
  WsLayout lay;
  LatDesc h_desc;
  LatDesc *d_desc;
  LatState *d_state;
  int32_t *d_order, *d_queue, *d_slots;
  double *d_scratch;
  void *d_trace;        // barriers the event loop last evaluated, [nv][8]
  bool stepped = false; // a kmc_step has filled d_trace
  uint8_t *d_occ;
  const unsigned char *mlp_blob = nullptr;
  LaunchTiming timing;  // events recorded by ALL_SITES launches (akmc_rates_timing)
  int device = 0;       // device current at create (where the workspace lives)
  // learned runtime forms (akmc_policy_attach, akmc_poisson_attach)
  const unsigned char *pol_blob = nullptr, *pt_blob = nullptr;
  int pol_dims[3] = {0, 0, 0}, pt_dims[3] = {0, 0, 0};
  float inv_tau = 1.0f;
};

extern "C" {

akmc_status akmc_workspace_bytes(const akmc_params *p, int32_t n_vac, size_t *bytes) {
  akmc_status s = check_params(p);
  if (s != AKMC_OK) return s;
  if (!bytes) return fail(AKMC_ERR_INVALID, "bytes is NULL");
  if (n_vac < 0 || n_vac > AKMC_MAX_VACANCIES)
    return fail(AKMC_ERR_INVALID, "n_vac must lie in [0, AKMC_MAX_VACANCIES]");
  *bytes = ws_layout(n_sites_of(p), n_vac).total;
  return AKMC_OK;
}

akmc_status akmc_lattice_create(const akmc_params *p, const uint8_t *occ_host,
                                const int32_t *slot_sites_host, void *d_ws, size_t ws_bytes,
                                void *hip_stream, akmc_handle *out) {
  akmc_status st = check_params(p);
  if (st != AKMC_OK) return st;
  if (!occ_host || !d_ws || !out) return fail(AKMC_ERR_INVALID, "NULL occupancy, workspace or out");
  if (!aligned(d_ws)) return fail(AKMC_ERR_INVALID, "workspace must be 256-byte aligned");
  if (p->barrier_model == AKMC_BARRIER_MLP && p->precision != AKMC_FP32)
    return fail(AKMC_ERR_UNSUPPORTED, "the learned barrier gives binary32 rates: use precision AKMC_FP32");
  if (p->barrier_model == AKMC_BARRIER_MLP && p->n_shells == 6)
    return fail(AKMC_ERR_UNSUPPORTED, "the learned barrier reads the two-shell bond footprint: use n_shells 2");
  const int64_t N = n_sites_of(p);
  std::vector<int32_t> slots;
  st = build_slots(p, occ_host, slot_sites_host, slots);
  if (st != AKMC_OK) return st;
  const int nv = (int)slots.size();
  const WsLayout lay = ws_layout(N, nv);
  if (ws_bytes < lay.total) return fail(AKMC_ERR_WORKSPACE, "workspace smaller than akmc_workspace_bytes");

  akmc_lattice *h = new (std::nothrow) akmc_lattice;
  if (!h) return fail(AKMC_ERR_INVALID, "out of host memory");
  h->p = *p;
  h->nv = nv;
  h->nsites = N;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(AKMC_ERR_HIP, "hipGetDevice failed");
  }
  h->stream = (hipStream_t)hip_stream;
  h->ws = (unsigned char *)d_ws;
  h->lay = lay;
  h->h_desc = make_desc(p, nv);
  h->d_desc = (LatDesc *)(h->ws + lay.desc);
  h->d_state = (LatState *)(h->ws + lay.state);
  h->d_order = (int32_t *)(h->ws + lay.order);
  h->d_queue = (int32_t *)(h->ws + lay.queue);
  h->d_slots = (int32_t *)(h->ws + lay.slots);
  h->d_scratch = (double *)(h->ws + lay.scratch);
  h->d_trace = h->ws + lay.trace;
  h->d_occ = h->ws + lay.occ;

  LatState s0;
  std::memset(&s0, 0, sizeof(s0));
  s0.t = p->time0;
  s0.n = p->event_counter0;
  s0.digest = p->digest0 ? p->digest0 : kFnvOffset;
  s0.frozen = 0;
  const int32_t zero = 0;
  hipError_t e;
  if ((e = hipMemcpyAsync(h->d_desc, &h->h_desc, sizeof(LatDesc), hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(h->d_state, &s0, sizeof(s0), hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(h->d_order, &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
      (nv > 0 && (e = hipMemcpyAsync(h->d_slots, slots.data(), sizeof(int32_t) * nv,
                                     hipMemcpyHostToDevice, h->stream)) != hipSuccess) ||
      (e = hipMemcpyAsync(h->d_occ, occ_host, (size_t)N, hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(h->stream)) != hipSuccess) {
    delete h;
    return hip_fail(e, "lattice_create copies");
  }
  *out = h;
  return AKMC_OK;
}

akmc_status akmc_rates_eval(akmc_handle h, int32_t mode, const int32_t *d_sites, int64_t n_sites,
                            void *d_rates_out, void *d_ea_out) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (!d_rates_out) return fail(AKMC_ERR_INVALID, "rates output is NULL");
  hipError_t e;
  switch (mode) {
    case AKMC_RATES_VACANCIES:
      e = launch_rates_sites(h->d_desc, h->h_desc, h->d_occ, h->d_slots, h->nv, h->p.precision,
                             d_rates_out, d_ea_out, h->stream);
      break;
    case AKMC_RATES_SITES:
      if (n_sites < 0) return fail(AKMC_ERR_INVALID, "n_sites must be >= 0");
      if (n_sites > 0 && !d_sites) return fail(AKMC_ERR_INVALID, "site list is NULL");
      e = launch_rates_sites(h->d_desc, h->h_desc, h->d_occ, d_sites, n_sites, h->p.precision,
                             d_rates_out, d_ea_out, h->stream);
      break;
    case AKMC_RATES_ALL_SITES:
      if ((reinterpret_cast<uintptr_t>(d_rates_out) & 15) ||
          (reinterpret_cast<uintptr_t>(d_ea_out) & 15))
        return fail(AKMC_ERR_INVALID, "ALL_SITES outputs must be 16-byte aligned");
      e = launch_rates_all(h->d_desc, h->h_desc, h->d_occ, h->p.precision, d_rates_out, d_ea_out,
                           h->stream, &h->timing);
      break;
    default:
      return fail(AKMC_ERR_INVALID, "unknown rates_eval mode");
  }
  if (e != hipSuccess) return hip_fail(e, "rates_eval launch");
  return AKMC_OK;
}

akmc_status akmc_rates_timing(akmc_handle h, void *start_event, void *stop_event) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  h->timing.start = (hipEvent_t)start_event;
  h->timing.stop = (hipEvent_t)stop_event;
  return AKMC_OK;
}

static akmc_status run_loop(akmc_handle h, int64_t n_events, double t_end, akmc_event *d_log);

akmc_status akmc_kmc_step(akmc_handle h, int64_t n_events, akmc_event *d_log) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (n_events < 0) return fail(AKMC_ERR_INVALID, "n_events must be >= 0");
  if (n_events == 0) return AKMC_OK;
  if (h->nv == 0) return fail(AKMC_ERR_FROZEN, "lattice has no vacancies");
  return run_loop(h, n_events, HUGE_VAL, d_log);
}

akmc_status akmc_kmc_run_until(akmc_handle h, double t_end, int64_t max_events, akmc_event *d_log) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (max_events < 0) return fail(AKMC_ERR_INVALID, "max_events must be >= 0");
  if (std::isnan(t_end)) return fail(AKMC_ERR_INVALID, "t_end is NaN");
  if (max_events == 0) return AKMC_OK;
  if (h->nv == 0) return fail(AKMC_ERR_FROZEN, "lattice has no vacancies");
  return run_loop(h, max_events, t_end, d_log);
}

static akmc_status run_loop(akmc_handle h, int64_t n_events, double t_end, akmc_event *d_log) {
  LoopArgs a;
  std::memset(&a, 0, sizeof(a));
  a.descs = h->d_desc;
  a.states = h->d_state;
  a.occ = h->d_occ;
  a.slots = h->d_slots;
  a.order = h->d_order;
  a.queue = h->d_queue;
  a.n_lat = 1;
  a.nv_max = h->nv;
  const bool mlp = h->p.barrier_model == AKMC_BARRIER_MLP;
  if (mlp && !h->mlp_blob) return fail(AKMC_ERR_INVALID, "barrier_model MLP: attach weights with akmc_mlp_attach first");
  a.mlp_blob = h->mlp_blob;
  a.ea_trace = h->d_trace;
  a.t_end = t_end;
  const bool lrn = h->pol_blob || h->pt_blob;
  if (lrn && mlp) return fail(AKMC_ERR_UNSUPPORTED, "the learned runtime forms use the pair barrier model");
  const bool far = h->p.n_shells == 6;
  if (far && event_loop_far_lds_bytes(h->nv, h->p.precision) > kLdsBytes)
    return fail(AKMC_ERR_UNSUPPORTED, "the vacancies' rate tree needs more than the 160 KiB of LDS of a workgroup");
  a.pol_blob = h->pol_blob;
  a.pt_blob = h->pt_blob;
  a.inv_tau = h->inv_tau;
  size_t lrn_lds = 0;
  if (lrn) {
    lrn_lds = event_loop_lrn_lds_bytes(h->nv, h->p.precision, h->pol_blob ? h->pol_dims : nullptr,
                                       h->pt_blob ? h->pt_dims : nullptr);
    if (lrn_lds > kLdsBytes)
      return fail(AKMC_ERR_UNSUPPORTED, "the vacancies' rate tree and the attached networks exceed the "
                                        "160 KiB of LDS of a workgroup");
  }
  // The LDS the loop leaves free in its workgroup holds the coarse vacancy
  // grid (at most 32 KiB).
  {
    const size_t base = far   ? event_loop_far_lds_bytes(h->nv, h->p.precision)
                        : lrn ? lrn_lds
                        : mlp ? event_loop_mlp_lds_bytes(h->nv, h->p.n_species)
                              : event_loop_lds_bytes(h->nv, 64, 1, h->p.precision);
    const int cap = base < kLdsBytes ? (int)std::min<size_t>(kLoopGridWords, (kLdsBytes - base) / 16 * 4) : 0;
    const int reach = far ? 6 : lrn ? 5 : 4;
    a.grid_words = h->p.refresh == AKMC_REFRESH_FULL
                       ? 0
                       : vac_grid(h->p.lx, h->p.ly, h->p.lz, h->nv, reach, cap).words;
    if (lrn)
      lrn_lds = event_loop_lrn_lds_bytes(h->nv, h->p.precision, h->pol_blob ? h->pol_dims : nullptr,
                                         h->pt_blob ? h->pt_dims : nullptr, a.grid_words);
  }
  Schedule s{64, 1, 1};
  for (int64_t done = 0; done < n_events; done += kChunkEvents) {
    const int64_t n = std::min(kChunkEvents, n_events - done);
    a.n_events = n;
    a.log = d_log ? d_log + done : nullptr;
    a.log_stride = n;
    const int full = h->p.refresh == AKMC_REFRESH_FULL;
    hipError_t e = far  ? launch_event_loop_far(a, h->p.precision, full, h->stream)
                   : lrn  ? launch_event_loop_lrn(a, h->p.precision, full, lrn_lds, h->stream)
                   : mlp ? launch_event_loop_mlp(a, full, h->p.n_species, h->stream)
                         : launch_event_loop(a, h->p.precision, full, s, h->stream);
    if (e != hipSuccess) return hip_fail(e, "kmc_step launch");
    h->stepped = true;
  }
  return AKMC_OK;
}

akmc_status akmc_loop_barriers(akmc_handle h, void *d_ea_out) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (!d_ea_out) return fail(AKMC_ERR_INVALID, "output is NULL");
  if (!h->stepped) return fail(AKMC_ERR_INVALID, "no kmc_step has run on this lattice yet");
  const size_t elem = h->p.precision == AKMC_FP32 ? sizeof(float) : sizeof(double);
  HIP_TRY(hipMemcpyAsync(d_ea_out, h->d_trace, elem * 8 * (size_t)h->nv, hipMemcpyDeviceToDevice,
                         h->stream));
  return AKMC_OK;
}

static akmc_status read_state(hipStream_t stream, const LatDesc *d_desc, const LatDesc &hd,
                              const LatState *d_state, const uint8_t *d_occ, const int32_t *d_slots,
                              double *d_scratch, int nv, int64_t nsites, int precision,
                              uint8_t *occ_host, int32_t *slots_host, akmc_summary *out) {
  HIP_TRY(hipStreamSynchronize(stream));
  LatState s;
  HIP_TRY(hipMemcpy(&s, d_state, sizeof(s), hipMemcpyDeviceToHost));
  if (slots_host && nv > 0)
    HIP_TRY(hipMemcpy(slots_host, d_slots, sizeof(int32_t) * nv, hipMemcpyDeviceToHost));
  std::vector<uint8_t> tmp;
  const uint8_t *occ = occ_host;
  if (out && !occ_host) {
    tmp.resize((size_t)nsites);
    occ = tmp.data();
  }
  if (occ) HIP_TRY(hipMemcpy((void *)occ, d_occ, (size_t)nsites, hipMemcpyDeviceToHost));
  if (!out) return AKMC_OK;
  std::memset(out, 0, sizeof(*out));
  out->t = s.t;
  out->n_events = s.n;
  out->gamma_tot = s.gamma_tot;
  out->digest = s.digest;
  out->n_ood = s.n_ood;
  out->n_vacancies = nv;
  out->frozen = s.frozen;
  {
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    out->loop_seconds = khz > 0 ? (double)s.busy_ticks / (1e3 * (double)khz) : 0.0;
  }
  for (int64_t i = 0; i < nsites; ++i) out->species_count[occ[i] & 7] += 1;
  if (nv > 0) {
    // Pair-model barriers and energy changes of the current candidates, for
    // the counts of negative forward and reverse barriers (compared in the
    // precision the kernel computed them in; inadmissible jumps give
    // Ea = +inf and dE = NaN and count in neither).
    hipError_t e = launch_rates_sites(d_desc, hd, d_occ, d_slots, nv, precision,
                                      (void *)(d_scratch + 8 * nv), (void *)d_scratch, stream,
                                      nullptr, (void *)(d_scratch + 16 * nv));
    if (e != hipSuccess) return hip_fail(e, "state_read barriers");
    HIP_TRY(hipStreamSynchronize(stream));
    const size_t n = (size_t)nv * 8;
    if (precision == AKMC_FP32) {
      std::vector<float> ea(n), de(n);
      HIP_TRY(hipMemcpy(ea.data(), d_scratch, sizeof(float) * n, hipMemcpyDeviceToHost));
      HIP_TRY(hipMemcpy(de.data(), d_scratch + 16 * nv, sizeof(float) * n, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < n; ++i) {
        out->n_neg_barrier += ea[i] < 0.0f;
        out->n_neg_reverse += ea[i] < de[i];
      }
    } else {
      std::vector<double> ea(n), de(n);
      HIP_TRY(hipMemcpy(ea.data(), d_scratch, sizeof(double) * n, hipMemcpyDeviceToHost));
      HIP_TRY(hipMemcpy(de.data(), d_scratch + 16 * nv, sizeof(double) * n, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < n; ++i) {
        out->n_neg_barrier += ea[i] < 0.0;
        out->n_neg_reverse += ea[i] < de[i];
      }
    }
  }
  return AKMC_OK;
}

akmc_status akmc_state_read(akmc_handle h, uint8_t *occ_host, int32_t *slot_sites_host,
                            akmc_summary *out) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  return read_state(h->stream, h->d_desc, h->h_desc, h->d_state, h->d_occ, h->d_slots,
                    h->d_scratch, h->nv, h->nsites, h->p.precision, occ_host, slot_sites_host, out);
}

akmc_status akmc_cluster_scratch_bytes(akmc_handle h, size_t *bytes) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (!bytes) return fail(AKMC_ERR_INVALID, "bytes is NULL");
  *bytes = 2 * up(sizeof(int32_t) * (size_t)h->nsites);
  return AKMC_OK;
}

akmc_status akmc_cluster_hist(akmc_handle h, int32_t species, int64_t max_size, int64_t *d_hist,
                              void *d_scratch, size_t scratch_bytes) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (species < 0 || species >= h->p.n_species)
    return fail(AKMC_ERR_INVALID, "species must lie in [0, n_species)");
  if (max_size < 1 || max_size > h->nsites)
    return fail(AKMC_ERR_INVALID, "max_size must lie in [1, number of sites]");
  if (!d_hist) return fail(AKMC_ERR_INVALID, "histogram output is NULL");
  const size_t half = up(sizeof(int32_t) * (size_t)h->nsites);
  if (!d_scratch) return fail(AKMC_ERR_INVALID, "scratch is NULL");
  if (scratch_bytes < 2 * half) return fail(AKMC_ERR_WORKSPACE, "cluster scratch too small");
  int32_t *parent = static_cast<int32_t *>(d_scratch);
  int32_t *size = reinterpret_cast<int32_t *>(static_cast<unsigned char *>(d_scratch) + half);
  const hipError_t e = launch_cluster_hist(h->d_occ, h->p.lx, h->p.ly, h->p.lz, species, max_size,
                                           d_hist, parent, size, h->stream);
  if (e != hipSuccess) return hip_fail(e, "cluster_hist launch");
  return AKMC_OK;
}

akmc_status akmc_cluster_hist_noalloc(akmc_handle h, int32_t species, int64_t max_size,
                                      int64_t *d_hist) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (species < 0 || species >= h->p.n_species)
    return fail(AKMC_ERR_INVALID, "species must lie in [0, n_species)");
  if (max_size < 1 || max_size > h->nsites)
    return fail(AKMC_ERR_INVALID, "max_size must lie in [1, number of sites]");
  if (!d_hist) return fail(AKMC_ERR_INVALID, "histogram output is NULL");
  if (h->nsites > AKMC_CLUSTER_STATIC_MAX_SITES)
    return fail(AKMC_ERR_UNSUPPORTED,
                "lattice has more sites than the library's cluster scratch holds "
                "(AKMC_CLUSTER_STATIC_MAX_SITES = 4194304): use akmc_cluster_hist");
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != h->device) HIP_TRY(hipSetDevice(h->device));
  int32_t *parent = nullptr, *size = nullptr;
  hipError_t e = cluster_static_scratch(&parent, &size);
  const char *what = "cluster scratch address (hipGetSymbolAddress)";
  if (e == hipSuccess) {
    e = launch_cluster_hist(h->d_occ, h->p.lx, h->p.ly, h->p.lz, species, max_size, d_hist,
                            parent, size, h->stream);
    what = "cluster_hist_noalloc launch";
  }
  if (cur != h->device) {
    const hipError_t e2 = hipSetDevice(cur);
    if (e == hipSuccess && e2 != hipSuccess) return hip_fail(e2, "hipSetDevice (restore)");
  }
  if (e != hipSuccess) return hip_fail(e, what);
  return AKMC_OK;
}

akmc_status akmc_lattice_destroy(akmc_handle h) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  delete h;
  return AKMC_OK;
}

const char *akmc_status_string(akmc_status s) {
  switch (s) {
    case AKMC_OK: return "ok";
    case AKMC_ERR_INVALID: return "invalid argument";
    case AKMC_ERR_WORKSPACE: return "workspace too small";
    case AKMC_ERR_HIP: return "HIP runtime error";
    case AKMC_ERR_FROZEN: return "frozen: total rate is zero";
    case AKMC_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char *akmc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ------------------------------------------------------------- batches

struct akmc_batch_s {
  int n_rep;
  int precision, refresh_full;
  hipStream_t stream;
  unsigned char *ws;
  std::vector<akmc_params> params;
  std::vector<LatDesc> h_descs;
  std::vector<int> nv;
  std::vector<int64_t> nsites;
  int nv_max;
  int grid_words;                     // LDS words of each group's vacancy grid
  LatDesc *d_descs;
  LatState *d_states;
  int32_t *d_order, *d_queue, *d_slots;
  double *d_scratch;
  uint8_t *d_occ;
  void *d_trace;                      // barriers the loop last evaluated, [slots][8]
  double *d_w;                        // workload proxy of every replica (Eq. 10)
  bool stepped = false;               // a launch has filled d_trace
  std::vector<int32_t> create_order;  // dispatch order chosen at create
  akmc_schedule sched;
  hipStream_t cap_stream = nullptr;   // capture-only stream (the legacy stream cannot capture)
  std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
};

namespace {

struct BatchLayout {
  size_t descs, states, order, queue, slots, scratch, trace, w, occ, total;
  std::vector<int64_t> occ_off, slot_off;
};

BatchLayout batch_layout(int n_rep, const akmc_params *p, const int32_t *n_vac) {
  BatchLayout b;
  size_t o = 0;
  b.descs = o;  o += up(sizeof(LatDesc) * (size_t)n_rep);
  b.states = o; o += up(sizeof(LatState) * (size_t)n_rep);
  b.order = o;  o += up(sizeof(int32_t) * (size_t)n_rep);
  b.queue = o;  o += up(sizeof(int32_t));
  int64_t ns = 0, nvmax = 1;
  for (int r = 0; r < n_rep; ++r) {
    b.slot_off.push_back(ns);
    ns += n_vac[r];
    nvmax = std::max<int64_t>(nvmax, n_vac[r]);
  }
  b.slots = o;   o += up(sizeof(int32_t) * (size_t)std::max<int64_t>(ns, 1));
  b.scratch = o; o += up(sizeof(double) * 24 * (size_t)nvmax);
  b.trace = o;   o += up(sizeof(double) * 8 * (size_t)std::max<int64_t>(ns, 1));
  b.w = o;       o += up(sizeof(double) * (size_t)n_rep);
  b.occ = o;
  int64_t oo = 0;
  for (int r = 0; r < n_rep; ++r) {
    b.occ_off.push_back(oo);
    oo += (int64_t)up((size_t)n_sites_of(&p[r]));
  }
  o += (size_t)oo;
  b.total = o;
  return b;
}

// The loop keeps every group's tree, lists, boxes and vacancy grid in LDS:
// a schedule is usable only if (64 / lanes) * waves groups of the largest
// replica fit.
bool schedule_fits(int nv_max, int group_lanes, int waves_per_block, int precision, int grid_words) {
  return event_loop_lds_bytes(nv_max, group_lanes, waves_per_block, precision, grid_words) <= kLdsBytes;
}

akmc_status check_schedule(const akmc_schedule *s) {
  if (!s) return fail(AKMC_ERR_INVALID, "schedule is NULL");
  if (s->group_lanes != 8 && s->group_lanes != 16 && s->group_lanes != 32 && s->group_lanes != 64)
    return fail(AKMC_ERR_INVALID, "group_lanes must be 8, 16, 32 or 64");
  if (s->waves_per_block != 1 && s->waves_per_block != 2 && s->waves_per_block != 4)
    return fail(AKMC_ERR_INVALID, "waves_per_block must be 1, 2 or 4");
  if (s->blocks < 0) return fail(AKMC_ERR_INVALID, "blocks must be >= 0");
  if (s->chunk_events <= 0) return fail(AKMC_ERR_INVALID, "chunk_events must be > 0");
  return AKMC_OK;
}

LoopArgs batch_args(const akmc_batch_s *b, int64_t n) {
  LoopArgs a;
  std::memset(&a, 0, sizeof(a));
  a.descs = b->d_descs;
  a.states = b->d_states;
  a.occ = b->d_occ;
  a.slots = b->d_slots;
  a.order = b->d_order;
  a.queue = b->d_queue;
  a.n_lat = b->n_rep;
  a.nv_max = b->nv_max;
  a.grid_words = b->grid_words;
  a.n_events = n;
  a.t_end = HUGE_VAL;
  a.ea_trace = b->d_trace;
  return a;
}

akmc_status batch_launch(akmc_batch_s *b, int64_t n, hipStream_t stream, double t_end = HUGE_VAL) {
  const Schedule s{b->sched.group_lanes, b->sched.waves_per_block, b->sched.blocks};
  LoopArgs a = batch_args(b, n);
  a.t_end = t_end;
  hipError_t e = launch_event_loop(a, b->precision, b->refresh_full, s, stream);
  if (e != hipSuccess) return hip_fail(e, "batch launch");
  b->stepped = true;
  return AKMC_OK;
}

// One chunk as a graph: [queue reset, persistent loop], captured once per
// (chunk, schedule, horizon) on the library's capture stream and replayed
// on the caller's stream.
akmc_status batch_graph_launch(akmc_batch_s *b, int64_t n, double t_end = HUGE_VAL) {
  int64_t tbits;
  std::memcpy(&tbits, &t_end, sizeof(tbits));
  std::vector<int64_t> key{n, b->sched.group_lanes, b->sched.waves_per_block, b->sched.blocks, tbits};
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    akmc_status st = batch_launch(b, n, b->cap_stream, t_end);
    hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
    if (st != AKMC_OK) {
      if (graph) hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    it = b->graphs.emplace(key, exec).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, b->stream));
  b->stepped = true;
  return AKMC_OK;
}

}  // namespace

extern "C" {

akmc_status akmc_batch_workspace_bytes(int32_t n_rep, const akmc_params *p, const int32_t *n_vac,
                                       size_t *bytes) {
  if (n_rep <= 0 || !p || !n_vac || !bytes) return fail(AKMC_ERR_INVALID, "bad batch arguments");
  for (int r = 0; r < n_rep; ++r) {
    akmc_status s = check_params(&p[r]);
    if (s != AKMC_OK) return s;
    if (n_vac[r] < 0 || n_vac[r] > AKMC_MAX_VACANCIES)
      return fail(AKMC_ERR_INVALID, "n_vac must lie in [0, AKMC_MAX_VACANCIES]");
  }
  *bytes = batch_layout(n_rep, p, n_vac).total;
  return AKMC_OK;
}

akmc_status akmc_batch_create(int32_t n_rep, const akmc_params *p, const uint8_t *const *occ_host,
                              const int32_t *const *slot_sites_host, void *d_ws, size_t ws_bytes,
                              void *hip_stream, akmc_batch *out) {
  if (n_rep <= 0 || !p || !occ_host || !d_ws || !out)
    return fail(AKMC_ERR_INVALID, "bad batch arguments");
  if (!aligned(d_ws)) return fail(AKMC_ERR_INVALID, "workspace must be 256-byte aligned");
  std::vector<int32_t> nv(n_rep);
  std::vector<std::vector<int32_t>> slots(n_rep);
  for (int r = 0; r < n_rep; ++r) {
    akmc_status s = check_params(&p[r]);
    if (s != AKMC_OK) return s;
    if (!occ_host[r]) return fail(AKMC_ERR_INVALID, "replica occupancy is NULL");
    if (p[r].precision != p[0].precision || p[r].refresh != p[0].refresh)
      return fail(AKMC_ERR_INVALID, "precision and refresh must agree across replicas");
    if (p[r].barrier_model != AKMC_BARRIER_PAIR)
      return fail(AKMC_ERR_UNSUPPORTED, "batches use the pair barrier model");
    if (p[r].n_shells != 2)
      return fail(AKMC_ERR_UNSUPPORTED, "batches use the first-and-second-neighbour pair model");
    s = build_slots(&p[r], occ_host[r], slot_sites_host ? slot_sites_host[r] : nullptr, slots[r]);
    if (s != AKMC_OK) return s;
    nv[r] = (int32_t)slots[r].size();
  }
  const BatchLayout lay = batch_layout(n_rep, p, nv.data());
  if (ws_bytes < lay.total) return fail(AKMC_ERR_WORKSPACE, "workspace smaller than akmc_batch_workspace_bytes");

  akmc_batch_s *b = new (std::nothrow) akmc_batch_s;
  if (!b) return fail(AKMC_ERR_INVALID, "out of host memory");
  b->n_rep = n_rep;
  b->precision = p[0].precision;
  b->refresh_full = p[0].refresh == AKMC_REFRESH_FULL;
  b->stream = (hipStream_t)hip_stream;
  b->ws = (unsigned char *)d_ws;
  b->params.assign(p, p + n_rep);
  b->nv.assign(nv.begin(), nv.end());
  b->nv_max = 1;
  for (int r = 0; r < n_rep; ++r) b->nv_max = std::max(b->nv_max, nv[r]);
  // Each group's vacancy grid is sized for the largest replica (at most
  // 2 KiB, so that small groups still pack several to a workgroup).
  b->grid_words = 0;
  if (!b->refresh_full)
    for (int r = 0; r < n_rep; ++r)
      b->grid_words = std::max(b->grid_words, vac_grid(p[r].lx, p[r].ly, p[r].lz, nv[r], 4, kBatchGridWords).words);
  b->d_descs = (LatDesc *)(b->ws + lay.descs);
  b->d_states = (LatState *)(b->ws + lay.states);
  b->d_order = (int32_t *)(b->ws + lay.order);
  b->d_queue = (int32_t *)(b->ws + lay.queue);
  b->d_slots = (int32_t *)(b->ws + lay.slots);
  b->d_scratch = (double *)(b->ws + lay.scratch);
  b->d_trace = b->ws + lay.trace;
  b->d_w = (double *)(b->ws + lay.w);
  b->d_occ = b->ws + lay.occ;
  // 8 lanes per replica, or the fewest lanes whose groups fit in LDS (64
  // lanes always fit: one group per wavefront).
  int g0 = 8;
  while (g0 < 64 && !schedule_fits(b->nv_max, g0, 1, b->precision, b->grid_words)) g0 *= 2;
  b->sched = akmc_schedule{g0, 1, 0, 0, 1 << 30};

  std::vector<LatState> states(n_rep);
  std::vector<double> weight(n_rep);
  std::vector<int32_t> order(n_rep);
  for (int r = 0; r < n_rep; ++r) {
    LatDesc d = make_desc(&p[r], nv[r]);
    d.occ_off = lay.occ_off[r];
    d.slot_off = lay.slot_off[r];
    b->h_descs.push_back(d);
    b->nsites.push_back(n_sites_of(&p[r]));
    LatState s;
    std::memset(&s, 0, sizeof(s));
    s.t = p[r].time0;
    s.n = p[r].event_counter0;
    s.digest = p[r].digest0 ? p[r].digest0 : kFnvOffset;
    s.frozen = nv[r] == 0 ? 1 : 0;
    states[r] = s;
    // Work proxy of Eq. 10: event multiplicity times the Arrhenius factor of
    // the matrix barrier at the replica's temperature.
    weight[r] = (double)nv[r] * 8.0 * std::exp(-p[r].e0[0] / (p[r].kb * p[r].temperature));
    order[r] = r;
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return weight[x] > weight[y]; });
  b->create_order = order;
  hipError_t e = hipSuccess;
  const hipStream_t st = b->stream;
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_descs, b->h_descs.data(), sizeof(LatDesc) * n_rep, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_states, states.data(), sizeof(LatState) * n_rep, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_order, order.data(), sizeof(int32_t) * n_rep, hipMemcpyHostToDevice, st);
  for (int r = 0; r < n_rep && e == hipSuccess; ++r) {
    if (nv[r] > 0)
      e = hipMemcpyAsync(b->d_slots + lay.slot_off[r], slots[r].data(), sizeof(int32_t) * nv[r],
                         hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->d_occ + lay.occ_off[r], occ_host[r], (size_t)b->nsites[r],
                         hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "batch_create copies");
  }
  *out = b;
  return AKMC_OK;
}

akmc_status akmc_batch_set_schedule(akmc_batch b, const akmc_schedule *s) {
  if (!b) return fail(AKMC_ERR_INVALID, "batch is NULL");
  akmc_status st = check_schedule(s);
  if (st != AKMC_OK) return st;
  if (!schedule_fits(b->nv_max, s->group_lanes, s->waves_per_block, b->precision, b->grid_words))
    return fail(AKMC_ERR_UNSUPPORTED,
                "schedule needs more than the 160 KiB of LDS of a workgroup: use more lanes per "
                "replica or fewer waves per block");
  b->sched = *s;
  return AKMC_OK;
}

akmc_status akmc_batch_step(akmc_batch b, int64_t n_events_per_replica) {
  if (!b) return fail(AKMC_ERR_INVALID, "batch is NULL");
  if (n_events_per_replica < 0) return fail(AKMC_ERR_INVALID, "n_events must be >= 0");
  int64_t done = 0;
  const int64_t chunk = std::min<int64_t>(b->sched.chunk_events, kChunkEvents);
  while (done < n_events_per_replica) {
    const int64_t n = std::min(chunk, n_events_per_replica - done);
    akmc_status st = b->sched.use_graph ? batch_graph_launch(b, n) : batch_launch(b, n, b->stream);
    if (st != AKMC_OK) return st;
    done += n;
  }
  return AKMC_OK;
}

akmc_status akmc_batch_autotune(akmc_batch b, int64_t trial_events, akmc_schedule *chosen) {
  if (!b) return fail(AKMC_ERR_INVALID, "batch is NULL");
  if (trial_events <= 0) return fail(AKMC_ERR_INVALID, "trial_events must be > 0");
  const int lanes[4] = {8, 16, 32, 64};
  const int waves[2] = {1, 2};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const akmc_schedule keep = b->sched;
  akmc_schedule best = keep;
  float best_ms = 1e30f;
  for (int G : lanes)
    for (int W : waves) {
      if (!schedule_fits(b->nv_max, G, W, b->precision, b->grid_words)) continue;
      akmc_schedule s = keep;
      s.group_lanes = G;
      s.waves_per_block = W;
      s.blocks = 0;
      s.use_graph = 0;
      s.chunk_events = trial_events;
      b->sched = s;
      HIP_TRY(hipEventRecord(e0, b->stream));
      akmc_status st = akmc_batch_step(b, trial_events);
      if (st != AKMC_OK) { b->sched = keep; return st; }
      HIP_TRY(hipEventRecord(e1, b->stream));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) { best_ms = ms; best = s; }
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  best.use_graph = keep.use_graph;
  best.chunk_events = keep.chunk_events;
  b->sched = best;
  if (chosen) *chosen = best;
  return AKMC_OK;
}

akmc_status akmc_batch_state_read(akmc_batch b, int32_t r, uint8_t *occ_host,
                                  int32_t *slot_sites_host, akmc_summary *out) {
  if (!b) return fail(AKMC_ERR_INVALID, "batch is NULL");
  if (r < 0 || r >= b->n_rep) return fail(AKMC_ERR_INVALID, "replica index out of range");
  const LatDesc &d = b->h_descs[r];
  return read_state(b->stream, b->d_descs + r, d, b->d_states + r, b->d_occ + d.occ_off,
                    b->d_slots + d.slot_off, b->d_scratch, b->nv[r], b->nsites[r], b->precision,
                    occ_host, slot_sites_host, out);
}

akmc_status akmc_batch_priority(akmc_batch b, double *d_w_out, int32_t *d_order_out) {
  if (!b) return fail(AKMC_ERR_INVALID, "batch is NULL");
  if (!b->stepped) {
    // A launch with no events evaluates every candidate and fills the trace.
    akmc_status st = batch_launch(b, 0, b->stream);
    if (st != AKMC_OK) return st;
  }
  hipError_t e = launch_priority(b->d_descs, b->d_trace, b->precision == AKMC_FP32, b->n_rep, b->d_w,
                                 b->d_order, b->stream);
  if (e != hipSuccess) return hip_fail(e, "batch priority launch");
  if (d_w_out)
    HIP_TRY(hipMemcpyAsync(d_w_out, b->d_w, sizeof(double) * b->n_rep, hipMemcpyDeviceToDevice, b->stream));
  if (d_order_out)
    HIP_TRY(hipMemcpyAsync(d_order_out, b->d_order, sizeof(int32_t) * b->n_rep, hipMemcpyDeviceToDevice,
                           b->stream));
  return AKMC_OK;
}

akmc_status akmc_batch_run_until(akmc_batch b, double t_end, int64_t max_events_per_replica,
                                 int32_t order) {
  if (!b) return fail(AKMC_ERR_INVALID, "batch is NULL");
  if (std::isnan(t_end)) return fail(AKMC_ERR_INVALID, "t_end is NaN");
  if (max_events_per_replica < 0) return fail(AKMC_ERR_INVALID, "max_events_per_replica must be >= 0");
  if (order == AKMC_ORDER_PRIORITY) {
    akmc_status st = akmc_batch_priority(b, nullptr, nullptr);
    if (st != AKMC_OK) return st;
  } else if (order == AKMC_ORDER_INDEX) {
    hipError_t e = launch_order_index(b->d_order, b->n_rep, b->stream);
    if (e != hipSuccess) return hip_fail(e, "order launch");
  } else if (order == AKMC_ORDER_CREATE) {
    HIP_TRY(hipMemcpyAsync(b->d_order, b->create_order.data(), sizeof(int32_t) * b->n_rep,
                           hipMemcpyHostToDevice, b->stream));
  } else {
    return fail(AKMC_ERR_INVALID, "order must be AKMC_ORDER_PRIORITY, _INDEX or _CREATE");
  }
  int64_t done = 0;
  const int64_t chunk = std::min<int64_t>(b->sched.chunk_events, kChunkEvents);
  while (done < max_events_per_replica) {
    const int64_t n = std::min(chunk, max_events_per_replica - done);
    akmc_status st = b->sched.use_graph ? batch_graph_launch(b, n, t_end)
                                        : batch_launch(b, n, b->stream, t_end);
    if (st != AKMC_OK) return st;
    done += n;
  }
  return AKMC_OK;
}

akmc_status akmc_batch_destroy(akmc_batch b) {
  if (!b) return fail(AKMC_ERR_INVALID, "batch is NULL");
  for (auto &kv : b->graphs) hipGraphExecDestroy(kv.second);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  delete b;
  return AKMC_OK;
}

}  // extern "C"

// ---------------------------------------------------------- surrogate

namespace {
akmc_status check_species(int32_t S) {
  if (S < 2 || S > AKMC_MAX_SPECIES) return fail(AKMC_ERR_INVALID, "n_species must lie in [2, 8]");
  return AKMC_OK;
}
int even_bits(int64_t n) {
  int b = 2;
  while ((int64_t(1) << b) < n) b += 2;
  return b;
}
}  // namespace

extern "C" {

akmc_status akmc_mlp_blob_bytes(int32_t n_species, size_t *bytes) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (!bytes) return fail(AKMC_ERR_INVALID, "bytes is NULL");
  *bytes = mlp_layout(n_species).total;
  return AKMC_OK;
}

akmc_status akmc_mlp_param_count(int32_t n_species, int32_t *count) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (!count) return fail(AKMC_ERR_INVALID, "count is NULL");
  *count = mlp_nparams(n_species);
  return AKMC_OK;
}

static akmc_status write_header(void *d_blob, int32_t S, float mu, float sigma, hipStream_t st) {
  MlpHeader h;
  std::memset(&h, 0, sizeof(h));
  h.S = S;
  h.k1 = mlp_k1(S);
  h.nparams = mlp_nparams(S);
  h.step = 0;
  h.mu = mu;
  h.sigma = sigma;
  HIP_TRY(hipMemcpyAsync(d_blob, &h, sizeof(h), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return AKMC_OK;
}

akmc_status akmc_mlp_init(void *d_blob, int32_t n_species, uint64_t seed, float mu, float sigma,
                          void *hip_stream) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (!d_blob || !aligned(d_blob)) return fail(AKMC_ERR_INVALID, "blob must be 256-byte aligned device memory");
  if (!(sigma > 0.f) || !std::isfinite(mu)) return fail(AKMC_ERR_INVALID, "need finite mu and sigma > 0");
  hipStream_t st = (hipStream_t)hip_stream;
  s = write_header(d_blob, n_species, mu, sigma, st);
  if (s != AKMC_OK) return s;
  hipError_t e = launch_mlp_init((unsigned char *)d_blob, n_species, seed, st);
  if (e != hipSuccess) return hip_fail(e, "mlp_init launch");
  return AKMC_OK;
}

akmc_status akmc_mlp_set_params(void *d_blob, int32_t n_species, const float *host_params,
                                float mu, float sigma, void *hip_stream) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (!d_blob || !aligned(d_blob) || !host_params) return fail(AKMC_ERR_INVALID, "bad blob or parameters");
  if (!(sigma > 0.f)) return fail(AKMC_ERR_INVALID, "sigma must be > 0");
  hipStream_t st = (hipStream_t)hip_stream;
  s = write_header(d_blob, n_species, mu, sigma, st);
  if (s != AKMC_OK) return s;
  const MlpLayout L = mlp_layout(n_species);
  const size_t nb = sizeof(float) * (size_t)mlp_nparams(n_species);
  unsigned char *b = (unsigned char *)d_blob;
  HIP_TRY(hipMemcpyAsync(b + L.params, host_params, nb, hipMemcpyHostToDevice, st));
  std::vector<float> zero((size_t)mlp_nparams(n_species), 0.f);
  HIP_TRY(hipMemcpyAsync(b + L.m, zero.data(), nb, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b + L.v, zero.data(), nb, hipMemcpyHostToDevice, st));
  hipError_t e = launch_mlp_sync(b, n_species, st);
  if (e != hipSuccess) return hip_fail(e, "mlp sync launch");
  HIP_TRY(hipStreamSynchronize(st));
  return AKMC_OK;
}

akmc_status akmc_mlp_get_params(const void *d_blob, int32_t n_species, float *host_params,
                                float *mu, float *sigma, void *hip_stream) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (!d_blob) return fail(AKMC_ERR_INVALID, "blob is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(hipStreamSynchronize(st));
  MlpHeader h;
  HIP_TRY(hipMemcpy(&h, d_blob, sizeof(h), hipMemcpyDeviceToHost));
  if (h.S != n_species) return fail(AKMC_ERR_INVALID, "blob holds a different species count");
  const MlpLayout L = mlp_layout(n_species);
  if (host_params)
    HIP_TRY(hipMemcpy(host_params, (const unsigned char *)d_blob + L.params,
                      sizeof(float) * (size_t)mlp_nparams(n_species), hipMemcpyDeviceToHost));
  if (mu) *mu = h.mu;
  if (sigma) *sigma = h.sigma;
  return AKMC_OK;
}

akmc_status akmc_env_encode(akmc_handle h, int32_t mode, const int32_t *d_sites, int64_t n_sites,
                            uint8_t *d_env, float *d_ea) {
  if (!h || !d_env) return fail(AKMC_ERR_INVALID, "handle or output is NULL");
  if (h->p.n_shells != 2)
    return fail(AKMC_ERR_UNSUPPORTED, "the surrogate's environment covers the first two shells only");
  const int32_t *sites;
  int64_t n;
  switch (mode) {
    case AKMC_RATES_VACANCIES: sites = h->d_slots; n = h->nv; break;
    case AKMC_RATES_SITES:
      if (n_sites < 0 || (n_sites > 0 && !d_sites)) return fail(AKMC_ERR_INVALID, "bad site list");
      sites = d_sites; n = n_sites; break;
    case AKMC_RATES_ALL_SITES: sites = nullptr; n = h->nsites; break;
    default: return fail(AKMC_ERR_INVALID, "unknown mode");
  }
  hipError_t e = launch_env_encode(h->d_desc, h->d_occ, sites, n, d_env, d_ea, h->stream);
  if (e != hipSuccess) return hip_fail(e, "env_encode launch");
  return AKMC_OK;
}

akmc_status akmc_mlp_fit_ood(void *d_blob, int32_t n_species, const uint8_t *d_env, int64_t n,
                             void *hip_stream) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (!d_blob || (n > 0 && !d_env) || n < 0) return fail(AKMC_ERR_INVALID, "bad blob or data");
  hipError_t e = launch_ood_fit((unsigned char *)d_blob, d_env, n, n_species, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "ood_fit launch");
  return AKMC_OK;
}

akmc_status akmc_mlp_forward(const void *d_blob, int32_t n_species, const uint8_t *d_env, int64_t n,
                             float *d_ea, void *hip_stream) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (!d_blob || n < 0 || (n > 0 && (!d_env || !d_ea))) return fail(AKMC_ERR_INVALID, "bad arguments");
  hipError_t e = launch_mlp_forward((const unsigned char *)d_blob, n_species, d_env, n, d_ea,
                                    (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "mlp_forward launch");
  return AKMC_OK;
}

akmc_status akmc_mlp_attach(akmc_handle h, const void *d_blob) {
  if (!h || !d_blob) return fail(AKMC_ERR_INVALID, "handle or blob is NULL");
  if (h->p.barrier_model != AKMC_BARRIER_MLP)
    return fail(AKMC_ERR_INVALID, "lattice was created with the pair barrier model");
  HIP_TRY(hipStreamSynchronize(h->stream));
  MlpHeader hd;
  HIP_TRY(hipMemcpy(&hd, d_blob, sizeof(hd), hipMemcpyDeviceToHost));
  if (hd.S != h->p.n_species || hd.k1 != mlp_k1(hd.S))
    return fail(AKMC_ERR_INVALID, "blob was built for a different species count");
  if (event_loop_mlp_lds_bytes(std::max(h->nv, 1), hd.S) > kLdsBytes)
    return fail(AKMC_ERR_UNSUPPORTED,
                "the vacancies' rate tree and the network's weights exceed the 160 KiB of LDS of a "
                "workgroup: use fewer vacancies or species");
  h->mlp_blob = (const unsigned char *)d_blob;
  return AKMC_OK;
}

akmc_status akmc_mlp_train_workspace_bytes(int32_t n_species, int32_t batch, size_t *bytes) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (batch <= 0 || batch % 16 || !bytes) return fail(AKMC_ERR_INVALID, "batch must be a positive multiple of 16");
  *bytes = mlp_partial_bytes(n_species, batch);
  return AKMC_OK;
}

akmc_status akmc_mlp_train(void *d_blob, int32_t n_species, const uint8_t *d_env, const float *d_ea,
                           int64_t n, const akmc_train_cfg *cfg, float *d_loss, void *d_work,
                           size_t work_bytes, void *hip_stream) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (!d_blob || !d_env || !d_ea || !cfg || !d_work || n <= 0 || n >= (int64_t(1) << 31))
    return fail(AKMC_ERR_INVALID, "bad training arguments");
  if (cfg->batch <= 0 || cfg->batch % 16 || cfg->epochs <= 0 || !(cfg->lr > 0.f))
    return fail(AKMC_ERR_INVALID, "bad training configuration");
  if (work_bytes < mlp_partial_bytes(n_species, cfg->batch)) return fail(AKMC_ERR_WORKSPACE, "training workspace too small");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t per_epoch = (n + cfg->batch - 1) / cfg->batch;
  const int64_t total = per_epoch * cfg->epochs;
  const int bits = even_bits(n);
  int64_t step = 0;
  for (int ep = 0; ep < cfg->epochs; ++ep) {
    uint64_t x[1];
    // one key per epoch, derived from the seed with a 64-bit mix
    uint64_t k = cfg->seed + 0x9E3779B97F4A7C15ull * (uint64_t)(ep + 1);
    k ^= k >> 31; k *= 0xBF58476D1CE4E5B9ull; k ^= k >> 27; k *= 0x94D049BB133111EBull; k ^= k >> 31;
    x[0] = k | 1ull;
    for (int64_t b = 0; b < per_epoch; ++b, ++step) {
      const int rows = (int)std::min<int64_t>(cfg->batch, n - b * cfg->batch);
      const double frac = total > 1 ? (double)step / (double)(total - 1) : 1.0;
      const float lr = (float)(cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) * (1.0 + std::cos(M_PI * frac)));
      hipError_t e = launch_mlp_step((unsigned char *)d_blob, n_species, d_env, d_ea, n, cfg->batch,
                                     rows, b * cfg->batch, cfg->shuffle ? x[0] : 0ull, bits, (float *)d_work, 1, lr,
                                     cfg->beta1, cfg->beta2, cfg->eps, cfg->weight_decay,
                                     (int)(step + 1), nullptr, d_loss ? d_loss + step : nullptr, st);
      if (e != hipSuccess) return hip_fail(e, "mlp training step");
    }
  }
  return AKMC_OK;
}

akmc_status akmc_mlp_grad(const void *d_blob, int32_t n_species, const uint8_t *d_env,
                          const float *d_ea, int32_t n, float *d_grad, float *d_loss, void *d_work,
                          size_t work_bytes, void *hip_stream) {
  akmc_status s = check_species(n_species);
  if (s != AKMC_OK) return s;
  if (!d_blob || !d_env || !d_ea || !d_grad || !d_work || n <= 0) return fail(AKMC_ERR_INVALID, "bad arguments");
  const int batch = (n + 15) / 16 * 16;
  if (work_bytes < mlp_partial_bytes(n_species, batch)) return fail(AKMC_ERR_WORKSPACE, "workspace too small");
  hipError_t e = launch_mlp_step((unsigned char *)d_blob, n_species, d_env, d_ea, n, batch, n, 0, 0,
                                 2, (float *)d_work, 0, 0.f, 0.f, 0.f, 0.f, 0.f, 0, d_grad, d_loss,
                                 (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "mlp_grad launch");
  return AKMC_OK;
}

}  // extern "C"

// ----------------------------------------------------- voxel ensemble

extern "C" {

akmc_status akmc_voxel_grid(const double *T, int32_t nx, int32_t nz, double e_eff, double kb,
                            double tol, int32_t *n_x, int32_t *n_z, double *t_vox, double *worst) {
  if (!T || !n_x || !n_z || !t_vox) return fail(AKMC_ERR_INVALID, "NULL argument");
  if (nx < 1 || nz < 1) return fail(AKMC_ERR_INVALID, "nx and nz must be >= 1");
  if (!(e_eff > 0.0) || !(kb > 0.0) || !(tol > 0.0) || !std::isfinite(e_eff) || !std::isfinite(kb) ||
      !std::isfinite(tol))
    return fail(AKMC_ERR_INVALID, "e_eff, kb and tol must be finite and > 0");
  for (int64_t q = 0; q < (int64_t)nx * nz; ++q)
    if (!(T[q] > 0.0) || !std::isfinite(T[q]))
      return fail(AKMC_ERR_INVALID, "temperature samples must be finite and > 0");
  int gx = 0, gz = 0;
  double w = 0.0;
  if (voxel_grid(T, nx, nz, e_eff, kb, tol, &gx, &gz, t_vox, &w) != 0)
    return fail(AKMC_ERR_INVALID, "no voxel grid meets the tolerance");
  *n_x = gx;
  *n_z = gz;
  if (worst) *worst = w;
  return AKMC_OK;
}

// ------------------------------------------------ learned runtime forms

akmc_status akmc_patchnet_blob_bytes(int32_t n_species, int32_t hidden, int32_t n_out, size_t *bytes) {
  if (n_species < 2 || n_species > AKMC_MAX_SPECIES) return fail(AKMC_ERR_INVALID, "n_species must lie in [2, 8]");
  if (hidden < 8 || hidden > kPatchMaxHidden || hidden % 8 != 0)
    return fail(AKMC_ERR_INVALID, "hidden must be a multiple of 8 in [8, 64]");
  if (n_out != 1 && n_out != 8) return fail(AKMC_ERR_INVALID, "n_out must be 1 (Poisson) or 8 (policy)");
  if (!bytes) return fail(AKMC_ERR_INVALID, "bytes is NULL");
  *bytes = patch_layout(n_species, hidden, n_out).total;
  return AKMC_OK;
}

static float round_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;   // to nearest, ties to even
  float y;
  std::memcpy(&y, &u, 4);
  return y;
}

akmc_status akmc_patchnet_set(void *d_blob, int32_t n_species, int32_t hidden, int32_t n_out,
                              const float *host_params) {
  size_t bytes = 0;
  akmc_status st = akmc_patchnet_blob_bytes(n_species, hidden, n_out, &bytes);
  if (st != AKMC_OK) return st;
  if (!d_blob || !host_params) return fail(AKMC_ERR_INVALID, "NULL blob or parameters");
  if (!aligned(d_blob)) return fail(AKMC_ERR_INVALID, "blob must be 256-byte aligned");
  const PatchLayout L = patch_layout(n_species, hidden, n_out);
  std::vector<unsigned char> img(L.total, 0);
  PatchHeader hdr{};
  hdr.S = n_species;
  hdr.H = hidden;
  hdr.n_out = n_out;
  hdr.nparams = L.nparams;
  hdr.magic = kPatchMagic;
  std::memcpy(img.data(), &hdr, sizeof(hdr));
  float *p = reinterpret_cast<float *>(img.data() + L.params);
  for (int x = 0; x < L.nparams; ++x) {
    const float v = host_params[x];
    if (!std::isfinite(v)) return fail(AKMC_ERR_INVALID, "parameters must be finite");
    const bool bias = (x >= L.ob1 && x < L.oW2) || (x >= L.ob2 && x < L.oW3) || x >= L.ob3;
    p[x] = bias ? v : round_bf16(v);
    if (!std::isfinite(p[x])) return fail(AKMC_ERR_INVALID, "a weight overflows bfloat16");
  }
  HIP_TRY(hipMemcpy(d_blob, img.data(), L.total, hipMemcpyHostToDevice));
  return AKMC_OK;
}

static akmc_status read_patch_header(const void *d_blob, PatchHeader *hdr) {
  if (!d_blob) return fail(AKMC_ERR_INVALID, "blob is NULL");
  HIP_TRY(hipMemcpy(hdr, d_blob, sizeof(PatchHeader), hipMemcpyDeviceToHost));
  if (hdr->magic != kPatchMagic || hdr->S < 2 || hdr->S > AKMC_MAX_SPECIES || hdr->H < 8 ||
      hdr->H > kPatchMaxHidden || hdr->H % 8 != 0 || (hdr->n_out != 1 && hdr->n_out != 8))
    return fail(AKMC_ERR_INVALID, "not a network blob written by akmc_patchnet_set");
  return AKMC_OK;
}

akmc_status akmc_patchnet_get(const void *d_blob, int32_t *n_species, int32_t *hidden, int32_t *n_out,
                              float *host_params) {
  PatchHeader hdr;
  akmc_status st = read_patch_header(d_blob, &hdr);
  if (st != AKMC_OK) return st;
  if (n_species) *n_species = hdr.S;
  if (hidden) *hidden = hdr.H;
  if (n_out) *n_out = hdr.n_out;
  if (host_params) {
    const PatchLayout L = patch_layout(hdr.S, hdr.H, hdr.n_out);
    HIP_TRY(hipMemcpy(host_params, static_cast<const unsigned char *>(d_blob) + L.params,
                      sizeof(float) * (size_t)L.nparams, hipMemcpyDeviceToHost));
  }
  return AKMC_OK;
}

akmc_status akmc_patchnet_eval(akmc_handle h, const void *d_blob, const int32_t *d_sites,
                               int64_t n_sites, float *d_out) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (n_sites < 0) return fail(AKMC_ERR_INVALID, "n_sites must be >= 0");
  if (n_sites > 0 && (!d_sites || !d_out)) return fail(AKMC_ERR_INVALID, "NULL sites or output");
  PatchHeader hdr;
  akmc_status st = read_patch_header(d_blob, &hdr);
  if (st != AKMC_OK) return st;
  if (hdr.S != h->p.n_species) return fail(AKMC_ERR_INVALID, "network species count differs from the lattice's");
  if (h->p.lx < 5 || h->p.ly < 5 || h->p.lz < 5)
    return fail(AKMC_ERR_INVALID, "the 64-neighbour observation needs lattice edges of at least 5 cells");
  hipError_t e = launch_patch_eval(h->d_desc, h->d_occ, static_cast<const unsigned char *>(d_blob), hdr.S,
                                   hdr.H, hdr.n_out, d_sites, n_sites, d_out, h->stream);
  if (e != hipSuccess) return hip_fail(e, "patchnet_eval launch");
  return AKMC_OK;
}

static akmc_status attach_net(akmc_handle h, const void *d_blob, int want_out, const unsigned char **slot,
                              int (&dims)[3]) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (!d_blob) {
    *slot = nullptr;
    return AKMC_OK;
  }
  PatchHeader hdr;
  akmc_status st = read_patch_header(d_blob, &hdr);
  if (st != AKMC_OK) return st;
  if (hdr.n_out != want_out)
    return fail(AKMC_ERR_INVALID, want_out == 8 ? "a policy blob has 8 outputs" : "a Poisson blob has 1 output");
  if (hdr.S != h->p.n_species) return fail(AKMC_ERR_INVALID, "network species count differs from the lattice's");
  if (h->p.lx < 5 || h->p.ly < 5 || h->p.lz < 5)
    return fail(AKMC_ERR_INVALID, "the 64-neighbour observation needs lattice edges of at least 5 cells");
  if (h->p.barrier_model != AKMC_BARRIER_PAIR || h->p.n_shells != 2)
    return fail(AKMC_ERR_UNSUPPORTED, "the learned runtime forms use the first-and-second-neighbour pair model");
  const int d[3] = {hdr.S, hdr.H, hdr.n_out};
  const unsigned char *pol = want_out == 8 ? static_cast<const unsigned char *>(d_blob) : h->pol_blob;
  const unsigned char *pt = want_out == 1 ? static_cast<const unsigned char *>(d_blob) : h->pt_blob;
  const size_t lds = event_loop_lrn_lds_bytes(h->nv, h->p.precision, pol ? (want_out == 8 ? d : h->pol_dims) : nullptr,
                                              pt ? (want_out == 1 ? d : h->pt_dims) : nullptr);
  if (lds > kLdsBytes)
    return fail(AKMC_ERR_UNSUPPORTED, "the vacancies' rate tree and the attached networks exceed the 160 KiB "
                                      "of LDS of a workgroup");
  *slot = static_cast<const unsigned char *>(d_blob);
  for (int q = 0; q < 3; ++q) dims[q] = d[q];
  return AKMC_OK;
}

akmc_status akmc_policy_attach(akmc_handle h, const void *d_blob, float tau) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  if (d_blob && !(tau > 0.0f && std::isfinite(tau))) return fail(AKMC_ERR_INVALID, "tau must be finite and > 0");
  akmc_status st = attach_net(h, d_blob, 8, &h->pol_blob, h->pol_dims);
  if (st == AKMC_OK && d_blob) h->inv_tau = 1.0f / tau;
  return st;
}

akmc_status akmc_poisson_attach(akmc_handle h, const void *d_blob) {
  if (!h) return fail(AKMC_ERR_INVALID, "handle is NULL");
  return attach_net(h, d_blob, 1, &h->pt_blob, h->pt_dims);
}

}  // extern "C"
