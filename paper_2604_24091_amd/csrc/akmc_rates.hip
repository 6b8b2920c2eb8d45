// Rate evaluation outside the event loop.
//
//  k_rates_sites: one thread per candidate (site, direction) of a site
//    list; gathers the bond counts straight from the occupancy and uses
//    exactly the arithmetic of the event loop, so VACANCIES mode returns
//    the loop's rates bit for bit.
//
//  k_rates_all: the bulk sweep over every lattice site (a vacancy placed
//    at each site in turn), nominally bound by the HBM write of the [N][8]
//    rate array.  A workgroup stages a brick of occupancy with a halo of
//    2 cells (4 along x, for dword-aligned rows) in LDS.  With the field
//        G'_A(q) = sum over the 14 bonds of q of D'_k[A][s_n],
//        D'_k[A][s] = D_k[A][s] - D_k[A][Fe],
//    the energy change of the jump p <- j (species A = s_j) is
//        dE = G'_A(p) - G'_A(j) + D1[A][s_p] - D1[A][A],
//    which equals the bond-count form up to rounding; measuring the field
//    against the all-Fe environment keeps it near zero, so binary32 keeps
//    its relative accuracy.  A target enters with its own species only.

#include <hip/hip_runtime.h>

#include "akmc_device.hpp"
#include "akmc_internal.hpp"

namespace akmc {

template <class Real> struct Tab;
template <> struct Tab<double> {
  __device__ static const double *D1(const LatDesc *d) { return d->D1; }
  __device__ static const double *D2(const LatDesc *d) { return d->D2; }
  __device__ static const double *e0(const LatDesc *d) { return d->e0; }
  __device__ static const double *Ds1(const LatDesc *d) { return d->Ds1; }
  __device__ static const double *Ds2(const LatDesc *d) { return d->Ds2; }
  __device__ static const double *K(const LatDesc *d) { return d->K; }
  __device__ static double nu(const LatDesc *d) { return d->nu; }
  __device__ static double kT(const LatDesc *d) { return d->kT; }
  __device__ static double beta(const LatDesc *d) { return d->beta; }
};
template <> struct Tab<float> {
  __device__ static const float *D1(const LatDesc *d) { return d->D1f; }
  __device__ static const float *D2(const LatDesc *d) { return d->D2f; }
  __device__ static const float *e0(const LatDesc *d) { return d->e0f; }
  __device__ static const float *Ds1(const LatDesc *d) { return d->Ds1f; }
  __device__ static const float *Ds2(const LatDesc *d) { return d->Ds2f; }
  __device__ static const float *K(const LatDesc *d) { return d->Kf; }
  __device__ static float nu(const LatDesc *d) { return d->nuf; }
  __device__ static float kT(const LatDesc *d) { return d->kTf; }
  __device__ static float beta(const LatDesc *d) { return d->betaf; }
};

template <class Real> __device__ __forceinline__ Real inf_of();
template <> __device__ __forceinline__ double inf_of<double>() { return __builtin_huge_val(); }
template <> __device__ __forceinline__ float inf_of<float>() { return __builtin_huge_valf(); }

// ----------------------------------------------------------- site list

template <class Real>
__global__ __launch_bounds__(256) void k_rates_sites(const LatDesc *__restrict__ d,
                                                     const uint8_t *__restrict__ occ,
                                                     const int32_t *__restrict__ sites,
                                                     int64_t n_sites, Real *__restrict__ rates,
                                                     Real *__restrict__ ea) {
  __shared__ Real sD1[64], sD2[64], se0[8];
  const int tid = threadIdx.x;
  if (tid < 64) { sD1[tid] = Tab<Real>::D1(d)[tid]; sD2[tid] = Tab<Real>::D2(d)[tid]; }
  if (tid < 8) se0[tid] = Tab<Real>::e0(d)[tid];
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * 256 + tid;
  if (c >= n_sites * 8) return;
  const int64_t a = c >> 3;
  const int k = (int)(c & 7);
  const Geo g = make_geo(d->lx, d->ly, d->lz);
  const int S = d->S, V = S - 1;
  const int i = sites ? sites[a] : (int)a;
  if (i < 0 || i >= 2 * g.ncell) {  // a listed site outside the lattice: no gather
    rates[c] = Real(__builtin_nan(""));
    if (ea) ea[c] = Real(__builtin_nan(""));
    return;
  }
  int X, Y, Z;
  pos_of(g, i, X, Y, Z);
  const int JX = wrapc(X + dir_sx(k), g.X2), JY = wrapc(Y + dir_sy(k), g.Y2),
            JZ = wrapc(Z + dir_sz(k), g.Z2);
  const int A = occ[site_of(g, JX, JY, JZ)];
  Real r, e;
  if (A == V) {
    r = Real(0);
    e = inf_of<Real>();
  } else {
    uint32_t c1i = 0, c1j = 0, c2i = 0, c2j = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int dx = dir_sx(q), dy = dir_sy(q), dz = dir_sz(q);
      c1i += onehot(occ[site_of(g, wrapc(X + dx, g.X2), wrapc(Y + dy, g.Y2), wrapc(Z + dz, g.Z2))]);
      c1j += onehot(occ[site_of(g, wrapc(JX + dx, g.X2), wrapc(JY + dy, g.Y2), wrapc(JZ + dz, g.Z2))]);
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const int s = (m & 1) ? -2 : 2, ax = m >> 1;
      const int dx = ax == 0 ? s : 0, dy = ax == 1 ? s : 0, dz = ax == 2 ? s : 0;
      c2i += onehot(occ[site_of(g, wrapc(X + dx, g.X2), wrapc(Y + dy, g.Y2), wrapc(Z + dz, g.Z2))]);
      c2j += onehot(occ[site_of(g, wrapc(JX + dx, g.X2), wrapc(JY + dy, g.Y2), wrapc(JZ + dz, g.Z2))]);
    }
    c1i -= onehot(A);           // N1(i) without j
    c1j -= onehot(occ[i]);      // N1(j) without i
    const Real de = delta_e_counts<Real>(c1i, c1j, c2i, c2j, sD1 + 8 * A, sD2 + 8 * A);
    e = se0[A] + Real(0.5) * de;
    r = rate_from_barrier(e, Tab<Real>::nu(d), Tab<Real>::kT(d));
  }
  rates[c] = r;
  if (ea) ea[c] = e;
}

// ---------------------------------------------------------- bulk sweep

template <class Real> struct Sweep;
// The rate of candidate p <- j as one exponential of the sum of a per-site
// term and a per-target term (see k_rates_all):
//   binary64:  ln r    = (Cn[A][s_p]  - h G'_A(p)) + h G'_{s_j}(j),  h = beta/2
//   binary32:  log2 r  = (C2f[A][s_p] - h G'_A(p)) + h G'_{s_j}(j),  h = (beta/2) log2(e)
template <> struct Sweep<double> {
  __device__ static double h(const LatDesc *d) { return d->half_beta; }
  __device__ static double table(const LatDesc *d, int i) { return d->Cn[i]; }
  __device__ static double target(double h, double H) { return h * H; }
  __device__ static double site(double c, double h, double g) { return c - h * g; }
  __device__ static double masked_site() { return -__builtin_huge_val(); }
  __device__ static double rate(double t, double e) { return exp(t + e); }
};
template <> struct Sweep<float> {
  __device__ static float h(const LatDesc *d) { return d->h2f; }
  __device__ static float table(const LatDesc *d, int i) { return d->C2f[i]; }
  __device__ static float target(float h, float H) { return h * H; }
  __device__ static float site(float c, float h, float g) { return c - h * g; }
  __device__ static float masked_site() { return -__builtin_huge_valf(); }
  __device__ static float rate(float t, float e) { return __builtin_amdgcn_exp2f(t + e); }
};

constexpr int kSweepThreads = 512;

template <int TX, int TY, int TZ>
struct SweepShape {
  // Occupancy brick: cells [-2, T+2) in y and z and [-8, T+8) in x, so that
  // every row starts on an 8-byte boundary and can be staged in 8-byte
  // vectors (TX a multiple of 8).
  static constexpr int PX = 8;
  static constexpr int EX = TX + 2 * PX, EY = TY + 4, EZ = TZ + 4, EV = EX * EY * EZ;
  static constexpr int ROWS = 2 * EY * EZ;
  static constexpr int HX = TX + 1, HY = TY + 1, HZ = TZ + 1, HV = HX * HY * HZ;  // field region
  static constexpr int NT = 2 * TX * TY * TZ;                                     // brick sites
  static constexpr int OCC_BYTES = (2 * EV + 15) & ~15;
  // per region site: bond counts (2 words), the target term, the field
  // (barrier output only); site terms: binary32 per lane (S planes of 256),
  // binary64 per brick site (S-1 planes of NT, twice with the barrier output)
  __host__ __device__ static constexpr size_t terms(int S, size_t real, bool with_ea) {
    return real == 4 ? (size_t)S * kSweepThreads : (size_t)(S - 1) * NT * (with_ea ? 2 : 1);
  }
  static size_t lds_bytes(int S, size_t real, bool with_ea) {
    return OCC_BYTES + (size_t)2 * HV * (8 + real + (with_ea ? real : 0)) +
           terms(S, real, with_ea) * real;
  }
};

// Region layout: corners (b = 0) at cells [0, T+1) and centres (b = 1) at
// cells [-1, T) of the brick, each stored at index h = c + b.  The targets
// of a corner at cell c are the centres at cells c - 1 + [s > 0], those of
// a centre the corners at c + [s > 0]; both sit at index h = c + [s > 0] of
// the other sublattice.
//
// With the field G'_A(q) = sum_s n1_s(q) Ds1[A][s] + n2_s(q) Ds2[A][s], the
// rate of p <- j (species A = s_j) is, in logarithms,
//   ln r = Cn[A][s_p] - h G'_A(p) + h G'_A(j),
// and a target enters only with its own species (A = s_j).  Phase 2 stores
// per region site its counts and its target term; phase 3 forms per brick
// site the term of every mover species (a per-lane table in LDS, whose
// entry for the vacancy code gives a zero rate) and combines it with the
// target terms of the 8 neighbours.
//
// Output: one lane per site writes its 8 rates as two (binary32) or four
// (binary64) 16-byte non-temporal vectors; neighbouring lanes write
// neighbouring 32- or 64-byte rows.
template <int TX, int TY, int TZ, int S, class Real, bool WITH_EA>
__global__ __launch_bounds__(kSweepThreads) void k_rates_all(const LatDesc *__restrict__ d,
                                                             const uint8_t *__restrict__ occ,
                                                             Real *__restrict__ rates,
                                                             Real *__restrict__ ea) {
  using Sh = SweepShape<TX, TY, TZ>;
  using SW = Sweep<Real>;
  constexpr int EX = Sh::EX, EY = Sh::EY, EZ = Sh::EZ, EV = Sh::EV, PX = Sh::PX;
  constexpr int HX = Sh::HX, HY = Sh::HY, HV = Sh::HV;
  constexpr int V = S - 1, NA = S - 1;
  constexpr int VW = 16 / (int)sizeof(Real);  // candidates per 16-byte store
  typedef Real vecw __attribute__((ext_vector_type(VW)));
  extern __shared__ __align__(16) unsigned char sweep_lds[];
  uint8_t *socc = sweep_lds;
  uint2 *sCnt = (uint2 *)(sweep_lds + Sh::OCC_BYTES);
  Real *sE = (Real *)(sCnt + 2 * HV);
  Real *sT = sE + 2 * HV;              // site terms
  Real *sH = sT + Sh::terms(S, sizeof(Real), WITH_EA);  // WITH_EA only
  __shared__ Real sC[64], sDs1[64], sDs2[64], se0[8], sK[64];

  const int tid = threadIdx.x;
  const int lx = d->lx, ly = d->ly, lz = d->lz;
  const int ncell = lx * ly * lz;
  if (tid < 64) {
    sC[tid] = SW::table(d, tid);
    sDs1[tid] = Tab<Real>::Ds1(d)[tid];
    sDs2[tid] = Tab<Real>::Ds2(d)[tid];
    if (WITH_EA) sK[tid] = Tab<Real>::K(d)[tid];
  }
  if (WITH_EA && tid < 8) se0[tid] = Tab<Real>::e0(d)[tid];

  const int ntx = (lx + TX - 1) / TX, nty = (ly + TY - 1) / TY;
  const int tile = blockIdx.x;
  const int x0 = (tile % ntx) * TX;
  const int y0 = ((tile / ntx) % nty) * TY;
  const int z0 = (tile / (ntx * nty)) * TZ;

  // Phase 1: occupancy brick of both sublattices, as 4*species (the shift of
  // that species' count nibble).  One conditional wrap per axis suffices
  // when every edge exceeds the brick (then x is staged in aligned dwords if
  // lx is a multiple of 4); small lattices take the general modulo byte by
  // byte.
  // x spans [x0 - PX, x0 + TX + PX) with x0 <= lx - 1: one wrap suffices
  // when lx >= TX + PX; y and z span 2 cells either side.
  const bool simple = lx >= TX + PX && ly > TY + 2 && lz > TZ + 2;
  static_assert(TX % 8 == 0 && PX % 8 == 0, "brick rows must start on 8-byte boundaries");
  if (simple && (lx & 7) == 0) {
    // EX / 8 vectors per row; with lx a multiple of 8 a vector never
    // straddles the periodic seam.
    constexpr int QW = EX / 8;
    for (int i = tid; i < Sh::ROWS * QW; i += kSweepThreads) {
      const int row = i / QW, w = i % QW;
      const int ey = row % EY;
      const int bz = row / EY;
      const int ez = bz % EZ;
      const int b = bz / EZ;
      int gx = x0 - PX + 8 * w, gy = y0 + ey - 2, gz = z0 + ez - 2;
      gx += gx < 0 ? lx : 0;  gx -= gx >= lx ? lx : 0;
      gy += gy < 0 ? ly : 0;  gy -= gy >= ly ? ly : 0;
      gz += gz < 0 ? lz : 0;  gz -= gz >= lz ? lz : 0;
      uint2 v = *(const uint2 *)(occ + (size_t)b * ncell + (gz * ly + gy) * lx + gx);
      v.x <<= 2; v.y <<= 2;  // codes < 8: no carry between bytes
      *(uint2 *)(socc + row * EX + 8 * w) = v;
    }
  } else if (simple && (lx & 3) == 0) {
    // 16 lanes per brick row (DW <= 16 dwords used), rows in pow-2 strides.
    constexpr int DW = EX / 4;
    static_assert(DW <= 16, "brick row wider than 16 dwords");
    const int w = tid & 15;
    for (int row = tid >> 4; row < Sh::ROWS; row += kSweepThreads / 16) {
      if (w >= DW) continue;
      const int ey = row % EY;
      const int bz = row / EY;
      const int ez = bz % EZ;
      const int b = bz / EZ;
      int gx = x0 - PX + 4 * w, gy = y0 + ey - 2, gz = z0 + ez - 2;
      gx += gx < 0 ? lx : 0;  gx -= gx >= lx ? lx : 0;
      gy += gy < 0 ? ly : 0;  gy -= gy >= ly ? ly : 0;
      gz += gz < 0 ? lz : 0;  gz -= gz >= lz ? lz : 0;
      const uint32_t v = *(const uint32_t *)(occ + (size_t)b * ncell + (gz * ly + gy) * lx + gx);
      *(uint32_t *)(socc + row * EX + 4 * w) = v << 2;  // codes < 8: no carry between bytes
    }
  } else {
    for (int r = tid; r < 2 * EV; r += kSweepThreads) {
      const int ex = r % EX;
      const int row = r / EX;
      const int ey = row % EY;
      const int bz = row / EY;
      const int ez = bz % EZ;
      const int b = bz / EZ;
      int gx = x0 + ex - PX, gy = y0 + ey - 2, gz = z0 + ez - 2;
      if (simple) {
        gx += gx < 0 ? lx : 0;  gx -= gx >= lx ? lx : 0;
        gy += gy < 0 ? ly : 0;  gy -= gy >= ly ? ly : 0;
        gz += gz < 0 ? lz : 0;  gz -= gz >= lz ? lz : 0;
      } else {
        gx = ((gx % lx) + lx) % lx;
        gy = ((gy % ly) + ly) % ly;
        gz = ((gz % lz) + lz) % lz;
      }
      socc[r] = (uint8_t)(occ[(size_t)b * ncell + (gz * ly + gy) * lx + gx] << 2);
    }
  }
  __syncthreads();

  auto oidx = [&](int b, int cx, int cy, int cz) {
    return b * EV + ((cz + 2) * EY + (cy + 2)) * EX + (cx + PX);
  };
  const Real h = SW::h(d);

  // Phase 2: for every region site q the bond counts (kept for the vacancy
  // role) and the target term from the field of q's own species.
  // Threads sit on fixed columns hx of the region's rows (HX sites each);
  // a pass covers RPP whole rows.
  constexpr int RPP = kSweepThreads / HX;
  const int hx = tid % HX, row0 = tid / HX;
  for (int row = row0; row0 < RPP && row < 2 * HY * Sh::HZ; row += RPP) {
    const int r = row * HX + hx;
    const int hy = row % HY;
    const int bz = row / HY;
    const int hz = bz % Sh::HZ;
    const int b = bz / Sh::HZ;
    const int cx = hx - b, cy = hy - b, cz = hz - b;
    // First shell: the other sublattice's cube of cells c-1..c (corner) or
    // c..c+1 (centre); second shell: same sublattice, +-1 cell per axis.
    const uint8_t *s1 = socc + oidx(1 - b, cx - 1 + b, cy - 1 + b, cz - 1 + b);
    const uint8_t *s2 = socc + oidx(b, cx, cy, cz);
    uint32_t c1 = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) c1 += 1u << s1[((q >> 2) & 1) + ((q >> 1) & 1) * EX + (q & 1) * (EX * EY)];
    const uint32_t c2 = (1u << s2[1]) + (1u << s2[-1]) + (1u << s2[EX]) + (1u << s2[-EX]) +
                        (1u << s2[EX * EY]) + (1u << s2[-EX * EY]);
    sCnt[r] = make_uint2(c1, c2);
    // A vacancy is never a target: its entry is computed for a mover, unused.
    const int A = min((int)s2[0] >> 2, NA - 1);
    Real g = Real(0);
#pragma unroll
    for (int s = 1; s < S; ++s)
      g = fma((Real)nib(c2, s), sDs2[A * S + s], fma((Real)nib(c1, s), sDs1[A * S + s], g));
    sE[r] = SW::target(h, g);
    if (WITH_EA) sH[r] = g;
  }
  __syncthreads();

  // Phase 3: the 8 candidates of every brick site.  The field of the
  // vacancy site for every mover species comes from its counts, with the
  // same chain as above.
  if constexpr (sizeof(Real) == 8) {
    // binary64: one lane per site forms the site terms (planes of NT), then
    // four lanes per site combine them with the target terms, two
    // candidates each, so that the costly exponentials run in short
    // independent chains.
    Real *sTs = sT, *sGs = sT + NA * Sh::NT;
    for (int t = tid; t < Sh::NT; t += kSweepThreads) {
      const int cx = t % TX;
      const int row = t / TX;
      const int cy = row % TY;
      const int bz = row / TY;
      const int cz = bz % TZ;
      const int b = bz / TZ;
      const int sp = socc[oidx(b, cx, cy, cz)] >> 2;
      const int ip = b * HV + ((cz + b) * HY + (cy + b)) * HX + (cx + b);
      const uint2 cn = sCnt[ip];
      Real g[NA];
#pragma unroll
      for (int A = 0; A < NA; ++A) g[A] = Real(0);
#pragma unroll
      for (int s = 1; s < S; ++s) {
        const Real n1 = (Real)nib(cn.x, s), n2 = (Real)nib(cn.y, s);
#pragma unroll
        for (int A = 0; A < NA; ++A) g[A] = fma(n2, sDs2[A * S + s], fma(n1, sDs1[A * S + s], g[A]));
      }
#pragma unroll
      for (int A = 0; A < NA; ++A) {
        sTs[A * Sh::NT + t] = SW::site(sC[A * S + sp], h, g[A]);
        if (WITH_EA) sGs[A * Sh::NT + t] = g[A];
      }
    }
    __syncthreads();
    constexpr int LPS = 8 / VW;
    for (int it = tid; it < Sh::NT * LPS; it += kSweepThreads) {
      const int t = it / LPS, part = it % LPS;
      const int cx = t % TX;
      const int row = t / TX;
      const int cy = row % TY;
      const int bz = row / TY;
      const int cz = bz % TZ;
      const int b = bz / TZ;
      const int gx = x0 + cx, gy = y0 + cy, gz = z0 + cz;
      if (gx >= lx || gy >= ly || gz >= lz) continue;
      const int sp = socc[oidx(b, cx, cy, cz)] >> 2;
      const int ij0 = (1 - b) * HV + (cz * HY + cy) * HX + cx;
      const uint8_t *s1 = socc + oidx(1 - b, cx - 1 + b, cy - 1 + b, cz - 1 + b);
      vecw w, we;
#pragma unroll
      for (int c = 0; c < VW; ++c) {
        const int k = part * VW + c;
        const int px = (k >> 2) & 1, py = (k >> 1) & 1, pz = k & 1;
        const int A = s1[px + py * EX + pz * (EX * EY)] >> 2;
        const int Ac = min(A, NA - 1);
        const int ij = ij0 + (pz * HY + py) * HX + px;
        const Real ts = A == V ? SW::masked_site() : sTs[Ac * Sh::NT + t];
        w[c] = SW::rate(ts, sE[ij]);
        if (WITH_EA)
          we[c] = A == V ? inf_of<Real>()
                         : se0[Ac] + Real(0.5) * ((sGs[Ac * Sh::NT + t] - sH[ij]) + sK[Ac * S + sp]);
      }
      const size_t site = (unsigned)(b * ncell + (gz * ly + gy) * lx + gx);
      __builtin_nontemporal_store(w, (vecw *)(rates + site * 8) + part);
      if (WITH_EA) __builtin_nontemporal_store(we, (vecw *)(ea + site * 8) + part);
    }
    return;
  }
  // binary32: one lane per site; the grid-uniform tables sit in scalar
  // registers and the site terms in a per-lane LDS table.
  const Real *Ds1 = Tab<Real>::Ds1(d), *Ds2 = Tab<Real>::Ds2(d);
  Real *myT = sT + tid;
  myT[NA * kSweepThreads] = SW::masked_site();  // code of the vacancy
  for (int t = tid; t < Sh::NT; t += kSweepThreads) {
    const int cx = t % TX;
    const int row = t / TX;
    const int cy = row % TY;
    const int bz = row / TY;
    const int cz = bz % TZ;
    const int b = bz / TZ;
    const int gx = x0 + cx, gy = y0 + cy, gz = z0 + cz;
    if (gx >= lx || gy >= ly || gz >= lz) continue;
    const int sp = socc[oidx(b, cx, cy, cz)] >> 2;
    const int ip = b * HV + ((cz + b) * HY + (cy + b)) * HX + (cx + b);
    const int ij0 = (1 - b) * HV + (cz * HY + cy) * HX + cx;
    const uint8_t *s1 = socc + oidx(1 - b, cx - 1 + b, cy - 1 + b, cz - 1 + b);
    const uint2 cn = sCnt[ip];
    Real g[NA];
#pragma unroll
    for (int A = 0; A < NA; ++A) g[A] = Real(0);
#pragma unroll
    for (int s = 1; s < S; ++s) {
      const Real n1 = (Real)nib(cn.x, s), n2 = (Real)nib(cn.y, s);
#pragma unroll
      for (int A = 0; A < NA; ++A) g[A] = fma(n2, Ds2[A * S + s], fma(n1, Ds1[A * S + s], g[A]));
    }
#pragma unroll
    for (int A = 0; A < NA; ++A) myT[A * kSweepThreads] = SW::site(sC[A * S + sp], h, g[A]);
    // Site indices stay below 2^31 (checked at create).
    const size_t site = (unsigned)(b * ncell + (gz * ly + gy) * lx + gx);
    vecw *out = (vecw *)(rates + site * 8);
    vecw *oe = WITH_EA ? (vecw *)(ea + site * 8) : nullptr;
    constexpr int NVEC = 8 / VW;
#pragma unroll
    for (int v = 0; v < NVEC; ++v) {
      vecw w, we;
#pragma unroll
      for (int c = 0; c < VW; ++c) {
        const int k = v * VW + c;
        const int px = (k >> 2) & 1, py = (k >> 1) & 1, pz = k & 1;
        const int A = s1[px + py * EX + pz * (EX * EY)] >> 2;
        const int ij = ij0 + (pz * HY + py) * HX + px;
        w[c] = SW::rate(myT[A * kSweepThreads], sE[ij]);
        if (WITH_EA) {
          Real ga = g[0];
#pragma unroll
          for (int m = 1; m < NA; ++m) ga = A == m ? g[m] : ga;
          const int Ac = min(A, NA - 1);
          we[c] = A == V ? inf_of<Real>() : se0[Ac] + Real(0.5) * ((ga - sH[ij]) + sK[Ac * S + sp]);
        }
      }
      __builtin_nontemporal_store(w, out + v);
      if (WITH_EA) __builtin_nontemporal_store(we, oe + v);
    }
  }
}

// ------------------------------------------------------------ launchers

hipError_t launch_rates_sites(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                              const int32_t *sites, int64_t n_sites, int precision, void *rates,
                              void *ea, hipStream_t stream) {
  if (n_sites <= 0) return hipSuccess;
  const int64_t nthreads = n_sites * 8;
  const unsigned blocks = (unsigned)((nthreads + 255) / 256);
  if (precision == AKMC_FP32)
    hipLaunchKernelGGL((k_rates_sites<float>), dim3(blocks), dim3(256), 0, stream, d_desc, occ,
                       sites, n_sites, (float *)rates, (float *)ea);
  else
    hipLaunchKernelGGL((k_rates_sites<double>), dim3(blocks), dim3(256), 0, stream, d_desc, occ,
                       sites, n_sites, (double *)rates, (double *)ea);
  return hipGetLastError();
}

template <int TX, int TY, int TZ, int S, class Real>
static hipError_t launch_sweep(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                               void *rates, void *ea, hipStream_t stream) {
  using Sh = SweepShape<TX, TY, TZ>;
  const unsigned tiles = (unsigned)(((h.lx + TX - 1) / TX) * ((h.ly + TY - 1) / TY) *
                                    ((h.lz + TZ - 1) / TZ));
  const size_t lds = Sh::lds_bytes(S, sizeof(Real), ea != nullptr);
  auto k = ea ? k_rates_all<TX, TY, TZ, S, Real, true> : k_rates_all<TX, TY, TZ, S, Real, false>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3(tiles), dim3(kSweepThreads), lds, stream, d_desc, occ, (Real *)rates,
                     (Real *)ea);
  return hipGetLastError();
}

template <int S, class Real>
static hipError_t launch_sweep_s(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                                 void *rates, void *ea, hipStream_t stream) {
  // binary64 takes the narrower brick so that several workgroups share a CU
  if (sizeof(Real) == 8) return launch_sweep<16, 4, 4, S, Real>(d_desc, h, occ, rates, ea, stream);
  return launch_sweep<32, 4, 4, S, Real>(d_desc, h, occ, rates, ea, stream);
}

template <class Real>
static hipError_t launch_sweep_r(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                                 void *rates, void *ea, hipStream_t stream) {
  switch (h.S) {
    case 2: return launch_sweep_s<2, Real>(d_desc, h, occ, rates, ea, stream);
    case 3: return launch_sweep_s<3, Real>(d_desc, h, occ, rates, ea, stream);
    case 4: return launch_sweep_s<4, Real>(d_desc, h, occ, rates, ea, stream);
    case 5: return launch_sweep_s<5, Real>(d_desc, h, occ, rates, ea, stream);
    case 6: return launch_sweep_s<6, Real>(d_desc, h, occ, rates, ea, stream);
    case 7: return launch_sweep_s<7, Real>(d_desc, h, occ, rates, ea, stream);
    case 8: return launch_sweep_s<8, Real>(d_desc, h, occ, rates, ea, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_rates_all(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                            int precision, void *rates, void *ea, hipStream_t stream) {
  if (precision == AKMC_FP32) return launch_sweep_r<float>(d_desc, h, occ, rates, ea, stream);
  return launch_sweep_r<double>(d_desc, h, occ, rates, ea, stream);
}

}  // namespace akmc
