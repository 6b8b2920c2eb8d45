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
//    2 cells (8 along x, for 8-byte aligned rows) in LDS.  With the field
//        G'_A(q) = sum over the 14 bonds of q of D'_k[A][s_n],
//        D'_k[A][s] = D_k[A][s] - D_k[A][Fe],
//    the energy change of the jump p <- j (species A = s_j) is
//        dE = G'_A(p) - G'_A(j) + D1[A][s_p] - D1[A][A],
//    which equals the bond-count form up to rounding; measuring the field
//    against the all-Fe environment keeps it near zero, so binary32 keeps
//    its relative accuracy.  A target enters with its own species only.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "akmc_device.hpp"
#include "akmc_internal.hpp"
#include "akmc_patch.hpp"

namespace akmc {

template <class Real> struct Tab;
template <> struct Tab<double> {
  __device__ static const double *D1(const LatDesc *d) { return d->D1; }
  __device__ static const double *D2(const LatDesc *d) { return d->D2; }
  __device__ static const double *e0(const LatDesc *d) { return d->e0; }
  __device__ static const double *Hs1(const LatDesc *d) { return d->Hs1; }
  __device__ static const double *Hs2(const LatDesc *d) { return d->Hs2; }
  __device__ static const double *K(const LatDesc *d) { return d->K; }
  __device__ static double nu(const LatDesc *d) { return d->nu; }
  __device__ static double kT(const LatDesc *d) { return d->kT; }
  __device__ static double beta(const LatDesc *d) { return d->beta; }
};
template <> struct Tab<float> {
  __device__ static const float *D1(const LatDesc *d) { return d->D1f; }
  __device__ static const float *D2(const LatDesc *d) { return d->D2f; }
  __device__ static const float *e0(const LatDesc *d) { return d->e0f; }
  __device__ static const float *Hs1(const LatDesc *d) { return d->Hs1f; }
  __device__ static const float *Hs2(const LatDesc *d) { return d->Hs2f; }
  __device__ static const float *K(const LatDesc *d) { return d->Kf; }
  __device__ static float nu(const LatDesc *d) { return d->nuf; }
  __device__ static float kT(const LatDesc *d) { return d->kTf; }
  __device__ static float beta(const LatDesc *d) { return d->betaf; }
};

template <class Real> struct TabFar;
template <> struct TabFar<double> {
  __device__ static const double *Dx(const LatDesc *d) { return &d->Dx[0][0]; }
};
template <> struct TabFar<float> {
  __device__ static const float *Dx(const LatDesc *d) { return &d->Dxf[0][0]; }
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
                                                     Real *__restrict__ ea, Real *__restrict__ de_out) {
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
    if (de_out) de_out[c] = Real(__builtin_nan(""));
    return;
  }
  int X, Y, Z;
  pos_of(g, i, X, Y, Z);
  const int JX = wrapc(X + dir_sx(k), g.X2), JY = wrapc(Y + dir_sy(k), g.Y2),
            JZ = wrapc(Z + dir_sz(k), g.Z2);
  const int A = occ[site_of(g, JX, JY, JZ)];
  Real r, e, de = Real(__builtin_nan(""));
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
    de = delta_e_counts<Real>(c1i, c1j, c2i, c2j, sD1 + 8 * A, sD2 + 8 * A);
    e = se0[A] + Real(0.5) * de;
    r = rate_from_barrier(e, Tab<Real>::nu(d), Tab<Real>::kT(d));
  }
  rates[c] = r;
  if (ea) ea[c] = e;
  if (de_out) de_out[c] = de;
}

// ------------------------------------------- pair model out to 6.0 A

// The 64 neighbours within 6.0 A with their shell (0..5), in the order of
// the observation (by length, then x, y, z).
struct Shell64 {
  int8_t d[kObsN][3];
  int8_t sh[kObsN];
};
constexpr Shell64 make_shell64() {
  Shell64 r{};
  const ObsTab t = make_obs();
  for (int m = 0; m < kObsN; ++m) {
    const int dx = t.d[m][0], dy = t.d[m][1], dz = t.d[m][2];
    const int r2 = dx * dx + dy * dy + dz * dz;
    r.d[m][0] = t.d[m][0];
    r.d[m][1] = t.d[m][1];
    r.d[m][2] = t.d[m][2];
    r.sh[m] = (int8_t)(r2 == 3 ? 0 : r2 == 4 ? 1 : r2 == 8 ? 2 : r2 == 11 ? 3 : r2 == 12 ? 4 : 5);
  }
  return r;
}
__constant__ Shell64 kShell64 = make_shell64();

// One thread per candidate of a site list, bond counts gathered straight
// from the occupancy (all six shells of i and of j = the target), the same
// arithmetic as the event loop's six-shell evaluation.
template <class Real>
__global__ __launch_bounds__(256) void k_rates_sites_far(const LatDesc *__restrict__ d,
                                                         const uint8_t *__restrict__ occ,
                                                         const int32_t *__restrict__ sites,
                                                         int64_t n_sites, Real *__restrict__ rates,
                                                         Real *__restrict__ ea, Real *__restrict__ de_out) {
  __shared__ Real sD1[64], sD2[64], sDx[256], se0[8];
  const int tid = threadIdx.x;
  if (tid < 64) { sD1[tid] = Tab<Real>::D1(d)[tid]; sD2[tid] = Tab<Real>::D2(d)[tid]; }
  sDx[tid] = TabFar<Real>::Dx(d)[tid];
  if (tid < 8) se0[tid] = Tab<Real>::e0(d)[tid];
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * 256 + tid;
  if (c >= n_sites * 8) return;
  const int64_t a = c >> 3;
  const int k = (int)(c & 7);
  const Geo g = make_geo(d->lx, d->ly, d->lz);
  const int S = d->S, V = S - 1;
  const int i = sites ? sites[a] : (int)a;
  if (i < 0 || i >= 2 * g.ncell) {
    rates[c] = Real(__builtin_nan(""));
    if (ea) ea[c] = Real(__builtin_nan(""));
    if (de_out) de_out[c] = Real(__builtin_nan(""));
    return;
  }
  int X, Y, Z;
  pos_of(g, i, X, Y, Z);
  const int kx = dir_sx(k), ky = dir_sy(k), kz = dir_sz(k);
  const int JX = wrapc(X + kx, g.X2), JY = wrapc(Y + ky, g.Y2), JZ = wrapc(Z + kz, g.Z2);
  const int A = occ[site_of(g, JX, JY, JZ)];
  Real r, e, de = Real(__builtin_nan(""));
  if (A == V) {
    r = Real(0);
    e = inf_of<Real>();
  } else {
    uint64_t ci[6] = {0, 0, 0, 0, 0, 0}, cj[6] = {0, 0, 0, 0, 0, 0};
    for (int m = 0; m < kObsN; ++m) {
      const int dx = kShell64.d[m][0], dy = kShell64.d[m][1], dz = kShell64.d[m][2];
      const int sh = kShell64.sh[m];
      // neighbour of i (skip j itself) and of j (skip i itself)
      if (!(dx == kx && dy == ky && dz == kz)) {
        const int si = occ[site_of(g, wrapc(X + dx, g.X2), wrapc(Y + dy, g.Y2), wrapc(Z + dz, g.Z2))];
        ci[sh] += 1ull << (8 * si);
      }
      if (!(dx == -kx && dy == -ky && dz == -kz)) {
        const int sj = occ[site_of(g, wrapc(JX + dx, g.X2), wrapc(JY + dy, g.Y2), wrapc(JZ + dz, g.Z2))];
        cj[sh] += 1ull << (8 * sj);
      }
    }
    de = delta_e_counts6<Real>(ci, cj, S, sD1 + 8 * A, sD2 + 8 * A, sDx, A);
    e = se0[A] + Real(0.5) * de;
    r = rate_from_barrier(e, Tab<Real>::nu(d), Tab<Real>::kT(d));
  }
  rates[c] = r;
  if (ea) ea[c] = e;
  if (de_out) de_out[c] = de;
}

// ---------------------------------------------------------- bulk sweep

template <class Real> struct Sweep;
// The rate of candidate p <- j from a per-site term and a per-target term
// (see k_rates_all), with the field accumulated from tables already scaled
// by h (hG = h G'):
//   binary64:  r = exp(Cn[A][s_p] - hG_A(p)) * exp(hG_{s_j}(j)),   h = beta/2
//   binary32:  r = 2^((C2f[A][s_p] - hG_A(p)) + hG_{s_j}(j)),      h = (beta/2) log2(e)
// binary64 takes the product of two factors, so that a site costs S-1
// exponentials for its movers plus one for its own target role instead of
// one per candidate (its costly exponential dominates); each factor must
// stay inside binary64's exponent range, which the host checks from the
// tables before it picks this kernel.  binary32's range is too narrow for
// the factors, and its hardware exponential is cheap: one per candidate.
// The barrier, when asked for, is e0[A] + (G'_A(p) - G'_A(j) + K[A][s_p]) / 2
// with G' = hG / h.
template <> struct Sweep<double> {
  static constexpr bool kFactor = true;
  __device__ static double inv_h(const LatDesc *d) { return d->inv_half_beta; }
  __device__ static double table(const LatDesc *d, int i) { return d->Cn[i]; }
  __device__ static double ex(double t) { return exp(t); }
};
template <> struct Sweep<float> {
  static constexpr bool kFactor = false;
  __device__ static float inv_h(const LatDesc *d) { return d->inv_h2f; }
  __device__ static float table(const LatDesc *d, int i) { return d->C2f[i]; }
  __device__ static float ex(float t) { return __builtin_amdgcn_exp2f(t); }
};

// Species count s of a packed nibble count vector c, as a real, from the
// even (c & 0x0f0f0f0f) or odd ((c >> 4) & 0x0f0f0f0f) nibbles.
template <class Real>
__device__ __forceinline__ Real count_of(uint32_t ev, uint32_t od, int s) {
  return (Real)(((s & 1) ? od : ev) >> (8 * (s >> 1)) & 0xffu);
}

// Whether either shell holds a vacancy (code V).  Vacancies are a tiny
// fraction of the sites, so the field chains add the vacancy terms last and
// only where a lane needs them: a wavefront without such a lane skips them.
__device__ __forceinline__ bool has_vacancy(uint32_t c1, uint32_t c2, int V) {
  return ((c1 | c2) >> (4 * V) & 15u) != 0u;
}

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
  // per region site: bond counts (2 words), the target term (binary32) or
  // factor (binary64) and, for the binary64 barrier output, its field; site
  // terms: binary32 per lane (S planes of kSweepThreads), binary64 factors
  // per brick site (S-1 planes of NT, twice with the barrier output)
  __host__ __device__ static constexpr size_t terms(int S, size_t real, bool with_ea) {
    return real == 4 ? (size_t)S * kSweepThreads : (size_t)(S - 1) * NT * (with_ea ? 2 : 1);
  }
  static size_t lds_bytes(int S, size_t real, bool with_ea) {
    return OCC_BYTES + (size_t)2 * HV * (8 + real + (with_ea && real == 8 ? real : 0)) +
           terms(S, real, with_ea) * real;
  }
};

// Region layout: corners (b = 0) at cells [0, T+1) and centres (b = 1) at
// cells [-1, T) of the brick, each stored at index h = c + b.  The targets
// of a corner at cell c are the centres at cells c - 1 + [s > 0], those of
// a centre the corners at c + [s > 0]; both sit at index h = c + [s > 0] of
// the other sublattice.
//
// With the field G'_A(q) = sum_s n1_s(q) Ds1[A][s] + n2_s(q) Ds2[A][s]
// (accumulated as hG = h G' from the scaled tables Hs = h Ds), the rate of
// p <- j (species A = s_j) is, in logarithms,
//   ln r = Cn[A][s_p] - hG_A(p) + hG_A(j),
// and a target enters only with its own species (A = s_j).  Phase 2 stores
// per region site its counts and its target term hG(q) (binary64: the
// factor exp(hG(q))); phase 3 forms per brick site the term of every mover
// species (a table in LDS whose entry for the vacancy code gives a zero
// rate) and combines it with the target terms of the 8 neighbours.
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
  constexpr int HX = Sh::HX, HY = Sh::HY, HZ = Sh::HZ, HV = Sh::HV;
  constexpr int V = S - 1, NA = S - 1;
  constexpr int VW = 16 / (int)sizeof(Real);  // candidates per 16-byte store
  typedef Real vecw __attribute__((ext_vector_type(VW)));
  extern __shared__ __align__(16) unsigned char sweep_lds[];
  uint8_t *socc = sweep_lds;
  uint2 *sCnt = (uint2 *)(sweep_lds + Sh::OCC_BYTES);
  Real *sE = (Real *)(sCnt + 2 * HV);  // target terms (binary32) or factors (binary64)
  Real *sT = sE + 2 * HV;              // site terms or factors
  Real *sH = sT + Sh::terms(S, sizeof(Real), WITH_EA);  // binary64 barrier output: hG
  __shared__ Real sC[64], sHs1[64], sHs2[64], se0[8], sK[64];

  const int tid = threadIdx.x;
  const int lx = d->lx, ly = d->ly, lz = d->lz;
  const int ncell = lx * ly * lz;
  if (tid < 64) {
    sC[tid] = SW::table(d, tid);
    sHs1[tid] = Tab<Real>::Hs1(d)[tid];
    sHs2[tid] = Tab<Real>::Hs2(d)[tid];
    if (WITH_EA) sK[tid] = Tab<Real>::K(d)[tid];
  }
  if (WITH_EA && tid < 8) se0[tid] = Tab<Real>::e0(d)[tid];

  // binary32: the grid-uniform field tables, read at the start into scalar
  // registers (rows of 8 at 8*A, the movers' rows only).
  Real H1[NA * 8], H2[NA * 8];
  if constexpr (sizeof(Real) == 4) {
    const Real *Hs1 = Tab<Real>::Hs1(d), *Hs2 = Tab<Real>::Hs2(d);
#pragma unroll
    for (int i = 0; i < NA * 8; ++i) {
      H1[i] = Hs1[i];
      H2[i] = Hs2[i];
    }
  }

  // One workgroup per brick, y fastest: workgroups are dealt to the 8 XCDs
  // in turn, each with an L2 of its own, so y-neighbouring bricks land on
  // different XCDs and a lattice row (its x run of one cache line or more)
  // is fetched by the XCD whose bricks hold it, plus the two whose y halos
  // reach it, instead of by every XCD whose brick holds a piece of it.
  const int nbx = (lx + TX - 1) / TX, nby = (ly + TY - 1) / TY;
  const int y0 = (int)(blockIdx.x % nby) * TY, x0 = (int)(blockIdx.x / nby % nbx) * TX;
  const int z0 = (int)(blockIdx.x / (nby * nbx)) * TZ;

  // Phase 1: occupancy brick of both sublattices, as 4*species (the shift of
  // that species' count nibble).  One conditional wrap per axis suffices
  // when every edge exceeds the brick: x spans [x0 - PX, x0 + TX + PX) with
  // x0 <= lx - 1, so one wrap suffices when lx >= TX + PX; y and z span 2
  // cells either side.  Small lattices take the general modulo byte by byte.
  const bool simple = lx >= TX + PX && ly > TY + 2 && lz > TZ + 2;
  static_assert(TX % 8 == 0 && PX % 8 == 0, "brick rows must start on 8-byte boundaries");
  if (simple && (lx & 7) == 0) {
    // QW lanes per row of one sublattice, the first QW*EY*EZ lanes (whole
    // wavefronts; the others skip): the indices are formed once and both
    // sublattices' loads are in flight together.  With lx a multiple of 8 a
    // vector never straddles the periodic seam.
    constexpr int QW = EX / 8;
    static_assert(QW * EY * EZ <= kSweepThreads, "one pass per sublattice");
    if (tid < QW * EY * EZ) {
      const int row = tid / QW, w = tid - row * QW;
      const int ey = row % EY, ez = row / EY;
      int gx = x0 - PX + 8 * w, gy = y0 + ey - 2, gz = z0 + ez - 2;
      gx += gx < 0 ? lx : 0;  gx -= gx >= lx ? lx : 0;
      gy += gy < 0 ? ly : 0;  gy -= gy >= ly ? ly : 0;
      gz += gz < 0 ? lz : 0;  gz -= gz >= lz ? lz : 0;
      const uint8_t *src = occ + (gz * ly + gy) * lx + gx;
      uint2 v0 = *(const uint2 *)src;
      uint2 v1 = *(const uint2 *)(src + ncell);
      // codes < 8: no carry between bytes
      v0.x <<= 2; v0.y <<= 2; v1.x <<= 2; v1.y <<= 2;
      uint8_t *dst = socc + (ez * EY + ey) * EX + 8 * w;
      *(uint2 *)dst = v0;
      *(uint2 *)(dst + EV) = v1;
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

  // Phase 2: for every region site q the bond counts (kept for the vacancy
  // role) and the target factor from the field of q's own species.  A thread
  // keeps one column hx and one row hy of the region and walks the z planes
  // of each sublattice BZP at a time (the planes b*HZ + hz congruent to its
  // first one modulo BZP), so that only the plane offset changes per step.
  constexpr int RPP = kSweepThreads / HX;  // region rows per pass
  constexpr int BZP = RPP / HY;            // planes per pass
  static_assert(BZP >= 1, "region row count");
  {
    const int hx = tid % HX, r0 = tid / HX;
    const int hy = r0 % HY, bz0 = r0 / HY;
    if (bz0 < BZP) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        // Region site (b, c = h - b): first shell on the other sublattice's
        // cube of cells c-1..c (corner) or c..c+1 (centre), i.e. h-1..h;
        // second shell on the same sublattice, +-1 cell per axis.
        const uint8_t *s1b = socc + oidx(1 - b, hx - 1, hy - 1, -1);
        const uint8_t *s2b = socc + oidx(b, hx - b, hy - b, -b);
        const int rb = (b * HZ * HY + hy) * HX + hx;
        const int hz0 = b == 0 ? bz0 : ((bz0 - HZ) % BZP + BZP) % BZP;
        for (int hz = hz0; hz < HZ; hz += BZP) {
          const int r = rb + hz * (HY * HX);
          const uint8_t *s1 = s1b + hz * (EY * EX);
          const uint8_t *s2 = s2b + hz * (EY * EX);
          uint32_t c1 = 0;
#pragma unroll
          for (int q = 0; q < 8; ++q) c1 += 1u << s1[((q >> 2) & 1) + ((q >> 1) & 1) * EX + (q & 1) * (EX * EY)];
          const uint32_t c2 = (1u << s2[1]) + (1u << s2[-1]) + (1u << s2[EX]) + (1u << s2[-EX]) +
                              (1u << s2[EX * EY]) + (1u << s2[-EX * EY]);
          sCnt[r] = make_uint2(c1, c2);
          const uint32_t e1 = c1 & 0x0f0f0f0fu, o1 = (c1 >> 4) & 0x0f0f0f0fu;
          const uint32_t e2 = c2 & 0x0f0f0f0fu, o2 = (c2 >> 4) & 0x0f0f0f0fu;
          // Row of q's own species (rows of 8; the vacancy's row is finite
          // and unused, a vacancy never being a target).
          const Real *t1 = sHs1 + 2 * s2[0], *t2 = sHs2 + 2 * s2[0];
          Real g = Real(0);
#pragma unroll
          for (int s = 1; s < V; ++s)
            g = fma(count_of<Real>(e2, o2, s), t2[s], fma(count_of<Real>(e1, o1, s), t1[s], g));
          if (has_vacancy(c1, c2, V))
            g = fma(count_of<Real>(e2, o2, V), t2[V], fma(count_of<Real>(e1, o1, V), t1[V], g));
          if constexpr (SW::kFactor) {
            sE[r] = SW::ex(g);
            if (WITH_EA) sH[r] = g;
          } else {
            sE[r] = g;
          }
        }
      }
    }
  }
  __syncthreads();

  // Phase 3: the 8 candidates of every brick site.  The field of the
  // vacancy site for every mover species comes from its counts, with the
  // same chain as above.
  if constexpr (sizeof(Real) == 8) {
    // binary64: one lane per site forms the site factors (planes of NT),
    // then four lanes per site combine them with the target factors, two
    // candidates each.
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
      const uint32_t e1 = cn.x & 0x0f0f0f0fu, o1 = (cn.x >> 4) & 0x0f0f0f0fu;
      const uint32_t e2 = cn.y & 0x0f0f0f0fu, o2 = (cn.y >> 4) & 0x0f0f0f0fu;
      Real g[NA];
#pragma unroll
      for (int A = 0; A < NA; ++A) g[A] = Real(0);
#pragma unroll
      for (int s = 1; s < V; ++s) {
        const Real n1 = count_of<Real>(e1, o1, s), n2 = count_of<Real>(e2, o2, s);
#pragma unroll
        for (int A = 0; A < NA; ++A) g[A] = fma(n2, sHs2[A * 8 + s], fma(n1, sHs1[A * 8 + s], g[A]));
      }
      if (has_vacancy(cn.x, cn.y, V)) {
        const Real n1 = count_of<Real>(e1, o1, V), n2 = count_of<Real>(e2, o2, V);
#pragma unroll
        for (int A = 0; A < NA; ++A) g[A] = fma(n2, sHs2[A * 8 + V], fma(n1, sHs1[A * 8 + V], g[A]));
      }
#pragma unroll
      for (int A = 0; A < NA; ++A) {
        sTs[A * Sh::NT + t] = SW::ex(sC[A * S + sp] - g[A]);
        if (WITH_EA) sGs[A * Sh::NT + t] = g[A];
      }
    }
    __syncthreads();
    const Real inv_h = SW::inv_h(d);
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
        const Real ts = A == V ? Real(0) : sTs[Ac * Sh::NT + t];
        w[c] = ts * sE[ij];
        if (WITH_EA)
          we[c] = A == V ? inf_of<Real>()
                         : se0[Ac] + Real(0.5) * ((sGs[Ac * Sh::NT + t] - sH[ij]) * inv_h + sK[Ac * S + sp]);
      }
      const size_t site = (unsigned)(b * ncell + (gz * ly + gy) * lx + gx);
      __builtin_nontemporal_store(w, (vecw *)(rates + site * 8) + part);
      if (WITH_EA) __builtin_nontemporal_store(we, (vecw *)(ea + site * 8) + part);
    }
    return;
  }
  // binary32: one lane per site; the field tables sit in scalar registers
  // and the site terms in a per-lane LDS table indexed by the target's code
  // (stored as 4*code, so that code * kSweepThreads is a single shift of
  // it); the vacancy's entry is -inf, which makes a masked rate exactly +0.
  const Real inv_h = SW::inv_h(d);
  Real *myT = sT + tid;
  myT[NA * kSweepThreads] = -__builtin_huge_valf();  // code of the vacancy: a zero rate
  // A workgroup's threads cover one sublattice of the brick: the cell of a
  // thread is fixed and the sublattice is the step.
  static_assert(sizeof(Real) == 8 || TX * TY * TZ == kSweepThreads, "one brick sublattice per pass");
  const int cx = tid % TX, cy = (tid / TX) % TY, cz = tid / (TX * TY);
  const int gx = x0 + cx, gy = y0 + cy, gz = z0 + cz;
  if (gx >= lx || gy >= ly || gz >= lz) return;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int sp = socc[oidx(b, cx, cy, cz)] >> 2;
    const int ip = b * HV + ((cz + b) * HY + (cy + b)) * HX + (cx + b);
    const int ij0 = (1 - b) * HV + (cz * HY + cy) * HX + cx;
    const uint8_t *s1 = socc + oidx(1 - b, cx - 1 + b, cy - 1 + b, cz - 1 + b);
    const uint2 cn = sCnt[ip];
    const uint32_t e1 = cn.x & 0x0f0f0f0fu, o1 = (cn.x >> 4) & 0x0f0f0f0fu;
    const uint32_t e2 = cn.y & 0x0f0f0f0fu, o2 = (cn.y >> 4) & 0x0f0f0f0fu;
    Real g[NA];
#pragma unroll
    for (int A = 0; A < NA; ++A) g[A] = Real(0);
#pragma unroll
    for (int s = 1; s < V; ++s) {
      const Real n1 = count_of<Real>(e1, o1, s), n2 = count_of<Real>(e2, o2, s);
#pragma unroll
      for (int A = 0; A < NA; ++A) g[A] = fma(n2, H2[A * 8 + s], fma(n1, H1[A * 8 + s], g[A]));
    }
    if (has_vacancy(cn.x, cn.y, V)) {
      const Real n1 = count_of<Real>(e1, o1, V), n2 = count_of<Real>(e2, o2, V);
#pragma unroll
      for (int A = 0; A < NA; ++A) g[A] = fma(n2, H2[A * 8 + V], fma(n1, H1[A * 8 + V], g[A]));
    }
#pragma unroll
    for (int A = 0; A < NA; ++A) myT[A * kSweepThreads] = sC[A * S + sp] - g[A];
    // Site indices stay below 2^31 (checked at create).
    const size_t site = (unsigned)(b * ncell + (gz * ly + gy) * lx + gx);
    vecw *out = (vecw *)(rates + site * 8);
    vecw *oe = WITH_EA ? (vecw *)(ea + site * 8) : nullptr;
    // All 8 rates first, then the row's stores back to back: a 128-byte
    // line is covered by the two store instructions of one wavefront, and
    // issuing them together lets the line be written to HBM once.
    constexpr int NVEC = 8 / VW;
    vecw w[NVEC], we[NVEC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int px = (k >> 2) & 1, py = (k >> 1) & 1, pz = k & 1;
      const int A4 = s1[px + py * EX + pz * (EX * EY)];  // 4 * code
      const int ij = ij0 + (pz * HY + py) * HX + px;
      w[k / VW][k % VW] = SW::ex(myT[A4 * (kSweepThreads / 4)] + sE[ij]);
      if (WITH_EA) {
        const int A = A4 >> 2;
        Real ga = g[0];
#pragma unroll
        for (int m = 1; m < NA; ++m) ga = A == m ? g[m] : ga;
        const int Ac = min(A, NA - 1);
        we[k / VW][k % VW] =
            A == V ? inf_of<Real>() : se0[Ac] + Real(0.5) * ((ga - sE[ij]) * inv_h + sK[Ac * S + sp]);
      }
    }
#pragma unroll
    for (int v = 0; v < NVEC; ++v) __builtin_nontemporal_store(w[v], out + v);
    if (WITH_EA) {
#pragma unroll
      for (int v = 0; v < NVEC; ++v) __builtin_nontemporal_store(we[v], oe + v);
    }
  }
}

// ------------------------------------------------------------ launchers

// A launch that records the caller's timing events, if any, at its kernel's
// start and end.
template <class K, class... Args>
static void launch_timed(K k, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                         const LaunchTiming *tm, Args... args) {
  if (tm && (tm->start || tm->stop))
    hipExtLaunchKernelGGL(k, grid, block, (uint32_t)lds, st, tm->start, tm->stop, 0u, args...);
  else
    hipLaunchKernelGGL(k, grid, block, lds, st, args...);
}

hipError_t launch_rates_sites(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                              const int32_t *sites, int64_t n_sites, int precision, void *rates,
                              void *ea, hipStream_t stream, const LaunchTiming *tm, void *de) {
  if (n_sites <= 0) return hipSuccess;
  const int64_t nthreads = n_sites * 8;
  const unsigned blocks = (unsigned)((nthreads + 255) / 256);
  if (h.n_shells == 6) {
    if (precision == AKMC_FP32)
      launch_timed(k_rates_sites_far<float>, dim3(blocks), dim3(256), 0, stream, tm, d_desc, occ, sites,
                   n_sites, (float *)rates, (float *)ea, (float *)de);
    else
      launch_timed(k_rates_sites_far<double>, dim3(blocks), dim3(256), 0, stream, tm, d_desc, occ, sites,
                   n_sites, (double *)rates, (double *)ea, (double *)de);
    return hipGetLastError();
  }
  if (precision == AKMC_FP32)
    launch_timed(k_rates_sites<float>, dim3(blocks), dim3(256), 0, stream, tm, d_desc, occ, sites,
                 n_sites, (float *)rates, (float *)ea, (float *)de);
  else
    launch_timed(k_rates_sites<double>, dim3(blocks), dim3(256), 0, stream, tm, d_desc, occ, sites,
                 n_sites, (double *)rates, (double *)ea, (double *)de);
  return hipGetLastError();
}

template <int TX, int TY, int TZ, int S, class Real>
static hipError_t launch_sweep(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                               void *rates, void *ea, hipStream_t stream, const LaunchTiming *tm) {
  using Sh = SweepShape<TX, TY, TZ>;
  const dim3 tiles((unsigned)(((h.lx + TX - 1) / TX) * ((h.ly + TY - 1) / TY) * ((h.lz + TZ - 1) / TZ)));
  const size_t lds = Sh::lds_bytes(S, sizeof(Real), ea != nullptr);
  auto k = ea ? k_rates_all<TX, TY, TZ, S, Real, true> : k_rates_all<TX, TY, TZ, S, Real, false>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  launch_timed(k, tiles, dim3(kSweepThreads), lds, stream, tm, d_desc, occ, (Real *)rates, (Real *)ea);
  return hipGetLastError();
}

template <int S, class Real>
static hipError_t launch_sweep_s(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                                 void *rates, void *ea, hipStream_t stream, const LaunchTiming *tm) {
  // binary64 takes the narrower brick so that several workgroups share a CU
  if constexpr (sizeof(Real) == 8)
    return launch_sweep<16, 4, 4, S, Real>(d_desc, h, occ, rates, ea, stream, tm);
  else
    return launch_sweep<16, 4, 8, S, Real>(d_desc, h, occ, rates, ea, stream, tm);
}

template <class Real>
static hipError_t launch_sweep_r(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                                 void *rates, void *ea, hipStream_t stream, const LaunchTiming *tm) {
  switch (h.S) {
    case 2: return launch_sweep_s<2, Real>(d_desc, h, occ, rates, ea, stream, tm);
    case 3: return launch_sweep_s<3, Real>(d_desc, h, occ, rates, ea, stream, tm);
    case 4: return launch_sweep_s<4, Real>(d_desc, h, occ, rates, ea, stream, tm);
    case 5: return launch_sweep_s<5, Real>(d_desc, h, occ, rates, ea, stream, tm);
    case 6: return launch_sweep_s<6, Real>(d_desc, h, occ, rates, ea, stream, tm);
    case 7: return launch_sweep_s<7, Real>(d_desc, h, occ, rates, ea, stream, tm);
    case 8: return launch_sweep_s<8, Real>(d_desc, h, occ, rates, ea, stream, tm);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_rates_all(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                            int precision, void *rates, void *ea, hipStream_t stream,
                            const LaunchTiming *tm) {
  // The six-shell model takes the per-candidate kernel over every site.
  if (h.n_shells == 6)
    return launch_rates_sites(d_desc, h, occ, nullptr, 2 * h.ncell, precision, rates, ea, stream, tm);
  if (precision == AKMC_FP32) return launch_sweep_r<float>(d_desc, h, occ, rates, ea, stream, tm);
  // The binary64 sweep's factors must stay inside the exponent range; tables
  // that could leave it take the per-candidate kernel over every site.
  if (!h.sweep_factor_ok)
    return launch_rates_sites(d_desc, h, occ, nullptr, 2 * h.ncell, precision, rates, ea, stream,
                              tm);
  return launch_sweep_r<double>(d_desc, h, occ, rates, ea, stream, tm);
}

}  // namespace akmc
