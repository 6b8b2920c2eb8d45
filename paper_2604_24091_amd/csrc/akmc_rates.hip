// Rate evaluation outside the event loop.
//
//  k_rates_sites: one thread per candidate (site, direction) of a site
//    list; gathers the bond counts straight from the occupancy and uses
//    exactly the arithmetic of the event loop, so VACANCIES mode returns
//    the loop's rates bit for bit.
//
//  k_rates_all: the bulk sweep over every lattice site (a vacancy placed
//    at each site in turn).  It is bound by the HBM write of the
//    [N][8] rate array.  A workgroup stages a brick of occupancy with a
//    2-cell halo in LDS, computes for every site q that can be a jump
//    target the field H(q) = sum over its 14 bonds of
//        D'_k[s_q][s_n] = D_k[s_q][s_n] - D_k[s_q][Fe],
//    and for every site p of the brick the same field G'_A(p) for each
//    mover species A.  Because the pair energy is a sum over bonds, the
//    energy change of the jump p <- j (species A = s_j) is
//        dE = G'_A(p) - H(j) + D1[A][s_p] - D1[A][A],
//    which equals the bond-count form up to rounding; measuring the field
//    against the all-Fe environment keeps it near zero, so binary32
//    keeps its relative accuracy.
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
    const Real de = delta_e_counts<Real>(c1i, c1j, c2i, c2j, sD1 + A * S, sD2 + A * S, S);
    e = se0[A] + Real(0.5) * de;
    r = rate_from_barrier(e, Tab<Real>::nu(d), Tab<Real>::kT(d));
  }
  rates[c] = r;
  if (ea) ea[c] = e;
}

// ---------------------------------------------------------- bulk sweep

template <class Real> struct Sweep;
template <> struct Sweep<double> {
  // ln r = Cn[A][s_p] + (beta/2) dG;  r = exp(ln r)
  __device__ static double C(const LatDesc *d, int i) { return d->Cn[i]; }
  __device__ static double h(const LatDesc *d) { return d->half_beta; }
  __device__ static double rate(double c, double h, double dg) { return exp(fma(h, dg, c)); }
};
template <> struct Sweep<float> {
  // log2 r = C2f[A][s_p] + h2f dG;  r = 2^(log2 r), one hardware exponential
  __device__ static float C(const LatDesc *d, int i) { return d->C2f[i]; }
  __device__ static float h(const LatDesc *d) { return d->h2f; }
  __device__ static float rate(float c, float h, float dg) {
    return __builtin_amdgcn_exp2f(fmaf(h, dg, c));
  }
};

constexpr int kSweepThreads = 256;

template <int TX, int TY, int TZ>
struct SweepShape {
  static constexpr int EX = TX + 4, EY = TY + 4, EZ = TZ + 4, EV = EX * EY * EZ;  // occupancy brick
  static constexpr int HX = TX + 1, HY = TY + 1, HZ = TZ + 1, HV = HX * HY * HZ;  // field region
  static constexpr int NT = 2 * TX * TY * TZ;                                     // brick sites
  static constexpr int OCC_BYTES = (2 * EV + 15) & ~15;
  static size_t lds_bytes(int S, size_t real) {
    return OCC_BYTES + (size_t)2 * HV * (size_t)(S - 1) * real;
  }
};

// Region layout of the field G'_A: corners (b = 0) at cells [0, T+1) and
// centres (b = 1) at cells [-1, T) of the brick, each stored at index
// h = c + b.  The targets of a corner at cell c are the centres at cells
// c - 1 + [s > 0], those of a centre the corners at c + [s > 0]; both sit
// at index h = c + [s > 0] of the other sublattice.
template <int TX, int TY, int TZ, class Real, bool WITH_EA>
__global__ __launch_bounds__(kSweepThreads) void k_rates_all(const LatDesc *__restrict__ d,
                                                             const uint8_t *__restrict__ occ,
                                                             Real *__restrict__ rates,
                                                             Real *__restrict__ ea) {
  using Sh = SweepShape<TX, TY, TZ>;
  constexpr int EX = Sh::EX, EY = Sh::EY, EV = Sh::EV;
  constexpr int HX = Sh::HX, HY = Sh::HY, HV = Sh::HV;
  extern __shared__ __align__(16) unsigned char sweep_lds[];
  uint8_t *socc = sweep_lds;
  Real *sG = (Real *)(sweep_lds + Sh::OCC_BYTES);
  __shared__ Real sDs1[64], sDs2[64], sC[64], sK[64], se0[8];

  const int tid = threadIdx.x;
  const int lx = d->lx, ly = d->ly, lz = d->lz;
  const int S = d->S, V = S - 1, NA = S - 1;
  const int ncell = lx * ly * lz;
  if (tid < 64) {
    sDs1[tid] = Tab<Real>::Ds1(d)[tid];
    sDs2[tid] = Tab<Real>::Ds2(d)[tid];
    sC[tid] = Sweep<Real>::C(d, tid);
    sK[tid] = Tab<Real>::K(d)[tid];
  }
  if (tid < 8) se0[tid] = Tab<Real>::e0(d)[tid];

  const int ntx = (lx + TX - 1) / TX, nty = (ly + TY - 1) / TY;
  const int tile = blockIdx.x;
  const int x0 = (tile % ntx) * TX;
  const int y0 = ((tile / ntx) % nty) * TY;
  const int z0 = (tile / (ntx * nty)) * TZ;

  // Phase 1: occupancy brick, cells [-2, T+2) of both sublattices, x fastest
  // across lanes.  One conditional wrap suffices when every edge exceeds
  // the brick; smaller lattices take the general modulo.
  const bool simple = lx > TX + 2 && ly > TY + 2 && lz > TZ + 2;
  for (int r = tid; r < 2 * EV; r += kSweepThreads) {
    const int ex = r % EX;
    const int row = r / EX;
    const int ey = row % EY;
    const int bz = row / EY;
    const int ez = bz % Sh::EZ;
    const int b = bz / Sh::EZ;
    int gx = x0 + ex - 2, gy = y0 + ey - 2, gz = z0 + ez - 2;
    if (simple) {
      gx += gx < 0 ? lx : 0;  gx -= gx >= lx ? lx : 0;
      gy += gy < 0 ? ly : 0;  gy -= gy >= ly ? ly : 0;
      gz += gz < 0 ? lz : 0;  gz -= gz >= lz ? lz : 0;
    } else {
      gx = ((gx % lx) + lx) % lx;
      gy = ((gy % ly) + ly) % ly;
      gz = ((gz % lz) + lz) % lz;
    }
    socc[r] = occ[b * ncell + (gz * ly + gy) * lx + gx];
  }
  __syncthreads();

  auto oidx = [&](int b, int cx, int cy, int cz) {
    return b * EV + ((cz + 2) * EY + (cy + 2)) * EX + (cx + 2);
  };

  // Phase 2: G'_A(q) for every mover species A at every region site:
  //   G'_A(q) = sum_s n1_s(q) Ds1[A][s] + n2_s(q) Ds2[A][s]   (s = 0 drops out)
  for (int r = tid; r < 2 * HV; r += kSweepThreads) {
    const int hx = r % HX;
    const int row = r / HX;
    const int hy = row % HY;
    const int bz = row / HY;
    const int hz = bz % Sh::HZ;
    const int b = bz / Sh::HZ;
    const int cx = hx - b, cy = hy - b, cz = hz - b;
    const int o = b ? 0 : -1;  // first shell of a corner: cells c-1..c; of a centre: c..c+1
    uint32_t c1 = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      c1 += onehot(socc[oidx(1 - b, cx + o + ((q >> 2) & 1), cy + o + ((q >> 1) & 1), cz + o + (q & 1))]);
    const uint32_t c2 =
        onehot(socc[oidx(b, cx + 1, cy, cz)]) + onehot(socc[oidx(b, cx - 1, cy, cz)]) +
        onehot(socc[oidx(b, cx, cy + 1, cz)]) + onehot(socc[oidx(b, cx, cy - 1, cz)]) +
        onehot(socc[oidx(b, cx, cy, cz + 1)]) + onehot(socc[oidx(b, cx, cy, cz - 1)]);
    Real g[8];
#pragma unroll
    for (int A = 0; A < 8; ++A) g[A] = Real(0);
    for (int s = 1; s < S; ++s) {
      const Real n1 = (Real)nib(c1, s), n2 = (Real)nib(c2, s);
#pragma unroll
      for (int A = 0; A < 8; ++A)
        if (A < NA) g[A] = fma(n2, sDs2[A * S + s], fma(n1, sDs1[A * S + s], g[A]));
    }
#pragma unroll
    for (int A = 0; A < 8; ++A)
      if (A < NA) sG[A * (2 * HV) + r] = g[A];
  }
  __syncthreads();

  // Phase 3: the 8 candidates of every brick site, from the field alone.
  const Real h = Sweep<Real>::h(d);
  for (int t = tid; t < Sh::NT; t += kSweepThreads) {
    const int cx = t % TX;
    const int row = t / TX;
    const int cy = row % TY;
    const int bz = row / TY;
    const int cz = bz % TZ;
    const int b = bz / TZ;
    const int gx = x0 + cx, gy = y0 + cy, gz = z0 + cz;
    if (gx >= lx || gy >= ly || gz >= lz) continue;
    const int sp = socc[oidx(b, cx, cy, cz)];
    // Field planes are species-major (plane A holds G'_A of every region
    // site), so neighbouring lanes read neighbouring words.
    const int ip = b * HV + ((cz + b) * HY + (cy + b)) * HX + (cx + b);
    const int ij0 = (1 - b) * HV + (cz * HY + cy) * HX + cx;
    const int o = b ? 0 : -1;
    Real rr[8], ee[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int px = (k >> 2) & 1, py = (k >> 1) & 1, pz = k & 1;
      const int A = socc[oidx(1 - b, cx + o + px, cy + o + py, cz + o + pz)];
      if (A == V) {
        rr[k] = Real(0);
        ee[k] = inf_of<Real>();
      } else {
        const Real gpa = sG[A * (2 * HV) + ip];
        const Real gja = sG[A * (2 * HV) + ij0 + (pz * HY + py) * HX + px];
        rr[k] = Sweep<Real>::rate(sC[A * S + sp], h, gja - gpa);
        if (WITH_EA) ee[k] = se0[A] + Real(0.5) * ((gpa - gja) + sK[A * S + sp]);
      }
    }
    const int64_t site = (int64_t)b * ncell + ((int64_t)gz * ly + gy) * lx + gx;
    Real *out = rates + site * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) __builtin_nontemporal_store(rr[k], out + k);
    if (WITH_EA) {
      Real *oe = ea + site * 8;
#pragma unroll
      for (int k = 0; k < 8; ++k) __builtin_nontemporal_store(ee[k], oe + k);
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

template <int TX, int TY, int TZ, class Real>
static hipError_t launch_sweep(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                               void *rates, void *ea, hipStream_t stream) {
  using Sh = SweepShape<TX, TY, TZ>;
  const unsigned tiles = (unsigned)(((h.lx + TX - 1) / TX) * ((h.ly + TY - 1) / TY) *
                                    ((h.lz + TZ - 1) / TZ));
  const size_t lds = Sh::lds_bytes(h.S, sizeof(Real));
  if (ea) {
    auto k = k_rates_all<TX, TY, TZ, Real, true>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(tiles), dim3(kSweepThreads), lds, stream, d_desc, occ, (Real *)rates, (Real *)ea);
  } else {
    auto k = k_rates_all<TX, TY, TZ, Real, false>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(tiles), dim3(kSweepThreads), lds, stream, d_desc, occ, (Real *)rates, (Real *)ea);
  }
  return hipGetLastError();
}

hipError_t launch_rates_all(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                            int precision, void *rates, void *ea, hipStream_t stream) {
  // The field holds S-1 values per region site: narrow the brick for many species.
  if (h.S <= 5) {
    if (precision == AKMC_FP32) return launch_sweep<32, 4, 4, float>(d_desc, h, occ, rates, ea, stream);
    return launch_sweep<32, 4, 4, double>(d_desc, h, occ, rates, ea, stream);
  }
  if (precision == AKMC_FP32) return launch_sweep<16, 4, 4, float>(d_desc, h, occ, rates, ea, stream);
  return launch_sweep<16, 4, 4, double>(d_desc, h, occ, rates, ea, stream);
}

}  // namespace akmc
