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

template <int TX, int TY, int TZ, class Real, bool WITH_EA>
__global__ __launch_bounds__(256) void k_rates_all(const LatDesc *__restrict__ d,
                                                   const uint8_t *__restrict__ occ,
                                                   Real *__restrict__ rates,
                                                   Real *__restrict__ ea) {
  constexpr int EX = TX + 4, EY = TY + 4, EZ = TZ + 4, EV = EX * EY * EZ;  // occupancy brick
  constexpr int HX = TX + 1, HY = TY + 1, HZ = TZ + 1, HV = HX * HY * HZ;  // target field
  constexpr int NT = 2 * TX * TY * TZ;                                     // brick sites
  constexpr int EVP = (2 * EV + 15) & ~15;
  __shared__ __align__(16) uint8_t socc[EVP];
  __shared__ Real sH[2 * HV];
  __shared__ Real sG[256 * 8];
  __shared__ Real sDs1[64], sDs2[64], sK[64], se0[8];

  const int tid = threadIdx.x;
  const int lx = d->lx, ly = d->ly, lz = d->lz;
  const int S = d->S, V = S - 1;
  const int ncell = lx * ly * lz;
  if (tid < 64) {
    sDs1[tid] = Tab<Real>::Ds1(d)[tid];
    sDs2[tid] = Tab<Real>::Ds2(d)[tid];
    sK[tid] = Tab<Real>::K(d)[tid];
  }
  if (tid < 8) se0[tid] = Tab<Real>::e0(d)[tid];

  const int ntx = (lx + TX - 1) / TX, nty = (ly + TY - 1) / TY;
  const int tile = blockIdx.x;
  const int x0 = (tile % ntx) * TX;
  const int y0 = ((tile / ntx) % nty) * TY;
  const int z0 = (tile / (ntx * nty)) * TZ;

  // Phase 1: occupancy brick, cells [-2, T+2) of both sublattices.
  for (int r = tid; r < 2 * EV; r += 256) {
    const int b = r / EV;
    int q = r - b * EV;
    const int ex = q % EX;
    q /= EX;
    const int ey = q % EY;
    const int ez = q / EY;
    int gx = x0 + ex - 2, gy = y0 + ey - 2, gz = z0 + ez - 2;
    gx = ((gx % lx) + lx) % lx;
    gy = ((gy % ly) + ly) % ly;
    gz = ((gz % lz) + lz) % lz;
    socc[r] = occ[b * ncell + (gz * ly + gy) * lx + gx];
  }
  __syncthreads();

  auto oidx = [&](int b, int cx, int cy, int cz) {
    return b * EV + ((cz + 2) * EY + (cy + 2)) * EX + (cx + 2);
  };
  // Bond counts of site (b, c) from the brick.
  auto counts = [&](int b, int cx, int cy, int cz, uint32_t &c1, uint32_t &c2) {
    const int o = b ? 0 : -1;  // first neighbours of a corner sit in cells c-1..c, of a centre in c..c+1
    c1 = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      c1 += onehot(socc[oidx(1 - b, cx + o + ((q >> 2) & 1), cy + o + ((q >> 1) & 1), cz + o + (q & 1))]);
    c2 = onehot(socc[oidx(b, cx + 1, cy, cz)]) + onehot(socc[oidx(b, cx - 1, cy, cz)]) +
         onehot(socc[oidx(b, cx, cy + 1, cz)]) + onehot(socc[oidx(b, cx, cy - 1, cz)]) +
         onehot(socc[oidx(b, cx, cy, cz + 1)]) + onehot(socc[oidx(b, cx, cy, cz - 1)]);
  };

  // Phase 2: H(q) for every possible target: corners at cells [0, T+1),
  // centres at cells [-1, T) (stored shifted by one cell).
  for (int r = tid; r < 2 * HV; r += 256) {
    const int b = r / HV;
    int q = r - b * HV;
    const int hx = q % HX;
    q /= HX;
    const int hy = q % HY;
    const int hz = q / HY;
    const int cx = hx - b, cy = hy - b, cz = hz - b;
    const int sq = socc[oidx(b, cx, cy, cz)];
    Real h = Real(0);
    if (sq != V) {
      uint32_t c1, c2;
      counts(b, cx, cy, cz, c1, c2);
      for (int s = 1; s < S; ++s) {
        h = fma((Real)nib(c1, s), sDs1[sq * S + s], h);
        h = fma((Real)nib(c2, s), sDs2[sq * S + s], h);
      }
    }
    sH[r] = h;
  }
  __syncthreads();

  // Phase 3: the 8 candidates of every brick site.
  const Real nu = Tab<Real>::nu(d), beta = Tab<Real>::beta(d);
  Real *myG = sG + tid * 8;
  for (int t = tid; t < NT; t += 256) {
    const int b = t / (TX * TY * TZ);
    int q = t - b * (TX * TY * TZ);
    const int cx = q % TX;
    q /= TX;
    const int cy = q % TY;
    const int cz = q / TY;
    const int gx = x0 + cx, gy = y0 + cy, gz = z0 + cz;
    if (gx >= lx || gy >= ly || gz >= lz) continue;
    const int sp = socc[oidx(b, cx, cy, cz)];
    uint32_t c1, c2;
    counts(b, cx, cy, cz, c1, c2);
    for (int A = 0; A < V; ++A) {
      Real g = Real(0);
      for (int s = 1; s < S; ++s) {
        g = fma((Real)nib(c1, s), sDs1[A * S + s], g);
        g = fma((Real)nib(c2, s), sDs2[A * S + s], g);
      }
      myG[A] = g;
    }
    const int o = b ? 0 : -1;
    Real rr[8], ee[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int px = (k >> 2) & 1, py = (k >> 1) & 1, pz = k & 1;
      const int A = socc[oidx(1 - b, cx + o + px, cy + o + py, cz + o + pz)];
      // Target j sits in the other sublattice's field at shifted cell c + [s > 0].
      const Real hj = sH[(1 - b) * HV + ((cz + pz) * HY + (cy + py)) * HX + (cx + px)];
      if (A == V) {
        rr[k] = Real(0);
        ee[k] = inf_of<Real>();
      } else {
        const Real de = (myG[A] - hj) + sK[A * S + sp];
        const Real e = se0[A] + Real(0.5) * de;
        ee[k] = e;
        rr[k] = nu * exp(-(e * beta));
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

hipError_t launch_rates_all(const LatDesc *d_desc, const LatDesc &h, const uint8_t *occ,
                            int precision, void *rates, void *ea, hipStream_t stream) {
  constexpr int TX = 32, TY = 4, TZ = 4;
  const unsigned tiles = (unsigned)(((h.lx + TX - 1) / TX) * ((h.ly + TY - 1) / TY) *
                                    ((h.lz + TZ - 1) / TZ));
  if (precision == AKMC_FP32) {
    if (ea)
      hipLaunchKernelGGL((k_rates_all<TX, TY, TZ, float, true>), dim3(tiles), dim3(256), 0,
                         stream, d_desc, occ, (float *)rates, (float *)ea);
    else
      hipLaunchKernelGGL((k_rates_all<TX, TY, TZ, float, false>), dim3(tiles), dim3(256), 0,
                         stream, d_desc, occ, (float *)rates, (float *)ea);
  } else {
    if (ea)
      hipLaunchKernelGGL((k_rates_all<TX, TY, TZ, double, true>), dim3(tiles), dim3(256), 0,
                         stream, d_desc, occ, (double *)rates, (double *)ea);
    else
      hipLaunchKernelGGL((k_rates_all<TX, TY, TZ, double, false>), dim3(tiles), dim3(256), 0,
                         stream, d_desc, occ, (double *)rates, (double *)ea);
  }
  return hipGetLastError();
}

}  // namespace akmc
