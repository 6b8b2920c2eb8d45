// Voxel ensemble on one GPU: temperature-guided discretisation of a wall
// thermal field (Sec. III-C1, the Eq. 9 tolerance on the intra-voxel rate
// variation) and dynamic voxel scheduling (Sec. III-C2): the workload proxy
// W_v of Eq. 10 computed on the device from every replica's current
// barriers, and the heaviest-first order the persistent event loop pulls
// replicas in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "akmc_internal.hpp"

namespace akmc {

// ------------------------------------------------------------ discretisation

namespace {

struct VoxelStat {
  double mean, lo, hi;
};

// Mean (summed row by row, x fastest), min and max of the samples of voxel
// (b, a) of a uniform n_x by n_z split; voxel a spans the sample columns
// floor(a*nx/n_x) .. floor((a+1)*nx/n_x) - 1, rows likewise.
VoxelStat voxel_stat(const double *T, int nx, int nz, int n_x, int n_z, int a, int b) {
  const int x0 = (int)((int64_t)a * nx / n_x), x1 = (int)((int64_t)(a + 1) * nx / n_x);
  const int z0 = (int)((int64_t)b * nz / n_z), z1 = (int)((int64_t)(b + 1) * nz / n_z);
  double s = 0.0, lo = INFINITY, hi = -INFINITY;
  for (int z = z0; z < z1; ++z)
    for (int x = x0; x < x1; ++x) {
      const double v = T[(int64_t)z * nx + x];
      s += v;
      lo = std::min(lo, v);
      hi = std::max(hi, v);
    }
  return VoxelStat{s / (double)((int64_t)(x1 - x0) * (z1 - z0)), lo, hi};
}

// Relative rate variation of Eq. 9 inside one voxel: E dT / (kB T^2) with
// T the voxel temperature and dT the spread of its samples.
double eq9(double e_eff, double kb, const VoxelStat &v) {
  return (e_eff * (v.hi - v.lo)) / (kb * v.mean * v.mean);
}

}  // namespace

int voxel_grid(const double *T, int nx, int nz, double e_eff, double kb, double tol, int *n_x_out,
               int *n_z_out, double *t_vox, double *worst_out) {
  // Grids in order of voxel count, then of column count; the first whose
  // every voxel meets the tolerance is the discretisation.  A grid of
  // single samples always does (zero spread).
  const int64_t total_max = (int64_t)nx * nz;
  for (int64_t total = 1; total <= total_max; ++total) {
    for (int n_x = 1; n_x <= nx; ++n_x) {
      if (total % n_x != 0 || total / n_x > nz) continue;
      const int n_z = (int)(total / n_x);
      double worst = 0.0;
      bool ok = true;
      for (int b = 0; b < n_z && ok; ++b)
        for (int a = 0; a < n_x; ++a) {
          const double w = eq9(e_eff, kb, voxel_stat(T, nx, nz, n_x, n_z, a, b));
          if (!(w <= tol)) {
            ok = false;
            break;
          }
          worst = std::max(worst, w);
        }
      if (!ok) continue;
      for (int b = 0; b < n_z; ++b)
        for (int a = 0; a < n_x; ++a)
          t_vox[(int64_t)b * n_x + a] = voxel_stat(T, nx, nz, n_x, n_z, a, b).mean;
      *n_x_out = n_x;
      *n_z_out = n_z;
      *worst_out = worst;
      return 0;
    }
  }
  return -1;
}

// ---------------------------------------------------------------- priority

namespace {

// W_v = M exp(-E/kT) per replica: M the admissible candidates of the current
// state (finite barriers in the loop's trace), E their mean barrier (summed
// in candidate order in binary64), kT the replica's.  One lane per replica.
template <class Real>
__global__ void k_priority(const LatDesc *__restrict__ descs, const Real *__restrict__ trace,
                           int n_rep, double *__restrict__ w_out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rep) return;
  const LatDesc &d = descs[r];
  const Real *ea = trace + d.slot_off * 8;
  int64_t m = 0;
  double s = 0.0;
  for (int c = 0; c < 8 * d.nv; ++c) {
    const double e = (double)ea[c];
    if (isinf(e)) continue;
    m += 1;
    s += e;
  }
  double w = 0.0;
  if (m > 0) {
    const double e_hat = s / (double)m;
    w = (double)m * exp(-(e_hat / d.kT));
  }
  w_out[r] = w;
}

// Dispatch order: replica r goes to position #{u : w_u > w_r, or w_u = w_r
// and u < r}, i.e. heaviest first with equal weights by index.  One lane per
// replica; the weights are read through LDS tiles.
__global__ void k_rank(const double *__restrict__ w, int n_rep, int32_t *__restrict__ order) {
  __shared__ double tile[256];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const double wr = r < n_rep ? w[r] : 0.0;
  int rank = 0;
  for (int t0 = 0; t0 < n_rep; t0 += 256) {
    const int u = t0 + (int)threadIdx.x;
    tile[threadIdx.x] = u < n_rep ? w[u] : 0.0;
    __syncthreads();
    const int cnt = std::min(256, n_rep - t0);
    for (int q = 0; q < cnt; ++q) {
      const double wu = tile[q];
      rank += (wu > wr || (wu == wr && t0 + q < r)) ? 1 : 0;
    }
    __syncthreads();
  }
  if (r < n_rep) order[rank] = r;
}

__global__ void k_iota(int32_t *order, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) order[r] = r;
}

}  // namespace

hipError_t launch_order_index(int32_t *d_order, int n_rep, hipStream_t st) {
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n_rep + 255) / 256)), dim3(256), 0, st, d_order, n_rep);
  return hipGetLastError();
}

hipError_t launch_priority(const LatDesc *d_descs, const void *d_trace, int fp32, int n_rep,
                           double *d_w, int32_t *d_order, hipStream_t st) {
  const int B = 256;
  const dim3 grid((unsigned)((n_rep + B - 1) / B));
  if (fp32)
    hipLaunchKernelGGL(k_priority<float>, grid, dim3(B), 0, st, d_descs,
                       static_cast<const float *>(d_trace), n_rep, d_w);
  else
    hipLaunchKernelGGL(k_priority<double>, grid, dim3(B), 0, st, d_descs,
                       static_cast<const double *>(d_trace), n_rep, d_w);
  hipLaunchKernelGGL(k_rank, grid, dim3(B), 0, st, d_w, n_rep, d_order);
  return hipGetLastError();
}

}  // namespace akmc
