// Solute cluster-size histogram: connected components of one species under
// first-neighbour adjacency on the periodic BCC lattice (the clustering
// descriptor of Sec. III-A2; Cu-rich precipitates, Sec. III-C1), by
// lock-free union-find.
//
// parent[p] always names a site of p's component with an index <= p, so
// every chain ends at the smallest index of a component (its root).  Hooking
// links the larger of two roots below the smaller with a compare-and-swap;
// path halving only ever replaces a pointer by one of its ancestors.  Both
// keep the invariant, so the result is the unique partition whatever the
// order in which waves run.  One launch per phase gives the grid-wide order
// between phases.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "akmc.h"
#include "akmc_device.hpp"

// Scratch of the allocation-free histogram: parent and size arrays of up to
// AKMC_CLUSTER_STATIC_MAX_SITES sites each (32 MiB per device).  Every
// device holds its own copy; host code reaches it only through the address
// that akmc::cluster_static_scratch resolves on that device (the name is a
// host-side stand-in, not a device address).
static __device__ __align__(256) int32_t scratch[2 * (size_t)AKMC_CLUSTER_STATIC_MAX_SITES];

namespace akmc {

namespace {

__device__ __forceinline__ int ld(const int *a, int i) {
  return __hip_atomic_load(a + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving.
__device__ __forceinline__ int find_root(int *parent, int x) {
  int px = ld(parent, x);
  while (px != x) {
    const int gx = ld(parent, px);
    if (gx != px) __hip_atomic_store(parent + x, gx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = px;
    px = gx;
  }
  return x;
}

// Site of the first neighbour of `site` in direction k (k = 4[sx>0] + 2[sy>0] + [sz>0]).
__device__ __forceinline__ int nbr1(const Geo &g, int X, int Y, int Z, int k) {
  return site_of(g, wrapc(X + dir_sx(k), g.X2), wrapc(Y + dir_sy(k), g.Y2), wrapc(Z + dir_sz(k), g.Z2));
}

__global__ void k_cc_init(const uint8_t *__restrict__ occ, int64_t n, int species,
                          int *__restrict__ parent, int *__restrict__ size,
                          unsigned long long *__restrict__ hist, int64_t nbins) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nbins) hist[p] = 0ull;
  if (p >= n) return;
  parent[p] = occ[p] == species ? (int)p : -1;
  size[p] = 0;
}

// Each edge is taken once, from its larger endpoint.
__global__ void k_cc_hook(const uint8_t *__restrict__ occ, int64_t n, int species, int lx, int ly,
                          int lz, int *parent) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || occ[p] != species) return;
  const Geo g = make_geo(lx, ly, lz);
  int X, Y, Z;
  pos_of(g, (int)p, X, Y, Z);
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    const int q = nbr1(g, X, Y, Z, k);
    if (q >= p || occ[q] != species) continue;
    int a = find_root(parent, (int)p), b = find_root(parent, q);
    // Bounded: every failed exchange moves one of the two roots to a
    // strictly smaller index.
    while (a != b) {
      const int hi = a > b ? a : b, lo = a > b ? b : a;
      int expect = hi;
      if (__hip_atomic_compare_exchange_strong(parent + hi, &expect, lo, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        break;
      // hi gained a parent meanwhile: continue from the new roots.
      a = find_root(parent, expect);
      b = find_root(parent, lo);
    }
  }
}

__global__ void k_cc_count(int64_t n, int *parent, int *size) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || ld(parent, (int)p) < 0) return;
  const int r = find_root(parent, (int)p);
  atomicAdd(size + r, 1);
}

__global__ void k_cc_hist(int64_t n, const int *__restrict__ parent, const int *__restrict__ size,
                          unsigned long long *hist, int64_t max_size) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || parent[p] != (int)p) return;
  const int64_t s = size[p];
  atomicAdd(hist + (s < max_size ? s : max_size), 1ull);
}

}  // namespace

hipError_t cluster_static_scratch(int32_t **parent, int32_t **size) {
  static std::mutex mu;
  static std::map<int, int32_t *> resolved;  // device -> device address of `scratch`
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = resolved.find(dev);
  if (it == resolved.end()) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = resolved.emplace(dev, static_cast<int32_t *>(ptr)).first;
  }
  *parent = it->second;
  *size = it->second + (size_t)AKMC_CLUSTER_STATIC_MAX_SITES;
  return hipSuccess;
}

hipError_t launch_cluster_hist(const uint8_t *d_occ, int lx, int ly, int lz, int species,
                               int64_t max_size, int64_t *d_hist, int *d_parent, int *d_size,
                               hipStream_t st) {
  const int64_t n = 2ll * lx * ly * lz;
  const int64_t nbins = max_size + 1;
  const int B = 256;
  const int64_t span = n > nbins ? n : nbins;
  unsigned long long *hist = reinterpret_cast<unsigned long long *>(d_hist);
  hipLaunchKernelGGL(k_cc_init, dim3((unsigned)((span + B - 1) / B)), dim3(B), 0, st, d_occ, n,
                     species, d_parent, d_size, hist, nbins);
  const dim3 grid((unsigned)((n + B - 1) / B));
  hipLaunchKernelGGL(k_cc_hook, grid, dim3(B), 0, st, d_occ, n, species, lx, ly, lz, d_parent);
  hipLaunchKernelGGL(k_cc_count, grid, dim3(B), 0, st, n, d_parent, d_size);
  hipLaunchKernelGGL(k_cc_hist, grid, dim3(B), 0, st, n, d_parent, d_size, hist, max_size);
  return hipGetLastError();
}

}  // namespace akmc
