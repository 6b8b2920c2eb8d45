// Local patch networks evaluated on listed sites (a vacancy's 64-neighbour
// observation read from the lattice): the same device forward the event
// loop runs for its learned runtime forms, over many observations.  Each
// block stages the network in LDS once; each wavefront evaluates one site
// at a time.
#include <hip/hip_runtime.h>

#include "akmc_device.hpp"
#include "akmc_internal.hpp"
#include "akmc_patch.hpp"

namespace akmc {

namespace {

__constant__ ObsTab kObsDev = make_obs();

constexpr int kPatchWaves = 4;

__global__ __launch_bounds__(64 * kPatchWaves) void k_patch_eval(
    const LatDesc *__restrict__ d, const uint8_t *__restrict__ occ, const unsigned char *blob,
    const int32_t *__restrict__ sites, int64_t n, float *__restrict__ out) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float *hbuf = (float *)lds + 64 * wave;
  uint8_t *codes = lds + 4 * 64 * kPatchWaves + 64 * wave;
  const PatchNet net = patch_stage(blob, lds + 4 * 64 * kPatchWaves + 64 * kPatchWaves, threadIdx.x,
                                   64 * kPatchWaves);
  __syncthreads();
  const Geo g = make_geo(d->lx, d->ly, d->lz);
  const int64_t nsites = 2ll * g.ncell;
  for (int64_t a = (int64_t)blockIdx.x * kPatchWaves + wave; a < n; a += (int64_t)gridDim.x * kPatchWaves) {
    const int i = sites[a];
    const bool ok = i >= 0 && i < nsites;   // uniform over the wavefront
    if (ok) {
      int X, Y, Z;
      pos_of(g, i, X, Y, Z);
      const int s = site_of(g, wrapc(X + kObsDev.d[lane][0], g.X2), wrapc(Y + kObsDev.d[lane][1], g.Y2),
                            wrapc(Z + kObsDev.d[lane][2], g.Z2));
      codes[lane] = occ[s];
    }
    wave_sync();
    if (ok) {
      const float y = patch_forward(net, codes, hbuf, lane);
      if (lane < net.n_out) out[a * net.n_out + lane] = y;
    } else if (lane < net.n_out) {
      out[a * net.n_out + lane] = __builtin_nanf("");
    }
    wave_sync();
  }
}

}  // namespace

size_t patch_eval_lds_bytes(int S, int H, int n_out) {
  return (size_t)(4 * 64 + 64) * kPatchWaves + (size_t)patch_lds_bytes(S, H, n_out);
}

hipError_t launch_patch_eval(const LatDesc *d_desc, const uint8_t *d_occ, const unsigned char *d_blob,
                             int S, int H, int n_out, const int32_t *d_sites, int64_t n, float *d_out,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = patch_eval_lds_bytes(S, H, n_out);
  hipError_t e = hipFuncSetAttribute((const void *)k_patch_eval,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t want = (n + kPatchWaves - 1) / kPatchWaves;
  const unsigned blocks = (unsigned)(want < 2048 ? want : 2048);
  hipLaunchKernelGGL(k_patch_eval, dim3(blocks), dim3(64 * kPatchWaves), lds, st, d_desc, d_occ, d_blob,
                     d_sites, n, d_out);
  return hipGetLastError();
}

}  // namespace akmc
