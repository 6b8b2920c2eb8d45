// Local patch networks of the learned runtime forms (Sec. III-A1 local
// policy, Sec. III-A3 Poisson time network): weight blob layout, the
// 64-neighbour observation and the device forward of one observation by
// one wavefront.
//
// Observation of a vacancy: the species of its 64 neighbours within 6.0 A
// (the cutoff and neighbour cap of Sec. IV-C; BCC shells 1-6 with 8, 6, 12,
// 24, 8, 6 sites), neighbour m being the m-th offset (in a/2 units) ordered
// by squared length, then x, y, z ascending.
//
// Network (hidden width H <= 64, n_out outputs: 8 logits for the policy, 1
// value for the Poisson network), binary32 arithmetic on bfloat16 weights:
//   h1[j] = relu(b1[j] + sum_m W1[m][code_m][j])            (m = 0..63 in order)
//   h2[j] = relu(b2[j] + sum_i h1[i] W2[i][j])              (one fma per i, ascending)
//   out[k] = b3[k] + sum_i h2[i] W3[i][k]                   (one fma per i, ascending)
// Lane j of the wavefront owns hidden unit j, lane k output k, so every sum
// runs in its stated order in one lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace akmc {

constexpr int kObsN = 64;
constexpr int kPatchMaxHidden = 64;

struct ObsTab {
  int8_t d[kObsN][3];
};

constexpr int obs_key(int dx, int dy, int dz) {
  // squared length first, then the components (each in [-4, 4])
  return (((dx * dx + dy * dy + dz * dz) * 16 + (dx + 4)) * 16 + (dy + 4)) * 16 + (dz + 4);
}

constexpr ObsTab make_obs() {
  ObsTab t{};
  int keys[kObsN] = {};
  int n = 0;
  for (int dx = -4; dx <= 4; ++dx)
    for (int dy = -4; dy <= 4; ++dy)
      for (int dz = -4; dz <= 4; ++dz) {
        const int odd = dx & 1;
        if ((dy & 1) != odd || (dz & 1) != odd) continue;  // not a lattice vector
        const int r2 = dx * dx + dy * dy + dz * dz;
        if (r2 == 0 || r2 > 16) continue;                   // within 2a = 5.73 A < 6.0 A < next shell
        if (n < kObsN) {
          keys[n] = obs_key(dx, dy, dz);
          t.d[n][0] = (int8_t)dx;
          t.d[n][1] = (int8_t)dy;
          t.d[n][2] = (int8_t)dz;
        }
        ++n;
      }
  // insertion sort by key
  for (int a = 1; a < kObsN; ++a)
    for (int b = a; b > 0 && keys[b - 1] > keys[b]; --b) {
      const int k = keys[b];
      keys[b] = keys[b - 1];
      keys[b - 1] = k;
      for (int c = 0; c < 3; ++c) {
        const int8_t v = t.d[b][c];
        t.d[b][c] = t.d[b - 1][c];
        t.d[b - 1][c] = v;
      }
    }
  return t;
}

// Blob: header, then binary32 parameters W1 [64][S][H], b1 [H], W2 [H][H],
// b2 [H], W3 [H][n_out], b3 [n_out] (weights hold bfloat16 values).
struct PatchHeader {
  int32_t S, H, n_out, nparams;
  int32_t magic;
  int32_t pad_[3];
};
constexpr int32_t kPatchMagic = 0x50617463;  // "Patc"

struct PatchLayout {
  int oW1, ob1, oW2, ob2, oW3, ob3, nparams;
  size_t params, total;
};

__host__ __device__ inline PatchLayout patch_layout(int S, int H, int n_out) {
  PatchLayout L;
  L.oW1 = 0;
  L.ob1 = L.oW1 + kObsN * S * H;
  L.oW2 = L.ob1 + H;
  L.ob2 = L.oW2 + H * H;
  L.oW3 = L.ob2 + H;
  L.ob3 = L.oW3 + H * n_out;
  L.nparams = L.ob3 + n_out;
  L.params = 256;
  L.total = L.params + (((size_t)L.nparams * 4 + 255) & ~size_t(255));
  return L;
}

// LDS bytes of one staged network: bf16 W1, W2, W3 and binary32 biases.
__host__ __device__ inline int patch_lds_bytes(int S, int H, int n_out) {
  const int w = 2 * (kObsN * S * H + H * H + H * n_out);
  return ((w + 15) & ~15) + 4 * ((2 * H + n_out + 3) & ~3);
}

// A network staged in LDS.
struct PatchNet {
  const unsigned short *w1, *w2, *w3;
  const float *b1, *b2, *b3;
  int S, H, n_out;
};

// Copies the blob's network into LDS at `dst` (patch_lds_bytes of it) with
// nthreads threads; returns the LDS view.  The bfloat16 weights are the
// upper halves of their binary32 values (exact: the blob holds bfloat16
// values).
__device__ inline PatchNet patch_stage(const unsigned char *blob, unsigned char *dst, int tid,
                                       int nthreads) {
  const PatchHeader *h = (const PatchHeader *)blob;
  const int S = h->S, H = h->H, no = h->n_out;
  const PatchLayout L = patch_layout(S, H, no);
  const float *p = (const float *)(blob + L.params);
  unsigned short *w = (unsigned short *)dst;
  const int nw1 = kObsN * S * H, nw2 = H * H, nw3 = H * no;
  for (int x = tid; x < nw1; x += nthreads) w[x] = (unsigned short)(__float_as_uint(p[L.oW1 + x]) >> 16);
  for (int x = tid; x < nw2; x += nthreads) w[nw1 + x] = (unsigned short)(__float_as_uint(p[L.oW2 + x]) >> 16);
  for (int x = tid; x < nw3; x += nthreads)
    w[nw1 + nw2 + x] = (unsigned short)(__float_as_uint(p[L.oW3 + x]) >> 16);
  float *b = (float *)(dst + ((2 * (nw1 + nw2 + nw3) + 15) & ~15));
  for (int x = tid; x < H; x += nthreads) {
    b[x] = p[L.ob1 + x];
    b[H + x] = p[L.ob2 + x];
  }
  for (int x = tid; x < no; x += nthreads) b[2 * H + x] = p[L.ob3 + x];
  PatchNet n;
  n.w1 = w;
  n.w2 = w + nw1;
  n.w3 = w + nw1 + nw2;
  n.b1 = b;
  n.b2 = b + H;
  n.b3 = b + 2 * H;
  n.S = S;
  n.H = H;
  n.n_out = no;
  return n;
}

__device__ __forceinline__ float bf16_to_f32(unsigned short v) {
  return __uint_as_float((uint32_t)v << 16);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward of one observation (codes[0..63] in LDS, species codes < S) by
// one full wavefront; hbuf is a 64-float LDS staging area.  Lane k < n_out
// returns output k (other lanes return 0).  Every lane must take part.
__device__ inline float patch_forward(const PatchNet &n, const uint8_t *codes, float *hbuf, int lane) {
  const int H = n.H, S = n.S;
  const int j = lane < H ? lane : H - 1;
  float acc = n.b1[j];
#pragma unroll 16
  for (int m = 0; m < kObsN; ++m) {
    const int c = codes[m];
    acc = acc + bf16_to_f32(n.w1[(m * S + c) * H + j]);
  }
  const float h1 = acc > 0.0f ? acc : 0.0f;
  wave_sync();
  if (lane < H) hbuf[lane] = h1;
  wave_sync();
  acc = n.b2[j];
  for (int i = 0; i < H; ++i) acc = fmaf(hbuf[i], bf16_to_f32(n.w2[i * H + j]), acc);
  const float h2 = acc > 0.0f ? acc : 0.0f;
  wave_sync();
  if (lane < H) hbuf[lane] = h2;
  wave_sync();
  const int k = lane < n.n_out ? lane : 0;
  acc = n.b3[k];
  for (int i = 0; i < H; ++i) acc = fmaf(hbuf[i], bf16_to_f32(n.w3[i * n.n_out + k]), acc);
  wave_sync();
  return lane < n.n_out ? acc : 0.0f;
}

}  // namespace akmc
