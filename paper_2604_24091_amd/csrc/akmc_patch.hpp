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
// Network (hidden width H a multiple of 8 up to 64, n_out outputs: 8 logits for the policy, 1
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

// Staged layout in LDS: W1 as in the blob ([64][S][H], lane j reads
// element j of a row), W2 and W3 transposed ([j][i] and [k][i], rows padded
// by 16 bytes) so that lane j reads its own 64 weights as eight 16-byte
// vectors, then the binary32 biases.
__host__ __device__ inline int patch_w1_elems(int S, int H) { return kObsN * S * H; }
// bf16 elements per transposed row: H rounded up to 8 (16-byte aligned rows),
// plus 8 of padding
__host__ __device__ inline int patch_ldt(int H) { return ((H + 7) & ~7) + 8; }
__host__ __device__ inline int patch_lds_bytes(int S, int H, int n_out) {
  const int w = 2 * (patch_w1_elems(S, H) + (H + n_out) * patch_ldt(H));
  return ((w + 15) & ~15) + 4 * ((2 * H + n_out + 3) & ~3);
}

// A network staged in LDS.
struct PatchNet {
  const unsigned short *w1, *w2t, *w3t;
  const float *b1, *b2, *b3;
  int S, H, n_out;
};

// Copies the blob's network into LDS at `dst` (patch_lds_bytes of it) with
// nthreads threads; returns the LDS view.  The bfloat16 weights are the
// upper halves of their binary32 values (exact: the blob holds bfloat16
// values).
// The LDS view of a network that patch_stage placed at `dst` (no copy).
__device__ inline PatchNet patch_view(const unsigned char *blob, unsigned char *dst) {
  const PatchHeader *h = (const PatchHeader *)blob;
  const int S = h->S, H = h->H, no = h->n_out;
  const int ld = patch_ldt(H), nw1 = patch_w1_elems(S, H);
  PatchNet n;
  n.w1 = (const unsigned short *)dst;
  n.w2t = n.w1 + nw1;
  n.w3t = n.w2t + H * ld;
  n.b1 = (const float *)(dst + ((2 * (nw1 + (H + no) * ld) + 15) & ~15));
  n.b2 = n.b1 + H;
  n.b3 = n.b1 + 2 * H;
  n.S = S;
  n.H = H;
  n.n_out = no;
  return n;
}

__device__ inline PatchNet patch_stage(const unsigned char *blob, unsigned char *dst, int tid,
                                       int nthreads) {
  const PatchHeader *h = (const PatchHeader *)blob;
  const int S = h->S, H = h->H, no = h->n_out;
  const PatchLayout L = patch_layout(S, H, no);
  const float *p = (const float *)(blob + L.params);
  const int ld = patch_ldt(H);
  unsigned short *w = (unsigned short *)dst;
  const int nw1 = patch_w1_elems(S, H);
  unsigned short *w2t = w + nw1, *w3t = w2t + H * ld;
  for (int x = tid; x < nw1; x += nthreads) w[x] = (unsigned short)(__float_as_uint(p[L.oW1 + x]) >> 16);
  for (int x = tid; x < H * H; x += nthreads) {
    const int i = x / H, j = x - i * H;  // W2[i][j] -> row j, column i
    w2t[j * ld + i] = (unsigned short)(__float_as_uint(p[L.oW2 + x]) >> 16);
  }
  for (int x = tid; x < H * no; x += nthreads) {
    const int i = x / no, k = x - i * no;  // W3[i][k] -> row k, column i
    w3t[k * ld + i] = (unsigned short)(__float_as_uint(p[L.oW3 + x]) >> 16);
  }
  float *b = (float *)(dst + ((2 * (nw1 + (H + no) * ld) + 15) & ~15));
  for (int x = tid; x < H; x += nthreads) {
    b[x] = p[L.ob1 + x];
    b[H + x] = p[L.ob2 + x];
  }
  for (int x = tid; x < no; x += nthreads) b[2 * H + x] = p[L.ob3 + x];
  PatchNet n;
  n.w1 = w;
  n.w2t = w2t;
  n.w3t = w3t;
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

// sum_i x[i] * w[i] for i = 0 .. H-1 in ascending order (one fma each),
// starting from acc (H a multiple of 8): x is the 64-float activation
// staging (read as 16-byte vectors, the same address in every lane), w a
// bf16 row of 16-byte aligned chunks.
__device__ __forceinline__ float patch_dot(const float *x, const unsigned short *w, int H, float acc) {
  for (int i0 = 0; i0 < H; i0 += 8) {
    const uint4 wv = *(const uint4 *)(w + i0);
    const float4 xa = *(const float4 *)(x + i0);
    const float4 xb = *(const float4 *)(x + i0 + 4);
    const uint32_t wr[4] = {wv.x, wv.y, wv.z, wv.w};
    const float xs[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t word = wr[e >> 1];
      const float we = __uint_as_float((e & 1) ? (word & 0xFFFF0000u) : (word << 16));
      acc = fmaf(xs[e], we, acc);
    }
  }
  return acc;
}

// Forward of one observation (codes[0..63] in LDS, 16-byte aligned, species
// codes < S) by one full wavefront; hbuf is a 64-float, 16-byte aligned LDS
// staging area.  Lane k < n_out returns output k (other lanes return 0).
// Every lane must take part.
__device__ inline float patch_forward(const PatchNet &n, const uint8_t *codes, float *hbuf, int lane) {
  const int H = n.H, S = n.S;
  const int j = lane < H ? lane : H - 1;
  // all 64 codes in scalar registers (the same 64 bytes in every lane), so
  // that each row offset is scalar arithmetic
  uint32_t cw[16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint4 v = *(const uint4 *)(codes + 16 * q);
    cw[4 * q] = __builtin_amdgcn_readfirstlane(v.x);
    cw[4 * q + 1] = __builtin_amdgcn_readfirstlane(v.y);
    cw[4 * q + 2] = __builtin_amdgcn_readfirstlane(v.z);
    cw[4 * q + 3] = __builtin_amdgcn_readfirstlane(v.w);
  }
  float acc = n.b1[j];
  const unsigned short *w1 = n.w1 + j;
#pragma unroll
  for (int m = 0; m < kObsN; ++m) {
    const int c = (int)((cw[m >> 2] >> (8 * (m & 3))) & 255u);
    acc = acc + bf16_to_f32(w1[(m * S + c) * H]);
  }
  const float h1 = acc > 0.0f ? acc : 0.0f;
  wave_sync();
  if (lane < H) hbuf[lane] = h1;
  wave_sync();
  acc = patch_dot(hbuf, n.w2t + j * patch_ldt(H), H, n.b2[j]);
  const float h2 = acc > 0.0f ? acc : 0.0f;
  wave_sync();
  if (lane < H) hbuf[lane] = h2;
  wave_sync();
  const int k = lane < n.n_out ? lane : 0;
  acc = patch_dot(hbuf, n.w3t + k * patch_ldt(H), H, n.b3[k]);
  wave_sync();
  return lane < n.n_out ? acc : 0.0f;
}

}  // namespace akmc
