// Learned barrier surrogate: layout of the weight blob and the device
// forward pass shared by the bulk inference, training and event-loop
// kernels.
//
// Network (per candidate): 27 footprint slots in the jump frame, one-hot
// over S species, zero-padded to K1 = 32*ceil(27*S/32) inputs;
//   h1 = gelu(x W1 + b1), h2 = gelu(h1 W2 + b2), y = h2 . w3 + b3,
//   Ea = mu + sigma*y,   gelu(z) = z/2 (1 + tanh(sqrt(2/pi)(z + 0.044715 z^3))).
// Weights and activations are bfloat16 on the matrix cores with binary32
// accumulation; biases, the output layer sum and the optimiser state are
// binary32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace akmc {

constexpr int kHid = 128;
// LDS row pitch of staged weights and activations, in bf16 elements: 16
// bytes beyond the data, so that the 16 lanes of a row group, which read
// 16 consecutive rows at the same column, fall on different banks.
constexpr int kPad = 8;
constexpr int kLdH = kHid + kPad;
__host__ __device__ constexpr int mlp_ld1(int k1) { return k1 + kPad; }
constexpr int kSlots = 27;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int mlp_k1(int S) { return 32 * ((kSlots * S + 31) / 32); }
// Bytes of a 16-row one-hot input tile at the largest species count (8); the
// tile and the 16-row activation tile of the forward share this area.
constexpr int kTileBytes = 2 * 16 * mlp_ld1(mlp_k1(8));
static_assert(kTileBytes >= 2 * 16 * kLdH, "the activation tile fits the shared area");
__host__ __device__ inline int mlp_nparams(int S) {
  const int k1 = mlp_k1(S);
  return k1 * kHid + kHid + kHid * kHid + kHid + kHid + 1;
}

// Header at the start of the blob.
struct MlpHeader {
  int32_t S, k1, nparams, step;
  float mu, sigma;
  int32_t ood_valid;
  int32_t pad_;
  int32_t ood_max[5][8];  // largest per-species count seen in training: 4 bond groups, then the moving species
};

// Byte offsets inside the blob; every segment 256-byte aligned.
struct MlpLayout {
  size_t hdr, params, m, v, w1t, w2t, w2r, total;
  // element offsets inside the parameter vector
  int oW1, ob1, oW2, ob2, ow3, ob3;
};

__host__ __device__ inline size_t mlp_up(size_t x) { return (x + 255) & ~size_t(255); }

__host__ __device__ inline MlpLayout mlp_layout(int S) {
  MlpLayout L;
  const int k1 = mlp_k1(S), np = mlp_nparams(S);
  size_t o = 0;
  L.hdr = o;    o += mlp_up(sizeof(MlpHeader));
  L.params = o; o += mlp_up(sizeof(float) * (size_t)np);
  L.m = o;      o += mlp_up(sizeof(float) * (size_t)np);
  L.v = o;      o += mlp_up(sizeof(float) * (size_t)np);
  L.w1t = o;    o += mlp_up(2 * (size_t)kHid * k1);
  L.w2t = o;    o += mlp_up(2 * (size_t)kHid * kHid);
  L.w2r = o;    o += mlp_up(2 * (size_t)kHid * kHid);
  L.total = o;
  L.oW1 = 0;
  L.ob1 = L.oW1 + k1 * kHid;
  L.oW2 = L.ob1 + kHid;
  L.ob2 = L.oW2 + kHid * kHid;
  L.ow3 = L.ob2 + kHid;
  L.ob3 = L.ow3 + kHid;
  return L;
}

// slot = f / S for 0 <= f < 224 and 2 <= S <= 8: f * ceil(2^16/S) >> 16 is
// exact there (the rounding excess stays below 224/2^16 < 1/S).
__device__ __forceinline__ int div_s(int f, int magic) { return (f * magic) >> 16; }
__host__ __device__ inline int s_magic(int S) { return (65536 + S - 1) / S; }

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even: the hardware conversion (v_cvt_pk_bf16_f32)
  return __builtin_bit_cast(unsigned short, (__bf16)f);
}
// Two values to bfloat16 with one conversion; the first in the low half.
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
__device__ __forceinline__ float bf2f(unsigned short h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// GELU in its tanh form, evaluated as z times a logistic function:
//   gelu(z) = z/2 (1 + tanh u) = z s,  s = 1 / (1 + e^{-2u}),
//   u = sqrt(2/pi) (z + 0.044715 z^3),
// with one hardware base-2 exponential and one reciprocal (about 1e-7
// relative, far below the bfloat16 rounding of the activations).  The
// exponent -2u log2(e) is formed as z (b + a z^2), b = -2 sqrt(2/pi) log2(e),
// a = 0.044715 b.
__device__ __forceinline__ float gelu_sig(float z) {
  const float b = -(2.0f * 0.7978845608028654f * 1.4426950408889634f);
  const float a = 0.044715f * b;
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * fmaf(a * z, z, b)));
}
__device__ __forceinline__ float gelu_f(float z) { return z * gelu_sig(z); }
// d/dz [z s] = s + z s (1 - s) 2u'(z),  u' = sqrt(2/pi) (1 + 3 * 0.044715 z^2)
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float c = 0.7978845608028654f;
  const float s = gelu_sig(z);
  return s + z * s * (1.0f - s) * (2.0f * c) * fmaf(3.0f * 0.044715f * z, z, 1.0f);
}

// Copies rows x cols bf16 values (cols a multiple of 8) from a dense array
// into LDS rows of pitch ld, 16 bytes per thread and step.
__device__ __forceinline__ void stage_rows(unsigned short *dst, const unsigned short *src, int rows,
                                           int cols, int ld, int tid, int nthreads) {
  const int per_row = cols / 8;
  for (int u = tid; u < rows * per_row; u += nthreads) {
    const int r = u / per_row, c8 = u - r * per_row;
    *(uint4 *)(dst + r * ld + 8 * c8) = *(const uint4 *)(src + r * cols + 8 * c8);
  }
}

// The same copy with eight loads in flight per thread before their stores,
// for kernels that stage the weights once per block before any other work
// (the registers are free then).
__device__ __forceinline__ void stage_rows8(unsigned short *dst, const unsigned short *src, int rows,
                                            int cols, int ld, int tid, int nthreads) {
  const int per_row = cols / 8, total = rows * per_row;
  int u = tid;
  for (; u + 7 * nthreads < total; u += 8 * nthreads) {
    uint4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int w = u + k * nthreads, r = w / per_row, c8 = w - r * per_row;
      v[k] = *(const uint4 *)(src + r * cols + 8 * c8);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int w = u + k * nthreads, r = w / per_row, c8 = w - r * per_row;
      *(uint4 *)(dst + r * ld + 8 * c8) = v[k];
    }
  }
  for (; u < total; u += nthreads) {
    const int r = u / per_row, c8 = u - r * per_row;
    *(uint4 *)(dst + r * ld + 8 * c8) = *(const uint4 *)(src + r * cols + 8 * c8);
  }
}

// One-hot input tile of 16 rows (bf16, pitch mlp_ld1(k1)) from 16 rows of
// 32 species codes (the first kSlots used): the wavefront clears the tile,
// then sets feature slot*S + code of every (row, slot); a code >= S sets
// nothing (rows without a candidate).
__device__ __forceinline__ void onehot_tile(const uint8_t *codes, unsigned short *atile, int S, int k1,
                                            int lane) {
  const int ld = mlp_ld1(k1);
  for (int u = lane; u < 16 * ld / 8; u += 64) *(uint4 *)(atile + 8 * u) = make_uint4(0u, 0u, 0u, 0u);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // Element u = lane + 64 j (row u / kSlots, slot u % kSlots): every code is
  // read before the first store; the source and tile offsets advance by 64
  // elements per j (64 = 2 kSlots + 10, so slot wraps at most once a step).
  constexpr int kJ = (16 * kSlots + 63) / 64;
  constexpr int kStep = 64 - 2 * kSlots;
  static_assert(kStep >= 0 && kStep < kSlots, "one wrap per step");
  int code[kJ];
  {
    int slot = lane % kSlots, src = (lane / kSlots) * 32 + slot;
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
      code[j] = lane + 64 * j < 16 * kSlots ? codes[src] : S;
      slot += kStep;
      src += 2 * 32 + kStep;
      if (slot >= kSlots) {
        slot -= kSlots;
        src += 32 - kSlots;
      }
    }
  }
  int slot = lane % kSlots;
  int d = (lane / kSlots) * ld + slot * S;
  const int step = 2 * ld + kStep * S, wrap = ld - kSlots * S;
#pragma unroll
  for (int j = 0; j < kJ; ++j) {
    if (code[j] < S) atile[d + code[j]] = 0x3F80;  // bf16 1.0
    slot += kStep;
    d += step;
    if (slot >= kSlots) {
      slot -= kSlots;
      d += wrap;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same tile straight from n rows of kSlots codes in global memory, rows
// row0 .. row0+15 (rows past n, and codes >= S, set no feature).
__device__ __forceinline__ void onehot_tile_rows(const uint8_t *env, int64_t row0, int64_t n,
                                                 unsigned short *atile, int S, int k1, int lane) {
  const int ld = mlp_ld1(k1);
  for (int u = lane; u < 16 * ld / 8; u += 64) *(uint4 *)(atile + 8 * u) = make_uint4(0u, 0u, 0u, 0u);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int rows = n - row0 < 16 ? (int)(n - row0) : 16;
  const uint8_t *src = env + row0 * kSlots;  // rows are contiguous: element u = row * kSlots + slot
  // Element u = lane + 64 j: every code is loaded before the first store,
  // and the tile offset row * ld + slot * S advances by 64 elements per j
  // (64 = 2 kSlots + 10, so slot wraps at most once per step).
  constexpr int kJ = (16 * kSlots + 63) / 64;
  static_assert(64 - 2 * kSlots >= 0 && 64 - 2 * kSlots < kSlots, "one wrap per step");
  const int nu = rows * kSlots;
  int code[kJ];
#pragma unroll
  for (int j = 0; j < kJ; ++j) code[j] = lane + 64 * j < nu ? src[lane + 64 * j] : S;
  int slot = lane % kSlots;
  int d = (lane / kSlots) * ld + slot * S;
  const int step = 2 * ld + (64 - 2 * kSlots) * S, wrap = ld - kSlots * S;
#pragma unroll
  for (int j = 0; j < kJ; ++j) {
    if (code[j] < S) atile[d + code[j]] = 0x3F80;  // bf16 1.0
    slot += 64 - 2 * kSlots;
    d += step;
    if (slot >= kSlots) {
      slot -= kSlots;
      d += wrap;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward pass of 16 rows by one wavefront.
//   env:   LDS, 16 rows x 32 bytes of species codes (27 used), or with
//          ATILE the one-hot tile built by onehot_tile
//   w1t:   LDS, bf16 [128][k1 + kPad]   (output feature major, padded rows)
//   w2t:   LDS, bf16 [128][kLdH]
//   hst:   LDS, bf16 [16][kLdH] staging of one activation tile
//   prm:   binary32 parameter vector (biases, w3, b3)
// Results per lane (C layout of the 16x16 matrix-core tiles: lane l holds
// rows 4*(l/16)+i, column 16*c + l%16 of tile c):
//   h1b[c][i], h2b[c][i]  bf16 activations; gp1/gp2 gelu'(z) (if GRAD);
//   y[i] for rows 4*(l/16)+i (sum over all columns, identical in the 16
//   lanes of a row group).
template <bool GRAD, bool ATILE = false>
__device__ __forceinline__ void mlp_fwd16(const uint8_t *env, const unsigned short *w1t,
                                          const unsigned short *w2t, unsigned short *hst,
                                          const float *prm, const MlpLayout &L, int S, int k1,
                                          unsigned short (&h1b)[8][4], unsigned short (&h2b)[8][4],
                                          float (&gp1)[8][4], float (&gp2)[8][4], float (&y)[4]) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
  // Layer 1: A from the one-hot codes (row r, features 32t + 8q .. +7).
  // The first product of every tile takes a zero accumulator operand.
  f32x4 acc[8];
  const int nk = k1 / 32;
  __builtin_assume(nk >= 1);  // k1 = 32 * ceil(27 S / 32) with S >= 2
  const int mg = s_magic(S);
  for (int t = 0; t < nk; ++t) {
    bf16x8 a;
    if (ATILE) {
      a = *(const bf16x8 *)((const unsigned short *)env + r * mlp_ld1(k1) + 32 * t + 8 * q);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int f = 32 * t + 8 * q + i;
        const int slot = div_s(f, mg), sp = f - slot * S;
        const bool one = slot < kSlots && env[r * 32 + slot] == sp;
        a[i] = __builtin_bit_cast(__bf16, (unsigned short)(one ? 0x3F80 : 0));
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const bf16x8 b = *(const bf16x8 *)(w1t + (16 * c + r) * mlp_ld1(k1) + 32 * t + 8 * q);
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          a, b, t == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[c], 0, 0, 0);
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const float bias = prm[L.ob1 + 16 * c + r];
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
      const float z0 = acc[c][i] + bias, z1 = acc[c][i + 1] + bias;
      const uint32_t hp = f2bf2(gelu_f(z0), gelu_f(z1));
      h1b[c][i] = (unsigned short)hp;
      h1b[c][i + 1] = (unsigned short)(hp >> 16);
      if (GRAD) {
        gp1[c][i] = gelu_grad_f(z0);
        gp1[c][i + 1] = gelu_grad_f(z1);
      }
      hst[(4 * q + i) * kLdH + 16 * c + r] = (unsigned short)hp;
      hst[(4 * q + i + 1) * kLdH + 16 * c + r] = (unsigned short)(hp >> 16);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // Layer 2: A = h1 rows from the staging tile.
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bf16x8 a = *(const bf16x8 *)(hst + r * kLdH + 32 * t + 8 * q);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const bf16x8 b = *(const bf16x8 *)(w2t + (16 * c + r) * kLdH + 32 * t + 8 * q);
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          a, b, t == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[c], 0, 0, 0);
    }
  }
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const float bias = prm[L.ob2 + 16 * c + r];
    const float w3 = bf2f(f2bf(prm[L.ow3 + 16 * c + r]));
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
      const float z0 = acc[c][i] + bias, z1 = acc[c][i + 1] + bias;
      const uint32_t hp = f2bf2(gelu_f(z0), gelu_f(z1));
      h2b[c][i] = (unsigned short)hp;
      h2b[c][i + 1] = (unsigned short)(hp >> 16);
      if (GRAD) {
        gp2[c][i] = gelu_grad_f(z0);
        gp2[c][i + 1] = gelu_grad_f(z1);
      }
      part[i] = fmaf(__builtin_bit_cast(float, hp << 16), w3, part[i]);
      part[i + 1] = fmaf(__builtin_bit_cast(float, hp & 0xffff0000u), w3, part[i + 1]);
    }
  }
  // Sum the 16 lanes of each row group (lanes 16q .. 16q+15).
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float v = part[i];
    v += __shfl_xor(v, 8, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 1, 16);
    y[i] = v + prm[L.ob3];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace akmc
