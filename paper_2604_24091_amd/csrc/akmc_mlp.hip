// Learned barrier surrogate on the matrix cores: environment encoding,
// bulk inference, training (forward, backward, AdamW) and initialisation.
//
// The paper turns its per-atom network evaluations into batched GEMMs on
// matrix units (Sec. III-B1, "swarm gathering"), in reduced precision with
// fused layers, and trains with AdamW at batch 256 (Sec. IV-C).  Here every
// wavefront owns 16 candidates (one 16-row tile of the bf16 16x16x32 MFMA);
// both layers and the activation run in one kernel with the weights staged
// in LDS.  Training splits a batch over wavefronts: each computes the
// gradient of its 16 rows (the weight gradients use the 16x16x16 MFMA with
// the 16 rows as the reduction dimension, reading the activations straight
// from the accumulator layout), and one update kernel sums the partial
// gradients in a fixed order and applies AdamW.
#include <hip/hip_runtime.h>

#include "akmc_device.hpp"
#include "akmc_internal.hpp"
#include "akmc_mlp.hpp"

#include <algorithm>

namespace akmc {

// ------------------------------------------------------------ encoding
// Species codes of the 27 footprint slots of candidate (i, k) in the frame
// where the jump points along (+,+,+): slot 0 the moving species; slots
// 1..7 N1(i) without j by reflected direction 0..6; 8..13 N2(i) by
// reflected 2NN index; 14..20 N1(j) without i by reflected direction 1..7;
// 21..26 N2(j).  Reflecting the axes where the jump is negative maps a
// direction d to d ^ (~k & 7) and swaps the +/- second neighbours of each
// reflected axis.
__global__ __launch_bounds__(256) void k_env_encode(const LatDesc *__restrict__ d,
                                                    const uint8_t *__restrict__ occ,
                                                    const int32_t *__restrict__ sites,
                                                    int64_t n_sites, uint8_t *__restrict__ env,
                                                    float *__restrict__ ea) {
  __shared__ double sD1[64], sD2[64], se0[8];
  const int tid = threadIdx.x;
  if (tid < 64) { sD1[tid] = d->D1[tid]; sD2[tid] = d->D2[tid]; }
  if (tid < 8) se0[tid] = d->e0[tid];
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * 256 + tid;
  if (c >= n_sites * 8) return;
  const int64_t a = c >> 3;
  const int k = (int)(c & 7);
  const Geo g = make_geo(d->lx, d->ly, d->lz);
  const int S = d->S, V = S - 1;
  uint8_t *out = env + c * kSlots;
  const int i = sites ? sites[a] : (int)a;
  if (i < 0 || i >= 2 * g.ncell) {
    for (int s = 0; s < kSlots; ++s) out[s] = (uint8_t)V;
    if (ea) ea[c] = __builtin_huge_valf();
    return;
  }
  int X, Y, Z;
  pos_of(g, i, X, Y, Z);
  const int flip = (~k) & 7;
  const int JX = wrapc(X + dir_sx(k), g.X2), JY = wrapc(Y + dir_sy(k), g.Y2),
            JZ = wrapc(Z + dir_sz(k), g.Z2);
  auto at = [&](int x, int y, int z) { return occ[site_of(g, wrapc(x, g.X2), wrapc(y, g.Y2), wrapc(z, g.Z2))]; };
  const int A = at(JX, JY, JZ);
  out[0] = (uint8_t)A;
  uint32_t c1i = 0, c1j = 0, c2i = 0, c2j = 0;
  for (int dd = 0; dd < 7; ++dd) {
    const int q = dd ^ flip;
    const uint8_t sp = (uint8_t)at(X + dir_sx(q), Y + dir_sy(q), Z + dir_sz(q));
    out[1 + dd] = sp;
    c1i += onehot(sp);
  }
  for (int dd = 1; dd < 8; ++dd) {
    const int q = dd ^ flip;
    const uint8_t sp = (uint8_t)at(JX + dir_sx(q), JY + dir_sy(q), JZ + dir_sz(q));
    out[13 + dd] = sp;
    c1j += onehot(sp);
  }
  for (int m = 0; m < 6; ++m) {
    const int axis = m >> 1;
    const int mm = ((flip >> (2 - axis)) & 1) ? (m ^ 1) : m;
    const int st = (mm & 1) ? -2 : 2;
    const int dx = axis == 0 ? st : 0, dy = axis == 1 ? st : 0, dz = axis == 2 ? st : 0;
    const uint8_t si = (uint8_t)at(X + dx, Y + dy, Z + dz);
    const uint8_t sj = (uint8_t)at(JX + dx, JY + dy, JZ + dz);
    out[8 + m] = si;
    out[21 + m] = sj;
    c2i += onehot(si);
    c2j += onehot(sj);
  }
  if (ea) {
    if (A == V) {
      ea[c] = __builtin_huge_valf();
    } else {
      const double de = delta_e_counts<double>(c1i, c1j, c2i, c2j, sD1 + 8 * A, sD2 + 8 * A);
      ea[c] = (float)(se0[A] + 0.5 * de);
    }
  }
}

// Largest per-species count of each bond group over a data set (for the
// out-of-distribution test of the surrogate).
__global__ __launch_bounds__(256) void k_ood_fit(const uint8_t *__restrict__ env, int64_t n, int S,
                                                 MlpHeader *__restrict__ hdr) {
  __shared__ int smax[5][8];
  const int tid = threadIdx.x;
  if (tid < 40) smax[tid >> 3][tid & 7] = 0;
  __syncthreads();
  int loc[5][8];
#pragma unroll
  for (int g = 0; g < 5; ++g)
#pragma unroll
    for (int s = 0; s < 8; ++s) loc[g][s] = 0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + tid; r < n; r += (int64_t)gridDim.x * 256) {
    const uint8_t *e = env + r * kSlots;
    if (e[0] == S - 1) continue;
    int cnt[5][8] = {};
    cnt[4][e[0] & 7] = 1;
    for (int s = 1; s < 8; ++s) cnt[0][e[s] & 7] += 1;
    for (int s = 8; s < 14; ++s) cnt[1][e[s] & 7] += 1;
    for (int s = 14; s < 21; ++s) cnt[2][e[s] & 7] += 1;
    for (int s = 21; s < 27; ++s) cnt[3][e[s] & 7] += 1;
#pragma unroll
    for (int g = 0; g < 5; ++g)
#pragma unroll
      for (int s = 0; s < 8; ++s) loc[g][s] = max(loc[g][s], cnt[g][s]);
  }
#pragma unroll
  for (int g = 0; g < 5; ++g)
#pragma unroll
    for (int s = 0; s < 8; ++s) atomicMax(&smax[g][s], loc[g][s]);
  __syncthreads();
  if (tid < 40) atomicMax(&hdr->ood_max[tid >> 3][tid & 7], smax[tid >> 3][tid & 7]);
  if (tid == 0 && blockIdx.x == 0) hdr->ood_valid = 1;
}

// ------------------------------------------------------ weight staging

// ------------------------------------------------------ bulk inference

// Per training wavefront: 16 rows of 32 codes, then one area for the
// one-hot input tile and, once layer 1 has read it, the 16-row activation
// tile (one wavefront's LDS operations take effect in program order).
constexpr int kWaveBytes = 512 + kTileBytes;

// Bulk inference: a block of up to kFwdWavesMax wavefronts shares the
// weights staged in LDS; each wavefront owns one tile area sized for the
// species count (fwd_wave_bytes), holding the one-hot input tile and, once
// layer 1 has read it, the 16-row activation tile (one wavefront's LDS
// operations take effect in program order).
constexpr int kFwdWavesMax = 16;
__host__ __device__ inline int fwd_wave_bytes(int k1) {
  const int a = 2 * 16 * mlp_ld1(k1), h = 2 * 16 * kLdH;
  return a > h ? a : h;
}

__global__ __launch_bounds__(64 * kFwdWavesMax) void k_mlp_forward(const unsigned char *__restrict__ blob,
                                                                   const uint8_t *__restrict__ env,
                                                                   int64_t n, float *__restrict__ ea) {
  extern __shared__ __align__(16) unsigned char mlp_lds[];
  const MlpHeader *hdr = (const MlpHeader *)blob;
  const int S = hdr->S, k1 = hdr->k1;
  const MlpLayout L = mlp_layout(S);
  unsigned short *w1t = (unsigned short *)mlp_lds;
  unsigned short *w2t = w1t + kHid * mlp_ld1(k1);
  unsigned char *per_wave = (unsigned char *)(w2t + kHid * kLdH);
  stage_rows8(w1t, (const unsigned short *)(blob + L.w1t), kHid, k1, mlp_ld1(k1), threadIdx.x, blockDim.x);
  stage_rows8(w2t, (const unsigned short *)(blob + L.w2t), kHid, kHid, kLdH, threadIdx.x, blockDim.x);
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
  unsigned short *atile = (unsigned short *)(per_wave + wave * fwd_wave_bytes(k1));
  unsigned short *hst = atile;
  const float *prm = (const float *)(blob + L.params);
  const float mu = hdr->mu, sigma = hdr->sigma;
  __syncthreads();
  const int64_t tiles = (n + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * nw + wave; tile < tiles; tile += (int64_t)gridDim.x * nw) {
    const int64_t row0 = tile * 16;
    unsigned short h1b[8][4], h2b[8][4];
    float gp1[8][4], gp2[8][4], y[4];
    onehot_tile_rows(env, row0, n, atile, S, k1, l);
    mlp_fwd16<false, true>((const uint8_t *)atile, w1t, w2t, hst, prm, L, S, k1, h1b, h2b, gp1, gp2, y);
    if ((l & 15) == 0) {
      const int q = l >> 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + 4 * q + i;
        if (row < n) ea[row] = mu + sigma * y[i];
      }
    }
  }
}

// ------------------------------------------------------------ training

constexpr int kTrainWaves = 4;

// Dataset row of batch position b: a keyed bijection of [0, n) (four-round
// Feistel network on the next power of two with cycle walking), a fresh
// permutation per epoch.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}
__device__ __forceinline__ int64_t permute_row(int64_t b, int64_t n, uint64_t key, int bits) {
  const int hb = bits / 2;
  const uint32_t lo_mask = (1u << hb) - 1u;
  uint32_t x = (uint32_t)b;
  do {
    uint32_t L = x >> hb, R = x & lo_mask;
    for (int rnd = 0; rnd < 4; ++rnd) {
      const uint32_t F = mix32(R ^ (uint32_t)(key >> (16 * rnd)) ^ (0x9E3779B9u * (rnd + 1))) & lo_mask;
      const uint32_t nl = R, nr = L ^ F;
      L = nl;
      R = nr;
    }
    x = (L << hb) | R;
  } while ((int64_t)x >= n);
  return (int64_t)x;
}

struct TrainArgs {
  const unsigned char *blob;
  const uint8_t *env;
  const float *ea;
  int64_t n;            // data set rows
  int32_t batch;        // rows per step (multiple of 16)
  int32_t rows;         // rows of this step (<= batch; the rest contribute nothing)
  int64_t start;        // first batch position of this step in the epoch order
  uint64_t perm_key;    // 0: identity order
  int32_t perm_bits;
  float *partial;       // [n_waves][nparams + 1] (last: loss partial)
};

__global__ __launch_bounds__(64 * kTrainWaves) void k_mlp_train_partial(TrainArgs ta) {
  extern __shared__ __align__(16) unsigned char mlp_lds[];
  const MlpHeader *hdr = (const MlpHeader *)ta.blob;
  const int S = hdr->S, k1 = hdr->k1, np = hdr->nparams;
  const MlpLayout L = mlp_layout(S);
  unsigned short *w1t = (unsigned short *)mlp_lds;
  unsigned short *w2t = w1t + kHid * mlp_ld1(k1);
  unsigned short *w2r = w2t + kHid * kLdH;
  unsigned char *per_wave = (unsigned char *)(w2r + kHid * kLdH);
  stage_rows8(w1t, (const unsigned short *)(ta.blob + L.w1t), kHid, k1, mlp_ld1(k1), threadIdx.x, blockDim.x);
  stage_rows8(w2t, (const unsigned short *)(ta.blob + L.w2t), kHid, kHid, kLdH, threadIdx.x, blockDim.x);
  stage_rows8(w2r, (const unsigned short *)(ta.blob + L.w2r), kHid, kHid, kLdH, threadIdx.x, blockDim.x);
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
  uint8_t *senv = per_wave + wave * kWaveBytes;
  unsigned short *hst = (unsigned short *)(senv + 512);
  unsigned short *atile = hst;
  const float *prm = (const float *)(ta.blob + L.params);
  const float mu = hdr->mu, sigma = hdr->sigma;
  const int gw = blockIdx.x * kTrainWaves + wave;  // wavefront index within the batch
  const int row0 = gw * 16;
  __shared__ float s_t[kTrainWaves][16];
  __shared__ int s_valid[kTrainWaves][16];
  if (l < 16) {
    const int b = row0 + l;
    float t = 0.f;
    int valid = 0;
    int64_t row = -1;
    if (b < ta.rows) {
      const int64_t pos = ta.start + b;
      row = ta.perm_key ? permute_row(pos, ta.n, ta.perm_key, ta.perm_bits) : pos;
    }
    for (int s = 0; s < 32; ++s)
      senv[l * 32 + s] = (row >= 0 && s < kSlots) ? ta.env[row * kSlots + s] : 0;
    if (row >= 0 && senv[l * 32] != S - 1) {
      valid = 1;
      t = (ta.ea[row] - mu) / sigma;
    }
    s_t[wave][l] = t;
    s_valid[wave][l] = valid;
  }
  __syncthreads();

  unsigned short h1b[8][4], h2b[8][4];
  float gp1[8][4], gp2[8][4], y[4];
  onehot_tile(senv, atile, S, k1, l);
  mlp_fwd16<true, true>((const uint8_t *)atile, w1t, w2t, hst, prm, L, S, k1, h1b, h2b, gp1, gp2, y);

  float *part = ta.partial + (size_t)gw * (size_t)(np + 1);
  const float inv_b = 2.0f / (float)max(ta.rows, 1);   // d(mean loss)/dy over this step's rows
  float dy[4];
  float lsum = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = 4 * q + i;
    const float d = s_valid[wave][row] ? (y[i] - s_t[wave][row]) : 0.f;
    dy[i] = d * inv_b;
    lsum += d * d;
  }
  // Loss and output-layer gradients (rows are spread over the 4 row groups).
  float db3 = dy[0] + dy[1] + dy[2] + dy[3];
  db3 += __shfl_xor(db3, 16, 64);
  db3 += __shfl_xor(db3, 32, 64);
  lsum += __shfl_xor(lsum, 16, 64);
  lsum += __shfl_xor(lsum, 32, 64);
  if (l == 0) {
    part[L.ob3] = db3;
    part[np] = lsum;
  }
  float dz2[8][4];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const float w3 = bf2f(f2bf(prm[L.ow3 + 16 * c + r]));
    float dw3 = 0.f, db2 = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dw3 = fmaf(bf2f(h2b[c][i]), dy[i], dw3);
      dz2[c][i] = dy[i] * w3 * gp2[c][i];
      db2 += dz2[c][i];
    }
    dw3 += __shfl_xor(dw3, 16, 64);
    dw3 += __shfl_xor(dw3, 32, 64);
    db2 += __shfl_xor(db2, 16, 64);
    db2 += __shfl_xor(db2, 32, 64);
    if (q == 0) {
      part[L.ow3 + 16 * c + r] = dw3;
      part[L.ob2 + 16 * c + r] = db2;
    }
  }
  // dW2[i][o] = sum_rows h1[row][i] dz2[row][o]: the 16 rows are the
  // reduction dimension; both operands are already in the accumulator layout.
  s16x4 dz2b[8];
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned short hb = f2bf(dz2[c][i]);
      dz2b[c][i] = (short)hb;
      hst[(4 * q + i) * kLdH + 16 * c + r] = hb;
    }
#pragma unroll
  for (int ti = 0; ti < 8; ++ti) {
    s16x4 a;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = (short)h1b[ti][i];
#pragma unroll
    for (int to = 0; to < 8; ++to) {
      f32x4 cacc = {0.f, 0.f, 0.f, 0.f};
      cacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, dz2b[to], cacc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) part[L.oW2 + (16 * ti + 4 * q + i) * kHid + 16 * to + r] = cacc[i];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // dh1 = dz2 W2^T (A = dz2 rows from the staging tile, B = W2 row-major).
  f32x4 acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bf16x8 a = *(const bf16x8 *)(hst + r * kLdH + 32 * t + 8 * q);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const bf16x8 b = *(const bf16x8 *)(w2r + (16 * c + r) * kLdH + 32 * t + 8 * q);
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
  }
  s16x4 dz1b[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    float db1 = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float dz = acc[c][i] * gp1[c][i];
      db1 += dz;
      dz1b[c][i] = (short)f2bf(dz);
    }
    db1 += __shfl_xor(db1, 16, 64);
    db1 += __shfl_xor(db1, 32, 64);
    if (q == 0) part[L.ob1 + 16 * c + r] = db1;
  }
  // dW1[f][n] = sum_rows x[row][f] dz1[row][n]; x from the species codes.
  const int nf = k1 / 16;
  for (int tf = 0; tf < nf; ++tf) {
    const int f = 16 * tf + r;
    const int slot = div_s(f, s_magic(S)), sp = f - slot * S;
    s16x4 a;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool one = slot < kSlots && senv[(4 * q + i) * 32 + slot] == sp;
      a[i] = (short)(one ? 0x3F80 : 0);
    }
#pragma unroll
    for (int tn = 0; tn < 8; ++tn) {
      f32x4 cacc = {0.f, 0.f, 0.f, 0.f};
      cacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, dz1b[tn], cacc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) part[L.oW1 + (16 * tf + 4 * q + i) * kHid + 16 * tn + r] = cacc[i];
    }
  }
}

// Sums the partial gradients in wavefront order and applies one AdamW step
// (decoupled weight decay, bias-corrected moments); refreshes the bf16
// copies.  grad_out (optional) receives the summed gradient instead of an
// update when apply == 0.
__global__ __launch_bounds__(256) void k_mlp_update(unsigned char *__restrict__ blob,
                                                    const float *__restrict__ partial, int n_waves,
                                                    int apply, float lr, float beta1, float beta2,
                                                    float eps, float wd, int step,
                                                    float *__restrict__ grad_out,
                                                    float *__restrict__ loss_out, float inv_rows) {
  MlpHeader *hdr = (MlpHeader *)blob;
  const int S = hdr->S, k1 = hdr->k1, np = hdr->nparams;
  const MlpLayout L = mlp_layout(S);
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p == 0 && loss_out) {
    float ls = 0.f;
    for (int w = 0; w < n_waves; ++w) ls += partial[(size_t)w * (np + 1) + np];
    *loss_out = ls * inv_rows;
  }
  if (p >= np) return;
  float g = 0.f;
  for (int w = 0; w < n_waves; ++w) g += partial[(size_t)w * (np + 1) + p];
  if (!apply) {
    grad_out[p] = g;
    return;
  }
  float *prm = (float *)(blob + L.params);
  float *m = (float *)(blob + L.m);
  float *v = (float *)(blob + L.v);
  float th = prm[p] * (1.0f - lr * wd);
  const float mm = beta1 * m[p] + (1.0f - beta1) * g;
  const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float bc1 = 1.0f - powf(beta1, (float)step), bc2 = 1.0f - powf(beta2, (float)step);
  th -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
  prm[p] = th;
  const unsigned short hb = f2bf(th);
  if (p < L.ob1) {
    const int f = p / kHid, nn = p - f * kHid;
    ((unsigned short *)(blob + L.w1t))[nn * k1 + f] = hb;
  } else if (p >= L.oW2 && p < L.ob2) {
    const int i = (p - L.oW2) / kHid, o = (p - L.oW2) - i * kHid;
    ((unsigned short *)(blob + L.w2t))[o * kHid + i] = hb;
    ((unsigned short *)(blob + L.w2r))[i * kHid + o] = hb;
  }
  if (p == 0) hdr->step = step;
}

// Writes the bf16 copies of the current parameters.
__global__ __launch_bounds__(256) void k_mlp_sync_bf16(unsigned char *__restrict__ blob) {
  const MlpHeader *hdr = (const MlpHeader *)blob;
  const int S = hdr->S, k1 = hdr->k1, np = hdr->nparams;
  const MlpLayout L = mlp_layout(S);
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const float *prm = (const float *)(blob + L.params);
  const unsigned short hb = f2bf(prm[p]);
  if (p < L.ob1) {
    const int f = p / kHid, nn = p - f * kHid;
    ((unsigned short *)(blob + L.w1t))[nn * k1 + f] = hb;
  } else if (p >= L.oW2 && p < L.ob2) {
    const int i = (p - L.oW2) / kHid, o = (p - L.oW2) - i * kHid;
    ((unsigned short *)(blob + L.w2t))[o * kHid + i] = hb;
    ((unsigned short *)(blob + L.w2r))[i * kHid + o] = hb;
  }
}

// Uniform initialisation from the Philox stream (counter = parameter
// index): W1 ~ U(-sqrt(3/27), +) (27 active inputs per row), W2 and w3 ~
// U(-sqrt(3/128), +), biases zero; moments zero.
__global__ __launch_bounds__(256) void k_mlp_init(unsigned char *__restrict__ blob, uint64_t seed) {
  const MlpHeader *hdr = (const MlpHeader *)blob;
  const int S = hdr->S, np = hdr->nparams;
  const MlpLayout L = mlp_layout(S);
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  float *prm = (float *)(blob + L.params);
  uint64_t x[4];
  philox4x64_10((uint64_t)p, 0, 0, 0, seed, 0x6d6c70ull, x);
  const float u = (float)((double)(x[0] >> 11) * 1.1102230246251565404e-16) * 2.0f - 1.0f;
  float a = 0.f;
  if (p < L.ob1) a = sqrtf(3.0f / 27.0f);
  else if (p >= L.oW2 && p < L.ob2) a = sqrtf(3.0f / kHid);
  else if (p >= L.ow3 && p < L.ob3) a = sqrtf(3.0f / kHid);
  prm[p] = a * u;
  ((float *)(blob + L.m))[p] = 0.f;
  ((float *)(blob + L.v))[p] = 0.f;
}

// ------------------------------------------------------------ launchers

static size_t fwd_weight_bytes(int S) { return (size_t)2 * kHid * mlp_ld1(mlp_k1(S)) + 2 * kHid * kLdH; }
static size_t train_lds(int S) {
  return (size_t)2 * kHid * mlp_ld1(mlp_k1(S)) + 2 * (size_t)2 * kHid * kLdH + kTrainWaves * kWaveBytes;
}

hipError_t launch_env_encode(const LatDesc *d_desc, const uint8_t *occ, const int32_t *sites,
                             int64_t n_sites, uint8_t *env, float *ea, hipStream_t stream) {
  if (n_sites <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_sites * 8 + 255) / 256);
  hipLaunchKernelGGL(k_env_encode, dim3(blocks), dim3(256), 0, stream, d_desc, occ, sites, n_sites, env, ea);
  return hipGetLastError();
}

hipError_t launch_ood_fit(unsigned char *blob, const uint8_t *env, int64_t n, int S, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_ood_fit, dim3(blocks), dim3(256), 0, stream, env, n, S, (MlpHeader *)blob);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const unsigned char *blob, int S, const uint8_t *env, int64_t n,
                              float *ea, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  // As many wavefronts per block as the LDS left by the weights holds, and
  // a persistent grid of as many blocks as the CUs hold at once.
  const size_t wbytes = fwd_weight_bytes(S), per = (size_t)fwd_wave_bytes(mlp_k1(S));
  const int waves = (int)std::min<size_t>(kFwdWavesMax, (kLdsBytes - wbytes) / per);
  const size_t lds = wbytes + (size_t)waves * per;
  hipError_t e = hipFuncSetAttribute((const void *)k_mlp_forward, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int64_t per_cu = std::max<int64_t>(1, (int64_t)(kLdsBytes / lds));
  const int64_t tiles = (n + 15) / 16;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + waves - 1) / waves, (int64_t)cus * per_cu));
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(64 * waves), lds, stream, blob, env, n, ea);
  return hipGetLastError();
}

hipError_t launch_mlp_init(unsigned char *blob, int S, uint64_t seed, hipStream_t stream) {
  const int np = mlp_nparams(S);
  hipLaunchKernelGGL(k_mlp_init, dim3((np + 255) / 256), dim3(256), 0, stream, blob, seed);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_sync_bf16, dim3((np + 255) / 256), dim3(256), 0, stream, blob);
  return hipGetLastError();
}

hipError_t launch_mlp_sync(unsigned char *blob, int S, hipStream_t stream) {
  const int np = mlp_nparams(S);
  hipLaunchKernelGGL(k_mlp_sync_bf16, dim3((np + 255) / 256), dim3(256), 0, stream, blob);
  return hipGetLastError();
}

// One step: partial gradients of `rows` rows (batch positions start ..
// start+rows-1 of the epoch order), then the sum and (if apply) AdamW.
hipError_t launch_mlp_step(unsigned char *blob, int S, const uint8_t *env, const float *ea,
                           int64_t n, int batch, int rows, int64_t start, uint64_t perm_key,
                           int perm_bits, float *partial, int apply, float lr, float beta1,
                           float beta2, float eps, float wd, int step, float *grad_out,
                           float *loss_out, hipStream_t stream) {
  const size_t lds = train_lds(S);
  hipError_t e = hipFuncSetAttribute((const void *)k_mlp_train_partial, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  TrainArgs ta;
  ta.blob = blob;
  ta.env = env;
  ta.ea = ea;
  ta.n = n;
  ta.batch = batch;
  ta.rows = rows;
  ta.start = start;
  ta.perm_key = perm_key;
  ta.perm_bits = perm_bits;
  ta.partial = partial;
  const int n_waves = batch / 16;
  const unsigned blocks = (unsigned)((n_waves + kTrainWaves - 1) / kTrainWaves);
  hipLaunchKernelGGL(k_mlp_train_partial, dim3(blocks), dim3(64 * kTrainWaves), lds, stream, ta);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int np = mlp_nparams(S);
  hipLaunchKernelGGL(k_mlp_update, dim3((np + 255) / 256), dim3(256), 0, stream, blob, partial,
                     (int)(blocks * kTrainWaves), apply, lr, beta1, beta2, eps, wd, step, grad_out,
                     loss_out, 1.0f / (float)std::max(rows, 1));
  return hipGetLastError();
}

size_t mlp_partial_bytes(int S, int batch) {
  const int n_waves = ((batch / 16 + kTrainWaves - 1) / kTrainWaves) * kTrainWaves;
  return sizeof(float) * (size_t)n_waves * (size_t)(mlp_nparams(S) + 1);
}

}  // namespace akmc
