// Learned barrier surrogate on the matrix cores: environment encoding,
// bulk inference, training (forward, backward, AdamW) and initialisation.
//
// The paper turns its per-atom network evaluations into batched GEMMs on
// matrix units (Sec. III-B1, "swarm gathering"), in reduced precision with
// fused layers, and trains with AdamW at batch 256 (Sec. IV-C).  Here every
// wavefront owns 16 candidates (one 16-row tile of the bf16 16x16x32 MFMA);
// both layers and the activation run in one kernel with the weights staged
// in LDS.  Training gives every 16 rows of a batch a block of 8
// wavefronts, one per 16 hidden units: each computes its tile of both
// layers and of the gradients (the weight gradients on the 16x16x16 MFMA
// with the 16 rows as the reduction dimension), the activation tiles pass
// through LDS, and one update kernel sums the blocks' partial gradients in
// a fixed order and applies AdamW.
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

// Partial gradients of one wavefront: nparams + 1 floats (the last is the
// loss partial), padded to a multiple of 4.  The weight matrices W1 and W2
// are stored in the order of the 16x16 MFMA accumulator tiles that produce
// them (tile by tile, lane by lane, the lane's 4 rows), so that each tile
// is one 16-byte store per lane; part_index maps a parameter index there.
__host__ __device__ inline int part_stride(int np) { return (np + 1 + 3) & ~3; }
__host__ __device__ inline int tile_pos(int row, int col) {
  return (((row >> 4) * (kHid / 16) + (col >> 4)) * 64 + ((row & 15) >> 2) * 16 + (col & 15)) * 4 + (row & 3);
}
__host__ __device__ inline int part_index(const MlpLayout &L, int p) {
  if (p < L.ob1) return L.oW1 + tile_pos(p / kHid, p % kHid);
  if (p >= L.oW2 && p < L.ob2) return L.oW2 + tile_pos((p - L.oW2) / kHid, (p - L.oW2) % kHid);
  return p;
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
  float *partial;       // [n_waves][part_stride(nparams)] (part_index order)
};

// One block of kTrainTileWaves wavefronts per 16 rows of the batch;
// wavefront w owns hidden units 16w .. 16w+15 of both layers, so each
// layer is one 16x16 matrix-core tile per wavefront, with the activation
// tiles exchanged in LDS.  The partial gradients of the 16 rows are the
// same numbers the whole-network-per-wavefront form gave: every tile and
// every reduction has the same operands in the same order (the output y is
// summed over the 8 tiles in tile order by every wavefront).
constexpr int kTrainTileWaves = kHid / 16;

__global__ __launch_bounds__(64 * kTrainTileWaves) void k_mlp_train_partial(TrainArgs ta) {
  extern __shared__ __align__(16) unsigned char mlp_lds[];
  const MlpHeader *hdr = (const MlpHeader *)ta.blob;
  const int S = hdr->S, k1 = hdr->k1, np = hdr->nparams;
  const MlpLayout L = mlp_layout(S);
  const int ld1 = mlp_ld1(k1);
  unsigned short *atile = (unsigned short *)mlp_lds;          // one-hot inputs [16][ld1]
  unsigned short *h1s = atile + 16 * ld1;                       // h1 [16][kLdH]
  unsigned short *h2s = h1s + 16 * kLdH;                        // h2 [16][kLdH]
  unsigned short *dzs = h2s + 16 * kLdH;                        // dz2 [16][kLdH]
  uint8_t *senv = (uint8_t *)(dzs + 16 * kLdH);                 // codes [16][32]
  const unsigned short *gw1t = (const unsigned short *)(ta.blob + L.w1t);  // [128][k1]
  const unsigned short *gw2t = (const unsigned short *)(ta.blob + L.w2t);  // [o][i]
  const unsigned short *gw2r = (const unsigned short *)(ta.blob + L.w2r);  // [i][o]
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
  const int col = 16 * w + r;  // this lane's hidden unit
  const float *prm = (const float *)(ta.blob + L.params);
  const float mu = hdr->mu, sigma = hdr->sigma;
  const int row0 = blockIdx.x * 16;
  // This lane's weight operands of all three products, read before the
  // batch rows so that their latency overlaps the setup.
  constexpr int kMaxT1 = mlp_k1(8) / 32;
  const int nk = k1 / 32;
  bf16x8 bw1[kMaxT1], bw2[4], bw2r[4];
  // Every chunk is loaded without a branch, so all are in flight together;
  // chunks past k1 read the last one again and are never used.
#pragma unroll
  for (int t = 0; t < kMaxT1; ++t)
    bw1[t] = *(const bf16x8 *)(gw1t + col * k1 + 32 * (t < nk ? t : nk - 1) + 8 * q);
  // The binary32 parameters this lane uses, read here rather than after the
  // barriers below (a read there would wait a full memory round trip).
  const float b1c = prm[L.ob1 + col], b2c = prm[L.ob2 + col], b3 = prm[L.ob3];
  const float w3c = bf2f(f2bf(prm[L.ow3 + col]));
  float w3r[kTrainTileWaves];
#pragma unroll
  for (int c = 0; c < kTrainTileWaves; ++c) w3r[c] = bf2f(f2bf(prm[L.ow3 + 16 * c + r]));
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    bw2[t] = *(const bf16x8 *)(gw2t + col * kHid + 32 * t + 8 * q);
    bw2r[t] = *(const bf16x8 *)(gw2r + col * kHid + 32 * t + 8 * q);
  }
  __shared__ float s_t[16];
  __shared__ int s_valid[16];
  // Batch rows, spread over the block: thread u < 16 * kSlots fetches code
  // `slot` of row `row` (rows past this step's count read as code 0 and
  // train nothing); the slot-0 thread also takes the row's target.  The
  // one-hot tile is cleared meanwhile, and filled after the barrier.
  const int tid = threadIdx.x;
  const int urow = tid / kSlots, uslot = tid - urow * kSlots;
  int ucode = S;
  if (tid < 16 * kSlots) {
    const int b = row0 + urow;
    int64_t drow = -1;
    if (b < ta.rows) {
      const int64_t pos = ta.start + b;
      drow = ta.perm_key ? permute_row(pos, ta.n, ta.perm_key, ta.perm_bits) : pos;
    }
    // the row's target is read beside its codes, not after them
    const float eav = uslot == 0 && drow >= 0 ? ta.ea[drow] : 0.f;
    ucode = drow >= 0 ? ta.env[drow * kSlots + uslot] : 0;
    senv[urow * 32 + uslot] = (uint8_t)ucode;
    if (uslot == 0) {
      const bool valid = drow >= 0 && ucode != S - 1;
      s_t[urow] = valid ? (eav - mu) / sigma : 0.f;
      s_valid[urow] = valid ? 1 : 0;
    }
  }
  for (int u = tid; u < 16 * ld1 / 8; u += 64 * kTrainTileWaves) *(uint4 *)(atile + 8 * u) = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  if (tid < 16 * kSlots && ucode < S) atile[urow * ld1 + uslot * S + ucode] = 0x3F80;  // bf16 1.0
  __syncthreads();

  // Layer 1, this wavefront's tile.
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < kMaxT1; ++t) {
    if (t >= nk) break;
    const bf16x8 a = *(const bf16x8 *)(atile + r * ld1 + 32 * t + 8 * q);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw1[t], acc, 0, 0, 0);
  }
  float gp1[4], gp2[4];
  {
    const float bias = b1c;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float z = acc[i] + bias;
      h1s[(4 * q + i) * kLdH + col] = f2bf(gelu_f(z));
      gp1[i] = gelu_grad_f(z);
    }
  }
  __syncthreads();

  // Layer 2, this wavefront's tile (A = all of h1).
  acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bf16x8 a = *(const bf16x8 *)(h1s + r * kLdH + 32 * t + 8 * q);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw2[t], acc, 0, 0, 0);
  }
  unsigned short h2b[4];
  {
    const float bias = b2c;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float z = acc[i] + bias;
      h2b[i] = f2bf(gelu_f(z));
      gp2[i] = gelu_grad_f(z);
      h2s[(4 * q + i) * kLdH + col] = h2b[i];
    }
  }
  __syncthreads();

  // Output of the 16 rows (every wavefront): lane (q, r) adds h2 w3 over
  // the 8 tiles in order, then the 16 lanes of each row group.
  float y[4];
  {
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < kTrainTileWaves; ++c) {
      const float w3 = w3r[c];
#pragma unroll
      for (int i = 0; i < 4; ++i) part[i] = fmaf(bf2f(h2s[(4 * q + i) * kLdH + 16 * c + r]), w3, part[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = part[i];
      v += __shfl_xor(v, 8, 16);
      v += __shfl_xor(v, 4, 16);
      v += __shfl_xor(v, 2, 16);
      v += __shfl_xor(v, 1, 16);
      y[i] = v + b3;
    }
  }

  float *part = ta.partial + (size_t)blockIdx.x * (size_t)part_stride(np);
  const float inv_b = 2.0f / (float)max(ta.rows, 1);   // d(mean loss)/dy over this step's rows
  float dy[4];
  float lsum = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = 4 * q + i;
    const float d = s_valid[row] ? (y[i] - s_t[row]) : 0.f;
    dy[i] = d * inv_b;
    lsum += d * d;
  }
  if (w == 0) {
    float db3 = dy[0] + dy[1] + dy[2] + dy[3];
    db3 += __shfl_xor(db3, 16, 64);
    db3 += __shfl_xor(db3, 32, 64);
    lsum += __shfl_xor(lsum, 16, 64);
    lsum += __shfl_xor(lsum, 32, 64);
    if (l == 0) {
      part[L.ob3] = db3;
      part[np] = lsum;
    }
  }
  // Output-layer gradients of this tile.
  s16x4 dz2b;
  {
    const float w3 = w3c;
    float dw3 = 0.f, db2 = 0.f;
    float dz2[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dw3 = fmaf(bf2f(h2b[i]), dy[i], dw3);
      dz2[i] = dy[i] * w3 * gp2[i];
      db2 += dz2[i];
    }
    dw3 += __shfl_xor(dw3, 16, 64);
    dw3 += __shfl_xor(dw3, 32, 64);
    db2 += __shfl_xor(db2, 16, 64);
    db2 += __shfl_xor(db2, 32, 64);
    if (q == 0) {
      part[L.ow3 + col] = dw3;
      part[L.ob2 + col] = db2;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned short hb = f2bf(dz2[i]);
      dz2b[i] = (short)hb;
      dzs[(4 * q + i) * kLdH + col] = hb;
    }
  }
  // dW2[i][o] for this tile's outputs o: the 16 rows are the reduction
  // dimension (A: h1 of input tile ti, B: dz2 of this tile).
#pragma unroll
  for (int ti = 0; ti < kTrainTileWaves; ++ti) {
    s16x4 a;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = (short)h1s[(4 * q + i) * kLdH + 16 * ti + r];
    f32x4 cacc = {0.f, 0.f, 0.f, 0.f};
    cacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, dz2b, cacc, 0, 0, 0);
    *(f32x4 *)(part + L.oW2 + ((ti * 8 + w) * 64 + l) * 4) = cacc;
  }
  __syncthreads();

  // dh1 of this tile's inputs = dz2 (all outputs) W2^T.
  acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bf16x8 a = *(const bf16x8 *)(dzs + r * kLdH + 32 * t + 8 * q);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw2r[t], acc, 0, 0, 0);
  }
  s16x4 dz1b;
  {
    float db1 = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float dz = acc[i] * gp1[i];
      db1 += dz;
      dz1b[i] = (short)f2bf(dz);
    }
    db1 += __shfl_xor(db1, 16, 64);
    db1 += __shfl_xor(db1, 32, 64);
    if (q == 0) part[L.ob1 + col] = db1;
  }
  // dW1[f][n] for this tile's units n: x from the species codes.
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
    f32x4 cacc = {0.f, 0.f, 0.f, 0.f};
    cacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, dz1b, cacc, 0, 0, 0);
    *(f32x4 *)(part + L.oW1 + ((tf * 8 + w) * 64 + l) * 4) = cacc;
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
  const size_t stride = (size_t)part_stride(np);
  // Sum over the blocks in block order, 16 reads in flight at a time.
  auto sum_parts = [&](int idx) {
    float acc = 0.f;
    int w = 0;
    for (; w + 16 <= n_waves; w += 16) {
      float v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = partial[(size_t)(w + k) * stride + idx];
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += v[k];
    }
    for (; w < n_waves; ++w) acc += partial[(size_t)w * stride + idx];
    return acc;
  };
  if (p == 0 && loss_out) *loss_out = sum_parts(np) * inv_rows;
  if (p >= np) return;
  const float g = sum_parts(part_index(L, p));
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
  return (size_t)2 * 16 * mlp_ld1(mlp_k1(S)) + (size_t)3 * 2 * 16 * kLdH + 16 * 32;
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
  const unsigned blocks = (unsigned)(batch / 16);
  hipLaunchKernelGGL(k_mlp_train_partial, dim3(blocks), dim3(64 * kTrainTileWaves), lds, stream, ta);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int np = mlp_nparams(S);
  hipLaunchKernelGGL(k_mlp_update, dim3((np + 255) / 256), dim3(256), 0, stream, blob, partial,
                     (int)blocks, apply, lr, beta1, beta2, eps, wd, step, grad_out,
                     loss_out, 1.0f / (float)std::max(rows, 1));
  return hipGetLastError();
}

size_t mlp_partial_bytes(int S, int batch) {
  return sizeof(float) * (size_t)(batch / 16) * (size_t)part_stride(mlp_nparams(S));
}

}  // namespace akmc
