// Device helpers of the vacancy-jump path: lattice positions, the Philox
// stream, the event digest and the per-candidate energy change.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "akmc_internal.hpp"

namespace akmc {

// ------------------------------------------------------------ positions
// A site is addressed by its position in units of a/2: X = 2x + b etc., in
// a periodic box of 2*lx x 2*ly x 2*lz.  The corner (b = 0) has even
// coordinates, the body centre (b = 1) odd ones.  First neighbours are the
// 8 offsets (+-1, +-1, +-1), second neighbours the 6 offsets +-2 along one
// axis, in the order (+x, -x, +y, -y, +z, -z).

struct Geo {
  int lx, ly, lz;
  int X2, Y2, Z2;   // box edges in a/2 units
  int ncell;
};

__device__ __forceinline__ Geo make_geo(int lx, int ly, int lz) {
  Geo g;
  g.lx = lx; g.ly = ly; g.lz = lz;
  g.X2 = 2 * lx; g.Y2 = 2 * ly; g.Z2 = 2 * lz;
  g.ncell = lx * ly * lz;
  return g;
}

__device__ __forceinline__ int wrapc(int v, int L2) {
  v = v < 0 ? v + L2 : v;
  return v >= L2 ? v - L2 : v;
}

__device__ __forceinline__ int site_of(const Geo &g, int X, int Y, int Z) {
  return (X & 1) * g.ncell + ((Z >> 1) * g.ly + (Y >> 1)) * g.lx + (X >> 1);
}

__device__ __forceinline__ void pos_of(const Geo &g, int site, int &X, int &Y, int &Z) {
  int b = site >= g.ncell ? 1 : 0;
  int r = site - b * g.ncell;
  int x = r % g.lx;
  r /= g.lx;
  int y = r % g.ly;
  int z = r / g.ly;
  X = 2 * x + b;
  Y = 2 * y + b;
  Z = 2 * z + b;
}

// Packed position (11 bits per axis; edges are limited to 1000 cells).
__device__ __forceinline__ int pack_pos(int X, int Y, int Z) { return X | (Y << 11) | (Z << 22); }
__device__ __forceinline__ int pos_x(int p) { return p & 2047; }
__device__ __forceinline__ int pos_y(int p) { return (p >> 11) & 2047; }
__device__ __forceinline__ int pos_z(int p) { return (p >> 22) & 2047; }

__device__ __forceinline__ int dir_sx(int k) { return ((k >> 2) & 1) ? 1 : -1; }
__device__ __forceinline__ int dir_sy(int k) { return ((k >> 1) & 1) ? 1 : -1; }
__device__ __forceinline__ int dir_sz(int k) { return (k & 1) ? 1 : -1; }

// -------------------------------------------------------------- Philox
// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11):
// multipliers 0xD2E7470EE14C6C93, 0xCA5A826395121157, key increments the
// golden-ratio and sqrt(3)-1 Weyl constants.
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Event n's uniforms: u1 in [0,1) from word 0, u2 in (0,1] from word 1.
__device__ __forceinline__ void event_uniforms(uint64_t seed, uint64_t stream, int64_t n,
                                               double &u1, double &u2) {
  uint64_t x[4];
  philox4x64_10((uint64_t)n, 0, 0, 0, seed, stream, x);
  const double two_m53 = 1.1102230246251565404e-16;  // 2^-53
  u1 = (double)(x[0] >> 11) * two_m53;
  u2 = (double)((x[1] >> 11) + 1) * two_m53;
}

// -------------------------------------------------------------- digest
// One event of the trajectory digest: the FNV-1a step (xor, then multiply by
// the 64-bit FNV prime modulo 2^64) on the word from | to << 32.
__device__ __forceinline__ uint64_t digest_event(uint64_t h, int32_t from, int32_t to) {
  const uint64_t w = (uint64_t)(uint32_t)from | ((uint64_t)(uint32_t)to << 32);
  return (h ^ w) * 0x100000001b3ull;
}

// ------------------------------------------------- candidate energetics
// Species counts are kept as 8 nibbles of a 32-bit word (one per species
// code); a shell has at most 8 members, so no nibble overflows.
__device__ __forceinline__ uint32_t onehot(int s) { return 1u << (4 * s); }
__device__ __forceinline__ int nib(uint32_t c, int s) { return (int)((c >> (4 * s)) & 15u); }
// Nibble s of c read as a 4-bit two's complement number.
__device__ __forceinline__ int nib_signed(uint32_t c, int s) {
  return (int)(c << (28 - 4 * s)) >> 28;
}

// Energy change from the bond counts, as one fused multiply-add chain over
// species codes, shell 1 first:  dE = sum_s dn1[s] D1[A][s] + dn2[s] D2[A][s]
// with dn1 = c1i - c1j (first shells of i without j and of j without i)
// and dn2 = c2i - c2j (second shells).  The counts are exact integers, so
// any way of gathering them gives the same bits.
//
// Rows hold 8 entries, zero past the species count: the extra terms are
// fma(0, 0, acc) = acc exactly (acc starts at +0 and is never -0), so the
// chain equals the one over s < S.  Every count nibble is at most 7 (7 or 6
// sites per group), so 8 + ci - cj stays within a nibble and one subtraction
// serves all species; xor with 8 turns each nibble into the 4-bit two's
// complement of dn.
template <class Real>
__device__ __forceinline__ Real delta_e_counts(uint32_t c1i, uint32_t c1j, uint32_t c2i,
                                               uint32_t c2j, const Real *D1row,
                                               const Real *D2row) {
  Real d1[8], d2[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    d1[s] = D1row[s];
    d2[s] = D2row[s];
  }
  const uint32_t e1 = ((c1i + 0x88888888u) - c1j) ^ 0x88888888u;
  const uint32_t e2 = ((c2i + 0x88888888u) - c2j) ^ 0x88888888u;
  Real acc = Real(0);
#pragma unroll
  for (int s = 0; s < 8; ++s) acc = fma((Real)nib_signed(e1, s), d1[s], acc);
#pragma unroll
  for (int s = 0; s < 8; ++s) acc = fma((Real)nib_signed(e2, s), d2[s], acc);
  return acc;
}

// Pair model out to 6.0 A: the energy change from per-shell species counts
// of the changed bonds, ci[m] (of i without j) and cj[m] (of j without i)
// holding one 8-bit count per species (shells hold at most 24 sites), as
// one fused multiply-add chain over shells 1..6, then species: shell 1 and
// 2 tables D1, D2, shells 3..6 in Dx (rows of 8 at 8*A, stride 64).
template <class Real>
__device__ __forceinline__ Real delta_e_counts6(const uint64_t (&ci)[6], const uint64_t (&cj)[6], int S,
                                                const Real *D1row, const Real *D2row, const Real *Dx,
                                                int A) {
  Real acc = Real(0);
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const Real *row = m == 0 ? D1row : m == 1 ? D2row : Dx + 64 * (m - 2) + 8 * A;
#pragma unroll
    for (int sp = 0; sp < 8; ++sp) {
      if (sp >= S) break;
      const int dn = (int)((ci[m] >> (8 * sp)) & 255u) - (int)((cj[m] >> (8 * sp)) & 255u);
      acc = fma(Real(dn), row[sp], acc);
    }
  }
  return acc;
}

__device__ __forceinline__ double rate_from_barrier(double ea, double nu, double kT) {
  double x = -(ea / kT);
  return nu * exp(x);
}
// binary32: nu * 2^(Ea * (-log2(e) / kT)) on the hardware base-2
// exponential (about 1 ulp); where the function is inlined into a loop the
// scale is computed once.
__device__ __forceinline__ float rate_from_barrier(float ea, float nu, float kT) {
  return nu * __builtin_amdgcn_exp2f(ea * (-1.44269504088896341f / kT));
}

}  // namespace akmc
