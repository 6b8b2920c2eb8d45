// Persistent residence-time event loop.
//
// One group of G lanes (G = 8, 16, 32 or 64, always inside one wavefront)
// owns one lattice for a whole launch and runs its events back to back
// with no host round trip.  Groups pull lattices from a device work queue
// in a given order (heaviest first for replica ensembles), so a launch can
// serve one lattice or a voxel ensemble of uneven replicas.
//
// Per event (all of it group-local, synchronised at wavefront level):
//   1. uniforms of event n from Philox4x64-10 (computed G events ahead,
//      one per lane, together with -ln u2);
//   2. selection: target = u1 * Gamma_tot, descended through a tree of
//      binary64 partial sums held in LDS (fan-out 8 at every level: 8
//      directions per slot, then groups of 8 slots, ...).  Every node is
//      a fixed function of its children (a scan within its group of 8), so
//      the sums do not depend on G, on which slots were refreshed, or on
//      the launch split;
//   3. dt = -ln(u2)/Gamma_tot, t += dt, digest update;
//   4. swap of atom and vacancy in the global occupancy;
//   5. local refresh: every slot whose vacancy lies within 4 half-lattice
//      units (Chebyshev, minimum image) of the old vacancy site is
//      re-evaluated; that covers every slot whose 58-site bond footprint
//      contains one of the two changed sites.  Each refreshed vacancy's
//      footprint is gathered once into a 7x7x7 LDS box and its 8
//      candidates read their bond counts from there;
//   6. the changed tree paths are re-summed.
#include <hip/hip_runtime.h>

#include "akmc_device.hpp"
#include "akmc_internal.hpp"
#include "akmc_mlp.hpp"
#include "akmc_patch.hpp"

namespace akmc {

// The 58 sites (offsets in a/2 units) that the bonds of any of the 8 jumps
// of a vacancy touch: the 8 first and 6 second neighbours, the 20 offsets
// with all components in {0, +-2} and two or three of them non-zero (first
// shells of the targets), and the 24 offsets with one component +-3 and the
// others +-1 (second shells of the targets).
struct FootTab {
  int8_t d[64][3];
  int n;
};

constexpr int iabs_c(int v) { return v < 0 ? -v : v; }

constexpr FootTab make_foot() {
  FootTab t{};
  int n = 0;
  for (int dz = -3; dz <= 3; ++dz)
    for (int dy = -3; dy <= 3; ++dy)
      for (int dx = -3; dx <= 3; ++dx) {
        const int ax = iabs_c(dx), ay = iabs_c(dy), az = iabs_c(dz);
        const bool odd = (ax & 1) && (ay & 1) && (az & 1);
        const int threes = (ax == 3) + (ay == 3) + (az == 3);
        const bool even = !(ax & 1) && !(ay & 1) && !(az & 1) && ax <= 2 && ay <= 2 && az <= 2 &&
                          (ax + ay + az) > 0;
        if ((odd && threes <= 1) || even) {
          t.d[n][0] = (int8_t)dx;
          t.d[n][1] = (int8_t)dy;
          t.d[n][2] = (int8_t)dz;
          ++n;
        }
      }
  t.n = n;
  return t;
}

constexpr FootTab kFootHost = make_foot();
static_assert(kFootHost.n == 58, "footprint of a vacancy has 58 sites");
__constant__ FootTab kFoot = make_foot();

constexpr int kFootN = 59;       // 58 gathered sites + the vacancy itself
constexpr int kBoxC = 3 + 7 * 3 + 49 * 3;
// With the learned runtime forms a vacancy's 64-neighbour observation also
// needs the 6 sites 4 half-cells away along an axis, outside the 7x7x7 box:
// they are gathered with the footprint and kept in box bytes kFarOff.. of
// their box, in the order (-x, -y, -z, +z, +y, +x) of the observation.
constexpr int kFootNL = kFootN + 6;
constexpr int kFarOff = 344;
static_assert(kFarOff >= 343 && kFarOff + 6 <= kBoxBytes, "far sites fit the box padding");
constexpr int kFarD[6][3] = {{-4, 0, 0}, {0, -4, 0}, {0, 0, -4}, {0, 0, 4}, {0, 4, 0}, {4, 0, 0}};

// Packed gather element: box byte (bits 0-10; the index 0..5 of a far site),
// offsets + 5 (bits 11-14, 15-18, 19-22), box number q (bits 23-28), centre
// flag (bit 29), far flag (bit 30); -1 for none.
__host__ __device__ constexpr int fe_pack(int bi, int dx, int dy, int dz, int q, bool centre, bool far) {
  return bi | ((dx + 5) << 11) | ((dy + 5) << 15) | ((dz + 5) << 19) | (q << 23) | ((int)centre << 29) |
         ((int)far << 30);
}
__device__ __forceinline__ int fe_dx(int f) { return ((f >> 11) & 15) - 5; }
__device__ __forceinline__ int fe_dy(int f) { return ((f >> 15) & 15) - 5; }
__device__ __forceinline__ int fe_dz(int f) { return ((f >> 19) & 15) - 5; }
__device__ __forceinline__ int fe_q(int f) { return (f >> 23) & 63; }
__device__ __forceinline__ bool fe_centre(int f) { return (f >> 29) & 1; }
__device__ __forceinline__ int fe_byte(int f) { return ((f >> 30) & 1) ? kFarOff + (f & 2047) : (f & 2047); }

// Pair model out to 6.0 A: an 11x11x11 box (offsets -5..5) holds the bonds
// of all 8 jumps of a vacancy: the 168 sites within 6.0 A of the vacancy or
// of one of its 8 targets.
constexpr int kBoxCF = 5 + 11 * 5 + 121 * 5;
constexpr int kFootFarN = 168;
struct FootFarTab {
  int8_t d[kFootFarN][3];
  int n;
};
constexpr bool within_6a(int dx, int dy, int dz) {
  const int odd = dx & 1;
  if ((dy & 1) != odd || (dz & 1) != odd) return false;
  const int r2 = dx * dx + dy * dy + dz * dz;
  return r2 > 0 && r2 <= 16;
}
constexpr FootFarTab make_foot_far() {
  FootFarTab t{};
  int n = 0;
  for (int dz = -5; dz <= 5; ++dz)
    for (int dy = -5; dy <= 5; ++dy)
      for (int dx = -5; dx <= 5; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        bool in = within_6a(dx, dy, dz);
        for (int k = 0; k < 8 && !in; ++k) {
          const int tx = (k >> 2) & 1 ? 1 : -1, ty = (k >> 1) & 1 ? 1 : -1, tz = k & 1 ? 1 : -1;
          in = (dx == tx && dy == ty && dz == tz) || within_6a(dx - tx, dy - ty, dz - tz);
        }
        if (!in) continue;
        if (n < kFootFarN) {
          t.d[n][0] = (int8_t)dx;
          t.d[n][1] = (int8_t)dy;
          t.d[n][2] = (int8_t)dz;
        }
        ++n;
      }
  t.n = n;
  return t;
}
constexpr FootFarTab kFootFarHost = make_foot_far();
static_assert(kFootFarHost.n == kFootFarN, "the bonds of a vacancy's 8 jumps touch 168 sites");
__constant__ FootFarTab kFootFar = make_foot_far();

// The 64 bond offsets with their shells (the observation order), as box
// offsets of the 11x11x11 box.
struct BondFar {
  int16_t off[kObsN];
  int8_t sh[kObsN];
};
constexpr BondFar make_bond_far() {
  BondFar r{};
  const ObsTab t = make_obs();
  for (int m = 0; m < kObsN; ++m) {
    const int dx = t.d[m][0], dy = t.d[m][1], dz = t.d[m][2];
    const int r2 = dx * dx + dy * dy + dz * dz;
    r.off[m] = (int16_t)(dx + 11 * dy + 121 * dz);
    r.sh[m] = (int8_t)(r2 == 3 ? 0 : r2 == 4 ? 1 : r2 == 8 ? 2 : r2 == 11 ? 3 : r2 == 12 ? 4 : 5);
  }
  return r;
}
// Used in fully unrolled loops only, so every entry folds into an immediate.
constexpr BondFar kBondFar = make_bond_far();
__constant__ BondFar kBondFarDev = make_bond_far();  // for per-lane (runtime) indices

// The 64 bonds of a jump's site in 8 groups of one shell each (the 24 of
// shell 3 in three groups), for the 8 lanes that count one candidate
// together: group p holds bond indices m[p][0..) (-1 past the end).
constexpr int kFarGroupShell[8] = {0, 1, 2, 3, 3, 3, 4, 5};
constexpr int kFarGroupMax = 12;
struct FarGroups {
  int8_t m[8][kFarGroupMax];
};
constexpr FarGroups make_far_groups() {
  FarGroups g{};
  int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int p = 0; p < 8; ++p)
    for (int u = 0; u < kFarGroupMax; ++u) g.m[p][u] = -1;
  for (int m = 0; m < kObsN; ++m)
    for (int p = 0; p < 8; ++p)
      if (kFarGroupShell[p] == kBondFar.sh[m] && cnt[p] < (p == 2 ? 12 : 8)) {
        g.m[p][cnt[p]++] = (int8_t)m;
        break;
      }
  return g;
}
constexpr bool far_groups_cover() {
  const FarGroups g = make_far_groups();
  int n = 0;
  for (int p = 0; p < 8; ++p)
    for (int u = 0; u < kFarGroupMax; ++u) n += g.m[p][u] >= 0;
  return n == kObsN;
}
static_assert(far_groups_cover(), "every bond in one group");
__constant__ FarGroups kFarGroups = make_far_groups();
constexpr int kFarNone = 0x7fff;  // no bond at this place of a group

// Box byte of each observation neighbour: inside the 7x7x7 box, or the far
// slot of an axis site 4 half-cells away.
struct ObsSrc {
  int16_t b[kObsN];
};
constexpr ObsSrc make_obs_src() {
  ObsSrc r{};
  const ObsTab t = make_obs();
  for (int m = 0; m < kObsN; ++m) {
    const int dx = t.d[m][0], dy = t.d[m][1], dz = t.d[m][2];
    int src = -1;
    for (int f = 0; f < 6; ++f)
      if (kFarD[f][0] == dx && kFarD[f][1] == dy && kFarD[f][2] == dz) src = kFarOff + f;
    if (src < 0) src = (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);
    r.b[m] = (int16_t)src;
  }
  return r;
}
constexpr ObsSrc kObsSrcHost = make_obs_src();
__constant__ ObsSrc kObsSrc = make_obs_src();

template <int G>
struct Group {
  int gw, gl, base;
  __device__ __forceinline__ uint64_t ballot(bool p) const {
    const uint64_t m = __builtin_amdgcn_ballot_w64(p);
    if (G == 64) return m;
    return (m >> base) & ((1ull << (G & 63)) - 1ull);
  }
  __device__ __forceinline__ uint64_t lanes_below() const {
    return gl == 0 ? 0ull : ((1ull << gl) - 1ull);
  }
  template <class T>
  __device__ __forceinline__ T bcast(T v, int src) const {
    return __shfl(v, base + src, 64);
  }
};

// Orders LDS traffic of the wavefront (a group never spans wavefronts).
__device__ __forceinline__ void gsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class Real>
struct Lds {
  double *part;     // [nv][8] partial sums over directions, part[v][7] = slot total
  double *q;        // tree levels
  int *pos;         // packed vacancy positions
  int *aff;         // refreshed slots, ascending
  int *la, *lb;     // group lists of the tree update
  uint8_t *spec;    // [nv][8] species of each candidate's target
  uint8_t *box;     // (G/8) footprint boxes
  Real *D1, *D2, *e0;
  Real *Dx;         // shells 3..6 of the pair model out to 6.0 A (4 rows of 64)
  double *ru1, *rw; // uniforms u1 and -ln u2 of the next G events
  double *tmp;      // G values exchanged between the lanes of a group
  uint32_t *grid;   // coarse vacancy counts (vac_grid), grid_words words
  int grid_words;
};

template <class Real>
__device__ __forceinline__ Lds<Real> carve(unsigned char *base, const GroupLayout &L) {
  Lds<Real> s;
  s.part = (double *)(base + L.off_part);
  s.q = (double *)(base + L.off_q);
  s.pos = (int *)(base + L.off_pos);
  s.aff = (int *)(base + L.off_aff);
  s.la = (int *)(base + L.off_la);
  s.lb = (int *)(base + L.off_lb);
  s.spec = base + L.off_spec;
  s.box = base + L.off_box;
  s.D1 = (Real *)(base + L.off_tab);
  s.D2 = s.D1 + 64;
  s.e0 = s.D2 + 64;
  s.Dx = s.e0 + 8;
  s.ru1 = (double *)(base + L.off_rng);
  s.rw = s.ru1 + L.G;
  s.tmp = (double *)(base + L.off_tmp);
  s.grid = (uint32_t *)(base + L.off_grid);
  s.grid_words = L.grid_words;
  return s;
}

// Rate of candidate k of the vacancy whose footprint sits in `box`.  Boxes
// hold 4*species (the shift of that species' count nibble).  Bond counts as
// in the site-list kernel: N1(i) without j, N1(j) without i, N2(i), N2(j).
// Returns the rate widened to binary64 and the target species.
template <class Real>
__device__ __forceinline__ double eval_box(const uint8_t *box, int k, int V, const Real *D1,
                                           const Real *D2, const Real *e0, Real nu, Real kT,
                                           int &A_out, Real &ea_out) {
  const int jb = kBoxC + dir_sx(k) + 7 * dir_sy(k) + 49 * dir_sz(k);
  const int a4 = box[jb];
  const int A = a4 >> 2;
  A_out = A;
  ea_out = Real(__builtin_huge_valf());
  if (A == V) return 0.0;
  uint32_t c1i = 0, c1j = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int off = dir_sx(q) + 7 * dir_sy(q) + 49 * dir_sz(q);
    c1i += 1u << box[kBoxC + off];
    c1j += 1u << box[jb + off];
  }
  const uint32_t c2i = (1u << box[kBoxC + 2]) + (1u << box[kBoxC - 2]) + (1u << box[kBoxC + 14]) +
                       (1u << box[kBoxC - 14]) + (1u << box[kBoxC + 98]) + (1u << box[kBoxC - 98]);
  const uint32_t c2j = (1u << box[jb + 2]) + (1u << box[jb - 2]) + (1u << box[jb + 14]) +
                       (1u << box[jb - 14]) + (1u << box[jb + 98]) + (1u << box[jb - 98]);
  c1i -= 1u << a4;
  c1j -= 1u << box[kBoxC];
  const Real de = delta_e_counts<Real>(c1i, c1j, c2i, c2j, D1 + 8 * A, D2 + 8 * A);
  const Real ea = e0[A] + Real(0.5) * de;
  ea_out = ea;
  return (double)rate_from_barrier(ea, nu, kT);
}

// Rate of candidate k with the pair model out to 6.0 A (box of 11^3, 4 *
// species per byte): per-shell species counts of the 63 bonds of i without
// j and of j without i, then the six-shell fma chain.
template <class Real>
__device__ __forceinline__ double eval_box6(const uint8_t *box, int k, int V, int S, const Real *D1,
                                            const Real *D2, const Real *Dx, const Real *e0, Real nu,
                                            Real kT, int &A_out, Real &ea_out) {
  const int dk = dir_sx(k) + 11 * dir_sy(k) + 121 * dir_sz(k);
  const int jb = kBoxCF + dk;
  const int a4 = box[jb];
  const int A = a4 >> 2;
  A_out = A;
  ea_out = Real(__builtin_huge_valf());
  if (A == V) return 0.0;
  uint64_t ci[6] = {0, 0, 0, 0, 0, 0}, cj[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < kObsN; ++m) {
    const int off = kBondFar.off[m];
    const int sh = kBondFar.sh[m];
    // bytes hold 4*species: << 1 gives 8*species
    const uint64_t bi = 1ull << (box[kBoxCF + off] << 1);
    const uint64_t bj = 1ull << (box[jb + off] << 1);
    if (off != dk) ci[sh] += bi;
    if (off != -dk) cj[sh] += bj;
  }
  const Real de = delta_e_counts6<Real>(ci, cj, S, D1 + 8 * A, D2 + 8 * A, Dx, A);
  const Real ea = e0[A] + Real(0.5) * de;
  ea_out = ea;
  return (double)rate_from_barrier(ea, nu, kT);
}

// The same rate on a full wavefront: lane 8k + p counts bond group p of
// candidate k (fo: this lane's group offsets, kFarNone past its end), the
// count words are collected in lane 8k by DPP row shifts (integer sums, so
// the counts are those eval_box6 forms) and lane 8k runs the six-shell chain.
// Returns the rate, species and barrier of candidate gl in lanes gl < 8.
// Every lane of the wavefront must call it.
template <int SHR>
__device__ __forceinline__ uint64_t row_shl64(uint64_t x) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, 0x100 + SHR, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), 0x100 + SHR, 0xF, 0xF, false);
  return (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32);
}
template <class Real>
__device__ __forceinline__ double eval_box6_wave(const uint8_t *box, int gl, const int (&fo)[kFarGroupMax],
                                                 int V, int S, const Real *D1, const Real *D2, const Real *Dx,
                                                 const Real *e0, Real nu, Real kT, int &A_out, Real &ea_out) {
  const int k = gl >> 3;
  const int dk = dir_sx(k) + 11 * dir_sy(k) + 121 * dir_sz(k);
  const int jb = kBoxCF + dk;
  uint64_t ci = 0, cj = 0;
#pragma unroll
  for (int u = 0; u < kFarGroupMax; ++u) {
    const int off = fo[u];
    if (off == kFarNone) continue;
    const uint64_t bi = 1ull << (box[kBoxCF + off] << 1);
    const uint64_t bj = 1ull << (box[jb + off] << 1);
    if (off != dk) ci += bi;
    if (off != -dk) cj += bj;
  }
  // lane 8k collects groups 1..7 (group 0 is its own)
  uint64_t wi[6], wj[6];
  wi[0] = ci;
  wj[0] = cj;
  wi[1] = row_shl64<1>(ci);
  wj[1] = row_shl64<1>(cj);
  wi[2] = row_shl64<2>(ci);
  wj[2] = row_shl64<2>(cj);
  wi[3] = row_shl64<3>(ci) + row_shl64<4>(ci) + row_shl64<5>(ci);
  wj[3] = row_shl64<3>(cj) + row_shl64<4>(cj) + row_shl64<5>(cj);
  wi[4] = row_shl64<6>(ci);
  wj[4] = row_shl64<6>(cj);
  wi[5] = row_shl64<7>(ci);
  wj[5] = row_shl64<7>(cj);
  const int A = box[jb] >> 2;
  double r = 0.0;
  Real ea = Real(__builtin_huge_valf());
  if ((gl & 7) == 0 && A != V) {
    const Real de = delta_e_counts6<Real>(wi, wj, S, D1 + 8 * A, D2 + 8 * A, Dx, A);
    ea = e0[A] + Real(0.5) * de;
    r = (double)rate_from_barrier(ea, nu, kT);
  }
  // candidate k's results from lane 8k to lane k
  const int src = 8 * (gl & 7);
  r = __hiloint2double(__shfl(__double2hiint(r), src), __shfl(__double2loint(r), src));
  ea_out = __shfl(ea, src);
  A_out = __shfl(A, src);
  return r;
}

// LDS of the learned barrier (one group per block): bf16 weights, the
// 64-row code staging, the activation staging tile, outputs, biases and
// output weights, the one-hot input tile.
struct MlpLds {
  unsigned short *w1t, *w2t, *hst;
  uint8_t *senv;
  float *yb;
  float *pb;  // biases b1, b2, output weights w3 and bias b3 (128, 128, 128, 1)
  unsigned short *atile;  // one-hot input tile, 16 rows of pitch mlp_ld1(k1); then layer 2's output
  int *cmd;               // to the helper wavefronts: 1 = a tile, 0 = the end of the launch
};

__host__ __device__ inline size_t mlp_loop_lds_bytes(int S) {
  return (size_t)2 * kHid * mlp_ld1(mlp_k1(S)) + (size_t)2 * kHid * kLdH + 64 * 32 + 2 * 16 * kLdH + 64 * 4 +
         (3 * kHid + 1) * 4 + 16 + (size_t)2 * 16 * mlp_ld1(mlp_k1(S)) + 16;
}

// The surrogate's LDS area of the event loop, at b (after the lattice).
__device__ inline MlpLds mlp_lds_at(unsigned char *b, int k1) {
  MlpLds ml;
  ml.w1t = (unsigned short *)b;
  ml.w2t = ml.w1t + kHid * mlp_ld1(k1);
  ml.senv = (uint8_t *)(ml.w2t + kHid * kLdH);
  ml.hst = (unsigned short *)(ml.senv + 64 * 32);
  ml.yb = (float *)(ml.hst + 16 * kLdH);
  ml.pb = ml.yb + 64;
  ml.atile = (unsigned short *)(((uintptr_t)(ml.pb + 3 * kHid + 1) + 15) & ~(uintptr_t)15);
  ml.cmd = (int *)(ml.atile + 16 * mlp_ld1(k1));
  return ml;
}

// Wavefronts of the surrogate loop's workgroup: the event loop runs on the
// first; all of them share each 16-row tile of the forward.
constexpr int kMlpWaves = 4;

// One 16-row tile of the surrogate forward (the one-hot inputs in atile) by
// the kMlpWaves wavefronts of the workgroup: wavefront w takes the kCpw
// hidden-unit tiles c = kCpw*w .. of both layers (the same matrix-core products,
// bias and GELU as the one-wavefront forward, h1 shared in hst, h2 written
// over atile); then wavefront w forms the outputs of rows 4*(l/16) + i for
// its i exactly as the one-wavefront forward does (each lane over c = 0..7
// in order, then its 16-lane row group) and stores them at yout[row].
// Every wavefront of the workgroup calls it, between the same barriers.
__device__ inline void mlp_tile_waves(const MlpLds &ml, int k1, int w, float *yout) {
  constexpr int kCpw = kHid / 16 / kMlpWaves;  // hidden-unit tiles per wavefront
  static_assert(kCpw * kMlpWaves == kHid / 16, "whole hidden-unit tiles per wavefront");
  const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
  const int ld1 = mlp_ld1(k1), nk = k1 / 32;
  __builtin_assume(nk >= 1);  // k1 = 32 * ceil(27 S / 32) with S >= 2
  // The first product of each layer takes a zero accumulator operand;
  // activations are converted to bfloat16 two at a time.
  f32x4 acc[kCpw];
  for (int t = 0; t < nk; ++t) {
    const bf16x8 a = *(const bf16x8 *)(ml.atile + r * ld1 + 32 * t + 8 * q);
#pragma unroll
    for (int cc = 0; cc < kCpw; ++cc) {
      const bf16x8 b = *(const bf16x8 *)(ml.w1t + (16 * (kCpw * w + cc) + r) * ld1 + 32 * t + 8 * q);
      acc[cc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          a, b, t == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[cc], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cc = 0; cc < kCpw; ++cc) {
    const int c = kCpw * w + cc;
    const float bias = ml.pb[16 * c + r];
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
      const uint32_t hp = f2bf2(gelu_f(acc[cc][i] + bias), gelu_f(acc[cc][i + 1] + bias));
      ml.hst[(4 * q + i) * kLdH + 16 * c + r] = (unsigned short)hp;
      ml.hst[(4 * q + i + 1) * kLdH + 16 * c + r] = (unsigned short)(hp >> 16);
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bf16x8 a = *(const bf16x8 *)(ml.hst + r * kLdH + 32 * t + 8 * q);
#pragma unroll
    for (int cc = 0; cc < kCpw; ++cc) {
      const bf16x8 b = *(const bf16x8 *)(ml.w2t + (16 * (kCpw * w + cc) + r) * kLdH + 32 * t + 8 * q);
      acc[cc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          a, b, t == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[cc], 0, 0, 0);
    }
  }
  unsigned short *h2 = ml.atile;  // every wavefront has read its inputs (barrier above)
#pragma unroll
  for (int cc = 0; cc < kCpw; ++cc) {
    const int c = kCpw * w + cc;
    const float bias = ml.pb[kHid + 16 * c + r];
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
      const uint32_t hp = f2bf2(gelu_f(acc[cc][i] + bias), gelu_f(acc[cc][i + 1] + bias));
      h2[(4 * q + i) * kLdH + 16 * c + r] = (unsigned short)hp;
      h2[(4 * q + i + 1) * kLdH + 16 * c + r] = (unsigned short)(hp >> 16);
    }
  }
  __syncthreads();
  constexpr int kIpw = 4 / kMlpWaves;  // output rows per lane and wavefront
  static_assert(kIpw * kMlpWaves == 4, "the four rows of a lane over the wavefronts");
#pragma unroll
  for (int ii = 0; ii < kIpw; ++ii) {
    const int i = kIpw * w + ii;
    float part = 0.f;
#pragma unroll
    for (int c = 0; c < kHid / 16; ++c)
      part = fmaf(bf2f(h2[(4 * q + i) * kLdH + 16 * c + r]), bf2f(f2bf(ml.pb[2 * kHid + 16 * c + r])), part);
    part += __shfl_xor(part, 8, 16);
    part += __shfl_xor(part, 4, 16);
    part += __shfl_xor(part, 2, 16);
    part += __shfl_xor(part, 1, 16);
    if (r == 0) yout[4 * q + i] = part + ml.pb[3 * kHid];
  }
  __syncthreads();
}

// KL: the most tree levels of any lattice of the launch (at most
// kMaxLevels); the level loops are unrolled that far.
// LRN: the learned runtime forms (policy selection, Poisson time); FAR: the
// pair model out to 6.0 A; both with one 64-lane group per launch.
template <int G, class Real, bool MLP = false, int KL = kMaxLevels, bool LRN = false, bool FAR = false>
struct Runner {
  // gather elements per box (the sites and the vacancy itself), per lane
  // and pass (G/8 boxes), box bytes, reach of a jump's changes in half-cells
  static constexpr int FN = FAR ? kFootFarN + 1 : LRN ? kFootNL : kFootN;
  static constexpr int FM = (FN + 7) / 8;
  static constexpr int BB = FAR ? kBoxBytesFar : kBoxBytes;
  static constexpr int REACH = FAR ? 6 : LRN ? 5 : 4;  // footprint reach + 1: bounds i from j's side
  LoopArgs a;
  Group<G> gp;
  int foot[FM];
  Lds<Real> s;
  Geo g;
  int S, V, nv, nlev;
  Real nu, kT;
  uint8_t *occ;
  // learned barrier
  MlpLds ml;
  MlpLayout mlay, play;  // play: offsets of the parameters staged in LDS
  const float *prm;
  float mu, sigma;
  int k1;
  int64_t n_ood;
  // Out-of-distribution bounds packed per bond group as nibbles (b | 8) of
  // the largest count seen per species (15: no bound), and the mask of
  // moving species seen in training.
  uint32_t oodw[4], seen;
  double top_q;   // lane c < 8: partial c of the top tree level (cached between events)
  // 64-lane groups keep tree levels 2 and 3 in registers as well: lane j
  // holds node j's value (the total of its child group; t2, t3) and its
  // inclusive partial (q2, q3), zero beyond the level's length.  The LDS
  // copy stays current for the general refresh path.
  double t2, q2, t3, q3;
  Real *eat;      // barrier trace of this lattice (LoopArgs::ea_trace) or NULL
  // learned runtime forms
  bool has_pol, has_pt;
  float inv_tau;
  PatchNet pol, pt;
  double *pg;     // [nv] total pair rate of each slot (policy selection)
  double *gv;     // [nv] Poisson network value of each slot
  double *wq;     // [64] selection weights of one refresh pass, lane order
  uint8_t *obs;   // [8][64] observation codes of one refresh pass
  float *hbuf;    // [64] activation staging
  int *lcmd;      // to the second wavefront (both networks): slots of a pass, 0 at the end
  bool split;     // the Poisson network runs on the second wavefront
  int obs_src;    // box byte of this lane's observation neighbour
  int fo[FAR ? kFarGroupMax : 1];  // six shells: this lane's bond group (box offsets)

  __device__ Runner(const LoopArgs &a_, const GroupLayout &L, const Group<G> &gp_,
                    const int (&foot_)[FM], unsigned char *lds)
      : a(a_), gp(gp_) {
    s = carve<Real>(lds, L);
    n_ood = 0;
    has_pol = has_pt = false;
    if (LRN) {
      unsigned char *b = lds + L.bytes;
      pg = (double *)b;
      gv = pg + a.nv_max;
      wq = gv + a.nv_max;
      hbuf = (float *)(wq + 64);
      obs = (uint8_t *)(hbuf + 64);
      lcmd = (int *)(obs + 8 * kObsN + 64 * 4);  // after the second wavefront's hbuf
      b = (unsigned char *)(lcmd + 4);
      has_pol = a.pol_blob != nullptr;
      has_pt = a.pt_blob != nullptr;
      split = has_pol && has_pt && blockDim.x > 64;
      obs_src = kObsSrc.b[gp.gl];
      inv_tau = a.inv_tau;
      if (has_pol) {
        pol = patch_stage(a.pol_blob, b, gp.gl, G);
        b += patch_lds_bytes(pol.S, pol.H, pol.n_out);
      }
      if (has_pt) pt = patch_stage(a.pt_blob, b, gp.gl, G);
      gsync();
    }
    if (MLP) {
      const MlpHeader *hdr = (const MlpHeader *)a.mlp_blob;
      const int Sm = hdr->S;
      k1 = hdr->k1;
      mlay = mlp_layout(Sm);
      prm = (const float *)(a.mlp_blob + mlay.params);
      mu = hdr->mu;
      sigma = hdr->sigma;
      ml = mlp_lds_at(lds + L.bytes, k1);
      stage_rows(ml.w1t, (const unsigned short *)(a.mlp_blob + mlay.w1t), kHid, k1, mlp_ld1(k1), gp.gl, G);
      stage_rows(ml.w2t, (const unsigned short *)(a.mlp_blob + mlay.w2t), kHid, kHid, kLdH, gp.gl, G);
      seen = 0u;
      for (int grp = 0; grp < 4; ++grp) {
        uint32_t w = 0u;
        for (int sp = 0; sp < 8; ++sp) {
          const int b = (hdr->ood_valid && sp < Sm) ? min(hdr->ood_max[grp][sp], 15) : 15;
          w |= (uint32_t)(b | 8) << (4 * sp);
        }
        oodw[grp] = w;
      }
      for (int sp = 0; sp < 8; ++sp)
        if (!hdr->ood_valid || hdr->ood_max[4][sp] >= 1) seen |= 1u << sp;
      // The forward's biases and output weights in LDS, with a layout whose
      // offsets point there (the weight matrices are staged above).
      for (int x = gp.gl; x < kHid; x += G) {
        ml.pb[x] = prm[mlay.ob1 + x];
        ml.pb[kHid + x] = prm[mlay.ob2 + x];
        ml.pb[2 * kHid + x] = prm[mlay.ow3 + x];
      }
      if (gp.gl == 0) ml.pb[3 * kHid] = prm[mlay.ob3];
      play = mlay;
      play.ob1 = 0;
      play.ob2 = kHid;
      play.ow3 = 2 * kHid;
      play.ob3 = 3 * kHid;
      gsync();
    }
#pragma unroll
    for (int m = 0; m < FM; ++m) foot[m] = foot_[m];
  }

  // Level l (1-based) of the tree: its nodes and their count.  Level m of
  // the layout holds ceil(nv_max / 8^(m-1)) nodes.
  __device__ __forceinline__ double *Q(int l) const {
    int o = 0;
    for (int m = 1; m < l; ++m) {
      const int sh = 3 * (m - 1);
      o += (a.nv_max + (1 << sh) - 1) >> sh;
    }
    return s.q + o;
  }
  __device__ __forceinline__ int nl(int l) const {
    const int sh = 3 * (l - 1);
    return (nv + (1 << sh) - 1) >> sh;
  }

  __device__ double node_value(int l, int u) const {
    if (l == 1) return s.part[u * 8 + 7];
    const int cnt = min(8, nl(l - 1) - 8 * u);
    return Q(l - 1)[8 * u + cnt - 1];
  }

  // Value held by lane c-D of the same 16-lane row (DPP row_shr:D).
  template <int D>
  __device__ __forceinline__ static double row_shr(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x110 + D, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x110 + D, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
  }

  // Inclusive sums within each 8-lane subgroup in a fixed order
  // (Kogge-Stone: y <- y[c-d] + y[c] for d = 1, 2, 4, where c >= d): lane c
  // returns the sum of x_0..x_c.  The order depends only on the 8 values,
  // never on how many lanes serve a lattice.  Every lane of the wavefront
  // must execute it.
  __device__ __forceinline__ static double subgroup_prefix(double x, int c) {
    double y = x;
    double t = row_shr<1>(y);
    if (c >= 1) y = t + y;
    t = row_shr<2>(y);
    if (c >= 2) y = t + y;
    t = row_shr<4>(y);
    if (c >= 4) y = t + y;
    return y;
  }

  // Value of x in lane src of this group (src uniform over the group).
  __device__ __forceinline__ double lane_value(double x, int src) const {
    if (G == 64) {
      const int lo = __builtin_amdgcn_readlane(__double2loint(x), src);
      const int hi = __builtin_amdgcn_readlane(__double2hiint(x), src);
      return __hiloint2double(hi, lo);
    }
    return __shfl(x, gp.base + src, 64);
  }

  // Re-sums the tree path above one refreshed slot v whose new total is
  // gv: every level's node values are read up front (a lane with nothing to
  // read loads a valid dummy and drops it, so no branch is taken), the one
  // node on the path takes the value just computed below it, and each
  // level's partials come from subgroup_prefix.  Returns Gamma_tot.
  __device__ double update_path(int v, double gv) {
    const int c = gp.gl & 7;
    const bool worker = gp.gl < 8;
    double x[KL + 1];
#pragma unroll
    for (int l = 1; l <= KL; ++l) {
      x[l] = 0.0;
      if (l <= nlev) {
        const int u = 8 * (v >> (3 * l)) + c;
        const bool ok = worker && u < nl(l);
        const int uu = ok ? u : 0;
        double val;
        if (l == 1) {
          val = s.part[uu * 8 + 7];
        } else {
          const int cnt = min(8, nl(l - 1) - 8 * uu);
          val = Q(l - 1)[8 * uu + cnt - 1];
        }
        x[l] = ok ? val : 0.0;
      }
    }
    double fresh = gv;
#pragma unroll
    for (int l = 1; l <= KL; ++l) {
      if (l <= nlev) {
        const int g = v >> (3 * l);
        if (c == ((v >> (3 * (l - 1))) & 7)) x[l] = fresh;
        const double pfx = subgroup_prefix(x[l], c);
        const int cnt = min(8, nl(l) - 8 * g);
        if (worker && c < cnt) Q(l)[8 * g + c] = pfx;
        if (l == nlev) top_q = pfx;
        fresh = lane_value(pfx, cnt - 1);
      }
    }
    gsync();
    return fresh;
  }

  // Learned-barrier rates of one refresh pass (all 64 lanes take part in the
  // matrix-core forward; lane q*8+k owns candidate k of pass slot q).
  __device__ double eval_mlp_pass(int np, int q, int k, int p0, int &vv) {
    const uint8_t *box = s.box + q * BB;
    int A = V;
    bool ood = false;
    float ea_pair = 0.f;
    uint8_t *row = ml.senv + gp.gl * 32;
    if (q >= np) {
      // Rows of lanes without a candidate take part in the last tile: code S
      // sets no input feature.
#pragma unroll
      for (int x = 0; x < kSlots; ++x) row[x] = (uint8_t)S;
    } else {
      vv = s.aff[p0 + q];
      const int flip = (~k) & 7;
      const int jb = kBoxC + dir_sx(k) + 7 * dir_sy(k) + 49 * dir_sz(k);
      // Every box byte is read before the first row byte is written (the
      // compiler cannot tell the row from the box, so a write between two
      // reads would make the second wait for the first).
      uint8_t n1i[8], n1j[8], n2i[6], n2j[6];
      A = box[jb] >> 2;
#pragma unroll
      for (int d2 = 0; d2 < 8; ++d2) {
        const int qq = d2 ^ flip;
        const int off = dir_sx(qq) + 7 * dir_sy(qq) + 49 * dir_sz(qq);
        n1i[d2] = box[kBoxC + off] >> 2;
        n1j[d2] = box[jb + off] >> 2;
      }
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        const int axis = m >> 1;
        const int mm = ((flip >> (2 - axis)) & 1) ? (m ^ 1) : m;
        const int off = ((mm & 1) ? -1 : 1) * (axis == 0 ? 2 : axis == 1 ? 14 : 98);
        n2i[m] = box[kBoxC + off] >> 2;
        n2j[m] = box[jb + off] >> 2;
      }
      row[0] = (uint8_t)A;
      uint32_t c1i = 0, c1j = 0, c2i = 0, c2j = 0;
#pragma unroll
      for (int d2 = 0; d2 < 8; ++d2) {
        if (d2 < 7) { row[1 + d2] = n1i[d2]; c1i += onehot(n1i[d2]); }
        if (d2 > 0) { row[13 + d2] = n1j[d2]; c1j += onehot(n1j[d2]); }
      }
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        row[8 + m] = n2i[m];
        row[21 + m] = n2j[m];
        c2i += onehot(n2i[m]);
        c2j += onehot(n2j[m]);
      }
      if (A != V) {
        // N1(i) without j does not contain the moving atom's site; the box
        // centre (the vacancy) is not part of N1(j) without i.
        const Real de = delta_e_counts<Real>(c1i, c1j, c2i, c2j, s.D1 + 8 * A, s.D2 + 8 * A);
        ea_pair = (float)(s.e0[A] + Real(0.5) * de);
        // A count nibble c exceeds its bound b exactly when (b + 8) - c has
        // its top bit clear (no borrow crosses nibbles: b + 8 - c >= 1).
        const uint32_t hi = 0x88888888u;
        ood = !((seen >> A) & 1u) || ((oodw[0] - c1i) & hi) != hi || ((oodw[1] - c2i) & hi) != hi ||
              ((oodw[2] - c1j) & hi) != hi || ((oodw[3] - c2j) & hi) != hi;
      }
    }
    gsync();
    const int ntiles = (np * 8 + 15) / 16;
    for (int t = 0; t < ntiles; ++t) {
      onehot_tile(ml.senv + t * 16 * 32, ml.atile, S, k1, gp.gl);
      // the helper wavefronts take their share of the tile
      if (gp.gl == 0) *ml.cmd = 1 + t;
      __syncthreads();
      mlp_tile_waves(ml, k1, 0, ml.yb + 16 * t);
    }
    double r = 0.0;
    const bool live = q < np && A != V;
    if (q < np) s.spec[vv * 8 + k] = (uint8_t)A;
    float ea = __builtin_huge_valf();
    if (live) {
      ea = ood ? ea_pair : mu + sigma * ml.yb[gp.gl];
      r = (double)rate_from_barrier(ea, (float)nu, (float)kT);
    }
    if (eat && q < np) eat[vv * 8 + k] = (Real)ea;
    n_ood += __popcll(gp.ballot(live && ood));
    return r;
  }

  // Re-evaluates the slots aff[0..na).  The footprint gathers of the first
  // pass are issued before this event's swap is stored (swap_lane0: lane 0
  // then stores occ[si] = A_new and occ[sj] = V), and the two swapped sites
  // are patched in the boxes, so the gathers never wait for the swap; the
  // stores of earlier events were completed by the caller's fence.
  __device__ void refresh(int na, int si, int sj, int a_new, bool swap_lane0,
                          akmc_event *ev, const akmc_event &rec) {
    constexpr int P = G / 8;
    for (int p0 = 0; p0 < na; p0 += P) {
      const int np = min(P, na - p0);
      int site[FM];
      uint8_t val[FM];
#pragma unroll
      for (int m = 0; m < FM; ++m) {
        const int f = foot[m];
        site[m] = -1;
        val[m] = (uint8_t)V;
        if (f < 0 || fe_q(f) >= np || fe_centre(f)) continue;
        const int pp = s.pos[s.aff[p0 + fe_q(f)]];
        const int X = wrapc(pos_x(pp) + fe_dx(f), g.X2);
        const int Y = wrapc(pos_y(pp) + fe_dy(f), g.Y2);
        const int Z = wrapc(pos_z(pp) + fe_dz(f), g.Z2);
        site[m] = site_of(g, X, Y, Z);
        val[m] = occ[site[m]];
      }
      if (p0 == 0 && swap_lane0 && gp.gl == 0) {
        occ[si] = (uint8_t)a_new;
        occ[sj] = (uint8_t)V;
        if (ev) *ev = rec;
      }
#pragma unroll
      for (int m = 0; m < FM; ++m) {
        const int f = foot[m];
        if (f < 0 || fe_q(f) >= np) continue;
        uint8_t v8 = val[m];
        if (site[m] == si) v8 = (uint8_t)a_new;
        else if (site[m] == sj) v8 = (uint8_t)V;
        s.box[fe_q(f) * BB + fe_byte(f)] = (uint8_t)(v8 << 2);
      }
      gsync();
      const int q = gp.gl >> 3, k = gp.gl & 7;
      double r = 0.0;
      int vv = 0;
      if (!MLP) {
        if (q < np) {
          vv = s.aff[p0 + q];
          int A;
          Real ea;
          if (FAR)
            r = eval_box6<Real>(s.box + q * BB, k, V, S, s.D1, s.D2, s.Dx, s.e0, nu, kT, A, ea);
          else
            r = eval_box<Real>(s.box + q * BB, k, V, s.D1, s.D2, s.e0, nu, kT, A, ea);
          s.spec[vv * 8 + k] = (uint8_t)A;
          if (eat) eat[vv * 8 + k] = ea;
        }
      } else {
        r = eval_mlp_pass(np, q, k, p0, vv);
      }
      if (LRN) r = learned_pass(np, p0, q, k, r, vv);
      // part[v][k] = r0 + r1 + ... + rk
      const double acc = subgroup_prefix(r, k);
      if (q < np) s.part[vv * 8 + k] = acc;
      gsync();
    }
  }

  // Learned runtime forms for the np slots aff[p0 ..] of one refresh pass
  // whose boxes are gathered (lane q*8+k holds the pair rate r of candidate
  // k of pass slot q, vv that slot): stores each slot's total pair rate and
  // Poisson value, and returns the weight the selection uses for this
  // lane's candidate (the policy's exp(z_hat), or r).
  __device__ double learned_pass(int np, int p0, int q, int k, double r, int vv) {
    static_assert(!LRN || G == 64, "the learned forms run on one 64-lane group");
    const int gl = gp.gl;
    const double pfx = subgroup_prefix(r, k);
    if (q < np && k == 7) pg[vv] = pfx;
    for (int qq = 0; qq < np; ++qq) obs[qq * kObsN + gl] = s.box[qq * BB + obs_src] >> 2;
    gsync();
    if (split) {
      // the second wavefront evaluates the Poisson network of these slots
      if (gl == 0) {
        lcmd[0] = np;
        lcmd[1] = p0;
      }
      __syncthreads();
    }
    for (int qq = 0; qq < np; ++qq) {
      const int v_q = s.aff[p0 + qq];
      if (has_pol) {
        const float z = patch_forward(pol, obs + qq * kObsN, hbuf, gl);
        if (gl < 8) {
          const bool ok = s.spec[v_q * 8 + gl] != (uint8_t)V;
          wq[qq * 8 + gl] = ok ? exp((double)(z * inv_tau)) : 0.0;
        }
      }
      if (has_pt && !split) {
        const float gval = patch_forward(pt, obs + qq * kObsN, hbuf, gl);
        if (gl == 0) gv[v_q] = (double)gval;
      }
    }
    if (split) __syncthreads();  // gv of these slots written
    gsync();
    return has_pol ? (q < np ? wq[gl] : 0.0) : r;
  }

  // Distinct parents (index >> 3) of an ascending list.
  __device__ int parents(const int *in, int n_in, int *out) {
    int n_out = 0;
    for (int b0 = 0; b0 < n_in; b0 += G) {
      const int idx = b0 + gp.gl;
      bool keep = false;
      int p = 0;
      if (idx < n_in) {
        p = in[idx] >> 3;
        keep = (idx == 0) || ((in[idx - 1] >> 3) != p);
      }
      const uint64_t m = gp.ballot(keep);
      if (keep) out[n_out + __popcll(m & gp.lanes_below())] = p;
      n_out += __popcll(m);
    }
    gsync();
    return n_out;
  }

  // Re-sums the level-l groups listed in grp[0..ng).
  __device__ void fold_level(int l, const int *grp, int ng) {
    constexpr int P = G / 8;
    for (int p0 = 0; p0 < ng; p0 += P) {
      const int q = gp.gl >> 3, c = gp.gl & 7;
      const bool live = q < min(P, ng - p0);
      int base = 0, cnt = 0;
      double x = 0.0;
      if (live) {
        base = grp[p0 + q] * 8;
        cnt = min(8, nl(l) - base);
        if (c < cnt) x = node_value(l, base + c);
      }
      const double acc = subgroup_prefix(x, c);
      if (live && c < cnt) Q(l)[base + c] = acc;
      gsync();
    }
  }

  __device__ void update_tree(int na) {
    int n = parents(s.aff, na, s.la);
    int *cur = s.la, *nxt = s.lb;
    for (int l = 1; l <= nlev; ++l) {
      fold_level(l, cur, n);
      if (l == nlev) break;
      n = parents(cur, n, nxt);
      int *t = cur; cur = nxt; nxt = t;
    }
  }

  __device__ double gamma_tot() {
    top_q = gp.gl < nl(nlev) ? Q(nlev)[gp.gl] : 0.0;
    if (G == 64 && nlev >= 2) {
      const bool in2 = gp.gl < nl(2);
      t2 = in2 ? node_value(2, gp.gl) : 0.0;
      q2 = in2 ? Q(2)[gp.gl] : 0.0;
      const bool in3 = nlev >= 3 && gp.gl < nl(3);
      t3 = in3 ? node_value(3, gp.gl) : 0.0;
      q3 = in3 ? Q(3)[gp.gl] : 0.0;
    }
    return Q(nlev)[nl(nlev) - 1];
  }

  // update_path for a 64-lane group with at least two levels: x1 (lane
  // c < 8) holds the totals of the 8 slots of v's level-1 group, read
  // before this event changed anything; levels 2 and 3 come from the
  // registers.  The same partials as update_path, the same LDS stores.
  __device__ double update_path_regs(int v, double gv, double x1) {
    const int gl = gp.gl, c = gl & 7;
    const int g1 = v >> 3, g2 = v >> 6;
    x1 = c == (v & 7) ? gv : x1;
    const double p1 = subgroup_prefix(x1, c);
    const int cnt1 = min(8, nv - 8 * g1);
    if (gl < cnt1) Q(1)[8 * g1 + gl] = p1;
    double fresh = lane_value(p1, cnt1 - 1);
    t2 = gl == g1 ? fresh : t2;
    q2 = subgroup_prefix(t2, c);
    const int cnt2 = min(8, nl(2) - 8 * g2);
    if ((gl >> 3) == g2 && c < cnt2) Q(2)[gl] = q2;
    fresh = lane_value(q2, 8 * g2 + cnt2 - 1);
    if (nlev == 2) {
      top_q = gl < 8 ? q2 : 0.0;
    } else {
      t3 = gl == g2 ? fresh : t3;
      q3 = subgroup_prefix(t3, c);
      const int cnt3 = nl(3);
      if (gl < cnt3) Q(3)[gl] = q3;
      top_q = gl < 8 ? q3 : 0.0;
      fresh = lane_value(q3, cnt3 - 1);
    }
    gsync();
    return fresh;
  }

  // The tree paths of the na <= 8 refreshed slots aff[0 .. na) at once (a
  // 64-lane group with tree levels 2 and 3 in registers): subgroup p
  // re-sums the level-1 group of slot aff[p] from the slot totals, the
  // register levels take every new group total and are re-summed once.
  // Each node is the same fixed function of its children as with one path
  // at a time (a group listed twice is summed twice, to the same values).
  __device__ double update_paths_regs(int na) {
    const int gl = gp.gl, c = gl & 7, p = gl >> 3;
    const int g1 = s.aff[min(p, na - 1)] >> 3;
    const int cnt1 = min(8, nv - 8 * g1);
    const double xr = s.part[(8 * g1 + min(c, cnt1 - 1)) * 8 + 7];  // unpredicated
    const double p1 = subgroup_prefix(c < cnt1 ? xr : 0.0, c);
    if (p < na && c < cnt1) Q(1)[8 * g1 + c] = p1;
    for (int pp = 0; pp < na; ++pp) {
      const int gg = __builtin_amdgcn_readlane(g1, 8 * pp);
      const int cc = min(8, nv - 8 * gg);
      const double tot = lane_value(p1, 8 * pp + cc - 1);
      t2 = gl == gg ? tot : t2;
    }
    q2 = subgroup_prefix(t2, c);
    const int n2 = nl(2);
    if (gl < n2) Q(2)[gl] = q2;
    double fresh;
    if (nlev == 2) {
      top_q = gl < 8 ? q2 : 0.0;
      fresh = lane_value(q2, n2 - 1);
    } else {
      for (int pp = 0; pp < na; ++pp) {
        const int gg = __builtin_amdgcn_readlane(g1, 8 * pp) >> 3;
        const int cc = min(8, n2 - 8 * gg);
        const double tot = lane_value(q2, 8 * gg + cc - 1);
        t3 = gl == gg ? tot : t3;
      }
      q3 = subgroup_prefix(t3, c);
      const int n3 = nl(3);
      if (gl < n3) Q(3)[gl] = q3;
      top_q = gl < 8 ? q3 : 0.0;
      fresh = lane_value(q3, n3 - 1);
    }
    gsync();
    return fresh;
  }

  // One selection step at level l >= 2 from the registers (a 64-lane
  // group): the children of the node whose first child is `base` sit in
  // lanes base .. base+cnt-1 of q (partials) and t (values).  The same
  // comparisons and fallback as the LDS step of the descent.
  __device__ __forceinline__ int select_regs(int l, int base, double q, double t, double &tgt) const {
    const int gl = gp.gl;
    const int cnt = min(8, nl(l) - base);
    const bool in = gl >= base && gl < base + cnt;
    uint64_t m = (gp.ballot(in && q > tgt) >> base) & 0xffull;
    int c;
    if (m) {
      c = __ffsll((unsigned long long)m) - 1;
    } else {
      const uint64_t m2 = (gp.ballot(in && t > 0.0) >> base) & 0xffull;
      c = m2 ? 63 - __clzll((long long)m2) : 0;
    }
    if (c > 0) tgt = tgt - lane_value(q, base + c - 1);
    return base + c;
  }

  // x of lane 15 of the previous 16-lane row (DPP row_bcast:15; rows in
  // row_mask only, the others receive 0), and of lane 31 (row_bcast:31).
  template <int CTRL, int ROWS>
  __device__ __forceinline__ static double row_bcast(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
  }

  // Sum of a per-slot array in an order fixed by nv alone: lane l adds
  // slots l, l + 64, ... in turn; each 16-lane row is summed by a
  // Kogge-Stone scan over DPP row shifts, the row totals are added by row
  // broadcasts (rows 0+1, 2+3, then both halves) and lane 63's total is
  // returned to every lane.  64-lane groups only.
  __device__ double slot_sum(const double *x) const {
    double acc = 0.0;
    for (int v = gp.gl; v < nv; v += 64) acc += x[v];
    acc += row_shr<1>(acc);
    acc += row_shr<2>(acc);
    acc += row_shr<4>(acc);
    acc += row_shr<8>(acc);
    acc += row_bcast<0x142, 0xA>(acc);
    acc += row_bcast<0x143, 0xC>(acc);
    return lane_value(acc, 63);
  }

  // Coarse vacancy grid (vac_grid): the cell of a position, and the count
  // field of a cell; the moved vacancy's count goes from cell to cell by
  // LDS atomics (no borrow: a count is at least 1 where it is decremented).
  __device__ __forceinline__ static int grid_cell(const VacGrid &vg, int X, int Y, int Z) {
    const int cx = min(X >> vg.lc, vg.nx - 1), cy = min(Y >> vg.lc, vg.ny - 1),
              cz = min(Z >> vg.lc, vg.nz - 1);
    return (cz * vg.ny + cy) * vg.nx + cx;
  }
  __device__ __forceinline__ int grid_count(const VacGrid &vg, int cell) const {
    const uint32_t w = s.grid[cell >> (5 - vg.fb)];
    return (int)((w >> ((cell << vg.fb) & 31)) & ((1u << (1 << vg.fb)) - 1u));
  }
  __device__ __forceinline__ void grid_inc(const VacGrid &vg, int cell) {
    atomicAdd(&s.grid[cell >> (5 - vg.fb)], 1u << ((cell << vg.fb) & 31));
  }
  __device__ __forceinline__ void grid_dec(const VacGrid &vg, int cell) {
    atomicSub(&s.grid[cell >> (5 - vg.fb)], 1u << ((cell << vg.fb) & 31));
  }

  __device__ void run(int lat) {
    const LatDesc *d = a.descs + lat;
    LatState *st = a.states + lat;
    const int gl = gp.gl;
    g = make_geo(d->lx, d->ly, d->lz);
    S = d->S;
    V = S - 1;
    nv = d->nv;
    occ = a.occ + d->occ_off;
    int32_t *slots = a.slots + d->slot_off;
    eat = a.ea_trace ? (Real *)a.ea_trace + d->slot_off * 8 : nullptr;
    akmc_event *evlog = a.log ? a.log + (int64_t)lat * a.log_stride : nullptr;
    const bool fp32 = sizeof(Real) == 4;
    for (int x = gl; x < 64; x += G) {
      s.D1[x] = fp32 ? (Real)d->D1f[x] : (Real)d->D1[x];
      s.D2[x] = fp32 ? (Real)d->D2f[x] : (Real)d->D2[x];
    }
    if (gl < 8) s.e0[gl] = fp32 ? (Real)d->e0f[gl] : (Real)d->e0[gl];
    if (FAR)
      for (int x = gl; x < 256; x += G) s.Dx[x] = fp32 ? (Real)(&d->Dxf[0][0])[x] : (Real)(&d->Dx[0][0])[x];
    if constexpr (FAR && G == 64) {
#pragma unroll
      for (int u = 0; u < kFarGroupMax; ++u) {
        const int m = kFarGroups.m[gl & 7][u];
        fo[u] = m >= 0 ? kBondFarDev.off[m] : kFarNone;
      }
    }
    nu = fp32 ? (Real)d->nuf : (Real)d->nu;
    kT = fp32 ? (Real)d->kTf : (Real)d->kT;
    const uint64_t seed = d->seed, stream = d->stream;
    const int time_mode = d->time_mode;
    const bool full = a.refresh_full != 0;

    nlev = 1;
    while (nl(nlev) > 8 && nlev < KL) ++nlev;

    double t = st->t;
    int64_t n = st->n;
    uint64_t dig = st->digest;
    int frozen = st->frozen;
    if (frozen) return;
    const int64_t clk0 = wall_clock64();

    // The vacancy grid rules out other slots near a jump in one LDS read
    // per lane; it only decides whether the exact scan runs.
    const VacGrid vg = vac_grid(g.lx, g.ly, g.lz, nv, REACH, s.grid_words);
    const bool use_grid = !full && vg.words > 0;
    if (use_grid) {
      for (int w = gl; w < vg.words; w += G) s.grid[w] = 0u;
      gsync();
    }
    for (int v = gl; v < nv; v += G) {
      int X, Y, Z;
      pos_of(g, slots[v], X, Y, Z);
      s.pos[v] = pack_pos(X, Y, Z);
      s.aff[v] = v;
      if (use_grid) grid_inc(vg, grid_cell(vg, X, Y, Z));
    }
    gsync();
    akmc_event none{};
    refresh(nv, -1, -1, 0, false, nullptr, none);
    update_tree(nv);
    double gtot = gamma_tot();
    // With the learned forms the tree holds the selection weights; the
    // physical total rate (time) and u(s) are sums over the slots.
    double gphys = gtot, uval = 0.0;
    if (LRN) {
      if (has_pol) gphys = slot_sum(pg);
      if (has_pt) uval = slot_sum(gv);
    }
    frozen = !(gtot > 0.0) || !(gphys > 0.0);

    double ru1v = 0.0, rwv = 0.0;
    // An event starts only while t < t_end (+inf unless the launch advances
    // lattices to a physical-time horizon), so the event that reaches the
    // horizon is the last one.
    for (int64_t e = 0; e < a.n_events && !frozen && t < a.t_end; ++e) {
      const int ce = (int)(e % G);
      if (ce == 0) {
        double u1, u2;
        event_uniforms(seed, stream, n + gl, u1, u2);
        if (G == 64) {  // lane c keeps event c's pair in registers
          ru1v = u1;
          rwv = -log(u2);
        } else {
          s.ru1[gl] = u1;
          s.rw[gl] = -log(u2);
          gsync();
        }
      }
      const double u1 = G == 64 ? lane_value(ru1v, ce) : s.ru1[ce];
      const double w = G == 64 ? lane_value(rwv, ce) : s.rw[ce];
      double tgt = u1 * gtot;

      // Selection: descend the tree of partial sums.  Levels nlev..1 hold
      // the slot tree; level 0 is the per-direction partials part[8v + k].
      // At each level the child is the first whose inclusive partial sum
      // exceeds the target, and the target drops by the partial sum before
      // it.  A full wavefront takes two levels per LDS round trip (lane
      // 8c + c' looks at grandchild c' of child c); the comparisons and
      // subtractions are the same, so the result does not depend on G.
      // The level loop is unrolled at compile time so that every level's
      // offsets are constants and the descent stays in scalar registers.
      int node = 0;
      bool skip = false;
      // A 64-lane group takes levels nlev .. 2 from the registers, then
      // levels 1 and 0 in one LDS round trip.
      int ltop = nlev;
      if (G == 64 && nlev >= 2) {
        if (nlev == 3) node = select_regs(3, 0, q3, t3, tgt);
        node = select_regs(2, nlev == 3 ? 8 * node : 0, q2, t2, tgt);
        ltop = 1;
      }
#pragma unroll
      for (int l = KL; l >= 0; --l) {
        if (l > ltop) continue;
        if (skip) {
          skip = false;
          continue;
        }
        const int base = (l == nlev) ? 0 : node * 8;
        if (G == 64 && l >= 1) {
          const int c = gl >> 3, c2 = gl & 7;
          const int cntA = min(8, nl(l) - base);
          const bool inA = c < cntA;
          const double *qa_p = Q(l) + base;
          // Every lane reads a valid entry (indices clamped into range), so
          // no read is predicated; out-of-range lanes are masked below.
          const double qa = qa_p[min(c, cntA - 1)];
          const double qp = qa_p[max(min(c, cntA - 1) - 1, 0)];
          const int baseB = 8 * (base + c);
          const int nlB = l >= 2 ? nl(l - 1) : 8 * nv;
          const bool inB = inA && c2 < min(8, nlB - baseB);
          const int ib = min(baseB + c2, nlB - 1);
          const double qb = l >= 2 ? Q(l - 1)[ib] : s.part[ib];
          // all three reads in one round trip: keeps the compiler from
          // moving the last two behind the first comparison
          __asm__ volatile("" ::"v"(qa), "v"(qp), "v"(qb));
          const uint64_t mA = gp.ballot(c2 == 0 && inA && qa > tgt);
          if (mA) {
            const int cs = (__ffsll((unsigned long long)mA) - 1) >> 3;
            const double t1 = c > 0 ? tgt - qp : tgt;
            const uint64_t mB = gp.ballot(c == cs && inB && qb > t1);
            const double t1u = lane_value(t1, 8 * cs);
            if (mB) {
              const int cb = (__ffsll((unsigned long long)mB) - 1) & 7;
              const double qbp = lane_value(qb, 8 * cs + (cb > 0 ? cb - 1 : 0));
              tgt = cb > 0 ? t1u - qbp : t1u;
              node = 8 * (base + cs) + cb;
              skip = true;
            } else {
              // No grandchild exceeds the target (rounding): level l-1
              // takes the single step below with its fallback.
              tgt = t1u;
              node = base + cs;
            }
            continue;
          }
        }
        const int cnt = l >= 1 ? min(8, nl(l) - base) : 8;
        const bool in = gl < cnt;
        double qv = 0.0;
        if (in) qv = l == 0 ? s.part[base + gl] : (l == nlev ? top_q : Q(l)[base + gl]);
        uint64_t m = gp.ballot(in && (qv > tgt)) & 0xffull;
        int c;
        if (m) {
          c = __ffsll((unsigned long long)m) - 1;
        } else if (l >= 1) {
          const double cv = in ? node_value(l, base + gl) : 0.0;
          const uint64_t m2 = gp.ballot(in && (cv > 0.0)) & 0xffull;
          c = m2 ? 63 - __clzll((long long)m2) : 0;
        } else {
          const uint64_t m2 = gp.ballot(in && (s.spec[base + gl] != V)) & 0xffull;
          c = m2 ? 63 - __clzll((long long)m2) : 0;
        }
        const double prev = lane_value(qv, c > 0 ? c - 1 : 0);
        if (c > 0) tgt = tgt - prev;
        node = base + c;
      }
      const int v = node >> 3, k = node & 7;
      // Totals of the 8 slots of v's level-1 group, for the tree update at
      // the end of the event (read together with the chosen candidate).
      double x1 = 0.0;
      if (G == 64 && nlev >= 2) {
        const int u = 8 * (v >> 3) + (gl & 7);
        x1 = gl < 8 && u < nv ? s.part[u * 8 + 7] : 0.0;
      }
      int A = s.spec[v * 8 + k];
      int pp = s.pos[v];
      if (G == 64) {  // one lattice per wavefront: keep the event's scalars in SGPRs
        A = __builtin_amdgcn_readfirstlane(A);
        pp = __builtin_amdgcn_readfirstlane(pp);
        // x1 arrives with A and pp (not re-read at its use)
        __asm__ volatile("" ::"v"(x1));
      }
      const int X = pos_x(pp), Y = pos_y(pp), Z = pos_z(pp);
      const int JX = wrapc(X + dir_sx(k), g.X2), JY = wrapc(Y + dir_sy(k), g.Y2),
                JZ = wrapc(Z + dir_sz(k), g.Z2);
      const int si = site_of(g, X, Y, Z), sj = site_of(g, JX, JY, JZ);
      // Poisson time (Eq. 7) needs the state after the jump: its dt is set
      // after the refresh.
      double dt = time_mode ? 1.0 / gphys : w / gphys;
      akmc_event rec;
      rec.n = n;
      rec.slot = v;
      rec.from_site = si;
      rec.to_site = sj;
      rec.dir = (uint8_t)k;
      rec.species = (uint8_t)A;
      rec.pad[0] = 0;
      rec.pad[1] = 0;
      rec.gamma_tot = gphys;
      rec.dt = dt;
      akmc_event *ev = evlog ? evlog + e : nullptr;
      const bool late_rec = LRN && has_pt;   // the record waits for Eq. 7's dt

      // Stores of earlier events are complete before any gather.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      // Footprint of the moved vacancy around its new site j, gathered
      // before the swap is stored; the two swapped sites are patched below.
      // Box 0 holds elements 0 .. kFootN-1, i.e. the first M0 of this lane.
      constexpr int M0 = (FN + G - 1) / G;
      int site0[M0];
      uint8_t val0[M0];
#pragma unroll
      for (int m = 0; m < M0; ++m) {
        const int f = foot[m];
        site0[m] = -1;
        val0[m] = (uint8_t)V;
        if (f < 0 || fe_q(f) != 0 || fe_centre(f)) continue;
        const int FX = wrapc(JX + fe_dx(f), g.X2);
        const int FY = wrapc(JY + fe_dy(f), g.Y2);
        const int FZ = wrapc(JZ + fe_dz(f), g.Z2);
        site0[m] = site_of(g, FX, FY, FZ);
        val0[m] = occ[site0[m]];
      }
      if (gl == 0) {
        occ[si] = (uint8_t)A;
        occ[sj] = (uint8_t)V;
        if (ev && !late_rec) *ev = rec;
      }
      if (gl == 0) s.pos[v] = pack_pos(JX, JY, JZ);
      gsync();

      // Slots whose footprint may contain i or j (always v itself).
      int na;
      if (full) {
        na = nv;
      } else {
        // Usually only v itself is that close: one ballot per 4G slots
        // decides, and the ordered list is built only when another slot
        // is affected.
        auto hits = [&](int b0, bool (&hit)[4]) {
          int qp[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) qp[u] = s.pos[min(b0 + u * G + gl, nv - 1)];  // unpredicated
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            // |d| to i and to j by sum-of-absolute-differences, then the
            // periodic image
            const int px = pos_x(qp[u]), py = pos_y(qp[u]), pz = pos_z(qp[u]);
            int dx = (int)__sad(px, X, 0u), dy = (int)__sad(py, Y, 0u), dz = (int)__sad(pz, Z, 0u);
            int ex = (int)__sad(px, JX, 0u), ey = (int)__sad(py, JY, 0u), ez = (int)__sad(pz, JZ, 0u);
            dx = min(dx, g.X2 - dx);
            dy = min(dy, g.Y2 - dy);
            dz = min(dz, g.Z2 - dz);
            ex = min(ex, g.X2 - ex);
            ey = min(ey, g.Y2 - ey);
            ez = min(ez, g.Z2 - ez);
            // a candidate's bonds lie within 3 half-cells of its vacancy
            // (5 with pairs out to 6.0 A), an observation within 4: REACH - 1
            // per axis; the slot is stale only if i or j lies that close
            hit[u] = b0 + u * G + gl < nv &&
                     (max(dx, max(dy, dz)) < REACH || max(ex, max(ey, ez)) < REACH);
          }
        };
        // The grid first: lane b < 8 reads the cell of (X +- R, Y +- R,
        // Z +- R) (bit 0, 1, 2 of b: + in x, y, z) and counts it without
        // the moved vacancy, still at i there; only if some vacancy may be
        // that close do all slots take the exact test.
        bool scan = true;
        if (use_grid) {
          const int ci = grid_cell(vg, X, Y, Z);
          int c = 0;
          if (gl < 8) {
            const int cell = grid_cell(vg, wrapc(X + ((gl & 1) ? REACH : -REACH), g.X2),
                                       wrapc(Y + ((gl & 2) ? REACH : -REACH), g.Y2),
                                       wrapc(Z + ((gl & 4) ? REACH : -REACH), g.Z2));
            c = grid_count(vg, cell) - (cell == ci ? 1 : 0);
          }
          scan = gp.ballot(c > 0) != 0;
          const int cj = grid_cell(vg, JX, JY, JZ);
          if (gl == 0 && cj != ci) {
            grid_dec(vg, ci);
            grid_inc(vg, cj);
          }
        }
        // One pass builds the ordered list of every slot the exact test
        // hits (v among them); only v means the fast path.
        na = 1;
        if (scan) {
          na = 0;
          for (int b0 = 0; b0 < nv; b0 += 4 * G) {
            bool hit[4];
            hits(b0, hit);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const uint64_t m = gp.ballot(hit[u]);
              if (hit[u]) s.aff[na + __popcll(m & gp.lanes_below())] = b0 + u * G + gl;
              na += __popcll(m);
            }
          }
          gsync();
        } else if (MLP || LRN) {
          if (gl == 0) s.aff[0] = v;
          gsync();
        }
      }
      if (!late_rec) t += dt;
      dig = digest_event(dig, si, sj);
      n += 1;

      if (na == 1) {
        // Only the moved vacancy: its box is already gathered.
#pragma unroll
        for (int m = 0; m < M0; ++m) {
          const int f = foot[m];
          if (f < 0 || fe_q(f) != 0) continue;
          uint8_t v8 = val0[m];
          if (fe_centre(f)) v8 = (uint8_t)V;
          else if (site0[m] == si) v8 = (uint8_t)A;
          else if (site0[m] == sj) v8 = (uint8_t)V;
          s.box[fe_byte(f)] = (uint8_t)(v8 << 2);
        }
        gsync();
        const int kk = gl & 7;
        double r = 0.0;
        if (MLP) {
          // the surrogate on this machine: a pass of one slot (aff[0] is v)
          int vq = v;
          r = eval_mlp_pass(1, gl >> 3, kk, 0, vq);
        } else if (gl < 8) {
          int Ak;
          Real ea;
          if (FAR && G < 64)
            r = eval_box6<Real>(s.box, kk, V, S, s.D1, s.D2, s.Dx, s.e0, nu, kT, Ak, ea);
          else if (!FAR)
            r = eval_box<Real>(s.box, kk, V, s.D1, s.D2, s.e0, nu, kT, Ak, ea);
          if (!FAR || G < 64) {
            s.spec[v * 8 + kk] = (uint8_t)Ak;
            if (eat) eat[v * 8 + kk] = ea;
          }
        }
        if constexpr (FAR && G == 64 && !MLP) {
          // six shells: all 64 lanes count, 8 per candidate
          int Ak;
          Real ea;
          r = eval_box6_wave<Real>(s.box, gl, fo, V, S, s.D1, s.D2, s.Dx, s.e0, nu, kT, Ak, ea);
          if (gl < 8) {
            s.spec[v * 8 + kk] = (uint8_t)Ak;
            if (eat) eat[v * 8 + kk] = ea;
          } else {
            r = 0.0;
          }
        }
        if (LRN) r = learned_pass(1, 0, gl >> 3, kk, r, v);
        const double pfx = subgroup_prefix(r, kk);
        if (gl < 8) s.part[v * 8 + kk] = pfx;
        gtot = G == 64 && nlev >= 2 ? update_path_regs(v, lane_value(pfx, 7), x1)
                                    : update_path(v, lane_value(pfx, 7));
      } else {
        refresh(na, si, sj, A, false, nullptr, rec);
        if (G == 64 && nlev >= 2 && na <= 8) {
          gtot = update_paths_regs(na);
        } else {
          update_tree(na);
          gtot = gamma_tot();
        }
      }
      if (LRN) {
        const double g_prev = gphys, u_prev = uval;
        gphys = has_pol ? slot_sum(pg) : gtot;
        if (has_pt) {
          uval = slot_sum(gv);
          // Eq. 7; a frozen successor drops its term (tau = 0 there)
          dt = gphys > 0.0 ? (u_prev - (g_prev / gphys) * uval) / g_prev : u_prev / g_prev;
          t += dt;
          rec.dt = dt;
          if (gl == 0 && ev) *ev = rec;
        }
      } else {
        gphys = gtot;
      }
      frozen = !(gtot > 0.0) || !(gphys > 0.0);
    }

    for (int v = gl; v < nv; v += G) {
      const int q = s.pos[v];
      slots[v] = site_of(g, pos_x(q), pos_y(q), pos_z(q));
    }
    if (gl == 0) {
      st->t = t;
      st->n = n;
      st->digest = dig;
      st->gamma_tot = gtot;
      st->frozen = frozen;
      st->n_ood += n_ood;
      st->busy_ticks += wall_clock64() - clk0;
    }
    gsync();
  }
};

template <int G, int WAVES, bool FP32, bool MLP = false, int KL = kMaxLevels, bool LRN = false,
          bool FAR = false>
__global__ __launch_bounds__(64 * (MLP ? kMlpWaves : WAVES)) void k_event_loop(LoopArgs a, GroupLayout L) {
  using Real = typename std::conditional<FP32, float, double>::type;
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (LRN && WAVES == 2 && wave != 0) {
    // The second wavefront of a learned loop with both networks (WAVES = 2):
    // the Poisson network of each refresh pass the first one announces (the
    // same forward, on its own activation buffer), until the end.
    static_assert(!LRN || (G == 64 && WAVES <= 2), "the learned loop runs one 64-lane group");
    const Lds<Real> sl = carve<Real>(lds, L);
    unsigned char *b = lds + L.bytes;
    double *gv = (double *)b + a.nv_max;
    const uint8_t *obs = (const uint8_t *)((double *)b + 2 * a.nv_max + 64) + 64 * 4;
    float *hbuf = (float *)(obs + 8 * kObsN);
    int *lcmd = (int *)(hbuf + 64);
    unsigned char *nets = (unsigned char *)(lcmd + 4);
    const PatchHeader *ph = (const PatchHeader *)a.pol_blob;
    const PatchNet pt = patch_view(a.pt_blob, nets + patch_lds_bytes(ph->S, ph->H, ph->n_out));
    for (;;) {
      __syncthreads();
      const int np = lcmd[0];
      if (np == 0) break;
      const int p0 = lcmd[1];
      for (int qq = 0; qq < np; ++qq) {
        const float gval = patch_forward(pt, obs + qq * kObsN, hbuf, lane);
        if (lane == 0) gv[sl.aff[p0 + qq]] = (double)gval;
      }
      __syncthreads();
    }
    return;
  }
  if (MLP && wave != 0) {
    // A helper wavefront of the surrogate loop: its share of each tile the
    // event loop (wavefront 0) announces, until the end of the launch.
    static_assert(!MLP || (G == 64 && WAVES == 1), "the surrogate loop runs one 64-lane group");
    const int k1 = ((const MlpHeader *)a.mlp_blob)->k1;
    const MlpLds ml = mlp_lds_at(lds + L.bytes, k1);
    for (;;) {
      __syncthreads();
      const int cmd = *ml.cmd;  // 1 + the tile's place in the pass, 0 at the end
      if (cmd == 0) break;
      mlp_tile_waves(ml, k1, wave, ml.yb + 16 * (cmd - 1));
    }
    return;
  }
  Group<G> gp;
  gp.gw = lane / G;
  gp.gl = lane % G;
  gp.base = gp.gw * G;
  const int gib = wave * (64 / G) + gp.gw;
  unsigned char *mine = lds + (size_t)gib * L.bytes;

  // This lane's share of the footprint gathers: element f = gl + G*m of the
  // (G/8) boxes of a refresh pass, packed as described at fe_dx (box byte,
  // offsets, box number q, centre and far flags); -1 if none.
  using Run = Runner<G, Real, MLP, KL, LRN, FAR>;
  constexpr int FN = Run::FN, FM = Run::FM;
  int foot[FM];
  constexpr int P = G / 8;
#pragma unroll
  for (int m = 0; m < FM; ++m) {
    const int f = gp.gl + G * m;
    if (f >= P * FN) {
      foot[m] = -1;
      continue;
    }
    const int q = f / FN, e = f % FN;
    if (FAR) {
      if (e == FN - 1) {
        foot[m] = fe_pack(kBoxCF, 0, 0, 0, q, true, false);
      } else {
        const int dx = kFootFar.d[e][0], dy = kFootFar.d[e][1], dz = kFootFar.d[e][2];
        foot[m] = fe_pack((dx + 5) + 11 * (dy + 5) + 121 * (dz + 5), dx, dy, dz, q, false, false);
      }
    } else if (e == FN - 1) {
      foot[m] = fe_pack(kBoxC, 0, 0, 0, q, true, false);
    } else if (e >= kFootN - 1) {
      const int fi = e - (kFootN - 1);  // order of kFarD: -x, -y, -z, +z, +y, +x
      const int axis = fi < 3 ? fi : 5 - fi, len = fi < 3 ? -4 : 4;
      const int dx = axis == 0 ? len : 0, dy = axis == 1 ? len : 0, dz = axis == 2 ? len : 0;
      foot[m] = fe_pack(fi, dx, dy, dz, q, false, true);
    } else {
      const int dx = kFoot.d[e][0], dy = kFoot.d[e][1], dz = kFoot.d[e][2];
      foot[m] = fe_pack((dx + 3) + 7 * (dy + 3) + 49 * (dz + 3), dx, dy, dz, q, false, false);
    }
  }

  Run run(a, L, gp, foot, mine);
  for (;;) {
    int idx = 0;
    if (gp.gl == 0) idx = atomicAdd(a.queue, 1);
    idx = gp.bcast(idx, 0);
    // one lattice per wavefront: its index, and everything derived from
    // it, is uniform (scalar registers and branches)
    if (G == 64) idx = __builtin_amdgcn_readfirstlane(idx);
    if (idx >= a.n_lat) break;
    int lat = a.order[idx];
    if (G == 64) lat = __builtin_amdgcn_readfirstlane(lat);
    run.run(lat);
  }
  if (MLP) {
    // releases the helper wavefronts
    if (lane == 0) *run.ml.cmd = 0;
    __syncthreads();
  }
  if (LRN && WAVES == 2 && run.split) {
    if (lane == 0) run.lcmd[0] = 0;
    __syncthreads();
  }
}

__global__ void k_queue_reset(int32_t *queue) { *queue = 0; }

hipError_t launch_queue_reset(int32_t *queue, hipStream_t stream) {
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, stream, queue);
  return hipGetLastError();
}

size_t event_loop_lds_bytes(int nv_max, int group_lanes, int waves_per_block, int precision,
                            int grid_words) {
  const GroupLayout L = make_layout(nv_max, group_lanes, precision == AKMC_FP32, 0, grid_words);
  return (size_t)L.bytes * (size_t)(64 / group_lanes) * (size_t)waves_per_block;
}

size_t event_loop_mlp_lds_bytes(int nv_max, int n_species, int grid_words) {
  return (size_t)make_layout(nv_max, 64, 1, 0, grid_words).bytes + mlp_loop_lds_bytes(n_species);
}

template <int G, int W, bool FP32>
static hipError_t launch_one(const LoopArgs &a, const Schedule &s, hipStream_t stream) {
  const GroupLayout L = make_layout(a.nv_max, G, FP32 ? 1 : 0, 0, a.grid_words);
  const size_t lds = (size_t)L.bytes * (64 / G) * W;
  // Lattices of at most 64 slots need two tree levels: a shorter unrolled
  // descent and re-sum.
  static_assert(kMaxLevels == 3, "level variants");
  auto kern = L.nlev_max <= 2 ? k_event_loop<G, W, FP32, false, 2> : k_event_loop<G, W, FP32, false, 3>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int blocks = s.blocks;
  const int groups_per_block = (64 / G) * W;
  const int need = (a.n_lat + groups_per_block - 1) / groups_per_block;
  if (blocks <= 0 || blocks > need) blocks = need;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * W), lds, stream, a, L);
  return hipGetLastError();
}

template <int G, bool FP32>
static hipError_t launch_w(const LoopArgs &a, const Schedule &s, hipStream_t stream) {
  switch (s.waves_per_block) {
    case 2: return launch_one<G, 2, FP32>(a, s, stream);
    case 4: return launch_one<G, 4, FP32>(a, s, stream);
    default: return launch_one<G, 1, FP32>(a, s, stream);
  }
}

template <bool FP32>
static hipError_t launch_g(const LoopArgs &a, const Schedule &s, hipStream_t stream) {
  switch (s.group_lanes) {
    case 8: return launch_w<8, FP32>(a, s, stream);
    case 16: return launch_w<16, FP32>(a, s, stream);
    case 32: return launch_w<32, FP32>(a, s, stream);
    default: return launch_w<64, FP32>(a, s, stream);
  }
}

hipError_t launch_event_loop_mlp(const LoopArgs &a, int refresh_full, int n_species,
                                 hipStream_t stream) {
  LoopArgs b = a;
  b.refresh_full = refresh_full;
  hipError_t e = launch_queue_reset(a.queue, stream);
  if (e != hipSuccess) return e;
  const GroupLayout L = make_layout(a.nv_max, 64, 1, 0, a.grid_words);
  const size_t lds = event_loop_mlp_lds_bytes(a.nv_max, n_species, a.grid_words);
  auto kern = k_event_loop<64, 1, true, true>;
  e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(1), dim3(64 * kMlpWaves), lds, stream, b, L);
  return hipGetLastError();
}

size_t event_loop_far_lds_bytes(int nv_max, int precision, int grid_words) {
  return (size_t)make_layout(nv_max, 64, precision == AKMC_FP32, 1, grid_words).bytes;
}

template <bool FP32>
static hipError_t launch_far(const LoopArgs &a, hipStream_t stream) {
  const GroupLayout L = make_layout(a.nv_max, 64, FP32 ? 1 : 0, 1, a.grid_words);
  auto kern = L.nlev_max <= 2 ? k_event_loop<64, 1, FP32, false, 2, false, true>
                              : k_event_loop<64, 1, FP32, false, 3, false, true>;
  const size_t lds = (size_t)L.bytes;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(1), dim3(64), lds, stream, a, L);
  return hipGetLastError();
}

hipError_t launch_event_loop_far(const LoopArgs &a, int precision, int refresh_full, hipStream_t stream) {
  LoopArgs b = a;
  b.refresh_full = refresh_full;
  hipError_t e = launch_queue_reset(a.queue, stream);
  if (e != hipSuccess) return e;
  return precision == AKMC_FP32 ? launch_far<true>(b, stream) : launch_far<false>(b, stream);
}

size_t event_loop_lrn_lds_bytes(int nv_max, int precision, const int pol_dims[3],
                                const int pt_dims[3], int grid_words) {
  const GroupLayout L = make_layout(nv_max, 64, precision == AKMC_FP32, 0, grid_words);
  size_t b = (size_t)L.bytes + 16 * (size_t)nv_max + 8 * 64 + 4 * 64 + kObsN * 8 + 4 * 64 + 16;
  if (pol_dims) b += (size_t)patch_lds_bytes(pol_dims[0], pol_dims[1], pol_dims[2]);
  if (pt_dims) b += (size_t)patch_lds_bytes(pt_dims[0], pt_dims[1], pt_dims[2]);
  return b;
}

template <bool FP32, int W>
static hipError_t launch_lrn_w(const LoopArgs &a, size_t lds, hipStream_t stream) {
  const GroupLayout L = make_layout(a.nv_max, 64, FP32 ? 1 : 0, 0, a.grid_words);
  auto kern = L.nlev_max <= 2 ? k_event_loop<64, W, FP32, false, 2, true>
                              : k_event_loop<64, W, FP32, false, 3, true>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(1), dim3(64 * W), lds, stream, a, L);
  return hipGetLastError();
}

template <bool FP32>
static hipError_t launch_lrn(const LoopArgs &a, size_t lds, hipStream_t stream) {
  // with both networks a second wavefront evaluates the Poisson network
  return a.pol_blob && a.pt_blob ? launch_lrn_w<FP32, 2>(a, lds, stream) : launch_lrn_w<FP32, 1>(a, lds, stream);
}

hipError_t launch_event_loop_lrn(const LoopArgs &a, int precision, int refresh_full, size_t lds,
                                 hipStream_t stream) {
  LoopArgs b = a;
  b.refresh_full = refresh_full;
  hipError_t e = launch_queue_reset(a.queue, stream);
  if (e != hipSuccess) return e;
  return precision == AKMC_FP32 ? launch_lrn<true>(b, lds, stream) : launch_lrn<false>(b, lds, stream);
}

hipError_t launch_event_loop(const LoopArgs &a, int precision, int refresh_full,
                             const Schedule &s, hipStream_t stream) {
  LoopArgs b = a;
  b.refresh_full = refresh_full;
  hipError_t e = launch_queue_reset(a.queue, stream);
  if (e != hipSuccess) return e;
  return precision == AKMC_FP32 ? launch_g<true>(b, s, stream) : launch_g<false>(b, s, stream);
}

}  // namespace akmc
