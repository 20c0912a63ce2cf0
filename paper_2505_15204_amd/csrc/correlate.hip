// correlate.hip — the correlator (Section 4, Eq. 3; Section 6.2.2) on the matrix cores.
//
// For one integration interval and one output channel the visibilities of all input pairs form
// R = X X^H, X the complex int8 voltages of the 2A inputs (antenna, polarisation) over the
// K = n_int n_favg (sample, fine channel) terms. Each input's terms are kept as interleaved
// (re, im) byte pairs, so one int8 dot product over 2K bytes gives, for rows r and c,
//   (re, im)_r . (re, im)_c = sum Xr[r] Xr[c] + Xi[r] Xi[c]       = Re R[r][c]
//   (im, ~re)_r . (re, im)_c = sum Xi[r] Xr[c] + (~Xr[r]) Xi[c]  = Im R[r][c] - sum Xi[c]
// with ~x = -x - 1 the bitwise complement (exact in int8, unlike -x for x = -128); the per-input
// sum of Xi over K is added back at the end. Both byte layouts are staged in LDS (planes P and
// Q), so the products read their operands directly. Each 32 x 32 output tile therefore needs two
// int32 accumulators and two v_mfma_i32_32x32x32_i8 per 16 terms, all exact
// (|R| <= 2 K 128^2 < 2^31 for K <= 65535). Only the tiles on or below the diagonal are
// formed. A workgroup of 12 waves owns up to 36 tiles (three per wave, along tile rows so that a
// row's operands are read once per step) of one (interval, channel), all of them up to 128
// antennas, so every input is staged once, and keeps their accumulators in registers over all of
// K; K is staged through LDS in chunks of 64 terms (each input's 128 bytes contiguous), and the
// global loads of the next chunk are issued before the current chunk's matrix products.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"

namespace blink {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kTile = 32;                 // MFMA tile (inputs)
constexpr int kKc = 64;                   // terms per LDS chunk
constexpr int kRow = 2 * kKc + 16;        // LDS row stride in bytes (spreads rows over the banks)
constexpr int kTilesPerWave = 3;
constexpr int kWaves = 12;
constexpr int kTilesPerGroup = kTilesPerWave * kWaves;
constexpr int kThreads = 64 * kWaves;
constexpr int kOctets = kKc / 8;               // 8-term octets per chunk
constexpr int kItemsPerSlab = 4 * kOctets;     // (8-input group, 8-term octet) pairs per 32-input slab

// Tile tau of the lower triangle in row order: (a, b), b <= a, tau = a (a + 1) / 2 + b (at most
// 16 tile rows).
__device__ __forceinline__ void tile_of(int tau, int& a, int& b) {
  int r = 0;
  while ((r + 1) * (r + 2) / 2 <= tau) ++r;
  a = r;
  b = tau - r * (r + 1) / 2;
}

// x / K rounded once to float for an integer |x| < 2^31 and K <= 65535: the value of
// (float)((double)x / K). Write K = d 2^a with d odd. A quotient q = x / K that is a float
// rounding midpoint is a dyadic rational, so d divides x. Divisibility by d is one multiply by the
// inverse of d modulo 2^32: |x| dinv mod 2^32 <= (2^32 - 1) / d exactly when d divides |x|, and
// the product is then the exact quotient |x| / d, whose conversion to float (round to nearest
// even) times 2^-a is q correctly rounded. When d does not divide x, q is no midpoint and lies at
// least 2^-49 (relative) from every midpoint (a nonzero difference of fractions with denominators
// K and 2^e), while qd = x * (1/K in FP64) is within 2^-52 of q, so (float)qd rounds q correctly.
// Both ways are computed and one is selected, without branches.
struct MeanDiv {
  double inv;        // 1 / K rounded to double
  unsigned dinv;     // inverse of the odd part d of K modulo 2^32
  unsigned bound;    // (2^32 - 1) / d
  float scale;       // 2^-a
};

__device__ __forceinline__ MeanDiv mean_div(int K) {
  MeanDiv m;
  m.inv = 1.0 / (double)K;
  const int a = __builtin_ctz((unsigned)K);
  const unsigned d = (unsigned)K >> a;
  unsigned di = d;                                   // Newton's iteration doubles the correct bits
  for (int i = 0; i < 5; ++i) di *= 2u - d * di;
  m.dinv = di;
  m.bound = 0xffffffffu / d;
  m.scale = __uint_as_float((unsigned)(127 - a) << 23);
  return m;
}

__device__ __forceinline__ float mean_rn(int x, const MeanDiv& m) {
  const unsigned ax = x < 0 ? 0u - (unsigned)x : (unsigned)x;
  const unsigned t = ax * m.dinv;
  const float fq = (float)((double)x * m.inv);
  const float fe = __uint2float_rn(t) * m.scale;
  const float fd = x < 0 ? -fe : fe;
  return t <= m.bound ? fd : fq;
}

// One staging item: 16 bytes (8 inputs, re and im) for each of 8 consecutive terms.
struct Staged {
  uint4 w[8];
};

// A workgroup of 12 waves owns 36 tiles: every tile of one (interval, channel) up to 128 antennas
// (8 slabs), so each input is staged once per chunk; larger arrays take several workgroups. Each
// thread stages at most one item (n_slabs * kItemsPerSlab <= 512 items up to 256 antennas).
// With DB (two plane buffers, up to 8 slabs) the staging waves store chunk i + 1 into one buffer
// while every wave forms chunk i's products from the other: one barrier per chunk, and the other
// waves' matrix products cover the staging's byte permutes on each SIMD.
template <bool DB>
__global__ __launch_bounds__(kThreads, 1) void k_correlate(CorrelateArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int IP = a.n_slabs * kTile;               // padded input count
  const size_t plane = (size_t)IP * kRow;
  unsigned char* x0 = lds;                        // plane P [IP][kRow]: (re, im) pairs, terms contiguous
  unsigned char* xq0 = lds + plane;               // plane Q [IP][kRow]: (im, ~re) pairs
  unsigned char* x1 = DB ? lds + 2 * plane : x0;  // second buffer (DB)
  unsigned char* xq1 = DB ? lds + 3 * plane : xq0;
  int* colsum = reinterpret_cast<int*>(lds + (DB ? 4 : 2) * plane);   // [IP]: sum of Xi over K
  __shared__ unsigned s_need;                     // bit s: slab s is used by this workgroup

  // Workgroups are dispatched to the 8 XCDs in turn (workgroup w to XCD w % 8): the n_groups
  // workgroups of one (interval, channel) pair are w, w + 8, ..., so they share one XCD's L2 and
  // the voltages they all stage are read from HBM once.
  const long w = blockIdx.x, span = 8L * a.n_groups;
  const int group = (int)((w % span) / 8);
  const long pair = (w / span) * 8 + w % 8;
  if (pair >= (long)a.T * a.C) return;             // padding workgroups of the last span
  const int t = (int)(pair / a.C), c = (int)(pair % a.C);
  const int ntiles = a.n_slabs * (a.n_slabs + 1) / 2;
  const int tau0 = group * kTilesPerGroup;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64), lane = (int)threadIdx.x % 64;
  const int n = lane % 32, g = lane / 32;
  int ta[kTilesPerWave], tb[kTilesPerWave], tv[kTilesPerWave];
#pragma unroll
  for (int u = 0; u < kTilesPerWave; ++u) {
    const int tau = tau0 + wave * kTilesPerWave + u;
    tv[u] = tau < ntiles;
    if (tv[u]) tile_of(tau, ta[u], tb[u]);
    else ta[u] = tb[u] = 0;
  }
  for (int i = threadIdx.x; i < IP; i += kThreads) colsum[i] = 0;
  if (threadIdx.x == 0) {
    unsigned need = 0;
    for (int k = 0; k < kTilesPerGroup && tau0 + k < ntiles; ++k) {
      int y, z;
      tile_of(tau0 + k, y, z);
      need |= (1u << y) | (1u << z);
    }
    s_need = need;
  }

  v16i re[kTilesPerWave], im[kTilesPerWave];
#pragma unroll
  for (int u = 0; u < kTilesPerWave; ++u) re[u] = im[u] = v16i{};

  const int K = a.n_int * a.n_favg;
  const int in2 = 2 * a.A;                          // inputs (antenna, polarisation)
  const size_t rec = (size_t)in2 * 2;               // bytes per (sample, fine channel)
  const int n_items = a.n_slabs * kItemsPerSlab;
  __syncthreads();
  const unsigned need = s_need;

  // item -> (8-input group rg, term octet o): consecutive items are the 8 octets of one input
  // group, so a global load of a wave reads 128-byte runs (8 groups) of 8 records, and the LDS
  // rows are stored without a swizzle: with the 144-byte row stride (9 16-byte slots) the 16
  // lanes of one LDS cycle write rows r and r + 8 of their groups at octets 0..7, slots 9 row + o,
  // all distinct modulo 16, and the operand reads (16 consecutive rows, one octet) are distinct too
  const int item = (int)threadIdx.x;
  const int o = item % kOctets, rg = item / kOctets, row0 = rg * 8, slab = rg / 4;
  const bool staged = item < n_items && ((need >> slab) & 1u);   // this thread writes rows of P, Q
  const bool on = staged && row0 < in2;                           // ... and loads voltages for them
  // global loads of one chunk's item of this thread (unused slabs, inputs past 2A and terms past K
  // are not loaded and stage zeros). Term k is (sample k / n_favg, fine channel k % n_favg) of the
  // block; one division per chunk.
  auto load = [&](int k0, Staged& st) {
    const int kb = k0 + 8 * o;
    int sl = kb / a.n_favg, fl = kb - sl * a.n_favg;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      st.w[e] = make_uint4(0, 0, 0, 0);
      if (on && kb + e < K) {
        const size_t at = ((size_t)(t * a.n_int + sl) * a.F + (size_t)(c * a.n_favg + fl)) * rec + (size_t)row0 * 2;
        st.w[e] = *reinterpret_cast<const uint4*>(a.volt + at);
      }
      if (++fl == a.n_favg) {
        fl = 0;
        ++sl;
      }
    }
  };
  // transpose: row row0 + r gets the (re, im) pairs of its 8 terms as one 16-byte vector in P and
  // the (im, ~re) pairs in Q (byte permutes of two loaded words each); the chunk's imaginary parts
  // of each row are added to colsum
  auto store = [&](const Staged& st, unsigned char* x, unsigned char* xq) {
    if (staged) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        // v_perm_b32 byte selectors (0-3: bytes of the second source, 4-7: of the first): row r's
        // (re, im) pair is bytes j, j + 1 of its word, j = 2 (r % 2)
        const unsigned j = 2u * (r % 2);
        const unsigned sel_p = j | (j + 1) << 8 | (j + 4) << 16 | (j + 5) << 24;
        const unsigned sel_q = (j + 1) | j << 8 | (j + 5) << 16 | (j + 4) << 24;
        unsigned d[4], e[4];
        int isum = 0;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const uint4& w0 = st.w[2 * h];
          const uint4& w1 = st.w[2 * h + 1];
          const unsigned a0 = r < 2 ? w0.x : r < 4 ? w0.y : r < 6 ? w0.z : w0.w;
          const unsigned a1 = r < 2 ? w1.x : r < 4 ? w1.y : r < 6 ? w1.z : w1.w;
          d[h] = __builtin_amdgcn_perm(a1, a0, sel_p);                 // (re, im) of terms 2h, 2h + 1
          e[h] = __builtin_amdgcn_perm(a1, a0, sel_q) ^ 0xff00ff00u;   // (im, ~re)
          isum = __builtin_amdgcn_sdot4((int)d[h], 0x01000100, isum, false);   // the two im bytes
        }
        const size_t at = (size_t)(row0 + r) * kRow + 16 * o;
        *reinterpret_cast<uint4*>(x + at) = make_uint4(d[0], d[1], d[2], d[3]);
        *reinterpret_cast<uint4*>(xq + at) = make_uint4(e[0], e[1], e[2], e[3]);
        if (isum) atomicAdd(&colsum[row0 + r], isum);
      }
    }
  };

  // the products of one staged chunk: the wave's tiles run along tile rows (row order), so the
  // row operands A and As are read once per tile row and step and reused by the following tiles
  // of that row
  auto products = [&](const unsigned char* x, const unsigned char* xq) {
#pragma unroll
    for (int kk = 0; kk < 2 * kKc; kk += 32) {
      const int q = kk / 16 + g;                    // this lane's term octet of the step
      v4i A = {}, As = {};
      int cur = -1;
#pragma unroll
      for (int u = 0; u < kTilesPerWave; ++u) {
        if (!tv[u]) continue;
        if (ta[u] != cur) {
          cur = ta[u];
          const int rowa = cur * kTile + n;
          const size_t oa = (size_t)rowa * kRow + 16 * q;
          A = *reinterpret_cast<const v4i*>(x + oa);
          As = *reinterpret_cast<const v4i*>(xq + oa);
        }
        const int rowb = tb[u] * kTile + n;
        const v4i B = *reinterpret_cast<const v4i*>(x + (size_t)rowb * kRow + 16 * q);
        re[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B, re[u], 0, 0, 0);
        im[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(As, B, im[u], 0, 0, 0);
      }
    }
  };
  Staged st;
  load(0, st);
  if constexpr (DB) {
    // chunk i + 1 (loaded during chunk i - 1) is stored into the free buffer and chunk i + 2
    // requested before chunk i's products; the barrier closes both the products' reads of one
    // buffer and the stores into the other
    store(st, x0, xq0);
    if (kKc < K) load(kKc, st);
    __syncthreads();
    int i = 0;
    for (int k0 = 0; k0 < K; k0 += kKc, ++i) {
      if (k0 + kKc < K) {
        store(st, (i & 1) ? x0 : x1, (i & 1) ? xq0 : xq1);
        if (k0 + 2 * kKc < K) load(k0 + 2 * kKc, st);
      }
      products((i & 1) ? x1 : x0, (i & 1) ? xq1 : xq0);
      __syncthreads();
    }
  } else {
    // one buffer: stage the registers into LDS, request the next chunk (answered during this
    // chunk's products), then the products
    for (int k0 = 0; k0 < K; k0 += kKc) {
      store(st, x0, xq0);
      __syncthreads();
      if (k0 + kKc < K) load(k0 + kKc, st);
      products(x0, xq0);
      __syncthreads();   // the chunk's operands are read before the next chunk overwrites them
    }
  }

  // Output: element v of the lane is R[32 a + 8 (v / 4) + 4 g + v % 4][32 b + n].
  const MeanDiv md = mean_div(K);
  const long B = (long)a.A * (a.A - 1) / 2;
#pragma unroll
  for (int u = 0; u < kTilesPerWave; ++u) {
    if (!tv[u]) continue;
    const int ci = tb[u] * kTile + n;
    const int csum = ci < in2 ? colsum[ci] : 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int ri = ta[u] * kTile + 8 * (v / 4) + 4 * g + v % 4;
      if (ri >= in2 || ci >= in2) continue;
      const int i = ri / 2, p = ri % 2, j = ci / 2, q = ci % 2;
      if (i < j) continue;
      // Im R = im + csum fits in int32 (|R| <= 2 K 128^2 < 2^31); the sum is formed modulo 2^32
      const float vr = mean_rn(re[u][v], md);
      const float vi = mean_rn((int)((unsigned)im[u][v] + (unsigned)csum), md);
      if (i == j) {
        if (a.autos) a.autos[(((size_t)t * a.C + c) * a.A + i) * 4 + 2 * p + q] = make_float2(vr, vi);
        continue;
      }
      int pp;
      if (a.pol_mode == 4) pp = 2 * p + q;
      else if (p == q) pp = p;
      else continue;
      const long b = (long)i * (i - 1) / 2 + j;
      a.vis[(((size_t)t * a.C + c) * a.pol_mode + pp) * B + b] = make_float2(vr, vi);
    }
  }
}

}  // namespace

// Two plane buffers when they fit the 160 KB of LDS (up to 8 slabs, 128 antennas), else one.
static bool correlate_db(int slabs) { return (size_t)slabs * kTile * (4 * kRow + sizeof(int)) <= 160 * 1024; }

size_t correlate_lds_bytes(int A) {
  const int slabs = (2 * A + kTile - 1) / kTile;
  return (size_t)slabs * kTile * ((correlate_db(slabs) ? 4 : 2) * kRow + sizeof(int));
}

hipError_t launch_correlate(const CorrelateArgs& a, hipStream_t s) {
  const int T = a.S / a.n_int, C = a.F / a.n_favg;
  if (T == 0 || C == 0) return hipSuccess;
  const int ntiles = a.n_slabs * (a.n_slabs + 1) / 2;
  const int n_groups = (ntiles + kTilesPerGroup - 1) / kTilesPerGroup;
  const long n_wg = 8L * n_groups * (((long)T * C + 7) / 8);
  if (n_wg > 0x7fffffffL) return hipErrorInvalidValue;
  CorrelateArgs b = a;
  b.C = C;
  b.T = T;
  b.n_groups = n_groups;
  const unsigned grid = (unsigned)n_wg;
  const size_t lds_bytes = correlate_lds_bytes(a.A);
  if (a.n_slabs * kItemsPerSlab > kThreads) return hipErrorInvalidValue;   // one item per thread
  const bool db = correlate_db(a.n_slabs);
  const void* fn = db ? reinterpret_cast<const void*>(k_correlate<true>)
                      : reinterpret_cast<const void*>(k_correlate<false>);
  if (lds_bytes > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  if (db) k_correlate<true><<<grid, kThreads, lds_bytes, s>>>(b);
  else k_correlate<false><<<grid, kThreads, lds_bytes, s>>>(b);
  return hipGetLastError();
}

}  // namespace blink
