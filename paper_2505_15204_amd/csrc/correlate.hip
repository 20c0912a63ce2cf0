// correlate.hip — the correlator (Section 4, Eq. 3; Section 6.2.2) on the matrix cores.
//
// For one integration interval and one output channel the visibilities of all input pairs form
// R = X X^H, X the complex int8 voltages of the 2A inputs (antenna, polarisation) over the
// K = n_int n_favg (sample, fine channel) terms. Each input's terms are kept as interleaved
// (re, im) byte pairs, so one int8 dot product over 2K bytes gives, for rows r and c,
//   (re, im)_r . (re, im)_c = sum Xr[r] Xr[c] + Xi[r] Xi[c]       = Re R[r][c]
//   (im, ~re)_r . (re, im)_c = sum Xi[r] Xr[c] + (~Xr[r]) Xi[c]  = Im R[r][c] - sum Xi[c]
// with ~x = -x - 1 the bitwise complement (exact in int8, unlike -x for x = -128); the per-input
// sum of Xi over K is added back at the end. Each 32 x 32 output tile therefore needs two
// int32 accumulators and two v_mfma_i32_32x32x32_i8 per 16 terms, all exact
// (|R| <= 2 K 128^2 < 2^31 for K <= 65535). Only the tiles on or below the diagonal are
// formed. A workgroup owns up to 12 tiles (three per wave) of one (interval, channel) and keeps
// their accumulators in registers over all of K; K is staged through LDS in chunks of 64 terms
// (each input's 128 bytes contiguous), and the global loads of the next chunk are issued before
// the current chunk's matrix products.
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
constexpr int kWaves = 4;
constexpr int kTilesPerGroup = kTilesPerWave * kWaves;
constexpr int kThreads = 64 * kWaves;
constexpr int kItemsPerSlab = 4 * (kKc / 8);   // (8-input group, 8-term octet) pairs per 32-input slab

// Tile tau of the lower triangle in row order: (a, b), b <= a, tau = a (a + 1) / 2 + b.
__device__ __forceinline__ void tile_of(int tau, int& a, int& b) {
  int r = (int)((sqrt(8.0 * tau + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > tau) --r;
  while ((r + 1) * (r + 2) / 2 <= tau) ++r;
  a = r;
  b = tau - r * (r + 1) / 2;
}

// (re, im) byte pairs -> (im, ~re)
__device__ __forceinline__ int swap_complement(int x) {
  const unsigned u = (unsigned)x;
  return (int)(((u >> 8) & 0x00ff00ffu) | ((~u << 8) & 0xff00ff00u));
}

// One staging item: 16 bytes (8 inputs, re and im) for each of 8 consecutive terms.
struct Staged {
  uint4 w[8];
};

// ITEMS: staging items per thread, n_slabs * kItemsPerSlab / kThreads rounded up (1 for up to 128
// antennas, 2 for up to 256).
template <int ITEMS>
__global__ __launch_bounds__(kThreads, 2) void k_correlate(CorrelateArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int IP = a.n_slabs * kTile;               // padded input count
  unsigned char* x = lds;                         // [IP][kRow]: (re, im) pairs, terms contiguous
  int* colsum = reinterpret_cast<int*>(lds + (size_t)IP * kRow);   // [IP]: sum of Xi over K
  __shared__ unsigned s_need;                     // bit s: slab s is used by this workgroup

  const int group = blockIdx.x, c = blockIdx.y, t = blockIdx.z;
  const int ntiles = a.n_slabs * (a.n_slabs + 1) / 2;
  const int tau0 = group * kTilesPerGroup;
  const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
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

  // item -> (slab, 8-input group v < 4, term octet o < kKc / 8)
  auto item_rows = [&](int item, int& slab, int& row0, int& o) {
    slab = item / kItemsPerSlab;
    const int rest = item % kItemsPerSlab;
    row0 = slab * kTile + (rest / (kKc / 8)) * 8;
    o = rest % (kKc / 8);
  };
  // global loads of one chunk's items of this thread (unused slabs, inputs past 2A and terms
  // past K are not loaded and stage zeros)
  auto load = [&](int k0, Staged (&st)[ITEMS]) {
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
      const int item = (int)threadIdx.x + m * kThreads;
      int slab, row0, o;
      item_rows(item, slab, row0, o);
      const bool on = item < n_items && ((need >> slab) & 1u) && row0 < in2;
      // term k = (sample k / n_favg, fine channel k % n_favg) of the block; one division per item
      const int kb = k0 + 8 * o;
      int sl = kb / a.n_favg, fl = kb - sl * a.n_favg;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        st[m].w[e] = make_uint4(0, 0, 0, 0);
        if (on && kb + e < K) {
          const size_t at = ((size_t)(t * a.n_int + sl) * a.F + (size_t)(c * a.n_favg + fl)) * rec + (size_t)row0 * 2;
          st[m].w[e] = *reinterpret_cast<const uint4*>(a.volt + at);
        }
        if (++fl == a.n_favg) {
          fl = 0;
          ++sl;
        }
      }
    }
  };
  // transpose: row row0 + r gets the (re, im) pairs of its 8 terms as one 16-byte vector; the
  // imaginary parts are summed per row in registers (a thread stages the same rows every chunk)
  int isums[ITEMS][8];
#pragma unroll
  for (int m = 0; m < ITEMS; ++m)
#pragma unroll
    for (int r = 0; r < 8; ++r) isums[m][r] = 0;
  auto store = [&](const Staged (&st)[ITEMS]) {
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
      const int item = (int)threadIdx.x + m * kThreads;
      int slab, row0, o;
      item_rows(item, slab, row0, o);
      if (!(item < n_items && ((need >> slab) & 1u))) continue;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        unsigned d[4];
        int isum = isums[m][r];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const uint4& w0 = st[m].w[2 * h];
          const uint4& w1 = st[m].w[2 * h + 1];
          const unsigned a0 = r < 2 ? w0.x : r < 4 ? w0.y : r < 6 ? w0.z : w0.w;
          const unsigned a1 = r < 2 ? w1.x : r < 4 ? w1.y : r < 6 ? w1.z : w1.w;
          const unsigned sh = 16 * (r % 2);
          d[h] = ((a0 >> sh) & 0xffffu) | (((a1 >> sh) & 0xffffu) << 16);
          isum = __builtin_amdgcn_sdot4((int)d[h], 0x01000100, isum, false);   // the two im bytes
        }
        *reinterpret_cast<uint4*>(x + (size_t)(row0 + r) * kRow + 16 * o) = make_uint4(d[0], d[1], d[2], d[3]);
        isums[m][r] = isum;
      }
    }
  };

  Staged st[ITEMS];
  load(0, st);
  for (int k0 = 0; k0 < K; k0 += kKc) {
    store(st);
    __syncthreads();
    if (k0 + kKc < K) load(k0 + kKc, st);          // answered during this chunk's products
#pragma unroll
    for (int u = 0; u < kTilesPerWave; ++u) {
      if (!tv[u]) continue;
      const unsigned char* pa = x + (size_t)(ta[u] * kTile + n) * kRow + 16 * g;
      const unsigned char* pb = x + (size_t)(tb[u] * kTile + n) * kRow + 16 * g;
#pragma unroll
      for (int kk = 0; kk < 2 * kKc; kk += 32) {
        const v4i A = *reinterpret_cast<const v4i*>(pa + kk);
        const v4i B = *reinterpret_cast<const v4i*>(pb + kk);
        v4i As;
        As.x = swap_complement(A.x);
        As.y = swap_complement(A.y);
        As.z = swap_complement(A.z);
        As.w = swap_complement(A.w);
        re[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B, re[u], 0, 0, 0);
        im[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(As, B, im[u], 0, 0, 0);
      }
    }
    __syncthreads();   // the chunk's operands are read before the next chunk overwrites them
  }
#pragma unroll
  for (int m = 0; m < ITEMS; ++m) {
    const int item = (int)threadIdx.x + m * kThreads;
    int slab, row0, o;
    item_rows(item, slab, row0, o);
    if (!(item < n_items && ((need >> slab) & 1u))) continue;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (isums[m][r]) atomicAdd(&colsum[row0 + r], isums[m][r]);
  }
  __syncthreads();

  // Output: element v of the lane is R[32 a + 8 (v / 4) + 4 g + v % 4][32 b + n].
  const double count = (double)K;
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
      const float vr = (float)((double)re[u][v] / count);
      const float vi = (float)(((double)im[u][v] + (double)csum) / count);
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

size_t correlate_lds_bytes(int A) {
  const int slabs = (2 * A + kTile - 1) / kTile;
  return (size_t)slabs * kTile * (kRow + sizeof(int));
}

hipError_t launch_correlate(const CorrelateArgs& a, hipStream_t s) {
  const int T = a.S / a.n_int, C = a.F / a.n_favg;
  if (T == 0 || C == 0) return hipSuccess;
  const int ntiles = a.n_slabs * (a.n_slabs + 1) / 2;
  dim3 grid((unsigned)((ntiles + kTilesPerGroup - 1) / kTilesPerGroup), (unsigned)C, (unsigned)T);
  CorrelateArgs b = a;
  b.C = C;
  const size_t lds_bytes = correlate_lds_bytes(a.A);
  const int items = (a.n_slabs * kItemsPerSlab + kThreads - 1) / kThreads;
  const void* fn = items <= 1 ? reinterpret_cast<const void*>(k_correlate<1>)
                              : reinterpret_cast<const void*>(k_correlate<2>);
  if (items > 2) return hipErrorInvalidValue;
  if (lds_bytes > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  if (items <= 1) k_correlate<1><<<grid, kThreads, lds_bytes, s>>>(b);
  else k_correlate<2><<<grid, kThreads, lds_bytes, s>>>(b);
  return hipGetLastError();
}

}  // namespace blink
