// correlate.hip — the correlator (Section 4, Eq. 3; Section 6.2.2) on the matrix cores.
//
// For one integration interval and one output channel the visibilities of all input pairs form
// R = X X^H, X the complex int8 voltages of the 2A inputs (antenna, polarisation) over the
// K = n_int n_favg (sample, fine channel) terms. With X = Xr + i Xi:
//   Re R = Xr Xr^T + Xi Xi^T,   Im R = Xi Xr^T - (Xr Xi^T),
// four real int8 products accumulated exactly in int32 by v_mfma_i32_32x32x32_i8 (|R| <=
// 2 K 128^2 < 2^31 for K <= 65535). Only the 32 x 32 tiles on or below the diagonal are
// formed. A workgroup owns up to 8 tiles of one (interval, channel) and keeps their
// accumulators in registers over all of K; K is staged through LDS in chunks of 64, transposed
// so that every input's 64 values are contiguous (the MFMA operands are 16 consecutive k of one
// input per lane).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"

namespace blink {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kTile = 32;                 // MFMA tile (inputs)
constexpr int kKc = 64;                   // k values per LDS chunk
constexpr int kRow = kKc + 16;            // LDS row stride in bytes (spreads rows over the banks)
constexpr int kTilesPerGroup = 8;         // tiles per workgroup (two per wave)
constexpr int kThreads = 256;

// Tile tau of the lower triangle in row order: (a, b), b <= a, tau = a (a + 1) / 2 + b.
__device__ __forceinline__ void tile_of(int tau, int& a, int& b) {
  int r = (int)((sqrt(8.0 * tau + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > tau) --r;
  while ((r + 1) * (r + 2) / 2 <= tau) ++r;
  a = r;
  b = tau - r * (r + 1) / 2;
}

__global__ __launch_bounds__(kThreads) void k_correlate(CorrelateArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int IP = a.n_slabs * kTile;               // padded input count
  unsigned char* xr = lds;                        // [IP][kRow]: real parts, k contiguous
  unsigned char* xi = lds + (size_t)IP * kRow;    // imaginary parts
  __shared__ unsigned s_need;                     // bit s: slab s is used by this workgroup

  const int group = blockIdx.x, c = blockIdx.y, t = blockIdx.z;
  const int ntiles = a.n_slabs * (a.n_slabs + 1) / 2;
  const int tau0 = group * kTilesPerGroup;
  const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
  const int n = lane % 32, g = lane / 32;
  // this wave's two tiles (tile index -1: none)
  int ta[2], tb[2], tv[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int tau = tau0 + wave * 2 + u;
    tv[u] = tau < ntiles;
    if (tv[u]) tile_of(tau, ta[u], tb[u]);
    else ta[u] = tb[u] = 0;
  }
  if (threadIdx.x == 0) {
    unsigned need = 0;
    for (int k = 0; k < kTilesPerGroup && tau0 + k < ntiles; ++k) {
      int x, y;
      tile_of(tau0 + k, x, y);
      need |= (1u << x) | (1u << y);
    }
    s_need = need;
  }

  v16i re[2], d1[2], d2[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) re[u] = d1[u] = d2[u] = v16i{};

  const int K = a.n_int * a.n_favg;
  const int in2 = 2 * a.A;                          // inputs (antenna, polarisation)
  const size_t rec = (size_t)in2 * 2;               // bytes per (sample, fine channel)
  __syncthreads();
  const unsigned need = s_need;
  for (int k0 = 0; k0 < K; k0 += kKc) {
    // Stage: item = (slab, 8-input vector v < 4, k quad q < 16). The thread reads the 16-byte
    // vector of 8 inputs (re, im) for k0 + 4q .. k0 + 4q + 3 and writes, for each input, four
    // consecutive k of the real and the imaginary plane.
    for (int item = threadIdx.x; item < a.n_slabs * 4 * (kKc / 4); item += kThreads) {
      const int slab = item / (4 * (kKc / 4)), rest = item % (4 * (kKc / 4));
      const int v = rest / (kKc / 4), q = rest % (kKc / 4);
      if (!((need >> slab) & 1u)) continue;
      const int row0 = slab * kTile + v * 8;
      uint32_t pr[8] = {0, 0, 0, 0, 0, 0, 0, 0}, pi[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (row0 < in2) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = k0 + 4 * q + e;
          if (k < K) {
            const int s = t * a.n_int + k / a.n_favg, f = c * a.n_favg + k % a.n_favg;
            const uint4 w = *reinterpret_cast<const uint4*>(a.volt + ((size_t)s * a.F + f) * rec + (size_t)row0 * 2);
            const uint32_t word[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int r = 0; r < 8; ++r) {
              const uint32_t h = (word[r / 2] >> (16 * (r % 2))) & 0xffffu;   // input row0 + r: re | im << 8
              pr[r] |= (h & 0xffu) << (8 * e);
              pi[r] |= (h >> 8) << (8 * e);
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        *reinterpret_cast<uint32_t*>(xr + (size_t)(row0 + r) * kRow + 4 * q) = pr[r];
        *reinterpret_cast<uint32_t*>(xi + (size_t)(row0 + r) * kRow + 4 * q) = pi[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (!tv[u]) continue;
      const unsigned char* ra = xr + (size_t)(ta[u] * kTile + n) * kRow;
      const unsigned char* ia = xi + (size_t)(ta[u] * kTile + n) * kRow;
      const unsigned char* rb = xr + (size_t)(tb[u] * kTile + n) * kRow;
      const unsigned char* ib = xi + (size_t)(tb[u] * kTile + n) * kRow;
#pragma unroll
      for (int kk = 0; kk < kKc; kk += 32) {
        const int off = kk + 16 * g;
        const v4i Ar = *reinterpret_cast<const v4i*>(ra + off), Ai = *reinterpret_cast<const v4i*>(ia + off);
        const v4i Br = *reinterpret_cast<const v4i*>(rb + off), Bi = *reinterpret_cast<const v4i*>(ib + off);
        re[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Ar, Br, re[u], 0, 0, 0);
        re[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Ai, Bi, re[u], 0, 0, 0);
        d1[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Ai, Br, d1[u], 0, 0, 0);
        d2[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Ar, Bi, d2[u], 0, 0, 0);
      }
    }
    __syncthreads();   // the chunk's operands are read before the next chunk overwrites them
  }

  // Output: element v of the lane is R[32 a + 8 (v / 4) + 4 g + v % 4][32 b + n].
  const double inv_count = (double)K;
  const long B = (long)a.A * (a.A - 1) / 2;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (!tv[u]) continue;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int ri = ta[u] * kTile + 8 * (v / 4) + 4 * g + v % 4, ci = tb[u] * kTile + n;
      if (ri >= in2 || ci >= in2) continue;
      const int i = ri / 2, p = ri % 2, j = ci / 2, q = ci % 2;
      if (i < j) continue;
      const float vr = (float)((double)re[u][v] / inv_count);
      const float vi = (float)(((double)d1[u][v] - (double)d2[u][v]) / inv_count);
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
  return (size_t)slabs * kTile * kRow * 2;
}

hipError_t launch_correlate(const CorrelateArgs& a, hipStream_t s) {
  const int T = a.S / a.n_int, C = a.F / a.n_favg;
  if (T == 0 || C == 0) return hipSuccess;
  const int ntiles = a.n_slabs * (a.n_slabs + 1) / 2;
  dim3 grid((unsigned)((ntiles + kTilesPerGroup - 1) / kTilesPerGroup), (unsigned)C, (unsigned)T);
  CorrelateArgs b = a;
  b.C = C;
  const size_t lds_bytes = correlate_lds_bytes(a.A);
  if (lds_bytes > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_correlate),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  k_correlate<<<grid, kThreads, lds_bytes, s>>>(b);
  return hipGetLastError();
}

}  // namespace blink
