// api.hip — C ABI of libblink.so (declared in include/blink.h): argument checks, workspace
// layout, chunking over (time, channel) pairs and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "blink.h"
#include "launch.hpp"

constexpr int kPrecForms = 3;   // BLINK_PREC_FP32, BLINK_PREC_SPLIT_F16, BLINK_PREC_SPLIT_BF16

// Scratch memory of blink_image_batch_noalloc: a fixed device array, so that the call allocates
// nothing. Each device holds its own copy (at its own address) once the library's code is loaded
// there. Host code never uses this name as a device address: blink_create looks the address up on
// its device (hipGetSymbolAddress) and keeps it in the context.
static __device__ __align__(256) unsigned char scratch[BLINK_STATIC_SCRATCH_BYTES];

struct blink_ctx_s {
  int device = 0;
  float2* tw_base = nullptr;      // stage-ordered twiddle tables for N = 8 .. 4096, concatenated,
                                  // then the split forms' DFT operand table
  float2* tw[13] = {};
  const uint4* dft_ops = nullptr;
  void* scratch = nullptr;        // this device's copy of the static scratch array
  bool broken = false;
  std::string err;
  // execution plan per (log2 N, weighting, precision form): fused-kernel strip width, row
  // transforms per workgroup, images per column/row launch pair (0 = as many as the workspace holds)
  struct Plan {
    int col_strip = 0, row_tpb = 0, group = 0, col_loop = 1;
  } plan[13][2][kPrecForms];
  // descriptor-path plan (blink_set_desc_plan) and device facts
  int desc_block = 512, desc_workgroups = 0, desc_form = BLINK_DESC_STAGED;
  int cu_count = 0;
  // kernel timing (blink_profile_enable)
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> records[BLINK_KERNEL_COUNT];
  std::vector<hipEvent_t> spare;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool valid_precision(int p) { return p >= 0 && p < kPrecForms; }

int log2_exact(int n) {
  if (n < BLINK_MIN_GRID || n > BLINK_MAX_GRID || (n & (n - 1))) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

blink_status fail(blink_ctx ctx, blink_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

blink_status hip_fail(blink_ctx ctx, hipError_t e, const char* where) {
  if (ctx) ctx->broken = true;
  return fail(ctx, BLINK_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

// Sets the context's device for the duration of a call and restores the caller's.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

hipEvent_t take_event(blink_ctx ctx) {
  if (!ctx->spare.empty()) {
    hipEvent_t e = ctx->spare.back();
    ctx->spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void release_records(blink_ctx ctx) {
  for (auto& v : ctx->records) {
    for (auto& pr : v) {
      ctx->spare.push_back(pr.first);
      ctx->spare.push_back(pr.second);
    }
    v.clear();
  }
}

// Brackets one kernel launch with events when timing is enabled.
struct KernelTimer {
  blink_ctx ctx;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  KernelTimer(blink_ctx c, int k, hipStream_t st) : ctx(c), kind(k), s(st) {
    if (!ctx->profiling) return;
    a = take_event(ctx);
    b = take_event(ctx);
    if (a && b) (void)hipEventRecord(a, s);
  }
  ~KernelTimer() {
    if (!a || !b) return;
    (void)hipEventRecord(b, s);
    ctx->records[kind].emplace_back(a, b);
  }
};

bool mul_ok(size_t a, size_t b, size_t* out) {
  if (a != 0 && b > SIZE_MAX / a) return false;
  *out = a * b;
  return true;
}

// ---------------------------------------------------------------- workspace layouts
struct Carve {
  size_t off = 0;
  bool ok = true;
  size_t take(size_t count, size_t elem) {
    size_t bytes;
    if (!mul_ok(count, elem, &bytes)) ok = false;
    size_t at = off;
    off = align_up(off + (ok ? bytes : 0));
    return at;
  }
};

struct BinLayout {
  size_t plc, off, kept, occ, ext = 0;   // ext: column extent per pair (fused path)
};

BinLayout carve_bins(Carve& c, size_t Q, size_t P, size_t B, size_t nstrips) {
  BinLayout L;
  L.plc = c.take(Q, 2 * B * sizeof(int2));
  L.off = c.take(Q, (nstrips + 1) * sizeof(int));
  L.kept = c.take(Q, sizeof(int));
  L.occ = c.take(Q, P * sizeof(int));
  L.ext = c.take(Q, sizeof(int));
  return L;
}

struct ImageLayout {
  BinLayout bins;
  size_t H, vc, total;   // vc: corrected visibilities of a chunk (blink_image_batch_corrected)
  bool ok;
};

// The fused path keeps at most kMaxGroupImages half-spectrum intermediates per launch pair
// unless a plan asks for more.
constexpr size_t kMaxGroupImages = 256;
// Largest number of strips one workgroup of the fused column kernel takes in turn (plan col_loop).
constexpr int kMaxColLoop = 64;

int min_col_strip(int logn, int uniform) {
  int opts[4];
  int n = blink::col_strip_options(logn, uniform != 0, opts);
  return n > 0 ? opts[n - 1] : 1;
}

ImageLayout image_layout(size_t Q, int P, int B, int logn, int uniform, size_t h_images, bool corrected = false) {
  const size_t N = size_t(1) << logn;
  const size_t nstrips = (N / 2) / min_col_strip(logn, uniform);
  Carve c;
  ImageLayout L;
  L.bins = carve_bins(c, Q, P, B, nstrips);
  L.H = c.take(h_images, N * (N / 2) * sizeof(float2));
  L.vc = corrected ? c.take(Q * (size_t)P, (size_t)B * sizeof(float2)) : 0;
  L.total = c.off;
  L.ok = c.ok;
  return L;
}

// Convolutional path: records of the strips each placement reaches, the grid-correction table and
// the intermediates.
struct ConvLayout {
  BinLayout bins;
  size_t corr, H, total;
  int rec_stride;
  bool ok;
};

ConvLayout conv_layout(size_t Q, int P, int B, int logn, int width, size_t h_images) {
  const size_t N = size_t(1) << logn;
  const int S = blink::conv_strip_width(logn);
  ConvLayout L;
  L.rec_stride = blink::conv_records_per_pair(B, width, S, logn);
  Carve c;
  L.bins.plc = c.take(Q, (size_t)L.rec_stride * 16);
  L.bins.off = c.take(Q, ((size_t)blink::conv_bins_per_pair(logn, S) + 1) * sizeof(int));
  L.bins.kept = c.take(Q, sizeof(int));
  L.bins.occ = c.take(Q, (size_t)P * sizeof(int));
  L.bins.ext = c.take(Q, sizeof(int));
  L.corr = c.take(N, sizeof(float));
  L.H = c.take(h_images, N * (N / 2) * sizeof(float2));
  L.total = c.off;
  L.ok = c.ok;
  return L;
}

bool conv_args_ok(int width, double beta, int logn) {
  return width >= 1 && width <= 16 && 2 * width < (1 << logn) && beta >= 0.0 && std::isfinite(beta) && beta <= 100.0;
}

struct GridLayout {
  BinLayout bins;
  size_t total;
  bool ok;
};

GridLayout grid_layout(size_t Q, int P, int B, int logn) {
  const size_t N = size_t(1) << logn;
  const size_t nstrips = N / blink::grid_strip_width(logn);
  Carve c;
  GridLayout L;
  L.bins = carve_bins(c, Q, P, B, nstrips);
  L.total = c.off;
  L.ok = c.ok;
  return L;
}

struct FftLayout {
  size_t H, total;
  bool ok;
};

FftLayout fft_layout(size_t n_img, int logn) {
  const size_t N = size_t(1) << logn;
  Carve c;
  FftLayout L;
  L.H = c.take(n_img, N * (N / 2) * sizeof(float2));
  L.total = c.off;
  L.ok = c.ok;
  return L;
}

template <class F>
size_t largest_fitting_chunk(size_t n_tc, size_t ws_bytes, F total_for) {
  // total_for(Q) is increasing in Q; find the largest Q <= n_tc that fits.
  size_t lo = 0, hi = n_tc;
  while (lo < hi) {
    size_t mid = lo + (hi - lo + 1) / 2;
    if (total_for(mid) <= ws_bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Shared argument checks of blink_grid and blink_image_batch. Order: sizes, enums, ctx, pointers.
blink_status check_problem(blink_ctx ctx, const void* vis, const void* uvw, const void* freq, int T,
                           int C, int P, int B, int grid_n, double pixel_scale, int weighting,
                           const void* out, void* ws, int* logn) {
  if (T < 0 || C < 0 || P < 1 || B < 0)
    return fail(ctx, BLINK_ERR_ARG, "negative size (T=%d C=%d P=%d B=%d) or P < 1", T, C, P, B);
  if (B > (1 << 30)) return fail(ctx, BLINK_ERR_SIZE, "B=%d exceeds 2^30 baselines", B);
  *logn = log2_exact(grid_n);
  if (*logn < 0)
    return fail(ctx, BLINK_ERR_SIZE, "grid_n=%d is not a power of two in [%d, %d]", grid_n,
                BLINK_MIN_GRID, BLINK_MAX_GRID);
  if (weighting != BLINK_WEIGHT_NATURAL && weighting != BLINK_WEIGHT_UNIFORM)
    return fail(ctx, BLINK_ERR_ARG, "unknown weighting %d", weighting);
  if (!(pixel_scale > 0.0) || !std::isfinite(pixel_scale))
    return fail(ctx, BLINK_ERR_ARG, "pixel_scale must be finite and > 0");
  if (!ctx) return BLINK_ERR_ARG;
  if (ctx->broken) return fail(ctx, BLINK_ERR_STATE, "context unusable after an earlier HIP error");
  const bool empty = (size_t)T * C == 0;
  if (!empty && (!vis && B > 0)) return fail(ctx, BLINK_ERR_ARG, "vis is NULL");
  if (!empty && (!uvw && B > 0)) return fail(ctx, BLINK_ERR_ARG, "uvw_m is NULL");
  if (!empty && !freq) return fail(ctx, BLINK_ERR_ARG, "freq_hz is NULL");
  if (!empty && !out) return fail(ctx, BLINK_ERR_ARG, "output array is NULL");
  if (!empty && !ws) return fail(ctx, BLINK_ERR_ARG, "workspace is NULL");
  if ((uintptr_t)ws % kAlign) return fail(ctx, BLINK_ERR_ARG, "workspace is not 256-byte aligned");
  return BLINK_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

int blink_version(void) { return 100; }

const char* blink_status_string(blink_status s) {
  switch (s) {
    case BLINK_OK: return "ok";
    case BLINK_ERR_ARG: return "invalid argument";
    case BLINK_ERR_SIZE: return "unsupported size or workspace too small";
    case BLINK_ERR_NOMEM: return "out of memory";
    case BLINK_ERR_HIP: return "HIP runtime error";
    case BLINK_ERR_STATE: return "context unusable";
  }
  return "unknown status";
}

const char* blink_last_error(blink_ctx ctx) {
  if (!ctx) return "no context";
  return ctx->err.c_str();
}

blink_status blink_create(blink_ctx* out, int hip_device) {
  if (!out) return BLINK_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return BLINK_ERR_HIP;
  if (hip_device < 0 || hip_device >= count) return BLINK_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return BLINK_ERR_HIP;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BLINK_ERR_HIP;
  blink_ctx ctx = new (std::nothrow) blink_ctx_s;
  if (!ctx) return BLINK_ERR_NOMEM;
  ctx->device = hip_device;
  ctx->cu_count = prop.multiProcessorCount;
  DeviceGuard g(hip_device);
  if (g.err != hipSuccess) {
    delete ctx;
    return BLINK_ERR_HIP;
  }
  {
    void* sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
      delete ctx;
      return BLINK_ERR_HIP;
    }
    ctx->scratch = sp;
  }
  size_t total = 0;
  for (int l = 3; l <= 12; ++l) total += (size_t)blink::twiddle_table_size(l);
  const size_t ops_off = (total + 1) / 2 * 2;     // 16-byte aligned (float2 units)
  total = ops_off + (size_t)blink::kDftOpsCount * 2;
  if (hipMalloc(&ctx->tw_base, total * sizeof(float2)) != hipSuccess) {
    delete ctx;
    return BLINK_ERR_NOMEM;
  }
  size_t off = 0;
  hipError_t e = hipSuccess;
  for (int l = 3; l <= 12 && e == hipSuccess; ++l) {
    ctx->tw[l] = ctx->tw_base + off;
    e = blink::launch_twiddles(ctx->tw[l], l, nullptr);
    off += (size_t)blink::twiddle_table_size(l);
  }
  ctx->dft_ops = (const uint4*)(ctx->tw_base + ops_off);
  if (e == hipSuccess) e = blink::launch_dft_operands(ctx->tw[4], (uint4*)(ctx->tw_base + ops_off), nullptr);
  for (int l = 3; l <= 12; ++l) {
    for (int u = 0; u < 2; ++u) {
      int col[4], row[4];
      blink::col_strip_options(l, u != 0, col);
      int nr = blink::row_block_options(l, row);
      // default: the widest strip, and the row block closest to 256 threads
      int t = (1 << l) / 16 > 0 ? (1 << l) / 16 : 1;
      int best = row[0];
      for (int i = 0; i < nr; ++i)
        if (row[i] * t <= 256) { best = row[i]; break; }
      for (int pf = 0; pf < kPrecForms; ++pf) {
        ctx->plan[l][u][pf].col_strip = col[0];
        ctx->plan[l][u][pf].row_tpb = best;
        ctx->plan[l][u][pf].group = 0;
        ctx->plan[l][u][pf].col_loop = 1;
      }
    }
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(ctx->tw_base);
    delete ctx;
    return BLINK_ERR_HIP;
  }
  *out = ctx;
  return BLINK_OK;
}

blink_status blink_destroy(blink_ctx ctx) {
  if (!ctx) return BLINK_OK;
  {
    DeviceGuard g(ctx->device);
    if (ctx->tw_base) (void)hipFree(ctx->tw_base);
    release_records(ctx);
    for (hipEvent_t e : ctx->spare) (void)hipEventDestroy(e);
  }
  delete ctx;
  return BLINK_OK;
}

blink_status blink_grid_workspace_size(int T, int C, int B, int grid_n, size_t* bytes) {
  if (!bytes || T < 0 || C < 0 || B < 0) return BLINK_ERR_ARG;
  const int logn = log2_exact(grid_n);
  if (logn < 0) return BLINK_ERR_SIZE;
  // P only sizes the small occupancy array; the maximum supported polarisation count is 4.
  GridLayout L = grid_layout((size_t)T * C, 4, B, logn);
  if (!L.ok) return BLINK_ERR_SIZE;
  *bytes = L.total;
  return BLINK_OK;
}

blink_status blink_workspace_size(blink_ctx, const blink_problem* p, size_t* bytes) {
  if (!p || !bytes) return BLINK_ERR_ARG;
  switch (p->entry) {
    case BLINK_ENTRY_GRID: return blink_grid_workspace_size(p->T, p->C, p->B, p->grid_n, bytes);
    case BLINK_ENTRY_IFFT2D: return blink_ifft2d_workspace_size(p->n_img, p->grid_n, p->precision, bytes);
    case BLINK_ENTRY_IMAGE_BATCH:
      return blink_image_batch_workspace_size(p->T, p->C, p->P, p->B, p->grid_n, p->weighting, p->precision, bytes);
    case BLINK_ENTRY_IMAGE_BATCH_CORRECTED:
      return blink_image_batch_corrected_workspace_size(p->T, p->C, p->P, p->B, p->grid_n, p->weighting,
                                                        p->precision, bytes);
    case BLINK_ENTRY_IMAGE_BATCH_CONV:
      return blink_image_batch_conv_workspace_size(p->T, p->C, p->P, p->B, p->grid_n, p->kernel_width,
                                                   p->precision, bytes);
    case BLINK_ENTRY_IMAGE_BATCH_DESC:
      return blink_desc_workspace_size(p->n_img, p->max_baselines, p->grid_n, p->workgroups > 0 ? p->workgroups : 512,
                                       bytes);
    case BLINK_ENTRY_DEDISPERSE: return blink_dedisperse_workspace_size(p->C, p->n_dm, bytes);
    default: return BLINK_ERR_ARG;
  }
}

blink_status blink_ifft2d_workspace_size(int n_img, int grid_n, int precision, size_t* bytes) {
  if (!bytes || n_img < 0) return BLINK_ERR_ARG;
  if (!valid_precision(precision)) return BLINK_ERR_ARG;
  const int logn = log2_exact(grid_n);
  if (logn < 0) return BLINK_ERR_SIZE;
  FftLayout L = fft_layout((size_t)n_img, logn);
  if (!L.ok) return BLINK_ERR_SIZE;
  *bytes = L.total;
  return BLINK_OK;
}

blink_status blink_image_batch_workspace_size(int T, int C, int P, int B, int grid_n, int weighting,
                                              int precision, size_t* bytes) {
  if (!bytes || T < 0 || C < 0 || P < 1 || B < 0) return BLINK_ERR_ARG;
  if (weighting != BLINK_WEIGHT_NATURAL && weighting != BLINK_WEIGHT_UNIFORM) return BLINK_ERR_ARG;
  if (!valid_precision(precision)) return BLINK_ERR_ARG;
  const int logn = log2_exact(grid_n);
  if (logn < 0) return BLINK_ERR_SIZE;
  const size_t n_img = (size_t)T * C * P;
  ImageLayout L = image_layout((size_t)T * C, P, B, logn, weighting,
                               n_img < kMaxGroupImages ? n_img : kMaxGroupImages);
  if (!L.ok) return BLINK_ERR_SIZE;
  *bytes = L.total;
  return BLINK_OK;
}

blink_status blink_image_batch_corrected_workspace_size(int T, int C, int P, int B, int grid_n, int weighting,
                                                        int precision, size_t* bytes) {
  if (!bytes || T < 0 || C < 0 || P < 1 || B < 0) return BLINK_ERR_ARG;
  if (weighting != BLINK_WEIGHT_NATURAL && weighting != BLINK_WEIGHT_UNIFORM) return BLINK_ERR_ARG;
  if (!valid_precision(precision)) return BLINK_ERR_ARG;
  const int logn = log2_exact(grid_n);
  if (logn < 0) return BLINK_ERR_SIZE;
  const size_t n_img = (size_t)T * C * P;
  ImageLayout L = image_layout((size_t)T * C, P, B, logn, weighting,
                               n_img < kMaxGroupImages ? n_img : kMaxGroupImages, true);
  if (!L.ok) return BLINK_ERR_SIZE;
  *bytes = L.total;
  return BLINK_OK;
}

blink_status blink_grid(blink_ctx ctx, const blink_cf32* vis, const uint8_t* flags, const double* uvw_m,
                        const double* freq_hz, int T, int C, int P, int B, int grid_n, double pixel_scale,
                        int weighting, blink_cf32* grids, int32_t* counts, double* weight_sum,
                        int32_t* cell_idx, int32_t* n_out, void* workspace, size_t workspace_bytes,
                        void* hip_stream) {
  int logn = 0;
  blink_status st = check_problem(ctx, vis, uvw_m, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting,
                                  grids, workspace, &logn);
  if (st != BLINK_OK) return st;
  if (P > 4) return fail(ctx, BLINK_ERR_ARG, "blink_grid supports P <= 4 polarisations");
  const size_t n_tc = (size_t)T * C;
  if (n_tc == 0) return BLINK_OK;
  const size_t Q = largest_fitting_chunk(n_tc, workspace_bytes,
                                         [&](size_t q) { return grid_layout(q, P, B, logn).total; });
  if (Q == 0) {
    return fail(ctx, BLINK_ERR_SIZE, "workspace of %zu bytes is smaller than one (t,c) pair needs (%zu)",
                workspace_bytes, grid_layout(1, P, B, logn).total);
  }
  if (Q * P > (size_t)INT32_MAX) return fail(ctx, BLINK_ERR_SIZE, "batch too large");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t N = size_t(1) << logn;
  const int S = blink::grid_strip_width(logn);
  int log_s = 0;
  while ((1 << log_s) < S) ++log_s;
  char* ws = (char*)workspace;
  GridLayout L = grid_layout(Q, P, B, logn);
  for (size_t tc0 = 0; tc0 < n_tc; tc0 += Q) {
    const int q = (int)((n_tc - tc0) < Q ? (n_tc - tc0) : Q);
    blink::BinArgs ba{};
    ba.uvw = uvw_m;
    ba.freq = freq_hz;
    ba.flags = flags;
    ba.tc0 = (int)tc0;
    ba.Q = q;
    ba.C = C;
    ba.B = B;
    ba.logn = logn;
    ba.log_strip = log_s;
    ba.ku_limit = (int)N;
    ba.P = P;
    ba.pixel_scale = pixel_scale;
    ba.plc = (int2*)(ws + L.bins.plc);
    ba.strip_off = (int*)(ws + L.bins.off);
    ba.n_kept = (int*)(ws + L.bins.kept);
    ba.occ = (int*)(ws + L.bins.occ);
    ba.cell_idx = cell_idx;
    ba.n_out = n_out;
    hipError_t e;
    {
      KernelTimer kt(ctx, BLINK_KERNEL_BIN, s);
      e = blink::launch_bin(ba, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "bin kernel");
    blink::GridArgs ga{};
    ga.vis = (const float2*)vis + tc0 * P * B;
    ga.plc = ba.plc;
    ga.strip_off = ba.strip_off;
    ga.Q = q;
    ga.P = P;
    ga.B = B;
    ga.logn = logn;
    ga.uniform = weighting;
    ga.grids = (float2*)grids + tc0 * P * N * N;
    ga.counts = counts ? counts + tc0 * N * N : nullptr;
    ga.occ = ba.occ;
    {
      KernelTimer kt(ctx, BLINK_KERNEL_GRID, s);
      e = blink::launch_grid_full(ga, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "grid kernel");
    if (weight_sum) {
      KernelTimer kt(ctx, BLINK_KERNEL_WEIGHTS, s);
      e = blink::launch_image_weights(ba.n_kept, ba.occ, weighting, P, 0, q * P, nullptr,
                                      weight_sum + tc0 * P, s);
      if (e != hipSuccess) return hip_fail(ctx, e, "weights kernel");
    }
  }
  return BLINK_OK;
}

blink_status blink_ifft2d(blink_ctx ctx, const blink_cf32* grids, const double* weight_sum, int n_img,
                          int grid_n, int precision, int shift, float* images, void* workspace,
                          size_t workspace_bytes, void* hip_stream) {
  if (n_img < 0) return fail(ctx, BLINK_ERR_ARG, "n_img < 0");
  const int logn = log2_exact(grid_n);
  if (logn < 0) return fail(ctx, BLINK_ERR_SIZE, "grid_n=%d is not a power of two in [8, 4096]", grid_n);
  if (!valid_precision(precision)) return fail(ctx, BLINK_ERR_ARG, "unsupported precision %d", precision);
  if (!ctx) return BLINK_ERR_ARG;
  if (ctx->broken) return fail(ctx, BLINK_ERR_STATE, "context unusable after an earlier HIP error");
  if (n_img == 0) return BLINK_OK;
  if (!grids || !images || !workspace) return fail(ctx, BLINK_ERR_ARG, "NULL grids, images or workspace");
  if ((uintptr_t)workspace % kAlign) return fail(ctx, BLINK_ERR_ARG, "workspace is not 256-byte aligned");
  const size_t Q = largest_fitting_chunk((size_t)n_img, workspace_bytes,
                                         [&](size_t q) { return fft_layout(q, logn).total; });
  if (Q == 0)
    return fail(ctx, BLINK_ERR_SIZE, "workspace of %zu bytes is smaller than one image needs (%zu)",
                workspace_bytes, fft_layout(1, logn).total);
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t N = size_t(1) << logn;
  char* ws = (char*)workspace;
  FftLayout L = fft_layout(Q, logn);
  for (size_t i0 = 0; i0 < (size_t)n_img; i0 += Q) {
    const int q = (int)(((size_t)n_img - i0) < Q ? ((size_t)n_img - i0) : Q);
    float2* H = (float2*)(ws + L.H);
    hipError_t e;
    {
      KernelTimer kt(ctx, BLINK_KERNEL_DENSE_COLFFT, s);
      e = blink::launch_dense_colfft((const float2*)grids + i0 * N * N, q, logn, shift != 0, precision, H,
                                     ctx->tw[logn], ctx->dft_ops, s);
    }
    if (e == hipSuccess) {
      blink::RowArgs ra{};
      ra.H = H;
      ra.images = images + i0 * N * N;
      ra.logn = logn;
      ra.P = 1;
      ra.img0 = (int)i0;
      ra.wmode = blink::kWeightUser;
      ra.w_user = weight_sum;
      ra.dft_ops = ctx->dft_ops;
      KernelTimer kt(ctx, BLINK_KERNEL_ROW_FFT, s);
      e = blink::launch_row_c2r(ra, q, ctx->plan[logn][0][precision].row_tpb, precision, ctx->tw[logn], s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "ifft2d kernels");
  }
  return BLINK_OK;
}

// blink_image_batch, and blink_image_batch_corrected when corr is non-null (checked by the caller).
static blink_status image_batch(blink_ctx ctx, const blink_cf32* vis, const uint8_t* flags, const double* uvw_m,
                                const double* freq_hz, int T, int C, int P, int B, int grid_n, double pixel_scale,
                                int weighting, int precision, int shift, const blink_corrections* corr,
                                float* images, double* weight_sum, int32_t* n_out, void* workspace,
                                size_t workspace_bytes, void* hip_stream) {
  int logn = 0;
  blink_status st = check_problem(ctx, vis, uvw_m, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting,
                                  images, workspace, &logn);
  if (st != BLINK_OK) return st;
  if (!valid_precision(precision)) return fail(ctx, BLINK_ERR_ARG, "unsupported precision %d", precision);
  const size_t n_tc = (size_t)T * C;
  if (n_tc == 0) return BLINK_OK;
  const bool corrected = corr != nullptr;
  const auto& plan = ctx->plan[logn][weighting][precision];
  const size_t want = plan.group > 0 ? (size_t)plan.group : kMaxGroupImages;
  size_t Q = largest_fitting_chunk(n_tc, workspace_bytes, [&](size_t q) {
    return image_layout(q, P, B, logn, weighting, q * P < want ? q * P : want, corrected).total;
  });
  size_t h_images = Q * P < want ? Q * P : want;
  if (Q == 0 && image_layout(1, P, B, logn, weighting, 1, corrected).total <= workspace_bytes) {
    Q = 1;                       // fall back to one intermediate at a time
    h_images = 1;
  }
  if (Q == 0)
    return fail(ctx, BLINK_ERR_SIZE, "workspace of %zu bytes is smaller than one (t,c) pair needs (%zu)",
                workspace_bytes, image_layout(1, P, B, logn, weighting, 1, corrected).total);
  if (Q * P > (size_t)INT32_MAX) return fail(ctx, BLINK_ERR_SIZE, "batch too large");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t N = size_t(1) << logn;
  const int S = plan.col_strip;
  int log_s = 0;
  while ((1 << log_s) < S) ++log_s;
  char* ws = (char*)workspace;
  ImageLayout L = image_layout(Q, P, B, logn, weighting, h_images, corrected);
  const int G = (int)h_images;
  for (size_t tc0 = 0; tc0 < n_tc; tc0 += Q) {
    const int q = (int)((n_tc - tc0) < Q ? (n_tc - tc0) : Q);
    blink::BinArgs ba{};
    ba.uvw = uvw_m;
    ba.freq = freq_hz;
    ba.flags = flags;
    ba.tc0 = (int)tc0;
    ba.Q = q;
    ba.C = C;
    ba.B = B;
    ba.logn = logn;
    ba.log_strip = log_s;
    ba.ku_limit = (int)(N / 2);
    ba.P = P;
    ba.pixel_scale = pixel_scale;
    ba.plc = (int2*)(ws + L.bins.plc);
    ba.strip_off = (int*)(ws + L.bins.off);
    ba.n_kept = (int*)(ws + L.bins.kept);
    ba.occ = (int*)(ws + L.bins.occ);
    ba.cell_idx = nullptr;
    ba.n_out = n_out;
    ba.ext = (int*)(ws + L.bins.ext);
    hipError_t e;
    {
      KernelTimer kt(ctx, BLINK_KERNEL_BIN, s);
      e = blink::launch_bin(ba, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "bin kernel");
    blink::ColArgs ca{};
    ca.vis = (const float2*)vis + tc0 * P * B;
    if (corrected) {
      // the corrected visibilities of this chunk replace vis for the gridding
      blink::CorrArgs xa{};
      xa.vis = ca.vis;
      xa.uvw = uvw_m;
      xa.freq = freq_hz;
      xa.gains = (const float2*)corr->gains;
      xa.tc0 = (int)tc0;
      xa.Q = q;
      xa.C = C;
      xa.P = P;
      xa.B = B;
      xa.n_ant = corr->n_ant;
      xa.l0 = corr->l0;
      xa.m0 = corr->m0;
      xa.n0m1 = std::sqrt(1.0 - corr->l0 * corr->l0 - corr->m0 * corr->m0) - 1.0;
      xa.out = (float2*)(ws + L.vc);
      {
        KernelTimer kt(ctx, BLINK_KERNEL_CORRECT, s);
        e = blink::launch_correct_vis(xa, s);
      }
      if (e != hipSuccess) return hip_fail(ctx, e, "visibility correction kernel");
      ca.vis = xa.out;
    }
    ca.plc = ba.plc;
    ca.strip_off = ba.strip_off;
    ca.Q = q;
    ca.P = P;
    ca.B = B;
    ca.logn = logn;
    ca.uniform = weighting;
    ca.shift = shift != 0;
    ca.H = (float2*)(ws + L.H);
    ca.occ = ba.occ;
    ca.dft_ops = ctx->dft_ops;
    ca.col_loop = plan.col_loop;
    ca.ext = ba.ext;
    const int n_img = q * P;
    blink::RowArgs ra{};
    ra.H = ca.H;
    ra.ext = ba.ext;
    ra.logn = logn;
    ra.P = P;
    ra.wmode = weighting == BLINK_WEIGHT_UNIFORM ? blink::kWeightUniform : blink::kWeightNatural;
    ra.n_kept = ba.n_kept;
    ra.occ = ba.occ;
    ra.weight_sum = weight_sum ? weight_sum + tc0 * P : nullptr;
    ra.dft_ops = ctx->dft_ops;
    // Images go through the two passes G at a time so that their intermediates can stay in the
    // last-level cache between the column and the row launch.
    for (int i0 = 0; i0 < n_img; i0 += G) {
      const int gi = (n_img - i0) < G ? (n_img - i0) : G;
      ca.img0 = i0;
      {
        KernelTimer kt(ctx, BLINK_KERNEL_GRID_COLFFT, s);
        e = blink::launch_grid_colfft(ca, gi, S, precision, ctx->tw[logn], s);
      }
      if (e != hipSuccess) return hip_fail(ctx, e, "grid+column FFT kernel");
      ra.img0 = i0;
      ra.images = images + (tc0 * P + i0) * N * N;
      {
        KernelTimer kt(ctx, BLINK_KERNEL_ROW_FFT, s);
        e = blink::launch_row_c2r(ra, gi, plan.row_tpb, precision, ctx->tw[logn], s);
      }
      if (e != hipSuccess) return hip_fail(ctx, e, "row FFT kernel");
    }
  }
  return BLINK_OK;
}

blink_status blink_image_batch(blink_ctx ctx, const blink_cf32* vis, const uint8_t* flags, const double* uvw_m,
                               const double* freq_hz, int T, int C, int P, int B, int grid_n, double pixel_scale,
                               int weighting, int precision, int shift, float* images, double* weight_sum,
                               int32_t* n_out, void* workspace, size_t workspace_bytes, void* hip_stream) {
  return image_batch(ctx, vis, flags, uvw_m, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting, precision, shift,
                     nullptr, images, weight_sum, n_out, workspace, workspace_bytes, hip_stream);
}

blink_status blink_image_batch_noalloc(blink_ctx ctx, const blink_cf32* vis, const uint8_t* flags,
                                       const double* uvw_m, const double* freq_hz, int T, int C, int P, int B,
                                       int grid_n, double pixel_scale, int weighting, int precision, int shift,
                                       float* images, double* weight_sum, int32_t* n_out, void* hip_stream) {
  if (!ctx) return BLINK_ERR_ARG;
  if (!ctx->scratch) return fail(ctx, BLINK_ERR_STATE, "no static scratch address on this context's device");
  const int logn = log2_exact(grid_n);
  if (logn >= 0 && P >= 1 && B >= 0 && (weighting == BLINK_WEIGHT_NATURAL || weighting == BLINK_WEIGHT_UNIFORM)) {
    const ImageLayout one = image_layout(1, P, B, logn, weighting, 1);
    if (!one.ok || one.total > BLINK_STATIC_SCRATCH_BYTES)
      return fail(ctx, BLINK_ERR_SIZE,
                  "one (t,c) pair of N=%d, P=%d, B=%d needs %zu bytes of scratch, more than the %zu bytes of the "
                  "static scratch of blink_image_batch_noalloc",
                  grid_n, P, B, one.total, (size_t)BLINK_STATIC_SCRATCH_BYTES);
  }
  // Kernel timing is not taken here: recording it may create events.
  const bool profiling = ctx->profiling;
  ctx->profiling = false;
  const blink_status st = image_batch(ctx, vis, flags, uvw_m, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting,
                                      precision, shift, nullptr, images, weight_sum, n_out, ctx->scratch,
                                      BLINK_STATIC_SCRATCH_BYTES, hip_stream);
  ctx->profiling = profiling;
  return st;
}

blink_status blink_image_batch_corrected(blink_ctx ctx, const blink_cf32* vis, const uint8_t* flags,
                                         const double* uvw_m, const double* freq_hz, int T, int C, int P, int B,
                                         int grid_n, double pixel_scale, int weighting, int precision, int shift,
                                         const blink_corrections* corr, float* images, double* weight_sum,
                                         int32_t* n_out, void* workspace, size_t workspace_bytes,
                                         void* hip_stream) {
  if (corr) {
    if (!(std::isfinite(corr->l0) && std::isfinite(corr->m0) && corr->l0 * corr->l0 + corr->m0 * corr->m0 < 1.0))
      return fail(ctx, BLINK_ERR_ARG, "phase centre (l0=%g, m0=%g) is not a direction (l0^2 + m0^2 < 1)", corr->l0,
                  corr->m0);
    if (corr->gains && (corr->n_ant < 2 || (long long)corr->n_ant * (corr->n_ant - 1) / 2 != (long long)B))
      return fail(ctx, BLINK_ERR_ARG, "n_ant=%d does not give B=%d cross baselines", corr->n_ant, B);
  }
  return image_batch(ctx, vis, flags, uvw_m, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting, precision, shift,
                     corr, images, weight_sum, n_out, workspace, workspace_bytes, hip_stream);
}

blink_status blink_correlate(blink_ctx ctx, const int8_t* volt, int S, int F, int A, int n_int, int n_favg,
                             int pol_mode, blink_cf32* vis, blink_cf32* autos, void* hip_stream) {
  if (!ctx) return BLINK_ERR_ARG;
  if (S < 0 || F < 0 || n_int < 1 || n_favg < 1 || (pol_mode != 2 && pol_mode != 4))
    return fail(ctx, BLINK_ERR_ARG, "bad correlator arguments (S=%d F=%d n_int=%d n_favg=%d pol_mode=%d)", S, F, n_int,
                n_favg, pol_mode);
  if (A < 4 || A > 256 || A % 4 != 0)
    return fail(ctx, BLINK_ERR_ARG, "the correlator takes 4 .. 256 antennas in multiples of 4 (A=%d)", A);
  if (S % n_int != 0 || F % n_favg != 0)
    return fail(ctx, BLINK_ERR_ARG, "n_int=%d must divide S=%d and n_favg=%d must divide F=%d", n_int, S, n_favg, F);
  if ((long long)n_int * n_favg > 65535 || S / n_int > 65535 || F / n_favg > 65535)
    return fail(ctx, BLINK_ERR_ARG, "n_int n_favg above 65535 or more than 65535 intervals or channels");
  if (S == 0 || F == 0) return BLINK_OK;
  if (!volt || !vis) return fail(ctx, BLINK_ERR_ARG, "null voltage or visibility pointer");
  if (reinterpret_cast<uintptr_t>(volt) % 16 != 0)
    return fail(ctx, BLINK_ERR_ARG, "the voltage array must be 16-byte aligned");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  blink::CorrelateArgs ca{};
  ca.volt = volt;
  ca.S = S;
  ca.F = F;
  ca.A = A;
  ca.n_int = n_int;
  ca.n_favg = n_favg;
  ca.pol_mode = pol_mode;
  ca.n_slabs = (2 * A + 31) / 32;
  ca.vis = (float2*)vis;
  ca.autos = (float2*)autos;
  hipError_t e;
  {
    KernelTimer kt(ctx, BLINK_KERNEL_CORRELATE, s);
    e = blink::launch_correlate(ca, s);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "correlator kernel");
  return BLINK_OK;
}

blink_status blink_dispersion_delays(const double* freq_hz, int C, double dt_s, const double* dm, int n_dm,
                                     int32_t* delays) {
  if (C < 1 || n_dm < 0 || !(dt_s > 0.0) || !std::isfinite(dt_s) || !freq_hz || (n_dm > 0 && (!dm || !delays)))
    return BLINK_ERR_ARG;
  double f_ref = 0.0;
  for (int c = 0; c < C; ++c) {
    if (!(freq_hz[c] > 0.0) || !std::isfinite(freq_hz[c])) return BLINK_ERR_ARG;
    f_ref = freq_hz[c] > f_ref ? freq_hz[c] : f_ref;
  }
  const double ref_mhz = f_ref / 1.0e6;
  constexpr double kDispersion = 4148.808;   // s MHz^2 cm^3 / pc
  for (int k = 0; k < n_dm; ++k) {
    if (!(dm[k] >= 0.0) || !std::isfinite(dm[k])) return BLINK_ERR_ARG;
    for (int c = 0; c < C; ++c) {
      const double f_mhz = freq_hz[c] / 1.0e6;
      const double steps = kDispersion * dm[k] * (1.0 / (f_mhz * f_mhz) - 1.0 / (ref_mhz * ref_mhz)) / dt_s;
      if (!(steps < 2.0e9)) return BLINK_ERR_ARG;
      delays[(size_t)k * C + c] = (int32_t)std::nearbyint(steps);
    }
  }
  return BLINK_OK;
}

blink_status blink_dedisperse_workspace_size(int C, int n_dm, size_t* bytes) {
  if (!bytes || C < 1 || n_dm < 0) return BLINK_ERR_ARG;
  *bytes = align_up((size_t)C * (size_t)n_dm * sizeof(int32_t));
  return BLINK_OK;
}

blink_status blink_dedisperse(blink_ctx ctx, const float* images, int T, int C, int grid_n, const int32_t* delays,
                              int n_dm, int t_out, float* out, void* workspace, size_t workspace_bytes,
                              void* hip_stream) {
  if (!ctx) return BLINK_ERR_ARG;
  const int logn = log2_exact(grid_n);
  if (logn < 0) return fail(ctx, BLINK_ERR_SIZE, "grid_n=%d unsupported", grid_n);
  if (T < 0 || C < 1 || n_dm < 0 || t_out < 0 || t_out > T || n_dm > 65535 || t_out > 65535)
    return fail(ctx, BLINK_ERR_ARG, "bad de-dispersion sizes (T=%d C=%d n_dm=%d t_out=%d)", T, C, n_dm, t_out);
  if (n_dm == 0 || t_out == 0) return BLINK_OK;
  if (!images || !delays || !out || !workspace) return fail(ctx, BLINK_ERR_ARG, "null pointer");
  const size_t table = (size_t)C * (size_t)n_dm * sizeof(int32_t);
  if (workspace_bytes < table)
    return fail(ctx, BLINK_ERR_SIZE, "workspace of %zu bytes is smaller than the delay table (%zu)", workspace_bytes,
                table);
  for (size_t i = 0; i < (size_t)C * n_dm; ++i)
    if (delays[i] < 0 || (long long)delays[i] > (long long)T - t_out)
      return fail(ctx, BLINK_ERR_ARG, "delay %d of entry %zu outside 0 .. T - t_out = %d", delays[i], i, T - t_out);
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = hipMemcpyAsync(workspace, delays, table, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "delay table copy");
  {
    KernelTimer kt(ctx, BLINK_KERNEL_DEDISPERSE, s);
    e = blink::launch_dedisperse(images, C, logn, (const int*)workspace, n_dm, t_out, out, s);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "de-dispersion kernel");
  return BLINK_OK;
}

blink_status blink_image_batch_conv_workspace_size(int T, int C, int P, int B, int grid_n, int kernel_width,
                                                   int precision, size_t* bytes) {
  if (!bytes || T < 0 || C < 0 || P < 1 || B < 0) return BLINK_ERR_ARG;
  if (!valid_precision(precision)) return BLINK_ERR_ARG;
  const int logn = log2_exact(grid_n);
  if (logn < 0) return BLINK_ERR_SIZE;
  if (!conv_args_ok(kernel_width, 0.0, logn)) return BLINK_ERR_ARG;
  const size_t n_img = (size_t)T * C * P;
  ConvLayout L = conv_layout((size_t)T * C, P, B, logn, kernel_width,
                             n_img < kMaxGroupImages ? n_img : kMaxGroupImages);
  if (!L.ok) return BLINK_ERR_SIZE;
  *bytes = L.total;
  return BLINK_OK;
}

blink_status blink_image_batch_conv(blink_ctx ctx, const blink_cf32* vis, const uint8_t* flags, const double* uvw_m,
                                    const double* freq_hz, int T, int C, int P, int B, int grid_n, double pixel_scale,
                                    int kernel_width, double kernel_beta, int precision, int shift, float* images,
                                    double* weight_sum, int32_t* n_out, void* workspace, size_t workspace_bytes,
                                    void* hip_stream) {
  int logn = 0;
  blink_status st = check_problem(ctx, vis, uvw_m, freq_hz, T, C, P, B, grid_n, pixel_scale, BLINK_WEIGHT_NATURAL,
                                  images, workspace, &logn);
  if (st != BLINK_OK) return st;
  if (!valid_precision(precision)) return fail(ctx, BLINK_ERR_ARG, "unsupported precision %d", precision);
  if (!conv_args_ok(kernel_width, kernel_beta, logn))
    return fail(ctx, BLINK_ERR_ARG, "kernel width %d (1..16, < N/2) or beta %g (0..100) out of range", kernel_width,
                kernel_beta);
  const size_t n_tc = (size_t)T * C;
  if (n_tc == 0) return BLINK_OK;
  const auto& plan = ctx->plan[logn][BLINK_WEIGHT_NATURAL][precision];
  // The nearest-cell plan's group size, capped at 192 MiB of full half spectra (48 images at
  // 1024^2: faster for this path than the nearest-cell plan's 64, whose column kernel per image
  // is shorter).
  const size_t h_bytes = (size_t(1) << (2 * logn - 1)) * sizeof(float2);
  const size_t cache_group = ((size_t)192 << 20) / h_bytes > 0 ? ((size_t)192 << 20) / h_bytes : 1;
  size_t want = plan.group > 0 ? (size_t)plan.group : kMaxGroupImages;
  if (want > cache_group) want = cache_group;
  size_t Q = largest_fitting_chunk(n_tc, workspace_bytes, [&](size_t q) {
    return conv_layout(q, P, B, logn, kernel_width, q * P < want ? q * P : want).total;
  });
  size_t h_images = Q * P < want ? Q * P : want;
  if (Q == 0 && conv_layout(1, P, B, logn, kernel_width, 1).total <= workspace_bytes) {
    Q = 1;
    h_images = 1;
  }
  if (Q == 0)
    return fail(ctx, BLINK_ERR_SIZE, "workspace of %zu bytes is smaller than one (t,c) pair needs (%zu)",
                workspace_bytes, conv_layout(1, P, B, logn, kernel_width, 1).total);
  if (Q * P > (size_t)INT32_MAX) return fail(ctx, BLINK_ERR_SIZE, "batch too large");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t N = size_t(1) << logn;
  const int S = blink::conv_strip_width(logn);
  int log_s = 0;
  while ((1 << log_s) < S) ++log_s;
  char* ws = (char*)workspace;
  ConvLayout L = conv_layout(Q, P, B, logn, kernel_width, h_images);
  const blink::ConvParams cp{kernel_width, kernel_beta};
  float* corr = (float*)(ws + L.corr);
  hipError_t e;
  {
    KernelTimer kt(ctx, BLINK_KERNEL_CONV_CORRECTION, s);
    e = blink::launch_conv_correction(corr, logn, cp, shift != 0, s);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "grid-correction kernel");
  const int G = (int)h_images;
  for (size_t tc0 = 0; tc0 < n_tc; tc0 += Q) {
    const int q = (int)((n_tc - tc0) < Q ? (n_tc - tc0) : Q);
    blink::BinArgs ba{};
    ba.uvw = uvw_m;
    ba.freq = freq_hz;
    ba.flags = flags;
    ba.tc0 = (int)tc0;
    ba.Q = q;
    ba.C = C;
    ba.B = B;
    ba.logn = logn;
    ba.log_strip = log_s;
    ba.ku_limit = (int)(N / 2);
    ba.P = P;
    ba.pixel_scale = pixel_scale;
    ba.plc = (int2*)(ws + L.bins.plc);
    ba.strip_off = (int*)(ws + L.bins.off);
    ba.n_kept = (int*)(ws + L.bins.kept);
    ba.occ = (int*)(ws + L.bins.occ);
    ba.cell_idx = nullptr;
    ba.n_out = n_out;
    ba.ext = (int*)(ws + L.bins.ext);
    {
      KernelTimer kt(ctx, BLINK_KERNEL_BIN, s);
      e = blink::launch_bin_conv(ba, cp, L.rec_stride, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "convolutional bin kernel");
    blink::ColArgs ca{};
    ca.vis = (const float2*)vis + tc0 * P * B;
    ca.plc = ba.plc;
    ca.strip_off = ba.strip_off;
    ca.Q = q;
    ca.P = P;
    ca.B = B;
    ca.logn = logn;
    ca.uniform = 0;
    ca.shift = shift != 0;
    ca.H = (float2*)(ws + L.H);
    ca.occ = ba.occ;
    ca.dft_ops = ctx->dft_ops;
    ca.rec_stride = L.rec_stride;
    ca.ext = ba.ext;
    const int n_img = q * P;
    blink::RowArgs ra{};
    ra.H = ca.H;
    ra.ext = ba.ext;
    ra.logn = logn;
    ra.P = P;
    ra.wmode = blink::kWeightNatural;
    ra.n_kept = ba.n_kept;
    ra.occ = ba.occ;
    ra.weight_sum = weight_sum ? weight_sum + tc0 * P : nullptr;
    ra.dft_ops = ctx->dft_ops;
    ra.corr = corr;
    for (int i0 = 0; i0 < n_img; i0 += G) {
      const int gi = (n_img - i0) < G ? (n_img - i0) : G;
      ca.img0 = i0;
      {
        KernelTimer kt(ctx, BLINK_KERNEL_GRID_COLFFT, s);
        e = blink::launch_grid_colfft_conv(ca, gi, cp, precision, ctx->tw[logn], s);
      }
      if (e != hipSuccess) return hip_fail(ctx, e, "convolutional grid + column FFT kernel");
      ra.img0 = i0;
      ra.images = images + (tc0 * P + i0) * N * N;
      {
        KernelTimer kt(ctx, BLINK_KERNEL_ROW_FFT, s);
        e = blink::launch_row_c2r(ra, gi, plan.row_tpb, precision, ctx->tw[logn], s);
      }
      if (e != hipSuccess) return hip_fail(ctx, e, "row FFT kernel");
    }
  }
  return BLINK_OK;
}

blink_status blink_image_average(blink_ctx ctx, const float* images, int T, int C, int P, int grid_n, int axes,
                                 float* out, void* hip_stream) {
  if (T < 0 || C < 0 || P < 0 || axes < 0 || axes > 7) return fail(ctx, BLINK_ERR_ARG, "bad sizes or axes %d", axes);
  const int logn = log2_exact(grid_n);
  if (logn < 0) return fail(ctx, BLINK_ERR_SIZE, "grid_n=%d unsupported", grid_n);
  if (!ctx) return BLINK_ERR_ARG;
  if (ctx->broken) return fail(ctx, BLINK_ERR_STATE, "context unusable after an earlier HIP error");
  if ((size_t)T * C * P == 0) return BLINK_OK;
  if (!images || !out) return fail(ctx, BLINK_ERR_ARG, "NULL images or out");
  if ((uintptr_t)images % 16 || (uintptr_t)out % 16) return fail(ctx, BLINK_ERR_ARG, "arrays must be 16-byte aligned");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e;
  {
    KernelTimer kt(ctx, BLINK_KERNEL_AVERAGE, s);
    e = blink::launch_image_average(images, T, C, P, logn, axes, out, s);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "image average kernel");
  return BLINK_OK;
}

// ---------------------------------------------------------------- uneven batches
}  // extern "C"

namespace {

struct DescLayout {
  size_t valid, order, counter, status, plc, strip_off, H, total;
  bool ok;
};

DescLayout desc_layout(size_t n_img, size_t max_b, size_t max_n, size_t slots) {
  Carve c;
  DescLayout L;
  L.valid = c.take(n_img, sizeof(int));
  L.order = c.take(n_img, sizeof(int));
  L.counter = c.take(1, sizeof(int));
  L.status = c.take(1, sizeof(int));
  L.plc = c.take(slots, 2 * max_b * sizeof(int2));
  L.strip_off = c.take(slots, (max_n / 2 + 1) * sizeof(int));
  L.H = c.take(slots, max_n * (max_n / 2) * sizeof(float2));
  L.total = c.off;
  L.ok = c.ok;
  return L;
}

// Staged form: per-image placements, strip offsets, counts and extents (by position in the
// order), the chunk table and the chunk buffer, which holds as many of the largest images' half
// spectra as fit 256 MiB (at least one, at most the batch). An image touches only the columns
// below its extent, so a chunk's working set is that fraction of the buffer (about 220 MiB with
// the uneven benchmark's extents, which the 256 MB last-level cache holds between the chunk's
// two launches; 128, 192, 320, 384 and 512 MiB were slower on it).
struct StagedLayout {
  size_t valid, order, counter, status, chunks, plc, strip_off, kept, occ, ext, H, total;
  int max_chunks;
  int64_t chunk_elems;
  bool ok;
};

StagedLayout staged_layout(size_t n_img, size_t max_b, size_t max_n) {
  StagedLayout L;
  int max_logn = 0;
  while ((size_t(1) << max_logn) < max_n) ++max_logn;
  const int64_t h = (int64_t)max_n * (int64_t)(max_n / 2);
  int64_t cap = ((int64_t)256 << 20) / (h * (int64_t)sizeof(float2));
  if (cap > (int64_t)n_img) cap = (int64_t)n_img;   // a batch of few images needs no more
  if (cap < 1) cap = 1;
  L.chunk_elems = h * cap;
  int64_t mc = 0;                   // the chunk slots reserved for every grid size up to the largest
  for (int l = 3; l <= max_logn; ++l) mc += blink::staged_slots(l, L.chunk_elems, (int)n_img);
  L.max_chunks = (int)(mc < (int64_t)1 << 30 ? mc : (int64_t)1 << 30);
  Carve c;
  L.valid = c.take(n_img, sizeof(int));
  L.order = c.take(n_img, sizeof(int));
  L.counter = c.take(1, sizeof(int));
  L.status = c.take(1, sizeof(int));
  L.chunks = c.take((size_t)L.max_chunks, sizeof(int4));
  L.plc = c.take(n_img, 2 * max_b * sizeof(int2));
  L.strip_off = c.take(n_img, (max_n / 2 + 1) * sizeof(int));
  L.kept = c.take(n_img, sizeof(int));
  L.occ = c.take(n_img, sizeof(int));
  L.ext = c.take(n_img, sizeof(int));
  L.H = c.take((size_t)L.chunk_elems, sizeof(float2));
  L.total = c.off;
  L.ok = c.ok;
  return L;
}

struct DescCall {
  const blink_image_desc* desc;
  int n_img;
  const blink_cf32* vis;
  int64_t vis_len;
  const double* uvw;
  int64_t uvw_len;
  const uint8_t* flags;
  int64_t flags_len;
  int max_b, max_n, weighting, precision, shift;
  float* images;
  int64_t images_len;
  double* weight_sum;
  int32_t* n_out;
  int32_t* status;
  void* ws;
  size_t ws_bytes;
};

blink_status check_desc(blink_ctx ctx, const DescCall& c, int* max_logn) {
  if (c.n_img < 0 || c.max_b < 0 || c.vis_len < 0 || c.uvw_len < 0 || c.flags_len < 0 || c.images_len < 0)
    return fail(ctx, BLINK_ERR_ARG, "negative count or length");
  if (c.max_b > (1 << 30)) return fail(ctx, BLINK_ERR_SIZE, "max_baselines exceeds 2^30");
  *max_logn = log2_exact(c.max_n);
  if (*max_logn < 0) return fail(ctx, BLINK_ERR_SIZE, "max_grid_n=%d is not a power of two in [8, 4096]", c.max_n);
  if (c.weighting != BLINK_WEIGHT_NATURAL && c.weighting != BLINK_WEIGHT_UNIFORM)
    return fail(ctx, BLINK_ERR_ARG, "unknown weighting %d", c.weighting);
  if (!valid_precision(c.precision)) return fail(ctx, BLINK_ERR_ARG, "unsupported precision %d", c.precision);
  if (!ctx) return BLINK_ERR_ARG;
  if (ctx->broken) return fail(ctx, BLINK_ERR_STATE, "context unusable after an earlier HIP error");
  if (c.n_img == 0) return BLINK_OK;
  if (!c.desc || !c.images || !c.ws) return fail(ctx, BLINK_ERR_ARG, "NULL desc, images or workspace");
  if ((c.vis_len > 0 && !c.vis) || (c.uvw_len > 0 && !c.uvw))
    return fail(ctx, BLINK_ERR_ARG, "NULL vis or uvw_m with a nonzero length");
  if ((uintptr_t)c.ws % kAlign) return fail(ctx, BLINK_ERR_ARG, "workspace is not 256-byte aligned");
  return BLINK_OK;
}

int desc_block_for(blink_ctx ctx, int weighting) { return weighting ? 512 : ctx->desc_block; }

// The common descriptor-pass arguments of both forms.
blink::DescArgs desc_args(blink_ctx ctx, const DescCall& c, int max_logn, int block) {
  blink::DescArgs a{};
  a.desc = c.desc;
  a.n_img = c.n_img;
  a.vis = (const float2*)c.vis;
  a.vis_len = c.vis_len;
  a.uvw = c.uvw;
  a.uvw_len = c.uvw_len;
  a.flags = c.flags;
  a.flags_len = c.flags_len;
  a.max_b = c.max_b;
  a.max_logn = max_logn;
  a.weighting = c.weighting;
  a.shift = c.shift != 0;
  a.block = block;
  a.images = c.images;
  a.images_len = c.images_len;
  a.weight_sum = c.weight_sum;
  a.n_out = c.n_out;
  a.strip_stride = c.max_n / 2 + 1;
  for (int l = 3; l <= 12; ++l) a.tw[l] = ctx->tw[l];
  a.dft_ops = ctx->dft_ops;
  return a;
}

// Staged form: the descriptor pass, one binning launch, then for every grid size from the largest
// down and every chunk slot reserved for it, the chunk's column launch and row launch with the
// batched path's plan for that size (strip width, strips per workgroup, row block).
blink_status run_desc_staged(blink_ctx ctx, const DescCall& c, int max_logn, hipStream_t s) {
  StagedLayout L = staged_layout(c.n_img, c.max_b, c.max_n);
  if (!L.ok || L.total > c.ws_bytes)
    return fail(ctx, BLINK_ERR_SIZE, "workspace of %zu bytes is smaller than the %zu bytes the staged form needs",
                c.ws_bytes, L.total);
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  char* ws = (char*)c.ws;
  blink::DescArgs a = desc_args(ctx, c, max_logn, desc_block_for(ctx, c.weighting));
  a.status = c.status ? c.status : (int32_t*)(ws + L.status);
  a.valid = (int*)(ws + L.valid);
  a.order = (int*)(ws + L.order);
  a.counter = (int*)(ws + L.counter);
  a.plc = (int2*)(ws + L.plc);
  a.strip_off = (int*)(ws + L.strip_off);
  a.H = (float2*)(ws + L.H);
  a.chunks = (int4*)(ws + L.chunks);
  a.max_chunks = L.max_chunks;
  a.chunk_elems = L.chunk_elems;
  a.kept = (int*)(ws + L.kept);
  a.occ = (int*)(ws + L.occ);
  a.ext = (int*)(ws + L.ext);
  for (int l = 3; l <= 12; ++l) {
    int ls = 0;
    while ((1 << (ls + 1)) <= ctx->plan[l][c.weighting][c.precision].col_strip) ++ls;
    a.col_log_strip[l] = ls;
  }
  hipError_t e;
  {
    KernelTimer kt(ctx, BLINK_KERNEL_DESC_PREP, s);
    e = blink::launch_desc_prep(a, s);
  }
  if (e == hipSuccess) {
    KernelTimer kt(ctx, BLINK_KERNEL_BIN, s);
    e = blink::launch_desc_bin(a, s);
  }
  int j = 0;
  for (int l = max_logn; l >= 3 && e == hipSuccess; --l) {
    const auto& plan = ctx->plan[l][c.weighting][c.precision];
    const int cap = blink::staged_capacity(l, L.chunk_elems, c.n_img);
    const int slots = blink::staged_slots(l, L.chunk_elems, c.n_img);
    for (int m = 0; m < slots && e == hipSuccess; ++m, ++j) {
      {
        KernelTimer kt(ctx, BLINK_KERNEL_GRID_COLFFT, s);
        e = blink::launch_chunk_colfft(a, j, l, plan.col_strip, plan.col_loop, cap, c.precision, s);
      }
      if (e == hipSuccess) {
        KernelTimer kt(ctx, BLINK_KERNEL_ROW_FFT, s);
        e = blink::launch_chunk_row(a, j, l, plan.row_tpb, cap, c.precision, s);
      }
    }
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "uneven-batch staged kernels");
  return BLINK_OK;
}

blink_status run_desc(blink_ctx ctx, const DescCall& c, hipStream_t s) {
  int max_logn = 0;
  blink_status st = check_desc(ctx, c, &max_logn);
  if (st != BLINK_OK || c.n_img == 0) return st;
  if (ctx->desc_form == BLINK_DESC_STAGED) return run_desc_staged(ctx, c, max_logn, s);
  const int block = desc_block_for(ctx, c.weighting);
  const int per_cu = blink::persistent_blocks_per_cu(block, c.weighting != 0, c.precision);
  if (per_cu <= 0) return fail(ctx, BLINK_ERR_ARG, "persistent kernel with %d threads is not available", block);
  size_t wg = ctx->desc_workgroups > 0 ? (size_t)ctx->desc_workgroups : (size_t)per_cu * ctx->cu_count;
  if (wg > (size_t)c.n_img) wg = (size_t)c.n_img;
  while (wg > 1 && desc_layout(c.n_img, c.max_b, c.max_n, wg).total > c.ws_bytes) wg = wg / 2 > 1 ? wg / 2 : 1;
  while (desc_layout(c.n_img, c.max_b, c.max_n, wg + 1).total <= c.ws_bytes && wg < (size_t)c.n_img &&
         wg < (ctx->desc_workgroups > 0 ? (size_t)ctx->desc_workgroups : (size_t)per_cu * ctx->cu_count))
    ++wg;
  DescLayout L = desc_layout(c.n_img, c.max_b, c.max_n, wg);
  if (!L.ok || L.total > c.ws_bytes)
    return fail(ctx, BLINK_ERR_SIZE, "workspace of %zu bytes is smaller than the %zu bytes one slot needs", c.ws_bytes,
                L.total);
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  char* ws = (char*)c.ws;
  blink::DescArgs a = desc_args(ctx, c, max_logn, block);
  a.status = c.status ? c.status : (int32_t*)(ws + L.status);
  a.valid = (int*)(ws + L.valid);
  a.order = (int*)(ws + L.order);
  a.counter = (int*)(ws + L.counter);
  a.plc = (int2*)(ws + L.plc);
  a.strip_off = (int*)(ws + L.strip_off);
  a.H = (float2*)(ws + L.H);
  hipError_t e;
  {
    KernelTimer kt(ctx, BLINK_KERNEL_DESC_PREP, s);
    e = blink::launch_desc_prep(a, s);
  }
  if (e == hipSuccess) {
    KernelTimer kt(ctx, BLINK_KERNEL_PERSISTENT, s);
    e = blink::launch_persistent(a, (int)wg, c.precision, s);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "uneven-batch kernels");
  return BLINK_OK;
}

}  // namespace

struct blink_graph_s {
  blink_ctx ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

blink_status blink_desc_workspace_size(int n_img, int max_baselines, int max_grid_n, int workgroups, size_t* bytes) {
  if (!bytes || n_img < 0 || max_baselines < 0 || workgroups < 1) return BLINK_ERR_ARG;
  if (log2_exact(max_grid_n) < 0) return BLINK_ERR_SIZE;
  DescLayout L = desc_layout((size_t)n_img, (size_t)max_baselines, (size_t)max_grid_n,
                             (size_t)(workgroups < n_img ? workgroups : (n_img > 0 ? n_img : 1)));
  StagedLayout S = staged_layout((size_t)n_img, (size_t)max_baselines, (size_t)max_grid_n);
  if (!L.ok || !S.ok) return BLINK_ERR_SIZE;
  *bytes = L.total > S.total ? L.total : S.total;
  return BLINK_OK;
}

blink_status blink_image_batch_desc(blink_ctx ctx, const blink_image_desc* desc, int n_img, const blink_cf32* vis,
                                    int64_t vis_len, const double* uvw_m, int64_t uvw_len, const uint8_t* flags,
                                    int64_t flags_len, int max_baselines, int max_grid_n, int weighting,
                                    int precision, int shift, float* images, int64_t images_len,
                                    double* weight_sum, int32_t* n_out, int32_t* status, void* workspace,
                                    size_t workspace_bytes, void* hip_stream) {
  DescCall c{desc, n_img, vis, vis_len, uvw_m, uvw_len, flags, flags_len, max_baselines, max_grid_n, weighting,
             precision, shift, images, images_len, weight_sum, n_out, status, workspace, workspace_bytes};
  return run_desc(ctx, c, (hipStream_t)hip_stream);
}

blink_status blink_get_desc_plan(blink_ctx ctx, int* block_threads, int* workgroups) {
  if (!ctx) return BLINK_ERR_ARG;
  if (block_threads) *block_threads = ctx->desc_block;
  if (workgroups) *workgroups = ctx->desc_workgroups;
  return BLINK_OK;
}

blink_status blink_get_desc_form(blink_ctx ctx, int* form) {
  if (!ctx || !form) return BLINK_ERR_ARG;
  *form = ctx->desc_form;
  return BLINK_OK;
}

blink_status blink_set_desc_form(blink_ctx ctx, int form) {
  if (!ctx) return BLINK_ERR_ARG;
  if (form != BLINK_DESC_PERSISTENT && form != BLINK_DESC_STAGED)
    return fail(ctx, BLINK_ERR_ARG, "unknown descriptor-path form %d", form);
  ctx->desc_form = form;
  return BLINK_OK;
}

blink_status blink_set_desc_plan(blink_ctx ctx, int block_threads, int workgroups) {
  if (!ctx) return BLINK_ERR_ARG;
  if ((block_threads != 512 && block_threads != 1024) || workgroups < 0)
    return fail(ctx, BLINK_ERR_ARG, "descriptor plan needs block 512 or 1024 and workgroups >= 0");
  ctx->desc_block = block_threads;
  ctx->desc_workgroups = workgroups;
  return BLINK_OK;
}

blink_status blink_autotune_desc(blink_ctx ctx, const blink_image_desc* desc, int n_img, const blink_cf32* vis,
                                 int64_t vis_len, const double* uvw_m, int64_t uvw_len, const uint8_t* flags,
                                 int64_t flags_len, int max_baselines, int max_grid_n, int weighting, int precision,
                                 int shift, float* images, int64_t images_len, double* weight_sum, int32_t* n_out,
                                 int32_t* status, void* workspace, size_t workspace_bytes, void* hip_stream,
                                 int* block_threads, int* workgroups, double* best_ms) {
  DescCall c{desc, n_img, vis, vis_len, uvw_m, uvw_len, flags, flags_len, max_baselines, max_grid_n, weighting,
             precision, shift, images, images_len, weight_sum, n_out, status, workspace, workspace_bytes};
  int max_logn = 0;
  blink_status st = check_desc(ctx, c, &max_logn);
  if (st != BLINK_OK) return st;
  const int sb = ctx->desc_block, sw = ctx->desc_workgroups, sf = ctx->desc_form;
  const bool was_profiling = ctx->profiling;
  ctx->profiling = false;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    ctx->profiling = was_profiling;
    return hip_fail(ctx, hipErrorOutOfMemory, "hipEventCreate");
  }
  const int blocks[] = {512, 1024};
  // the staged form is timed only when the workspace holds its layout
  const bool staged_fits = n_img > 0 && staged_layout(n_img, max_baselines, max_grid_n).total <= workspace_bytes;
  double best = 1e300;
  int bb = sb, bw = sw, bf = sf;
  blink_status result = BLINK_OK;
  for (int form = BLINK_DESC_PERSISTENT; form <= BLINK_DESC_STAGED && result == BLINK_OK; ++form) {
    if (form == BLINK_DESC_STAGED && !staged_fits) continue;
    for (int bi = 0; bi < 2 && result == BLINK_OK; ++bi) {
      if (weighting && blocks[bi] != 512) continue;
      // the staged form takes the batched path's per-size plans: one timing, with block 512
      if (form == BLINK_DESC_STAGED && blocks[bi] != 512) continue;
      const int resident = blink::persistent_blocks_per_cu(blocks[bi], weighting != 0, precision) * ctx->cu_count;
      const int counts[] = {0, resident / 2, resident / 4};
      for (int wi = 0; wi < 3 && result == BLINK_OK; ++wi) {
        if (wi > 0 && (counts[wi] < 1 || form == BLINK_DESC_STAGED)) continue;
        ctx->desc_form = form;
        ctx->desc_block = blocks[bi];
        ctx->desc_workgroups = counts[wi];
        double t = 1e300;
        for (int rep = 0; rep < 3 && result == BLINK_OK; ++rep) {
          hipError_t he = hipEventRecord(e0, s);
          result = run_desc(ctx, c, s);
          if (he == hipSuccess) he = hipEventRecord(e1, s);
          if (he == hipSuccess) he = hipEventSynchronize(e1);
          float ms = 0.f;
          if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
          if (he != hipSuccess && result == BLINK_OK) result = hip_fail(ctx, he, "autotune timing");
          if (rep > 0 && ms < t) t = ms;
        }
        if (result == BLINK_OK && t < best) {
          best = t;
          bb = ctx->desc_block;
          bw = ctx->desc_workgroups;
          bf = ctx->desc_form;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->profiling = was_profiling;
  if (result != BLINK_OK) {
    ctx->desc_block = sb;
    ctx->desc_workgroups = sw;
    ctx->desc_form = sf;
    return result;
  }
  ctx->desc_block = bb;
  ctx->desc_workgroups = bw;
  ctx->desc_form = bf;
  result = run_desc(ctx, c, s);
  if (block_threads) *block_threads = bb;
  if (workgroups) *workgroups = bw;
  if (best_ms) *best_ms = best;
  return result;
}

blink_status blink_graph_create_desc(blink_ctx ctx, const blink_image_desc* desc, int n_img, const blink_cf32* vis,
                                     int64_t vis_len, const double* uvw_m, int64_t uvw_len, const uint8_t* flags,
                                     int64_t flags_len, int max_baselines, int max_grid_n, int weighting,
                                     int precision, int shift, float* images, int64_t images_len,
                                     double* weight_sum, int32_t* n_out, int32_t* status, void* workspace,
                                     size_t workspace_bytes, blink_graph* out) {
  if (!out) return BLINK_ERR_ARG;
  *out = nullptr;
  DescCall c{desc, n_img, vis, vis_len, uvw_m, uvw_len, flags, flags_len, max_baselines, max_grid_n, weighting,
             precision, shift, images, images_len, weight_sum, n_out, status, workspace, workspace_bytes};
  int max_logn = 0;
  blink_status st = check_desc(ctx, c, &max_logn);
  if (st != BLINK_OK) return st;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  blink_graph gr = new (std::nothrow) blink_graph_s;
  if (!gr) return BLINK_ERR_NOMEM;
  gr->ctx = ctx;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  const bool was_profiling = ctx->profiling;
  ctx->profiling = false;                       // no event records inside the graph
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = run_desc(ctx, c, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &gr->graph);
    if (st == BLINK_OK && e2 != hipSuccess) e = e2;
  }
  ctx->profiling = was_profiling;
  if (e == hipSuccess && st == BLINK_OK) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess || st != BLINK_OK) {
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
    if (st != BLINK_OK) return st;
    return hip_fail(ctx, e, "graph capture");
  }
  *out = gr;
  return BLINK_OK;
}

blink_status blink_graph_launch(blink_graph graph, void* hip_stream) {
  if (!graph || !graph->exec) return BLINK_ERR_ARG;
  DeviceGuard g(graph->ctx->device);
  hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(graph->ctx, e, "hipGraphLaunch");
  return BLINK_OK;
}

blink_status blink_graph_destroy(blink_graph graph) {
  if (!graph) return BLINK_OK;
  {
    DeviceGuard g(graph->ctx->device);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
  }
  delete graph;
  return BLINK_OK;
}

blink_status blink_plan_options(int grid_n, int weighting, int* col_strips, int* n_col, int* row_blocks,
                                int* n_row) {
  const int logn = log2_exact(grid_n);
  if (logn < 0) return BLINK_ERR_SIZE;
  if (weighting != 0 && weighting != 1) return BLINK_ERR_ARG;
  int col[4], row[4];
  const int nc = blink::col_strip_options(logn, weighting != 0, col);
  const int nr = blink::row_block_options(logn, row);
  if (n_col) *n_col = nc;
  if (n_row) *n_row = nr;
  for (int i = 0; i < nc && col_strips; ++i) col_strips[i] = col[i];
  for (int i = 0; i < nr && row_blocks; ++i) row_blocks[i] = row[i];
  return BLINK_OK;
}

blink_status blink_get_plan(blink_ctx ctx, int grid_n, int weighting, int precision, int* col_strip, int* row_block,
                            int* group, int* col_loop) {
  const int logn = log2_exact(grid_n);
  if (logn < 0) return fail(ctx, BLINK_ERR_SIZE, "grid_n=%d unsupported", grid_n);
  if (!ctx || (weighting != 0 && weighting != 1) || !valid_precision(precision)) return BLINK_ERR_ARG;
  const auto& p = ctx->plan[logn][weighting][precision];
  if (col_strip) *col_strip = p.col_strip;
  if (row_block) *row_block = p.row_tpb;
  if (group) *group = p.group;
  if (col_loop) *col_loop = p.col_loop;
  return BLINK_OK;
}

blink_status blink_set_plan(blink_ctx ctx, int grid_n, int weighting, int precision, int col_strip, int row_block,
                            int group, int col_loop) {
  const int logn = log2_exact(grid_n);
  if (logn < 0) return fail(ctx, BLINK_ERR_SIZE, "grid_n=%d unsupported", grid_n);
  if (!ctx || (weighting != 0 && weighting != 1) || group < 0 || !valid_precision(precision)) return BLINK_ERR_ARG;
  if (col_loop < 1 || col_loop > kMaxColLoop)
    return fail(ctx, BLINK_ERR_ARG, "col_loop=%d outside 1..%d", col_loop, kMaxColLoop);
  int col[4], row[4];
  const int nc = blink::col_strip_options(logn, weighting != 0, col);
  const int nr = blink::row_block_options(logn, row);
  bool okc = false, okr = false;
  for (int i = 0; i < nc; ++i) okc |= col[i] == col_strip;
  for (int i = 0; i < nr; ++i) okr |= row[i] == row_block;
  if (!okc || !okr)
    return fail(ctx, BLINK_ERR_ARG, "plan (col_strip=%d, row_block=%d) is not a compiled option for N=%d", col_strip,
                row_block, grid_n);
  auto& p = ctx->plan[logn][weighting][precision];
  p.col_strip = col_strip;
  p.row_tpb = row_block;
  p.group = group;
  p.col_loop = col_loop;
  return BLINK_OK;
}

blink_status blink_autotune_image_batch(blink_ctx ctx, const blink_cf32* vis, const uint8_t* flags,
                                        const double* uvw_m, const double* freq_hz, int T, int C, int P, int B,
                                        int grid_n, double pixel_scale, int weighting, int precision, int shift,
                                        float* images, double* weight_sum, int32_t* n_out, void* workspace,
                                        size_t workspace_bytes, void* hip_stream, int* col_strip, int* row_block,
                                        int* group, int* col_loop, double* best_ms) {
  int logn = 0;
  blink_status st = check_problem(ctx, vis, uvw_m, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting, images,
                                  workspace, &logn);
  if (st != BLINK_OK) return st;
  if (!valid_precision(precision)) return fail(ctx, BLINK_ERR_ARG, "unsupported precision %d", precision);
  const auto saved = ctx->plan[logn][weighting][precision];
  const bool was_profiling = ctx->profiling;
  ctx->profiling = false;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(ctx, g.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    ctx->profiling = was_profiling;
    return hip_fail(ctx, hipErrorOutOfMemory, "hipEventCreate");
  }
  int col[4], row[4];
  const int nc = blink::col_strip_options(logn, weighting != 0, col);
  const int nr = blink::row_block_options(logn, row);
  const int groups[] = {16, 24, 32, 48, 64, 96, 128, 256};
  constexpr int n_groups = (int)(sizeof(groups) / sizeof(groups[0]));
  double best = 1e300;
  auto best_plan = saved;
  blink_status result = BLINK_OK;
  auto& p = ctx->plan[logn][weighting][precision];
  // time the context's current plan for (grid_n, weighting, precision): best of two runs after one
  auto time_plan = [&]() {
    double t = 1e300;
    for (int rep = 0; rep < 3 && result == BLINK_OK; ++rep) {
      hipError_t he = hipEventRecord(e0, s);
      result = blink_image_batch(ctx, vis, flags, uvw_m, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting,
                                 precision, shift, images, weight_sum, n_out, workspace, workspace_bytes, hip_stream);
      if (he == hipSuccess) he = hipEventRecord(e1, s);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess && result == BLINK_OK) result = hip_fail(ctx, he, "autotune timing");
      if (rep > 0 && ms < t) t = ms;        // the first run warms caches and code
    }
    if (result == BLINK_OK && t < best) {
      best = t;
      best_plan = p;
    }
  };
  // every (group, strip width, row block) with one strip per column workgroup, then 2, 4, .. 16
  // strips per workgroup for every group with the best strip width and row block of those (the
  // best group can change with the strips per workgroup)
  for (int gi = 0; gi < n_groups && result == BLINK_OK; ++gi) {
    for (int ci = 0; ci < nc && result == BLINK_OK; ++ci) {
      for (int ri = 0; ri < nr && result == BLINK_OK; ++ri) {
        p.col_strip = col[ci];
        p.row_tpb = row[ri];
        p.group = groups[gi];
        p.col_loop = 1;
        time_plan();
      }
    }
  }
  if (result == BLINK_OK) {
    const auto first = best_plan;
    const int nstrips = (1 << logn) / 2 / first.col_strip;
    for (int gi = 0; gi < n_groups && result == BLINK_OK; ++gi) {
      for (int loop = 2; loop <= 16 && loop <= nstrips && result == BLINK_OK; loop *= 2) {
        p = first;
        p.group = groups[gi];
        p.col_loop = loop;
        time_plan();
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->profiling = was_profiling;
  ctx->plan[logn][weighting][precision] = result == BLINK_OK ? best_plan : saved;
  if (result != BLINK_OK) return result;
  // leave a result computed with the chosen plan in the outputs
  result = blink_image_batch(ctx, vis, flags, uvw_m, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting, precision,
                             shift, images, weight_sum, n_out, workspace, workspace_bytes, hip_stream);
  if (col_strip) *col_strip = best_plan.col_strip;
  if (row_block) *row_block = best_plan.row_tpb;
  if (group) *group = best_plan.group;
  if (col_loop) *col_loop = best_plan.col_loop;
  if (best_ms) *best_ms = best;
  return result;
}

blink_status blink_profile_enable(blink_ctx ctx, int enable) {
  if (!ctx) return BLINK_ERR_ARG;
  release_records(ctx);
  ctx->profiling = enable != 0;
  return BLINK_OK;
}

blink_status blink_profile_read(blink_ctx ctx, int kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches || kernel < 0 || kernel >= BLINK_KERNEL_COUNT) return BLINK_ERR_ARG;
  DeviceGuard g(ctx->device);
  double sum = 0.0;
  for (auto& pr : ctx->records[kernel]) {
    hipError_t e = hipEventSynchronize(pr.second);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) return hip_fail(ctx, e, "blink_profile_read");
    sum += ms;
  }
  *total_ms = sum;
  *launches = (int64_t)ctx->records[kernel].size();
  return BLINK_OK;
}

}  // extern "C"
