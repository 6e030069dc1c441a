// Shared host/device helpers of the mrpie library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>

#include "mrpie.h"
#include "fft.hpp"

namespace mrpie {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

#define MRPIE_HIP(call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return ::mrpie::hip_fail(e_, #call); \
  } while (0)

inline int n_index(int N) {
  switch (N) {
    case 64: return 0;
    case 128: return 1;
    case 192: return 2;
    case 256: return 3;
    case 32: return 4;
    default: return -1;
  }
}

// Roots of unity w_N^e = exp(-2 pi i e / N), e < N, for the four sizes;
// written by k_init_twiddles in double precision and rounded once.  Each
// translation unit holds its own copy (no relocatable device code).
static __device__ float2 g_tw[5][256];
static __device__ double2 g_tw64[5][256];

static __global__ void k_init_twiddles() {
  const int idx = blockIdx.x;
  const int N = idx == 0 ? 64 : idx == 1 ? 128 : idx == 2 ? 192 : idx == 3 ? 256 : 32;
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)e / (double)N, &s, &c);
    g_tw[idx][e] = make_float2((float)c, (float)s);
    g_tw64[idx][e] = make_double2(c, s);
  }
}

static inline int launch_init_twiddles(hipStream_t s) {
  hipLaunchKernelGGL(k_init_twiddles, dim3(5), dim3(256), 0, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_init_twiddles");
  return MRPIE_OK;
}

// Copy the N-entry twiddle table to LDS (NT: the kernel's fixed workgroup
// size, 0 = read blockDim.x).
template <int N, int NT = 0>
__device__ __forceinline__ void load_twiddles(float2* s_tw) {
  constexpr int idx = N == 64 ? 0 : N == 128 ? 1 : N == 192 ? 2 : N == 256 ? 3 : 4;
  for (int i = threadIdx.x; i < N; i += wg_threads<NT>()) s_tw[i] = g_tw[idx][i];
}
template <int N, int NT = 0>
__device__ __forceinline__ void load_twiddles(double2* s_tw) {
  constexpr int idx = N == 64 ? 0 : N == 128 ? 1 : N == 192 ? 2 : N == 256 ? 3 : 4;
  for (int i = threadIdx.x; i < N; i += wg_threads<NT>()) s_tw[i] = g_tw64[idx][i];
}

// Wave reductions (64-wide waves, every lane active).  DPP row shifts by
// 1, 2, 4, 8 leave in lane 15 of each row of 16 the reduction of its row
// (lanes shifted in from outside a row read 0, the identity of both
// reductions below); the four row results are then combined in a fixed
// order through scalar registers.  The result is uniform over the wave.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float lane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffLL), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// max over the wave of NON-NEGATIVE values
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp_f<0x111>(v));  // row_shr:1
  v = fmaxf(v, dpp_f<0x112>(v));  // row_shr:2
  v = fmaxf(v, dpp_f<0x114>(v));  // row_shr:4
  v = fmaxf(v, dpp_f<0x118>(v));  // row_shr:8
  return fmaxf(fmaxf(lane_f(v, 15), lane_f(v, 31)), fmaxf(lane_f(v, 47), lane_f(v, 63)));
}
// sum over the wave, in a fixed order (deterministic)
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0x111>(v);
  v += dpp_d<0x112>(v);
  v += dpp_d<0x114>(v);
  v += dpp_d<0x118>(v);
  return (lane_d(v, 15) + lane_d(v, 31)) + (lane_d(v, 47) + lane_d(v, 63));
}
// Workgroup reductions.  red: >= 16 floats of LDS; v >= 0.  All threads
// get the result.
__device__ __forceinline__ float block_max(float v, float* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  lds_barrier();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  lds_barrier();
  float r = red[0];
  for (int i = 1; i < nw; ++i) r = fmaxf(r, red[i]);
  return r;
}
// max of two values over the workgroup with one pair of barriers.  red: >= 32
// floats of LDS; a, b >= 0.
__device__ __forceinline__ void block_max2(float a, float b, float* red, float& ra, float& rb) {
  a = wave_max(a);
  b = wave_max(b);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  lds_barrier();
  if ((threadIdx.x & 63) == 0) {
    red[w] = a;
    red[16 + w] = b;
  }
  lds_barrier();
  ra = red[0];
  rb = red[16];
  for (int i = 1; i < nw; ++i) {
    ra = fmaxf(ra, red[i]);
    rb = fmaxf(rb, red[16 + i]);
  }
}
// red: >= 16 doubles of LDS; fixed summation order (deterministic).
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  lds_barrier();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  lds_barrier();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += red[i];
  return r;
}

__device__ __forceinline__ void flag_status(int* status, int bit) {
  if (status) atomicOr(status, bit);
}

// Box corner n = floor(p + 0.5) clamped to [0, lim]; sets the clamp bit.
__device__ __forceinline__ int box_corner(float p, int lim, int* status) {
  float q = floorf(p + 0.5f);
  if (!(q >= 0.0f && q <= (float)lim)) {  // also catches NaN
    flag_status(status, MRPIE_STATUS_POS_CLAMPED);
    q = (q > (float)lim) ? (float)lim : 0.0f;
  }
  return (int)q;
}

// XCD-aware unit index: consecutive workgroups are dispatched round-robin
// over the 8 XCDs; give each XCD a contiguous range of units so that units
// sharing cache lines share an L2.  Requires nunits % 8 == 0 and
// gridDim.x == nunits.
__device__ __forceinline__ int xcd_unit(int b, int nunits) {
  const int per = nunits >> 3;
  return (b & 7) * per + (b >> 3);
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Raise a kernel's dynamic-LDS limit once to at least `bytes` (host-side
// attribute; done outside any stream capture the first time a size is seen).
hipError_t ensure_lds(const void* kernel, size_t bytes);

// The current device's side stream (non-blocking, default priority) and
// its ring of kSideEvents events (no timing), created on first use.  A call
// that forks work onto it holds side_mutex() while it issues that work, so
// calls from several host threads do not interleave their event records.
constexpr int kSideEvents = 16;
int side_stream(hipStream_t* out, hipEvent_t** events);
std::mutex& side_mutex();

// ---------------------------------------------------------------- timing
// Sampled per-kernel timing (diagnostic): when enabled, every `stride`-th
// launch of a timed kernel class is launched with hipExtLaunchKernelGGL and
// a start / stop event pair, so the events carry that dispatch's own start
// and end time on its stream; mrpie_timing_read() averages them.
enum TimedKernel {
  TK_ROWS = 0, TK_COLS = 1, TK_REG = 2, TK_GEMM = 3, TK_ADJ = 4, TK_LDS = 5, TK_UPD = 6, TK_GAT = 7, TK_COUNT = 8
};
struct TimedLaunch {
  hipEvent_t start = nullptr, stop = nullptr;
};
// `units`: the launch's grid.y (jobs of a sweep pass, positions of an
// adjoint pass, pairs of a registration pass), averaged per class.
TimedLaunch timing_slot(int kind, int units);

// units: what the timing record averages for this launch (jobs, positions
// or pairs it processes)
template <typename K, typename... A>
inline void launch_ku(int kind, int units, K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, A... args) {
  const TimedLaunch t = timing_slot(kind, units);
  if (t.start) hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, s, t.start, t.stop, 0u, args...);
  else hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}
// ... with grid.y units
template <typename K, typename... A>
inline void launch_k(int kind, K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, A... args) {
  launch_ku(kind, (int)grid.y, kernel, grid, block, lds, s, args...);
}

}  // namespace mrpie
