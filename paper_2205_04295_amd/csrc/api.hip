// Host-side services of the mrpie C ABI: errors, validation, twiddles, and
// the FFT / modulus test hooks.
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "common.hpp"

namespace mrpie {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  set_error("HIP error '%s' in %s", hipGetErrorString(e), what);
  return MRPIE_EDEVICE;
}

// ------------------------------------------------------------ LDS limits
hipError_t ensure_lds(const void* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> done;
  std::lock_guard<std::mutex> lk(mu);
  auto it = done.find(kernel);
  if (it != done.end() && it->second >= bytes) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done[kernel] = bytes;
  return e;
}

// ------------------------------------------------------------ side stream
// One non-blocking stream (default priority) and a ring of events per
// device, created on first use, for work the library overlaps with a
// latency-bound sweep on the caller's stream.
namespace {
constexpr int kMaxDevices = 16;
struct Side {
  hipStream_t stream = nullptr;
  hipEvent_t ev[kSideEvents] = {};
};
Side g_side[kMaxDevices];
std::mutex g_side_mu;
}  // namespace

std::mutex& side_mutex() {
  static std::mutex mu;
  return mu;
}

int side_stream(hipStream_t* out, hipEvent_t** events) {
  int dev = 0;
  MRPIE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MRPIE_EDEVICE, "device %d beyond the side-stream table", dev);
  std::lock_guard<std::mutex> lk(g_side_mu);
  Side& sd = g_side[dev];
  if (!sd.stream) {
    MRPIE_HIP(hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking));
    for (int i = 0; i < kSideEvents; ++i) MRPIE_HIP(hipEventCreateWithFlags(&sd.ev[i], hipEventDisableTiming));
  }
  *out = sd.stream;
  *events = sd.ev;
  return MRPIE_OK;
}

// ------------------------------------------------------------ timing
namespace {
constexpr int kEvPairs = 8192;
struct Timing {
  int stride = 0;
  long long seen[TK_COUNT] = {};
  hipEvent_t ev[2 * kEvPairs] = {};
  int kind[kEvPairs] = {};
  int units[kEvPairs] = {};
  int used = 0;
  bool created = false;
};
Timing g_timing;
}  // namespace

TimedLaunch timing_slot(int kind, int units) {
  Timing& T = g_timing;
  TimedLaunch t;
  if (T.stride <= 0) return t;
  if ((T.seen[kind]++ % T.stride) != 0 || T.used >= kEvPairs) return t;
  const int slot = T.used++;
  T.kind[slot] = kind;
  T.units[slot] = units;
  t.start = T.ev[2 * slot];
  t.stop = T.ev[2 * slot + 1];
  return t;
}

// ------------------------------------------------------------ FFT test hook
// Row pass: one workgroup per (array, row); unnormalised transform of the
// row times `scale`.
template <int N, bool INV>
__global__ __launch_bounds__(256) void k_fft_rows(float2* data, float scale) {
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* a = tw + N;
  float2* b = a + N;
  load_twiddles<N>(tw);
  float2* row = data + (size_t)blockIdx.x * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) a[i] = row[i];
  __syncthreads();
  float2* r = fft_lds<N, INV>(a, b, 1, tw);
  for (int i = threadIdx.x; i < N; i += blockDim.x) row[i] = cscale(r[i], scale);
}

// Column pass: one workgroup per (array, stripe of WC columns).
template <int N, bool INV, int WC>
__global__ __launch_bounds__(256) void k_fft_cols(float2* data, float scale) {
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* a = tw + N;
  float2* b = a + WC * N;
  load_twiddles<N>(tw);
  const int per = N / WC;
  const int arr = blockIdx.x / per;
  const int c0 = (blockIdx.x - arr * per) * WC;
  float2* base = data + (size_t)arr * N * N + c0;
  for (int i = threadIdx.x; i < N * WC; i += blockDim.x) {
    const int k = i / WC, cc = i - k * WC;
    a[cc * N + k] = base[(size_t)k * N + cc];
  }
  __syncthreads();
  float2* r = fft_lds<N, INV>(a, b, WC, tw);
  for (int i = threadIdx.x; i < N * WC; i += blockDim.x) {
    const int k = i / WC, cc = i - k * WC;
    base[(size_t)k * N + cc] = cscale(r[cc * N + k], scale);
  }
}

template <int N>
static int fft2_impl(int B, float2* d, int inverse, hipStream_t s) {
  constexpr int WC = 4;
  const float sc = 1.0f / sqrtf((float)N);
  const size_t lr = (3 * N) * sizeof(float2);
  const size_t lc = (N + 2 * WC * N) * sizeof(float2);
  if (inverse) {
    hipLaunchKernelGGL((k_fft_rows<N, true>), dim3(B * N), dim3(256), lr, s, d, sc);
    hipLaunchKernelGGL((k_fft_cols<N, true, WC>), dim3(B * (N / WC)), dim3(256), lc, s, d, sc);
  } else {
    hipLaunchKernelGGL((k_fft_rows<N, false>), dim3(B * N), dim3(256), lr, s, d, sc);
    hipLaunchKernelGGL((k_fft_cols<N, false, WC>), dim3(B * (N / WC)), dim3(256), lc, s, d, sc);
  }
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

// ---------------------------------------------------------- modulus hook
__global__ void k_modulus(float2* psi, const float* I, int N, int M) {
  const size_t NN = (size_t)N * N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < NN; i += (size_t)gridDim.x * blockDim.x) {
    float S = 0.f;
    for (int p = 0; p < M; ++p) S += cabs2(psi[p * NN + i]);
    const float sq = sqrtf(fmaxf(I[i], 0.f));
    const float f = S > 0.f ? sq / sqrtf(S) : 0.f;
    for (int p = 0; p < M; ++p) psi[p * NN + i] = cscale(psi[p * NN + i], f);
  }
}

}  // namespace mrpie

using namespace mrpie;

extern "C" {

const char* mrpie_version(void) { return "mrpie 0.1 (gfx950)"; }

const char* mrpie_last_error(void) { return g_err; }

int mrpie_timing_enable(int32_t stride) {
  Timing& T = g_timing;
  if (stride < 0) return fail(MRPIE_EINVAL, "stride < 0");
  if (stride > 0 && !T.created) {
    // no system-scope fence when the stop event is recorded: the fence would
    // write the L2 back and lengthen exactly the dispatch being timed
    for (int i = 0; i < 2 * kEvPairs; ++i)
      MRPIE_HIP(hipEventCreateWithFlags(&T.ev[i], hipEventDisableSystemFence));
    T.created = true;
  }
  T.stride = stride;
  T.used = 0;
  for (int k = 0; k < TK_COUNT; ++k) T.seen[k] = 0;
  return MRPIE_OK;
}

int mrpie_timing_read(double* avg_ms, int64_t* count, double* avg_units, int32_t nkinds) {
  Timing& T = g_timing;
  if (!avg_ms || !count || nkinds < 1) return fail(MRPIE_EINVAL, "bad arguments");
  for (int k = 0; k < nkinds; ++k) {
    avg_ms[k] = 0.0;
    count[k] = 0;
    if (avg_units) avg_units[k] = 0.0;
  }
  for (int i = 0; i < T.used; ++i) {
    MRPIE_HIP(hipEventSynchronize(T.ev[2 * i + 1]));
    float ms = 0.f;
    MRPIE_HIP(hipEventElapsedTime(&ms, T.ev[2 * i], T.ev[2 * i + 1]));
    const int k = T.kind[i];
    if (k < nkinds) {
      avg_ms[k] += ms;
      count[k] += 1;
      if (avg_units) avg_units[k] += T.units[i];
    }
  }
  for (int k = 0; k < nkinds; ++k)
    if (count[k]) {
      avg_ms[k] /= (double)count[k];
      if (avg_units) avg_units[k] /= (double)count[k];
    }
  T.used = 0;
  for (int k = 0; k < TK_COUNT; ++k) T.seen[k] = 0;
  return MRPIE_OK;
}

int mrpie_fft2(int32_t N, int32_t B, void* data, int32_t inverse, void* stream) {
  if (n_index(N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", N);
  if (B < 0) return fail(MRPIE_EINVAL, "B=%d < 0", B);
  if (B == 0) return MRPIE_OK;
  if (!data) return fail(MRPIE_EINVAL, "data is NULL");
  hipStream_t s = (hipStream_t)stream;
  int rc = launch_init_twiddles(s);
  if (rc) return rc;
  float2* d = (float2*)data;
  switch (N) {
    case 32: return fft2_impl<32>(B, d, inverse, s);
    case 64: return fft2_impl<64>(B, d, inverse, s);
    case 128: return fft2_impl<128>(B, d, inverse, s);
    case 192: return fft2_impl<192>(B, d, inverse, s);
    default: return fft2_impl<256>(B, d, inverse, s);
  }
}

int mrpie_modulus(int32_t N, int32_t M, void* psi, const float* intens, void* stream) {
  if (N < 1) return fail(MRPIE_EINVAL, "N=%d < 1", N);
  if (M < 1 || M > MRPIE_MAX_MODES) return fail(M < 1 ? MRPIE_EINVAL : MRPIE_EUNSUPPORTED, "M=%d not in [1,8]", M);
  if (!psi || !intens) return fail(MRPIE_EINVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  const size_t NN = (size_t)N * N;
  const int blocks = (int)std::min<size_t>((NN + 255) / 256, 4096);
  hipLaunchKernelGGL(k_modulus, dim3(blocks), dim3(256), 0, s, (float2*)psi, intens, N, M);
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

}  // extern "C"
