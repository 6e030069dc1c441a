// Autotuner of the sweep's launch shapes (FFT radix plan per pass, threads
// per row workgroup, detector columns per column workgroup, in-place FFTs in
// batches, and the one-workgroup LDS sweep for probes whose modes fit the
// LDS), per probe size N, mode class of M and batch class.  It times every
// candidate on a synthetic problem of the requested shape, on the device,
// and installs the fastest.  Only the timing matters: the synthetic data
// (a hash of the element index) are well-conditioned but meaningless.
#include <algorithm>
#include <vector>

#include "sweep.hpp"

namespace mrpie {

namespace {

struct TuneLayout {
  size_t obj, probe, pos, I, ws, job, total;
  int H;
};

TuneLayout tune_layout(int N, int M, int J) {
  TuneLayout L{};
  L.H = 3 * N;
  const size_t NN = (size_t)N * N;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = ws_align(off + bytes); return o; };
  L.obj = take((size_t)L.H * L.H * 8);
  L.probe = take((size_t)M * NN * 8);
  L.pos = take((size_t)J * 8);
  L.I = take((size_t)J * NN * 4);
  L.ws = take(ws_layout(N, M, 1).total);
  L.job = off;  // bytes per job
  L.total = off;
  return L;
}

__device__ __forceinline__ float hash01(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return (float)(x >> 8) * (1.0f / 16777216.0f);
}

// Job b's synthetic problem: a unit-magnitude object with a small phase, a
// probe of unit-scale modes, integer positions anywhere in the object and
// intensities of the model's mean level.
__global__ void k_tune_fill(char* base, size_t job_bytes, size_t o_obj, size_t o_probe, size_t o_pos, size_t o_I,
                            int H, int N, int M, int J) {
  char* jb = base + (size_t)blockIdx.y * job_bytes;
  const unsigned seed = 0x9e3779b9U * (blockIdx.y + 1);
  const size_t NN = (size_t)N * N;
  const size_t nobj = (size_t)H * H, nprobe = (size_t)M * NN, nI = (size_t)J * NN;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nobj; i += stride) {
    float s, c;
    sincosf(0.2f * hash01(seed ^ (unsigned)i), &s, &c);
    ((float2*)(jb + o_obj))[i] = make_float2(c, s);
  }
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nprobe; i += stride)
    ((float2*)(jb + o_probe))[i] =
        make_float2(hash01(seed + 7u * (unsigned)i) - 0.5f, hash01(seed + 7u * (unsigned)i + 3u) - 0.5f);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nI; i += stride)
    ((float*)(jb + o_I))[i] = 2.0f * (float)M * hash01(seed * 31u + (unsigned)i);
  // positions along a Fermat spiral around the object's centre (golden-angle
  // steps of about 0.04 N: the ~70 % overlap of consecutive probes of the
  // paper's scans, shrunk for long runs so the spiral stays inside), the
  // scan pattern whose box moves the row passes are built for
  const float c0 = fminf(0.0394f * (float)N, 0.95f * (float)(H - N) / (2.f * sqrtf((float)J)));
  const float ctr = 0.5f * (float)(H - N);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)J; i += stride) {
    const float r = c0 * sqrtf((float)i), th = 2.39996323f * (float)i;  // golden angle in radians
    float sn, cs;
    sincosf(th, &sn, &cs);
    ((float*)(jb + o_pos))[2 * i] = floorf(ctr + r * sn + 0.5f);
    ((float*)(jb + o_pos))[2 * i + 1] = floorf(ctr + r * cs + 0.5f);
  }
}

int candidates(int N, int M, bool batched, std::vector<Tuning>& out) {
  out.clear();
  for (int rr : {4, 8})
    for (int cr : {4, 8})
      for (int th : {256, 512})
        for (int cw : {1, 4})
          for (int ip : {0, 1})
            for (int sp : {0, 1}) {
              // the in-place and split options shape multi-job launches only
              if ((ip || sp) && !batched) continue;
              out.push_back(Tuning{rr, cr, th, 0, cw, ip, sp});
            }
  if (lds_sweep_fits(N, M)) out.push_back(Tuning{8, 8, 256, MRPIE_MAX_MODES, 1, 0, 0});
  return (int)out.size();
}

}  // namespace

}  // namespace mrpie

using namespace mrpie;

extern "C" {

int mrpie_tuning_candidates(int32_t N, int32_t M, int32_t batched, mrpie_tuning* out, int32_t cap) {
  if (n_index(N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", N);
  if (batched < 0 || batched > 2) return fail(MRPIE_EINVAL, "batched=%d not in {0, 1, 2}", batched);
  if (M < 1 || M > MRPIE_MAX_MODES) return fail(MRPIE_EINVAL, "M=%d not in [1, 8]", M);
  std::vector<Tuning> c;
  const int n = candidates(N, M, batched != 0, c);
  for (int i = 0; out && i < std::min<int>(n, cap); ++i)
    out[i] = mrpie_tuning{c[i].rows_radix, c[i].cols_radix, c[i].rows_threads, c[i].lds_sweep, c[i].cols_width,
                          c[i].rows_inplace, c[i].rows_split};
  return n;
}

int mrpie_autotune_workspace_size(int32_t N, int32_t M, int32_t batch, int32_t J, size_t* bytes) {
  if (n_index(N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", N);
  if (M < 1 || M > MRPIE_MAX_MODES) return fail(MRPIE_EINVAL, "M=%d not in [1, 8]", M);
  if (batch < 1 || batch > 1024 || J < 1 || J > 100000) return fail(MRPIE_EINVAL, "batch=%d J=%d", batch, J);
  if (!bytes) return fail(MRPIE_EINVAL, "bytes is NULL");
  *bytes = tune_layout(N, M, J).job * (size_t)batch;
  return MRPIE_OK;
}

int mrpie_autotune(int32_t N, int32_t M, int32_t batch, int32_t J, int32_t reps, void* ws, size_t ws_bytes,
                   mrpie_tuning* best, float* cand_ms, void* stream) {
  size_t need = 0;
  int rc = mrpie_autotune_workspace_size(N, M, batch, J, &need);
  if (rc) return rc;
  if (reps < 1 || reps > 100) return fail(MRPIE_EINVAL, "reps=%d not in [1, 100]", reps);
  if (!ws || ws_bytes < need) return fail(MRPIE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  MRPIE_HIP(hipStreamIsCapturing(s, &cap));
  if (cap != hipStreamCaptureStatusNone) return fail(MRPIE_EINVAL, "the autotuner times on the host: not under capture");
  const TuneLayout L = tune_layout(N, M, J);
  char* base = (char*)ws;
  hipLaunchKernelGGL(k_tune_fill, dim3(256, batch), dim3(256), 0, s, base, L.job, L.obj, L.probe, L.pos, L.I, L.H,
                     N, M, J);
  MRPIE_HIP(hipGetLastError());
  std::vector<JobRec> jobs((size_t)batch);
  for (int b = 0; b < batch; ++b) {
    char* jb = base + (size_t)b * L.job;
    jobs[b] = JobRec{(float2*)(jb + L.obj), (float2*)(jb + L.probe), (const float*)(jb + L.pos),
                     (const float*)(jb + L.I), jb + L.ws, nullptr, L.H, L.H, N, M, J, 1};
  }
  const Common c{1.f, 1.f, 1.f, 0.1f, 0, 0};
  std::vector<Tuning> cands;
  const bool batched = batch > 1;
  const int n = candidates(N, M, batched, cands);
  const int nb = batch;  // the call class of `batch` jobs
  const Tuning saved = get_tuning(N, M, nb);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MRPIE_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MRPIE_EDEVICE, "hipEventCreate failed");
  }
  // Round-robin over the candidates, `reps` timed rounds after one warm-up
  // round, each candidate keeping its best time: a drift of the clocks
  // during the run then shifts every candidate alike instead of favouring
  // the ones timed while the GPU ran fastest.
  std::vector<float> t_best((size_t)n, 0.f);
  for (int r = 0; r <= reps && rc == MRPIE_OK; ++r) {
    for (int i = 0; i < n && rc == MRPIE_OK; ++i) {
      set_tuning(N, M, nb, cands[i]);
      hipError_t e = hipEventRecord(e0, s);
      if (e == hipSuccess) rc = run_sweep(c, jobs.data(), batch, nullptr, s);
      if (rc == MRPIE_OK && e == hipSuccess) e = hipEventRecord(e1, s);
      if (rc == MRPIE_OK && e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (rc == MRPIE_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess && rc == MRPIE_OK) rc = hip_fail(e, "autotune timing");
      if (r > 0 && (r == 1 || ms < t_best[i])) t_best[i] = ms;
    }
  }
  float best_ms = 0.f;
  int best_i = -1;
  for (int i = 0; i < n && rc == MRPIE_OK; ++i) {
    if (cand_ms) cand_ms[i] = t_best[i];
    if (best_i < 0 || t_best[i] < best_ms) {
      best_ms = t_best[i];
      best_i = i;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != MRPIE_OK || best_i < 0) {
    set_tuning(N, M, nb, saved);
    return rc ? rc : fail(MRPIE_EDEVICE, "no candidate ran");
  }
  const Tuning& t = cands[best_i];
  set_tuning(N, M, nb, t);
  if (best)
    *best = mrpie_tuning{t.rows_radix, t.cols_radix, t.rows_threads, t.lds_sweep, t.cols_width, t.rows_inplace,
                         t.rows_split};
  return MRPIE_OK;
}

}  // extern "C"
