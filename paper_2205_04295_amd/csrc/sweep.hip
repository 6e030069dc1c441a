// The sequential M-rPIE sweep on gfx950 (Methods, "M-rPIE algorithm",
// Eq. 4-7).
//
// A position step is split at the two transposes of the 2-D FFT into two
// launches; kernel boundaries are the device-wide sync points (a graph-
// replayed launch costs less on MI355X than a cross-XCD grid barrier):
//
//   k_cols  (step s):   per column stripe, all modes: forward column FFT,
//                       mode-summed modulus replacement (Eq. 7), inverse
//                       column FFT, in place in psi[s&1]; accumulates the
//                       Fourier error.
//   k_rows  (s-1 -> s): per probe row r: inverse row FFTs of psi[(s-1)&1],
//                       probe update of row r (Eq. 5) and object update of
//                       the box rows that become rows of the next box or
//                       leave it (Eq. 6), then gather of row r of the next
//                       box, exit waves P_p o (Eq. 1/4) and forward row FFTs
//                       into psi[s&1].
//
// Probe, patch and spectra are double-buffered by step parity, so inside a
// k_rows launch every buffer a unit reads is disjoint from every buffer any
// unit writes; the object rows a unit writes are exactly the rows it then
// re-gathers (it merges them from LDS), so the sweep needs no atomics and is
// bitwise deterministic.  The O update of step s-1 and the gather of step s
// happen in one launch, which keeps rPIE's order: position s reads the
// object after position s-1 has been written.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace mrpie {

enum RowMode { ROWS_HEAD = 0, ROWS_MID = 1, ROWS_TAIL = 2 };

struct SweepArgs {
  int H, W, N, M, J, T;
  float alpha_obj, alpha_probe, beta, gamma;
  int iter_offset, probe_update_start;
  float2* obj;
  float2* probe[2];   // probe[s&1] is the probe used at step s
  const float* pos;   // [J][2]
  const float* I;     // [J][N][N]
  float2* psi[2];     // [M][N][N]
  float2* patch[2];   // [N][N]
  float* pmax[2];     // [N] per-row max of sum_p |P_p|^2 of probe[s&1]
  float* omax[2];     // [N] per-row max of |o_s|^2
  int* box[2];        // [2] integer corner of the box gathered at step s
  double* err_acc;    // [T][kErrSlots]
  int* status;
  const int* iter_dev;  // iteration counter (relative to the call)
};

constexpr int kErrSlots = 256;
constexpr int kCols = 2;  // columns per k_cols workgroup

// ---------------------------------------------------------------- k_rows
template <int N>
__global__ __launch_bounds__(256) void k_rows(SweepArgs a, int jn, int mode) {
  extern __shared__ float2 smem[];
  const int M = a.M;
  float2* tw = smem;                 // N
  float2* pn = tw + N;               // M*N  new probe row r
  float2* orow = pn + M * N;         // N    updated object row (box-prev row rb1)
  float2* bufA = orow + N;           // 3*M*N
  float2* bufB = bufA + 3 * M * N;   // 3*M*N
  __shared__ float redf[16];
  __shared__ float s_omax, s_pmax;

  const int r = blockIdx.x;
  const int it = *a.iter_dev;
  const int s = it * a.J + jn;
  const bool has_prev = mode != ROWS_HEAD;
  const bool has_next = mode != ROWS_TAIL;
  const int cur = s & 1, prv = (s - 1) & 1;
  const size_t NN = (size_t)N * N;

  load_twiddles<N>(tw);

  // next box corner from the current position estimate
  int ny_n = 0, nx_n = 0;
  if (has_next) {
    ny_n = box_corner(a.pos[2 * jn], a.H - N, a.status);
    nx_n = box_corner(a.pos[2 * jn + 1], a.W - N, a.status);
    if (r == 0 && threadIdx.x == 0) {
      a.box[cur][0] = ny_n;
      a.box[cur][1] = nx_n;
    }
  }
  int ny_p = 0, nx_p = 0, rb1 = -1, rb2 = -1;
  if (has_prev) {
    ny_p = a.box[prv][0];
    nx_p = a.box[prv][1];
    if (has_next) {
      const int dy = ny_n - ny_p;
      if (r + dy >= 0 && r + dy < N) rb1 = r + dy;
      if (dy > 0 && r < min(N, dy)) rb2 = r;
      if (dy < 0 && r < min(N, -dy)) rb2 = max(0, N + dy) + r;
    } else {
      rb1 = r;
    }
  }

  float* pmax_out = a.pmax[cur];
  if (has_prev) {
    // ---- reductions of the previous step's max terms
    float vo = 0.f, vp = 0.f;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      vo = fmaxf(vo, a.omax[prv][i]);
      vp = fmaxf(vp, a.pmax[prv][i]);
    }
    vo = block_max(vo, redf);
    vp = block_max(vp, redf + 8);
    if (threadIdx.x == 0) {
      s_omax = vo;
      s_pmax = vp;
    }
    // distinct rows needing an inverse row FFT: slot 0 = probe row r,
    // slot 1 = rb1, slot 2 = rb2 (slots equal to r are served by slot 0)
    const int nsl = 3;
    const float2* src = a.psi[prv];
    for (int i = threadIdx.x; i < nsl * M * N; i += blockDim.x) {
      const int sl = i / (M * N);
      const int rem = i - sl * M * N;
      const int p = rem / N, c = rem - p * N;
      const int row = sl == 0 ? r : (sl == 1 ? rb1 : rb2);
      if (row >= 0 && (sl == 0 || row != r)) bufA[i] = src[p * NN + (size_t)row * N + c];
      else bufA[i] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    float2* res = fft_lds<N, true>(bufA, bufB, nsl * M, tw);
    const float omax = s_omax, pmaxv = s_pmax;

    // ---- probe update of row r (Eq. 5), from the pre-update o and P
    const int it_abs = a.iter_offset + (s - 1) / a.J;
    const bool upd_p = it_abs >= a.probe_update_start;
    const float2* Pold = a.probe[prv];
    float2* Pnew = a.probe[cur];
    const float2* patch = a.patch[prv];
    float pm = 0.f;
    bool bad = false;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
      const float2 o = patch[(size_t)r * N + c];
      const float o2 = cabs2(o);
      const float dP = a.beta * omax + (1.f - a.beta) * o2;
      const float g = (upd_p && dP != 0.f) ? a.alpha_probe / dP : 0.f;
      float ps = 0.f;
      for (int p = 0; p < M; ++p) {
        const float2 P = Pold[p * NN + (size_t)r * N + c];
        const float2 d = csub(res[p * N + c], cmul(P, o));
        const float2 Pn = cadd(P, cscale(cmulc(d, o), g));
        pn[p * N + c] = Pn;
        Pnew[p * NN + (size_t)r * N + c] = Pn;
        ps += cabs2(Pn);
      }
      bad |= !isfinite(ps);
      pm = fmaxf(pm, ps);
    }
    pm = block_max(pm, redf);
    if (threadIdx.x == 0) pmax_out[r] = pm;

    // ---- object update (Eq. 6) of box rows rb1 / rb2
    for (int slot = 1; slot <= 2; ++slot) {
      const int rb = slot == 1 ? rb1 : rb2;
      if (rb < 0) continue;
      const int bs = (rb == r) ? 0 : slot;
      const float2* dres = res + bs * M * N;
      float2* orow_g = a.obj + (size_t)(ny_p + rb) * a.W + nx_p;
      for (int c = threadIdx.x; c < N; c += blockDim.x) {
        const float2 o = patch[(size_t)rb * N + c];
        float Ps = 0.f;
        float2 num = make_float2(0.f, 0.f);
        for (int p = 0; p < M; ++p) {
          const float2 P = Pold[p * NN + (size_t)rb * N + c];
          const float2 d = csub(dres[p * N + c], cmul(P, o));
          num = cadd(num, cmulc(d, P));
          Ps += cabs2(P);
        }
        const float dO = a.gamma * pmaxv + (1.f - a.gamma) * Ps;
        const float g = dO != 0.f ? a.alpha_obj / dO : 0.f;
        const float2 on = cadd(o, cscale(num, g));
        bad |= !(isfinite(on.x) && isfinite(on.y));
        orow_g[c] = on;
        if (slot == 1) orow[c] = on;
      }
    }
    if (bad) flag_status(a.status, MRPIE_STATUS_NONFINITE);
    __syncthreads();
  }

  if (!has_next) return;

  // ---- gather row r of the next box, merging the row just updated
  const int gy = ny_n + r;
  const float2* grow = a.obj + (size_t)gy * a.W;
  float2* patch_n = a.patch[cur];
  const float2* Pcur = a.probe[cur];
  float om = 0.f, pm0 = 0.f;
  for (int c = threadIdx.x; c < N; c += blockDim.x) {
    const int gx = nx_n + c;
    float2 o;
    if (rb1 >= 0 && gx >= nx_p && gx < nx_p + N) o = orow[gx - nx_p];
    else o = grow[gx];
    patch_n[(size_t)r * N + c] = o;
    om = fmaxf(om, cabs2(o));
    float ps = 0.f;
    for (int p = 0; p < M; ++p) {
      const float2 P = has_prev ? pn[p * N + c] : Pcur[p * NN + (size_t)r * N + c];
      ps += cabs2(P);
      bufA[p * N + c] = cmul(P, o);
    }
    pm0 = fmaxf(pm0, ps);
  }
  om = block_max(om, redf);
  if (!has_prev) pm0 = block_max(pm0, redf + 8);
  if (threadIdx.x == 0) {
    a.omax[cur][r] = om;
    if (!has_prev) pmax_out[r] = pm0;
  }
  __syncthreads();
  float2* res = fft_lds<N, false>(bufA, bufB, M, tw);
  float2* dst = a.psi[cur];
  for (int i = threadIdx.x; i < M * N; i += blockDim.x) {
    const int p = i / N, c = i - p * N;
    dst[p * NN + (size_t)r * N + c] = res[i];
  }
}

// ---------------------------------------------------------------- k_cols
template <int N, int WC>
__global__ __launch_bounds__(256) void k_cols(SweepArgs a, int jn) {
  extern __shared__ float2 smem[];
  const int M = a.M;
  float2* tw = smem;
  float2* bufA = tw + N;
  float2* bufB = bufA + M * WC * N;
  __shared__ double redd[16];
  const int it = *a.iter_dev;
  const int s = it * a.J + jn;
  const size_t NN = (size_t)N * N;
  const int nunits = N / WC;
  const int u = xcd_unit(blockIdx.x, nunits);
  const int c0 = u * WC;
  float2* psi = a.psi[s & 1];
  const float* I = a.I + (size_t)jn * NN;

  load_twiddles<N>(tw);
  for (int i = threadIdx.x; i < M * N * WC; i += blockDim.x) {
    const int p = i / (N * WC);
    const int rem = i - p * N * WC;
    const int k = rem / WC, cc = rem - k * WC;
    bufA[(p * WC + cc) * N + k] = psi[p * NN + (size_t)k * N + c0 + cc];
  }
  __syncthreads();
  float2* F = fft_lds<N, false>(bufA, bufB, M * WC, tw);
  float2* G = (F == bufA) ? bufB : bufA;
  // modulus replacement, Eq. 7; the 2-D transform here is unnormalised
  // (N x unitary) and the inverse will be too, so the factor carries 1/N.
  const float invN = 1.0f / (float)N;
  double e = 0.0;
  bool bad = false;
  for (int i = threadIdx.x; i < N * WC; i += blockDim.x) {
    const int k = i / WC, cc = i - k * WC;
    float S = 0.f;
    for (int p = 0; p < M; ++p) S += cabs2(F[(p * WC + cc) * N + k]);
    const float Au = sqrtf(S);
    const float sq = sqrtf(fmaxf(I[(size_t)k * N + c0 + cc], 0.f));
    const float d = Au * invN - sq;
    e += (double)d * (double)d;
    bad |= !isfinite(S);
    const float f = S > 0.f ? sq / Au * invN : 0.f;
    for (int p = 0; p < M; ++p) G[(p * WC + cc) * N + k] = cscale(F[(p * WC + cc) * N + k], f);
  }
  if (bad) flag_status(a.status, MRPIE_STATUS_NONFINITE);
  __syncthreads();
  float2* H = fft_lds<N, true>(G, F, M * WC, tw);
  for (int i = threadIdx.x; i < M * N * WC; i += blockDim.x) {
    const int p = i / (N * WC);
    const int rem = i - p * N * WC;
    const int k = rem / WC, cc = rem - k * WC;
    psi[p * NN + (size_t)k * N + c0 + cc] = H[(p * WC + cc) * N + k];
  }
  e = block_sum(e, redd);
  if (threadIdx.x == 0) a.err_acc[(size_t)it * kErrSlots + u] += e;
}

// ------------------------------------------------------- small kernels
__global__ void k_zero_words(int* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}
__global__ void k_advance(int* iter_dev) {
  if (threadIdx.x == 0) *iter_dev += 1;
}
// per-block partial sums of max(I, 0), fixed order
__global__ __launch_bounds__(256) void k_isum_partial(const float* I, size_t n, double* part) {
  __shared__ double red[16];
  double v = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v += (double)fmaxf(I[i], 0.f);
  v = block_sum(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}
__global__ __launch_bounds__(256) void k_finalize_err(const double* err_acc, const double* part, int nparts,
                                                     int T, float* err_out) {
  __shared__ double red[16];
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += part[i];
  const double isum = block_sum(v, red);
  for (int t = 0; t < T; ++t) {
    double e = 0.0;
    for (int i = threadIdx.x; i < kErrSlots; i += blockDim.x) e += err_acc[(size_t)t * kErrSlots + i];
    e = block_sum(e, red);
    if (threadIdx.x == 0) err_out[t] = (float)(isum > 0.0 ? e / isum : e);
  }
}
__global__ void k_copy(float2* dst, const float2* src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) dst[i] = src[i];
}

// ------------------------------------------------------------ host side
constexpr int kIsumParts = 1024;

struct SweepLayout {
  size_t psi[2], patch[2], probe1, pmax[2], omax[2], box[2], err, isum, iter, total;
};

static SweepLayout sweep_layout(const mrpie_problem* pb, const mrpie_params* pr) {
  SweepLayout L{};
  const size_t NN = (size_t)pb->N * pb->N;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  for (int i = 0; i < 2; ++i) L.psi[i] = take(pb->M * NN * 8);
  for (int i = 0; i < 2; ++i) L.patch[i] = take(NN * 8);
  L.probe1 = take(pb->M * NN * 8);
  for (int i = 0; i < 2; ++i) L.pmax[i] = take(pb->N * 4);
  for (int i = 0; i < 2; ++i) L.omax[i] = take(pb->N * 4);
  for (int i = 0; i < 2; ++i) L.box[i] = take(16);
  L.err = take((size_t)std::max(pr->iterations, 1) * kErrSlots * 8);
  L.isum = take(kIsumParts * 8);
  L.iter = take(16);
  L.total = off;
  return L;
}

static size_t rows_lds(int N, int M) { return (size_t)(N + M * N + N + 6 * M * N) * 8; }
static size_t cols_lds(int N, int M) { return (size_t)(N + 2 * M * kCols * N) * 8; }

template <int N>
static int sweep_impl(const mrpie_problem* pb, const mrpie_params* pr, SweepArgs& a, float* err_out,
                      char* ws, const SweepLayout& L, hipStream_t s) {
  const size_t lr = rows_lds(N, pb->M), lc = cols_lds(N, pb->M);
  if (lr > 65536)
    MRPIE_HIP(hipFuncSetAttribute((const void*)k_rows<N>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr));
  if (lc > 65536)
    MRPIE_HIP(hipFuncSetAttribute((const void*)k_cols<N, kCols>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lc));
  const dim3 blk(256);
  const int J = pb->J, T = pr->iterations;
  auto rows = [&](int jn, int mode) {
    TimingScope ts(TK_ROWS, s);
    hipLaunchKernelGGL(k_rows<N>, dim3(N), blk, lr, s, a, jn, mode);
  };
  auto cols = [&](int jn) {
    TimingScope ts(TK_COLS, s);
    hipLaunchKernelGGL((k_cols<N, kCols>), dim3(N / kCols), blk, lc, s, a, jn);
  };
  for (int it = 0; it < T; ++it) {
    for (int j = 0; j < J; ++j) {
      rows(j, (it == 0 && j == 0) ? ROWS_HEAD : ROWS_MID);
      cols(j);
    }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, (int*)(ws + L.iter));
  }
  rows(0, ROWS_TAIL);
  MRPIE_HIP(hipGetLastError());
  // final probe lives in probe[(T*J)&1]
  if (((long long)T * J) & 1) {
    const size_t n = (size_t)pb->M * pb->N * pb->N;
    hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, a.probe[0], (const float2*)a.probe[1], n);
  }
  if (err_out) {
    const size_t nI = (size_t)J * pb->N * pb->N;
    hipLaunchKernelGGL(k_isum_partial, dim3(kIsumParts), dim3(256), 0, s, a.I, nI, (double*)(ws + L.isum));
    hipLaunchKernelGGL(k_finalize_err, dim3(1), dim3(256), 0, s, (const double*)(ws + L.err),
                       (const double*)(ws + L.isum), kIsumParts, T, err_out);
  }
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

}  // namespace mrpie

using namespace mrpie;

extern "C" {

int mrpie_validate(const mrpie_problem* pb, const mrpie_params* pr) {
  if (!pb || !pr) return fail(MRPIE_EINVAL, "null problem or params");
  if (n_index(pb->N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {64,128,192,256}", pb->N);
  if (pb->M < 1) return fail(MRPIE_EINVAL, "M=%d < 1", pb->M);
  if (pb->M > MRPIE_MAX_MODES) return fail(MRPIE_EUNSUPPORTED, "M=%d > %d", pb->M, MRPIE_MAX_MODES);
  if (pb->J < 1) return fail(MRPIE_EINVAL, "J=%d < 1", pb->J);
  if (pb->H < pb->N || pb->W < pb->N) return fail(MRPIE_EINVAL, "object %dx%d smaller than the probe %d", pb->H, pb->W, pb->N);
  if ((long long)pb->H * pb->W >= (1LL << 31)) return fail(MRPIE_EINVAL, "object too large");
  if ((long long)pb->J * pb->N * pb->N >= (1LL << 40)) return fail(MRPIE_EINVAL, "too many patterns");
  auto finite = [](float v) { return std::isfinite(v); };
  if (!finite(pr->alpha_obj) || !finite(pr->alpha_probe)) return fail(MRPIE_EINVAL, "non-finite step size");
  if (!(pr->beta >= 0.f && pr->beta <= 1.f)) return fail(MRPIE_EINVAL, "beta=%g not in [0,1]", pr->beta);
  if (!(pr->gamma >= 0.f && pr->gamma <= 1.f)) return fail(MRPIE_EINVAL, "gamma=%g not in [0,1]", pr->gamma);
  if (pr->iterations < 0 || pr->iterations > 100000) return fail(MRPIE_EINVAL, "iterations=%d", pr->iterations);
  if (pr->iter_offset < 0) return fail(MRPIE_EINVAL, "iter_offset=%d < 0", pr->iter_offset);
  if (pr->subpixel != 0 && pr->subpixel != 1) return fail(MRPIE_EINVAL, "subpixel must be 0 or 1");
  if (pr->refine != 0 && pr->refine != 1) return fail(MRPIE_EINVAL, "refine must be 0 or 1");
  if (pr->refine) {
    if (pr->upsample < 1 || pr->upsample > 1000) return fail(MRPIE_EINVAL, "upsample=%d not in [1,1000]", pr->upsample);
    if (pr->xcorr_norm != 0 && pr->xcorr_norm != 1) return fail(MRPIE_EINVAL, "xcorr_norm must be 0 or 1");
    if (!(pr->adam_b1 >= 0.f && pr->adam_b1 < 1.f) || !(pr->adam_b2 >= 0.f && pr->adam_b2 < 1.f))
      return fail(MRPIE_EINVAL, "Adam betas must be in [0,1)");
    if (!(pr->adam_eps > 0.f) || !finite(pr->adam_lr)) return fail(MRPIE_EINVAL, "bad Adam lr/eps");
  }
  if (pr->subpixel || pr->refine) return fail(MRPIE_EUNSUPPORTED, "subpixel / refine not built in this library");
  return MRPIE_OK;
}

int mrpie_workspace_size(const mrpie_problem* pb, const mrpie_params* pr, size_t* bytes) {
  int rc = mrpie_validate(pb, pr);
  if (rc) return rc;
  if (!bytes) return fail(MRPIE_EINVAL, "bytes is NULL");
  *bytes = sweep_layout(pb, pr).total;
  return MRPIE_OK;
}

int mrpie_rpie(const mrpie_problem* pb, const mrpie_params* pr, void* obj, void* probe, float* pos,
               float* adam, const float* intens, float* err_out, int32_t* status, void* ws, size_t ws_bytes,
               void* stream) {
  int rc = mrpie_validate(pb, pr);
  if (rc) return rc;
  if (!obj || !probe || !pos || !intens) return fail(MRPIE_EINVAL, "null array pointer");
  if (pr->refine && !adam) return fail(MRPIE_EINVAL, "adam state is NULL with refine = 1");
  const SweepLayout L = sweep_layout(pb, pr);
  if (!ws || ws_bytes < L.total) return fail(MRPIE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
  if (pr->iterations == 0) return MRPIE_OK;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  SweepArgs a{};
  a.H = pb->H; a.W = pb->W; a.N = pb->N; a.M = pb->M; a.J = pb->J; a.T = pr->iterations;
  a.alpha_obj = pr->alpha_obj; a.alpha_probe = pr->alpha_probe; a.beta = pr->beta; a.gamma = pr->gamma;
  a.iter_offset = pr->iter_offset; a.probe_update_start = pr->probe_update_start;
  a.obj = (float2*)obj;
  a.probe[0] = (float2*)probe;
  a.probe[1] = (float2*)(w + L.probe1);
  a.pos = pos;
  a.I = intens;
  for (int i = 0; i < 2; ++i) {
    a.psi[i] = (float2*)(w + L.psi[i]);
    a.patch[i] = (float2*)(w + L.patch[i]);
    a.pmax[i] = (float*)(w + L.pmax[i]);
    a.omax[i] = (float*)(w + L.omax[i]);
    a.box[i] = (int*)(w + L.box[i]);
  }
  a.err_acc = (double*)(w + L.err);
  a.status = status;
  a.iter_dev = (const int*)(w + L.iter);
  rc = launch_init_twiddles(s);
  if (rc) return rc;
  // clear the error accumulators and the iteration counter (fill kernel:
  // safe under graph capture)
  hipLaunchKernelGGL(k_zero_words, dim3(64), dim3(256), 0, s, (int*)(w + L.err),
                     (size_t)pr->iterations * kErrSlots * 2);
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, (int*)(w + L.iter), (size_t)4);
  MRPIE_HIP(hipGetLastError());
  switch (pb->N) {
    case 64: return sweep_impl<64>(pb, pr, a, err_out, w, L, s);
    case 128: return sweep_impl<128>(pb, pr, a, err_out, w, L, s);
    case 192: return sweep_impl<192>(pb, pr, a, err_out, w, L, s);
    default: return sweep_impl<256>(pb, pr, a, err_out, w, L, s);
  }
}

}  // extern "C"
