// The M-rPIE sweep of one reconstruction in one workgroup, for probes whose
// modes fit the LDS together (Methods, "M-rPIE algorithm", Eq. 4-7):
// M * N^2 <= 16384 complex values, i.e. 32^2 x up to 8 modes, 64^2 x up to
// 4, 128^2 x 1.
//
// A 1024-thread workgroup owns the whole job: the probe modes stay in
// registers for the whole call (thread k holds pixels k, k + 1024, ...),
// the exit waves of all modes are written to LDS, transformed there by a
// radix-8/4 Stockham 2-D FFT (rows, then columns), the mode-summed modulus
// replacement (Eq. 7) is applied in place, the inverse 2-D FFT follows, and
// the simultaneous probe (Eq. 5) and object (Eq. 6) updates leave the
// patch in the object with ordinary stores.  The next position's gather
// reads those stores after a workgroup barrier, so rPIE's order holds with
// no device-wide synchronisation at all: one launch covers every position
// and iteration.  Many jobs run as many workgroups of one launch.
//
// LDS layout: mode planes of N rows with a padded pitch of N + 1 values
// (spreads the row-direction butterflies over the banks), plus the N-entry
// twiddle table.  When two copies of the planes fit, the FFT stages
// ping-pong between them (one barrier per stage); otherwise each stage
// reads its inputs into registers, synchronises, and writes in place.
#include <algorithm>
#include <vector>

#include "sweep.hpp"

namespace mrpie {

constexpr int kLdsThreads = 1024;
// float2 values of dynamic LDS a variant may use (160 KiB less the static
// reduction scratch)
constexpr int kLdsBudget = 20480 - 64;

// threadIdx.x as a value the compiler cannot see through: index arithmetic
// derived from it stays inside the position loop instead of being hoisted
// out of it (which would keep hundreds of addresses live and spill).
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

template <int N, int MM>
struct LdsCfg {
  static constexpr int NN = N * N;
  static constexpr int PITCH = N + 1;
  static constexpr int PLANE = N * PITCH;
  static constexpr int PPT = NN / kLdsThreads;  // pixels per thread
  static constexpr int FIELD = MM * PLANE;
  static constexpr bool PP = 2 * FIELD + N <= kLdsBudget;
  static constexpr int BYTES = (FIELD * (PP ? 2 : 1) + N) * 8;
  static_assert(FIELD + N <= kLdsBudget, "modes do not fit the LDS");
  static_assert(PPT >= 1 && NN % kLdsThreads == 0, "unsupported N");
};

// One Stockham stage over M planes along x (AY = false) or y (AY = true).
// PP: src and dst are different buffers; otherwise src == dst and every
// thread reads all of its inputs before anyone writes.
template <int N, int R, int NS, bool INV, bool AY, int MM, bool PP>
__device__ __forceinline__ void lstage(const float2* src, float2* dst, int M, const float2* __restrict__ tw) {
  using C = LdsCfg<N, MM>;
  constexpr int Q = N / R;
  constexpr int TWS = N / (NS * R);
  constexpr int PER = N * Q;  // butterflies per plane
  constexpr int BPT = (MM * PER + kLdsThreads - 1) / kLdsThreads;
  constexpr int ES = AY ? C::PITCH : 1;  // element stride along the transform
  const int total = M * PER;
  const int tx = opaque_tid();
  float2 v[BPT][R];
  int base[BPT], jj[BPT];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int t = tx + b * kLdsThreads;
    base[b] = 0;
    jj[b] = 0;
    if (t < total) {
      const int p = t / PER, rem = t - p * PER;
      int j, bs;
      if constexpr (AY) {  // consecutive threads: consecutive columns x
        j = rem / N;
        bs = p * C::PLANE + (rem - j * N);
      } else {             // consecutive threads: consecutive j within a row
        const int y = rem / Q;
        j = rem - y * Q;
        bs = p * C::PLANE + y * C::PITCH;
      }
      base[b] = bs;
      jj[b] = j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = src[bs + (j + r * Q) * ES];
    }
  }
  if constexpr (!PP) __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int t = tx + b * kLdsThreads;
    if (t < total) {
      const int j = jj[b];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * TWS];
          if constexpr (INV) w.y = -w.y;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      dftR<R, INV>(v[b]);
      const int o = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[base[b] + (o + r * NS) * ES] = v[b][r];
    }
  }
  __syncthreads();
}

// Unnormalised 2-D transform of M planes (rows, then columns).  Returns the
// buffer that holds the result (a, or b when the stages ping-pong).
template <int N, bool INV, int MM>
__device__ __forceinline__ float2* lds_fft2(float2* a, float2* b, int M, const float2* tw) {
  using C = LdsCfg<N, MM>;
  constexpr bool PP = C::PP;
  using P = Plan8<N>;
  constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2];
  static_assert(P::R[3] == 1, "plan too long");
  float2* cur = a;
  float2* oth = PP ? b : a;
#define MRPIE_LSTEP(R_, NS_, AY_)                                        \
  lstage<N, R_, NS_, INV, AY_, MM, PP>(cur, PP ? oth : cur, M, tw);      \
  if constexpr (PP) {                                                    \
    float2* t_ = cur;                                                    \
    cur = oth;                                                           \
    oth = t_;                                                            \
  }
  MRPIE_LSTEP(R0, 1, false)
  MRPIE_LSTEP(R1, R0, false)
  if constexpr (R2 > 1) { MRPIE_LSTEP(R2, R0 * R1, false) }
  MRPIE_LSTEP(R0, 1, true)
  MRPIE_LSTEP(R1, R0, true)
  if constexpr (R2 > 1) { MRPIE_LSTEP(R2, R0 * R1, true) }
#undef MRPIE_LSTEP
  return cur;
}

template <int N, int MM>
__device__ __forceinline__ void lds_sweep_body(const Common& cm, const JobRec& jb, float2* smem, float* red,
                                               double* redd) {
  using C = LdsCfg<N, MM>;
  constexpr int NN = C::NN, PPT = C::PPT;
  constexpr bool KEEP = MM * PPT <= 8;
  const int M = jb.M, H = jb.H, W = jb.W, J = jb.J;
  const int tid0 = threadIdx.x;
  float2* fa = smem;
  float2* fb = C::PP ? smem + C::FIELD : smem;
  float2* tw = smem + C::FIELD * (C::PP ? 2 : 1);
  load_twiddles<N>(tw);
  const WsLayout L = ws_layout(N, M, jb.T);
  double* errs = (double*)(jb.ws + L.err);
  double* isums = (double*)(jb.ws + L.isum);
  const float invN = 1.0f / (float)N;

  // the probe modes at this thread's pixels, for the whole call
  float2 Pr[MM][PPT];
#pragma unroll
  for (int p = 0; p < MM; ++p)
#pragma unroll
    for (int k = 0; k < PPT; ++k) Pr[p][k] = p < M ? jb.probe[(size_t)p * NN + tid0 + k * kLdsThreads] : make_float2(0.f, 0.f);

  for (int it = 0; it < jb.T; ++it) {
    const bool upd_p = cm.iter_offset + it >= cm.probe_update_start;
    double eacc = 0.0, iacc = 0.0;
    for (int j = 0; j < J; ++j) {
      const int ny = box_corner(jb.pos[2 * j], H - N, jb.status);
      const int nx = box_corner(jb.pos[2 * j + 1], W - N, jb.status);
      const float* Ij = jb.I + (size_t)j * NN;
      float2* ob = jb.obj + (size_t)ny * W + nx;

      // ---- gather (Eq. 4) and the maxima of the denominators.  With few
      //      values per thread the patch and the pattern stay in registers
      //      across the transforms; otherwise (KEEP false) they are read
      //      again where they are used, which keeps the kernel within its
      //      128 registers.
      int tid = opaque_tid();
      float2 o[PPT];
      float Iv[PPT];
      float om = 0.f, pm = 0.f;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int i = tid + k * kLdsThreads, y = i / N, x = i - y * N;
        if constexpr (KEEP) Iv[k] = Ij[i];
        o[k] = ob[(size_t)y * W + x];
      }
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        om = fmaxf(om, cabs2(o[k]));
        float ps = 0.f;
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) ps += cabs2(Pr[p][k]);
        pm = fmaxf(pm, ps);
      }
      float omax, pmax;
      block_max2(om, pm, red, omax, pmax);

      // ---- exit waves (Eq. 1) into the LDS planes
      tid = opaque_tid();
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int i = tid + k * kLdsThreads, y = i / N, x = i - y * N;
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) fa[p * C::PLANE + y * C::PITCH + x] = cmul(Pr[p][k], o[k]);
      }
      __syncthreads();
      float2* F = lds_fft2<N, false, MM>(fa, fb, M, tw);

      // ---- mode-summed modulus replacement (Eq. 7); the forward and
      //      inverse transforms are unnormalised, so the factor carries 1/N
      bool bad = false;
      tid = opaque_tid();
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int i = tid + k * kLdsThreads, y = i / N, x = i - y * N;
        const int li = y * C::PITCH + x;
        float S = 0.f;
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) S += cabs2(F[p * C::PLANE + li]);
        // hardware reciprocal square root and square root (about 1 ulp)
        const float rs = S > 0.f ? __builtin_amdgcn_rsqf(S) : 0.f;
        const float Au = S * rs;
        const float sq = __builtin_amdgcn_sqrtf(fmaxf(KEEP ? Iv[k] : Ij[i], 0.f));
        const float d = Au * invN - sq;
        eacc += (double)d * (double)d;
        iacc += (double)fmaxf(KEEP ? Iv[k] : Ij[i], 0.f);
        bad |= !isfinite(S);
        const float f = sq * rs * invN;
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) F[p * C::PLANE + li] = cscale(F[p * C::PLANE + li], f);
      }
      __syncthreads();
      float2* G = lds_fft2<N, true, MM>(F, F == fa ? fb : fa, M, tw);

      // ---- probe (Eq. 5) and object (Eq. 6) updates from the pre-update o, P
      tid = opaque_tid();
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int i = tid + k * kLdsThreads, y = i / N, x = i - y * N;
        const int li = y * C::PITCH + x;
        const float2 ok = KEEP ? o[k] : ob[(size_t)y * W + x];
        const float dP = cm.beta * omax + (1.f - cm.beta) * cabs2(ok);
        const float gP = (upd_p && dP != 0.f) ? cm.alpha_probe * __builtin_amdgcn_rcpf(dP) : 0.f;
        float Ps = 0.f, Pn = 0.f;
        float2 num = make_float2(0.f, 0.f);
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) {
            const float2 P = Pr[p][k];
            const float2 d = csub(G[p * C::PLANE + li], cmul(P, ok));
            num = cadd(num, cmulc(d, P));
            Ps += cabs2(P);
            Pr[p][k] = cadd(P, cscale(cmulc(d, ok), gP));
            Pn += cabs2(Pr[p][k]);
          }
        const float dO = cm.gamma * pmax + (1.f - cm.gamma) * Ps;
        const float g = dO != 0.f ? cm.alpha_obj * __builtin_amdgcn_rcpf(dO) : 0.f;
        const float2 on = cadd(ok, cscale(num, g));
        bad |= !(isfinite(on.x) && isfinite(on.y) && isfinite(Pn));
        ob[(size_t)y * W + x] = on;
      }
      if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
      // the next gather reads these stores; the LDS planes are reused
      __syncthreads();
    }
    eacc = block_sum(eacc, redd);
    iacc = block_sum(iacc, redd);
    if (tid0 == 0) {
      errs[(size_t)it * kErrSlots] = eacc;
      isums[(size_t)it * kErrSlots] = iacc;
    }
  }
#pragma unroll
  for (int p = 0; p < MM; ++p)
#pragma unroll
    for (int k = 0; k < PPT; ++k)
      if (p < M) jb.probe[(size_t)p * NN + tid0 + k * kLdsThreads] = Pr[p][k];
}

// variant of (N, M): capacity MM in modes; -1 when the modes do not fit
static __host__ __device__ inline int lds_variant(int N, int M) {
  if (M < 1) return -1;
  if (N == 32 && M <= 8) return 0;
  if (N == 64 && M <= 1) return 1;
  if (N == 64 && M <= 2) return 2;
  if (N == 64 && M <= 4) return 3;
  if (N == 128 && M <= 1) return 4;
  return -1;
}

__global__ __launch_bounds__(1024) void k_lds_sweep(const LaunchArgs a) {
  extern __shared__ float2 smem[];
  __shared__ float red[32];
  __shared__ double redd[16];
  const JobRec& jb = a.job[blockIdx.x];
  switch (lds_variant(jb.N, jb.M)) {
    case 0: lds_sweep_body<32, 8>(a.c, jb, smem, red, redd); break;
    case 1: lds_sweep_body<64, 1>(a.c, jb, smem, red, redd); break;
    case 2: lds_sweep_body<64, 2>(a.c, jb, smem, red, redd); break;
    case 3: lds_sweep_body<64, 4>(a.c, jb, smem, red, redd); break;
    case 4: lds_sweep_body<128, 1>(a.c, jb, smem, red, redd); break;
    default: break;
  }
}

static size_t lds_bytes(int v) {
  switch (v) {
    case 0: return LdsCfg<32, 8>::BYTES;
    case 1: return LdsCfg<64, 1>::BYTES;
    case 2: return LdsCfg<64, 2>::BYTES;
    case 3: return LdsCfg<64, 4>::BYTES;
    case 4: return LdsCfg<128, 1>::BYTES;
    default: return 0;
  }
}

bool lds_sweep_fits(int N, int M) { return lds_variant(N, M) >= 0; }

int run_lds_sweep(const Common& c, const JobRec* jobs, int njobs, float* const* err_out, hipStream_t s) {
  int rc = launch_init_twiddles(s);
  if (rc) return rc;
  for (int c0 = 0; c0 < njobs; c0 += kMaxJobsPerLaunch) {
    const int nb = std::min(kMaxJobsPerLaunch, njobs - c0);
    LaunchArgs a{};
    a.c = c;
    a.njobs = nb;
    size_t lds = 0;
    std::vector<float*> eo((size_t)nb);
    for (int b = 0; b < nb; ++b) {
      a.job[b] = jobs[c0 + b];
      const int v = lds_variant(jobs[c0 + b].N, jobs[c0 + b].M);
      if (v < 0) return fail(MRPIE_EUNSUPPORTED, "job does not fit the LDS sweep");
      lds = std::max(lds, lds_bytes(v));
      eo[(size_t)b] = err_out ? err_out[c0 + b] : nullptr;
    }
    MRPIE_HIP(ensure_lds((const void*)k_lds_sweep, lds));
    launch_zero_err(a, nb, s);
    launch_k(TK_LDS, k_lds_sweep, dim3(nb), dim3(kLdsThreads), lds, s, a);
    launch_finish(a, nb, eo.data(), s, false);
    MRPIE_HIP(hipGetLastError());
  }
  return MRPIE_OK;
}

}  // namespace mrpie
