// M-rPIE sweep with subpixel positions and XCORR_A position refinement
// (Methods, "M-rPIE algorithm", Eq. 4-7, and "Adam-based position
// refinement", Eq. 8-9, Alg. 1), on gfx950.
//
// A position at pos = n + f (n = floor(pos + 0.5)) is cropped at n and moved
// by the fraction f with a band-limited Fourier phase ramp, o = S_f(crop);
// the object update is moved back, O[box] += S_{-f}(delta_o).  Each Fourier
// move costs one 2-D FFT round trip, so a position takes six launches
// (R = row pass over probe rows, C = column pass over detector columns):
//
//   k_sp_gather  (R, s-1 -> s)  inverse row FFT of S_{-f} delta_o of step
//                s-1, object update of the box rows that are rows of box s
//                or leave it; gather crop rows of box s (merged), row FFT
//   k_sp_ramp    (C, s)  column FFT, x e^{+2 pi i k.f/N} / N^2, inverse
//   k_sp_exit    (R, s)  inverse row FFT -> o_s; exit waves P_p o_s, row FFTs
//   k_cols       (C, s)  modulus replacement (Eq. 7), shared with the
//                integer-crop sweep
//   k_sp_update  (R, s)  inverse row FFTs -> psi'; probe update of row r
//                (Eq. 5); delta_o row r (Eq. 6); row FFT of delta_o
//   k_sp_ramp    (C, s)  column FFT, x e^{-2 pi i k.f/N} / N^2, inverse
//
// With refinement the patch before (o_s) and after (o_s + delta_o) the
// update are recorded for the registration batch that follows each
// iteration.  Every workgroup writes only its own rows / columns of each
// buffer, so the path is deterministic like the integer-crop sweep.
#include <algorithm>
#include <cmath>

#include "register.hpp"
#include "sweep.hpp"

namespace mrpie {

__device__ __forceinline__ size_t pick2(const size_t (&a)[2], int i) { return i ? a[1] : a[0]; }

struct SpArgs {
  LaunchArgs la;  // one job (la.job[0])
  int subpixel;
  float2* reg_ref;
  float2* reg_mov;
  int record_start;
};

__device__ __forceinline__ bool recording(const SpArgs& a, const JobRec& jb, int t) {
  return a.reg_ref && (a.la.c.iter_offset + t / jb.J) >= a.record_start;
}

// ---------------------------------------------------------------- gather
template <int N>
__device__ void sp_gather(const SpArgs& a, const JobRec& jb, int t, int mode, float2* smem) {
  const int r = blockIdx.x;
  const int total = jb.J * jb.T;
  if (r >= N) return;
  const bool has_prev = mode != 0, has_next = mode != 2;
  const int cur = t & 1, prv = (t + 1) & 1;
  const int jn = has_next ? t % jb.J : 0;
  (void)total;
  const WsLayout L = ws_layout(N, jb.M, jb.T);
  char* ws = jb.ws;
  const int c = threadIdx.x;
  const bool lane = c < N;
  float2* tw = smem;
  float2* orow = tw + N;
  float2* A = orow + N;       // 2*N
  float2* B = A + 2 * N;      // 2*N

  int ny_n = 0, nx_n = 0;
  float fy = 0.f, fx = 0.f;
  if (has_next) {
    const float py = jb.pos[2 * jn], px = jb.pos[2 * jn + 1];
    ny_n = box_corner(py, jb.H - N, jb.status);
    nx_n = box_corner(px, jb.W - N, jb.status);
    if (a.subpixel) {
      fy = py - (float)ny_n;
      fx = px - (float)nx_n;
      if (!(fy >= -0.5f && fy < 0.5f)) fy = 0.f;  // clamped corner: no move
      if (!(fx >= -0.5f && fx < 0.5f)) fx = 0.f;
    }
  }
  const int* bp = (const int*)(ws + pick2(L.box, prv));
  int ny_p = 0, nx_p = 0, rb1 = -1, rb2 = -1;
  if (has_prev) {
    ny_p = bp[0];
    nx_p = bp[1];
    if (has_next) {
      const int dy = ny_n - ny_p;
      if (r + dy >= 0 && r + dy < N) rb1 = r + dy;
      if (dy > 0 && r < min(N, dy)) rb2 = r;
      if (dy < 0 && r < min(N, -dy)) rb2 = max(0, N + dy) + r;
    } else {
      rb1 = r;
    }
  }
  const float2* db = (const float2*)(ws + L.db);
  float2 d1 = make_float2(0.f, 0.f), d2 = d1, o1 = d1, o2 = d1, og = d1;
  if (lane) {
    if (rb1 >= 0) {
      d1 = db[(size_t)rb1 * N + c];
      o1 = jb.obj[(size_t)(ny_p + rb1) * jb.W + nx_p + c];
    }
    if (rb2 >= 0) {
      d2 = db[(size_t)rb2 * N + c];
      o2 = jb.obj[(size_t)(ny_p + rb2) * jb.W + nx_p + c];
    }
    if (has_next) {
      const int gx = nx_n + c;
      if (!(rb1 >= 0 && gx >= nx_p && gx < nx_p + N)) og = jb.obj[(size_t)(ny_n + r) * jb.W + gx];
    }
  }
  if (has_next && r == 0 && c == 0) {
    int* bc = (int*)(ws + pick2(L.box, cur));
    bc[0] = ny_n;
    bc[1] = nx_n;
    bc[2] = __float_as_int(fy);
    bc[3] = __float_as_int(fx);
  }
  load_twiddles<N>(tw);
  if (has_prev) {
    if (lane) {
      A[c] = d1;
      A[N + c] = d2;
    }
    __syncthreads();
    float2* R = fft_lds<N, true>(A, B, 2, tw);
    bool bad = false;
    if (lane) {
      if (rb1 >= 0) {
        const float2 on = cadd(o1, R[c]);
        jb.obj[(size_t)(ny_p + rb1) * jb.W + nx_p + c] = on;
        orow[c] = on;
        bad |= !(isfinite(on.x) && isfinite(on.y));
      }
      if (rb2 >= 0) {
        const float2 on = cadd(o2, R[N + c]);
        jb.obj[(size_t)(ny_p + rb2) * jb.W + nx_p + c] = on;
        bad |= !(isfinite(on.x) && isfinite(on.y));
      }
    }
    if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
    __syncthreads();
  }
  if (!has_next) return;
  if (lane) {
    const int gx = nx_n + c;
    A[c] = (rb1 >= 0 && gx >= nx_p && gx < nx_p + N) ? orow[gx - nx_p] : og;
  }
  __syncthreads();
  float2* R = fft_lds<N, false>(A, B, 1, tw);
  float2* cb = (float2*)(ws + L.cb);
  if (lane) cb[(size_t)r * N + c] = R[c];
}

// ---------------------------------------------------------------- ramp
// Column pass of the Fourier move: column FFT of buffer `which` (0 = crop
// spectra, +f; 1 = update spectra, -f), phase ramp and the 1/N^2 of the
// unnormalised 2-D round trip, inverse column FFT, in place.
template <int N>
__device__ void sp_ramp(const SpArgs& a, const JobRec& jb, int t, int which, float2* smem) {
  const int u = xcd_unit(blockIdx.x, gridDim.x);
  if (u >= N || t >= jb.J * jb.T) return;
  const WsLayout L = ws_layout(N, jb.M, jb.T);
  char* ws = jb.ws;
  float2* buf = (float2*)(ws + (which == 0 ? L.cb : L.db));
  const int* bc = (const int*)(ws + pick2(L.box, t & 1));
  const float fy = __int_as_float(bc[2]), fx = __int_as_float(bc[3]);
  const float sg = which == 0 ? 1.f : -1.f;
  const int k = threadIdx.x;
  const bool lane = k < N;
  float2* tw = smem;
  float2* A = tw + N;
  float2* B = A + N;
  float2 v = make_float2(0.f, 0.f);
  if (lane) v = buf[(size_t)k * N + u];
  load_twiddles<N>(tw);
  if (lane) A[k] = v;
  __syncthreads();
  float2* F = fft_lds<N, false>(A, B, 1, tw);
  float2* G = (F == A) ? B : A;
  if (lane) {
    const int ky = k < N / 2 ? k : k - N;   // fftfreq order, Nyquist -> -N/2
    const int kx = u < N / 2 ? u : u - N;
    float sn, cs;
    sincospif(sg * 2.f * ((float)ky * fy + (float)kx * fx) / (float)N, &sn, &cs);
    const float s2 = 1.f / ((float)N * (float)N);
    G[k] = cscale(cmul(F[k], make_float2(cs, sn)), s2);
  }
  __syncthreads();
  float2* H = fft_lds<N, true>(G, F, 1, tw);
  if (lane) buf[(size_t)k * N + u] = H[k];
}

// ---------------------------------------------------------------- exit waves
template <int N>
__device__ void sp_exit(const SpArgs& a, const JobRec& jb, int t, float2* smem) {
  constexpr int MM = MRPIE_MAX_MODES;
  const int r = blockIdx.x;
  if (r >= N || t >= jb.J * jb.T) return;
  const int M = jb.M;
  const int cur = t & 1, jn = t % jb.J;
  const WsLayout L = ws_layout(N, M, jb.T);
  char* ws = jb.ws;
  const size_t NN = (size_t)N * N;
  const int c = threadIdx.x;
  const bool lane = c < N;
  float2* tw = smem;
  float2* A = tw + N;          // (M+1)*N
  float2* B = A + (M + 1) * N; // (M+1)*N
  __shared__ float redf[16];
  const float2* Pc = cur == 0 ? jb.probe : (const float2*)(ws + L.probe1);
  float2 cbv = make_float2(0.f, 0.f);
  float2 P[MM];
  if (lane) {
    cbv = ((const float2*)(ws + L.cb))[(size_t)r * N + c];
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) P[p] = Pc[p * NN + (size_t)r * N + c];
  }
  load_twiddles<N>(tw);
  if (lane) A[c] = cbv;
  __syncthreads();
  float2* R = fft_lds<N, true>(A, B, 1, tw);
  float2* W = (R == A) ? B : A;
  float om = 0.f, pm = 0.f;
  if (lane) {
    const float2 o = R[c];
    ((float2*)(ws + pick2(L.patch, cur)))[(size_t)r * N + c] = o;
    if (recording(a, jb, t)) a.reg_ref[((size_t)jn * N + r) * N + c] = o;
    om = cabs2(o);
    float ps = 0.f;
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        ps += cabs2(P[p]);
        W[p * N + c] = cmul(P[p], o);
      }
    pm = ps;
  }
  om = block_max(om, redf);
  pm = block_max(pm, redf + 8);
  if (threadIdx.x == 0) {
    ((float*)(ws + pick2(L.omax, cur)))[r] = om;
    ((float*)(ws + pick2(L.pmax, cur)))[r] = pm;
  }
  float2* S = fft_lds<N, false>(W, R, M, tw);
  float2* dst = (float2*)(ws + pick2(L.psi, cur));
  for (int i = threadIdx.x; i < M * N; i += blockDim.x) {
    const int p = i / N, cc = i - p * N;
    dst[p * NN + (size_t)r * N + cc] = S[i];
  }
}

// ---------------------------------------------------------------- updates
template <int N>
__device__ void sp_update(const SpArgs& a, const JobRec& jb, int t, float2* smem) {
  constexpr int MM = MRPIE_MAX_MODES;
  const int r = blockIdx.x;
  if (r >= N || t >= jb.J * jb.T) return;
  const int M = jb.M;
  const int cur = t & 1, nxt = (t + 1) & 1, jn = t % jb.J;
  const Common& cm = a.la.c;
  const WsLayout L = ws_layout(N, M, jb.T);
  char* ws = jb.ws;
  const size_t NN = (size_t)N * N;
  const int c = threadIdx.x;
  const bool lane = c < N;
  float2* tw = smem;
  float2* A = tw + N;      // M*N
  float2* B = A + M * N;   // M*N
  __shared__ float redf[16];
  const float2* Pold = cur == 0 ? jb.probe : (const float2*)(ws + L.probe1);
  float2* Pnew = nxt == 0 ? jb.probe : (float2*)(ws + L.probe1);
  const float2* psi = (const float2*)(ws + pick2(L.psi, cur));
  float2 pv[MM], P[MM];
  float2 o = make_float2(0.f, 0.f);
  float om_in = 0.f, pm_in = 0.f;
  if (lane) {
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        pv[p] = psi[p * NN + (size_t)r * N + c];
        P[p] = Pold[p * NN + (size_t)r * N + c];
      }
    o = ((const float2*)(ws + pick2(L.patch, cur)))[(size_t)r * N + c];
    om_in = ((const float*)(ws + pick2(L.omax, cur)))[c];
    pm_in = ((const float*)(ws + pick2(L.pmax, cur)))[c];
  }
  load_twiddles<N>(tw);
  if (lane) {
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) A[p * N + c] = pv[p];
  }
  const float omax = block_max(om_in, redf);
  const float pmaxv = block_max(pm_in, redf + 8);
  float2* R = fft_lds<N, true>(A, B, M, tw);
  float2* W = (R == A) ? B : A;
  const int it_abs = cm.iter_offset + t / jb.J;
  const bool upd_p = it_abs >= cm.probe_update_start;
  bool bad = false;
  if (lane) {
    const float o2 = cabs2(o);
    const float dP = cm.beta * omax + (1.f - cm.beta) * o2;
    const float gp = (upd_p && dP != 0.f) ? cm.alpha_probe / dP : 0.f;
    float Ps = 0.f;
    float2 num = make_float2(0.f, 0.f);
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        const float2 d = csub(R[p * N + c], cmul(P[p], o));
        num = cadd(num, cmulc(d, P[p]));
        Ps += cabs2(P[p]);
        const float2 Pn = cadd(P[p], cscale(cmulc(d, o), gp));
        Pnew[p * NN + (size_t)r * N + c] = Pn;
        bad |= !(isfinite(Pn.x) && isfinite(Pn.y));
      }
    const float dO = cm.gamma * pmaxv + (1.f - cm.gamma) * Ps;
    const float go = dO != 0.f ? cm.alpha_obj / dO : 0.f;
    const float2 dlt = cscale(num, go);
    if (recording(a, jb, t)) a.reg_mov[((size_t)jn * N + r) * N + c] = cadd(o, dlt);
    W[c] = dlt;
  }
  if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
  __syncthreads();
  float2* S = fft_lds<N, false>(W, R, 1, tw);
  if (lane) ((float2*)(ws + L.db))[(size_t)r * N + c] = S[c];
}

// ---------------------------------------------------------------- kernels
#define MRPIE_DISPATCH(FN, ...)                         \
  switch (jb.N) {                                       \
    case 32: FN<32>(__VA_ARGS__); break;                \
    case 64: FN<64>(__VA_ARGS__); break;                \
    case 128: FN<128>(__VA_ARGS__); break;              \
    case 192: FN<192>(__VA_ARGS__); break;              \
    default: FN<256>(__VA_ARGS__); break;               \
  }

__global__ __launch_bounds__(256) void k_sp_gather(const SpArgs a, int t, int mode) {
  extern __shared__ float2 smem[];
  const JobRec& jb = a.la.job[0];
  MRPIE_DISPATCH(sp_gather, a, jb, t, mode, smem)
}
__global__ __launch_bounds__(256) void k_sp_ramp(const SpArgs a, int t, int which) {
  extern __shared__ float2 smem[];
  const JobRec& jb = a.la.job[0];
  MRPIE_DISPATCH(sp_ramp, a, jb, t, which, smem)
}
__global__ __launch_bounds__(256) void k_sp_exit(const SpArgs a, int t) {
  extern __shared__ float2 smem[];
  const JobRec& jb = a.la.job[0];
  MRPIE_DISPATCH(sp_exit, a, jb, t, smem)
}
__global__ __launch_bounds__(256) void k_sp_update(const SpArgs a, int t) {
  extern __shared__ float2 smem[];
  const JobRec& jb = a.la.job[0];
  MRPIE_DISPATCH(sp_update, a, jb, t, smem)
}

// the modulus column pass of the integer-crop sweep (sweep.hip)

int run_sweep_subpixel(const Common& c, const JobRec& jb, const SubpixelExtra& ex, int it0, int iters, bool head,
                       bool tail, hipStream_t s) {
  return run_sweep_subpixel_range(c, jb, ex, it0 * jb.J, (it0 + iters) * jb.J, head, tail, s);
}

int run_sweep_subpixel_range(const Common& c, const JobRec& jb, const SubpixelExtra& ex, int t0, int t1, bool head,
                             bool tail, hipStream_t s) {
  int rc = launch_init_twiddles(s);
  if (rc) return rc;
  SpArgs a{};
  a.la.c = c;
  a.la.njobs = 1;
  a.la.job[0] = jb;
  a.subpixel = ex.subpixel;
  a.reg_ref = ex.reg_ref;
  a.reg_mov = ex.reg_mov;
  a.record_start = ex.record_start;
  const int N = jb.N, M = jb.M;
  const size_t lg = (size_t)(N + N + 4 * N) * 8;
  const size_t le = (size_t)(N + 2 * (M + 1) * N) * 8;
  const size_t lu = (size_t)(N + 2 * M * N) * 8;
  const size_t lr = (size_t)(N + 2 * N) * 8;
  MRPIE_HIP(ensure_lds((const void*)k_sp_exit, le));
  MRPIE_HIP(ensure_lds((const void*)k_sp_update, lu));
  const dim3 g(N), blk(256);
  for (int t = t0; t < t1; ++t) {
    hipLaunchKernelGGL(k_sp_gather, g, blk, lg, s, a, t, (t == t0 && head) ? 0 : 1);
    hipLaunchKernelGGL(k_sp_ramp, g, blk, lr, s, a, t, 0);
    hipLaunchKernelGGL(k_sp_exit, g, blk, le, s, a, t);
    launch_cols_pass(a.la, N, 1, t, s);
    hipLaunchKernelGGL(k_sp_update, g, blk, lu, s, a, t);
    hipLaunchKernelGGL(k_sp_ramp, g, blk, lr, s, a, t, 1);
  }
  if (tail) hipLaunchKernelGGL(k_sp_gather, g, blk, lg, s, a, t1, 2);
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

}  // namespace mrpie
