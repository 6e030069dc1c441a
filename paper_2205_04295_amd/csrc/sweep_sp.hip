// M-rPIE sweep with subpixel positions and XCORR_A position refinement
// (Methods, "M-rPIE algorithm", Eq. 4-7, and "Adam-based position
// refinement", Eq. 8-9, Alg. 1), on gfx950.
//
// A position at pos = n + f (n = floor(pos + 0.5)) is cropped at n and moved
// by the fraction f with a band-limited Fourier phase ramp, o = S_f(crop);
// the object update is moved back, O[box] += S_{-f}(delta_o).  The ramp
// e^{2 pi i (k_y f_y + k_x f_x) / N} factors into one ramp per axis, so the
// move along x is a row FFT, ramp and inverse row FFT inside a row pass and
// the move along y the same inside a column pass; both ride on the passes
// that the exit waves' 2-D FFT needs anyway, and a position takes four
// launches (R = one workgroup per patch row, C = one per patch column):
//
//   k_sp_rows_gather (R, s-1 -> s)  x back-move of delta_o of step s-1 and
//                    object update of the box rows that are rows of box s or
//                    leave it; gather crop rows of box s (merged), x move
//   k_sp_cols_exit   (C, s)  y move -> o_s; exit waves P_p o_s (Eq. 4);
//                    column FFTs; maxima of |o|^2 and sum_p |P_p|^2
//   k_sp_rows_mod    (R, s)  row FFTs, mode-summed modulus replacement
//                    (Eq. 7), inverse row FFTs
//   k_sp_cols_update (C, s)  inverse column FFTs -> psi'; probe update (Eq. 5)
//                    and delta_o (Eq. 6) of column u; y back-move of delta_o
//
// Near field (Eq. 2 with a general D_z): the Fresnel transfer function
// H(k) = exp(-i pi (k_y^2 + k_x^2) / N_F) also factors per axis, so
// D_z = F^-1 H F is a y propagation (column FFT, h_y, inverse column FFT)
// followed by an x propagation (the same along rows).  The exit-wave column
// pass propagates along y, the modulus row pass propagates along x, applies
// the modulus constraint in the detector plane and propagates back along x
// with conj(h_x), and the update column pass propagates back along y with
// conj(h_y): still four launches per position.
//
// XCORR_B (refinement against the measured data) records the modelled
// detector amplitude A_j (before the modulus replacement) and sqrt(I_j) in
// the modulus row pass, as the pair the registration compares.
//
// A move whose fraction is exactly 0 is skipped (the crop is used as is), so
// integer positions take no Fourier round trip at all.  With refinement the
// patch before (o_s) and after (o_s + delta_o) the update are recorded for
// the registration.  Every workgroup writes only its own rows / columns of
// each buffer, so the path is deterministic like the integer-crop sweep.
#include <algorithm>
#include <cmath>

#include "register.hpp"
#include "sweep.hpp"

namespace mrpie {

// Every kernel of this file runs 256 threads per workgroup.
constexpr int kSpThreads = 256;


struct SpArgs {
  Common c;
  JobRec jb;
  int subpixel;
  float2* reg_ref;
  float2* reg_mov;
  int record_start;
  int xcb;        // 1: record (A_j, sqrt(I_j)) for XCORR_B, 0: (o_j, o'_j) for XCORR_A
  float fresnel;  // Fresnel number of the N x N window; 0: far field
};

__device__ __forceinline__ bool recording(const SpArgs& a, int t) {
  return a.reg_ref && (a.c.iter_offset + t / a.jb.J) >= a.record_start;
}

// One axis of the Fresnel transfer function with the 1/N of that axis'
// unnormalised round trip: exp(sg i pi ks^2 / N_F) / N for FFT index k
// (signed frequency ks in fftfreq order).  The phase is reduced in double
// precision (ks^2 / N_F reaches 10^4 rad).
__device__ __forceinline__ float2 fresnel1(int k, float nf, float sg, int N) {
  const int ks = k < N / 2 ? k : k - N;
  double sn, cs;
  sincospi((double)sg * (double)(ks * ks) / (double)nf, &sn, &cs);
  const double s = 1.0 / (double)N;
  return make_float2((float)(cs * s), (float)(sn * s));
}

// Box corner and fraction of position j; the fraction is 0 for a clamped
// corner and with subpixel moves off.  The positions do not change within a
// launch sequence (the refining sweep moves them only after its last step of
// an iteration), so every pass recomputes the boxes it needs.
__device__ __forceinline__ void box_frac(const SpArgs& a, int j, int N, int* ny, int* nx, float* fy, float* fx,
                                         int* status) {
  const JobRec& jb = a.jb;
  const float py = jb.pos[2 * j], px = jb.pos[2 * j + 1];
  *ny = box_corner(py, jb.H - N, status);
  *nx = box_corner(px, jb.W - N, status);
  float y = 0.f, x = 0.f;
  if (a.subpixel) {
    y = py - (float)*ny;
    x = px - (float)*nx;
    if (!(y >= -0.5f && y < 0.5f)) y = 0.f;
    if (!(x >= -0.5f && x < 0.5f)) x = 0.f;
  }
  *fy = y;
  *fx = x;
}

// e^{sg 2 pi i k f / N} / N for FFT index k (signed frequency in fftfreq
// order, Nyquist -> -N/2): one axis of the ramp and the 1/N of that axis'
// unnormalised round trip.
__device__ __forceinline__ float2 ramp1(int k, float f, float sg, int N) {
  const int ks = k < N / 2 ? k : k - N;
  float sn, cs;
  sincospif(sg * 2.f * (float)ks * f / (float)N, &sn, &cs);
  const float s = 1.f / (float)N;
  return make_float2(cs * s, sn * s);
}

// ---------------------------------------------------------------- R: update + gather
template <int N>
__device__ void sp_rows_gather(const SpArgs& a, int t, int mode, float2* smem) {
  const JobRec& jb = a.jb;
  const int r = blockIdx.x;
  if (r >= N) return;
  const bool has_prev = mode != 0, has_next = mode != 2;
  const WsLayout L = ws_layout(N, jb.M, jb.T);
  char* ws = jb.ws;
  const int c = threadIdx.x;
  const bool lane = c < N;
  float2* tw = smem;
  float2* orow = tw + N;
  float2* A = orow + N;  // 2N
  float2* B = A + 2 * N; // 2N

  int ny_n = 0, nx_n = 0, ny_p = 0, nx_p = 0;
  float fy_n = 0.f, fx_n = 0.f, fy_p = 0.f, fx_p = 0.f;
  if (has_next) box_frac(a, t % jb.J, N, &ny_n, &nx_n, &fy_n, &fx_n, jb.status);
  if (has_prev) box_frac(a, (t - 1) % jb.J, N, &ny_p, &nx_p, &fy_p, &fx_p, nullptr);
  // rows of box s-1 this workgroup updates: rb1 = the one that is row r of
  // box s, rb2 = one that leaves the box
  int rb1 = -1, rb2 = -1;
  if (has_prev) {
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
  load_twiddles<N, kSpThreads>(tw);
  if (has_prev) {
    float2 e1 = d1, e2 = d2;
    if (fx_p != 0.f) {  // x back-move (db is already moved back along y)
      if (lane) {
        A[c] = d1;
        A[N + c] = d2;
      }
      __syncthreads();
      float2* F = fft_lds<N, false, false, kSpThreads>(A, B, 2, tw);
      float2* G = (F == A) ? B : A;
      if (lane) {
        const float2 w = ramp1(c, fx_p, -1.f, N);
        G[c] = cmul(F[c], w);
        G[N + c] = cmul(F[N + c], w);
      }
      __syncthreads();
      float2* H = fft_lds<N, true, false, kSpThreads>(G, F, 2, tw);
      if (lane) {
        e1 = H[c];
        e2 = H[N + c];
      }
    }
    bool bad = false;
    if (lane) {
      if (rb1 >= 0) {
        const float2 on = cadd(o1, e1);
        jb.obj[(size_t)(ny_p + rb1) * jb.W + nx_p + c] = on;
        orow[c] = on;
        bad |= !(isfinite(on.x) && isfinite(on.y));
      }
      if (rb2 >= 0) {
        const float2 on = cadd(o2, e2);
        jb.obj[(size_t)(ny_p + rb2) * jb.W + nx_p + c] = on;
        bad |= !(isfinite(on.x) && isfinite(on.y));
      }
    }
    if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
    __syncthreads();
  }
  if (!has_next) return;
  // crop row r of box s (the part inside box s-1 taken from the row just
  // updated), x move
  float2 v = make_float2(0.f, 0.f);
  if (lane) {
    // (a value select on an in-range read: no pointer select over address spaces)
    const int xo = nx_n + c - nx_p;
    const float2 ov = orow[min(max(xo, 0), N - 1)];
    v = (rb1 >= 0 && xo >= 0 && xo < N) ? ov : og;
  }
  float2* cb = (float2*)(ws + L.cb) + (size_t)r * N;
  if (fx_n != 0.f) {
    if (lane) A[c] = v;
    __syncthreads();
    float2* F = fft_lds<N, false, false, kSpThreads>(A, B, 1, tw);
    float2* G = (F == A) ? B : A;
    if (lane) G[c] = cmul(F[c], ramp1(c, fx_n, 1.f, N));
    __syncthreads();
    fft_lds_store<N, true, false, kSpThreads>(G, F, 1, tw, [&](int, int cc, float2 w) { cb[cc] = w; });
  } else if (lane) {
    cb[c] = v;
  }
}

// ---------------------------------------------------------------- C: exit waves
template <int N>
__device__ void sp_cols_exit(const SpArgs& a, int t, float2* smem) {
  constexpr int MM = MRPIE_MAX_MODES;
  const JobRec& jb = a.jb;
  const int u = xcd_unit(blockIdx.x, gridDim.x);
  if (u >= N || t >= jb.J * jb.T) return;
  const int M = jb.M, jn = t % jb.J;
  const WsLayout L = ws_layout(N, M, jb.T);
  char* ws = jb.ws;
  const size_t NN = (size_t)N * N;
  const int k = threadIdx.x;
  const bool lane = k < N;
  float2* tw = smem;
  float2* A = tw + N;     // M N
  float2* B = A + M * N;  // M N
  __shared__ float redf[32];
  int ny, nx;
  float fy, fx;
  box_frac(a, jn, N, &ny, &nx, &fy, &fx, nullptr);
  const float2* Pc = (t & 1) == 0 ? jb.probe : (const float2*)(ws + L.probe1);
  float2 v = make_float2(0.f, 0.f);
  float2 P[MM];
  if (lane) {
    v = ((const float2*)(ws + L.cb))[(size_t)k * N + u];
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) P[p] = Pc[p * NN + (size_t)k * N + u];
  }
  load_twiddles<N, kSpThreads>(tw);
  float2 o = v;
  if (fy != 0.f) {  // y move
    if (lane) A[k] = v;
    __syncthreads();
    float2* F = fft_lds<N, false, false, kSpThreads>(A, B, 1, tw);
    float2* G = (F == A) ? B : A;
    if (lane) G[k] = cmul(F[k], ramp1(k, fy, 1.f, N));
    __syncthreads();
    float2* H = fft_lds<N, true, false, kSpThreads>(G, F, 1, tw);
    if (lane) o = H[k];
    __syncthreads();
  }
  float om = 0.f, pm = 0.f;
  if (lane) {
    ((float2*)(ws + L.patch[0]))[(size_t)k * N + u] = o;
    if (!a.xcb && recording(a, t)) a.reg_ref[((size_t)jn * N + k) * N + u] = o;
    om = cabs2(o);
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        pm += cabs2(P[p]);
        A[p * N + k] = cmul(P[p], o);
      }
  }
  block_max2(om, pm, redf, om, pm);  // (its barriers also publish A)
  if (threadIdx.x == 0) {
    ((float*)(ws + L.omax[0]))[u] = om;
    ((float*)(ws + L.pmax[0]))[u] = pm;
  }
  float2* psi = (float2*)(ws + L.psi[0]);
  auto store = [&](int p, int kk, float2 v) { psi[p * NN + (size_t)kk * N + u] = v; };
  if (a.fresnel > 0.f) {  // near field: y propagation, F_y^-1 h_y F_y
    float2* S = fft_lds<N, false, false, kSpThreads>(A, B, M, tw);
    float2* G = (S == A) ? B : A;
    if (lane) {
      const float2 h = fresnel1(k, a.fresnel, -1.f, N);
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) G[p * N + k] = cmul(S[p * N + k], h);
    }
    __syncthreads();
    fft_lds_store<N, true, false, kSpThreads>(G, S, M, tw, store);
  } else {
    fft_lds_store<N, false, false, kSpThreads>(A, B, M, tw, store);
  }
}

// ---------------------------------------------------------------- R: modulus
template <int N>
__device__ void sp_rows_mod(const SpArgs& a, int t, float2* smem) {
  constexpr int MM = MRPIE_MAX_MODES;
  const JobRec& jb = a.jb;
  const int r = blockIdx.x;
  if (r >= N || t >= jb.J * jb.T) return;
  const int M = jb.M, it = t / jb.J, jn = t - it * jb.J;
  const WsLayout L = ws_layout(N, M, jb.T);
  char* ws = jb.ws;
  const size_t NN = (size_t)N * N;
  const int c = threadIdx.x;
  const bool lane = c < N;
  float2* tw = smem;
  float2* A = tw + N;     // M N
  float2* B = A + M * N;  // M N
  float2* psi = (float2*)(ws + L.psi[0]);
  // per-wave partials of the Fourier error and of the intensity sum
  const size_t slot = (size_t)it * kErrSlots + r * 4 + (c >> 6);
  double* err_slot = (double*)(ws + L.err) + slot;
  double* isum_slot = (double*)(ws + L.isum) + slot;
  const double err_old = (c & 63) == 0 ? *err_slot : 0.0;
  const double isum_old = (c & 63) == 0 ? *isum_slot : 0.0;
  float Iv = 0.f;
  if (lane) {
    Iv = jb.I[(size_t)jn * NN + (size_t)r * N + c];
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) A[p * N + c] = psi[p * NN + (size_t)r * N + c];
  }
  load_twiddles<N, kSpThreads>(tw);
  __syncthreads();
  const bool near = a.fresnel > 0.f;
  float2* F = fft_lds<N, false, false, kSpThreads>(A, B, M, tw);
  float2* G = (F == A) ? B : A;
  if (near) {  // x propagation to the detector plane, F_x^-1 h_x F_x
    if (lane) {
      const float2 h = fresnel1(c, a.fresnel, -1.f, N);
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) G[p * N + c] = cmul(F[p * N + c], h);
    }
    __syncthreads();
    F = fft_lds<N, true, false, kSpThreads>(G, F, M, tw);
    G = (F == A) ? B : A;
  }
  // Eq. 7.  Far field: the 2-D transform here is unnormalised (N x unitary)
  // and so is the inverse, so the scale factor carries one 1/N.  Near field:
  // the propagated field is exact (each axis' round trip carries its 1/N).
  double e = 0.0, isv = 0.0;
  if (lane) {
    const float sc = near ? 1.0f : 1.0f / (float)N;
    float S = 0.f;
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) S += cabs2(F[p * N + c]);
    const float rs = S > 0.f ? __builtin_amdgcn_rsqf(S) : 0.f;
    const float Au = S * rs;
    const float sq = __builtin_amdgcn_sqrtf(fmaxf(Iv, 0.f));
    const float d = Au * sc - sq;
    e = (double)d * (double)d;
    isv = (double)fmaxf(Iv, 0.f);
    if (!isfinite(S)) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
    if (a.xcb && recording(a, t)) {  // XCORR_B pair: model amplitude, measured amplitude
      const size_t off = ((size_t)jn * N + r) * N + c;
      a.reg_ref[off] = make_float2(Au * sc, 0.f);
      a.reg_mov[off] = make_float2(sq, 0.f);
    }
    const float f = sq * rs * sc;
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) G[p * N + c] = cscale(F[p * N + c], f);
  }
  __syncthreads();
  auto store = [&](int p, int cc, float2 v) { psi[p * NN + (size_t)r * N + cc] = v; };
  if (near) {  // back along x, F_x^-1 conj(h_x) F_x
    float2* K = fft_lds<N, false, false, kSpThreads>(G, F, M, tw);
    float2* Q = (K == A) ? B : A;
    if (lane) {
      const float2 h = fresnel1(c, a.fresnel, 1.f, N);
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) Q[p * N + c] = cmul(K[p * N + c], h);
    }
    __syncthreads();
    fft_lds_store<N, true, false, kSpThreads>(Q, K, M, tw, store);
  } else {
    fft_lds_store<N, true, false, kSpThreads>(G, F, M, tw, store);
  }
  e = wave_sum(e);
  isv = wave_sum(isv);
  if ((c & 63) == 0) {
    *err_slot = err_old + e;
    *isum_slot = isum_old + isv;
  }
}

// ---------------------------------------------------------------- C: updates
template <int N>
__device__ void sp_cols_update(const SpArgs& a, int t, float2* smem) {
  constexpr int MM = MRPIE_MAX_MODES;
  const JobRec& jb = a.jb;
  const int u = xcd_unit(blockIdx.x, gridDim.x);
  if (u >= N || t >= jb.J * jb.T) return;
  const int M = jb.M, jn = t % jb.J;
  const Common& cm = a.c;
  const WsLayout L = ws_layout(N, M, jb.T);
  char* ws = jb.ws;
  const size_t NN = (size_t)N * N;
  const int k = threadIdx.x;
  const bool lane = k < N;
  float2* tw = smem;
  float2* A = tw + N;     // M N
  float2* B = A + M * N;  // M N
  __shared__ float redf[32];
  int ny, nx;
  float fy, fx;
  box_frac(a, jn, N, &ny, &nx, &fy, &fx, nullptr);
  const float2* Pold = (t & 1) == 0 ? jb.probe : (const float2*)(ws + L.probe1);
  float2* Pnew = (t & 1) == 0 ? (float2*)(ws + L.probe1) : jb.probe;
  const float2* psi = (const float2*)(ws + L.psi[0]);
  float2 P[MM];
  float2 o = make_float2(0.f, 0.f);
  float om_in = 0.f, pm_in = 0.f;
  if (lane) {
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        A[p * N + k] = psi[p * NN + (size_t)k * N + u];
        P[p] = Pold[p * NN + (size_t)k * N + u];
      }
    o = ((const float2*)(ws + L.patch[0]))[(size_t)k * N + u];
    om_in = ((const float*)(ws + L.omax[0]))[k];
    pm_in = ((const float*)(ws + L.pmax[0]))[k];
  }
  load_twiddles<N, kSpThreads>(tw);
  float omax, pmaxv;
  block_max2(om_in, pm_in, redf, omax, pmaxv);  // (its barriers also publish A)
  float2* R;
  if (a.fresnel > 0.f) {  // near field: back along y, F_y^-1 conj(h_y) F_y
    float2* F = fft_lds<N, false, false, kSpThreads>(A, B, M, tw);
    float2* G = (F == A) ? B : A;
    if (lane) {
      const float2 h = fresnel1(k, a.fresnel, 1.f, N);
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) G[p * N + k] = cmul(F[p * N + k], h);
    }
    __syncthreads();
    R = fft_lds<N, true, false, kSpThreads>(G, F, M, tw);
  } else {
    R = fft_lds<N, true, false, kSpThreads>(A, B, M, tw);
  }
  float2* W = (R == A) ? B : A;
  const int it_abs = cm.iter_offset + t / jb.J;
  const bool upd_p = it_abs >= cm.probe_update_start;
  bool bad = false;
  float2 dlt = make_float2(0.f, 0.f);
  if (lane) {
    const float o2 = cabs2(o);
    const float dP = cm.beta * omax + (1.f - cm.beta) * o2;
    const float gp = (upd_p && dP != 0.f) ? cm.alpha_probe / dP : 0.f;
    float Ps = 0.f;
    float2 num = make_float2(0.f, 0.f);
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        const float2 d = csub(R[p * N + k], cmul(P[p], o));
        num = cadd(num, cmulc(d, P[p]));
        Ps += cabs2(P[p]);
        const float2 Pn = cadd(P[p], cscale(cmulc(d, o), gp));
        Pnew[p * NN + (size_t)k * N + u] = Pn;
        bad |= !(isfinite(Pn.x) && isfinite(Pn.y));
      }
    const float dO = cm.gamma * pmaxv + (1.f - cm.gamma) * Ps;
    const float go = dO != 0.f ? cm.alpha_obj / dO : 0.f;
    dlt = cscale(num, go);
    if (!a.xcb && recording(a, t)) a.reg_mov[((size_t)jn * N + k) * N + u] = cadd(o, dlt);
  }
  if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
  float2* db = (float2*)(ws + L.db) + u;
  if (fy != 0.f) {  // y back-move of delta_o
    if (lane) W[k] = dlt;
    __syncthreads();
    float2* F = fft_lds<N, false, false, kSpThreads>(W, R, 1, tw);
    float2* G = (F == W) ? R : W;
    if (lane) G[k] = cmul(F[k], ramp1(k, fy, -1.f, N));
    __syncthreads();
    fft_lds_store<N, true, false, kSpThreads>(G, F, 1, tw, [&](int, int kk, float2 v) { db[(size_t)kk * N] = v; });
  } else if (lane) {
    db[(size_t)k * N] = dlt;
  }
}

// ---------------------------------------------------------------- kernels
// The job comes as leading scalar arguments (positions, workspace, object,
// probe, tick, mode, shape), which gfx950 preloads into SGPRs, so a launch's
// first loads do not wait for a kernel-argument fetch; the rest follows.
#define MRPIE_SP_PARAMS                                                                                        \
  const float *pos, char *ws, float2 *obj, float2 *probe, int t, int mode, int J, int T, int NM, int H, int W, \
      const float *I, int *status, float2 *reg_ref, float2 *reg_mov, int subpixel, int record_start, int xcb,    \
      float fresnel, const Common c
#define MRPIE_SP_ARGS                                                                                  \
  SpArgs a;                                                                                            \
  a.c = c;                                                                                             \
  a.jb = JobRec{obj, probe, pos, I, ws, status, H, W, NM & 0xffff, NM >> 16, J, T};                    \
  a.subpixel = subpixel;                                                                               \
  a.reg_ref = reg_ref;                                                                                 \
  a.reg_mov = reg_mov;                                                                                 \
  a.record_start = record_start;                                                                       \
  a.xcb = xcb;                                                                                         \
  a.fresnel = fresnel;
#define MRPIE_DISPATCH(FN, ...)              \
  switch (a.jb.N) {                          \
    case 32: FN<32>(__VA_ARGS__); break;     \
    case 64: FN<64>(__VA_ARGS__); break;     \
    case 128: FN<128>(__VA_ARGS__); break;   \
    case 192: FN<192>(__VA_ARGS__); break;   \
    default: FN<256>(__VA_ARGS__); break;    \
  }

__global__ __launch_bounds__(256) void k_sp_rows_gather(MRPIE_SP_PARAMS) {
  extern __shared__ float2 smem[];
  MRPIE_SP_ARGS
  MRPIE_DISPATCH(sp_rows_gather, a, t, mode, smem)
}
__global__ __launch_bounds__(256) void k_sp_cols_exit(MRPIE_SP_PARAMS) {
  extern __shared__ float2 smem[];
  MRPIE_SP_ARGS
  MRPIE_DISPATCH(sp_cols_exit, a, t, smem)
}
__global__ __launch_bounds__(256) void k_sp_rows_mod(MRPIE_SP_PARAMS) {
  extern __shared__ float2 smem[];
  MRPIE_SP_ARGS
  MRPIE_DISPATCH(sp_rows_mod, a, t, smem)
}
__global__ __launch_bounds__(256) void k_sp_cols_update(MRPIE_SP_PARAMS) {
  extern __shared__ float2 smem[];
  MRPIE_SP_ARGS
  MRPIE_DISPATCH(sp_cols_update, a, t, smem)
}

int run_sweep_subpixel(const Common& c, const JobRec& jb, const SubpixelExtra& ex, int it0, int iters, bool head,
                       bool tail, hipStream_t s) {
  const int t0 = it0 * jb.J, t1 = (it0 + iters) * jb.J;
  int rc = launch_init_twiddles(s);
  if (rc) return rc;
  const int N = jb.N, M = jb.M;
  const int NM = N | (M << 16);
  const size_t lg = (size_t)(N + N + 4 * N) * 8;
  const size_t lm = (size_t)(N + 2 * M * N) * 8;
  MRPIE_HIP(ensure_lds((const void*)k_sp_cols_exit, lm));
  MRPIE_HIP(ensure_lds((const void*)k_sp_rows_mod, lm));
  MRPIE_HIP(ensure_lds((const void*)k_sp_cols_update, lm));
  const dim3 g(N), blk(kSpThreads);
#define MRPIE_SP_LAUNCH(K, L, T_, MODE)                                                                        \
  hipLaunchKernelGGL(K, g, blk, L, s, jb.pos, jb.ws, jb.obj, jb.probe, T_, MODE, jb.J, jb.T, NM, jb.H, jb.W, jb.I, \
                     jb.status, ex.reg_ref, ex.reg_mov, ex.subpixel, ex.record_start, ex.xcb, ex.fresnel, c)
  for (int t = t0; t < t1; ++t) {
    MRPIE_SP_LAUNCH(k_sp_rows_gather, lg, t, (t == t0 && head) ? 0 : 1);
    MRPIE_SP_LAUNCH(k_sp_cols_exit, lm, t, 0);
    MRPIE_SP_LAUNCH(k_sp_rows_mod, lm, t, 0);
    MRPIE_SP_LAUNCH(k_sp_cols_update, lm, t, 0);
  }
  if (tail) MRPIE_SP_LAUNCH(k_sp_rows_gather, lg, t1, 2);
#undef MRPIE_SP_LAUNCH
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

}  // namespace mrpie
