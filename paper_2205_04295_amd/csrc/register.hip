// Subpixel registration (Methods, "Adam-based position refinement": the
// 2-D phase correlation of Guizar-Sicairos et al. 2008, refined by a
// matrix-product DFT evaluated only around the coarse peak, no zero-padding)
// and the modified Adam step of Alg. 1 (Eq. 8-9), on gfx950.
//
// The whole registration runs in double precision so that its integer peaks
// (coarse lag and upsampled-window argmax) are those of an exact evaluation:
// float rounding of the 65536-term sums is larger than the gap between
// neighbouring samples near the peak of the upsampled surface.
//
// Pipeline for a batch of B (ref, mov) pairs of N x N complex64 patches:
//   k_reg_rows   row FFTs of ref and mov (complex128)
//   k_reg_cols   column FFTs, X = F(ref) conj(F(mov)) [phase-normalised],
//                stored; inverse column FFT of X
//   k_reg_coarse inverse row FFT -> |F^-1 X|^2, per-row first maximum
//   k_reg_s0     first maximum in row-major order -> signed integer lag s0
//   k_reg_gemm1  T = K (X . e^{2 pi i k.s0/N})   [U x N] x [N x N]
//   k_reg_gemm2  C = T K^T, per-tile first maximum of |C|^2
//   k_reg_final  window argmax (u*, v*) -> shift s0 + ((u*, v*) - c)/up
// with K[u][k] = exp(+2 pi i k (u - c) / (N up)), k the signed frequency,
// U = ceil(1.5 up), c = floor(U/2): the coarse lag is folded into X as a
// diagonal phase so one K serves every pair.
#include <algorithm>
#include <cmath>

#include "register.hpp"

namespace mrpie {

__device__ __forceinline__ int signed_freq(int k, int N) { return k < (N + 1) / 2 ? k : k - N; }

// first-maximum order: larger value first; equal values -> smaller index
__device__ __forceinline__ bool better(double v, long long i, double bv, long long bi) {
  return v > bv || (v == bv && i < bi);
}

struct ArgMax {
  double v;
  long long i;
};

// first-maximum argmax over one wave (all lanes get the result)
__device__ __forceinline__ ArgMax wave_argmax(double v, long long i) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const long long oi = __shfl_xor(i, o, 64);
    if (better(ov, oi, v, i)) { v = ov; i = oi; }
  }
  return ArgMax{v, i};
}

// workgroup argmax with the first-maximum rule (all threads get the result)
__device__ __forceinline__ ArgMax block_argmax(double v, long long i, double* rv, long long* ri) {
  const ArgMax wm = wave_argmax(v, i);
  v = wm.v;
  i = wm.i;
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { rv[w] = v; ri[w] = i; }
  __syncthreads();
  ArgMax r{rv[0], ri[0]};
  for (int k = 1; k < nw; ++k)
    if (better(rv[k], ri[k], r.v, r.i)) { r.v = rv[k]; r.i = ri[k]; }
  return r;
}

// ---------------------------------------------------------------- FFT passes
// Row passes take kRegRW rows per workgroup (one wave per row at N = 256),
// so every thread of the workgroup has a butterfly in every radix-4 stage.
constexpr int kRegRW = 4;

template <int N>
__global__ __launch_bounds__(256) void k_reg_rows(const RegArgs a) {
  __shared__ double2 tw[N];
  __shared__ double2 A[kRegRW * N], B[kRegRW * N];
  const int r0 = blockIdx.x * kRegRW, b = blockIdx.y, which = blockIdx.z;
  const float2* src = (which == 0 ? a.ref : a.mov) + ((size_t)b * N + r0) * N;
  load_twiddles<N>(tw);
  for (int i = threadIdx.x; i < kRegRW * N; i += blockDim.x) {
    const float2 v = src[i];
    A[i] = make_double2((double)v.x, (double)v.y);
  }
  __syncthreads();
  double2* R = fft_lds<N, false>(A, B, kRegRW, tw);
  double2* dst = a.work + (((size_t)b * 2 + which) * N + r0) * N;
  for (int i = threadIdx.x; i < kRegRW * N; i += blockDim.x) dst[i] = R[i];
}

// CW adjacent columns per workgroup, so every access moves CW * 16
// contiguous bytes of a row; pixel q of the group is row k = q / CW, column
// c = q % CW.  LDS (dynamic): twiddles, then one buffer of 2 CW transforms
// (ref and mov of each column) transformed in place (the same butterflies
// as the ping-pong plan, half the LDS: twice the workgroups per CU).
constexpr int kRegCW = 4;
constexpr size_t reg_cols_lds(int N) { return (size_t)(N + 2 * kRegCW * N) * 16; }

template <int N>
__global__ __launch_bounds__(256) void k_reg_cols(const RegArgs a) {
  constexpr int CW = kRegCW, PIX = (N * CW + 255) / 256;
  extern __shared__ double2 dsm[];
  double2* tw = dsm;
  double2* A = tw + N;           // ref column c at c * N, mov at (CW + c) * N
  const int u0 = blockIdx.x * CW, b = blockIdx.y, tid = threadIdx.x;
  double2* w0 = a.work + (size_t)b * 2 * N * N;  // ref spectra -> later F^-1 over columns of X
  double2* w1 = w0 + (size_t)N * N;              // mov spectra -> later X
  load_twiddles<N>(tw);
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    A[c * N + k] = w0[(size_t)k * N + u0 + c];
    A[(CW + c) * N + k] = w1[(size_t)k * N + u0 + c];
  }
  __syncthreads();
  fft_lds_inplace<N, false, true, 2 * CW, 256>(A, 2 * CW, tw);
  const double2* F = A;
  double2* G = A;  // X over the ref transforms: each thread rewrites only the pixels it reads
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    double2 x = cmulc(F[c * N + k], F[(CW + c) * N + k]);  // F(ref) conj(F(mov))
    if (a.norm) {
      const double m = hypot(x.x, x.y);
      x = m > 0.0 ? make_double2(x.x / m, x.y / m) : make_double2(0.0, 0.0);
    }
    w1[(size_t)k * N + u0 + c] = x;
    G[c * N + k] = x;
  }
  __syncthreads();
  fft_lds_inplace<N, true, true, CW, 256>(G, CW, tw);
  const double2* H = G;
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    w0[(size_t)k * N + u0 + c] = H[c * N + k];
  }
}

// kRegRW rows per workgroup; wave w scans row r0 + w of the inverse
// transform for its first maximum (requires 64 kRegRW threads).
template <int N>
__global__ __launch_bounds__(256) void k_reg_coarse(const RegArgs a) {
  __shared__ double2 tw[N];
  __shared__ double2 A[kRegRW * N], B[kRegRW * N];
  const int r0 = blockIdx.x * kRegRW, b = blockIdx.y;
  const double2* src = a.work + ((size_t)b * 2 * N + r0) * N;
  load_twiddles<N>(tw);
  for (int i = threadIdx.x; i < kRegRW * N; i += blockDim.x) A[i] = src[i];
  __syncthreads();
  double2* R = fft_lds<N, true>(A, B, kRegRW, tw);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, r = r0 + w;
  double v = -1.0;
  long long idx = (long long)r * N + N;
  for (int i = lane; i < N; i += 64) {
    const double m = cabs2(R[w * N + i]);
    const long long ii = (long long)r * N + i;
    if (better(m, ii, v, idx)) { v = m; idx = ii; }
  }
  const ArgMax m = wave_argmax(v, idx);
  if (lane == 0) {
    a.rowmax_v[(size_t)b * N + r] = m.v;
    a.rowmax_i[(size_t)b * N + r] = m.i;
  }
}

__global__ __launch_bounds__(256) void k_reg_s0(const RegArgs a, int N) {
  __shared__ double rv[16];
  __shared__ long long ri[16];
  const int b = blockIdx.x;
  double v = -1.0;
  long long idx = (long long)N * N;
  for (int r = threadIdx.x; r < N; r += blockDim.x) {
    const double m = a.rowmax_v[(size_t)b * N + r];
    const long long ii = a.rowmax_i[(size_t)b * N + r];
    if (better(m, ii, v, idx)) { v = m; idx = ii; }
  }
  const ArgMax m = block_argmax(v, idx, rv, ri);
  if (threadIdx.x == 0) {
    const int py = (int)(m.i / N), px = (int)(m.i % N);
    a.s0[2 * b] = py > N / 2 ? py - N : py;
    a.s0[2 * b + 1] = px > N / 2 ? px - N : px;
    a.peak[4 * b] = py;
    a.peak[4 * b + 1] = px;
  }
}

// K[u][k] = exp(+2 pi i k_signed (u - c) / (N up)), u < U
__global__ void k_reg_kmat(const RegArgs a, int N) {
  const int U = a.U;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < U * N; i += gridDim.x * blockDim.x) {
    const int u = i / N, k = i - u * N;
    const double ph = 2.0 * (double)signed_freq(k, N) * (double)(u - a.c) / ((double)N * (double)a.up);
    double s, c;
    sincospi(ph, &s, &c);
    a.K[i] = make_double2(c, s);
  }
}

// Register blocks of the two GEMMs: RB = 4 (64 x 64 output tiles, 16
// complex FMAs per 8 LDS reads) for large windows, RB = 2 (32-row tiles)
// for small ones, whose last 64-row tile would be mostly empty (upsample
// 1000, 256 pairs: 28.6 against 35.0 ms; upsample 100: 1.77 against 1.82
// ms with RB = 2).  Every output sums its terms in k order whatever RB is.
inline int gemm_rb(int U) { return U > 320 ? 4 : 2; }

// T[b][u][kx] = sum_ky K[u][ky] X[b][ky][kx] e^{2 pi i (ky s0y + kx s0x)/N}
// Tile: 16 RB u x 64 kx per workgroup, ky in chunks of 16 staged in LDS;
// each of the 16 x 16 threads accumulates an RB x 4 block.
constexpr int G1_RJ = 4, G1_TX = 16 * G1_RJ, G1_KC = 16;
template <int N, int G1_RI>
__global__ __launch_bounds__(256) void k_reg_gemm1(const RegArgs a) {
  constexpr int G1_TU = 16 * G1_RI;
  __shared__ double2 Ks[G1_TU][G1_KC + 1];
  __shared__ double2 Xs[G1_KC][G1_TX + 1];
  __shared__ double2 tw[N];  // exp(-2 pi i e / N): the lag phase is an N-th root of unity
  const int b = blockIdx.z;
  const int u0 = blockIdx.y * G1_TU, x0 = blockIdx.x * G1_TX;
  const int U = a.U;
  const double2* X = a.work + ((size_t)b * 2 + 1) * N * N;
  const int s0y = a.s0[2 * b], s0x = a.s0[2 * b + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;  // 16 x 16 threads
  double2 acc[G1_RI][G1_RJ];
#pragma unroll
  for (int i = 0; i < G1_RI; ++i)
#pragma unroll
    for (int j = 0; j < G1_RJ; ++j) acc[i][j] = make_double2(0.0, 0.0);
  load_twiddles<N>(tw);
  __syncthreads();
  for (int k0 = 0; k0 < N; k0 += G1_KC) {
    for (int i = threadIdx.x; i < G1_TU * G1_KC; i += blockDim.x) {
      const int uu = i / G1_KC, kk = i - uu * G1_KC;
      const int u = u0 + uu;
      Ks[uu][kk] = u < U ? a.K[(size_t)u * N + k0 + kk] : make_double2(0.0, 0.0);
    }
    for (int i = threadIdx.x; i < G1_KC * G1_TX; i += blockDim.x) {
      const int kk = i / G1_TX, xx = i - kk * G1_TX;
      const int ky = k0 + kk, kx = x0 + xx;
      if (kx >= N) { Xs[kk][xx] = make_double2(0.0, 0.0); continue; }
      const double2 x = X[(size_t)ky * N + kx];
      // e^{2 pi i e / N} with e = (ky s0y + kx s0x) mod N = conj(tw[e])
      int e = (signed_freq(ky, N) * s0y + signed_freq(kx, N) * s0x) % N;
      e += e < 0 ? N : 0;
      Xs[kk][xx] = cmulc(x, tw[e]);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < G1_KC; ++kk) {
      double2 kv[G1_RI], xv[G1_RJ];
#pragma unroll
      for (int i = 0; i < G1_RI; ++i) kv[i] = Ks[ty + 16 * i][kk];
#pragma unroll
      for (int j = 0; j < G1_RJ; ++j) xv[j] = Xs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < G1_RI; ++i)
#pragma unroll
        for (int j = 0; j < G1_RJ; ++j) {
          acc[i][j].x = fma(kv[i].x, xv[j].x, fma(-kv[i].y, xv[j].y, acc[i][j].x));
          acc[i][j].y = fma(kv[i].x, xv[j].y, fma(kv[i].y, xv[j].x, acc[i][j].y));
        }
    }
    __syncthreads();
  }
  double2* T = a.T + (size_t)b * U * N;
#pragma unroll
  for (int i = 0; i < G1_RI; ++i) {
    const int u = u0 + ty + 16 * i;
    if (u >= U) continue;
#pragma unroll
    for (int j = 0; j < G1_RJ; ++j)
      if (x0 + tx + 16 * j < N) T[(size_t)u * N + x0 + tx + 16 * j] = acc[i][j];
  }
}

// C[b][u][v] = sum_kx T[b][u][kx] K[v][kx]; per-tile first maximum of |C|^2.
// Tile 16 RB u x 16 RB v, kx in chunks of 16; each thread an RB x RB block.
constexpr int G2_KC = 16;
template <int N, int G2_R>
__global__ __launch_bounds__(256) void k_reg_gemm2(const RegArgs a) {
  constexpr int G2_T = 16 * G2_R;
  __shared__ double2 Ts[G2_T][G2_KC + 1];
  __shared__ double2 Ks[G2_T][G2_KC + 1];
  __shared__ double rv[16];
  __shared__ long long ri[16];
  const int b = blockIdx.z;
  const int u0 = blockIdx.y * G2_T, v0 = blockIdx.x * G2_T;
  const int U = a.U;
  const double2* T = a.T + (size_t)b * U * N;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double2 acc[G2_R][G2_R];
#pragma unroll
  for (int i = 0; i < G2_R; ++i)
#pragma unroll
    for (int j = 0; j < G2_R; ++j) acc[i][j] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < N; k0 += G2_KC) {
    for (int i = threadIdx.x; i < G2_T * G2_KC; i += blockDim.x) {
      const int rr = i / G2_KC, kk = i - rr * G2_KC;
      const int u = u0 + rr, v = v0 + rr;
      Ts[rr][kk] = u < U ? T[(size_t)u * N + k0 + kk] : make_double2(0.0, 0.0);
      Ks[rr][kk] = v < U ? a.K[(size_t)v * N + k0 + kk] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < G2_KC; ++kk) {
      double2 tv[G2_R], kv[G2_R];
#pragma unroll
      for (int i = 0; i < G2_R; ++i) tv[i] = Ts[ty + 16 * i][kk];
#pragma unroll
      for (int j = 0; j < G2_R; ++j) kv[j] = Ks[tx + 16 * j][kk];
#pragma unroll
      for (int i = 0; i < G2_R; ++i)
#pragma unroll
        for (int j = 0; j < G2_R; ++j) {
          acc[i][j].x = fma(tv[i].x, kv[j].x, fma(-tv[i].y, kv[j].y, acc[i][j].x));
          acc[i][j].y = fma(tv[i].x, kv[j].y, fma(tv[i].y, kv[j].x, acc[i][j].y));
        }
    }
    __syncthreads();
  }
  double best = -1.0;
  long long bi = (long long)U * U;
#pragma unroll
  for (int i = 0; i < G2_R; ++i)
#pragma unroll
    for (int j = 0; j < G2_R; ++j) {
      const int u = u0 + ty + 16 * i, v = v0 + tx + 16 * j;
      if (u < U && v < U) {
        const double m = cabs2(acc[i][j]);
        const long long ii = (long long)u * U + v;
        if (better(m, ii, best, bi)) { best = m; bi = ii; }
      }
    }
  const ArgMax m = block_argmax(best, bi, rv, ri);
  if (threadIdx.x == 0) {
    const int tiles = gridDim.x * gridDim.y;
    const int t = blockIdx.y * gridDim.x + blockIdx.x;
    a.tile_v[(size_t)b * tiles + t] = m.v;
    a.tile_i[(size_t)b * tiles + t] = m.i;
  }
}

__global__ __launch_bounds__(64) void k_reg_final(const RegArgs a, int tiles) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.B) return;
  double v = -1.0;
  long long idx = (long long)a.U * a.U;
  for (int t = 0; t < tiles; ++t) {
    const double m = a.tile_v[(size_t)b * tiles + t];
    const long long ii = a.tile_i[(size_t)b * tiles + t];
    if (better(m, ii, v, idx)) { v = m; idx = ii; }
  }
  const int u = (int)(idx / a.U), w = (int)(idx % a.U);
  a.peak[4 * b + 2] = u;
  a.peak[4 * b + 3] = w;
  const double up = (double)a.up;
  a.shift[2 * b] = (float)((double)a.s0[2 * b] + (double)(u - a.c) / up);
  a.shift[2 * b + 1] = (float)((double)a.s0[2 * b + 1] + (double)(w - a.c) / up);
}

// ---------------------------------------------------------------- Adam
// Alg. 1 with the measured shift as the gradient; the position moves by
// +lr mhat / (sqrt(vhat) + eps) (Eq. 8-9) and is clamped to the object.
__global__ void k_adam(int J, float* pos, float* st, const float* g, int t, float lr, float b1, float b2,
                       float eps, float ymax, float xmax, const int* active) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  if (active && !active[0]) return;
  const double bc1 = 1.0 - pow((double)b1, (double)t);
  const double bc2 = 1.0 - pow((double)b2, (double)t);
  for (int a = 0; a < 2; ++a) {
    const double gj = (double)g[2 * j + a];
    const double m = (double)b1 * (double)st[4 * j + a] + (1.0 - (double)b1) * gj;
    const double v = (double)b2 * (double)st[4 * j + 2 + a] + (1.0 - (double)b2) * gj * gj;
    st[4 * j + a] = (float)m;
    st[4 * j + 2 + a] = (float)v;
    double p = (double)pos[2 * j + a] + (double)lr * (m / bc1) / (sqrt(v / bc2) + (double)eps);
    const double lim = a == 0 ? (double)ymax : (double)xmax;
    p = p < 0.0 ? 0.0 : (p > lim ? lim : p);
    pos[2 * j + a] = (float)p;
  }
}

// ---------------------------------------------------------------- host
int reg_window(int up, int* U, int* c) {
  *U = (int)std::ceil(1.5 * (double)up);
  *c = *U / 2;
  return MRPIE_OK;
}

RegLayout reg_layout(int N, int B, int up) {
  RegLayout L{};
  int U, c;
  reg_window(up, &U, &c);
  const int chunk = std::max(1, std::min(B, kRegChunk));
  const int t2 = 16 * gemm_rb(U);
  const int tiles = ((U + t2 - 1) / t2) * ((U + t2 - 1) / t2);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = ws_align(off + bytes); return o; };
  L.chunk = chunk;
  L.work = take((size_t)chunk * 2 * N * N * 16);
  L.K = take((size_t)U * N * 16);
  L.T = take((size_t)chunk * U * N * 16);
  L.rowmax_v = take((size_t)chunk * N * 8);
  L.rowmax_i = take((size_t)chunk * N * 8);
  L.s0 = take((size_t)chunk * 2 * 4);
  L.tile_v = take((size_t)chunk * tiles * 8);
  L.tile_i = take((size_t)chunk * tiles * 8);
  L.total = off;
  return L;
}

template <int N>
static int register_impl(int B, const float2* ref, const float2* mov, int up, int norm, float* shift, int32_t* peak,
                         char* ws, const RegLayout& L, hipStream_t s) {
  int U, c;
  reg_window(up, &U, &c);
  RegArgs a{};
  a.U = U;
  a.c = c;
  a.up = up;
  a.norm = norm;
  a.work = (double2*)(ws + L.work);
  a.K = (double2*)(ws + L.K);
  a.T = (double2*)(ws + L.T);
  a.rowmax_v = (double*)(ws + L.rowmax_v);
  a.rowmax_i = (long long*)(ws + L.rowmax_i);
  a.s0 = (int*)(ws + L.s0);
  a.tile_v = (double*)(ws + L.tile_v);
  a.tile_i = (long long*)(ws + L.tile_i);
  MRPIE_HIP(ensure_lds((const void*)k_reg_cols<N>, reg_cols_lds(N)));
  hipLaunchKernelGGL(k_reg_kmat, dim3(64), dim3(256), 0, s, a, N);
  const int rb = gemm_rb(U), gt = (U + 16 * rb - 1) / (16 * rb);
  const auto kg1 = rb == 4 ? k_reg_gemm1<N, 4> : k_reg_gemm1<N, 2>;
  const auto kg2 = rb == 4 ? k_reg_gemm2<N, 4> : k_reg_gemm2<N, 2>;
  for (int b0 = 0; b0 < B; b0 += L.chunk) {
    const int nb = std::min(L.chunk, B - b0);
    a.B = nb;
    a.ref = ref + (size_t)b0 * N * N;
    a.mov = mov + (size_t)b0 * N * N;
    a.shift = shift + 2 * (size_t)b0;
    a.peak = peak + 4 * (size_t)b0;
    hipLaunchKernelGGL(k_reg_rows<N>, dim3(N / kRegRW, nb, 2), dim3(256), 0, s, a);
    launch_k(TK_REG, k_reg_cols<N>, dim3(N / kRegCW, nb), dim3(256), reg_cols_lds(N), s, a);
    hipLaunchKernelGGL(k_reg_coarse<N>, dim3(N / kRegRW, nb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_reg_s0, dim3(nb), dim3(256), 0, s, a, N);
    launch_k(TK_GEMM, kg1, dim3((N + G1_TX - 1) / G1_TX, (U + 16 * rb - 1) / (16 * rb), nb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(kg2, dim3(gt, gt, nb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_reg_final, dim3((nb + 63) / 64), dim3(64), 0, s, a, gt * gt);
  }
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

int run_register(int N, int B, const float2* ref, const float2* mov, int up, int norm, float* shift, int32_t* peak,
                 void* ws, size_t ws_bytes, hipStream_t s) {
  const RegLayout L = reg_layout(N, B, up);
  if (!ws || ws_bytes < L.total) return fail(MRPIE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
  int rc = launch_init_twiddles(s);
  if (rc) return rc;
  char* w = (char*)ws;
  switch (N) {
    case 32: return register_impl<32>(B, ref, mov, up, norm, shift, peak, w, L, s);
    case 64: return register_impl<64>(B, ref, mov, up, norm, shift, peak, w, L, s);
    case 128: return register_impl<128>(B, ref, mov, up, norm, shift, peak, w, L, s);
    case 192: return register_impl<192>(B, ref, mov, up, norm, shift, peak, w, L, s);
    default: return register_impl<256>(B, ref, mov, up, norm, shift, peak, w, L, s);
  }
}

int launch_adam(int J, float* pos, float* adam, const float* g, int t, const mrpie_params* pr, int ymax, int xmax,
                hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((J + 255) / 256), dim3(256), 0, s, J, pos, adam, g, t, pr->adam_lr, pr->adam_b1,
                     pr->adam_b2, pr->adam_eps, (float)ymax, (float)xmax, (const int*)nullptr);
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

}  // namespace mrpie

using namespace mrpie;

extern "C" {

int mrpie_register_workspace_size(int32_t N, int32_t B, int32_t upsample, size_t* bytes) {
  if (n_index(N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", N);
  if (B < 0 || upsample < 1 || upsample > 1000 || !bytes) return fail(MRPIE_EINVAL, "bad arguments");
  *bytes = reg_layout(N, std::max(B, 1), upsample).total;
  return MRPIE_OK;
}

int mrpie_register(int32_t N, int32_t B, const void* ref, const void* mov, int32_t upsample, int32_t norm,
                   float* shift, int32_t* peak, void* ws, size_t ws_bytes, void* stream) {
  if (n_index(N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", N);
  if (B < 0) return fail(MRPIE_EINVAL, "B=%d < 0", B);
  if (upsample < 1 || upsample > 1000) return fail(MRPIE_EINVAL, "upsample=%d not in [1,1000]", upsample);
  if (norm != 0 && norm != 1) return fail(MRPIE_EINVAL, "norm must be 0 or 1");
  if (B == 0) return MRPIE_OK;
  if (!ref || !mov || !shift || !peak) return fail(MRPIE_EINVAL, "null pointer");
  return run_register(N, B, (const float2*)ref, (const float2*)mov, upsample, norm, shift, peak, ws, ws_bytes,
                      (hipStream_t)stream);
}

int mrpie_adam(int32_t J, const mrpie_params* pr, int32_t ymax, int32_t xmax, float* pos, float* adam,
               const float* g, int32_t t, void* stream) {
  if (!pr || J < 0 || t < 1 || ymax < 0 || xmax < 0) return fail(MRPIE_EINVAL, "bad arguments");
  if (!(pr->adam_b1 >= 0.f && pr->adam_b1 < 1.f) || !(pr->adam_b2 >= 0.f && pr->adam_b2 < 1.f))
    return fail(MRPIE_EINVAL, "Adam betas must be in [0,1)");
  if (!(pr->adam_eps > 0.f) || !std::isfinite(pr->adam_lr)) return fail(MRPIE_EINVAL, "bad Adam lr/eps");
  if (J == 0) return MRPIE_OK;
  if (!pos || !adam || !g) return fail(MRPIE_EINVAL, "null pointer");
  return launch_adam(J, pos, adam, g, t, pr, ymax, xmax, (hipStream_t)stream);
}

}  // extern "C"
