// Amplitude loss of the mixed-state forward model and its hand-written
// adjoint (gradients w.r.t. object, probe modes and subpixel positions) on
// gfx950.  The forward model is the paper's Eq. 4 with the crop moved by a
// band-limited Fourier shift; the loss and adjoint are an extension of it:
//
//   o_j = S_f(crop_j),  Psi_pj = F(P_p o_j),  A_j = sqrt(sum_p |Psi_pj|^2)
//   L   = sum_j sum_k (A_j - sqrt(I_j))^2
//   chi_pj = F^-1((1 - sqrt(I_j)/A_j) Psi_pj)            (0 where A_j = 0)
//   dL/dP_p   = 2 sum_j conj(o_j) chi_pj
//   dL/do_j   = g_j = 2 sum_p conj(P_p) chi_pj
//   dL/dO     = sum_j S_{-f}(g_j) scattered into box j
//   dL/df_j   = Re sum_k conj(F g_j)(k) (2 pi i k / N) (F o_j)(k)
// (gradients of complex arrays in the dL/dRe + i dL/dIm convention; F is the
// unitary DFT.)  Nothing is stored between the forward and backward passes:
// the backward recomputes the exit waves.
//
// Positions are independent, so every pass runs on a chunk of positions at
// once (grid.y = position in chunk), with the 2-D FFTs split into row and
// column passes like the sweep.  Overlapping boxes and the probe sum are
// reduced in position order by separate kernels, never with atomics, so the
// result is deterministic.
#include <algorithm>
#include <cmath>

#include "adjoint.hpp"

namespace mrpie {

// The FFT passes of this file run 256 threads per workgroup.
constexpr int kAdjThreads = 256;

__device__ __forceinline__ size_t chunk_off(int b, int N) { return (size_t)b * N * N; }

// The 2-D transforms are split into row and column passes, and the Fourier
// move is separable, S_f = S_y S_x: S_y moves along columns by fy
// (e^{+2 pi i ky fy/N}), S_x along rows by fx.  Each 1-D move, each
// component of the position gradient and each back-move then rides in a
// pass over the axis it acts on:
//   P1 (cols): crop columns -> C = S_y(crop)
//   P2 (rows): o = S_x(C); exit waves P_p o, row FFTs
//   P3 (cols): column FFTs; loss and modulus weight; inverse column FFTs
//   P4 (rows): inverse row FFTs -> chi_p; probe-gradient terms; g;
//              dL/df_x = Re <g, d_x o>; h = S_{-x}(g)
//   P5 (cols): dL/df_y = Re <h, d_y C>; S_{-y}(h) = S_{-f}(g)
// (<a, b> = sum conj(a) b, d_x and d_y the band-limited derivatives along x
// and y; S_x is unitary and commutes with d_y, so Re <g, d_y o> =
// Re <S_{-x} g, d_y S_y crop>.)  A 1-D term of the gradient is the
// unnormalised-DFT Parseval sum (1/N) sum_k Re(conj(F a)(k) (2 pi i k/N)
// (F b)(k)) over each row or column.

__device__ __forceinline__ void frac_of(const AdjArgs& a, int j, int N, float* fy, float* fx) {
  *fy = 0.f;
  *fx = 0.f;
  if (!a.subpixel) return;
  const float py = a.pos[2 * j], px = a.pos[2 * j + 1];
  const float qy = floorf(py + 0.5f), qx = floorf(px + 0.5f);
  if (qy >= 0.f && qy <= (float)(a.H - N)) *fy = py - qy;
  if (qx >= 0.f && qx <= (float)(a.W - N)) *fx = px - qx;
}

__device__ __forceinline__ float2 ramp(int ky, int kx, float fy, float fx, float sg, int N) {
  float sn, cs;
  sincospif(sg * 2.f * ((float)ky * fy + (float)kx * fx) / (float)N, &sn, &cs);
  return make_float2(cs, sn);
}

// Column passes work on CW adjacent columns per workgroup, so every global
// access moves CW * 8 contiguous bytes of a row; pixel q of the group is row
// k = q / CW, column c = q % CW (consecutive threads: consecutive columns).
constexpr int kAdjCW1 = 8;  // passes with one transform per column
constexpr int kAdjCWM = 4;  // the mode pass (M transforms per column)
static_assert(kAdjCWM * 64 == kAdjThreads, "the mode pass stores one loss partial per wave and column");

__device__ __forceinline__ int col_group(int nunits) {
  return (nunits & 7) == 0 ? xcd_unit(blockIdx.x, nunits) : (int)blockIdx.x;
}


// P1 (cols): crop columns u0.. of position j0 + b, gathered from the object;
// C = S_y(crop) = F_y^-1(F_y(crop) e^{+2 pi i ky fy/N}) -> Cp
template <int N>
__device__ void adj_p1(const AdjArgs& a, float2* smem) {
  constexpr int CW = kAdjCW1, PIX = (N * CW + 255) / 256;
  constexpr int PT = col_pitch<N, CW, true>();  // LDS pitch (padded intermediates)
  const int u = col_group(gridDim.x), b = blockIdx.y;
  if (u >= N / CW) return;
  const int u0 = u * CW, j = a.j0 + b, tid = threadIdx.x;
  const int ny = box_corner(a.pos[2 * j], a.H - N, a.status);
  const int nx = box_corner(a.pos[2 * j + 1], a.W - N, a.status);
  float fy, fx;
  frac_of(a, j, N, &fy, &fx);
  float2* tw = smem;
  float2* A = tw + N;       // transform c at c * PT
  float2* B = A + CW * PT;
  float2 v[PIX];
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    v[i] = a.obj[(size_t)(ny + k) * a.W + nx + u0 + c];
  }
  load_twiddles<N, kAdjThreads>(tw);
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    A[c * PT + k] = v[i];
  }
  __syncthreads();
  float2* F = fft_lds<N, false, false, kAdjThreads, PT, true>(A, B, CW, tw);
  float2* G = (F == A) ? B : A;
  const float invN = 1.f / (float)N;
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    const int ky = k < N / 2 ? k : k - N;
    G[c * PT + k] = cscale(cmul(F[c * PT + k], ramp(ky, 0, fy, 0.f, 1.f, N)), invN);
  }
  __syncthreads();
  float2* H = fft_lds<N, true, false, kAdjThreads, PT, true>(G, F, CW, tw);
  float2* cp = a.Cp + chunk_off(b, N);
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    cp[(size_t)k * N + u0 + c] = H[c * PT + k];
  }
}

// Row passes that hold one row of a position per thread take this many
// positions per workgroup step, so that each FFT call keeps more of the
// workgroup's threads busy (one 256-point row keeps 32 of 256 busy in a
// radix-8 stage).
constexpr int kAdjRowPos = 2;

// P2 (rows): row r of C; o = S_x(C) (-> Ob); exit waves P_p o, row FFTs ->
// Psi.  A workgroup takes row r of kAdjRowPos consecutive positions, so each
// FFT call transforms that many rows (or M times as many) at once.
template <int N>
__device__ void adj_p2(const AdjArgs& a, float2* smem) {
  constexpr int MM = MRPIE_MAX_MODES;
  const int r = blockIdx.x, b0 = kAdjRowPos * blockIdx.y, M = a.M;
  const int ns = min(kAdjRowPos, a.nb - b0);  // positions of this workgroup
  const size_t NN = (size_t)N * N;
  float2* tw = smem;
  constexpr int PT = col_pitch<N, 1, true>();  // LDS pitch (padded intermediates)
  float2* A = tw + N;                    // kAdjRowPos M PT
  float2* B = A + kAdjRowPos * M * PT;   // kAdjRowPos M PT
  const int c = threadIdx.x;
  const int kx = c < N / 2 ? c : c - N;
  float2 v[kAdjRowPos], P[MM];
  float fx[kAdjRowPos] = {};
  if (c < N) {
#pragma unroll
    for (int q = 0; q < kAdjRowPos; ++q)
      if (q < ns) v[q] = a.Cp[chunk_off(b0 + q, N) + (size_t)r * N + c];
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) P[p] = a.probe[p * NN + (size_t)r * N + c];
  }
#pragma unroll
  for (int q = 0; q < kAdjRowPos; ++q) {
    float fy;
    if (q < ns) frac_of(a, a.j0 + b0 + q, N, &fy, &fx[q]);
  }
  load_twiddles<N, kAdjThreads>(tw);
  if (c < N) {
#pragma unroll
    for (int q = 0; q < kAdjRowPos; ++q)
      if (q < ns) A[q * PT + c] = v[q];
  }
  __syncthreads();
  float2* X = fft_lds<N, false, false, kAdjThreads, PT, true>(A, B, ns, tw);
  float2* Y = (X == A) ? B : A;
  if (c < N) {
#pragma unroll
    for (int q = 0; q < kAdjRowPos; ++q)
      if (q < ns) Y[q * PT + c] = cscale(cmul(X[q * PT + c], ramp(0, kx, 0.f, fx[q], 1.f, N)), 1.f / (float)N);
  }
  __syncthreads();
  float2* R = fft_lds<N, true, false, kAdjThreads, PT, true>(Y, X, ns, tw);
  float2* W = (R == A) ? B : A;
  if (c < N) {
#pragma unroll
    for (int q = 0; q < kAdjRowPos; ++q)
      if (q < ns) {
        const float2 o = R[q * PT + c];
        a.Ob[chunk_off(b0 + q, N) + (size_t)r * N + c] = o;
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) W[(q * M + p) * PT + c] = cmul(P[p], o);
      }
  }
  __syncthreads();
  fft_lds_store<N, false, false, kAdjThreads, PT, true>(W, R, ns * M, tw, [&](int t, int cc, float2 v) {
    const int q = t / M, p = t - q * M;
    a.Psi[((size_t)(b0 + q) * M + p) * NN + (size_t)r * N + cc] = v;
  });
}

// P3 (cols): Psi -> A, loss partial; chi = F^-1((1 - sqrt(I)/A) Psi)
// IP: in-place transforms (one M CW N buffer instead of two, so more
// workgroups share a CU; used while the register arrays it needs stay small)
// The mode pass takes kAdjP3Group consecutive positions per workgroup (up to
// four modes; one with more, where the prefetch registers would spill) and
// loads the next position's spectra and pattern columns while the current
// one's transforms run.
constexpr int kAdjP3Group = 4;
__host__ __device__ constexpr int adj_p3_group(int mm) { return mm <= 4 ? kAdjP3Group : 1; }

template <int N, int MM, bool IP>
__device__ void adj_p3(const AdjArgs& a, float2* smem) {
  constexpr int CW = kAdjCWM, PIX = (N * CW + 255) / 256, GRP = adj_p3_group(MM);
  const int u = col_group(gridDim.x), M = a.M;
  if (u >= N / CW) return;
  const int b0 = blockIdx.y * GRP, b1 = min(b0 + GRP, a.nb);
  const int u0 = u * CW, tid = threadIdx.x;
  const size_t NN = (size_t)N * N;
  float2* tw = smem;
  constexpr int PT = col_pitch<N, CW, true>();  // LDS pitch (padded intermediates)
  float2* A = tw + N;          // transform (p, c) at (p * CW + c) * PT
  float2* B = IP ? A : A + M * CW * PT;
  // pixel q = tid + 256 i of the group: row k = q / CW, column c = q % CW
  float2 nv[PIX][MM];
  float nI[PIX];
  auto fetch = [&](int bb) {
    const float2* psi = a.Psi + (size_t)bb * M * NN;
    const float* Ij = a.I + (size_t)(a.j0 + bb) * NN;
#pragma unroll
    for (int i = 0; i < PIX; ++i) {
      const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
      if (q >= N * CW) continue;
      const size_t off = (size_t)k * N + u0 + c;
      nI[i] = Ij[off];
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) nv[i][p] = psi[p * NN + off];
    }
  };
  if (b0 < b1) fetch(b0);
  load_twiddles<N, kAdjThreads>(tw);
  const float invN = 1.f / (float)N;
  for (int bb = b0; bb < b1; ++bb) {
    float Iv[PIX];
#pragma unroll
    for (int i = 0; i < PIX; ++i) {
      const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
      if (q >= N * CW) continue;
      Iv[i] = nI[i];
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) A[(p * CW + c) * PT + k] = nv[i][p];
    }
    if (bb + 1 < b1) fetch(bb + 1);
    lds_barrier();
    float2* F;
    if constexpr (IP) {
      fft_lds_inplace<N, false, false, MM * CW, 256, kAdjThreads, PT, true>(A, M * CW, tw);
      F = A;
    } else {
      F = fft_lds<N, false, false, kAdjThreads, PT, true>(A, B, M * CW, tw);
    }
    float2* G = IP ? F : ((F == A) ? B : A);  // (in place: each thread rescales the pixels it reads)
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < PIX; ++i) {
      const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
      if (q >= N * CW) continue;
      float S = 0.f;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) S += cabs2(F[(p * CW + c) * PT + k]);
      // hardware reciprocal square root and square root (about 1 ulp)
      const float rs = S > 0.f ? __builtin_amdgcn_rsqf(S) : 0.f;
      const float Au = S * rs;
      const float sq = __builtin_amdgcn_sqrtf(fmaxf(Iv[i], 0.f));
      const float d = Au * invN - sq;
      e += (double)d * (double)d;
      // (1 - sqrt(I)/A) with A = Au / N, and the 1/N^2 of the unnormalised
      // inverse 2-D transform
      const float wgt = S > 0.f ? (1.f - sq * (float)N * rs) * invN * invN : 0.f;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) G[(p * CW + c) * PT + k] = cscale(F[(p * CW + c) * PT + k], wgt);
    }
    lds_barrier();
    const float2* H;
    if constexpr (IP) {
      fft_lds_inplace<N, true, false, MM * CW, 256, kAdjThreads, PT, true>(G, M * CW, tw);
      H = G;
    } else {
      H = fft_lds<N, true, false, kAdjThreads, PT, true>(G, F, M * CW, tw);
    }
    float2* psi = a.Psi + (size_t)bb * M * NN;
#pragma unroll
    for (int i = 0; i < PIX; ++i) {
      const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
      if (q >= N * CW) continue;
      const size_t off = (size_t)k * N + u0 + c;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) psi[p * NN + off] = H[(p * CW + c) * PT + k];
    }
    // one partial per wave, in the slots of the group's CW columns (no
    // workgroup reduction per position)
    e = wave_sum(e);
    if ((tid & 63) == 0) a.loss_part[(size_t)bb * N + u0 + (tid >> 6)] = e;
    lds_barrier();  // this position's reads of the LDS buffers end before the next one's writes
  }
}

// The mode pass for radix-8 three-stage plans (N >= 128) with the first and
// last FFT stages in registers: each thread loads the inputs of its
// first-stage butterflies straight from the spectra, the last forward stage
// leaves each of CW * N / RL threads every mode of one column at RL
// frequencies, so the loss, the modulus weight and the first inverse stage
// need no LDS round trip, and the last inverse stage stores straight to the
// workspace.  The next position's butterfly inputs and pattern values are
// loaded while the current one's LDS stages run.
template <int N, int MM, bool IP>
__device__ void adj_p3_rd(const AdjArgs& a, float2* smem) {
  using P = Plan8<N>;
  constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2];
  static_assert(R2 > 1 && P::R[3] == 1, "three-stage plans only");
  constexpr int CW = kAdjCWM, GRP = adj_p3_group(MM), NT = kAdjThreads;
  constexpr int RL = R2, Q0 = N / R0, QL = N / RL;
  constexpr int IT1 = (MM * CW * Q0 + NT - 1) / NT;  // first-stage butterflies per thread
  static_assert(CW * QL <= NT, "one mode-sum thread per (column, frequency group)");
  constexpr int PT = col_pitch<N, CW>();             // LDS pitch of a transform
  constexpr int MB2 = (MM * CW * (N / R1) + NT - 1) / NT;
  const int u = col_group(gridDim.x), M = a.M;
  if (u >= N / CW) return;
  const int b0 = blockIdx.y * GRP, b1 = min(b0 + GRP, a.nb);
  const int u0 = u * CW, tid = threadIdx.x;
  const size_t NN = (size_t)N * N;
  float2* tw = smem;
  float2* A = tw + N;                    // transform (p, c) at (p * CW + c) * PT
  float2* B = IP ? A : A + M * CW * PT;
  const int nb1 = M * CW * Q0;
  const bool ms = tid < CW * QL;
  const int mc = tid % CW, mj = tid / CW;  // mode-sum thread: column, frequency group
  // butterfly b = tid + NT i: column c = b % CW, index j = (b / CW) % Q0 of
  // transform (p, c), p = b / (CW Q0), rows j + Q0 r
  float2 nv[IT1][R0];
  float nI[RL];
  auto fetch = [&](int bb) {
    const float2* psi = a.Psi + (size_t)bb * M * NN;
#pragma unroll
    for (int i = 0; i < IT1; ++i) {
      const int b = tid + NT * i;
      if (b < nb1) {
        const int c = b % CW, j = (b / CW) % Q0, p = b / (CW * Q0);
#pragma unroll
        for (int r = 0; r < R0; ++r) nv[i][r] = psi[p * NN + (size_t)(j + Q0 * r) * N + u0 + c];
      }
    }
    if (ms) {
      const float* Ij = a.I + (size_t)(a.j0 + bb) * NN;
#pragma unroll
      for (int r = 0; r < RL; ++r) nI[r] = Ij[(size_t)(mj + QL * r) * N + u0 + mc];
    }
  };
  if (b0 < b1) fetch(b0);
  load_twiddles<N, NT>(tw);
  const float invN = 1.f / (float)N;
  for (int bb = b0; bb < b1; ++bb) {
    // forward stage 1 (no twiddles) -> LDS
#pragma unroll
    for (int i = 0; i < IT1; ++i) {
      const int b = tid + NT * i;
      if (b < nb1) {
        const int c = b % CW, j = (b / CW) % Q0, p = b / (CW * Q0);
        dftR<R0, false>(nv[i]);
#pragma unroll
        for (int r = 0; r < R0; ++r) A[(p * CW + c) * PT + j * R0 + r] = nv[i][r];
      }
    }
    float Iv[RL];
#pragma unroll
    for (int r = 0; r < RL; ++r) Iv[r] = nI[r];
    if (bb + 1 < b1) fetch(bb + 1);
    lds_barrier();
    // forward stage 2
    if constexpr (IP) {
      stage_inplace<N, R1, R0, false, MB2, NT, PT>(A, M * CW, tw);
    } else {
      stage<N, R1, R0, false, NT, PT>(A, B, M * CW, tw);
      lds_barrier();
    }
    // forward stage 3 (every mode of one column per thread), loss, modulus
    // weight, inverse stage 1
    float2 X[MM][RL];
    if (ms) {
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) {
          const float2* src = B + (p * CW + mc) * PT;
#pragma unroll
          for (int r = 0; r < RL; ++r) X[p][r] = src[mj + QL * r];
        }
    }
    if constexpr (IP) lds_barrier();  // every read of the buffer before it is overwritten
    double e = 0.0;
    if (ms) {
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) {
#pragma unroll
          for (int r = 1; r < RL; ++r) X[p][r] = cmul(X[p][r], tw[r * mj]);
          dftR<RL, false>(X[p]);
        }
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        float S = 0.f;
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) S += cabs2(X[p][r]);
        // hardware reciprocal square root and square root (about 1 ulp)
        const float rs = S > 0.f ? __builtin_amdgcn_rsqf(S) : 0.f;
        const float Au = S * rs;
        const float sq = __builtin_amdgcn_sqrtf(fmaxf(Iv[r], 0.f));
        const float d = Au * invN - sq;
        e += (double)d * (double)d;
        // (1 - sqrt(I)/A) with A = Au / N, and the 1/N^2 of the unnormalised
        // inverse 2-D transform
        const float wgt = S > 0.f ? (1.f - sq * (float)N * rs) * invN * invN : 0.f;
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) X[p][r] = cscale(X[p][r], wgt);
      }
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) {
          dftR<RL, true>(X[p]);
          float2* dst = A + (p * CW + mc) * PT;
#pragma unroll
          for (int r = 0; r < RL; ++r) dst[mj * RL + r] = X[p][r];
        }
    }
    lds_barrier();
    // inverse stage 2
    if constexpr (IP) {
      stage_inplace<N, R1, RL, true, MB2, NT, PT>(A, M * CW, tw);
    } else {
      stage<N, R1, RL, true, NT, PT>(A, B, M * CW, tw);
      lds_barrier();
    }
    // inverse stage 3 -> the workspace
    float2* psi = a.Psi + (size_t)bb * M * NN;
#pragma unroll
    for (int i = 0; i < IT1; ++i) {
      const int b = tid + NT * i;
      if (b < nb1) {
        const int c = b % CW, j = (b / CW) % Q0, p = b / (CW * Q0);
        const float2* src = B + (p * CW + c) * PT;
        float2 w8[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) w8[r] = src[j + Q0 * r];
#pragma unroll
        for (int r = 1; r < R0; ++r) {
          float2 w = tw[r * j];
          w.y = -w.y;
          w8[r] = cmul(w8[r], w);
        }
        dftR<R0, true>(w8);
#pragma unroll
        for (int r = 0; r < R0; ++r) psi[p * NN + (size_t)(j + Q0 * r) * N + u0 + c] = w8[r];
      }
    }
    // one partial per wave, in the slots of the group's CW columns
    e = wave_sum(e);
    if ((tid & 63) == 0) a.loss_part[(size_t)bb * N + u0 + (tid >> 6)] = e;
    lds_barrier();  // this position's reads of the LDS buffers end before the next one's writes
  }
}

// P4 (rows): chi row r; g = 2 sum_p conj(P_p) chi_p; the x part of the
// position gradient from F_x g and F_x o; h = S_{-x}(g) -> G.  A workgroup
// takes row r of kAdjGroup consecutive positions, kAdjRowPos at a time (each
// FFT call transforms all of their rows), and sums their probe-gradient terms
// 2 conj(o) chi_p in registers; the group's partial replaces row r of its
// first position's Psi (which only this workgroup reads), so the probe
// gradient is reduced from one array per group.  Each wave stores its own
// partial of the x gradient (no workgroup barrier per position).
constexpr int kAdjGroup = 8;

template <int N, int MM>
__device__ void adj_p4(const AdjArgs& a, float2* smem) {
  const int r = blockIdx.x, M = a.M;
  const int NB = M > 2 ? kAdjRowPos * M : 2 * kAdjRowPos;  // transforms per buffer: the step's modes, then its g and o
  const int b0 = blockIdx.y * kAdjGroup, b1 = min(b0 + kAdjGroup, a.nb);
  const size_t NN = (size_t)N * N;
  float2* tw = smem;
  constexpr int PT = col_pitch<N, 1, true>();  // LDS pitch (padded intermediates)
  float2* A = tw + N;        // NB PT
  float2* B = A + NB * PT;   // NB PT
  const int c = threadIdx.x, wave = threadIdx.x >> 6;
  const int kx = c < N / 2 ? c : c - N;
  const size_t roff = (size_t)r * N + c;
  float2 P[MM], acc[MM];
#pragma unroll
  for (int p = 0; p < MM; ++p) {
    acc[p] = make_float2(0.f, 0.f);
    if (p < M && c < N) P[p] = a.probe[p * NN + roff];
  }
  load_twiddles<N, kAdjThreads>(tw);
  // software pipeline: the next step's spectra rows and o rows are loaded
  // into registers while this step's transforms run (the LDS barriers of
  // the transforms leave those loads in flight)
  float2 nv[kAdjRowPos][MM], no[kAdjRowPos];
  auto fetch = [&](int bb) {
    if (c >= N) return;
#pragma unroll
    for (int q = 0; q < kAdjRowPos; ++q)
      if (bb + q < b1) {
        no[q] = a.Ob[chunk_off(bb + q, N) + roff];
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) nv[q][p] = a.Psi[((size_t)(bb + q) * M + p) * NN + roff];
      }
  };
  if (b0 < b1) fetch(b0);
  for (int b = b0; b < b1; b += kAdjRowPos) {
    const int ns = min(kAdjRowPos, b1 - b);
    float fx[kAdjRowPos] = {};
#pragma unroll
    for (int q = 0; q < kAdjRowPos; ++q) {
      float fy;
      if (q < ns) frac_of(a, a.j0 + b + q, N, &fy, &fx[q]);
    }
    float2 o[kAdjRowPos];
    if (c < N) {
#pragma unroll
      for (int q = 0; q < kAdjRowPos; ++q)
        if (q < ns) {
          o[q] = no[q];
#pragma unroll
          for (int p = 0; p < MM; ++p)
            if (p < M) A[(q * M + p) * PT + c] = nv[q][p];
        }
    }
    if (b + kAdjRowPos < b1) fetch(b + kAdjRowPos);
    lds_barrier();
    float2* R = fft_lds<N, true, false, kAdjThreads, PT, true>(A, B, ns * M, tw);
    float2* W = (R == A) ? B : A;
    if (c < N) {
#pragma unroll
      for (int q = 0; q < kAdjRowPos; ++q)
        if (q < ns) {
          float2 g = make_float2(0.f, 0.f);
#pragma unroll
          for (int p = 0; p < MM; ++p)
            if (p < M) {
              const float2 chi = R[(q * M + p) * PT + c];
              acc[p] = cadd(acc[p], cscale(cmulc(chi, o[q]), 2.f));   // 2 chi conj(o)
              g = cadd(g, cmulc(chi, P[p]));
            }
          W[(2 * q) * PT + c] = cscale(g, 2.f);
          W[(2 * q + 1) * PT + c] = o[q];
        }
    }
    lds_barrier();
    float2* S = fft_lds<N, false, false, kAdjThreads, PT, true>(W, R, 2 * ns, tw);  // F_x g, F_x o
    float2* T = (S == A) ? B : A;
    double gx[kAdjRowPos] = {};
    if (c < N) {
#pragma unroll
      for (int q = 0; q < kAdjRowPos; ++q)
        if (q < ns) {
          const float2 fg = S[(2 * q) * PT + c];
          // Re conj(F g) (i w) F o = -w Im(conj(F g) F o), w = 2 pi kx / N
          const float2 cf = cmulc(S[(2 * q + 1) * PT + c], fg);  // F o conj(F g)
          gx[q] = -2.0 * M_PI * (double)kx / (double)N * (double)cf.y / (double)N;
          T[q * PT + c] = cscale(cmul(fg, ramp(0, kx, 0.f, fx[q], -1.f, N)), 1.f / (float)N);
        }
    }
    lds_barrier();
    fft_lds_store<N, true, false, kAdjThreads, PT, true>(T, S, ns, tw, [&](int q, int cc, float2 v) {
      a.G[chunk_off(b + q, N) + (size_t)r * N + cc] = v;
    });
#pragma unroll
    for (int q = 0; q < kAdjRowPos; ++q)
      if (q < ns) {
        const double v = wave_sum(gx[q]);
        if ((threadIdx.x & 63) == 0 && a.subpixel)
          a.pos_part[((size_t)(b + q) * N + r) * kPosSlots + 1 + wave] = v;
      }
    lds_barrier();  // A, B are reused by the next step
  }
  if (c < N) {
    float2* part = a.Psi + (size_t)b0 * M * NN;
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) part[p * NN + roff] = acc[p];
  }
}

// P5 (cols): the y part of the position gradient from F_y h and F_y C;
// S_{-y}(h) = S_{-f}(g) -> G (the object-gradient term)
template <int N>
__device__ void adj_p5(const AdjArgs& a, float2* smem) {
  constexpr int CW = kAdjCW1, PIX = (N * CW + 255) / 256;
  constexpr int PT = col_pitch<N, CW, true>();  // LDS pitch (padded intermediates)
  const int u = col_group(gridDim.x), b = blockIdx.y;
  if (u >= N / CW) return;
  const int u0 = u * CW, j = a.j0 + b, tid = threadIdx.x;
  float fy, fx;
  frac_of(a, j, N, &fy, &fx);
  float2* tw = smem;
  float2* A = tw + N;
  float2* B = A + CW * PT;
  __shared__ double redd[16];
  float2* g = a.G + chunk_off(b, N);
  const float2* cp = a.Cp + chunk_off(b, N);
  float2 hv[PIX], cv[PIX];
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    cv[i] = cp[(size_t)k * N + u0 + c];
    hv[i] = g[(size_t)k * N + u0 + c];
  }
  load_twiddles<N, kAdjThreads>(tw);
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    A[c * PT + k] = cv[i];
  }
  __syncthreads();
  float2* F = fft_lds<N, false, false, kAdjThreads, PT, true>(A, B, CW, tw);  // F_y C
  float2* X = (F == A) ? B : A;
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    cv[i] = F[c * PT + k];
    X[c * PT + k] = hv[i];
  }
  __syncthreads();
  float2* Fh = fft_lds<N, false, false, kAdjThreads, PT, true>(X, F, CW, tw);  // F_y h
  float2* Y = (Fh == A) ? B : A;
  double gy = 0.0;
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    const int ky = k < N / 2 ? k : k - N;
    const float2 fh = Fh[c * PT + k];
    const float2 cf = cmulc(cv[i], fh);  // F C conj(F h)
    gy += -2.0 * M_PI * (double)ky / (double)N * (double)cf.y / (double)N;
    Y[c * PT + k] = cscale(cmul(fh, ramp(ky, 0, fy, 0.f, -1.f, N)), 1.f / (float)N);
  }
  __syncthreads();
  float2* H = fft_lds<N, true, false, kAdjThreads, PT, true>(Y, Fh, CW, tw);
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + 256 * i, k = q / CW, c = q - k * CW;
    if (q >= N * CW) continue;
    g[(size_t)k * N + u0 + c] = H[c * PT + k];
  }
  gy = block_sum(gy, redd);
  // one partial per column group, in the slot of its first column
  if (tid < CW && a.subpixel) a.pos_part[((size_t)b * N + u0 + tid) * kPosSlots] = tid == 0 ? gy : 0.0;
}

// P1 for radix-8 three-stage plans (N >= 128) with the first and last FFT
// stages in registers, kAdjCWR columns per workgroup: the first stage takes
// the global loads, the last forward stage leaves each of kAdjCWR * N / RL
// threads one column at RL frequencies, where the ramp and the first
// inverse stage run without an LDS round trip, and the last inverse stage
// stores straight to the workspace.  (The same for P5, with two fields per
// column, was slower than its staged version: 111.6 against 102.0 us per
// 256 positions at 256^2.)
constexpr int kAdjCWR = 4;

template <int N>
struct AdjRd {
  using P = Plan8<N>;
  static constexpr int R0 = P::R[0], R1 = P::R[1], RL = P::R[2];
  static_assert(RL > 1 && P::R[3] == 1, "three-stage plans only");
  static constexpr int Q0 = N / R0, QL = N / RL, CW = kAdjCWR;
  static constexpr int PT = col_pitch<N, CW>();  // LDS pitch of a transform
  static_assert(CW * QL <= kAdjThreads, "one ramp thread per (column, frequency group)");
};

template <int N>
__device__ void adj_p1_rd(const AdjArgs& a, float2* smem) {
  using D = AdjRd<N>;
  constexpr int R0 = D::R0, R1 = D::R1, RL = D::RL, Q0 = D::Q0, QL = D::QL, CW = D::CW, PT = D::PT;
  constexpr int NT = kAdjThreads;
  const int u = col_group(gridDim.x), b = blockIdx.y;
  if (u >= N / CW) return;
  const int u0 = u * CW, j = a.j0 + b, tid = threadIdx.x;
  const int ny = box_corner(a.pos[2 * j], a.H - N, a.status);
  const int nx = box_corner(a.pos[2 * j + 1], a.W - N, a.status);
  float fy, fx;
  frac_of(a, j, N, &fy, &fx);
  float2* tw = smem;
  float2* A = tw + N;       // transform c at c * PT
  float2* B = A + CW * PT;
  // first-stage butterfly tid: column c = tid % CW, index jj = tid / CW
  const bool s1 = tid < CW * Q0;
  const int c1 = tid % CW, j1 = tid / CW;
  float2 v[R0];
  if (s1) {
#pragma unroll
    for (int r = 0; r < R0; ++r) v[r] = a.obj[(size_t)(ny + j1 + Q0 * r) * a.W + nx + u0 + c1];
  }
  load_twiddles<N, NT>(tw);
  if (s1) {
    dftR<R0, false>(v);
#pragma unroll
    for (int r = 0; r < R0; ++r) A[c1 * PT + j1 * R0 + r] = v[r];
  }
  __syncthreads();
  stage<N, R1, R0, false, NT, PT>(A, B, CW, tw);
  __syncthreads();
  // last forward stage, the ramp e^{+2 pi i ky fy / N} / N, first inverse stage
  const bool ms = tid < CW * QL;
  const int mc = tid % CW, mj = tid / CW;
  if (ms) {
    float2 X[RL];
#pragma unroll
    for (int r = 0; r < RL; ++r) X[r] = B[mc * PT + mj + QL * r];
#pragma unroll
    for (int r = 1; r < RL; ++r) X[r] = cmul(X[r], tw[r * mj]);
    dftR<RL, false>(X);
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int k = mj + QL * r, ky = k < N / 2 ? k : k - N;
      X[r] = cscale(cmul(X[r], ramp(ky, 0, fy, 0.f, 1.f, N)), 1.f / (float)N);
    }
    dftR<RL, true>(X);
#pragma unroll
    for (int r = 0; r < RL; ++r) A[mc * PT + mj * RL + r] = X[r];
  }
  __syncthreads();
  stage<N, R1, RL, true, NT, PT>(A, B, CW, tw);
  __syncthreads();
  if (s1) {
#pragma unroll
    for (int r = 0; r < R0; ++r) v[r] = B[c1 * PT + j1 + Q0 * r];
#pragma unroll
    for (int r = 1; r < R0; ++r) {
      float2 w = tw[r * j1];
      w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    dftR<R0, true>(v);
    float2* cp = a.Cp + chunk_off(b, N);
#pragma unroll
    for (int r = 0; r < R0; ++r) cp[(size_t)(j1 + Q0 * r) * N + u0 + c1] = v[r];
  }
}

template <int N>
__device__ void adj_p1_any(const AdjArgs& a, float2* smem) {
  if constexpr (N >= 128) adj_p1_rd<N>(a, smem);
  else adj_p1<N>(a, smem);
}

#define MRPIE_ADJ_KERNEL(NAME, FN)                       \
  __global__ __launch_bounds__(256) void NAME(const AdjArgs a) { \
    extern __shared__ float2 smem[];                     \
    switch (a.N) {                                       \
      case 32: FN<32>(a, smem); break;                   \
      case 64: FN<64>(a, smem); break;                   \
      case 128: FN<128>(a, smem); break;                 \
      case 192: FN<192>(a, smem); break;                 \
      default: FN<256>(a, smem); break;                  \
    }                                                    \
  }
MRPIE_ADJ_KERNEL(k_adj_p1, adj_p1_any)
MRPIE_ADJ_KERNEL(k_adj_p2, adj_p2)
// the mode pass per bound MM >= M on the modes (register arrays of the
// in-place transforms)
template <int MM>
__global__ __launch_bounds__(256) void k_adj_p3(const AdjArgs a) {
  constexpr bool IP = MM <= 4;
  extern __shared__ float2 smem[];
  switch (a.N) {
    case 32: adj_p3<32, MM, IP>(a, smem); break;
    case 64: adj_p3<64, MM, IP>(a, smem); break;
    case 128: adj_p3_rd<128, MM, IP>(a, smem); break;
    case 192: adj_p3_rd<192, MM, IP>(a, smem); break;
    default: adj_p3_rd<256, MM, IP>(a, smem); break;
  }
}
template <int MM>
__global__ __launch_bounds__(256) void k_adj_p4(const AdjArgs a) {
  extern __shared__ float2 smem[];
  switch (a.N) {
    case 32: adj_p4<32, MM>(a, smem); break;
    case 64: adj_p4<64, MM>(a, smem); break;
    case 128: adj_p4<128, MM>(a, smem); break;
    case 192: adj_p4<192, MM>(a, smem); break;
    default: adj_p4<256, MM>(a, smem); break;
  }
}
MRPIE_ADJ_KERNEL(k_adj_p5, adj_p5)

// ---------------------------------------------------------------- reductions
// loss += sum over the chunk's (position, column) partials, in order: each
// of kLossBlocks workgroups sums one contiguous range, then one workgroup
// adds the range sums
constexpr int kLossBlocks = 64;
__global__ __launch_bounds__(256) void k_adj_loss_part(const AdjArgs a, int nb) {
  __shared__ double red[16];
  const int n = nb * a.N, per = (n + kLossBlocks - 1) / kLossBlocks;
  const int i0 = blockIdx.x * per, i1 = min(n, i0 + per);
  double v = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) v += a.loss_part[i];
  v = block_sum(v, red);
  if (threadIdx.x == 0) a.loss_blk[blockIdx.x] = v;
}

__global__ __launch_bounds__(64) void k_adj_loss(const AdjArgs a) {
  __shared__ double red[16];
  double v = a.loss_blk[threadIdx.x];
  v = block_sum(v, red);
  if (threadIdx.x == 0) *a.loss_acc += v;
}

// grad_pos[j] = sum over columns of the position partials
__global__ __launch_bounds__(256) void k_adj_pos(const AdjArgs a, int nb) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  double gy = 0.0, gx = 0.0;
  for (int u = threadIdx.x; u < a.N; u += blockDim.x) {
    const double* pp = a.pos_part + ((size_t)b * a.N + u) * kPosSlots;
    gy += pp[0];
    gx += (pp[1] + pp[2]) + (pp[3] + pp[4]);
  }
  gy = block_sum(gy, red);
  gx = block_sum(gx, red);
  if (threadIdx.x == 0) {
    a.grad_pos[2 * (a.j0 + b)] = a.subpixel ? (float)gy : 0.f;
    a.grad_pos[2 * (a.j0 + b) + 1] = a.subpixel ? (float)gx : 0.f;
  }
}

// grad_P += the chunk's group partials of 2 chi conj(o), in position order
__global__ __launch_bounds__(256) void k_adj_probe(const AdjArgs a, int nb) {
  const size_t MNN = (size_t)a.M * a.N * a.N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < MNN; i += (size_t)gridDim.x * blockDim.x) {
    float2 s = a.grad_probe[i];
    for (int b = 0; b < nb; b += kAdjGroup) s = cadd(s, a.Psi[(size_t)b * MNN + i]);
    a.grad_probe[i] = s;
  }
}

// grad_O += the chunk's S_{-f}(g) patches at their boxes, in position order.
// One workgroup per 16 x 16 object tile; it lists the overlapping boxes
// first, so each pixel visits only those.
constexpr int kObjTile = 16;
__global__ __launch_bounds__(256) void k_adj_object(const AdjArgs a, int nb) {
  __shared__ int lst[kAdjChunk];
  __shared__ int boxes[kAdjChunk][2];
  __shared__ int cnt;
  const int N = a.N;
  const int ty0 = blockIdx.y * kObjTile, tx0 = blockIdx.x * kObjTile;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int j = a.j0 + b;
    const int ny = box_corner(a.pos[2 * j], a.H - N, nullptr);
    const int nx = box_corner(a.pos[2 * j + 1], a.W - N, nullptr);
    boxes[b][0] = ny;
    boxes[b][1] = nx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int n = 0;
    for (int b = 0; b < nb; ++b) {
      const int ny = boxes[b][0], nx = boxes[b][1];
      if (ny < ty0 + kObjTile && ny + N > ty0 && nx < tx0 + kObjTile && nx + N > tx0) lst[n++] = b;
    }
    cnt = n;
  }
  __syncthreads();
  const int y = ty0 + threadIdx.x / kObjTile, x = tx0 + threadIdx.x % kObjTile;
  if (y >= a.H || x >= a.W) return;
  float2 s = a.grad_obj[(size_t)y * a.W + x];
  for (int q = 0; q < cnt; ++q) {
    const int b = lst[q];
    const int dy = y - boxes[b][0], dx = x - boxes[b][1];
    if (dy >= 0 && dy < N && dx >= 0 && dx < N) s = cadd(s, a.G[chunk_off(b, N) + (size_t)dy * N + dx]);
  }
  a.grad_obj[(size_t)y * a.W + x] = s;
}

__global__ void k_adj_zero(float2* p, size_t n, double* d) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_float2(0.f, 0.f);
  if (d && blockIdx.x == 0 && threadIdx.x == 0) *d = 0.0;
}

__global__ void k_adj_loss_out(const double* acc, double* out) {
  if (threadIdx.x == 0) *out = *acc;
}

// ---------------------------------------------------------------- host
AdjLayout adj_layout(int N, int M, int J) {
  AdjLayout L{};
  const int B = std::max(1, std::min(J, kAdjChunk));
  const size_t NN = (size_t)N * N;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = ws_align(off + bytes); return o; };
  L.chunk = B;
  L.Cp = take((size_t)B * NN * 8);
  L.Ob = take((size_t)B * NN * 8);
  L.G = take((size_t)B * NN * 8);
  L.Psi = take((size_t)B * M * NN * 8);
  L.loss_part = take((size_t)B * N * 8);
  L.pos_part = take((size_t)B * N * kPosSlots * 8);
  L.loss_blk = take((size_t)kLossBlocks * 8);
  L.loss_acc = take(16);
  L.total = off;
  return L;
}

int run_adjoint(const mrpie_problem* pb, int subpixel, const float2* obj, const float2* probe, const float* pos,
                const float* intens, double* loss_out, float2* gobj, float2* gprobe, float* gpos, int32_t* status,
                void* ws, size_t ws_bytes, hipStream_t s) {
  const int N = pb->N, M = pb->M, J = pb->J;
  const AdjLayout L = adj_layout(N, M, J);
  if (!ws || ws_bytes < L.total) return fail(MRPIE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
  int rc = launch_init_twiddles(s);
  if (rc) return rc;
  char* w = (char*)ws;
  const bool grads = gobj != nullptr;
  AdjArgs a{};
  a.H = pb->H; a.W = pb->W; a.N = N; a.M = M; a.J = J; a.subpixel = subpixel;
  a.obj = obj; a.probe = probe; a.pos = pos; a.I = intens; a.status = status;
  a.Cp = (float2*)(w + L.Cp); a.Ob = (float2*)(w + L.Ob); a.G = (float2*)(w + L.G); a.Psi = (float2*)(w + L.Psi);
  a.loss_part = (double*)(w + L.loss_part); a.pos_part = (double*)(w + L.pos_part);
  a.loss_blk = (double*)(w + L.loss_blk);
  a.loss_acc = (double*)(w + L.loss_acc);
  a.grad_obj = gobj; a.grad_probe = gprobe; a.grad_pos = gpos;
  hipLaunchKernelGGL(k_adj_zero, dim3(1), dim3(64), 0, s, (float2*)nullptr, (size_t)0, a.loss_acc);
  if (grads) {
    hipLaunchKernelGGL(k_adj_zero, dim3(2048), dim3(256), 0, s, gobj, (size_t)pb->H * pb->W, (double*)nullptr);
    hipLaunchKernelGGL(k_adj_zero, dim3(256), dim3(256), 0, s, gprobe, (size_t)M * N * N, (double*)nullptr);
  }
  // LDS of the row passes (kAdjRowPos M transforms; P4 at least 2 kAdjRowPos)
  // at the padded pitch
  // col_pitch<N, 1, true>(), of the single-field column passes (kAdjCW1
  // transforms) and of the mode column pass at col_pitch<N, CW, true>()
  const size_t pr = (size_t)(N + N / 16 + 15) / 16 * 16;
  const size_t l2 = (N + 2 * kAdjRowPos * M * pr) * 8, l4 = (N + 2 * kAdjRowPos * std::max(M, 2) * pr) * 8;
  const size_t pbase = pr, p1 = pbase + 16 / kAdjCW1, pm = pbase + 16 / kAdjCWM;
  const size_t lc1 = (size_t)(N + 2 * kAdjCW1 * p1) * 8, lcm = (size_t)(N + (M <= 4 ? 1 : 2) * M * kAdjCWM * pm) * 8;
  // from N = 128 P1 takes kAdjCWR columns per workgroup at the pitch
  // N + 16 / kAdjCWR
  const bool rd = N >= 128;
  const int cw1 = rd ? kAdjCWR : kAdjCW1;
  const size_t lp1 = rd ? (N + 2 * kAdjCWR * ((size_t)N + 16 / kAdjCWR)) * 8 : lc1;
  MRPIE_HIP(ensure_lds((const void*)k_adj_p1, lp1));
  MRPIE_HIP(ensure_lds((const void*)k_adj_p2, l2));
  const auto kp4 = M <= 1 ? k_adj_p4<1> : M <= 2 ? k_adj_p4<2> : M <= 4 ? k_adj_p4<4> : k_adj_p4<MRPIE_MAX_MODES>;
  MRPIE_HIP(ensure_lds((const void*)kp4, l4));
  MRPIE_HIP(ensure_lds((const void*)k_adj_p5, lc1));
  const auto kp3 = M <= 1 ? k_adj_p3<1> : M <= 2 ? k_adj_p3<2> : M <= 4 ? k_adj_p3<4> : k_adj_p3<MRPIE_MAX_MODES>;
  const int g3 = adj_p3_group(M <= 4 ? 4 : MRPIE_MAX_MODES);  // positions per workgroup of k_adj_p3
  MRPIE_HIP(ensure_lds((const void*)kp3, lcm));
  for (int j0 = 0; j0 < J; j0 += L.chunk) {
    const int nb = std::min(L.chunk, J - j0);
    a.j0 = j0;
    a.nb = nb;
    const dim3 gp1(N / cw1, nb), g1(N / kAdjCW1, nb), blk(kAdjThreads);
    hipLaunchKernelGGL(k_adj_p1, gp1, blk, lp1, s, a);
    hipLaunchKernelGGL(k_adj_p2, dim3(N, (nb + kAdjRowPos - 1) / kAdjRowPos), blk, l2, s, a);
    launch_ku(TK_ADJ, nb, kp3, dim3(N / kAdjCWM, (nb + g3 - 1) / g3), blk, lcm, s, a);  // timed per position
    hipLaunchKernelGGL(k_adj_loss_part, dim3(kLossBlocks), blk, 0, s, a, nb);
    hipLaunchKernelGGL(k_adj_loss, dim3(1), dim3(kLossBlocks), 0, s, a);
    if (grads) {
      hipLaunchKernelGGL(kp4, dim3(N, (nb + kAdjGroup - 1) / kAdjGroup), blk, l4, s, a);
      hipLaunchKernelGGL(k_adj_p5, g1, blk, lc1, s, a);
      hipLaunchKernelGGL(k_adj_pos, dim3(nb), blk, 0, s, a, nb);
      hipLaunchKernelGGL(k_adj_probe, dim3(512), blk, 0, s, a, nb);
      hipLaunchKernelGGL(k_adj_object, dim3((pb->W + kObjTile - 1) / kObjTile, (pb->H + kObjTile - 1) / kObjTile),
                         blk, 0, s, a, nb);
    }
  }
  if (loss_out) hipLaunchKernelGGL(k_adj_loss_out, dim3(1), dim3(64), 0, s, (const double*)a.loss_acc, loss_out);
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

}  // namespace mrpie

using namespace mrpie;

extern "C" {

int mrpie_grad_workspace_size(const mrpie_problem* pb, size_t* bytes) {
  if (!pb || !bytes) return fail(MRPIE_EINVAL, "null argument");
  if (n_index(pb->N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", pb->N);
  if (pb->M < 1 || pb->M > MRPIE_MAX_MODES || pb->J < 1 || pb->H < pb->N || pb->W < pb->N)
    return fail(pb->M > MRPIE_MAX_MODES ? MRPIE_EUNSUPPORTED : MRPIE_EINVAL, "bad problem shape");
  *bytes = adj_layout(pb->N, pb->M, pb->J).total;
  return MRPIE_OK;
}

static int adj_check(const mrpie_problem* pb, int subpixel, const void* obj, const void* probe, const float* pos,
                     const float* intens) {
  size_t n;
  int rc = mrpie_grad_workspace_size(pb, &n);
  if (rc) return rc;
  if (subpixel != 0 && subpixel != 1) return fail(MRPIE_EINVAL, "subpixel must be 0 or 1");
  if ((long long)pb->H * pb->W >= (1LL << 31)) return fail(MRPIE_EINVAL, "object too large");
  if (!obj || !probe || !pos || !intens) return fail(MRPIE_EINVAL, "null array pointer");
  return MRPIE_OK;
}

int mrpie_loss(const mrpie_problem* pb, int32_t subpixel, const void* obj, const void* probe, const float* pos,
               const float* intens, double* loss_out, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  int rc = adj_check(pb, subpixel, obj, probe, pos, intens);
  if (rc) return rc;
  if (!loss_out) return fail(MRPIE_EINVAL, "loss_out is NULL");
  return run_adjoint(pb, subpixel, (const float2*)obj, (const float2*)probe, pos, intens, loss_out, nullptr, nullptr,
                     nullptr, status, ws, ws_bytes, (hipStream_t)stream);
}

int mrpie_adjoint(const mrpie_problem* pb, int32_t subpixel, const void* obj, const void* probe, const float* pos,
                  const float* intens, double* loss_out, void* grad_obj, void* grad_probe, float* grad_pos,
                  int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  int rc = adj_check(pb, subpixel, obj, probe, pos, intens);
  if (rc) return rc;
  if (!grad_obj || !grad_probe || !grad_pos) return fail(MRPIE_EINVAL, "null gradient pointer");
  return run_adjoint(pb, subpixel, (const float2*)obj, (const float2*)probe, pos, intens, loss_out,
                     (float2*)grad_obj, (float2*)grad_probe, grad_pos, status, ws, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"
