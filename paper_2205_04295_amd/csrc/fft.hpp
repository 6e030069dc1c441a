// Batched 1-D complex FFTs staged in LDS for gfx950.
//
// Mixed-radix Stockham auto-sort: every stage reads R points at stride N/R,
// applies the twiddles w_N^(r * (j mod Ns) * N/(Ns R)), performs an R-point
// DFT in registers and writes them at stride Ns; the buffers ping-pong in
// LDS, one workgroup barrier per stage.  Radices 8/4/3 cover the probe sizes
// N in {64, 128, 192, 256}: 64 = 8*8, 128 = 8*4*4, 192 = 8*8*3,
// 256 = 8*8*4.  Twiddles are the N-th roots of unity rounded to float from
// double-precision values (table written once per call by a small kernel).
//
// All transforms are unnormalised (sum over e^{-+2 pi i k n / N}); callers
// fold the 1/N of the unitary 2-D transform into one multiply.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace mrpie {

struct c32 {
  float x, y;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2* v) {
  float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  float2 a2 = cadd(v[1], v[3]), a3 = rot90<INV>(csub(v[1], v[3]));
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  const float h = 0.70710678118654752440f;
  // split into even / odd halves, two 4-point DFTs, combine with w_8^k
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // w_8^1 = (1 -+ i)/sqrt2, w_8^2 = -+i, w_8^3 = (-1 -+ i)/sqrt2
  float2 o1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                  : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
  float2 o2 = rot90<INV>(o[2]);
  float2 o3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                  : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2* v) {
  const float c = -0.5f;
  const float s = INV ? 0.86602540378443864676f : -0.86602540378443864676f;
  float2 t1 = cadd(v[1], v[2]);
  float2 t2 = csub(v[1], v[2]);
  float2 m1 = make_float2(v[0].x + c * t1.x, v[0].y + c * t1.y);
  float2 m2 = make_float2(-s * t2.y, s * t2.x);  // i s t2
  v[0] = cadd(v[0], t1);
  v[1] = cadd(m1, m2);
  v[2] = csub(m1, m2);
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else dft2<INV>(v[0], v[1]);
}

// Stage plans (radix per stage, first to last; 1 = no stage).
//   Plan8: fewest stages (radix 8), for throughput-bound batches.
//   Plan4: radix 4 (+2 / 3), twice the threads per transform and half the
//          work per thread and stage: shorter latency for small batches.
template <int N> struct Plan8;
template <> struct Plan8<64>  { static constexpr int R[4] = {8, 8, 1, 1}; };
template <> struct Plan8<128> { static constexpr int R[4] = {8, 4, 4, 1}; };
template <> struct Plan8<192> { static constexpr int R[4] = {8, 8, 3, 1}; };
template <> struct Plan8<256> { static constexpr int R[4] = {8, 8, 4, 1}; };
template <int N> struct Plan4;
template <> struct Plan4<64>  { static constexpr int R[4] = {4, 4, 4, 1}; };
template <> struct Plan4<128> { static constexpr int R[4] = {4, 4, 4, 2}; };
template <> struct Plan4<192> { static constexpr int R[4] = {4, 4, 4, 3}; };
template <> struct Plan4<256> { static constexpr int R[4] = {4, 4, 4, 4}; };

// One Stockham stage over `nb` transforms of length N stored contiguously
// (transform t at src + t*N).  tw: N-th roots w_N^e = exp(-2 pi i e / N).
template <int N, int R, int NS, bool INV>
__device__ __forceinline__ void stage(const float2* __restrict__ src, float2* __restrict__ dst, int nb,
                                      const float2* __restrict__ tw) {
  constexpr int Q = N / R;
  constexpr int TWS = N / (NS * R);
  const int total = nb * Q;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int b = t / Q;
    const int j = t - b * Q;
    const float2* s = src + b * N;
    float2* d = dst + b * N;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * Q];
    if constexpr (NS > 1) {
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * k * TWS];  // r*k*TWS < N
        if constexpr (INV) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    dftR<R, INV>(v);
    const int o = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) d[o + r * NS] = v[r];
  }
}

// Full N-point transforms of `nb` contiguous rows in LDS buffer `a`, using
// `b` as the ping-pong partner.  Returns the buffer holding the result.
// Callers must __syncthreads() before (data ready); the result is ready on
// return (a barrier ends every stage).
template <int N, bool INV, bool R4 = true>
__device__ float2* fft_lds(float2* a, float2* b, int nb, const float2* __restrict__ tw) {
  using P = typename std::conditional<R4, Plan4<N>, Plan8<N>>::type;
  constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2], R3 = P::R[3];
  stage<N, R0, 1, INV>(a, b, nb, tw);
  __syncthreads();
  stage<N, R1, R0, INV>(b, a, nb, tw);
  __syncthreads();
  if constexpr (R2 == 1) return a;
  stage<N, R2, R0 * R1, INV>(a, b, nb, tw);
  __syncthreads();
  if constexpr (R3 == 1) return b;
  stage<N, R3, R0 * R1 * R2, INV>(b, a, nb, tw);
  __syncthreads();
  return a;
}

}  // namespace mrpie
