// Batched 1-D complex FFTs staged in LDS for gfx950, in float (complex64)
// or double (complex128) precision.
//
// Mixed-radix Stockham auto-sort: every stage reads R points at stride N/R,
// applies the twiddles w_N^(r * (j mod Ns) * N/(Ns R)), performs an R-point
// DFT in registers and writes them at stride Ns; the buffers ping-pong in
// LDS, one workgroup barrier per stage.  Radices 8/4/3/2 cover the probe
// sizes N in {32, 64, 128, 192, 256}.  Twiddles are the N-th roots of unity from
// double-precision sincospi (rounded once to float for the float path).
//
// All transforms are unnormalised (sum over e^{-+2 pi i k n / N}); callers
// fold the 1/N of the unitary 2-D transform into one multiply.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace mrpie {

template <typename C> struct real_of;
template <> struct real_of<float2> { using type = float; };
template <> struct real_of<double2> { using type = double; };

__device__ __forceinline__ float2 mk(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ double2 mk(double x, double y) { return make_double2(x, y); }

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C>
__device__ __forceinline__ C cmulc(C a, C b) {  // a * conj(b)
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return mk(a.x + b.x, a.y + b.y); }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return mk(a.x - b.x, a.y - b.y); }
template <typename C, typename R>
__device__ __forceinline__ C cscale(C a, R s) { return mk(a.x * s, a.y * s); }
template <typename C>
__device__ __forceinline__ auto cabs2(C a) { return a.x * a.x + a.y * a.y; }
template <typename C>
__device__ __forceinline__ C cconj(C a) { return mk(a.x, -a.y); }

// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C>
__device__ __forceinline__ C rot90(C a) {
  return INV ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft2(C* v) {
  C t = v[0];
  v[0] = cadd(t, v[1]);
  v[1] = csub(t, v[1]);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft4(C* v) {
  C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  C a2 = cadd(v[1], v[3]), a3 = rot90<INV>(csub(v[1], v[3]));
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft8(C* v) {
  using R = typename real_of<C>::type;
  const R h = (R)0.70710678118654752440;
  // split into even / odd halves, two 4-point DFTs, combine with w_8^k
  C e[4] = {v[0], v[2], v[4], v[6]};
  C o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // w_8^1 = (1 -+ i)/sqrt2, w_8^2 = -+i, w_8^3 = (-1 -+ i)/sqrt2
  C o1 = INV ? mk(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
             : mk(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
  C o2 = rot90<INV>(o[2]);
  C o3 = INV ? mk(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
             : mk(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft3(C* v) {
  using R = typename real_of<C>::type;
  const R c = (R)-0.5;
  const R s = INV ? (R)0.86602540378443864676 : (R)-0.86602540378443864676;
  C t1 = cadd(v[1], v[2]);
  C t2 = csub(v[1], v[2]);
  C m1 = mk(v[0].x + c * t1.x, v[0].y + c * t1.y);
  C m2 = mk(-s * t2.y, s * t2.x);  // i s t2
  v[0] = cadd(v[0], t1);
  v[1] = cadd(m1, m2);
  v[2] = csub(m1, m2);
}

template <int R, bool INV, typename C>
__device__ __forceinline__ void dftR(C* v) {
  if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else dft2<INV>(v);
}

// Stage plans (radix per stage, first to last; 1 = no stage).
//   Plan8: fewest stages (radix 8), for throughput-bound batches.
//   Plan4: radix 4 (+2 / 3), twice the threads per transform and half the
//          work per thread and stage: shorter latency for small batches.
template <int N> struct Plan8;
template <> struct Plan8<32>  { static constexpr int R[4] = {8, 4, 1, 1}; };
template <> struct Plan8<64>  { static constexpr int R[4] = {8, 8, 1, 1}; };
template <> struct Plan8<128> { static constexpr int R[4] = {8, 4, 4, 1}; };
template <> struct Plan8<192> { static constexpr int R[4] = {8, 8, 3, 1}; };
template <> struct Plan8<256> { static constexpr int R[4] = {8, 8, 4, 1}; };
template <int N> struct Plan4;
template <> struct Plan4<32>  { static constexpr int R[4] = {4, 4, 2, 1}; };
template <> struct Plan4<64>  { static constexpr int R[4] = {4, 4, 4, 1}; };
template <> struct Plan4<128> { static constexpr int R[4] = {4, 4, 4, 2}; };
template <> struct Plan4<192> { static constexpr int R[4] = {4, 4, 4, 3}; };
template <> struct Plan4<256> { static constexpr int R[4] = {4, 4, 4, 4}; };

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// orders global memory, which on gfx9 means waiting for every outstanding
// global load and store of the wave (one counter covers both); the FFT
// stages and the block reductions only exchange data through LDS, so with
// this barrier stores issued before a transform drain while it runs and
// loads issued for later use stay in flight.  Code that hands global memory
// from one wave to another must still use __syncthreads().
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Threads per workgroup: NT when the caller's kernel has a fixed size,
// else blockDim.x.  (blockDim.x is read from the implicit kernel arguments
// with a vector load and a wait on every outstanding load, each time a
// stage loop needs it; a compile-time size costs nothing.)
template <int NT>
__device__ __forceinline__ int wg_threads() {
  if constexpr (NT > 0) return NT;
  else return (int)blockDim.x;
}

// One Stockham stage over `nb` transforms of length N stored contiguously
// (transform t at src + t*N).  tw: N-th roots w_N^e = exp(-2 pi i e / N).
// Padded layout of the buffers between two stages (opt-in): element i of a
// transform sits at i + i / 16.  The first stage of a Stockham plan writes
// each thread's R outputs to R consecutive elements, so in the natural
// layout the 16 lanes an LDS access serves at once write 8R bytes apart and
// share a handful of banks (8-way for radix 8); one pad element every 16
// spreads them over distinct banks.  Inputs of the first stage and outputs
// of the last stay in the natural layout, so callers never see the padding.
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }
template <int N>
constexpr int padded_len() {
  return N + N / 16;
}

// PITCH: distance in elements between consecutive transforms (>= N, or >=
// padded_len<N>() with padded intermediates); PIN / POUT: the stage reads /
// writes the padded layout.
template <int N, int R, int NS, bool INV, int NT = 0, int PITCH = N, bool PIN = false, bool POUT = false,
          typename C>
__device__ __forceinline__ void stage(const C* __restrict__ src, C* __restrict__ dst, int nb,
                                      const C* __restrict__ tw) {
  static_assert(!(PIN || POUT) || PITCH >= padded_len<N>(), "padded layout needs a longer pitch");
  constexpr int Q = N / R;
  constexpr int TWS = N / (NS * R);
  const int total = nb * Q;
  for (int t = threadIdx.x; t < total; t += wg_threads<NT>()) {
    const int b = t / Q;
    const int j = t - b * Q;
    const C* s = src + b * PITCH;
    C* d = dst + b * PITCH;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[PIN ? pad16(j + r * Q) : j + r * Q];
    if constexpr (NS > 1) {
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = tw[r * k * TWS];  // r*k*TWS < N
        if constexpr (INV) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    dftR<R, INV>(v);
    const int o = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) d[POUT ? pad16(o + r * NS) : o + r * NS] = v[r];
  }
}

// Full N-point transforms of `nb` contiguous rows in LDS buffer `a`, using
// `b` as the ping-pong partner.  Returns the buffer holding the result.
// Callers must synchronise before (data ready in LDS); the result is ready
// on return (an LDS barrier ends every stage).  NT: the kernel's fixed workgroup
// size (0: read blockDim.x); PITCH: transform b starts at element b * PITCH;
// PAD: padded layout between stages (PITCH >= padded_len<N>()).
template <int N, bool INV, bool R4 = true, int NT = 0, int PITCH = N, bool PAD = false, typename C>
__device__ C* fft_lds(C* a, C* b, int nb, const C* __restrict__ tw) {
  using P = typename std::conditional<R4, Plan4<N>, Plan8<N>>::type;
  constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2], R3 = P::R[3];
  stage<N, R0, 1, INV, NT, PITCH, false, PAD>(a, b, nb, tw);
  lds_barrier();
  stage<N, R1, R0, INV, NT, PITCH, PAD, PAD && (R2 > 1)>(b, a, nb, tw);
  lds_barrier();
  if constexpr (R2 == 1) return a;
  stage<N, R2, R0 * R1, INV, NT, PITCH, PAD, PAD && (R3 > 1)>(a, b, nb, tw);
  lds_barrier();
  if constexpr (R3 == 1) return b;
  stage<N, R3, R0 * R1 * R2, INV, NT, PITCH, PAD, false>(b, a, nb, tw);
  lds_barrier();
  return a;
}

// fft_lds whose last stage hands its outputs to `store(t, k, v)` (element k
// of transform t) instead of writing them to LDS: the caller's global
// stores leave from registers, without the last LDS round trip and barrier.
template <int N, bool INV, bool R4 = true, int NT = 0, int PITCH = N, bool PAD = false, typename C, typename S>
__device__ void fft_lds_store(C* a, C* b, int nb, const C* __restrict__ tw, S store) {
  using P = typename std::conditional<R4, Plan4<N>, Plan8<N>>::type;
  constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2], R3 = P::R[3];
  constexpr int NS = R3 > 1 ? R0 * R1 * R2 : R2 > 1 ? R0 * R1 : R0;  // span before the last stage
  constexpr int RL = R3 > 1 ? R3 : R2 > 1 ? R2 : R1;                // last radix
  static_assert(NS * RL == N, "plan covers N");
  const C* src;
  stage<N, R0, 1, INV, NT, PITCH, false, PAD>(a, b, nb, tw);
  lds_barrier();
  if constexpr (R2 == 1) {
    src = b;
  } else {
    stage<N, R1, R0, INV, NT, PITCH, PAD, PAD>(b, a, nb, tw);
    lds_barrier();
    if constexpr (R3 == 1) {
      src = a;
    } else {
      stage<N, R2, R0 * R1, INV, NT, PITCH, PAD, PAD>(a, b, nb, tw);
      lds_barrier();
      src = b;
    }
  }
  // last stage: butterfly j < NS of transform t reads j + NS r, writes the
  // natural-order outputs j + NS r
  constexpr int TWS = 1;  // N / (NS * RL)
  const int total = nb * NS;
  for (int q = threadIdx.x; q < total; q += wg_threads<NT>()) {
    const int t = q / NS, j = q - t * NS;
    const C* sp = src + t * PITCH;
    C v[RL];
#pragma unroll
    for (int r = 0; r < RL; ++r) v[r] = sp[PAD ? pad16(j + r * NS) : j + r * NS];
#pragma unroll
    for (int r = 1; r < RL; ++r) {
      C w = tw[r * j * TWS];
      if constexpr (INV) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    dftR<RL, INV>(v);
#pragma unroll
    for (int r = 0; r < RL; ++r) store(t, j + r * NS, v[r]);
  }
}

// In-place variant: every thread first reads the inputs of all of its
// butterflies into registers, the workgroup synchronises, then every thread
// writes its outputs over the same buffer — one buffer instead of two, at
// the price of a second barrier per stage.  MAXB bounds the butterflies per
// thread (nb * N / R / blockDim.x, rounded up).
template <int N, int R, int NS, bool INV, int MAXB, int NT = 0, int PITCH = N, bool PIN = false, bool POUT = false,
          typename C>
__device__ __forceinline__ void stage_inplace(C* buf, int nb, const C* __restrict__ tw) {
  static_assert(!(PIN || POUT) || PITCH >= padded_len<N>(), "padded layout needs a longer pitch");
  constexpr int Q = N / R;
  constexpr int TWS = N / (NS * R);
  const int total = nb * Q;
  C v[MAXB][R];
  int bs[MAXB], jj[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int t = threadIdx.x + i * wg_threads<NT>();
    bs[i] = 0;
    jj[i] = 0;
    if (t < total) {
      const int b = t / Q, j = t - b * Q;
      bs[i] = b * PITCH;
      jj[i] = j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[b * PITCH + (PIN ? pad16(j + r * Q) : j + r * Q)];
    }
  }
  lds_barrier();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int t = threadIdx.x + i * wg_threads<NT>();
    if (t < total) {
      const int j = jj[i];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C w = tw[r * k * TWS];
          if constexpr (INV) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      dftR<R, INV>(v[i]);
      const int o = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[bs[i] + (POUT ? pad16(o + r * NS) : o + r * NS)] = v[i][r];
    }
  }
  lds_barrier();
}

// fft_lds_inplace whose last stage hands its outputs to `store(t, k, v)`
// (see fft_lds_store); the last stage only reads the buffer.
template <int N, bool INV, bool R4, int MAXNB, int MINT, int NT = 0, int PITCH = N, bool PAD = false, typename C,
          typename S>
__device__ void fft_lds_inplace_store(C* buf, int nb, const C* __restrict__ tw, S store) {
  using P = typename std::conditional<R4, Plan4<N>, Plan8<N>>::type;
  constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2], R3 = P::R[3];
  constexpr int NS = R3 > 1 ? R0 * R1 * R2 : R2 > 1 ? R0 * R1 : R0;
  constexpr int RL = R3 > 1 ? R3 : R2 > 1 ? R2 : R1;
  static_assert(NS * RL == N, "plan covers N");
  stage_inplace<N, R0, 1, INV, (MAXNB * (N / R0) + MINT - 1) / MINT, NT, PITCH, false, PAD>(buf, nb, tw);
  if constexpr (R2 > 1)
    stage_inplace<N, R1, R0, INV, (MAXNB * (N / R1) + MINT - 1) / MINT, NT, PITCH, PAD, PAD>(buf, nb, tw);
  if constexpr (R3 > 1)
    stage_inplace<N, R2, R0 * R1, INV, (MAXNB * (N / R2) + MINT - 1) / MINT, NT, PITCH, PAD, PAD>(buf, nb, tw);
  const int total = nb * NS;
  for (int q = threadIdx.x; q < total; q += wg_threads<NT>()) {
    const int t = q / NS, j = q - t * NS;
    const C* sp = buf + t * PITCH;
    C v[RL];
#pragma unroll
    for (int r = 0; r < RL; ++r) v[r] = sp[PAD ? pad16(j + r * NS) : j + r * NS];
#pragma unroll
    for (int r = 1; r < RL; ++r) {
      C w = tw[r * j];
      if constexpr (INV) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    dftR<RL, INV>(v);
#pragma unroll
    for (int r = 0; r < RL; ++r) store(t, j + r * NS, v[r]);
  }
}

// Full in-place transforms of `nb` (<= MAXNB) contiguous rows of `buf`
// with at least `MINT` threads per workgroup (exactly NT when NT > 0).
// Same contract as fft_lds; the result is in `buf`.
template <int N, bool INV, bool R4, int MAXNB, int MINT, int NT = 0, int PITCH = N, bool PAD = false, typename C>
__device__ void fft_lds_inplace(C* buf, int nb, const C* __restrict__ tw) {
  using P = typename std::conditional<R4, Plan4<N>, Plan8<N>>::type;
  constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2], R3 = P::R[3];
  stage_inplace<N, R0, 1, INV, (MAXNB * (N / R0) + MINT - 1) / MINT, NT, PITCH, false, PAD>(buf, nb, tw);
  stage_inplace<N, R1, R0, INV, (MAXNB * (N / R1) + MINT - 1) / MINT, NT, PITCH, PAD, PAD && (R2 > 1)>(buf, nb, tw);
  if constexpr (R2 > 1)
    stage_inplace<N, R2, R0 * R1, INV, (MAXNB * (N / R2) + MINT - 1) / MINT, NT, PITCH, PAD, PAD && (R3 > 1)>(
        buf, nb, tw);
  if constexpr (R3 > 1)
    stage_inplace<N, R3, R0 * R1 * R2, INV, (MAXNB * (N / R3) + MINT - 1) / MINT, NT, PITCH, PAD, false>(buf, nb, tw);
}

// LDS pitch (complex float elements) of the transforms of a column pass that
// holds CW adjacent detector columns: its global-to-LDS transposes put
// consecutive lanes on consecutive columns, so with a pitch of N (a multiple
// of 32 elements) the CW lanes of one row hit the same LDS banks; 16 / CW
// extra elements move each column's transform to other banks, so the 16 lanes
// an LDS access serves at once touch 16 distinct bank pairs.
// With padded intermediates (PAD) the pitch starts from padded_len<N>()
// rounded up to 16 elements.
template <int N, int CW, bool PAD = false>
constexpr int col_pitch() {
  constexpr int base = PAD ? (padded_len<N>() + 15) / 16 * 16 : N;
  return CW > 1 ? base + 16 / CW : base;
}

}  // namespace mrpie
