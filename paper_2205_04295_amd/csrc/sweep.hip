// The sequential M-rPIE sweep on gfx950 (Methods, "M-rPIE algorithm",
// Eq. 4-7).
//
// A position step is split at the two transposes of the 2-D FFT into two
// launches; kernel boundaries are the device-wide sync points (on MI355X a
// graph-replayed launch costs less than a cross-XCD grid barrier):
//
//   k_cols  (step s):   one workgroup per detector column, all modes:
//                       forward column FFT, mode-summed modulus replacement
//                       (Eq. 7), inverse column FFT, in place in psi[s&1];
//                       accumulates the Fourier error.
//   k_rows  (s-1 -> s): one workgroup per probe row r: inverse row FFTs of
//                       psi[(s-1)&1]; probe update of row r (Eq. 5); object
//                       update (Eq. 6) of the box rows that are rows of the
//                       next box or leave it; gather of row r of the next
//                       box, exit waves P_p o (Eq. 1/4) and forward row FFTs
//                       into psi[s&1].
//
// Probe, patch and spectra are double-buffered by step parity, so inside a
// k_rows launch every buffer a workgroup reads is disjoint from every buffer
// any workgroup writes; the object rows a workgroup writes are exactly the
// rows it then re-gathers (merged from LDS).  The sweep has no atomics on
// data and is bitwise deterministic.  The object update of step s-1 and the
// gather of step s are one launch, which keeps rPIE's order: position s
// reads the object after position s-1 has written it.
//
// Batching: blockIdx.y selects a job from the launch's job table; every job
// advances one position per tick (lock-step), so many independent
// reconstructions of different N, M, J fill the GPU that one sweep cannot.
// A job table holds at most 36 jobs: more jobs queue in launch lanes, each
// starting at a later tick (its own step is the tick minus its start).
// Batches of 16 or more jobs (by default) split the row work into two
// launches, k_upd (the update of step s-1) and k_gat (the gather of step
// s), which read every row of the spectra once and keep no patch copy (see
// the split passes below).  Every global load a workgroup needs is issued at
// kernel start, before the first LDS stage, so each launch pays one memory
// latency; the LDS barriers of the transforms leave global stores draining.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "register.hpp"
#include "sweep.hpp"

namespace mrpie {

// select one of a pair without dynamic indexing (keeps the layout in SGPRs)
__device__ __forceinline__ size_t pick(const size_t (&a)[2], int i) { return i ? a[1] : a[0]; }

// IP: the inverse row FFTs run in place (one 3MN buffer instead of two:
// more workgroups per CU, one more barrier per stage) — for batches.
// SINGLE: the single-job launch.  Batches use the padded layout between FFT
// stages (fewer LDS bank conflicts; a single job's latency chain would only
// see its extra index arithmetic), and only a single job touches the next
// pattern row early (a prefetch for its latency-bound column pass; in a
// batch, which is bound by memory traffic, it would be a second read).
// Index of spectra element (row k, column c) in a buffer the single-job
// passes exchange: row-major, or (TILE) in column groups of eight,
// ((c / 8) N + k) 8 + c % 8, so a row is written in 64-byte segments and a
// column read touches half the cache lines it would in row-major order.  The
// row pass writes its row transforms tiled and the column pass reads them
// tiled (column pass 6.1 -> 5.6 us, row pass 8.5 -> 8.8 us at 256^2 x 3);
// the column pass writes its results row-major, which the next row pass
// reads in whole lines (tiled reads there cost more than they saved).
constexpr int kTileCols = 8;
template <int N, bool TILE>
__device__ __forceinline__ size_t sidx(int k, int c) {
  if constexpr (TILE) return ((size_t)(c / kTileCols) * N + k) * kTileCols + (c % kTileCols);
  else return (size_t)k * N + c;
}

template <int N, bool R4, int MM, bool IP = false, bool SINGLE = false>
__device__ __forceinline__ void rows_body(const Common& cm, const JobRec& jb, int t, float2* smem) {
  const int M = jb.M;
  const int total = jb.J * jb.T;
  const int r = blockIdx.x;
  if (t < 0 || t > total || r >= N) return;
  const bool has_prev = t > 0, has_next = t < total;
  const int cur = t & 1, prv = (t + 1) & 1;
  const int jn = has_next ? t % jb.J : 0;
  const WsLayout L = ws_layout(N, M, jb.T);
  char* ws = jb.ws;
  const size_t NN = (size_t)N * N;
  const int tid = threadIdx.x;
  const bool lane = tid < N;  // this thread owns column `tid`

  constexpr bool PAD = !SINGLE;
  constexpr int PT = col_pitch<N, 1, PAD>();  // LDS pitch of a transform
  float2* tw = smem;               // N
  float2* orow = tw + N;           // N   updated object row (box-prev row rb1)
  float2* bufA = orow + N;         // 2*M*PT
  float2* bufB = IP ? bufA + M * PT : bufA + 2 * M * PT;  // forward-FFT partner (IP: inside bufA)
  __shared__ float redf[32];

  const float2* psi_prev = (const float2*)(ws + pick(L.psi, prv));
  const float2* patch_prev = (const float2*)(ws + pick(L.patch, prv));
  const float2* Pold = prv == 0 ? jb.probe : (const float2*)(ws + L.probe1);
  float2* Pnew = cur == 0 ? jb.probe : (float2*)(ws + L.probe1);

  // ---- issue every global load up front.  The probe row r (slot 0), its
  //      patch row and spectra and the max partials do not depend on the box
  //      geometry, so they are issued before the positions are even read;
  //      the rows that depend on the boxes follow.
  float2 pv[2][MM];      // psi_prev rows (row-transformed spectra)
  float2 Pq[2][MM];      // old probe at the slot rows
  float2 oq[2];          // old patch at the slot rows
  float2 og = make_float2(0.f, 0.f);  // object value of the next box row, outside the updated row
  float2 Ph[MM];         // probe row r when there is no previous step
  float om_in = 0.f, pm_in = 0.f, i_touch = 0.f;
  const int c = tid;
  if (lane) {
    const size_t off = (size_t)r * N + c;
    if (has_prev) {
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) {
          pv[0][p] = psi_prev[p * NN + sidx<N, false>(r, c)];
          Pq[0][p] = Pold[p * NN + off];
        }
      oq[0] = patch_prev[off];
      om_in = ((const float*)(ws + pick(L.omax, prv)))[c];
      pm_in = ((const float*)(ws + pick(L.pmax, prv)))[c];
    } else {
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) Ph[p] = Pnew[p * NN + off];
    }
    // touch row r of this step's pattern so the column pass that follows
    // finds it in the memory-side cache instead of HBM
    if (SINGLE && has_next) i_touch = jb.I[(size_t)jn * NN + off];
  }

  // ---- box geometry
  int ny_n = 0, nx_n = 0;
  if (has_next) {
    ny_n = box_corner(jb.pos[2 * jn], jb.H - N, jb.status);
    nx_n = box_corner(jb.pos[2 * jn + 1], jb.W - N, jb.status);
  }
  int ny_p = 0, nx_p = 0, rb1 = -1, rb2 = -1;
  if (has_prev) {
    // the previous box, recomputed from the (read-only) positions: no wait
    // for a value another XCD wrote one launch earlier (its clamp bit was
    // set when it was gathered)
    const int jp = (t - 1) % jb.J;
    ny_p = box_corner(jb.pos[2 * jp], jb.H - N, nullptr);
    nx_p = box_corner(jb.pos[2 * jp + 1], jb.W - N, nullptr);
    if (has_next) {
      const int dy = ny_n - ny_p;
      if (r + dy >= 0 && r + dy < N) rb1 = r + dy;
      if (dy > 0 && r < min(N, dy)) rb2 = r;
      if (dy < 0 && r < min(N, -dy)) rb2 = max(0, N + dy) + r;
    } else {
      rb1 = r;
    }
  }
  // distinct box rows needing an inverse row FFT: slot 0 is the probe row r,
  // slot 1 the box row that moves into the next box (rb1, when dy != 0 and
  // r + dy is inside) or the one that leaves it (rb2, dy < 0 and r < -dy;
  // for dy > 0 the leaving row is r itself).  The two cases exclude each
  // other, so at most two rows are transformed.
  const bool u1 = rb1 >= 0 && rb1 != r, u2 = rb2 >= 0 && rb2 != r;
  const int rows[2] = {r, u1 ? rb1 : rb2};
  const int ns = has_prev ? 1 + (int)(u1 || u2) : 0;
  if (lane) {
#pragma unroll
    for (int q = 1; q < 2; ++q) {
      if (q >= ns) break;
      const size_t off = (size_t)rows[q] * N + c;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) {
          pv[q][p] = psi_prev[p * NN + sidx<N, false>(rows[q], c)];
          Pq[q][p] = Pold[p * NN + off];
        }
      oq[q] = patch_prev[off];
    }
    if (has_next) {
      const int gx = nx_n + c;
      const bool merged = rb1 >= 0 && gx >= nx_p && gx < nx_p + N;
      if (!merged) og = jb.obj[(size_t)(ny_n + r) * jb.W + gx];
    }
  }
  load_twiddles<N>(tw);

  float2 Pn[MM];
  bool bad = false;
  float pm_row = 0.f;  // sum_p |P_p|^2 of the new probe at (r, c)
  if (has_prev) {
    if (lane) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (q >= ns) break;
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) bufA[(q * M + p) * PT + c] = pv[q][p];
      }
    }
    float omax, pmaxv;
    block_max2(om_in, pm_in, redf, omax, pmaxv);  // (contains the barrier before the FFT)
    float2* res;
    if constexpr (IP) {
      fft_lds_inplace<N, true, R4, 2 * MM, 256, 0, PT, PAD>(bufA, ns * M, tw);
      res = bufA;
    } else {
      res = fft_lds<N, true, R4, 0, PT, PAD>(bufA, bufB, ns * M, tw);
    }

    // ---- probe update of row r (Eq. 5) from the pre-update o and P
    const int it_abs = cm.iter_offset + (t - 1) / jb.J;
    const bool upd_p = it_abs >= cm.probe_update_start;
    if (lane) {
      const float2 o = oq[0];
      const float o2 = cabs2(o);
      const float dP = cm.beta * omax + (1.f - cm.beta) * o2;
      const float g = (upd_p && dP != 0.f) ? cm.alpha_probe / dP : 0.f;
      float ps = 0.f;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) {
          const float2 P = Pq[0][p];
          const float2 d = csub(res[p * PT + c], cmul(P, o));
          Pn[p] = cadd(P, cscale(cmulc(d, o), g));
          Pnew[p * NN + (size_t)r * N + c] = Pn[p];
          ps += cabs2(Pn[p]);
        }
      bad |= !isfinite(ps);
    }

    // ---- object update (Eq. 6) of box rows rb1 / rb2: slot 0 when one of
    //      them is the probe row r, slots 1.. otherwise
    if (lane) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const bool is_obj = q == 0 ? (rb1 == r || rb2 == r) : (q < ns);
        if (!is_obj) continue;
        const int rb = rows[q];
        const float2 o = oq[q];
        float Ps = 0.f;
        float2 num = make_float2(0.f, 0.f);
#pragma unroll
        for (int p = 0; p < MM; ++p)
          if (p < M) {
            const float2 P = Pq[q][p];
            const float2 d = csub(res[(q * M + p) * PT + c], cmul(P, o));
            num = cadd(num, cmulc(d, P));
            Ps += cabs2(P);
          }
        const float dO = cm.gamma * pmaxv + (1.f - cm.gamma) * Ps;
        const float g = dO != 0.f ? cm.alpha_obj / dO : 0.f;
        const float2 on = cadd(o, cscale(num, g));
        bad |= !(isfinite(on.x) && isfinite(on.y));
        jb.obj[(size_t)(ny_p + rb) * jb.W + nx_p + c] = on;
        if (rb == rb1) orow[c] = on;
      }
    }
    if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
    lds_barrier();  // publishes orow; the probe and object stores drain meanwhile
  } else {
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) Pn[p] = Ph[p];
  }

  if (!has_next) return;

  // ---- gather row r of the next box (merging the row just updated),
  //      exit waves and forward row FFTs
  float om = 0.f;
  if (lane) {
    const int gx = nx_n + c;
    const float2 o = (rb1 >= 0 && gx >= nx_p && gx < nx_p + N) ? orow[gx - nx_p] : og;
    ((float2*)(ws + pick(L.patch, cur)))[(size_t)r * N + c] = o;
    om = cabs2(o);
    float ps = 0.f;
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        ps += cabs2(Pn[p]);
        bufA[p * PT + c] = cmul(Pn[p], o);
      }
    pm_row = ps;
  }
  float pm;
  block_max2(om, pm_row, redf, om, pm);  // (its barriers also publish bufA)
  if (tid == 0) {
    ((float*)(ws + pick(L.omax, cur)))[r] = om;
    ((float*)(ws + pick(L.pmax, cur)))[r] = pm;
  }
  float2* dst = (float2*)(ws + pick(L.psi, cur));
  fft_lds_store<N, false, R4, 0, PT, PAD>(bufA, bufB, M, tw, [&](int p, int cc, float2 v) {
    dst[p * NN + sidx<N, SINGLE>(r, cc)] = v;
  });
  if (SINGLE && i_touch < -3.0e38f) flag_status(jb.status, 0);  // keeps the touch load
}

// Split row passes for batches (three launches per position: update rows,
// gather rows, columns).  The fused row pass above needs, in each workgroup,
// the inverse transforms of two rows of the previous spectra whenever the
// box moves vertically: probe row r (for the exit waves of next-box row r)
// and box row r + dy (the object row that becomes next-box row r).  With the
// update and the gather in launches of their own, every previous-box row is
// inverse-transformed exactly once and the pre-update patch is read straight
// from the object (the update is the only writer of its row), so a position
// moves (4M + 2.5) N^2 x 8 B read and (3M + 1) N^2 x 8 B written instead of
// about (5M + 3.5) and (3M + 2): less traffic for batches, which are bound by
// memory traffic; one more launch, which only a single sweep's latency
// chain would feel.  The probe is updated in place (each row by the one
// workgroup that owns it), so no copy-back is needed at the end.

// Each split pass of mode capacity MM <= 4 takes two consecutive rows per
// workgroup, so every FFT call transforms 2M rows at once (one 256-point row
// of M modes keeps only 32 M of 256 threads busy in a radix-8 stage); with
// MM = 8 the doubled register arrays would cost more occupancy than that
// gains, so it keeps one.
__host__ __device__ constexpr int split_rows(int mm) { return mm <= 4 ? 2 : 1; }

// Update of step t-1 (Eq. 5, Eq. 6) for previous-box rows q0 = split_rows(MM)
// blockIdx.x, q0 + 1, ...: inverse row FFTs of their spectra, probe rows and
// object rows from the pre-update o and P.
template <int N, bool R4, int MM, bool IP>
__device__ __forceinline__ void upd_body(const Common& cm, const JobRec& jb, int t, float2* smem) {
  constexpr int RP = split_rows(MM);
  const int M = jb.M;
  const int total = jb.J * jb.T;
  const int q0 = blockIdx.x * RP;
  if (t < 1 || t > total || q0 >= N) return;
  const int st = t - 1, prv = st & 1;
  const WsLayout L = ws_layout(N, M, jb.T);
  const size_t NN = (size_t)N * N;
  const int tid = threadIdx.x, c = tid;
  const bool lane = tid < N;
  constexpr int PT = col_pitch<N, 1, true>();  // LDS pitch of a transform (padded intermediates)
  float2* tw = smem;
  float2* bufA = tw + N;              // transform (s, p) at (s M + p) PT
  float2* bufB = bufA + RP * M * PT;  // ping-pong partner (not used in place)
  __shared__ float redf[32];

  const float2* psi = (const float2*)(jb.ws + pick(L.psi, prv));
  const int jp = st % jb.J;
  const int ny = box_corner(jb.pos[2 * jp], jb.H - N, nullptr);  // flagged by its gather
  const int nx = box_corner(jb.pos[2 * jp + 1], jb.W - N, nullptr);
  float2 pv[RP][MM], Pq[RP][MM], o[RP];
  float om_in = 0.f, pm_in = 0.f;
  if (lane) {
#pragma unroll
    for (int s = 0; s < RP; ++s) {
      const int q = q0 + s;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) {
          pv[s][p] = psi[p * NN + (size_t)q * N + c];
          Pq[s][p] = jb.probe[p * NN + (size_t)q * N + c];
        }
      o[s] = jb.obj[(size_t)(ny + q) * jb.W + nx + c];
    }
    om_in = ((const float*)(jb.ws + pick(L.omax, prv)))[c];
    pm_in = ((const float*)(jb.ws + pick(L.pmax, prv)))[c];
  }
  load_twiddles<N>(tw);
  if (lane) {
#pragma unroll
    for (int s = 0; s < RP; ++s)
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) bufA[(s * M + p) * PT + c] = pv[s][p];
  }
  float omax, pmaxv;
  block_max2(om_in, pm_in, redf, omax, pmaxv);  // (contains the barrier before the FFT)
  float2* res;
  if constexpr (IP) {
    fft_lds_inplace<N, true, R4, RP * MM, 256, 0, PT, true>(bufA, RP * M, tw);
    res = bufA;
  } else {
    res = fft_lds<N, true, R4, 0, PT, true>(bufA, bufB, RP * M, tw);
  }
  const int it_abs = cm.iter_offset + st / jb.J;
  const bool upd_p = it_abs >= cm.probe_update_start;
  bool bad = false;
  if (lane) {
#pragma unroll
    for (int s = 0; s < RP; ++s) {
      const int q = q0 + s;
      const float o2 = cabs2(o[s]);
      const float dP = cm.beta * omax + (1.f - cm.beta) * o2;
      const float gP = (upd_p && dP != 0.f) ? cm.alpha_probe / dP : 0.f;
      float ps = 0.f, Ps = 0.f;
      float2 num = make_float2(0.f, 0.f);
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) {
          const float2 P = Pq[s][p];
          const float2 d = csub(res[(s * M + p) * PT + c], cmul(P, o[s]));
          const float2 Pn = cadd(P, cscale(cmulc(d, o[s]), gP));
          jb.probe[p * NN + (size_t)q * N + c] = Pn;
          ps += cabs2(Pn);
          num = cadd(num, cmulc(d, P));
          Ps += cabs2(P);
        }
      bad |= !isfinite(ps);
      const float dO = cm.gamma * pmaxv + (1.f - cm.gamma) * Ps;
      const float gO = dO != 0.f ? cm.alpha_obj / dO : 0.f;
      const float2 on = cadd(o[s], cscale(num, gO));
      bad |= !(isfinite(on.x) && isfinite(on.y));
      jb.obj[(size_t)(ny + q) * jb.W + nx + c] = on;
    }
  }
  if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
}

// Gather of step t for box rows r0 = split_rows(MM) blockIdx.x, r0 + 1, ...: the
// object rows (already updated by step t-1), exit waves with the updated
// probe rows (Eq. 1, 4), the row maxima the next update needs, forward row
// FFTs into the spectra.
template <int N, bool R4, int MM, bool IP>
__device__ __forceinline__ void gat_body(const JobRec& jb, int t, float2* smem) {
  constexpr int RP = split_rows(MM);
  const int M = jb.M;
  const int total = jb.J * jb.T;
  const int r0 = blockIdx.x * RP;
  if (t < 0 || t >= total || r0 >= N) return;
  const int cur = t & 1, jn = t % jb.J;
  const WsLayout L = ws_layout(N, M, jb.T);
  const size_t NN = (size_t)N * N;
  const int tid = threadIdx.x, c = tid;
  const bool lane = tid < N;
  constexpr int PT = col_pitch<N, 1, true>();  // LDS pitch of a transform (padded intermediates)
  float2* tw = smem;
  float2* bufA = tw + N;              // transform (s, p) at (s M + p) PT
  float2* bufB = bufA + RP * M * PT;
  __shared__ float redf[64];

  const int ny = box_corner(jb.pos[2 * jn], jb.H - N, jb.status);
  const int nx = box_corner(jb.pos[2 * jn + 1], jb.W - N, jb.status);
  float2 o[RP], Pn[RP][MM];
  if (lane) {
#pragma unroll
    for (int s = 0; s < RP; ++s) {
      o[s] = jb.obj[(size_t)(ny + r0 + s) * jb.W + nx + c];
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) Pn[s][p] = jb.probe[p * NN + (size_t)(r0 + s) * N + c];
    }
  }
  load_twiddles<N>(tw);
  float om[RP] = {}, pm_row[RP] = {};
  if (lane) {
#pragma unroll
    for (int s = 0; s < RP; ++s) {
      om[s] = cabs2(o[s]);
      float ps = 0.f;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) {
          ps += cabs2(Pn[s][p]);
          bufA[(s * M + p) * PT + c] = cmul(Pn[s][p], o[s]);
        }
      pm_row[s] = ps;
    }
  }
  float omr[RP], pmr[RP];
#pragma unroll
  for (int s = 0; s < RP; ++s)  // (the first reduction's barriers also publish bufA)
    block_max2(om[s], pm_row[s], redf + 32 * s, omr[s], pmr[s]);
  if (tid == 0) {
#pragma unroll
    for (int s = 0; s < RP; ++s) {
      ((float*)(jb.ws + pick(L.omax, cur)))[r0 + s] = omr[s];
      ((float*)(jb.ws + pick(L.pmax, cur)))[r0 + s] = pmr[s];
    }
  }
  float2* dst = (float2*)(jb.ws + pick(L.psi, cur));
  auto store = [&](int sp, int cc, float2 v) {  // transform sp = s M + p
    const int s = sp / M, p = sp - s * M;
    dst[p * NN + (size_t)(r0 + s) * N + cc] = v;
  };
  if constexpr (IP) fft_lds_inplace_store<N, false, R4, RP * MM, 256, 0, PT, true>(bufA, RP * M, tw, store);
  else fft_lds_store<N, false, R4, 0, PT, true>(bufA, bufB, RP * M, tw, store);
}

// Column pass of step t: CW adjacent detector columns per workgroup (all
// modes), so that every global access of the pass moves CW * 8 contiguous
// bytes of a row (CW = 1: a single column, the shortest latency; CW = 4:
// a quarter of the cache-line traffic, for batches that fill the GPU).
// IP: the column FFTs run in place (one buffer: more workgroups per CU in
// batches).
template <int N, bool R4, int MM, int CW, bool IP = false, bool TILE = false>
__device__ __forceinline__ void cols_body(const JobRec& jb, int t, float2* smem) {
  const int M = jb.M;
  const int total = jb.J * jb.T;
  if (t < 0 || t >= total) return;
  const int u = xcd_unit(blockIdx.x, gridDim.x);  // column group of this workgroup
  if (u >= N / CW) return;
  const int u0 = u * CW;
  const int it = t / jb.J, jn = t - it * jb.J;
  const WsLayout L = ws_layout(N, M, jb.T);
  const size_t NN = (size_t)N * N;
  float2* psi = (float2*)(jb.ws + pick(L.psi, t & 1));
  const float* Ij = jb.I + (size_t)jn * NN;
  constexpr int NT = 256;               // threads
  constexpr int PIX = (N * CW + NT - 1) / NT;  // detector pixels per thread
  const int tid = threadIdx.x;

  constexpr bool PAD = true;             // padded layout between FFT stages
  constexpr int PT = col_pitch<N, CW, PAD>();  // LDS pitch of a transform
  float2* tw = smem;
  float2* bufA = tw + N;                // transform (p, c) at (p * CW + c) * PT
  float2* bufB = IP ? bufA : bufA + M * CW * PT;
  // per-wave partials of the Fourier error and of the intensity sum that
  // normalises it (kErrSlots / 256 waves per unit)
  const size_t slot = (size_t)it * kErrSlots + u * (NT / 64) + (tid >> 6);
  double* err_slot = (double*)(jb.ws + L.err) + slot;
  double* isum_slot = (double*)(jb.ws + L.isum) + slot;
  const double err_old = (tid & 63) == 0 ? *err_slot : 0.0;
  const double isum_old = (tid & 63) == 0 ? *isum_slot : 0.0;
  // pixel q = tid + NT * i of the group: row k = q / CW, column c = q % CW
  // (consecutive threads read consecutive columns of a row)
  float Iv[PIX];
  float2 v[PIX][MM];
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + NT * i;
    if (q < N * CW) {
      const int k = q / CW, c = q - k * CW;
      const size_t off = (size_t)k * N + u0 + c;
      Iv[i] = Ij[off];
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) v[i][p] = psi[p * NN + sidx<N, TILE>(k, u0 + c)];
    }
  }
  load_twiddles<N, 256>(tw);
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + NT * i;
    if (q < N * CW) {
      const int k = q / CW, c = q - k * CW;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) bufA[(p * CW + c) * PT + k] = v[i][p];
    }
  }
  __syncthreads();
  float2* F;
  if constexpr (IP) {
    fft_lds_inplace<N, false, R4, MM * CW, 256, 256, PT, PAD>(bufA, M * CW, tw);
    F = bufA;
  } else {
    F = fft_lds<N, false, R4, 256, PT, PAD>(bufA, bufB, M * CW, tw);
  }
  float2* G = IP ? F : ((F == bufA) ? bufB : bufA);
  // Eq. 7: the 2-D transform here is unnormalised (N x unitary) and so is
  // the inverse, so the scale factor carries one 1/N.
  const float invN = 1.0f / (float)N;
  double e = 0.0, isv = 0.0;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + NT * i;
    if (q < N * CW) {
      const int k = q / CW, c = q - k * CW;
      isv += (double)fmaxf(Iv[i], 0.f);
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
      bad |= !isfinite(S);
      const float f = sq * rs * invN;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) G[(p * CW + c) * PT + k] = cscale(F[(p * CW + c) * PT + k], f);
    }
  }
  if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
  __syncthreads();
  float2* H;
  if constexpr (IP) {
    fft_lds_inplace<N, true, R4, MM * CW, 256, 256, PT, PAD>(G, M * CW, tw);
    H = G;
  } else {
    H = fft_lds<N, true, R4, 256, PT, PAD>(G, F, M * CW, tw);
  }
#pragma unroll
  for (int i = 0; i < PIX; ++i) {
    const int q = tid + NT * i;
    if (q < N * CW) {
      const int k = q / CW, c = q - k * CW;
      const size_t off = (size_t)k * N + u0 + c;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) psi[p * NN + sidx<N, false>(k, u0 + c)] = H[(p * CW + c) * PT + k];
    }
  }
  e = wave_sum(e);
  isv = wave_sum(isv);
  if ((tid & 63) == 0) {
    *err_slot = err_old + e;
    *isum_slot = isum_old + isv;
  }
}

// Column pass of one column with the first and last FFT stages in
// registers (radix-8 plans, N >= 128, one column per workgroup): the
// forward transform's first stage takes the global loads directly, its
// last stage leaves each thread j < N/RL every mode at the frequencies
// j + (N/RL) r, so the mode-summed modulus (Eq. 7) and the first inverse
// stage need no LDS round trip, and the inverse transform's last stage
// stores straight to global memory: four barriers instead of eight.
template <int N, int MM, bool TILE = false>
__device__ __forceinline__ void cols_body_rd(const JobRec& jb, int t, float2* smem) {
  using P = Plan8<N>;
  constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2];
  static_assert(R2 > 1 && P::R[3] == 1, "three-stage plans only");
  constexpr int RL = R2;           // last forward radix = first inverse radix
  constexpr int Q0 = N / R0;       // butterflies per transform of the first stage
  constexpr int QL = N / RL;       // threads of the mode-sum stage
  const int M = jb.M;
  const int total = jb.J * jb.T;
  if (t < 0 || t >= total) return;
  const int u = xcd_unit(blockIdx.x, gridDim.x);
  if (u >= N) return;
  const int it = t / jb.J, jn = t - it * jb.J;
  const WsLayout L = ws_layout(N, M, jb.T);
  const size_t NN = (size_t)N * N;
  float2* psi = (float2*)(jb.ws + pick(L.psi, t & 1));
  const float* Ij = jb.I + (size_t)jn * NN;
  const int tid = threadIdx.x;

  float2* tw = smem;
  float2* bufA = tw + N;           // M N
  float2* bufB = bufA + M * N;     // M N

  const size_t slot = (size_t)it * kErrSlots + u * 4 + (tid >> 6);
  double* err_slot = (double*)(jb.ws + L.err) + slot;
  double* isum_slot = (double*)(jb.ws + L.isum) + slot;
  const double err_old = (tid & 63) == 0 ? *err_slot : 0.0;
  const double isum_old = (tid & 63) == 0 ? *isum_slot : 0.0;

  // first-stage inputs (thread (p, j): rows j + Q0 r of mode p) and the
  // patterns of the mode-sum threads
  const bool s0 = tid < M * Q0;
  const int p0 = tid / Q0, j0 = tid - p0 * Q0;
  float2 v[R0];
  if (s0) {
#pragma unroll
    for (int r = 0; r < R0; ++r) v[r] = psi[p0 * NN + sidx<N, TILE>(j0 + Q0 * r, u)];
  }
  float Iv[RL];
  if (tid < QL) {
#pragma unroll
    for (int r = 0; r < RL; ++r) Iv[r] = Ij[(size_t)(tid + QL * r) * N + u];
  }
  load_twiddles<N, 256>(tw);
  // forward stage 1 (no twiddles) -> LDS
  if (s0) {
    dftR<R0, false>(v);
#pragma unroll
    for (int r = 0; r < R0; ++r) bufA[p0 * N + j0 * R0 + r] = v[r];
  }
  __syncthreads();
  // forward stage 2, LDS -> LDS
  stage<N, R1, R0, false, 256>(bufA, bufB, M, tw);
  __syncthreads();
  // forward stage 3 (every mode per thread), modulus, inverse stage 1
  double e = 0.0, isv = 0.0;
  if (tid < QL) {
    float2 X[MM][RL];
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
#pragma unroll
        for (int r = 0; r < RL; ++r) X[p][r] = bufB[p * N + tid + QL * r];
#pragma unroll
        for (int r = 1; r < RL; ++r) X[p][r] = cmul(X[p][r], tw[r * tid]);
        dftR<RL, false>(X[p]);
      }
    const float invN = 1.0f / (float)N;
    bool bad = false;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      float S = 0.f;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) S += cabs2(X[p][r]);
      const float rs = S > 0.f ? __builtin_amdgcn_rsqf(S) : 0.f;
      const float Au = S * rs;
      const float sq = __builtin_amdgcn_sqrtf(fmaxf(Iv[r], 0.f));
      const float d = Au * invN - sq;
      e += (double)d * (double)d;
      isv += (double)fmaxf(Iv[r], 0.f);
      bad |= !isfinite(S);
      const float f = sq * rs * invN;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) X[p][r] = cscale(X[p][r], f);
    }
    if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        dftR<RL, true>(X[p]);
#pragma unroll
        for (int r = 0; r < RL; ++r) bufA[p * N + tid * RL + r] = X[p][r];
      }
  }
  __syncthreads();
  // inverse stage 2, LDS -> LDS
  stage<N, R1, RL, true, 256>(bufA, bufB, M, tw);
  __syncthreads();
  // inverse stage 3 -> global
  if (s0) {
#pragma unroll
    for (int r = 0; r < R0; ++r) v[r] = bufB[p0 * N + j0 + Q0 * r];
#pragma unroll
    for (int r = 1; r < R0; ++r) {
      float2 w = tw[r * j0];
      w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    dftR<R0, true>(v);
#pragma unroll
    for (int r = 0; r < R0; ++r) psi[p0 * NN + sidx<N, false>(j0 + Q0 * r, u)] = v[r];
  }
  e = wave_sum(e);
  isv = wave_sum(isv);
  if ((tid & 63) == 0) {
    *err_slot = err_old + e;
    *isum_slot = isum_old + isv;
  }
}

// The register-direct column pass for CW > 1 adjacent columns per workgroup
// (radix-8 three-stage plans): the same stage layout as cols_body_rd with
// CW M transforms, transform (p, c) at (p CW + c) PT; IP: one buffer, each
// LDS stage reading all of its inputs before any thread writes (one more
// barrier per stage, half the LDS).
// Consecutive threads take consecutive columns, so every global access
// moves CW * 8 contiguous bytes of a row; the pitch N + 16 / CW puts the CW
// transforms of one row index in different LDS banks.
template <int N, int MM, int CW, bool IP>
__device__ __forceinline__ void cols_body_rdw(const JobRec& jb, int t, float2* smem) {
  using P = Plan8<N>;
  constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2];
  static_assert(R2 > 1 && P::R[3] == 1, "three-stage plans only");
  constexpr int RL = R2;                         // last forward radix = first inverse radix
  constexpr int Q0 = N / R0;                     // butterflies per transform of the first stage
  constexpr int QL = N / RL;                     // mode-sum threads per column
  constexpr int NT = 256;
  constexpr int IT1 = (MM * CW * Q0 + NT - 1) / NT;  // first-stage butterflies per thread
  static_assert(CW * QL <= NT, "one mode-sum thread per (column, frequency group)");
  constexpr int PT = col_pitch<N, CW>();         // LDS pitch of a transform
  const int M = jb.M;
  const int total = jb.J * jb.T;
  if (t < 0 || t >= total) return;
  const int u = xcd_unit(blockIdx.x, gridDim.x);  // column group of this workgroup
  if (u >= N / CW) return;
  const int u0 = u * CW;
  const int it = t / jb.J, jn = t - it * jb.J;
  const WsLayout L = ws_layout(N, M, jb.T);
  const size_t NN = (size_t)N * N;
  float2* psi = (float2*)(jb.ws + pick(L.psi, t & 1));
  const float* Ij = jb.I + (size_t)jn * NN;
  const int tid = threadIdx.x;

  float2* tw = smem;
  float2* bufA = tw + N;                    // M CW PT
  float2* bufB = IP ? bufA : bufA + M * CW * PT;  // M CW PT

  const size_t slot = (size_t)it * kErrSlots + u * (NT / 64) + (tid >> 6);
  double* err_slot = (double*)(jb.ws + L.err) + slot;
  double* isum_slot = (double*)(jb.ws + L.isum) + slot;
  const double err_old = (tid & 63) == 0 ? *err_slot : 0.0;
  const double isum_old = (tid & 63) == 0 ? *isum_slot : 0.0;

  // first-stage inputs: butterfly b = tid + NT i is column c = b % CW,
  // index j = (b / CW) % Q0 of transform (p, c), p = b / (CW Q0): rows
  // j + Q0 r; and the patterns of the mode-sum threads
  const int nb1 = M * CW * Q0;
  float2 v[IT1][R0];
#pragma unroll
  for (int i = 0; i < IT1; ++i) {
    const int b = tid + NT * i;
    if (b < nb1) {
      const int c = b % CW, j = (b / CW) % Q0, p = b / (CW * Q0);
#pragma unroll
      for (int r = 0; r < R0; ++r) v[i][r] = psi[p * NN + (size_t)(j + Q0 * r) * N + u0 + c];
    }
  }
  const bool ms = tid < CW * QL;
  const int mc = tid % CW, mj = tid / CW;  // mode-sum thread: column, frequency group
  float Iv[RL];
  if (ms) {
#pragma unroll
    for (int r = 0; r < RL; ++r) Iv[r] = Ij[(size_t)(mj + QL * r) * N + u0 + mc];
  }
  load_twiddles<N, NT>(tw);
  // forward stage 1 (no twiddles) -> LDS
#pragma unroll
  for (int i = 0; i < IT1; ++i) {
    const int b = tid + NT * i;
    if (b < nb1) {
      const int c = b % CW, j = (b / CW) % Q0, p = b / (CW * Q0);
      dftR<R0, false>(v[i]);
#pragma unroll
      for (int r = 0; r < R0; ++r) bufA[(p * CW + c) * PT + j * R0 + r] = v[i][r];
    }
  }
  __syncthreads();
  // forward stage 2, LDS -> LDS
  constexpr int MB2 = (MM * CW * (N / R1) + NT - 1) / NT;  // butterflies per thread of stage 2
  if constexpr (IP) {
    stage_inplace<N, R1, R0, false, MB2, NT, PT>(bufA, M * CW, tw);
  } else {
    stage<N, R1, R0, false, NT, PT>(bufA, bufB, M * CW, tw);
    __syncthreads();
  }
  // forward stage 3 (every mode of one column per thread), modulus,
  // inverse stage 1
  double e = 0.0, isv = 0.0;
  float2 X[MM][RL];
  if (ms) {
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        const float2* src = bufB + (p * CW + mc) * PT;
#pragma unroll
        for (int r = 0; r < RL; ++r) X[p][r] = src[mj + QL * r];
      }
  }
  if constexpr (IP) lds_barrier();  // every read of the buffer before it is overwritten
  if (ms) {
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
#pragma unroll
        for (int r = 1; r < RL; ++r) X[p][r] = cmul(X[p][r], tw[r * mj]);
        dftR<RL, false>(X[p]);
      }
    const float invN = 1.0f / (float)N;
    bool bad = false;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      float S = 0.f;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) S += cabs2(X[p][r]);
      const float rs = S > 0.f ? __builtin_amdgcn_rsqf(S) : 0.f;
      const float Au = S * rs;
      const float sq = __builtin_amdgcn_sqrtf(fmaxf(Iv[r], 0.f));
      const float d = Au * invN - sq;
      e += (double)d * (double)d;
      isv += (double)fmaxf(Iv[r], 0.f);
      bad |= !isfinite(S);
      const float f = sq * rs * invN;
#pragma unroll
      for (int p = 0; p < MM; ++p)
        if (p < M) X[p][r] = cscale(X[p][r], f);
    }
    if (bad) flag_status(jb.status, MRPIE_STATUS_NONFINITE);
#pragma unroll
    for (int p = 0; p < MM; ++p)
      if (p < M) {
        dftR<RL, true>(X[p]);
        float2* dst = bufA + (p * CW + mc) * PT;
#pragma unroll
        for (int r = 0; r < RL; ++r) dst[mj * RL + r] = X[p][r];
      }
  }
  __syncthreads();
  // inverse stage 2, LDS -> LDS
  if constexpr (IP) {
    stage_inplace<N, R1, RL, true, MB2, NT, PT>(bufA, M * CW, tw);
  } else {
    stage<N, R1, RL, true, NT, PT>(bufA, bufB, M * CW, tw);
    __syncthreads();
  }
  // inverse stage 3 -> global
#pragma unroll
  for (int i = 0; i < IT1; ++i) {
    const int b = tid + NT * i;
    if (b < nb1) {
      const int c = b % CW, j = (b / CW) % Q0, p = b / (CW * Q0);
      const float2* src = bufB + (p * CW + c) * PT;
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
  e = wave_sum(e);
  isv = wave_sum(isv);
  if ((tid & 63) == 0) {
    *err_slot = err_old + e;
    *isum_slot = isum_old + isv;
  }
}

// R4: radix-4 FFT plan (else radix 8); MM: register capacity in probe modes
// (jobs of the launch have M <= MM), so small M does not pay the register
// cost (and occupancy) of the largest.  `tg` is the launch tick; a job runs
// its own step tg - t0 (t0 = 0 unless the job waited for an earlier job of
// its launch lane).
template <bool R4, int MM, bool IP>
__global__ __launch_bounds__(512) void k_rows(const LaunchArgs a, int tg) {
  extern __shared__ float2 smem[];
  const JobRec& jb = a.job[blockIdx.y];
  const int t = tg - jb.t0;
  switch (jb.N) {
    case 32: rows_body<32, R4, MM, IP>(a.c, jb, t, smem); break;
    case 64: rows_body<64, R4, MM, IP>(a.c, jb, t, smem); break;
    case 128: rows_body<128, R4, MM, IP>(a.c, jb, t, smem); break;
    case 192: rows_body<192, R4, MM, IP>(a.c, jb, t, smem); break;
    default: rows_body<256, R4, MM, IP>(a.c, jb, t, smem); break;
  }
}

template <bool R4, int MM, bool IP>
__global__ __launch_bounds__(512) void k_upd(const LaunchArgs a, int tg) {
  extern __shared__ float2 smem[];
  const JobRec& jb = a.job[blockIdx.y];
  const int t = tg - jb.t0;
  switch (jb.N) {
    case 32: upd_body<32, R4, MM, IP>(a.c, jb, t, smem); break;
    case 64: upd_body<64, R4, MM, IP>(a.c, jb, t, smem); break;
    case 128: upd_body<128, R4, MM, IP>(a.c, jb, t, smem); break;
    case 192: upd_body<192, R4, MM, IP>(a.c, jb, t, smem); break;
    default: upd_body<256, R4, MM, IP>(a.c, jb, t, smem); break;
  }
}

template <bool R4, int MM, bool IP>
__global__ __launch_bounds__(512) void k_gat(const LaunchArgs a, int tg) {
  extern __shared__ float2 smem[];
  const JobRec& jb = a.job[blockIdx.y];
  const int t = tg - jb.t0;
  switch (jb.N) {
    case 32: gat_body<32, R4, MM, IP>(jb, t, smem); break;
    case 64: gat_body<64, R4, MM, IP>(jb, t, smem); break;
    case 128: gat_body<128, R4, MM, IP>(jb, t, smem); break;
    case 192: gat_body<192, R4, MM, IP>(jb, t, smem); break;
    default: gat_body<256, R4, MM, IP>(jb, t, smem); break;
  }
}

template <bool R4, int MM, int CW, bool IP>
__global__ __launch_bounds__(256) void k_cols(const LaunchArgs a, int tg) {
  extern __shared__ float2 smem[];
  const JobRec& jb = a.job[blockIdx.y];
  const int t = tg - jb.t0;
  constexpr bool RD = !R4 && CW == 1 && !IP;
  constexpr bool RDW = !R4 && CW > 1;
  switch (jb.N) {
    case 32: cols_body<32, R4, MM, CW, IP>(jb, t, smem); break;
    case 64: cols_body<64, R4, MM, CW, IP>(jb, t, smem); break;
    case 128:
      if constexpr (RD) cols_body_rd<128, MM>(jb, t, smem);
      else if constexpr (RDW) cols_body_rdw<128, MM, CW, IP>(jb, t, smem);
      else cols_body<128, R4, MM, CW, IP>(jb, t, smem);
      break;
    case 192:
      if constexpr (RD) cols_body_rd<192, MM>(jb, t, smem);
      else if constexpr (RDW) cols_body_rdw<192, MM, CW, IP>(jb, t, smem);
      else cols_body<192, R4, MM, CW, IP>(jb, t, smem);
      break;
    default:
      if constexpr (RD) cols_body_rd<256, MM>(jb, t, smem);
      else if constexpr (RDW) cols_body_rdw<256, MM, CW, IP>(jb, t, smem);
      else cols_body<256, R4, MM, CW, IP>(jb, t, smem);
      break;
  }
}

// Single-job launches take the job as leading scalar arguments (NM = N |
// M << 16), which gfx950 preloads into SGPRs: the first loads of a launch
// do not wait for a kernel-argument fetch (about 1 us per launch).
template <bool R4, int MM>
__global__ __launch_bounds__(512) void k_rows1(char* ws, float2* obj, float2* probe, const float* pos, int t, int J,
                                               int T, int NM, int H, int W, const float* I, int* status,
                                               const Common c) {
  extern __shared__ float2 smem[];
  const JobRec jb{obj, probe, pos, I, ws, status, H, W, NM & 0xffff, NM >> 16, J, T};
  switch (jb.N) {
    case 32: rows_body<32, R4, MM, false, true>(c, jb, t, smem); break;
    case 64: rows_body<64, R4, MM, false, true>(c, jb, t, smem); break;
    case 128: rows_body<128, R4, MM, false, true>(c, jb, t, smem); break;
    case 192: rows_body<192, R4, MM, false, true>(c, jb, t, smem); break;
    default: rows_body<256, R4, MM, false, true>(c, jb, t, smem); break;
  }
}

template <bool R4, int MM, int CW>
__global__ __launch_bounds__(256) void k_cols1(char* ws, const float* I, int t, int J, int T, int NM, int* status) {
  extern __shared__ float2 smem[];
  const JobRec jb{nullptr, nullptr, nullptr, I, ws, status, 0, 0, NM & 0xffff, NM >> 16, J, T};
  // radix-8 plans with one column per workgroup: stages in registers at
  // both ends from N = 128 on
  constexpr bool RD = !R4 && CW == 1;
  switch (jb.N) {
    case 32: cols_body<32, R4, MM, CW, false, true>(jb, t, smem); break;
    case 64: cols_body<64, R4, MM, CW, false, true>(jb, t, smem); break;
    case 128:
      if constexpr (RD) cols_body_rd<128, MM, true>(jb, t, smem);
      else cols_body<128, R4, MM, CW, false, true>(jb, t, smem);
      break;
    case 192:
      if constexpr (RD) cols_body_rd<192, MM, true>(jb, t, smem);
      else cols_body<192, R4, MM, CW, false, true>(jb, t, smem);
      break;
    default:
      if constexpr (RD) cols_body_rd<256, MM, true>(jb, t, smem);
      else cols_body<256, R4, MM, CW, false, true>(jb, t, smem);
      break;
  }
}

using SweepKernel = void (*)(const LaunchArgs, int);
using RowsKernel1 = void (*)(char*, float2*, float2*, const float*, int, int, int, int, int, int, const float*, int*,
                             const Common);
using ColsKernel1 = void (*)(char*, const float*, int, int, int, int, int*);

static int mode_class(int M) { return M <= 1 ? 1 : M <= 2 ? 2 : M <= 4 ? 4 : 8; }
// Register capacity of the multi-job kernels: one more class for 5 or 6
// modes, so batches whose largest job has 5 modes (a common mix) do not pay
// the register arrays (and occupancy) of 8.
static int batch_mode_class(int M) { return M <= 4 ? mode_class(M) : M <= 6 ? 6 : 8; }

template <bool R4, bool IP>
static SweepKernel pick_rows(int mc) {
  switch (mc) {
    case 1: return k_rows<R4, 1, IP>;
    case 2: return k_rows<R4, 2, IP>;
    case 4: return k_rows<R4, 4, IP>;
    case 6: return k_rows<R4, 6, IP>;
    default: return k_rows<R4, 8, IP>;
  }
}
template <bool R4, int CW, bool IP>
static SweepKernel pick_cols(int mc) {
  switch (mc) {
    case 1: return k_cols<R4, 1, CW, IP>;
    case 2: return k_cols<R4, 2, CW, IP>;
    case 4: return k_cols<R4, 4, CW, IP>;
    case 6: return k_cols<R4, 6, CW, IP>;
    default: return k_cols<R4, 8, CW, IP>;
  }
}
template <bool R4, bool IP>
static SweepKernel pick_upd(int mc) {
  switch (mc) {
    case 1: return k_upd<R4, 1, IP>;
    case 2: return k_upd<R4, 2, IP>;
    case 4: return k_upd<R4, 4, IP>;
    case 6: return k_upd<R4, 6, IP>;
    default: return k_upd<R4, 8, IP>;
  }
}
template <bool R4, bool IP>
static SweepKernel pick_gat(int mc) {
  switch (mc) {
    case 1: return k_gat<R4, 1, IP>;
    case 2: return k_gat<R4, 2, IP>;
    case 4: return k_gat<R4, 4, IP>;
    case 6: return k_gat<R4, 6, IP>;
    default: return k_gat<R4, 8, IP>;
  }
}
template <bool R4>
static RowsKernel1 pick_rows1(int mc) {
  switch (mc) {
    case 1: return k_rows1<R4, 1>;
    case 2: return k_rows1<R4, 2>;
    case 4: return k_rows1<R4, 4>;
    default: return k_rows1<R4, 8>;
  }
}
template <bool R4, int CW>
static ColsKernel1 pick_cols1(int mc) {
  switch (mc) {
    case 1: return k_cols1<R4, 1, CW>;
    case 2: return k_cols1<R4, 2, CW>;
    case 4: return k_cols1<R4, 4, CW>;
    default: return k_cols1<R4, 8, CW>;
  }
}
static RowsKernel1 rows_kernel1(int radix, int M) {
  return radix == 8 ? pick_rows1<false>(mode_class(M)) : pick_rows1<true>(mode_class(M));
}
static ColsKernel1 cols_kernel1(int radix, int width, int M) {
  const int mc = mode_class(M);
  if (width == 4) return radix == 8 ? pick_cols1<false, 4>(mc) : pick_cols1<true, 4>(mc);
  return radix == 8 ? pick_cols1<false, 1>(mc) : pick_cols1<true, 1>(mc);
}
static SweepKernel rows_kernel(int radix, bool inplace, int maxM) {
  const int mc = batch_mode_class(maxM);
  if (inplace) return radix == 8 ? pick_rows<false, true>(mc) : pick_rows<true, true>(mc);
  return radix == 8 ? pick_rows<false, false>(mc) : pick_rows<true, false>(mc);
}
static SweepKernel upd_kernel(int radix, bool inplace, int maxM) {
  const int mc = batch_mode_class(maxM);
  if (inplace) return radix == 8 ? pick_upd<false, true>(mc) : pick_upd<true, true>(mc);
  return radix == 8 ? pick_upd<false, false>(mc) : pick_upd<true, false>(mc);
}
static SweepKernel gat_kernel(int radix, bool inplace, int maxM) {
  const int mc = batch_mode_class(maxM);
  if (inplace) return radix == 8 ? pick_gat<false, true>(mc) : pick_gat<true, true>(mc);
  return radix == 8 ? pick_gat<false, false>(mc) : pick_gat<true, false>(mc);
}
// multi-job launches; in place only with 4 columns per workgroup
static SweepKernel cols_kernel(int radix, int width, bool inplace, int maxM) {
  const int mc = batch_mode_class(maxM);
  if (width == 4 && inplace) return radix == 8 ? pick_cols<false, 4, true>(mc) : pick_cols<true, 4, true>(mc);
  if (width == 4) return radix == 8 ? pick_cols<false, 4, false>(mc) : pick_cols<true, 4, false>(mc);
  return radix == 8 ? pick_cols<false, 1, false>(mc) : pick_cols<true, 1, false>(mc);
}

// ------------------------------------------------------- small kernels
__global__ void k_zero_err(const LaunchArgs a) {
  const JobRec& jb = a.job[blockIdx.y];
  const WsLayout L = ws_layout(jb.N, jb.M, jb.T);
  double* e = (double*)(jb.ws + L.err);
  double* is = (double*)(jb.ws + L.isum);
  const size_t n = (size_t)(jb.T > 0 ? jb.T : 1) * kErrSlots;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    e[i] = 0.0;
    is[i] = 0.0;
  }
}

struct ErrOut {
  float* p[kMaxJobsPerLaunch];
};

// err_out[it] = sum of the iteration's error partials / sum of its
// intensity partials (both accumulated by the column passes)
__global__ __launch_bounds__(256) void k_finish(const LaunchArgs a, const ErrOut eo) {
  __shared__ double red[16];
  const JobRec& jb = a.job[blockIdx.y];
  const WsLayout L = ws_layout(jb.N, jb.M, jb.T);
  float* out = eo.p[blockIdx.y];
  if (!out) return;
  const double* err = (const double*)(jb.ws + L.err);
  const double* isp = (const double*)(jb.ws + L.isum);
  for (int t = 0; t < jb.T; ++t) {
    double e = 0.0, v = 0.0;
    for (int i = threadIdx.x; i < kErrSlots; i += blockDim.x) {
      e += err[(size_t)t * kErrSlots + i];
      v += isp[(size_t)t * kErrSlots + i];
    }
    e = block_sum(e, red);
    v = block_sum(v, red);
    if (threadIdx.x == 0) out[t] = (float)(v > 0.0 ? e / v : e);
  }
}

// the final probe lives in buffer (J*T)&1; copy it back when that is the
// workspace buffer
__global__ void k_probe_back(const LaunchArgs a) {
  const JobRec& jb = a.job[blockIdx.y];
  if (((long long)jb.J * jb.T) % 2 == 0) return;
  const WsLayout L = ws_layout(jb.N, jb.M, jb.T);
  const float2* src = (const float2*)(jb.ws + L.probe1);
  const size_t n = (size_t)jb.M * jb.N * jb.N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    jb.probe[i] = src[i];
}

// ------------------------------------------------------------ tuning
// Launch shapes of the sweep, per (N, batch class): FFT radix plan of each
// pass, threads per row workgroup, and up to which mode count a job whose
// modes fit the LDS runs the one-workgroup sweep.  The defaults were the
// fastest measured on MI355X: radix 8 in both passes with 256 threads for
// 256^2 x 3; the one-workgroup sweep for 32^2 (5 modes: 9.3 against 12.9 us
// per position) and 64^2 x 1 (9.6 against 11.6 us), the passes from 64^2 x 3
// (13.3 against 20.0 us) and 128^2 x 1 (12.3 against 42.3 us) on, where one
// CU's vector ALUs and LDS bandwidth bound the one-workgroup sweep; one
// detector column per column workgroup for a single sweep (19.5 against
// 23.3 us per position at 256^2 x 3), four in batches (8 jobs: 52.1 against
// 57.2 us per lock-step position, 32 jobs: 168 against 182 us); in-place
// inverse row FFTs in batches (8 jobs: 45.4 against 49.7 us, 32 jobs: 140
// against 164 us), ping-pong for a single sweep.  The
// autotuner measures the alternatives on the device for any (N, M, batch).
// Per (N, mode class, batch class); mode classes M = 1, 2, 3-4, 5-8 (the
// single-job kernels' register capacities; the multi-job kernels split the
// last class into 5-6 and 7-8).
static Tuning g_tune[5][4][3];
static bool g_tune_set[5][4][3];
static std::mutex g_tune_mu;

// Call classes: a single job, batches of 2 to kLargeBatch - 1 jobs, larger
// batches (the batch sizes where the in-place and split options pay differ).
constexpr int kLargeBatch = 16;
static int batch_class(int nb) { return nb <= 1 ? 0 : nb < kLargeBatch ? 1 : 2; }
int batch_class_jobs(int cls) { return cls <= 0 ? 1 : cls == 1 ? 2 : kLargeBatch; }
static int mode_index(int M) { return M <= 1 ? 0 : M <= 2 ? 1 : M <= 4 ? 2 : 3; }

// The one-workgroup LDS sweep is the default for a single small job only: in
// a batch, small jobs ride along in the shared row / column launches, which
// the other jobs' launches pay for anyway (uneven 64-job batch: 439k -> 480k
// positions x iterations / s eager, 310k -> 337k as a replayed graph, where
// the LDS sweep's long single launch would otherwise run ahead of the passes
// on the one stream).
Tuning default_tuning(int N, int nb) {
  const int bc = batch_class(nb);
  const int lds = bc ? 0 : N == 32 ? MRPIE_MAX_MODES : N == 64 ? 1 : 0;
  return Tuning{8, 8, 256, lds, bc ? 4 : 1, bc ? 1 : 0, bc == 2 ? 1 : 0};
}

Tuning get_tuning(int N, int M, int nb) {
  const int ni = n_index(N), mi = mode_index(M), bc = batch_class(nb);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (ni >= 0 && g_tune_set[ni][mi][bc]) return g_tune[ni][mi][bc];
  return default_tuning(N, nb);
}

void set_tuning(int N, int M, int nb, const Tuning& t) {
  const int ni = n_index(N), bc = batch_class(nb);
  if (ni < 0) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int mi = 0; mi < 4; ++mi)
    if (M <= 0 || mi == mode_index(M)) {
      g_tune[ni][mi][bc] = t;
      g_tune_set[ni][mi][bc] = true;
    }
}

// ------------------------------------------------------------ host driver
// LDS of the row passes: twiddles, the updated object row and the transforms
// at the padded pitch col_pitch<N, 1, true>()
static int row_pitch(int N) { return (N + N / 16 + 15) / 16 * 16; }
static size_t rows_lds(int N, int M, bool inplace) {
  return (size_t)(N + N + (inplace ? 2 : 4) * M * row_pitch(N)) * 8;
}
// LDS of the column pass: twiddles and the transforms at the padded pitch
// col_pitch<N, cw, true>() (the one-column register-direct variant uses
// less)
static size_t cols_lds(int N, int M, int cw, bool inplace) {
  const int base = (N + N / 16 + 15) / 16 * 16;
  const int pitch = cw > 1 ? base + 16 / cw : base;
  return (size_t)(N + (inplace ? 1 : 2) * cw * M * pitch) * 8;
}
static size_t split_lds(int N, int M, bool inplace, int rows) {
  return (size_t)(N + (inplace ? 1 : 2) * rows * M * row_pitch(N)) * 8;
}

// The column pass runs in place with the row pass only in calls of this many
// jobs or more: it doubles the workgroups per CU but adds a barrier per
// stage, which pays once the launches are throughput bound (measured at
// 256^2 x 3 with one launch chain per call: 32 jobs 122 against 134 us per
// lock-step position, 8 jobs 41.9 against 41.1 us).
constexpr int kColsInplaceJobs = 16;

void launch_zero_err(const LaunchArgs& a, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_err, dim3(8, nb), dim3(256), 0, s, a);
}

void launch_finish(const LaunchArgs& a, int nb, float* const* err_out, hipStream_t s, bool probe_back) {
  ErrOut eo{};
  for (int b = 0; b < nb; ++b) eo.p[b] = err_out ? err_out[b] : nullptr;
  if (probe_back) hipLaunchKernelGGL(k_probe_back, dim3(64, nb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_finish, dim3(1, nb), dim3(256), 0, s, a, eo);
}

// One launch group: the jobs of one stream that share every launch (a
// single-job call takes the scalar-argument kernels).  The jobs are dealt to
// at most kMaxJobsPerLaunch lanes: the longest first, each to the lane that
// frees up first, where it starts one tick after the lane's previous job
// took its last update.  Every tick's launches carry the jobs the lanes are
// running at that tick, so a launch never exceeds kMaxJobsPerLaunch jobs and
// carries no finished job, and the short jobs of an uneven batch queue
// behind each other in the lanes instead of taking launches of their own.
struct PassGroup {
  LaunchArgs a{};  // single-job calls: the job
  int maxTot = 0;  // last tick of the group
  bool single = false;  // a single-job call: the scalar-argument kernels
  bool split = false;   // update / gather / column launches per position
  int srows = 1;        // rows per workgroup of the split passes
  int width = 1;
  size_t lr = 0, lc = 0, lu = 0;
  dim3 rblk;
  SweepKernel kr = nullptr, kc = nullptr, ku = nullptr, kg = nullptr;
  RowsKernel1 kr1 = nullptr;
  ColsKernel1 kc1 = nullptr;
  hipStream_t s = nullptr;
  std::vector<JobRec> jobs;             // every job of the group, start ticks set
  std::vector<float*> err;
  std::vector<std::vector<int>> lanes;  // the jobs of each lane, in start order
  std::vector<size_t> cur;              // per lane: its current job
};

static long long job_ticks(const JobRec& jb) { return (long long)jb.J * jb.T; }

// Deal the jobs to the lanes and set their start ticks.
static int deal_lanes(PassGroup& g) {
  const int n = (int)g.jobs.size();
  const int nl = std::min(n, kMaxJobsPerLaunch);
  std::vector<int> order(n);
  for (int b = 0; b < n; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return job_ticks(g.jobs[x]) > job_ticks(g.jobs[y]); });
  std::vector<long long> load(nl, 0);
  g.lanes.assign(nl, {});
  g.cur.assign(nl, 0);
  long long last = 0;
  for (int b : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    const long long tot = job_ticks(g.jobs[b]);
    if (tot == 0) continue;  // no iterations: nothing to launch
    g.jobs[b].t0 = (int)load[l];
    load[l] += tot + 1;      // job ticks 0 .. tot
    if (load[l] > INT32_MAX) return fail(MRPIE_EINVAL, "batched call: a launch lane exceeds 2^31 ticks");
    last = std::max(last, load[l] - 1);
    g.lanes[l].push_back(b);
  }
  g.maxTot = (int)last;
  return MRPIE_OK;
}

// `call_jobs` (the jobs of the whole call) picks the tuning class and the
// kernels, so a job computes the same bits whichever group and stream it is
// dealt to.
static int prepare_group(PassGroup& g, const Common& c, const JobRec* const* jobs, float* const* err, int nb,
                         int call_jobs, hipStream_t s, const Tuning* force) {
  g.s = s;
  int maxN = 64, maxM = 1;
  for (int b = 0; b < nb; ++b) {
    g.jobs.push_back(*jobs[b]);
    g.jobs.back().t0 = 0;
    g.err.push_back(err[b]);
    maxN = std::max(maxN, jobs[b]->N);
    maxM = std::max(maxM, jobs[b]->M);
  }
  const Tuning tu = force ? *force : get_tuning(maxN, maxM, call_jobs);
  const bool ip = call_jobs > 1 && tu.rows_inplace;
  const bool cip = ip && tu.cols_width == 4 && call_jobs >= kColsInplaceJobs;
  for (const JobRec& jb : g.jobs) g.lr = std::max(g.lr, rows_lds(jb.N, jb.M, ip));
  for (const JobRec& jb : g.jobs) g.lc = std::max(g.lc, cols_lds(jb.N, jb.M, tu.cols_width, cip));
  g.width = tu.cols_width;
  g.rblk = dim3(tu.rows_threads);
  g.single = call_jobs == 1;
  if (g.single) {
    g.a.c = c;
    g.a.njobs = 1;
    g.a.job[0] = g.jobs[0];
    g.maxTot = (int)job_ticks(g.jobs[0]);
    g.kr1 = rows_kernel1(tu.rows_radix, g.jobs[0].M);
    g.kc1 = cols_kernel1(tu.cols_radix, tu.cols_width, g.jobs[0].M);
    MRPIE_HIP(ensure_lds((const void*)g.kr1, g.lr));
    MRPIE_HIP(ensure_lds((const void*)g.kc1, g.lc));
    return MRPIE_OK;
  }
  const int rc = deal_lanes(g);
  if (rc) return rc;
  if (tu.rows_split) {
    g.split = true;
    g.srows = split_rows(batch_mode_class(maxM));
    for (const JobRec& jb : g.jobs) g.lu = std::max(g.lu, split_lds(jb.N, jb.M, ip, g.srows));
    g.ku = upd_kernel(tu.rows_radix, ip, maxM);
    g.kg = gat_kernel(tu.rows_radix, ip, maxM);
    g.kc = cols_kernel(tu.cols_radix, tu.cols_width, cip, maxM);
    MRPIE_HIP(ensure_lds((const void*)g.ku, g.lu));
    MRPIE_HIP(ensure_lds((const void*)g.kg, g.lu));
    MRPIE_HIP(ensure_lds((const void*)g.kc, g.lc));
  } else {
    g.kr = rows_kernel(tu.rows_radix, ip, maxM);
    g.kc = cols_kernel(tu.cols_radix, tu.cols_width, cip, maxM);
    MRPIE_HIP(ensure_lds((const void*)g.kr, g.lr));
    MRPIE_HIP(ensure_lds((const void*)g.kc, g.lc));
  }
  return MRPIE_OK;
}

// The job tables of tick t: `all` the jobs running (their steps 0 .. J T),
// `upd` those with a previous step to update (1 .. J T), `nxt` those with a
// step to gather (0 .. J T - 1).  Largest probe size of each in *_n.
struct TickTables {
  LaunchArgs all, upd, nxt;
  int all_n = 0, upd_n = 0, nxt_n = 0;
};

static void tick_tables(PassGroup& g, const Common& c, int t, TickTables& tt) {
  tt.all.c = tt.upd.c = tt.nxt.c = c;
  int na = 0, nu = 0, nn = 0;
  for (size_t l = 0; l < g.lanes.size(); ++l) {
    const std::vector<int>& q = g.lanes[l];
    size_t& k = g.cur[l];
    while (k < q.size() && g.jobs[q[k]].t0 + job_ticks(g.jobs[q[k]]) < t) ++k;
    if (k == q.size() || g.jobs[q[k]].t0 > t) continue;
    const JobRec& jb = g.jobs[q[k]];
    const long long lt = t - jb.t0;
    tt.all.job[na++] = jb;
    tt.all_n = std::max(tt.all_n, jb.N);
    if (lt > 0) {
      tt.upd.job[nu++] = jb;
      tt.upd_n = std::max(tt.upd_n, jb.N);
    }
    if (lt < job_ticks(jb)) {
      tt.nxt.job[nn++] = jb;
      tt.nxt_n = std::max(tt.nxt_n, jb.N);
    }
  }
  tt.all.njobs = na;
  tt.upd.njobs = nu;
  tt.nxt.njobs = nn;
}

// tick t of a group: the (t-1 -> t) row pass and the column pass of step t
static void launch_tick(PassGroup& g, const Common& c, int t) {
  const dim3 blk(256);
  if (g.single) {
    const JobRec& jb = g.a.job[0];
    const int NM = jb.N | (jb.M << 16);
    launch_k(TK_ROWS, g.kr1, dim3(jb.N, 1), g.rblk, g.lr, g.s, jb.ws, jb.obj, jb.probe, jb.pos, t, jb.J, jb.T, NM,
             jb.H, jb.W, jb.I, jb.status, c);
    if (t < g.maxTot)
      launch_k(TK_COLS, g.kc1, dim3(jb.N / g.width, 1), blk, g.lc, g.s, jb.ws, jb.I, t, jb.J, jb.T, NM, jb.status);
    return;
  }
  TickTables tt;
  tick_tables(g, c, t, tt);
  if (g.split) {
    if (tt.upd.njobs) launch_k(TK_UPD, g.ku, dim3(tt.upd_n / g.srows, tt.upd.njobs), g.rblk, g.lu, g.s, tt.upd, t);
    if (tt.nxt.njobs) {
      launch_k(TK_GAT, g.kg, dim3(tt.nxt_n / g.srows, tt.nxt.njobs), g.rblk, g.lu, g.s, tt.nxt, t);
      launch_k(TK_COLS, g.kc, dim3(tt.nxt_n / g.width, tt.nxt.njobs), blk, g.lc, g.s, tt.nxt, t);
    }
    return;
  }
  if (tt.all.njobs) launch_k(TK_ROWS, g.kr, dim3(tt.all_n, tt.all.njobs), g.rblk, g.lr, g.s, tt.all, t);
  if (tt.nxt.njobs) launch_k(TK_COLS, g.kc, dim3(tt.nxt_n / g.width, tt.nxt.njobs), blk, g.lc, g.s, tt.nxt, t);
}

// The per-job launches before and after the passes (error partials cleared;
// the final probe copied back, the errors reduced), kMaxJobsPerLaunch jobs
// at a time.
static void launch_group_edges(const PassGroup& g, const Common& c, bool after) {
  if (g.single) {
    if (!after) hipLaunchKernelGGL(k_zero_err, dim3(8, 1), dim3(256), 0, g.s, g.a);
    else launch_finish(g.a, 1, g.err.data(), g.s, true);
    return;
  }
  const int n = (int)g.jobs.size();
  for (int c0 = 0; c0 < n; c0 += kMaxJobsPerLaunch) {
    const int nb = std::min(kMaxJobsPerLaunch, n - c0);
    LaunchArgs a{};
    a.c = c;
    a.njobs = nb;
    for (int b = 0; b < nb; ++b) a.job[b] = g.jobs[c0 + b];
    // (the split passes update the probe in place: nothing to copy back)
    if (!after) hipLaunchKernelGGL(k_zero_err, dim3(8, nb), dim3(256), 0, g.s, a);
    else launch_finish(a, nb, g.err.data() + c0, g.s, !g.split);
  }
}

// Row / column passes, lock-step over the jobs.  With a second stream `s2`
// (already forked from `s`) the jobs are dealt alternately to the two
// streams, one launch group each, and the launches of both groups are
// issued tick by tick.  A launch of a few jobs leaves most of the GPU idle
// while it waits on memory, so the other stream's launches fill it
// (measured at 256^2 x 3: 8 jobs 198k -> 219k, 32 jobs 266k -> 287k
// positions x iterations / s; four streams gained less than two).
static int run_passes(const Common& c, const JobRec* jobs, int njobs, float* const* err_out, hipStream_t s,
                      hipStream_t s2, const Tuning* force) {
  const int ns = s2 ? 2 : 1;
  std::vector<PassGroup> groups(ns);
  for (int k = 0; k < ns; ++k) {
    std::vector<const JobRec*> js;
    std::vector<float*> es;
    for (int b = k; b < njobs; b += ns) {
      js.push_back(&jobs[b]);
      es.push_back(err_out ? err_out[b] : nullptr);
    }
    const int rc = prepare_group(groups[k], c, js.data(), es.data(), (int)js.size(), njobs, k == 0 ? s : s2, force);
    if (rc) return rc;
  }
  int maxTot = 0;
  for (const PassGroup& g : groups) {
    launch_group_edges(g, c, false);
    maxTot = std::max(maxTot, g.maxTot);
  }
  for (int t = 0; t <= maxTot; ++t)
    for (PassGroup& g : groups)
      if (g.maxTot > 0 && t <= g.maxTot) launch_tick(g, c, t);
  for (const PassGroup& g : groups) launch_group_edges(g, c, true);
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

// Jobs whose modes fit the LDS (and whose tuning allows it) run the
// one-workgroup sweep; the rest run the row / column passes.  With two or
// more jobs the call forks the library's side stream from `s` (after the
// twiddle tables are written on `s`) and joins it back at the end: the LDS
// sweep and every second job of the passes run there, the rest on `s`.
// Under stream capture everything stays on `s`: a replayed graph of one
// launch chain is faster than one of two interleaved chains (8 jobs at
// 256^2 x 3: 204k against 146k positions x iterations / s).
int run_sweep(const Common& c, const JobRec* jobs, int njobs, float* const* err_out, hipStream_t s,
              const Tuning* force) {
  std::vector<JobRec> lj, pj;
  std::vector<float*> le, pe;
  for (int b = 0; b < njobs; ++b) {
    const JobRec& jb = jobs[b];
    const int lds_max = force ? force->lds_sweep : get_tuning(jb.N, jb.M, njobs).lds_sweep;
    const bool lds = jb.M <= lds_max && lds_sweep_fits(jb.N, jb.M);
    (lds ? lj : pj).push_back(jb);
    (lds ? le : pe).push_back(err_out ? err_out[b] : nullptr);
  }
  int rc = launch_init_twiddles(s);
  if (rc) return rc;
  hipStream_t s2 = nullptr;
  hipEvent_t* ev = nullptr;
  std::unique_lock<std::mutex> lk;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  MRPIE_HIP(hipStreamIsCapturing(s, &cap));
  if (njobs >= 2 && cap == hipStreamCaptureStatusNone) {
    rc = side_stream(&s2, &ev);
    if (rc) return rc;
    lk = std::unique_lock<std::mutex>(side_mutex());
    MRPIE_HIP(hipEventRecord(ev[0], s));
    MRPIE_HIP(hipStreamWaitEvent(s2, ev[0], 0));
  }
  if (!lj.empty()) rc = run_lds_sweep(c, lj.data(), (int)lj.size(), le.data(), s2 ? s2 : s);
  if (!rc && !pj.empty())
    rc = run_passes(c, pj.data(), (int)pj.size(), pe.data(), s, pj.size() >= 2 ? s2 : nullptr, force);
  if (s2) {  // joined also after an error, so `s` never runs ahead of the side stream's work
    MRPIE_HIP(hipEventRecord(ev[1], s2));
    MRPIE_HIP(hipStreamWaitEvent(s, ev[1], 0));
  }
  return rc;
}

// Workspace of mrpie_rpie: the sweep layout, then (refinement only) the
// recorded patch pairs, shifts, peaks and the registration workspace.
struct RefineLayout {
  size_t ref, mov, shift, peak, reg, total;
};

static RefineLayout refine_layout(const mrpie_problem* pb, const mrpie_params* pr) {
  RefineLayout R{};
  size_t off = ws_layout(pb->N, pb->M, pr->iterations).total;
  auto take = [&](size_t bytes) { size_t o = off; off = ws_align(off + bytes); return o; };
  if (pr->refine) {
    const size_t NN = (size_t)pb->N * pb->N;
    R.ref = take((size_t)pb->J * NN * 8);
    R.mov = take((size_t)pb->J * NN * 8);
    R.shift = take((size_t)pb->J * 8);
    R.peak = take((size_t)pb->J * 16);
    R.reg = take(reg_layout(pb->N, pb->J, pr->upsample).total);
  }
  R.total = off;
  return R;
}

size_t rpie_ws_total(const mrpie_problem* pb, const mrpie_params* pr) { return refine_layout(pb, pr).total; }

int run_refining_sweep(const Common& c, const JobRec& jb, const mrpie_params* pr, float* adam, float* err_out,
                       hipStream_t s) {
  mrpie_problem pb{jb.H, jb.W, jb.N, jb.M, jb.J};
  const RefineLayout R = refine_layout(&pb, pr);
  int rc = MRPIE_OK;
  LaunchArgs la{};
  la.c = c;
  la.njobs = 1;
  la.job[0] = jb;
  launch_zero_err(la, 1, s);
  SubpixelExtra ex{pr->subpixel, nullptr, nullptr, pr->refine_start};
  ex.xcb = pr->refine ? pr->xcorr_point : 0;
  ex.fresnel = pr->propagator ? pr->fresnel : 0.f;
  if (!pr->refine) {
    rc = run_sweep_subpixel(c, jb, ex, 0, jb.T, true, true, s);
    if (rc) return rc;
  } else {
    ex.reg_ref = (float2*)(jb.ws + R.ref);
    ex.reg_mov = (float2*)(jb.ws + R.mov);
    float* shift = (float*)(jb.ws + R.shift);
    int32_t* peak = (int32_t*)(jb.ws + R.peak);
    const size_t reg_bytes = reg_layout(jb.N, jb.J, pr->upsample).total;
    // Per iteration: the sweep (recording every position's patch before and
    // after its update once refinement has started), the registration of
    // all J pairs, the Adam step.  The registration runs after the sweep on
    // the same stream: overlapping it with the latency-bound sweep on a
    // second stream slowed the sweep by about what it hid (256^2 x 3, 1600
    // positions, upsample 100: 50.1 against 49.0 ms per iteration).
    for (int it = 0; it < jb.T; ++it) {
      const int it_abs = pr->iter_offset + it;
      rc = run_sweep_subpixel(c, jb, ex, it, 1, true, true, s);
      if (rc) return rc;
      if (it_abs < pr->refine_start) continue;
      rc = run_register(jb.N, jb.J, ex.reg_ref, ex.reg_mov, pr->upsample, pr->xcorr_norm, shift, peak,
                        jb.ws + R.reg, reg_bytes, s);
      if (rc) return rc;
      rc = launch_adam(jb.J, (float*)jb.pos, adam, shift, it_abs - pr->refine_start + 1, pr, jb.H - jb.N,
                       jb.W - jb.N, s);
      if (rc) return rc;
    }
  }
  float* eo[1] = {err_out};
  launch_finish(la, 1, eo, s);
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

int check_tuning(const mrpie_tuning* t) {
  if (!t) return fail(MRPIE_EINVAL, "tuning is NULL");
  if ((t->rows_radix != 4 && t->rows_radix != 8) || (t->cols_radix != 4 && t->cols_radix != 8))
    return fail(MRPIE_EINVAL, "radix must be 4 or 8");
  if (t->rows_threads != 256 && t->rows_threads != 512) return fail(MRPIE_EINVAL, "rows_threads must be 256 or 512");
  if (t->lds_sweep < 0 || t->lds_sweep > MRPIE_MAX_MODES) return fail(MRPIE_EINVAL, "lds_sweep must be in [0, 8]");
  if (t->cols_width != 1 && t->cols_width != 4) return fail(MRPIE_EINVAL, "cols_width must be 1 or 4");
  if (t->rows_inplace != 0 && t->rows_inplace != 1) return fail(MRPIE_EINVAL, "rows_inplace must be 0 or 1");
  if (t->rows_split != 0 && t->rows_split != 1) return fail(MRPIE_EINVAL, "rows_split must be 0 or 1");
  return MRPIE_OK;
}

}  // namespace mrpie

using namespace mrpie;

extern "C" {

int mrpie_validate(const mrpie_problem* pb, const mrpie_params* pr) {
  if (!pb || !pr) return fail(MRPIE_EINVAL, "null problem or params");
  if (n_index(pb->N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", pb->N);
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
  if ((long long)pr->iterations * pb->J >= (1LL << 30)) return fail(MRPIE_EINVAL, "iterations x J too large");
  if (pr->iter_offset < 0) return fail(MRPIE_EINVAL, "iter_offset=%d < 0", pr->iter_offset);
  if (pr->subpixel != 0 && pr->subpixel != 1) return fail(MRPIE_EINVAL, "subpixel must be 0 or 1");
  if (pr->refine != 0 && pr->refine != 1) return fail(MRPIE_EINVAL, "refine must be 0 or 1");
  if (pr->refine) {
    if (pr->upsample < 1 || pr->upsample > 1000) return fail(MRPIE_EINVAL, "upsample=%d not in [1,1000]", pr->upsample);
    if (pr->xcorr_norm != 0 && pr->xcorr_norm != 1) return fail(MRPIE_EINVAL, "xcorr_norm must be 0 or 1");
    if (!(pr->adam_b1 >= 0.f && pr->adam_b1 < 1.f) || !(pr->adam_b2 >= 0.f && pr->adam_b2 < 1.f))
      return fail(MRPIE_EINVAL, "Adam betas must be in [0,1)");
    if (!(pr->adam_eps > 0.f) || !finite(pr->adam_lr)) return fail(MRPIE_EINVAL, "bad Adam lr/eps");
    if (pr->xcorr_point != 0 && pr->xcorr_point != 1) return fail(MRPIE_EINVAL, "xcorr_point must be 0 or 1");
  }
  if (pr->propagator != 0 && pr->propagator != 1) return fail(MRPIE_EINVAL, "propagator must be 0 or 1");
  if (pr->propagator && !(pr->fresnel > 0.f && finite(pr->fresnel)))
    return fail(MRPIE_EINVAL, "fresnel=%g must be a finite number > 0 for the near field", pr->fresnel);
  return MRPIE_OK;
}

int mrpie_workspace_size(const mrpie_problem* pb, const mrpie_params* pr, size_t* bytes) {
  int rc = mrpie_validate(pb, pr);
  if (rc) return rc;
  if (!bytes) return fail(MRPIE_EINVAL, "bytes is NULL");
  *bytes = rpie_ws_total(pb, pr);
  return MRPIE_OK;
}

int mrpie_rpie(const mrpie_problem* pb, const mrpie_params* pr, void* obj, void* probe, float* pos,
               float* adam, const float* intens, float* err_out, int32_t* status, void* ws, size_t ws_bytes,
               void* stream) {
  int rc = mrpie_validate(pb, pr);
  if (rc) return rc;
  if (!obj || !probe || !pos || !intens) return fail(MRPIE_EINVAL, "null array pointer");
  if (pr->refine && !adam) return fail(MRPIE_EINVAL, "adam state is NULL with refine = 1");
  const size_t need = rpie_ws_total(pb, pr);
  if (!ws || ws_bytes < need) return fail(MRPIE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  if (pr->iterations == 0) return MRPIE_OK;
  hipStream_t s = (hipStream_t)stream;
  Common c{pr->alpha_obj, pr->alpha_probe, pr->beta, pr->gamma, pr->iter_offset, pr->probe_update_start};
  JobRec jb{(float2*)obj, (float2*)probe, pos, intens, (char*)ws, status,
            pb->H, pb->W, pb->N, pb->M, pb->J, pr->iterations};
  float* eo[1] = {err_out};
  if (!pr->subpixel && !pr->refine && !pr->propagator) return run_sweep(c, &jb, 1, eo, s);
  return run_refining_sweep(c, jb, pr, adam, err_out, s);
}

int mrpie_set_tuning(int32_t N, int32_t M, int32_t batched, const mrpie_tuning* t) {
  if (n_index(N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", N);
  if (batched < 0 || batched > 2) return fail(MRPIE_EINVAL, "batched=%d not in {0, 1, 2}", batched);
  if (M < 0 || M > MRPIE_MAX_MODES) return fail(MRPIE_EINVAL, "M=%d not in [0, 8]", M);
  int rc = check_tuning(t);
  if (rc) return rc;
  set_tuning(N, M, batch_class_jobs(batched),
             Tuning{t->rows_radix, t->cols_radix, t->rows_threads, t->lds_sweep, t->cols_width, t->rows_inplace,
                    t->rows_split});
  return MRPIE_OK;
}

int mrpie_get_tuning(int32_t N, int32_t M, int32_t batched, mrpie_tuning* t) {
  if (n_index(N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", N);
  if (batched < 0 || batched > 2) return fail(MRPIE_EINVAL, "batched=%d not in {0, 1, 2}", batched);
  if (M < 1 || M > MRPIE_MAX_MODES) return fail(MRPIE_EINVAL, "M=%d not in [1, 8]", M);
  if (!t) return fail(MRPIE_EINVAL, "tuning is NULL");
  const Tuning u = get_tuning(N, M, batch_class_jobs(batched));
  t->rows_radix = u.rows_radix;
  t->cols_radix = u.cols_radix;
  t->rows_threads = u.rows_threads;
  t->lds_sweep = u.lds_sweep;
  t->cols_width = u.cols_width;
  t->rows_inplace = u.rows_inplace;
  t->rows_split = u.rows_split;
  return MRPIE_OK;
}

int mrpie_rpie_batched(int32_t njobs, const mrpie_job* jobs, const mrpie_params* pr, const mrpie_tuning* tuning,
                       void* stream) {
  if (njobs < 0) return fail(MRPIE_EINVAL, "njobs=%d < 0", njobs);
  if (tuning) {
    int rc = check_tuning(tuning);
    if (rc) return rc;
  }
  if (njobs == 0) return MRPIE_OK;
  if (!jobs || !pr) return fail(MRPIE_EINVAL, "null jobs or params");
  if (pr->subpixel || pr->refine || pr->propagator)
    return fail(MRPIE_EUNSUPPORTED, "batched sweeps take integer crops, no refinement and the far field "
                                    "(subpixel=%d refine=%d propagator=%d)", pr->subpixel, pr->refine, pr->propagator);
  std::vector<JobRec> recs((size_t)njobs);
  std::vector<float*> errs((size_t)njobs);
  for (int b = 0; b < njobs; ++b) {
    const mrpie_job& j = jobs[b];
    int rc = mrpie_validate(&j.problem, pr);
    if (rc) return fail(rc, "job %d: %s", b, mrpie_last_error());
    if (!j.obj || !j.probe || !j.pos || !j.intens) return fail(MRPIE_EINVAL, "job %d: null array pointer", b);
    const WsLayout L = ws_layout(j.problem.N, j.problem.M, pr->iterations);
    if (!j.ws || j.ws_bytes < L.total)
      return fail(MRPIE_EWORKSPACE, "job %d: workspace %zu < %zu bytes", b, j.ws_bytes, L.total);
    recs[b] = JobRec{(float2*)j.obj, (float2*)j.probe, j.pos, j.intens, (char*)j.ws, j.status,
                     j.problem.H, j.problem.W, j.problem.N, j.problem.M, j.problem.J, pr->iterations};
    errs[b] = j.err_out;
  }
  if (pr->iterations == 0) return MRPIE_OK;
  Common c{pr->alpha_obj, pr->alpha_probe, pr->beta, pr->gamma, pr->iter_offset, pr->probe_update_start};
  Tuning tu{};
  if (tuning)
    tu = Tuning{tuning->rows_radix, tuning->cols_radix, tuning->rows_threads, tuning->lds_sweep, tuning->cols_width,
                tuning->rows_inplace, tuning->rows_split};
  return run_sweep(c, recs.data(), njobs, errs.data(), (hipStream_t)stream, tuning ? &tu : nullptr);
}

}  // extern "C"
