// Data structures of the M-rPIE sweep shared by the plain and batched
// drivers (Methods, "M-rPIE algorithm", Eq. 4-7).
#pragma once
#include "common.hpp"

namespace mrpie {

constexpr int kErrSlots = 1024;  // per-iteration error partials (one per wave of each column unit)
constexpr int kMaxJobsPerLaunch = 36;

// Parameters shared by all jobs of one call.
struct Common {
  float alpha_obj, alpha_probe, beta, gamma;
  int iter_offset, probe_update_start;
};

// One reconstruction (job).  `ws` is this job's private workspace.
struct JobRec {
  float2* obj;        // [H][W]
  float2* probe;      // [M][N][N]  (probe buffer 0: the caller's array)
  const float* pos;   // [J][2]
  const float* I;     // [J][N][N]
  char* ws;
  int* status;
  int H, W, N, M, J, T;
  int t0 = 0;         // first tick of the job in its launch lane (batched calls)
};

struct LaunchArgs {
  Common c;
  int njobs;
  JobRec job[kMaxJobsPerLaunch];
};

// Workspace layout of one job; identical on host and device.
struct WsLayout {
  size_t psi[2], patch[2], probe1, pmax[2], omax[2], err, isum, cb, db, total;
};

__host__ __device__ inline size_t ws_align(size_t x) { return (x + 255) & ~size_t(255); }

__host__ __device__ inline WsLayout ws_layout(int N, int M, int T) {
  WsLayout L{};
  const size_t NN = (size_t)N * N;
  size_t off = 0;
#define MRPIE_TAKE(field, bytes) \
  field = off;                   \
  off = ws_align(off + (bytes));
  MRPIE_TAKE(L.psi[0], M * NN * 8)
  MRPIE_TAKE(L.psi[1], M * NN * 8)
  MRPIE_TAKE(L.patch[0], NN * 8)
  MRPIE_TAKE(L.patch[1], NN * 8)
  MRPIE_TAKE(L.probe1, M * NN * 8)
  MRPIE_TAKE(L.pmax[0], (size_t)N * 4)
  MRPIE_TAKE(L.pmax[1], (size_t)N * 4)
  MRPIE_TAKE(L.omax[0], (size_t)N * 4)
  MRPIE_TAKE(L.omax[1], (size_t)N * 4)
  MRPIE_TAKE(L.err, (size_t)(T > 0 ? T : 1) * kErrSlots * 8)
  MRPIE_TAKE(L.isum, (size_t)(T > 0 ? T : 1) * kErrSlots * 8)  // same slots: sums of max(I, 0)
  MRPIE_TAKE(L.cb, NN * 8)   // subpixel path: crop rows moved along x
  MRPIE_TAKE(L.db, NN * 8)   // subpixel path: object update moved back along y
#undef MRPIE_TAKE
  L.total = off;
  return L;
}

// Launch shape of the two sweep passes (chosen per N and batch class).
struct Tuning {
  int rows_radix;    // 4 or 8: FFT plan of the row pass
  int cols_radix;    // 4 or 8: FFT plan of the column pass
  int rows_threads;  // 256 or 512 threads per row workgroup
  int lds_sweep;     // jobs with M <= lds_sweep whose modes fit the LDS run the
                     // one-workgroup sweep (0: never)
  int cols_width;    // 1 or 4 adjacent detector columns per column workgroup
  int rows_inplace;  // 1: multi-job row passes run their inverse FFTs in place
  int rows_split;    // 1: multi-job calls run the update and the gather row
                     // passes as launches of their own (three per position)
};
// The tuning of (N, mode class of M, batch class of nb jobs): the one set
// for it, else the default.  set_tuning with M = 0 sets every mode class.
Tuning get_tuning(int N, int M, int nb);
void set_tuning(int N, int M, int nb, const Tuning& t);
Tuning default_tuning(int N, int nb);
// A job count of call class cls (0: one job, 1: 2-15 jobs, 2: 16 or more).
int batch_class_jobs(int cls);
// validates a caller's tuning (MRPIE_OK or MRPIE_EINVAL with a message)
int check_tuning(const mrpie_tuning* t);

// Subpixel / refining sweep (four launches per position): iterations
// [it0, it0 + iters) of job `jb`; head: the first step has no previous one,
// tail: the last step's update is applied before returning.  `reg_ref`,
// `reg_mov` ([J][N][N] each) receive the patch before and after its update
// from iteration record_start on, when set.
struct SubpixelExtra {
  int subpixel;      // 0: fractions forced to 0 (refinement on integer crops)
  float2* reg_ref;
  float2* reg_mov;
  int record_start;  // absolute iteration from which pairs are recorded
  int xcb = 0;       // 1: XCORR_B pairs (model amplitude, sqrt(I)); 0: XCORR_A (o_j, o'_j)
  float fresnel = 0.f;  // near-field Fresnel number; 0: far field
};
int run_sweep_subpixel(const Common& c, const JobRec& jb, const SubpixelExtra& ex, int it0, int iters, bool head,
                       bool tail, hipStream_t s);
size_t rpie_ws_total(const mrpie_problem* pb, const mrpie_params* pr);
int run_refining_sweep(const Common& c, const JobRec& jb, const mrpie_params* pr, float* adam, float* err_out,
                       hipStream_t s);

// Launch helpers shared by the sweep drivers: clear the per-iteration error
// partials; finish (copy the probe back from the workspace buffer when
// `probe_back`, sum the intensities, write err_out).
void launch_zero_err(const LaunchArgs& a, int nb, hipStream_t s);
void launch_finish(const LaunchArgs& a, int nb, float* const* err_out, hipStream_t s, bool probe_back = true);

// One-workgroup sweep of jobs whose M modes of N x N fit the LDS together
// (M N^2 <= 16384); every job of `jobs` must fit.
bool lds_sweep_fits(int N, int M);
int run_lds_sweep(const Common& c, const JobRec* jobs, int njobs, float* const* err_out, hipStream_t s);

// Host driver: runs `T` iterations (per job) of the sweep for every job in
// `jobs` (any mix of N and M), lock-step by position: tick t performs the
// transition (t-1 -> t) row pass and the column pass of step t of every job
// that has one.  Writes err_out[b][T_b] when err_out[b] != nullptr.
// `force` (may be null) replaces the installed tuning for every launch.
int run_sweep(const Common& c, const JobRec* jobs, int njobs, float* const* err_out, hipStream_t s,
              const Tuning* force = nullptr);

}  // namespace mrpie
