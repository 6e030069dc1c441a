/* mrpie.h — C ABI of the MI355X (gfx950) multi-mode rPIE hot path.
 *
 * Method: Guzzi et al., "A modular software framework for the design and
 * implementation of ptychography algorithms" (SciComPty), arXiv 2205.04295,
 * Methods section: the mixed-state forward model (Eq. 1-4), the M-rPIE
 * object/probe updates (Eq. 5-6) with the modulus-corrected wave (Eq. 7),
 * and the Adam-driven cross-correlation position refinement (Eq. 8-9,
 * Alg. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex arrays are complex64: interleaved (re, im) float pairs,
 *    C-contiguous (last index fastest).  Real arrays are float32.
 *  - Every array argument is DEVICE memory owned by the caller; the library
 *    never allocates, frees or keeps a pointer after the call returns.
 *    Scratch comes from a caller-provided device workspace whose size the
 *    matching *_workspace_size function returns (0 when none is needed).
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the
 *    default stream) and performs no host<->device synchronisation and no
 *    device-memory allocation, so it may be recorded into a HIP graph
 *    (batched calls of two or more jobs also fork work to an internal
 *    stream and join it back before returning control of `stream`, see
 *    mrpie_rpie_batched).
 *  - The object O is [H][W]; probe modes P are [M][N][N]; positions are
 *    [J][2] floats (y, x): the top-left corner of the N x N box in object
 *    pixels; diffraction intensities are [J][N][N] in FFT order (zero
 *    frequency at [0][0], no fftshift).
 *  - The propagator D_z (Eq. 2) is the unitary 2-D DFT (far field) unless
 *    mrpie_params.propagator selects the near-field transfer function.
 *  - Return codes: MRPIE_OK, or a negative MRPIE_E* code for errors found
 *    on the host before anything is launched (then nothing is launched and
 *    mrpie_last_error() gives a message, per calling thread).  Numerical
 *    trouble found on the device while running sets bits in the
 *    caller-provided int32 `status` word (never cleared by the library).
 *  - Calls on distinct workspaces are reentrant.  Calls sharing one
 *    workspace must be ordered on one stream.
 */
#ifndef MRPIE_H
#define MRPIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRPIE_OK 0
#define MRPIE_EINVAL (-1)       /* bad shape, parameter or null pointer */
#define MRPIE_EUNSUPPORTED (-2) /* N not in {32,64,128,192,256} or M > 8 */
#define MRPIE_EDEVICE (-3)      /* HIP runtime error (message in mrpie_last_error) */
#define MRPIE_EWORKSPACE (-4)   /* workspace missing or too small */

/* device status bits (OR-ed into *status) */
#define MRPIE_STATUS_NONFINITE 1   /* a NaN/Inf reached the object, probe or error */
#define MRPIE_STATUS_POS_CLAMPED 2 /* a box corner was outside [0,H-N]x[0,W-N]
                                      (or not finite) and was clamped */

#define MRPIE_MAX_MODES 8

/* Problem shape.  H, W: object rows / columns; N: probe side (32, 64, 128,
 * 192 or 256); M: number of mutually incoherent probe modes (1..8, Eq. 4);
 * J: number of scan positions. */
typedef struct {
  int32_t H, W, N, M, J;
} mrpie_problem;

/* Reconstruction parameters.
 *  alpha_obj, alpha_probe : step sizes alpha_O, alpha_P (Eq. 6, Eq. 5)
 *  beta  : probe-denominator weight, beta |o_j|^2_max + (1-beta)|o_j|^2
 *          (Eq. 5), in [0, 1]
 *  gamma : object-denominator weight, gamma (sum_p|P_p|^2)_max +
 *          (1-gamma) sum_p|P_p|^2 (Eq. 6), in [0, 1].
 *          beta = gamma = 1 is M-ePIE.
 *  iterations : number of sweeps over all positions, in scan order
 *  iter_offset: absolute index of the first iteration (resume); it drives
 *          probe_update_start, refine_start and Adam's step counter
 *  probe_update_start: the probe is updated only in iterations >= this
 *  subpixel : 0 = crop at the nearest integer corner floor(pos + 0.5);
 *          1 = also move the crop by the fractional part with a Fourier
 *          phase ramp and move the object update back by the same amount
 *  refine : 1 = XCORR_A position refinement (register o_j against the
 *          updated o'_j, Adam step per position, Eq. 8-9 and Alg. 1) in
 *          iterations >= refine_start
 *  upsample : registration upsampling factor (window ceil(1.5 up) samples)
 *  xcorr_norm: 0 = plain cross-power spectrum (the default reading for
 *          refinement: the paper says it follows the SciPy-ecosystem
 *          implementation of Guizar-Sicairos et al., and the plain
 *          cross-power is the one that moves the positions on the
 *          refinement workload), 1 = phase-normalised (the paper's phrase
 *          "weighted phase correlation" admits both)
 *  adam_lr, adam_b1, adam_b2, adam_eps : Adam hyper-parameters
 *  xcorr_point : where refinement compares (Methods, "Adam-based position
 *          refinement", the XCORR_A / XCORR_B switch): 0 = XCORR_A, the
 *          patch o_j against its update o'_j; 1 = XCORR_B, the modelled
 *          detector amplitude sqrt(sum_p |D_z(P_p o_j)|^2) (before the
 *          modulus replacement) against the measured sqrt(I_j)
 *  propagator : D_z of Eq. 2.  0 = far field, the unitary 2-D DFT
 *          (intensities in FFT order); 1 = near field, the paraxial Fresnel
 *          transfer function D_z = F^-1 H F with H(k) = exp(-i pi (k_y^2 +
 *          k_x^2) / fresnel) on the signed integer frequencies of the N x N
 *          window and D_{-z} = F^-1 conj(H) F (intensities in detector-pixel
 *          order)
 *  fresnel : Fresnel number (N delta)^2 / (lambda z) of the N x N window,
 *          > 0 when propagator = 1 (ignored otherwise)                    */
typedef struct {
  float alpha_obj, alpha_probe, beta, gamma;
  int32_t iterations, iter_offset, probe_update_start;
  int32_t subpixel;
  int32_t refine, refine_start, upsample, xcorr_norm;
  float adam_lr, adam_b1, adam_b2, adam_eps;
  int32_t xcorr_point, propagator;
  float fresnel;
} mrpie_params;

/* Library version string (static storage). */
const char* mrpie_version(void);

/* Message for the last error returned on the calling thread ("" if none). */
const char* mrpie_last_error(void);

/* Host-only check of a problem and parameter set (no GPU needed).
 * Returns MRPIE_OK, MRPIE_EINVAL or MRPIE_EUNSUPPORTED. */
int mrpie_validate(const mrpie_problem* pb, const mrpie_params* pr);

/* Bytes of device workspace mrpie_rpie needs for (pb, pr); host-only. */
int mrpie_workspace_size(const mrpie_problem* pb, const mrpie_params* pr, size_t* bytes);

/* The sequential M-rPIE sweep (Methods, "M-rPIE algorithm"; Eq. 4-7, with
 * Eq. 8-9 / Alg. 1 when pr->refine = 1).
 *
 * For it in [0, iterations) and j in [0, J) in order: gather o_j from obj at
 * pos[j]; form psi_p = P_p o_j for every mode; Psi_p = D_z psi_p; replace
 * the mode-summed modulus by sqrt(intens[j]) (zero where the model is 0;
 * intensities are clamped at 0); psi'_p = D_{-z} Psi'_p; update the probe
 * (Eq. 5) and the object box (Eq. 6) simultaneously from the pre-update
 * o_j and P_p.
 *
 *  obj    [H][W]    complex64, in/out
 *  probe  [M][N][N] complex64, in/out
 *  pos    [J][2]    float32, in (in/out when refine = 1)
 *  adam   [J][4]    float32 (m_y, m_x, v_y, v_x), in/out when refine = 1,
 *                   may be NULL otherwise
 *  intens [J][N][N] float32, in
 *  err_out[iterations] float32, out: sum_j sum (|Psi| - sqrt(I))^2 /
 *                   sum_j sum I for each iteration (may be NULL)
 *  status int32, OR-ed with MRPIE_STATUS_* bits (may be NULL)
 *  ws, ws_bytes     workspace of at least mrpie_workspace_size bytes
 * The result is deterministic: the same inputs give bitwise equal outputs.
 * With refine = 1 each iteration's sweep records every position's pair
 * (XCORR_A: the patch before and after its update; XCORR_B: the modelled
 * and the measured detector amplitude), then all J pairs are registered
 * and the Adam step is taken, in order on `stream`.  Subpixel moves,
 * refinement and the near-field propagator run the four-launch position
 * step; the plain far-field sweep runs two launches per position (or one
 * workgroup per job for probes whose modes fit the LDS).  No device memory
 * is allocated. */
int mrpie_rpie(const mrpie_problem* pb, const mrpie_params* pr, void* obj, void* probe,
               float* pos, float* adam, const float* intens, float* err_out, int32_t* status,
               void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sweep as mrpie_rpie, same arguments and results, but without a caller
 * workspace.  Its scratch is a static device array of the library of
 * MRPIE_NOALLOC_MAX_BYTES (16 MiB) per GPU, held by every GPU the library
 * runs on until the process ends; its device address is looked up once per
 * device (with that device current) on the first call there.  Problems
 * whose mrpie_workspace_size exceeds MRPIE_NOALLOC_MAX_BYTES are refused
 * with MRPIE_EWORKSPACE before anything is launched (256^2 probes: up to 8
 * modes for up to 100 iterations per call, 3 modes for up to ~550).  No
 * device memory is allocated or freed, by the library or any library it
 * calls.  The current device must be the one `stream` belongs to.  All
 * calls on one GPU share its array, which keeps the last call's contents
 * (the sweep writes every scratch value before reading it): calls ordered
 * on one stream are safe, calls that overlap on one GPU (two streams, two
 * host threads) race and give undefined results. */
#define MRPIE_NOALLOC_MAX_BYTES ((size_t)16 << 20)
int mrpie_rpie_noalloc(const mrpie_problem* pb, const mrpie_params* pr, void* obj, void* probe,
                       float* pos, float* adam, const float* intens, float* err_out, int32_t* status,
                       void* stream);

/* One reconstruction of a batch: its shape, its arrays (device memory, as
 * for mrpie_rpie) and its own workspace (mrpie_workspace_size bytes for its
 * problem and the shared parameters). */
typedef struct {
  mrpie_problem problem;
  void* obj;            /* [H][W] complex64, in/out */
  void* probe;          /* [M][N][N] complex64, in/out */
  float* pos;           /* [J][2] float32, in */
  const float* intens;  /* [J][N][N] float32, in */
  float* err_out;       /* [iterations] float32, out (may be NULL) */
  int32_t* status;      /* int32 status word (may be NULL) */
  void* ws;
  size_t ws_bytes;
} mrpie_job;

/* Launch shape of the sweep's passes, per probe size N, mode class of M
 * (M = 1, 2, 3-4, 5-8) and call class (batched = 0: single-job mrpie_rpie;
 * 1: mrpie_rpie_batched with 2 to 15 jobs; 2: with 16 or more jobs).
 * rows_radix / cols_radix: 4 or 8, the radix of the LDS Stockham FFT
 * stages of the row / column pass (radix 4: more threads per transform,
 * shorter latency; radix 8: fewer stages, less LDS traffic); rows_threads:
 * 256 or 512 threads per row workgroup; lds_sweep in [0, 8]: a job with
 * M <= lds_sweep whose modes fit the LDS together (M N^2 <= 16384: 32^2
 * with up to 8 modes, 64^2 with up to 4, 128^2 with 1) runs as one
 * workgroup that keeps the probe in registers and the 2-D FFT in LDS for
 * the whole call; other jobs run the row / column passes (default for
 * single-job calls: 8 for N = 32, 1 for N = 64, 0 otherwise; 0 in batches,
 * where small jobs ride along in the shared launches); cols_width: 1 or 4 adjacent detector
 * columns per column-pass workgroup (1: shortest latency for a single
 * sweep; 4: coalesced 32-byte row segments, for batches); rows_inplace: 1
 * runs the inverse row FFTs of multi-job launches in place (half the row
 * pass's LDS: more workgroups per CU, one more barrier per FFT stage), and
 * the column FFTs too in calls of 16 or more jobs (with cols_width 4); 0
 * ping-pongs two buffers; rows_split: 1 makes multi-job calls run the row
 * work of a position as two launches, the update of the previous position
 * (inverse row FFTs, Eq. 5 and Eq. 6, the probe updated in place) and the
 * gather of the next (exit waves, forward row FFTs), so every row of the
 * previous spectra is transformed once and no patch copy is kept (three
 * launches per position, less memory traffic); 0 fuses them into one row
 * pass (two launches per position; single-job calls always fuse).  The
 * installed setting is process-wide host state (guarded by a lock); results
 * do not depend on it beyond float rounding.  mrpie_autotune times the candidates on the device and installs
 * the fastest.  mrpie_set_tuning with M = 0 sets every mode class of
 * (N, batched); mrpie_get_tuning takes M in [1, 8]. */
typedef struct {
  int32_t rows_radix, cols_radix, rows_threads, lds_sweep, cols_width, rows_inplace, rows_split;
} mrpie_tuning;
int mrpie_set_tuning(int32_t N, int32_t M, int32_t batched, const mrpie_tuning* t);
int mrpie_get_tuning(int32_t N, int32_t M, int32_t batched, mrpie_tuning* t);

/* Batched M-rPIE: runs mrpie_rpie's sweep (same parameters for every job;
 * refine, subpixel and propagator must be 0, else MRPIE_EUNSUPPORTED) on
 * `njobs` independent reconstructions of any mix of N, M, J and object
 * size, lock-step by position: every launch advances one position of every
 * running job, so one pair of launches carries the work of many jobs.  The
 * jobs of a stream run in at most 36 launch lanes (the job table of one
 * launch); a share of more than 36 jobs is dealt to the lanes longest job
 * first, and a job starts once the job ahead of it in its lane has taken
 * its last step.  Jobs run concurrently, so they must not share object,
 * probe, workspace or error-curve memory (positions and intensities are
 * only read and may be shared; so may status words).
 * Each job's object and probe match those of a mrpie_rpie call on that job
 * alone to float rounding (the single-job column pass keeps its first and
 * last FFT stages in registers; jobs that run the one-workgroup LDS sweep in
 * both are bitwise equal); the error curve may differ in the summation
 * order of its partial sums.  With two or more jobs, every second job runs
 * on an internal non-blocking stream (default priority; the first such call
 * on a device creates it and 16 events, kept until the process ends),
 * forked from `stream` and joined back into it before the call returns, so
 * two lock-step launch sequences share the GPU (jobs whose modes fit the
 * LDS run their one-workgroup sweep there too); while `stream` is being
 * captured into a graph, all launches stay on `stream`.  `jobs` is a HOST
 * array read during the call.  `tuning` (may be NULL) sets the launch shape
 * of every launch of this call; NULL uses the installed tuning of each
 * launch group's (N, mode class, batch class).  Each job brings its own
 * workspace (jobs of different shapes need different sizes) and its own
 * status word (jobs may share one). */
int mrpie_rpie_batched(int32_t njobs, const mrpie_job* jobs, const mrpie_params* pr, const mrpie_tuning* tuning,
                       void* stream);

/* Autotuner of the launch shapes for probe size N, the mode class of M and
 * the call class of `batch` jobs (1: single mrpie_rpie calls; 2-15 and
 * 16 or more: the two classes of mrpie_rpie_batched calls).  mrpie_autotune fills its workspace with `batch`
 * synthetic problems of shape (N, M, J positions along a Fermat spiral with
 * about 70 % overlap between consecutive probes, object 3N x 3N), runs one
 * sweep iteration with every candidate (mrpie_tuning_candidates lists them,
 * in order) in reps + 1 round-robin rounds on `stream` (the first round warms
 * up), timed with HIP events, keeps each candidate's fastest timed run,
 * installs the best
 * candidate for that (N, mode class, batch class) as mrpie_set_tuning
 * would, and returns it in *best (may be NULL).  cand_ms (may be NULL)
 * receives each candidate's time in ms.  The call waits on the host for its
 * timing events, so it may not be captured into a graph; it allocates no
 * device memory (workspace: mrpie_autotune_workspace_size bytes, reps in
 * [1, 100]).  mrpie_tuning_candidates writes up to `cap` candidates to
 * `out` (may be NULL) and returns their number (or a negative error). */
int mrpie_tuning_candidates(int32_t N, int32_t M, int32_t batched, mrpie_tuning* out, int32_t cap);
int mrpie_autotune_workspace_size(int32_t N, int32_t M, int32_t batch, int32_t J, size_t* bytes);
int mrpie_autotune(int32_t N, int32_t M, int32_t batch, int32_t J, int32_t reps, void* ws, size_t ws_bytes,
                   mrpie_tuning* best, float* cand_ms, void* stream);

/* Test hook: in-place unitary 2-D DFT (D_z, Eq. 2; inverse = 1 gives
 * D_{-z}) of B contiguous N x N complex64 arrays.  N in {32,64,128,192,256}. */
int mrpie_fft2(int32_t N, int32_t B, void* data, int32_t inverse, void* stream);

/* Test hook: in-place modulus replacement of Eq. 7 on M detector-plane
 * modes Psi [M][N][N] (unitary scale) with intensity I [N][N]:
 * Psi_p <- sqrt(max(I,0)) / sqrt(sum_n |Psi_n|^2) * Psi_p, 0 where the sum
 * is 0. */
int mrpie_modulus(int32_t N, int32_t M, void* psi, const float* intens, void* stream);

/* Subpixel registration of B pairs of N x N complex64 patches (Methods,
 * "Adam-based position refinement": 2-D phase correlation after
 * Guizar-Sicairos et al. 2008 with the matrix-multiply DFT evaluated only
 * around the coarse peak, no zero-padding).
 *  ref, mov [B][N][N] complex64 device arrays (pairs b = ref[b], mov[b])
 *  upsample : up >= 1; window U = ceil(1.5 up) samples per axis at spacing
 *             1/up, centred (index floor(U/2)) on the integer peak
 *  norm     : 0 = plain cross-power F(ref) conj(F(mov)); 1 = divided by its
 *             modulus (zero where the modulus is zero)
 *  shift [B][2] float32 out: (y, x) with mov(r) ~ ref(r + shift)
 *  peak  [B][4] int32 out: coarse argmax (row, col) of |F^-1 X| in FFT
 *             order (lags above N/2 are negative) and window argmax (u, v);
 *             ties go to the first maximum in row-major order
 * Computed in double precision throughout.  Workspace:
 * mrpie_register_workspace_size(N, B, upsample). */
int mrpie_register_workspace_size(int32_t N, int32_t B, int32_t upsample, size_t* bytes);
int mrpie_register(int32_t N, int32_t B, const void* ref, const void* mov, int32_t upsample, int32_t norm,
                   float* shift, int32_t* peak, void* ws, size_t ws_bytes, void* stream);

/* Modified Adam step of Alg. 1 for J positions (one reconstruction
 * iteration t >= 1): g [J][2] is the measured shift (the gradient);
 * adam [J][4] = (m_y, m_x, v_y, v_x) in/out; pos [J][2] in/out moves by
 * +adam_lr * mhat / (sqrt(vhat) + adam_eps) per axis (Eq. 8-9) and is
 * clamped to [0, ymax] x [0, xmax] (ymax = H - N, xmax = W - N). */
int mrpie_adam(int32_t J, const mrpie_params* pr, int32_t ymax, int32_t xmax, float* pos, float* adam,
               const float* g, int32_t t, void* stream);

/* Amplitude loss of the mixed-state forward model (Eq. 4, with the crop of
 * box j moved by the fractional position when subpixel = 1) and its
 * hand-written adjoint.
 *   L = sum_j sum_k (A_j(k) - sqrt(max(I_j(k), 0)))^2,
 *   A_j = sqrt(sum_p |D_z(P_p o_j)|^2),  o_j = S_f(crop of obj at pos[j])
 * mrpie_loss writes L (double, device) to loss_out.  mrpie_adjoint also
 * writes (overwriting) the gradients of L w.r.t. the object grad_obj [H][W]
 * and the probe modes grad_probe [M][N][N] (complex64, dL/dRe + i dL/dIm),
 * and w.r.t. the positions grad_pos [J][2] float32 through the Fourier
 * shift (zero when subpixel = 0; the integer corner is piecewise constant).
 * loss_out may be NULL for mrpie_adjoint.  Exit waves are recomputed, not
 * stored; overlapping boxes and the probe sum are reduced in position order
 * (deterministic).  Workspace: mrpie_grad_workspace_size. */
int mrpie_grad_workspace_size(const mrpie_problem* pb, size_t* bytes);
int mrpie_loss(const mrpie_problem* pb, int32_t subpixel, const void* obj, const void* probe, const float* pos,
               const float* intens, double* loss_out, int32_t* status, void* ws, size_t ws_bytes, void* stream);
int mrpie_adjoint(const mrpie_problem* pb, int32_t subpixel, const void* obj, const void* probe, const float* pos,
                  const float* intens, double* loss_out, void* grad_obj, void* grad_probe, float* grad_pos,
                  int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Canvas map of a scan (Results, the sparse-scan figure): canvas [H][W]
 * float32 (out, overwritten) = sum over positions j of the mode-summed
 * probe intensity sum_p |P_p|^2 (probe [M][N][N] complex64) placed at box
 * corner floor(pos[j] + 0.5) (pos [J][2] float32), i.e. how strongly each
 * object pixel is illuminated.  Corners outside [0, H-N] x [0, W-N] are
 * clamped and flagged in *status (may be NULL), as in the sweep.  Summed
 * in double precision in scan order (deterministic).  Workspace:
 * mrpie_canvas_workspace_size(N) bytes (the probe power map). */
int mrpie_canvas_workspace_size(int32_t N, size_t* bytes);
int mrpie_canvas(const mrpie_problem* pb, const void* probe, const float* pos, float* canvas, int32_t* status,
                 void* ws, size_t ws_bytes, void* stream);

/* Diagnostic kernel timing (not for use under graph capture).
 * mrpie_timing_enable(stride): from now on, every stride-th launch of each
 * timed kernel class is launched with a start / stop event pair of its own
 * dispatch (hipExtLaunchKernelGGL) on the stream it is launched on (stride
 * = 0 switches timing off).  Classes: 0 = sweep row pass (k_rows, k_rows1),
 * 1 = sweep column pass (k_cols, k_cols1), 2 = registration column pass
 * (k_reg_cols), 3 = registration window GEMM (k_reg_gemm1), 4 = adjoint
 * modulus pass (k_adj_p3), 5 = one-workgroup LDS sweep (k_lds_sweep),
 * 6 = split update pass (k_upd), 7 = split gather pass (k_gat).
 * The events are created without the system-scope fence, which would
 * otherwise write the L2 back inside the timed dispatch.
 * mrpie_timing_read(avg_ms[nkinds], count[nkinds], avg_units[nkinds],
 * nkinds): waits for the recorded events, returns the mean duration, the
 * number of timed launches and the mean number of units those launches
 * process (jobs per sweep pass, positions per adjoint pass, pairs per
 * registration pass;
 * avg_units may be NULL) per class, and clears the record.  Host-side
 * state, one per process. */
int mrpie_timing_enable(int32_t stride);
int mrpie_timing_read(double* avg_ms, int64_t* count, double* avg_units, int32_t nkinds);

#ifdef __cplusplus
}
#endif
#endif /* MRPIE_H */
