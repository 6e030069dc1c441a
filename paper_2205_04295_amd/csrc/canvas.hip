// Canvas map of a scan (Results, the sparse-scan figure): the sum over
// positions of the mode-summed probe intensity sum_p |P_p|^2, placed at each
// position's integer box corner floor(pos + 0.5).  It shows how strongly each
// object pixel is illuminated, which decides where a reconstruction can
// recover the object.
//
// k_probe_power writes sum_p |P_p|^2 once; k_canvas gives every output pixel
// one thread, which walks the positions in scan order (corners staged in
// LDS, 256 per round) and adds the probe power at its offset inside every
// box that contains it, in double precision.  No atomics: the sum order is
// the scan order, so the map is deterministic.
#include "sweep.hpp"

namespace mrpie {

__global__ __launch_bounds__(256) void k_probe_power(const float2* __restrict__ P, float* __restrict__ pw, int NN,
                                                     int M) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NN; i += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int p = 0; p < M; ++p) s += cabs2(P[(size_t)p * NN + i]);
    pw[i] = s;
  }
}

// 16 x 16 output pixels per workgroup.
__global__ __launch_bounds__(256) void k_canvas(const float* __restrict__ pw, const float* __restrict__ pos, int J,
                                                int N, int H, int W, float* __restrict__ canvas, int* status) {
  __shared__ int cy[256], cx[256];
  const int x = blockIdx.x * 16 + (threadIdx.x & 15);
  const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
  double acc = 0.0;
  for (int j0 = 0; j0 < J; j0 += 256) {
    const int j = j0 + threadIdx.x;
    __syncthreads();
    if (j < J) {
      // the clamp bit is set once per position, by the first workgroup
      int* st = (blockIdx.x == 0 && blockIdx.y == 0) ? status : nullptr;
      cy[threadIdx.x] = box_corner(pos[2 * j], H - N, st);
      cx[threadIdx.x] = box_corner(pos[2 * j + 1], W - N, st);
    }
    __syncthreads();
    const int n = min(256, J - j0);
    for (int k = 0; k < n; ++k) {
      const int dy = y - cy[k], dx = x - cx[k];
      if ((unsigned)dy < (unsigned)N && (unsigned)dx < (unsigned)N) acc += (double)pw[dy * N + dx];
    }
  }
  if (y < H && x < W) canvas[(size_t)y * W + x] = (float)acc;
}

}  // namespace mrpie

using namespace mrpie;

extern "C" {

int mrpie_canvas_workspace_size(int32_t N, size_t* bytes) {
  if (n_index(N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", N);
  if (!bytes) return fail(MRPIE_EINVAL, "bytes is NULL");
  *bytes = (size_t)N * N * sizeof(float);
  return MRPIE_OK;
}

int mrpie_canvas(const mrpie_problem* pb, const void* probe, const float* pos, float* canvas, int32_t* status,
                 void* ws, size_t ws_bytes, void* stream) {
  if (!pb) return fail(MRPIE_EINVAL, "null problem");
  if (n_index(pb->N) < 0) return fail(MRPIE_EUNSUPPORTED, "N=%d not in {32,64,128,192,256}", pb->N);
  if (pb->M < 1 || pb->M > MRPIE_MAX_MODES) return fail(MRPIE_EINVAL, "M=%d not in [1, 8]", pb->M);
  if (pb->J < 0) return fail(MRPIE_EINVAL, "J=%d < 0", pb->J);
  if (pb->H < pb->N || pb->W < pb->N) return fail(MRPIE_EINVAL, "object %dx%d smaller than the probe %d", pb->H,
                                                  pb->W, pb->N);
  if ((long long)pb->H * pb->W >= (1LL << 31)) return fail(MRPIE_EINVAL, "object too large");
  if (!probe || !canvas || (pb->J > 0 && !pos)) return fail(MRPIE_EINVAL, "null array pointer");
  const size_t need = (size_t)pb->N * pb->N * sizeof(float);
  if (!ws || ws_bytes < need) return fail(MRPIE_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  const int NN = pb->N * pb->N;
  hipLaunchKernelGGL(k_probe_power, dim3((NN + 255) / 256), dim3(256), 0, s, (const float2*)probe, (float*)ws, NN,
                     pb->M);
  hipLaunchKernelGGL(k_canvas, dim3((pb->W + 15) / 16, (pb->H + 15) / 16), dim3(256), 0, s, (const float*)ws, pos,
                     pb->J, pb->N, pb->H, pb->W, canvas, status);
  MRPIE_HIP(hipGetLastError());
  return MRPIE_OK;
}

}  // extern "C"
