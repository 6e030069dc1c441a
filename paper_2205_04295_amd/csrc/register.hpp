// Registration / Adam interfaces shared by the registration entry point and
// the refining sweep.
#pragma once
#include "common.hpp"
#include "sweep.hpp"

namespace mrpie {

constexpr int kRegChunk = 256;  // pairs registered per pass over the workspace

struct RegArgs {
  int B, U, c, up, norm;
  const float2* ref;   // [B][N][N]
  const float2* mov;   // [B][N][N]
  double2* work;       // [chunk][2][N][N]
  double2* K;          // [U][N]
  double2* T;          // [chunk][U][N]
  double* rowmax_v;    // [chunk][N]
  long long* rowmax_i; // [chunk][N]
  int* s0;             // [chunk][2]
  double* tile_v;      // [chunk][tiles]
  long long* tile_i;   // [chunk][tiles]
  float* shift;        // [B][2]
  int32_t* peak;       // [B][4]
};

struct RegLayout {
  int chunk;
  size_t work, K, T, rowmax_v, rowmax_i, s0, tile_v, tile_i, total;
};

RegLayout reg_layout(int N, int B, int up);
int reg_window(int up, int* U, int* c);
int run_register(int N, int B, const float2* ref, const float2* mov, int up, int norm, float* shift, int32_t* peak,
                 void* ws, size_t ws_bytes, hipStream_t s);
int launch_adam(int J, float* pos, float* adam, const float* g, int t, const mrpie_params* pr, int ymax, int xmax,
                hipStream_t s);

}  // namespace mrpie
