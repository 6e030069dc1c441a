// Loss / adjoint interfaces.
#pragma once
#include "common.hpp"
#include "sweep.hpp"

namespace mrpie {

constexpr int kAdjChunk = 256;  // positions processed per pass

struct AdjArgs {
  int H, W, N, M, J, subpixel, j0, nb;  // nb: positions in the current chunk
  const float2* obj;
  const float2* probe;
  const float* pos;
  const float* I;
  int* status;
  float2* Cp;          // [chunk][N][N] crop spectra -> o
  float2* Fo;          // [chunk][N][N] F(o), unnormalised
  float2* G;           // [chunk][N][N] g -> S_{-f}(g)
  float2* Psi;         // [chunk][M][N][N] Psi -> chi; slot of each group's first
                       // position -> the group's probe-gradient partial
  double* loss_part;   // [chunk][N]
  double* pos_part;    // [chunk][N][2]
  double* loss_blk;    // [kLossBlocks] partial sums of loss_part
  double* loss_acc;
  float2* grad_obj;
  float2* grad_probe;
  float* grad_pos;
};

struct AdjLayout {
  int chunk;
  size_t Cp, Fo, G, Psi, loss_part, pos_part, loss_blk, loss_acc, total;
};

AdjLayout adj_layout(int N, int M, int J);

}  // namespace mrpie
