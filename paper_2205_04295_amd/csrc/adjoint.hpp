// Loss / adjoint interfaces.
#pragma once
#include "common.hpp"
#include "sweep.hpp"

namespace mrpie {

constexpr int kAdjChunk = 256;  // positions processed per pass
constexpr int kPosSlots = 5;    // position-gradient partials per (position, row or column)

struct AdjArgs {
  int H, W, N, M, J, subpixel, j0, nb;  // nb: positions in the current chunk
  const float2* obj;
  const float2* probe;
  const float* pos;
  const float* I;
  int* status;
  float2* Cp;          // [chunk][N][N] S_y(crop): the crop moved along y
  float2* Ob;          // [chunk][N][N] o = S_x(S_y(crop))
  float2* G;           // [chunk][N][N] S_{-x}(g) -> S_{-f}(g)
  float2* Psi;         // [chunk][M][N][N] row spectra of the exit waves -> row
                       // spectra of chi; slot of each group's first position
                       // -> the group's probe-gradient partial
  double* loss_part;   // [chunk][N]: the mode pass's partial of each wave, in the
                       // slot of its column group's column of the same index
  double* pos_part;    // [chunk][N][kPosSlots]: [b][u][0] y part per column
                       // group (first column's slot), [b][r][1 + w] x part
                       // of row r from wave w
  double* loss_blk;    // [kLossBlocks] partial sums of loss_part
  double* loss_acc;
  float2* grad_obj;
  float2* grad_probe;
  float* grad_pos;
};

struct AdjLayout {
  int chunk;
  size_t Cp, Ob, G, Psi, loss_part, pos_part, loss_blk, loss_acc, total;
};

AdjLayout adj_layout(int N, int M, int J);

}  // namespace mrpie
