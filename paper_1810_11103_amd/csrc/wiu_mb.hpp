// Index frames of block sides for multi-block grids (host and device).
//
// Sides: 0 x low, 1 x high, 2 y low, 3 y high.  Along side s a node has a
// position t, counted counterclockwise around its block, and a depth d
// inward (0 on the side).  Two right-handed blocks meet with their
// counterclockwise orders opposed: position t of one side is position
// n - 1 - t of the other, and the ghost layer m >= 1 of one block is the
// node layer m - 1 of the other.
#pragma once

#include "wenoiu.h"
#include "wiu_device.hpp"

namespace wiu {

__host__ __device__ inline int mb_side_len(int s, int nx, int ny) { return s < 2 ? ny : nx; }

// node (a, c) at (t, d) along side s of an nx x ny block
__host__ __device__ inline void mb_side_node(int s, int nx, int ny, int t, int d, int& a, int& c) {
  if (s == 0) { a = d; c = ny - 1 - t; }
  else if (s == 1) { a = nx - 1 - d; c = t; }
  else if (s == 2) { a = t; c = d; }
  else { a = nx - 1 - t; c = ny - 1 - d; }
}

// (t, d) along side s of position (a, c)
__host__ __device__ inline void mb_side_frame(int s, int nx, int ny, int a, int c, int& t, int& d) {
  if (s == 0) { t = ny - 1 - c; d = a; }
  else if (s == 1) { t = c; d = nx - 1 - a; }
  else if (s == 2) { t = a; d = c; }
  else { t = nx - 1 - a; d = ny - 1 - c; }
}

// Position (a, c) beyond side s of an nx x ny block as the position
// (a2, c2) of the neighbour (nx2 x ny2) across its side s2.
__host__ __device__ inline void mb_through(int s, int nx, int ny, int s2, int nx2, int ny2, int a, int c, int& a2,
                                           int& c2) {
  int t, d;
  mb_side_frame(s, nx, ny, a, c, t, d);
  mb_side_node(s2, nx2, ny2, mb_side_len(s, nx, ny) - 1 - t, -d - 1, a2, c2);
}

// Coordinate source of one block for the coupled metrics (device table).
struct MbCoord {
  int nx, ny, bcx, bcy;
  double Lx, Ly;
  long long offX;       // x at X_all + offX, y right after
  int side[4], nbr[4], nbr_side[4];
  double shift[4][2];
};

// Host: whether a block set obeys the rules stated with wiu_block (also
// for blocks without interfaces), and the dimensions of one block.
bool mb_blocks_ok(const wiu_block* blocks, int n);
Dims mb_dims(const wiu_block& b);

}  // namespace wiu
