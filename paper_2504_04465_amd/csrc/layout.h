// layout.h -- device layout of a built grid: cells of each level are placed
// in bricks of 64 cells (4x4x4 in 3-D, 8x8 in 2-D) so that one wavefront
// updates one brick.  Within a level, bricks follow the Z order of their
// coordinates and cells the Z order inside the brick, which is the level's Z
// order with the holes of partly filled bricks left as unused slots.
//
// A cell whose every pull source is the same-level cell at x - xi_i, inside
// its own brick or one of the 3^D - 1 bricks around it, is a *bulk* cell: its
// sources follow from the brick's neighbour table and its position in the
// brick, and no per-cell neighbour list is read.  Every other cell (coarse
// and fine ghosts, boundary layers, cells next to walls or solid bodies, or
// sources across a periodic wrap the brick arithmetic does not reproduce)
// keeps an explicit row of pull sources, an *exception row*.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "grid_builder.h"
#include "lattice.h"

namespace lbm {

struct DeviceLayout {
  int D = 0, sh = 0, bs = 0;          // brick edge bs = 1 << sh
  int nb = 0, nbp = 0;                // 3^D neighbour bricks (incl. itself), row length
  int64_t nslot = 0;                  // total slots, a multiple of 64
  int64_t soff[9] = {0};              // level l owns slots [soff[l], soff[l+1])
  std::vector<int32_t> slot_of;       // [n cells] slot of a canonical cell
  std::vector<int32_t> cell_of;       // [nslot] canonical cell, or -1 for a hole
  std::vector<int32_t> nbrick;        // [nslot / 64][nbp] brick id (slot / 64), or -1
  std::vector<uint64_t> xmask;        // [nslot / 64] lanes that use an exception row
  std::vector<int32_t> xbase;         // [nslot / 64] first exception row of the brick
  std::vector<int32_t> xrow_of;       // [n cells] exception row of a cell, or -1
  int64_t nx = 0, xstride = 0;        // exception rows and row stride (multiple of 64)
  // pull sources of the exception rows, SoA [Q-1][xstride], over slots:
  //   >= vbase: coalesced slot of a coarse ghost, >= 0: a slot of the same
  //   level (the cell's own slot where it keeps its value), -1 bounce-back,
  //   -2 - k moving wall of face k; vbase = nslot
  std::vector<int32_t> xnbr;
};

// Per exception row, bit i set where population i pulls from the slot the
// bulk gather's brick arithmetic gives (the neighbour brick of its direction,
// at the local coordinates wrapped into it): a two-buffer pull takes that
// address for the row's cell and reads the explicit source of the others only.
void regular_pulls(const DeviceLayout &y, const LatticeInfo &lat, std::vector<uint64_t> *out);

// periodic[a]: axis a wraps.  Returns 0 or -1 (*err set).
int build_layout(const HostGrid &g, const LatticeInfo &lat, const bool periodic[3], DeviceLayout *out,
                 std::string *err);

// Z-order position of local coordinates inside a brick (x in bit 0).
inline int brick_local(int D, int sh, int x, int y, int z) {
  int r = 0;
  for (int b = 0; b < sh; ++b) {
    r |= ((x >> b) & 1) << (D * b);
    r |= ((y >> b) & 1) << (D * b + 1);
    if (D == 3) r |= ((z >> b) & 1) << (D * b + 2);
  }
  return r;
}

}  // namespace lbm
