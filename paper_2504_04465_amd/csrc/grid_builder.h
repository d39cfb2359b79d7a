// grid_builder.h -- host construction of the static refined grid (Secs. 4.3
// and 4.4 of the paper): level-grouped, Z-order cells, flags, pull neighbour
// list, coarse-ghost list with child table and unknown populations, boundary
// layers and sponge strength.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "lattice.h"

namespace lbm {

enum NodeFlag : uint8_t {
  F_COARSE_GHOST = 1,
  F_FINE_GHOST = 2,
  F_BC_NEUMANN = 4,
  F_BC_EQ = 8,
  F_SPONGE = 16,
  F_MOVING = 32,  // device copy only: a population comes from a moving wall
  F_HOLE = 64,    // device copy only: a slot of a brick without a cell
};

enum { NBR_NONE = -1, NBR_SOLID = -2 };  // moving wall on face k: -3 - k
enum { BC_PERIODIC = 0, BC_WALL = 1, BC_MOVING_WALL = 2, BC_NEUMANN = 3, BC_EQUILIBRIUM = 4 };

struct MaskView {
  const uint8_t *data = nullptr;
  int32_t lo[3] = {0, 0, 0};
  int32_t n[3] = {0, 0, 0};
  uint8_t at(int32_t x, int32_t y, int32_t z) const {
    if (!data) return 0;
    const int64_t a = (int64_t)x - lo[0], b = (int64_t)y - lo[1], c = (int64_t)z - lo[2];
    if (a < 0 || b < 0 || c < 0 || a >= n[0] || b >= n[1] || c >= n[2]) return 0;
    return data[a + (int64_t)n[0] * (b + (int64_t)n[1] * c)];
  }
};

struct FaceSpec {
  int kind;
  double rho, u[3], T;
  int extrapolate_rho;
  double sponge_sigma_max, sponge_width;
};

struct HostGrid {
  int D = 0, L = 0, Q = 0, B = 0;
  int32_t ext[3] = {1, 1, 1};
  int64_t n = 0;
  int64_t off[9] = {0};              // level l owns cells [off[l], off[l+1])
  std::vector<int32_t> xyz;          // [n][3]
  std::vector<int8_t> lev;           // [n]
  std::vector<uint8_t> flag;         // [n]
  std::vector<int32_t> nbr;          // canonical values, SoA [Q-1][n]
  std::vector<int32_t> ghost_cell;   // coarse ghosts, canonical order
  int64_t goff[9] = {0};             // ghosts of level l: [goff[l], goff[l+1])
  std::vector<int32_t> child;        // [n_ghost][2^D]
  std::vector<uint64_t> unknown;     // [n_ghost] bit i: population i coalesced
  std::vector<int32_t> bc_cell;      // boundary-layer cells, canonical order
  std::vector<int32_t> bc_src;       // their source cells
  std::vector<int8_t> bc_face;       // face whose values apply
  int64_t boff[9] = {0};             // boundary cells of level l
  std::vector<int32_t> bc_src_all;   // [n], -1 for cells outside boundary layers
  std::vector<double> sigma;         // [n] sponge strength (empty if none)
  std::vector<double> rho_inf;       // [n] sponge target density
};

// Returns 0, -1 (argument error) or -2 (mask error); *err receives the text.
int build_grid(const LatticeInfo &lat, int dim, const int32_t ext[3], int L,
               const MaskView *refine, const MaskView *solid, const FaceSpec faces[6],
               HostGrid *out, std::string *err);

}  // namespace lbm
