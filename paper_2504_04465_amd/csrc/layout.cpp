// layout.cpp -- brick placement of a built grid and the exception rows of
// the cells whose pull sources the brick arithmetic does not give.
#include "layout.h"

#include <algorithm>
#include <cstring>

namespace lbm {

namespace {

inline int64_t floordiv(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

struct LevelBricks {
  int32_t lo[3] = {0, 0, 0}, n[3] = {1, 1, 1};  // brick bounding box
  std::vector<int32_t> rank;                     // dense over the box, -1 if absent
  int64_t lin(int64_t x, int64_t y, int64_t z) const {
    return (x - lo[0]) + (int64_t)n[0] * ((y - lo[1]) + (int64_t)n[1] * (z - lo[2]));
  }
  int32_t find(int64_t x, int64_t y, int64_t z) const {
    if (x < lo[0] || y < lo[1] || z < lo[2] || x >= lo[0] + n[0] || y >= lo[1] + n[1] || z >= lo[2] + n[2])
      return -1;
    return rank[lin(x, y, z)];
  }
};

}  // namespace

int build_layout(const HostGrid &g, const LatticeInfo &lat, const bool periodic[3], DeviceLayout *out,
                 std::string *err) {
  DeviceLayout &y = *out;
  y = DeviceLayout();
  const int D = g.D, Qm = g.Q - 1;
  y.D = D;
  y.sh = D == 3 ? 2 : 3;
  y.bs = 1 << y.sh;
  y.nb = D == 3 ? 27 : 9;
  y.nbp = D == 3 ? 32 : 16;
  if (lat.B > y.bs) {
    if (err) *err = "lattice reach exceeds the brick edge";
    return -1;
  }
  const int sh = y.sh, bs = y.bs;
  const int64_t n = g.n;
  y.slot_of.assign(n, -1);
  std::vector<LevelBricks> lb(g.L);
  std::vector<std::vector<int32_t>> bxyz(g.L);  // brick coordinates per rank
  int64_t slots = 0;
  for (int l = 0; l < g.L; ++l) {
    y.soff[l] = slots;
    const int64_t c0 = g.off[l], c1 = g.off[l + 1];
    LevelBricks &B = lb[l];
    if (c1 > c0) {
      int32_t mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
      for (int64_t c = c0; c < c1; ++c)
        for (int a = 0; a < 3; ++a) {
          const int32_t v = a < D ? (g.xyz[3 * c + a] >> sh) : 0;
          mn[a] = std::min(mn[a], v);
          mx[a] = std::max(mx[a], v);
        }
      for (int a = 0; a < 3; ++a) {
        B.lo[a] = mn[a];
        B.n[a] = mx[a] - mn[a] + 1;
      }
      B.rank.assign((size_t)B.n[0] * B.n[1] * B.n[2], -1);
    }
    // cells come in Z order, so the cells of one brick are contiguous and
    // bricks appear in the Z order of their coordinates
    int32_t nbk = 0;
    int64_t prev = -1;
    for (int64_t c = c0; c < c1; ++c) {
      const int32_t x = g.xyz[3 * c], yy = g.xyz[3 * c + 1], z = D == 3 ? g.xyz[3 * c + 2] : 0;
      const int64_t k = B.lin(x >> sh, yy >> sh, D == 3 ? (z >> sh) : 0);
      if (k != prev) {
        if (B.rank[k] >= 0) {
          if (err) *err = "cells of a brick are not contiguous in the level order";
          return -1;
        }
        B.rank[k] = nbk++;
        bxyz[l].push_back(x >> sh);
        bxyz[l].push_back(yy >> sh);
        bxyz[l].push_back(D == 3 ? (z >> sh) : 0);
        prev = k;
      }
      const int loc = brick_local(D, sh, x & (bs - 1), yy & (bs - 1), z & (bs - 1));
      y.slot_of[c] = (int32_t)(slots + (int64_t)B.rank[k] * 64 + loc);
    }
    slots += (int64_t)nbk * 64;
  }
  y.soff[g.L] = slots;
  y.nslot = slots;
  if (slots >= INT32_MAX / 2) {
    if (err) *err = "grid too large for 32-bit slot indices";
    return -1;
  }
  y.cell_of.assign(slots, -1);
  for (int64_t c = 0; c < n; ++c) y.cell_of[y.slot_of[c]] = (int32_t)c;
  const int64_t nbrk = slots / 64;
  // neighbour bricks, with periodic wrap where the level extent is a whole
  // number of bricks (otherwise the cells at the wrap use exception rows)
  y.nbrick.assign((size_t)nbrk * y.nbp, -1);
  for (int l = 0; l < g.L; ++l) {
    const int64_t b0 = y.soff[l] / 64;
    const int64_t nbk = (y.soff[l + 1] - y.soff[l]) / 64;
    int64_t eb[3];
    bool wrap[3];
    for (int a = 0; a < 3; ++a) {
      const int64_t e = a < D ? ((int64_t)g.ext[a] << l) : 1;
      wrap[a] = a < D && periodic[a] && e % bs == 0;
      eb[a] = a < D ? e / bs : 1;
    }
    for (int64_t r = 0; r < nbk; ++r) {
      const int64_t bx = bxyz[l][3 * r], by = bxyz[l][3 * r + 1], bz = bxyz[l][3 * r + 2];
      for (int dir = 0; dir < y.nb; ++dir) {
        int64_t q[3] = {bx + dir % 3 - 1, by + (dir / 3) % 3 - 1, D == 3 ? bz + dir / 9 - 1 : 0};
        for (int a = 0; a < D; ++a)
          if (wrap[a]) q[a] = ((q[a] % eb[a]) + eb[a]) % eb[a];
        const int32_t rk = lb[l].find(q[0], q[1], q[2]);
        y.nbrick[(size_t)(b0 + r) * y.nbp + dir] = rk < 0 ? -1 : (int32_t)(b0 + rk);
      }
    }
  }
  // which cells need an exception row
  const uint8_t explicit_flags = F_COARSE_GHOST | F_FINE_GHOST | F_BC_NEUMANN | F_BC_EQ;
  std::vector<uint8_t> special(n, 0);
  for (size_t k = 0; k < g.child.size(); ++k)
    if (g.child[k] >= 0) special[g.child[k]] = 1;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < n; ++c) {
    if (special[c] || (g.flag[c] & explicit_flags)) {
      special[c] = 1;
      continue;
    }
    const int32_t x = g.xyz[3 * c], yy = g.xyz[3 * c + 1], z = D == 3 ? g.xyz[3 * c + 2] : 0;
    const int32_t lc[3] = {x & (bs - 1), yy & (bs - 1), z & (bs - 1)};
    const int64_t brick = y.slot_of[c] / 64;
    bool ok = true;
    for (int i = 1; i <= Qm && ok; ++i) {
      const int32_t s = g.nbr[(size_t)(i - 1) * n + c];
      if (s < 0) {
        ok = false;
        break;
      }
      int dir = 0, pw = 1;
      int32_t q[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a) {
        if (a < D) {
          const int64_t p = lc[a] - lat.c[i][a];
          const int64_t w = floordiv(p, bs);
          q[a] = (int32_t)(p - w * bs);
          dir += (int)(w + 1) * pw;
          pw *= 3;
        }
      }
      const int32_t nbid = y.nbrick[(size_t)brick * y.nbp + dir];
      if (nbid < 0) {
        ok = false;
        break;
      }
      const int64_t slot = (int64_t)nbid * 64 + brick_local(D, sh, q[0], q[1], q[2]);
      if (slot != y.slot_of[s]) ok = false;
    }
    special[c] = ok ? 0 : 1;
  }
  // exception rows: brick masks, prefix bases, rows in brick order
  y.xmask.assign(nbrk, 0ull);
  y.xbase.assign(nbrk, 0);
  y.xrow_of.assign(n, -1);
  for (int64_t c = 0; c < n; ++c)
    if (special[c]) {
      const int64_t s = y.slot_of[c];
      y.xmask[s / 64] |= 1ull << (s & 63);
    }
  int64_t rows = 0;
  for (int64_t b = 0; b < nbrk; ++b) {
    y.xbase[b] = (int32_t)rows;
    rows += __builtin_popcountll(y.xmask[b]);
  }
  y.nx = rows;
  y.xstride = std::max<int64_t>(64, ((rows + 63) / 64) * 64);
  std::vector<int32_t> gidx(n, -1);
  for (size_t k = 0; k < g.ghost_cell.size(); ++k) gidx[g.ghost_cell[k]] = (int32_t)k;
  y.xnbr.assign((size_t)Qm * y.xstride, -1);
  const int64_t vbase = y.nslot;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < n; ++c) {
    if (!special[c]) continue;
    const int64_t s = y.slot_of[c], b = s / 64;
    const uint64_t below = (s & 63) ? (y.xmask[b] & ((1ull << (s & 63)) - 1)) : 0ull;
    const int64_t row = y.xbase[b] + __builtin_popcountll(below);
    y.xrow_of[c] = (int32_t)row;
    for (int i = 0; i < Qm; ++i) {
      const int32_t v = g.nbr[(size_t)i * n + c];
      int32_t o;
      // a coarse ghost reads its coalesced slot for every population the
      // coarse level does not supply: no source, or another coarse ghost
      if (v >= 0) o = (gidx[c] >= 0 && gidx[v] >= 0) ? (int32_t)(vbase + gidx[c]) : y.slot_of[v];
      else if (v == NBR_NONE) o = gidx[c] >= 0 ? (int32_t)(vbase + gidx[c]) : (int32_t)s;
      else if (v == NBR_SOLID) o = -1;
      else o = -2 - (-3 - v);
      y.xnbr[(size_t)i * y.xstride + row] = o;
    }
  }
  return 0;
}

void regular_pulls(const DeviceLayout &y, const LatticeInfo &lat, std::vector<uint64_t> *out) {
  const int D = y.D, sh = y.sh, bs = y.bs, Qm = lat.Q - 1;
  const int64_t nbrk = (int64_t)y.xmask.size();
  out->assign((size_t)std::max<int64_t>(y.nx, 1), 0ull);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t b = 0; b < nbrk; ++b) {
    int64_t row = y.xbase[b];
    for (uint64_t m = y.xmask[b]; m; m &= m - 1, ++row) {
      const int lane = __builtin_ctzll(m);
      int lc[3] = {0, 0, 0};
      for (int k = 0; k < sh; ++k)
        for (int a = 0; a < D; ++a) lc[a] |= ((lane >> (D * k + a)) & 1) << k;
      uint64_t bits = 0;
      for (int i = 1; i <= Qm; ++i) {
        int dir = 0, pw = 1, q[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
          const int64_t p = lc[a] - lat.c[i][a];
          const int64_t w = floordiv(p, bs);
          q[a] = (int)(p - w * bs);
          dir += (int)(w + 1) * pw;
          pw *= 3;
        }
        const int32_t nb = y.nbrick[(size_t)b * y.nbp + dir];
        if (nb >= 0 && (int64_t)y.xnbr[(size_t)(i - 1) * y.xstride + row] ==
                           (int64_t)nb * 64 + brick_local(D, sh, q[0], q[1], q[2]))
          bits |= 1ull << i;
      }
      (*out)[row] = bits;
    }
  }
}

}  // namespace lbm
