// grid_device.hip -- the refined grid (level regions, coarse-ghost strips,
// Z-order cells, flags, pull neighbour list, boundary layers, sponge,
// coarse-ghost tables; Secs. 3.2, 4.3-4.4) and its brick layout, built on
// the GPU.  Every step is the host builder's rule applied per cell in
// parallel; the Z order of a level is a radix sort of the Morton keys of
// its cells, the lists in canonical order are prefix sums over flags, and
// the checks raise bits in an error word read back at the host builder's
// check points, so that both builders report the same error first.
#include "grid_device.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

// the sponge ramp is evaluated in the host builder's operation order
#pragma clang fp contract(off)

namespace lbm {
namespace {

enum : uint8_t { S_INR = 1, S_REF = 2, S_STRIP = 4, S_PRE = 8, S_EXIST = 16 };
enum : int {
  E_NEST = 1, E_IFACE = 2, E_CUT = 4, E_BOTH = 8, E_OVERLAP = 16, E_NOSRC = 32, E_SRCBC = 64, E_ORPHAN = 128,
  E_BRICK = 256
};

constexpr int TPB = 256;

struct DMask {
  const uint8_t *data;
  int32_t lo[3], n[3];
  __device__ uint8_t at(int32_t x, int32_t y, int32_t z) const {
    if (!data) return 0;
    const int64_t a = (int64_t)x - lo[0], b = (int64_t)y - lo[1], c = (int64_t)z - lo[2];
    if (a < 0 || b < 0 || c < 0 || a >= n[0] || b >= n[1] || c >= n[2]) return 0;
    return data[a + (int64_t)n[0] * (b + (int64_t)n[1] * c)];
  }
};

struct DLevel {
  int32_t E[3], lo[3], n[3];
  uint8_t *st;
  int32_t *idx;
  __host__ __device__ int64_t size() const { return (int64_t)n[0] * n[1] * n[2]; }
  __device__ bool inside(int64_t x, int64_t y, int64_t z) const {
    return x >= lo[0] && y >= lo[1] && z >= lo[2] && x < lo[0] + n[0] && y < lo[1] + n[1] && z < lo[2] + n[2];
  }
  __device__ int64_t lin(int64_t x, int64_t y, int64_t z) const {
    return (x - lo[0]) + (int64_t)n[0] * ((y - lo[1]) + (int64_t)n[1] * (z - lo[2]));
  }
  __device__ void coords(int64_t id, int32_t &X, int32_t &Y, int32_t &Z) const {
    X = (int32_t)(id % n[0]) + lo[0];
    Y = (int32_t)((id / n[0]) % n[1]) + lo[1];
    Z = (int32_t)(id / ((int64_t)n[0] * n[1])) + lo[2];
  }
};

struct DGrid {
  DLevel lv[8];
  int L, D, B;
  int32_t ext[3];
  int periodic[3];
};

struct DLat {
  int Q;
  int c[37][3];
};

struct DFaces {
  int kind[6];
  double rho[6], smax[6], width[6];
};

inline unsigned grid_for(int64_t n) {
  const int64_t b = (n + TPB - 1) / TPB;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 20));
}

// for kernels that end in a few atomics on one shared word per wavefront
// (bounding boxes): a grid of at most 2048 blocks, each thread striding over
// more cells, keeps those atomics from queueing behind each other
inline unsigned grid_few(int64_t n) { return std::min<unsigned>(grid_for(n), 2048u); }

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// ---- level regions ---------------------------------------------------------
__global__ void k_state(DLevel v, DLevel p, DMask wp, DMask wr, int l, int L, int D) {
  GRID_STRIDE(id, v.size()) {
    int32_t X, Y, Z;
    v.coords(id, X, Y, Z);
    uint8_t s = 0;
    if (l == 0) {
      s = S_INR;
    } else {
      const int32_t PX = X >> 1, PY = Y >> 1, PZ = D == 3 ? Z >> 1 : 0;
      if ((p.st[p.lin(PX, PY, PZ)] & S_INR) && wp.at(PX, PY, PZ)) s = S_INR;
    }
    if (l + 1 < L && wr.at(X, Y, Z)) s |= S_REF;
    v.st[id] = s;
  }
}

__global__ void k_nest(DLevel v, DMask w, int *err) {
  const int64_t N = (int64_t)w.n[0] * w.n[1] * w.n[2];
  GRID_STRIDE(k, N) {
    if (!w.data[k]) continue;
    const int32_t X = (int32_t)(k % w.n[0]) + w.lo[0];
    const int32_t Y = (int32_t)((k / w.n[0]) % w.n[1]) + w.lo[1];
    const int32_t Z = (int32_t)(k / ((int64_t)w.n[0] * w.n[1])) + w.lo[2];
    if (!v.inside(X, Y, Z) || !(v.st[v.lin(X, Y, Z)] & S_INR)) atomicOr(err, E_NEST);
  }
}

// refined cells within Chebyshev distance B of an unrefined in-domain cell
__global__ void k_strip(DLevel v, DMask w, int D, int B, int3 per) {
  const int RZ = D == 3 ? B : 0;
  const int periodic[3] = {per.x, per.y, per.z};
  GRID_STRIDE(id, v.size()) {
    if (!(v.st[id] & S_REF)) continue;
    int32_t X, Y, Z;
    v.coords(id, X, Y, Z);
    bool hit = false;
    for (int dz = -RZ; dz <= RZ && !hit; ++dz)
      for (int dy = -B; dy <= B && !hit; ++dy)
        for (int dx = -B; dx <= B && !hit; ++dx) {
          int32_t q[3] = {X + dx, Y + dy, Z + dz};
          bool outside = false;
          for (int a = 0; a < D; ++a) {
            if (q[a] >= 0 && q[a] < v.E[a]) continue;
            if (periodic[a]) q[a] = ((q[a] % v.E[a]) + v.E[a]) % v.E[a];
            else outside = true;
          }
          if (!outside && !w.at(q[0], q[1], q[2])) hit = true;
        }
    if (hit) v.st[id] |= S_STRIP;
  }
}

__global__ void k_iface(DLevel v, DLevel p, int D, int *err) {
  GRID_STRIDE(id, v.size()) {
    if (!(v.st[id] & S_REF)) continue;
    int32_t X, Y, Z;
    v.coords(id, X, Y, Z);
    if (p.st[p.lin(X >> 1, Y >> 1, D == 3 ? Z >> 1 : 0)] & S_STRIP) atomicOr(err, E_IFACE);
  }
}

__global__ void k_exist(DLevel v, DMask sv) {
  GRID_STRIDE(id, v.size()) {
    uint8_t s = v.st[id];
    const bool pre = (s & S_INR) && (!(s & S_REF) || (s & S_STRIP));
    if (!pre) continue;
    s |= S_PRE;
    int32_t X, Y, Z;
    v.coords(id, X, Y, Z);
    if (!sv.at(X, Y, Z)) s |= S_EXIST;
    v.st[id] = s;
  }
}

__global__ void k_cut(DLevel v, DLevel f, int D, int *err) {
  const int NCH = 1 << D;
  GRID_STRIDE(id, v.size()) {
    if (!(v.st[id] & S_STRIP)) continue;
    int32_t X, Y, Z;
    v.coords(id, X, Y, Z);
    int nf = 0;
    for (int o = 0; o < NCH; ++o) {
      const int32_t cx = 2 * X + (o & 1), cy = 2 * Y + ((o >> 1) & 1), cz = D == 3 ? 2 * Z + ((o >> 2) & 1) : 0;
      if (f.inside(cx, cy, cz) && (f.st[f.lin(cx, cy, cz)] & S_EXIST)) ++nf;
    }
    const bool fluid = (v.st[id] & S_EXIST) != 0;
    if (fluid ? nf == 0 : nf != 0) atomicOr(err, E_CUT);
  }
}

// ---- canonical order ---------------------------------------------------------
__global__ void k_flag_exist(DLevel v, int32_t *fl) {
  GRID_STRIDE(id, v.size()) fl[id] = (v.st[id] & S_EXIST) ? 1 : 0;
}

// Morton key of absolute coordinates, x in the lowest bit of each group:
// the order of the recursive subdivision of the level's root cube
__device__ inline uint64_t morton(int D, int bits, uint32_t x, uint32_t y, uint32_t z) {
  uint64_t k = 0;
  for (int b = 0; b < bits; ++b) {
    k |= (uint64_t)((x >> b) & 1u) << (D * b);
    k |= (uint64_t)((y >> b) & 1u) << (D * b + 1);
    if (D == 3) k |= (uint64_t)((z >> b) & 1u) << (D * b + 2);
  }
  return k;
}

__global__ void k_keys(DLevel v, int D, int bits, const int32_t *fl, const int32_t *pos, uint64_t *keys,
                       int32_t *ids) {
  GRID_STRIDE(id, v.size()) {
    if (!fl[id]) continue;
    int32_t X, Y, Z;
    v.coords(id, X, Y, Z);
    keys[pos[id]] = morton(D, bits, (uint32_t)X, (uint32_t)Y, (uint32_t)Z);
    ids[pos[id]] = (int32_t)id;
  }
}

__global__ void k_place(DLevel v, const int32_t *ids, int64_t cnt, int64_t base, int l, int32_t *xyz, int8_t *lev) {
  GRID_STRIDE(k, cnt) {
    const int64_t id = ids[k], c = base + k;
    int32_t X, Y, Z;
    v.coords(id, X, Y, Z);
    xyz[3 * c] = X;
    xyz[3 * c + 1] = Y;
    xyz[3 * c + 2] = Z;
    lev[c] = (int8_t)l;
    v.idx[id] = (int32_t)c;
  }
}

// ---- flags, neighbour list, boundary layers, sponge --------------------------
__global__ void k_flags(DGrid G, int64_t n, const int32_t *xyz, const int8_t *lev, uint8_t *flag, int *err) {
  const int D = G.D;
  GRID_STRIDE(c, n) {
    const int l = lev[c];
    const int32_t X = xyz[3 * c], Y = xyz[3 * c + 1], Z = xyz[3 * c + 2];
    uint8_t fl = 0;
    const DLevel &v = G.lv[l];
    if (v.st[v.lin(X, Y, Z)] & S_STRIP) fl |= F_COARSE_GHOST;
    if (l > 0) {
      const DLevel &p = G.lv[l - 1];
      if (p.st[p.lin(X >> 1, Y >> 1, D == 3 ? Z >> 1 : 0)] & S_STRIP) fl |= F_FINE_GHOST;
    }
    if ((fl & (F_COARSE_GHOST | F_FINE_GHOST)) == (F_COARSE_GHOST | F_FINE_GHOST)) atomicOr(err, E_BOTH);
    flag[c] = fl;
  }
}

__global__ void k_nbr(DGrid G, DLat lat, DFaces F, int64_t n, const int32_t *xyz, const int8_t *lev, int32_t *nbr) {
  const int D = G.D;
  GRID_STRIDE(c, n) {
    const DLevel &v = G.lv[lev[c]];
    for (int i = 1; i < lat.Q; ++i) {
      int32_t q[3];
      int nout = 0, outf[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a) {
        q[a] = xyz[3 * c + a] - lat.c[i][a];
        if (a >= D) continue;
        if (q[a] >= 0 && q[a] < v.E[a]) continue;
        if (G.periodic[a]) q[a] = ((q[a] % v.E[a]) + v.E[a]) % v.E[a];
        else outf[nout++] = 2 * a + (q[a] >= v.E[a] ? 1 : 0);
      }
      int32_t val = NBR_NONE;
      if (nout > 0) {
        bool wall = false;
        int mov = -1;
        for (int k = 0; k < nout; ++k) {
          const int kind = F.kind[outf[k]];
          if (kind == BC_WALL) wall = true;
          if (kind == BC_MOVING_WALL && mov < 0) mov = outf[k];
        }
        val = wall ? NBR_SOLID : (mov >= 0 ? -3 - mov : NBR_NONE);
      } else if (v.inside(q[0], q[1], q[2])) {
        const int64_t id = v.lin(q[0], q[1], q[2]);
        if (v.st[id] & S_EXIST) val = v.idx[id];
        else if (v.st[id] & S_PRE) val = NBR_SOLID;
      }
      nbr[(int64_t)(i - 1) * n + c] = val;
    }
  }
}

__global__ void k_bc(DGrid G, DFaces F, int64_t n, const int32_t *xyz, const int8_t *lev, uint8_t *flag,
                     int32_t *src_all, int8_t *bcf, int *err) {
  const int D = G.D, B = G.B;
  GRID_STRIDE(c, n) {
    const int l = lev[c];
    const DLevel &v = G.lv[l];
    int32_t src[3] = {xyz[3 * c], xyz[3 * c + 1], xyz[3 * c + 2]};
    int eqf = -1, nef = -1;
    for (int fc = 0; fc < 2 * D; ++fc) {
      const int kind = F.kind[fc], a = fc / 2;
      if (kind != BC_NEUMANN && kind != BC_EQUILIBRIUM) continue;
      const int32_t E = v.E[a], x = xyz[3 * c + a];
      const bool in = (fc & 1) ? x >= E - B : x < B;
      if (!in) continue;
      src[a] = (fc & 1) ? E - 1 - B : B;
      if (kind == BC_EQUILIBRIUM && eqf < 0) eqf = fc;
      if (kind == BC_NEUMANN && nef < 0) nef = fc;
    }
    src_all[c] = -1;
    bcf[c] = -1;
    if (eqf < 0 && nef < 0) continue;
    if (flag[c] & (F_COARSE_GHOST | F_FINE_GHOST)) {
      atomicOr(err, E_OVERLAP);
      continue;
    }
    int32_t sid = -1;
    if (v.inside(src[0], src[1], src[2])) sid = v.idx[v.lin(src[0], src[1], src[2])];
    if (sid < 0) {
      atomicOr(err, E_NOSRC);
      continue;
    }
    src_all[c] = sid;
    bcf[c] = (int8_t)(eqf >= 0 ? eqf : nef);
    flag[c] |= eqf >= 0 ? F_BC_EQ : F_BC_NEUMANN;
  }
}

__global__ void k_bc_check(int64_t n, int Qm, const uint8_t *flag, const int32_t *src_all, const int32_t *nbr,
                           int *err) {
  GRID_STRIDE(c, n) {
    const int32_t s = src_all[c];
    if (s >= 0 && (flag[s] & (F_BC_EQ | F_BC_NEUMANN))) atomicOr(err, E_SRCBC);
    if (flag[c] & (F_COARSE_GHOST | F_FINE_GHOST | F_BC_EQ | F_BC_NEUMANN)) continue;
    for (int i = 0; i < Qm; ++i)
      if (nbr[(int64_t)i * n + c] == NBR_NONE) atomicOr(err, E_ORPHAN);
  }
}

__global__ void k_sponge(DGrid G, DFaces F, int64_t n, const int32_t *xyz, const int8_t *lev, uint8_t *flag,
                         double *sigma, double *rho_inf) {
  const int D = G.D;
  GRID_STRIDE(c, n) {
    const int l = lev[c];
    double best = 0.0, rinf = 1.0;
    for (int fc = 0; fc < 2 * D; ++fc) {
      if (F.kind[fc] == BC_PERIODIC || F.smax[fc] <= 0.0 || F.width[fc] <= 0.0) continue;
      const int a = fc / 2;
      const double centre = (xyz[3 * c + a] + 0.5) / (double)(1 << l);
      const double dist = (fc & 1) ? G.ext[a] - centre : centre;
      const double r0 = 1.0 - dist / F.width[fc];
      const double r1 = 0.0 < r0 ? r0 : 0.0;  // max(0, .), first argument on ties
      const double ramp = r1 < 1.0 ? r1 : 1.0;  // min(1, .)
      const double s = F.smax[fc] * ramp;
      if (s > best) {
        best = s;
        rinf = F.rho[fc];
      }
    }
    sigma[c] = best;
    rho_inf[c] = rinf;
    if (best > 0.0) flag[c] |= F_SPONGE;
  }
}

// ---- lists in canonical order --------------------------------------------------
__global__ void k_flag_bits(int64_t n, const uint8_t *flag, uint8_t bits, int32_t *out) {
  GRID_STRIDE(c, n) out[c] = (flag[c] & bits) ? 1 : 0;
}
__global__ void k_flag_nonneg(int64_t n, const int32_t *v, int32_t *out) {
  GRID_STRIDE(c, n) out[c] = v[c] >= 0 ? 1 : 0;
}
__global__ void k_scatter_list(int64_t n, const int32_t *fl, const int32_t *pos, int32_t *list) {
  GRID_STRIDE(c, n) if (fl[c]) list[pos[c]] = (int32_t)c;
}
__global__ void k_bc_list(int64_t nb, const int32_t *cells, const int32_t *src_all, const int8_t *bcf,
                          int32_t *src, int8_t *face) {
  GRID_STRIDE(k, nb) {
    const int32_t c = cells[k];
    src[k] = src_all[c];
    face[k] = bcf[c];
  }
}

__global__ void k_child_unknown(DGrid G, int Q, int64_t ng, int64_t n, const int32_t *ghost, const int32_t *xyz,
                                const int8_t *lev, const int32_t *nbr, const uint8_t *flag, int32_t *child,
                                uint64_t *unknown) {
  const int D = G.D, NCH = 1 << D;
  GRID_STRIDE(k, ng) {
    const int64_t c = ghost[k];
    const DLevel &f = G.lv[lev[c] + 1];
    for (int o = 0; o < NCH; ++o) {
      const int32_t X = 2 * xyz[3 * c] + (o & 1), Y = 2 * xyz[3 * c + 1] + ((o >> 1) & 1);
      const int32_t Z = D == 3 ? 2 * xyz[3 * c + 2] + ((o >> 2) & 1) : 0;
      child[k * NCH + o] = f.inside(X, Y, Z) ? f.idx[f.lin(X, Y, Z)] : -1;
    }
    uint64_t m = 0;
    for (int i = 1; i < Q; ++i) {
      const int32_t v = nbr[(int64_t)(i - 1) * n + c];
      if (v == NBR_NONE || (v >= 0 && (flag[v] & F_COARSE_GHOST))) m |= (uint64_t)1 << i;
    }
    unknown[k] = m;
  }
}

// ---- brick layout ----------------------------------------------------------------
__device__ inline int brick_local_d(int D, int sh, int x, int y, int z) {
  int r = 0;
  for (int b = 0; b < sh; ++b) {
    r |= ((x >> b) & 1) << (D * b);
    r |= ((y >> b) & 1) << (D * b + 1);
    if (D == 3) r |= ((z >> b) & 1) << (D * b + 2);
  }
  return r;
}

// 1 where a cell starts a brick (cells of a level come in Z order), and the
// level's brick bounding box
// min and max of v over the wavefront, then one atomic per wavefront: a
// device-wide bounding box without every thread queueing on six words
__device__ inline void bbox_add(int *bbox, const int32_t (&lo)[3], const int32_t (&hi)[3]) {
  int32_t m[6] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      m[a] = min(m[a], __shfl_xor(m[a], o));
      m[3 + a] = max(m[3 + a], __shfl_xor(m[3 + a], o));
    }
  if ((threadIdx.x & 63) == 0 && m[0] <= m[3])
    for (int a = 0; a < 3; ++a) {
      atomicMin(&bbox[a], m[a]);
      atomicMax(&bbox[3 + a], m[3 + a]);
    }
}

__global__ void k_brick_start(int64_t c0, int64_t cnt, int D, int sh, const int32_t *xyz, int32_t *start,
                              int *bbox) {
  int32_t lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  GRID_STRIDE(k, cnt) {
    const int64_t c = c0 + k;
    int32_t b[3];
    for (int a = 0; a < 3; ++a) b[a] = a < D ? (xyz[3 * c + a] >> sh) : 0;
    bool s = k == 0;
    if (!s)
      for (int a = 0; a < 3; ++a)
        if ((a < D ? (xyz[3 * (c - 1) + a] >> sh) : 0) != b[a]) s = true;
    start[k] = s ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
      lo[a] = min(lo[a], b[a]);
      hi[a] = max(hi[a], b[a]);
    }
  }
  bbox_add(bbox, lo, hi);
}

struct DBricks {
  int32_t lo[3], n[3];
  int32_t *rank;
  __device__ int32_t find(int64_t x, int64_t y, int64_t z) const {
    if (x < lo[0] || y < lo[1] || z < lo[2] || x >= lo[0] + n[0] || y >= lo[1] + n[1] || z >= lo[2] + n[2])
      return -1;
    return rank[(x - lo[0]) + (int64_t)n[0] * ((y - lo[1]) + (int64_t)n[1] * (z - lo[2]))];
  }
};

__global__ void k_brick_rank(DBricks B, int64_t c0, int64_t cnt, int64_t b0, int D, int sh, const int32_t *xyz,
                             const int32_t *start, const int32_t *rk, int32_t *bxyz, int *err) {
  GRID_STRIDE(k, cnt) {
    if (!start[k]) continue;
    const int64_t c = c0 + k;
    int32_t b[3];
    for (int a = 0; a < 3; ++a) b[a] = a < D ? (xyz[3 * c + a] >> sh) : 0;
    const int64_t li = (b[0] - B.lo[0]) + (int64_t)B.n[0] * ((b[1] - B.lo[1]) + (int64_t)B.n[1] * (b[2] - B.lo[2]));
    if (atomicCAS(&B.rank[li], -1, rk[k]) != -1) atomicOr(err, E_BRICK);
    for (int a = 0; a < 3; ++a) bxyz[3 * (b0 + rk[k]) + a] = b[a];
  }
}

__global__ void k_slot(int64_t c0, int64_t cnt, int64_t s0, int D, int sh, const int32_t *xyz,
                       const int32_t *start, const int32_t *rk, int32_t *slot_of) {
  const int bs = 1 << sh;
  GRID_STRIDE(k, cnt) {
    const int64_t c = c0 + k;
    const int64_t r = rk[k] + start[k] - 1;
    const int loc = brick_local_d(D, sh, xyz[3 * c] & (bs - 1), xyz[3 * c + 1] & (bs - 1),
                                  D == 3 ? (xyz[3 * c + 2] & (bs - 1)) : 0);
    slot_of[c] = (int32_t)(s0 + r * 64 + loc);
  }
}

__global__ void k_cell_of(int64_t n, const int32_t *slot_of, int32_t *cell_of) {
  GRID_STRIDE(c, n) cell_of[slot_of[c]] = (int32_t)c;
}

__global__ void k_nbrick(DBricks B, int64_t nbk, int64_t b0, int D, int nb, int nbp, int3 wrap, int3 eb,
                         const int32_t *bxyz, int32_t *nbrick) {
  const int w[3] = {wrap.x, wrap.y, wrap.z};
  const int64_t e[3] = {eb.x, eb.y, eb.z};
  GRID_STRIDE(r, nbk) {
    const int64_t bx = bxyz[3 * (b0 + r)], by = bxyz[3 * (b0 + r) + 1], bz = bxyz[3 * (b0 + r) + 2];
    for (int dir = 0; dir < nb; ++dir) {
      int64_t q[3] = {bx + dir % 3 - 1, by + (dir / 3) % 3 - 1, D == 3 ? bz + dir / 9 - 1 : 0};
      for (int a = 0; a < D; ++a)
        if (w[a]) q[a] = ((q[a] % e[a]) + e[a]) % e[a];
      const int32_t rk = B.find(q[0], q[1], q[2]);
      nbrick[(b0 + r) * nbp + dir] = rk < 0 ? -1 : (int32_t)(b0 + rk);
    }
  }
}

__global__ void k_mark_children(int64_t nc, const int32_t *child, uint8_t *special) {
  GRID_STRIDE(k, nc) if (child[k] >= 0) special[child[k]] = 1;
}

__device__ inline int64_t floordiv_d(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// cells whose pull sources the brick arithmetic does not give
__global__ void k_special(DLat lat, int64_t n, int D, int sh, int nbp, const int32_t *xyz, const uint8_t *flag,
                          const int32_t *nbr, const int32_t *slot_of, const int32_t *nbrick, uint8_t *special) {
  const int bs = 1 << sh;
  const uint8_t explicit_flags = F_COARSE_GHOST | F_FINE_GHOST | F_BC_NEUMANN | F_BC_EQ;
  GRID_STRIDE(c, n) {
    if (special[c] || (flag[c] & explicit_flags)) {
      special[c] = 1;
      continue;
    }
    const int32_t lc[3] = {xyz[3 * c] & (bs - 1), xyz[3 * c + 1] & (bs - 1), D == 3 ? (xyz[3 * c + 2] & (bs - 1)) : 0};
    const int64_t brick = slot_of[c] / 64;
    bool ok = true;
    for (int i = 1; i < lat.Q && ok; ++i) {
      const int32_t s = nbr[(int64_t)(i - 1) * n + c];
      if (s < 0) {
        ok = false;
        break;
      }
      int dir = 0, pw = 1;
      int32_t q[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a) {
        if (a < D) {
          const int64_t p = lc[a] - lat.c[i][a];
          const int64_t w = floordiv_d(p, bs);
          q[a] = (int32_t)(p - w * bs);
          dir += (int)(w + 1) * pw;
          pw *= 3;
        }
      }
      const int32_t nbid = nbrick[brick * nbp + dir];
      if (nbid < 0) {
        ok = false;
        break;
      }
      const int64_t slot = (int64_t)nbid * 64 + brick_local_d(D, sh, q[0], q[1], q[2]);
      if (slot != slot_of[s]) ok = false;
    }
    special[c] = ok ? 0 : 1;
  }
}

__global__ void k_xmask(int64_t n, const uint8_t *special, const int32_t *slot_of, unsigned long long *xmask) {
  GRID_STRIDE(c, n) {
    if (!special[c]) continue;
    const int64_t s = slot_of[c];
    atomicOr(&xmask[s / 64], 1ull << (s & 63));
  }
}

__global__ void k_popc(int64_t nb, const unsigned long long *xmask, int32_t *cnt) {
  GRID_STRIDE(b, nb) cnt[b] = __popcll(xmask[b]);
}

__global__ void k_gidx(int64_t ng, const int32_t *ghost, int32_t *gidx) {
  GRID_STRIDE(k, ng) gidx[ghost[k]] = (int32_t)k;
}

__global__ void k_xrows(int64_t n, int Qm, int64_t xstride, int64_t vbase, const uint8_t *special,
                        const int32_t *slot_of, const unsigned long long *xmask, const int32_t *xbase,
                        const int32_t *nbr, const int32_t *gidx, int32_t *xrow_of, int32_t *xnbr) {
  GRID_STRIDE(c, n) {
    if (!special[c]) continue;
    const int64_t s = slot_of[c], b = s / 64;
    const unsigned long long below = (s & 63) ? (xmask[b] & ((1ull << (s & 63)) - 1)) : 0ull;
    const int64_t row = xbase[b] + __popcll(below);
    xrow_of[c] = (int32_t)row;
    for (int i = 0; i < Qm; ++i) {
      const int32_t v = nbr[(int64_t)i * n + c];
      int32_t o;
      if (v >= 0) o = (gidx[c] >= 0 && gidx[v] >= 0) ? (int32_t)(vbase + gidx[c]) : slot_of[v];
      else if (v == NBR_NONE) o = gidx[c] >= 0 ? (int32_t)(vbase + gidx[c]) : (int32_t)s;
      else if (v == NBR_SOLID) o = -1;
      else o = -2 - (-3 - v);
      xnbr[(int64_t)i * xstride + row] = o;
    }
  }
}

// ---- remesh sources ----------------------------------------------------------------
// dense index of the old flow cells of one level over their bounding box
struct DFlow {
  int32_t lo[3], n[3];
  int32_t *map;
  __device__ int32_t find(int64_t x, int64_t y, int64_t z) const {
    if (!map || x < lo[0] || y < lo[1] || z < lo[2] || x >= lo[0] + n[0] || y >= lo[1] + n[1] ||
        z >= lo[2] + n[2])
      return -1;
    return map[(x - lo[0]) + (int64_t)n[0] * ((y - lo[1]) + (int64_t)n[1] * (z - lo[2]))];
  }
};
struct DFlows {
  DFlow lv[8];
  int L, D, deepest;
};

// the cells of a level are contiguous: one launch per level, [c0, c0 + cnt)
__global__ void k_flow_bbox(int64_t c0, int64_t cnt, const int32_t *xyz, const uint8_t *flag, int *bbox) {
  int32_t lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  GRID_STRIDE(k, cnt) {
    const int64_t c = c0 + k;
    if (flag[c] & F_FINE_GHOST) continue;
    for (int a = 0; a < 3; ++a) {
      lo[a] = min(lo[a], xyz[3 * c + a]);
      hi[a] = max(hi[a], xyz[3 * c + a]);
    }
  }
  bbox_add(bbox, lo, hi);
}

__global__ void k_flow_map(DFlows F, int64_t n, const int32_t *xyz, const int8_t *lev, const uint8_t *flag) {
  GRID_STRIDE(c, n) {
    if (flag[c] & F_FINE_GHOST) continue;
    const DFlow &f = F.lv[lev[c]];
    const int64_t x = xyz[3 * c] - f.lo[0], y = xyz[3 * c + 1] - f.lo[1], z = xyz[3 * c + 2] - f.lo[2];
    f.map[x + (int64_t)f.n[0] * (y + (int64_t)f.n[1] * z)] = (int32_t)c;
  }
}

// The sources of one new cell in the host's order: the old cell at the same
// place on the same or a coarser level (weight 1), else the old cells
// inside it, depth first, children with x slowest, weights halved per axis
// and level, then divided by their sum.  MODE 0 counts them (and returns
// the sum through *tot), MODE 1 writes them.
template <int MODE>
__device__ inline int cell_sources(const DFlows &F, int l, int64_t x, int64_t y, int64_t z, double *tot,
                                   int32_t *src, double *wt) {
  for (int up = l; up >= 0; --up) {
    const int s = l - up;
    const int32_t c = F.lv[up].find(x >> s, y >> s, z >> s);
    if (c >= 0) {
      if (MODE == 1) {
        src[0] = c;
        wt[0] = 1.0;
      } else {
        *tot = 1.0;
      }
      return 1;
    }
  }
  struct Fr {
    int l, o;
    int64_t x, y, z;
    double w;
  };
  Fr stk[8];
  int sp = 0, k = 0;
  const int NCH = 1 << F.D;
  double sum = 0.0;
  const double norm = MODE == 1 ? *tot : 1.0;
  if (l < F.deepest) stk[sp++] = Fr{l, 0, x, y, z, 1.0 / (double)NCH};
  while (sp > 0) {
    Fr &f = stk[sp - 1];
    if (f.o == NCH) {
      --sp;
      continue;
    }
    const int o = f.o++;
    const int ox = F.D == 3 ? o >> 2 : o >> 1, oy = F.D == 3 ? (o >> 1) & 1 : o & 1, oz = F.D == 3 ? o & 1 : 0;
    const int64_t cx = 2 * f.x + ox, cy = 2 * f.y + oy, cz = F.D == 3 ? 2 * f.z + oz : 0;
    const int32_t c = F.lv[f.l + 1].find(cx, cy, cz);
    if (c >= 0) {
      if (MODE == 1) {
        src[k] = c;
        wt[k] = f.w / norm;
      }
      sum += f.w;
      ++k;
    } else if (f.l + 1 < F.deepest) {
      const double w = f.w / (double)NCH;
      const int nl = f.l + 1;
      stk[sp++] = Fr{nl, 0, cx, cy, cz, w};
    }
  }
  if (MODE == 0) *tot = sum;
  return k;
}

__global__ void k_src_count(DFlows F, int64_t n, const int32_t *xyz, const int8_t *lev, int64_t *cnt, double *tot,
                            unsigned long long *bad) {
  GRID_STRIDE(j, n) {
    double t = 0.0;
    const int k = cell_sources<0>(F, lev[j], xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2], &t, nullptr, nullptr);
    if (k == 0 || !(t > 0.0)) atomicMin(bad, (unsigned long long)j);
    cnt[j] = k;
    tot[j] = t;
  }
}

__global__ void k_src_fill(DFlows F, int64_t n, const int32_t *xyz, const int8_t *lev, const int64_t *off,
                           const double *tot, int32_t *src, double *wt) {
  GRID_STRIDE(j, n) {
    double t = tot[j];
    cell_sources<1>(F, lev[j], xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2], &t, src + off[j], wt + off[j]);
  }
}

// ---- host side ---------------------------------------------------------------------
struct Pool {
  const DevAlloc &da;
  std::vector<void *> held;
  bool failed = false;
  explicit Pool(const DevAlloc &d) : da(d) {}
  ~Pool() {
    for (void *p : held) da.release(p, da.ctx);
  }
  template <class T>
  T *take(size_t count) {
    void *p = da.alloc(std::max<size_t>(count, 1) * sizeof(T), da.ctx);
    if (!p) failed = true;
    else held.push_back(p);
    return (T *)p;
  }
};

int fail(std::string *err, int code, const char *msg) {
  if (err) *err = msg;
  return code;
}

// exclusive prefix sum of n int32 values (n >= 1); returns the total
hipError_t exclusive_sum(Pool &pool, const int32_t *in, int32_t *out, int64_t n, hipStream_t s, int64_t *total) {
  size_t tb = 0;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, tb, in, out, (int)n, s);
  if (e != hipSuccess) return e;
  void *tmp = pool.take<char>(tb);
  if (!tmp) return hipErrorOutOfMemory;
  if ((e = hipcub::DeviceScan::ExclusiveSum(tmp, tb, in, out, (int)n, s)) != hipSuccess) return e;
  int32_t last[2];
  if ((e = hipMemcpyAsync(&last[0], out + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(&last[1], in + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  *total = (int64_t)last[0] + last[1];
  return hipSuccess;
}

template <class T>
hipError_t down(std::vector<T> &dst, const T *src, size_t count, hipStream_t s) {
  dst.resize(count);
  if (!count) return hipSuccess;
  return hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s);
}

}  // namespace

#define DEV_TRY(x)                                                        \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) return fail(err, -3, hipGetErrorString(e_));    \
  } while (0)
#define DEV_MEM(p)                                                               \
  do {                                                                           \
    if (!(p)) return fail(err, -3, "device grid build: allocation failed");     \
  } while (0)

int build_grid_device(const LatticeInfo &lat, int dim, const int32_t ext_in[3], int L, const MaskView *refine,
                      const MaskView *solid, const FaceSpec faces[6], const bool periodic[3], const DevAlloc &da,
                      hipStream_t st, HostGrid *out, DeviceLayout *yo, DeviceGridArrays *keep, std::string *err) {
  // ---- argument checks, as the host builder makes them ----
  if (dim != lat.D) return fail(err, -1, "dimension does not match the lattice");
  if (L < 1 || L > 8) return fail(err, -1, "level count must be 1..8");
  int32_t ext[3];
  for (int a = 0; a < 3; ++a) {
    ext[a] = a < dim ? ext_in[a] : 1;
    if (ext[a] < 1) return fail(err, -1, "extent must be positive");
    if (a < dim && ((int64_t)ext[a] << (L - 1)) >= (1 << 21))
      return fail(err, -1, "finest extent exceeds 2^21 cells per axis");
  }
  bool per[3];
  for (int a = 0; a < 3; ++a) {
    per[a] = false;
    if (a >= dim) continue;
    const bool p0 = faces[2 * a].kind == BC_PERIODIC, p1 = faces[2 * a + 1].kind == BC_PERIODIC;
    if (p0 != p1) return fail(err, -2, "periodic faces must come in pairs");
    per[a] = p0;
    if (p0 && ext[a] <= lat.B) return fail(err, -1, "periodic extent must exceed the lattice reach");
    for (int s = 0; s < 2; ++s)
      if (faces[2 * a + s].kind < 0 || faces[2 * a + s].kind > 4) return fail(err, -1, "unknown face kind");
  }
  (void)periodic;
  const int D = dim, B = lat.B, Q = lat.Q, Qm = Q - 1, NCH = 1 << D;
  for (int l = 0; l + 1 < L; ++l)
    for (int a = 0; a < 3; ++a) {
      const int64_t E = a < dim ? ((int64_t)ext[a] << l) : 1;
      if (refine[l].data && (refine[l].lo[a] < 0 || refine[l].n[a] < 0 || refine[l].lo[a] + refine[l].n[a] > E))
        return fail(err, -1, "refine mask window outside its level");
    }
  for (int l = 0; solid && l < L; ++l)
    for (int a = 0; a < 3; ++a) {
      const int64_t E = a < dim ? ((int64_t)ext[a] << l) : 1;
      if (solid[l].data && (solid[l].lo[a] < 0 || solid[l].n[a] < 0 || solid[l].lo[a] + solid[l].n[a] > E))
        return fail(err, -1, "solid mask window outside its level");
    }

  Pool pool(da);
  int *derr = pool.take<int>(1);
  DEV_MEM(derr);
  DEV_TRY(hipMemsetAsync(derr, 0, sizeof(int), st));
  auto errors = [&](int *h) -> hipError_t {
    hipError_t e = hipMemcpyAsync(h, derr, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
  };
  const unsigned T = TPB;

  // masks on the device
  auto upload_mask = [&](const MaskView &m, DMask *dm) -> int {
    dm->data = nullptr;
    for (int a = 0; a < 3; ++a) {
      dm->lo[a] = m.lo[a];
      dm->n[a] = m.n[a];
    }
    if (!m.data) return 0;
    const size_t bytes = (size_t)m.n[0] * m.n[1] * m.n[2];
    uint8_t *p = pool.take<uint8_t>(bytes);
    if (!p) return -1;
    if (bytes && hipMemcpyAsync(p, m.data, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return -1;
    dm->data = p;
    return 0;
  };
  std::vector<DMask> dref(std::max(1, L - 1)), dsol(L);
  for (int l = 0; l + 1 < L; ++l)
    if (upload_mask(refine[l], &dref[l]) != 0) return fail(err, -3, "device grid build: mask upload failed");
  for (int l = 0; l < L; ++l) {
    MaskView none;
    if (upload_mask(solid ? solid[l] : none, &dsol[l]) != 0)
      return fail(err, -3, "device grid build: mask upload failed");
  }
  DMask nomask{};

  // ---- dense boxes and region membership ----
  DGrid G{};
  G.L = L;
  G.D = D;
  G.B = B;
  for (int a = 0; a < 3; ++a) {
    G.ext[a] = ext[a];
    G.periodic[a] = per[a] ? 1 : 0;
  }
  const int3 per3 = make_int3(G.periodic[0], G.periodic[1], G.periodic[2]);
  for (int l = 0; l < L; ++l) {
    DLevel &v = G.lv[l];
    for (int a = 0; a < 3; ++a) v.E[a] = a < dim ? (ext[a] << l) : 1;
    if (l == 0) {
      for (int a = 0; a < 3; ++a) {
        v.lo[a] = 0;
        v.n[a] = v.E[a];
      }
    } else {
      const MaskView &w = refine[l - 1];
      const DLevel &p = G.lv[l - 1];
      bool empty = !w.data;
      for (int a = 0; a < 3 && !empty; ++a) {
        if (a >= dim) {
          v.lo[a] = 0;
          v.n[a] = 1;
          continue;
        }
        const int32_t a0 = std::max(w.lo[a], p.lo[a]);
        const int32_t a1 = std::min(w.lo[a] + w.n[a], p.lo[a] + p.n[a]);
        if (a1 <= a0) {
          empty = true;
          break;
        }
        v.lo[a] = 2 * a0;
        v.n[a] = 2 * (a1 - a0);
      }
      if (empty)
        for (int a = 0; a < 3; ++a) {
          v.lo[a] = 0;
          v.n[a] = 0;
        }
    }
    const int64_t N = v.size();
    v.st = pool.take<uint8_t>(N);
    v.idx = pool.take<int32_t>(N);
    DEV_MEM(v.st);
    DEV_MEM(v.idx);
    if (N > 0) {
      DEV_TRY(hipMemsetAsync(v.idx, 0xff, sizeof(int32_t) * N, st));
      const DLevel pz = l > 0 ? G.lv[l - 1] : v;
      hipLaunchKernelGGL(k_state, dim3(grid_for(N)), dim3(T), 0, st, v, pz, l > 0 ? dref[l - 1] : nomask,
                         l + 1 < L ? dref[l] : nomask, l, L, D);
    }
    // nesting
    if (l + 1 < L && refine[l].data) {
      const int64_t NW = (int64_t)refine[l].n[0] * refine[l].n[1] * refine[l].n[2];
      if (NW > 0) hipLaunchKernelGGL(k_nest, dim3(grid_for(NW)), dim3(T), 0, st, v, dref[l], derr);
      int h = 0;
      DEV_TRY(errors(&h));
      if (h & E_NEST) return fail(err, -2, "refine mask is not nested in its level");
    }
    if (l + 1 < L && N > 0) hipLaunchKernelGGL(k_strip, dim3(grid_for(N)), dim3(T), 0, st, v, dref[l], D, B, per3);
    if (l >= 1 && l + 1 < L) {
      if (N > 0) hipLaunchKernelGGL(k_iface, dim3(grid_for(N)), dim3(T), 0, st, v, G.lv[l - 1], D, derr);
      int h = 0;
      DEV_TRY(errors(&h));
      if (h & E_IFACE) return fail(err, -2, "refinement interfaces are too close");
    }
    if (N > 0) hipLaunchKernelGGL(k_exist, dim3(grid_for(N)), dim3(T), 0, st, v, dsol[l]);
  }
  for (int l = 0; l + 1 < L; ++l) {
    const int64_t N = G.lv[l].size();
    if (N > 0) hipLaunchKernelGGL(k_cut, dim3(grid_for(N)), dim3(T), 0, st, G.lv[l], G.lv[l + 1], D, derr);
  }
  {
    int h = 0;
    DEV_TRY(errors(&h));
    if (h & E_CUT) return fail(err, -2, "a solid body cuts a refinement interface");
  }

  // ---- canonical order: level-major, Z order inside a level ----
  HostGrid &g = *out;
  g = HostGrid();
  g.D = D;
  g.L = L;
  g.Q = Q;
  g.B = B;
  for (int a = 0; a < 3; ++a) g.ext[a] = ext[a];
  std::vector<int64_t> cnt(L, 0);
  std::vector<int32_t *> ord(L, nullptr);
  int64_t total = 0;
  for (int l = 0; l < L; ++l) {
    const DLevel &v = G.lv[l];
    const int64_t N = v.size();
    g.off[l] = total;
    if (N == 0) continue;
    int32_t *fl = pool.take<int32_t>(N), *pos = pool.take<int32_t>(N);
    DEV_MEM(fl);
    DEV_MEM(pos);
    hipLaunchKernelGGL(k_flag_exist, dim3(grid_for(N)), dim3(T), 0, st, v, fl);
    int64_t m = 0;
    DEV_TRY(exclusive_sum(pool, fl, pos, N, st, &m));
    cnt[l] = m;
    total += m;
    if (m == 0) continue;
    int32_t emax = std::max(v.E[0], std::max(v.E[1], D == 3 ? v.E[2] : 1));
    int bits = 0;
    while ((1 << bits) < emax) ++bits;
    uint64_t *k0 = pool.take<uint64_t>(m), *k1 = pool.take<uint64_t>(m);
    int32_t *i0 = pool.take<int32_t>(m), *i1 = pool.take<int32_t>(m);
    DEV_MEM(k0);
    DEV_MEM(k1);
    DEV_MEM(i0);
    DEV_MEM(i1);
    hipLaunchKernelGGL(k_keys, dim3(grid_for(N)), dim3(T), 0, st, v, D, bits, fl, pos, k0, i0);
    size_t tb = 0;
    const int end_bit = std::max(1, D * bits);
    DEV_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k0, k1, i0, i1, (int)m, 0, end_bit, st));
    void *tmp = pool.take<char>(tb);
    DEV_MEM(tmp);
    DEV_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tb, k0, k1, i0, i1, (int)m, 0, end_bit, st));
    ord[l] = i1;
  }
  g.off[L] = total;
  if (total >= INT32_MAX / 2) return fail(err, -1, "grid too large for 32-bit cell indices");
  const int64_t n = total;
  g.n = n;
  // the tables the caller keeps come from its allocator directly
  auto kept = [&](size_t bytes) -> void * {
    if (!keep) return pool.take<char>(bytes);
    return da.alloc(std::max<size_t>(bytes, 1), da.ctx);
  };
  int32_t *xyz = (int32_t *)kept(sizeof(int32_t) * 3 * n);
  int8_t *lev = (int8_t *)kept(n);
  uint8_t *flag = (uint8_t *)kept(n);
  int32_t *nbr = (int32_t *)kept(sizeof(int32_t) * Qm * n);
  if (keep) {
    keep->xyz = xyz;
    keep->lev = lev;
    keep->flag = flag;
    keep->nbr = nbr;
    keep->n = n;
    keep->Qm = Qm;
  }
  int32_t *src_all = pool.take<int32_t>(n);
  int8_t *bcf = pool.take<int8_t>(n);
  int32_t *fl = pool.take<int32_t>(n), *pos = pool.take<int32_t>(n);
  DEV_MEM(xyz);
  DEV_MEM(lev);
  DEV_MEM(flag);
  DEV_MEM(nbr);
  DEV_MEM(src_all);
  DEV_MEM(bcf);
  DEV_MEM(fl);
  DEV_MEM(pos);
  for (int l = 0; l < L; ++l)
    if (cnt[l] > 0)
      hipLaunchKernelGGL(k_place, dim3(grid_for(cnt[l])), dim3(T), 0, st, G.lv[l], ord[l], cnt[l], g.off[l], l, xyz,
                         lev);
  DLat dl{};
  dl.Q = Q;
  for (int i = 0; i < Q; ++i)
    for (int a = 0; a < 3; ++a) dl.c[i][a] = lat.c[i][a];
  DFaces df{};
  for (int k = 0; k < 6; ++k) {
    df.kind[k] = faces[k].kind;
    df.rho[k] = faces[k].rho;
    df.smax[k] = faces[k].sponge_sigma_max;
    df.width[k] = faces[k].sponge_width;
  }

  // ---- flags ----
  if (n > 0) hipLaunchKernelGGL(k_flags, dim3(grid_for(n)), dim3(T), 0, st, G, n, xyz, lev, flag, derr);
  {
    int h = 0;
    DEV_TRY(errors(&h));
    if (h & E_BOTH) return fail(err, -2, "a cell is both a coarse and a fine ghost");
  }
  // ---- pull neighbour list ----
  if (n > 0) hipLaunchKernelGGL(k_nbr, dim3(grid_for(n)), dim3(T), 0, st, G, dl, df, n, xyz, lev, nbr);
  // ---- boundary layers ----
  if (n > 0) hipLaunchKernelGGL(k_bc, dim3(grid_for(n)), dim3(T), 0, st, G, df, n, xyz, lev, flag, src_all, bcf, derr);
  {
    int h = 0;
    DEV_TRY(errors(&h));
    if (h & E_OVERLAP) return fail(err, -2, "a boundary layer overlaps a refinement interface");
    if (h & E_NOSRC) return fail(err, -2, "a boundary cell has no fluid source");
  }
  if (n > 0) hipLaunchKernelGGL(k_bc_check, dim3(grid_for(n)), dim3(T), 0, st, n, Qm, flag, src_all, nbr, derr);
  {
    int h = 0;
    DEV_TRY(errors(&h));
    if (h & E_SRCBC) return fail(err, -2, "a boundary source lies in a boundary layer");
    if (h & E_ORPHAN) return fail(err, -2, "a bulk cell has no streaming source");
  }
  // per-level offsets of a flagged list in canonical order: the exclusive
  // sum at each level's first cell
  auto level_offsets = [&](const int32_t *p, int64_t tot, int64_t *o) -> hipError_t {
    for (int l = 0; l < L; ++l) {
      if (g.off[l] >= n) {
        o[l] = tot;
        continue;
      }
      int32_t v = 0;
      hipError_t e = hipMemcpyAsync(&v, p + g.off[l], sizeof(int32_t), hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return e;
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
      o[l] = v;
    }
    o[L] = tot;
    return hipSuccess;
  };
  int64_t nbc = 0;
  int32_t *bc_cell = nullptr, *bc_src = nullptr;
  int8_t *bc_face = nullptr;
  if (n > 0) {
    hipLaunchKernelGGL(k_flag_nonneg, dim3(grid_for(n)), dim3(T), 0, st, n, src_all, fl);
    DEV_TRY(exclusive_sum(pool, fl, pos, n, st, &nbc));
    DEV_TRY(level_offsets(pos, nbc, g.boff));
    bc_cell = pool.take<int32_t>(nbc);
    bc_src = pool.take<int32_t>(nbc);
    bc_face = pool.take<int8_t>(nbc);
    DEV_MEM(bc_cell);
    DEV_MEM(bc_src);
    DEV_MEM(bc_face);
    hipLaunchKernelGGL(k_scatter_list, dim3(grid_for(n)), dim3(T), 0, st, n, fl, pos, bc_cell);
    if (nbc > 0)
      hipLaunchKernelGGL(k_bc_list, dim3(grid_for(nbc)), dim3(T), 0, st, nbc, bc_cell, src_all, bcf, bc_src, bc_face);
  } else {
    for (int l = 0; l <= L; ++l) g.boff[l] = 0;
  }
  // ---- pressure sponge ----
  bool any_sponge = false;
  for (int fc = 0; fc < 2 * D; ++fc)
    if (faces[fc].kind != BC_PERIODIC && faces[fc].sponge_sigma_max > 0.0 && faces[fc].sponge_width > 0.0)
      any_sponge = true;
  double *sigma = nullptr, *rho_inf = nullptr;
  if (any_sponge) {
    sigma = pool.take<double>(n);
    rho_inf = pool.take<double>(n);
    DEV_MEM(sigma);
    DEV_MEM(rho_inf);
    if (n > 0)
      hipLaunchKernelGGL(k_sponge, dim3(grid_for(n)), dim3(T), 0, st, G, df, n, xyz, lev, flag, sigma, rho_inf);
  }
  // ---- coarse ghosts: list, child table, unknown populations ----
  int64_t ng = 0;
  int32_t *ghost = nullptr, *child = nullptr;
  uint64_t *unknown = nullptr;
  if (n > 0) {
    hipLaunchKernelGGL(k_flag_bits, dim3(grid_for(n)), dim3(T), 0, st, n, flag, (uint8_t)F_COARSE_GHOST, fl);
    DEV_TRY(exclusive_sum(pool, fl, pos, n, st, &ng));
    DEV_TRY(level_offsets(pos, ng, g.goff));
  } else {
    for (int l = 0; l <= L; ++l) g.goff[l] = 0;
  }
  ghost = pool.take<int32_t>(ng);
  child = pool.take<int32_t>((size_t)ng * NCH);
  unknown = pool.take<uint64_t>(ng);
  DEV_MEM(ghost);
  DEV_MEM(child);
  DEV_MEM(unknown);
  if (ng > 0) {
    hipLaunchKernelGGL(k_scatter_list, dim3(grid_for(n)), dim3(T), 0, st, n, fl, pos, ghost);
    hipLaunchKernelGGL(k_child_unknown, dim3(grid_for(ng)), dim3(T), 0, st, G, Q, ng, n, ghost, xyz, lev, nbr, flag,
                       child, unknown);
  }

  // ---- brick layout ----
  DeviceLayout &y = *yo;
  y = DeviceLayout();
  y.D = D;
  y.sh = D == 3 ? 2 : 3;
  y.bs = 1 << y.sh;
  y.nb = D == 3 ? 27 : 9;
  y.nbp = D == 3 ? 32 : 16;
  if (lat.B > y.bs) return fail(err, -1, "lattice reach exceeds the brick edge");
  const int sh = y.sh, bs = y.bs;
  int32_t *slot_of = (int32_t *)kept(sizeof(int32_t) * n);
  if (keep) keep->slot_of = slot_of;
  int32_t *bxyz = pool.take<int32_t>(3 * std::max<int64_t>(n, 1));  // at most one brick per cell
  int *bbox = pool.take<int>(6);
  DEV_MEM(slot_of);
  DEV_MEM(bxyz);
  DEV_MEM(bbox);
  std::vector<DBricks> lb(L);
  int64_t slots = 0;
  std::vector<int64_t> nbk(L, 0);
  for (int l = 0; l < L; ++l) {
    y.soff[l] = slots;
    const int64_t c0 = g.off[l], m = g.off[l + 1] - g.off[l];
    DBricks &Bk = lb[l];
    Bk.rank = nullptr;
    for (int a = 0; a < 3; ++a) {
      Bk.lo[a] = 0;
      Bk.n[a] = 1;
    }
    if (m == 0) continue;
    const int init[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
    DEV_TRY(hipMemcpyAsync(bbox, init, sizeof init, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_brick_start, dim3(grid_few(m)), dim3(T), 0, st, c0, m, D, sh, xyz, fl, bbox);
    int64_t nb = 0;
    DEV_TRY(exclusive_sum(pool, fl, pos, m, st, &nb));
    int hb[6];
    DEV_TRY(hipMemcpyAsync(hb, bbox, sizeof hb, hipMemcpyDeviceToHost, st));
    DEV_TRY(hipStreamSynchronize(st));
    for (int a = 0; a < 3; ++a) {
      Bk.lo[a] = hb[a];
      Bk.n[a] = hb[3 + a] - hb[a] + 1;
    }
    const int64_t nr = (int64_t)Bk.n[0] * Bk.n[1] * Bk.n[2];
    Bk.rank = pool.take<int32_t>(nr);
    DEV_MEM(Bk.rank);
    DEV_TRY(hipMemsetAsync(Bk.rank, 0xff, sizeof(int32_t) * nr, st));
    hipLaunchKernelGGL(k_brick_rank, dim3(grid_for(m)), dim3(T), 0, st, Bk, c0, m, slots / 64, D, sh, xyz, fl, pos,
                       bxyz, derr);
    hipLaunchKernelGGL(k_slot, dim3(grid_for(m)), dim3(T), 0, st, c0, m, slots, D, sh, xyz, fl, pos, slot_of);
    int h = 0;
    DEV_TRY(errors(&h));
    if (h & E_BRICK) return fail(err, -1, "cells of a brick are not contiguous in the level order");
    nbk[l] = nb;
    slots += nb * 64;
  }
  y.soff[L] = slots;
  y.nslot = slots;
  if (slots >= INT32_MAX / 2) return fail(err, -1, "grid too large for 32-bit slot indices");
  const int64_t nbrk = slots / 64;
  int32_t *cell_of = pool.take<int32_t>(slots);
  int32_t *nbrick = pool.take<int32_t>((size_t)nbrk * y.nbp);
  DEV_MEM(cell_of);
  DEV_MEM(nbrick);
  DEV_TRY(hipMemsetAsync(cell_of, 0xff, sizeof(int32_t) * std::max<int64_t>(slots, 1), st));
  DEV_TRY(hipMemsetAsync(nbrick, 0xff, sizeof(int32_t) * std::max<int64_t>(nbrk * y.nbp, 1), st));
  if (n > 0) hipLaunchKernelGGL(k_cell_of, dim3(grid_for(n)), dim3(T), 0, st, n, slot_of, cell_of);
  for (int l = 0; l < L; ++l) {
    if (nbk[l] == 0) continue;
    int wrap[3], eb[3];
    for (int a = 0; a < 3; ++a) {
      const int64_t e = a < D ? ((int64_t)ext[a] << l) : 1;
      wrap[a] = a < D && per[a] && e % bs == 0;
      eb[a] = (int)(a < D ? e / bs : 1);
    }
    hipLaunchKernelGGL(k_nbrick, dim3(grid_for(nbk[l])), dim3(T), 0, st, lb[l], nbk[l], y.soff[l] / 64, D, y.nb,
                       y.nbp, make_int3(wrap[0], wrap[1], wrap[2]), make_int3(eb[0], eb[1], eb[2]), bxyz, nbrick);
  }
  // exception rows
  uint8_t *special = pool.take<uint8_t>(n);
  unsigned long long *xmask = pool.take<unsigned long long>(nbrk);
  int32_t *pc = pool.take<int32_t>(nbrk), *xbase = pool.take<int32_t>(nbrk);
  int32_t *gidx = pool.take<int32_t>(n), *xrow_of = pool.take<int32_t>(n);
  DEV_MEM(special);
  DEV_MEM(xmask);
  DEV_MEM(pc);
  DEV_MEM(xbase);
  DEV_MEM(gidx);
  DEV_MEM(xrow_of);
  DEV_TRY(hipMemsetAsync(special, 0, std::max<int64_t>(n, 1), st));
  DEV_TRY(hipMemsetAsync(xmask, 0, sizeof(unsigned long long) * std::max<int64_t>(nbrk, 1), st));
  DEV_TRY(hipMemsetAsync(gidx, 0xff, sizeof(int32_t) * std::max<int64_t>(n, 1), st));
  DEV_TRY(hipMemsetAsync(xrow_of, 0xff, sizeof(int32_t) * std::max<int64_t>(n, 1), st));
  if (ng > 0)
    hipLaunchKernelGGL(k_mark_children, dim3(grid_for(ng * NCH)), dim3(T), 0, st, ng * NCH, child, special);
  if (n > 0) {
    hipLaunchKernelGGL(k_special, dim3(grid_for(n)), dim3(T), 0, st, dl, n, D, sh, y.nbp, xyz, flag, nbr, slot_of,
                       nbrick, special);
    hipLaunchKernelGGL(k_xmask, dim3(grid_for(n)), dim3(T), 0, st, n, special, slot_of, xmask);
  }
  int64_t rows = 0;
  if (nbrk > 0) {
    hipLaunchKernelGGL(k_popc, dim3(grid_for(nbrk)), dim3(T), 0, st, nbrk, xmask, pc);
    DEV_TRY(exclusive_sum(pool, pc, xbase, nbrk, st, &rows));
  }
  y.nx = rows;
  y.xstride = std::max<int64_t>(64, ((rows + 63) / 64) * 64);
  int32_t *xnbr = pool.take<int32_t>((size_t)Qm * y.xstride);
  DEV_MEM(xnbr);
  DEV_TRY(hipMemsetAsync(xnbr, 0xff, sizeof(int32_t) * (size_t)Qm * y.xstride, st));
  if (ng > 0) hipLaunchKernelGGL(k_gidx, dim3(grid_for(ng)), dim3(T), 0, st, ng, ghost, gidx);
  if (n > 0)
    hipLaunchKernelGGL(k_xrows, dim3(grid_for(n)), dim3(T), 0, st, n, Qm, y.xstride, y.nslot, special, slot_of,
                       xmask, xbase, nbr, gidx, xrow_of, xnbr);
  DEV_TRY(hipGetLastError());

  // ---- back to the host structures ----
  if (!keep) {
    DEV_TRY(down(g.xyz, xyz, 3 * n, st));
    DEV_TRY(down(g.nbr, nbr, (size_t)Qm * n, st));
  }
  DEV_TRY(down(g.lev, lev, n, st));
  DEV_TRY(down(g.flag, flag, n, st));
  DEV_TRY(down(g.bc_src_all, src_all, n, st));
  DEV_TRY(down(g.bc_cell, bc_cell, nbc, st));
  DEV_TRY(down(g.bc_src, bc_src, nbc, st));
  DEV_TRY(down(g.bc_face, bc_face, nbc, st));
  if (any_sponge) {
    DEV_TRY(down(g.sigma, sigma, n, st));
    DEV_TRY(down(g.rho_inf, rho_inf, n, st));
  }
  DEV_TRY(down(g.ghost_cell, ghost, ng, st));
  DEV_TRY(down(g.child, child, (size_t)ng * NCH, st));
  DEV_TRY(down(g.unknown, unknown, ng, st));
  DEV_TRY(down(y.slot_of, slot_of, n, st));
  DEV_TRY(down(y.cell_of, cell_of, slots, st));
  DEV_TRY(down(y.nbrick, nbrick, (size_t)nbrk * y.nbp, st));
  std::vector<unsigned long long> xm;
  DEV_TRY(down(xm, xmask, nbrk, st));
  DEV_TRY(down(y.xbase, xbase, nbrk, st));
  DEV_TRY(down(y.xrow_of, xrow_of, n, st));
  DEV_TRY(down(y.xnbr, xnbr, (size_t)Qm * y.xstride, st));
  DEV_TRY(hipStreamSynchronize(st));
  y.xmask.assign(xm.begin(), xm.end());
  return 0;
}

int fetch_host_mirror(const DeviceGridArrays &dg, HostGrid *g, hipStream_t st, std::string *err) {
  bool any = false;
  if (dg.xyz && g->xyz.empty()) {
    DEV_TRY(down(g->xyz, dg.xyz, 3 * dg.n, st));
    any = true;
  }
  if (dg.nbr && g->nbr.empty()) {
    DEV_TRY(down(g->nbr, dg.nbr, (size_t)dg.Qm * dg.n, st));
    any = true;
  }
  if (any) DEV_TRY(hipStreamSynchronize(st));
  return 0;
}

namespace {
__global__ void k_slot_flags(int64_t n, int Qm, const uint8_t *flag, const int32_t *nbr, const int32_t *slot_of,
                             uint8_t *out) {
  GRID_STRIDE(c, n) {
    uint8_t v = flag[c];
    for (int i = 0; i < Qm; ++i)
      if (nbr[(int64_t)i * n + c] <= -3) v |= F_MOVING;
    out[slot_of[c]] = v;
  }
}
}  // namespace

void launch_slot_flags(const DeviceGridArrays &dg, int64_t nslot, uint8_t *out, hipStream_t st) {
  hipMemsetAsync(out, F_HOLE, std::max<int64_t>(nslot, 1), st);
  if (dg.n > 0)
    hipLaunchKernelGGL(k_slot_flags, dim3(grid_for(dg.n)), dim3(TPB), 0, st, dg.n, dg.Qm, dg.flag, dg.nbr,
                       dg.slot_of, out);
}

int remesh_sources_device(const HostGrid &old, const DeviceGridArrays &dold, const HostGrid &nw,
                          const DeviceGridArrays &dnew, const DevAlloc &da, hipStream_t st, int64_t **d_off,
                          int32_t **d_src, double **d_wt, std::string *err) {
  *d_off = nullptr;
  *d_src = nullptr;
  *d_wt = nullptr;
  Pool pool(da);
  const int64_t no = old.n, nn = nw.n;
  const int L = old.L;
  const int32_t *oxyz = dold.xyz, *nxyz = dnew.xyz;
  const int8_t *olev = dold.lev, *nlev = dnew.lev;
  const uint8_t *oflag = dold.flag;
  if (!oxyz || !nxyz || !olev || !nlev || !oflag) return fail(err, -3, "remesh: device grid tables missing");
  int *bbox = pool.take<int>(6 * 8);
  int64_t *cnt = pool.take<int64_t>(nn + 1);
  double *tot = pool.take<double>(nn);
  unsigned long long *bad = pool.take<unsigned long long>(1);
  if (pool.failed) return fail(err, -3, "remesh: device allocation failed");
  std::vector<int> hb(6 * 8);
  for (int l = 0; l < 8; ++l)
    for (int a = 0; a < 3; ++a) {
      hb[6 * l + a] = INT_MAX;
      hb[6 * l + 3 + a] = INT_MIN;
    }
  DEV_TRY(hipMemcpyAsync(bbox, hb.data(), sizeof(int) * hb.size(), hipMemcpyHostToDevice, st));
  const unsigned T = TPB;
  for (int l = 0; l < L; ++l) {
    const int64_t m = old.off[l + 1] - old.off[l];
    if (m > 0)
      hipLaunchKernelGGL(k_flow_bbox, dim3(grid_few(m)), dim3(T), 0, st, old.off[l], m, oxyz, oflag, bbox + 6 * l);
  }
  DEV_TRY(hipMemcpyAsync(hb.data(), bbox, sizeof(int) * hb.size(), hipMemcpyDeviceToHost, st));
  DEV_TRY(hipStreamSynchronize(st));
  DFlows F{};
  F.L = L;
  F.D = nw.D;
  F.deepest = 0;
  for (int l = 0; l < L; ++l) {
    DFlow &f = F.lv[l];
    f.map = nullptr;
    if (hb[6 * l] > hb[6 * l + 3]) continue;  // no flow cell on this level
    F.deepest = l;
    int64_t sz = 1;
    for (int a = 0; a < 3; ++a) {
      f.lo[a] = hb[6 * l + a];
      f.n[a] = hb[6 * l + 3 + a] - hb[6 * l + a] + 1;
      sz *= f.n[a];
    }
    f.map = pool.take<int32_t>(sz);
    if (!f.map) return fail(err, -3, "remesh: device allocation failed");
    DEV_TRY(hipMemsetAsync(f.map, 0xff, sizeof(int32_t) * sz, st));
  }
  if (no > 0) hipLaunchKernelGGL(k_flow_map, dim3(grid_for(no)), dim3(T), 0, st, F, no, oxyz, olev, oflag);
  const unsigned long long none = ~0ull;
  DEV_TRY(hipMemcpyAsync(bad, &none, sizeof none, hipMemcpyHostToDevice, st));
  DEV_TRY(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (nn + 1), st));
  if (nn > 0) hipLaunchKernelGGL(k_src_count, dim3(grid_for(nn)), dim3(T), 0, st, F, nn, nxyz, nlev, cnt, tot, bad);
  unsigned long long hbad = none;
  DEV_TRY(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, st));
  DEV_TRY(hipStreamSynchronize(st));
  if (hbad != none) {
    if (err) *err = "remesh: new cell " + std::to_string(hbad) + " covers no flow cell of the old grid";
    return -1;
  }
  int64_t *off = (int64_t *)da.alloc(sizeof(int64_t) * (nn + 1), da.ctx);
  if (!off) return fail(err, -3, "remesh: device allocation failed");
  *d_off = off;
  size_t tb = 0;
  DEV_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, off, (int)(nn + 1), st));
  void *tmp = pool.take<char>(tb);
  if (!tmp) return fail(err, -3, "remesh: device allocation failed");
  DEV_TRY(hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt, off, (int)(nn + 1), st));
  int64_t total = 0;
  DEV_TRY(hipMemcpyAsync(&total, off + nn, sizeof total, hipMemcpyDeviceToHost, st));
  DEV_TRY(hipStreamSynchronize(st));
  *d_src = (int32_t *)da.alloc(sizeof(int32_t) * std::max<int64_t>(total, 1), da.ctx);
  *d_wt = (double *)da.alloc(sizeof(double) * std::max<int64_t>(total, 1), da.ctx);
  if (!*d_src || !*d_wt) return fail(err, -3, "remesh: device allocation failed");
  if (nn > 0)
    hipLaunchKernelGGL(k_src_fill, dim3(grid_for(nn)), dim3(T), 0, st, F, nn, nxyz, nlev, off, tot, *d_src, *d_wt);
  DEV_TRY(hipGetLastError());
  DEV_TRY(hipStreamSynchronize(st));
  return 0;
}

}  // namespace lbm
