// grid_builder.cpp -- host construction of the static refined grid.
//
// Level l (0 = coarsest) holds the cells of R_l outside R_{l+1}, plus the
// cells of R_{l+1} within Chebyshev distance B (in level-l cells) of its
// outside: these coarse ghosts overlap their children, the fine ghosts of
// level l+1 (Sec. 3.2; the buffer layer widened to B cells for high-order
// lattices).  Cells are grouped by level and ordered along the Z-order curve
// inside a level (Secs. 4.3-4.4).  Every level is processed on a dense box
// that bounds where it can exist, so memory follows the refined regions.
#include "grid_builder.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace lbm {
namespace {

enum : uint8_t { S_INR = 1, S_REF = 2, S_STRIP = 4, S_PRE = 8, S_EXIST = 16 };

struct LevelTmp {
  int32_t E[3] = {1, 1, 1};    // level extent
  int32_t lo[3] = {0, 0, 0};   // dense box
  int32_t n[3] = {0, 0, 0};
  std::vector<uint8_t> st;
  std::vector<int32_t> idx;
  bool inside(int32_t x, int32_t y, int32_t z) const {
    return x >= lo[0] && y >= lo[1] && z >= lo[2] && x < lo[0] + n[0] && y < lo[1] + n[1] &&
           z < lo[2] + n[2];
  }
  int64_t lin(int32_t x, int32_t y, int32_t z) const {
    return (int64_t)(x - lo[0]) + (int64_t)n[0] * ((int64_t)(y - lo[1]) + (int64_t)n[1] * (z - lo[2]));
  }
  int64_t size() const { return (int64_t)n[0] * n[1] * n[2]; }
};

struct Ctx {
  const LatticeInfo *lat;
  int D, L, B;
  int32_t ext[3];
  const FaceSpec *faces;
  bool periodic[3];
};

void zorder(const LevelTmp &lv, int D, int32_t x0, int32_t y0, int32_t z0, int32_t size,
            std::vector<int64_t> &out) {
  if (x0 >= lv.lo[0] + lv.n[0] || y0 >= lv.lo[1] + lv.n[1] || z0 >= lv.lo[2] + lv.n[2]) return;
  if (x0 + size <= lv.lo[0] || y0 + size <= lv.lo[1] || (D == 3 && z0 + size <= lv.lo[2])) return;
  if (size == 1) {
    const int64_t id = lv.lin(x0, y0, z0);
    if (lv.st[id] & S_EXIST) out.push_back(id);
    return;
  }
  const int32_t h = size / 2;
  for (int o = 0; o < (1 << D); ++o)
    zorder(lv, D, x0 + (o & 1) * h, y0 + ((o >> 1) & 1) * h, D == 3 ? z0 + ((o >> 2) & 1) * h : 0, h,
           out);
}

int fail(std::string *err, int code, const char *msg) {
  if (err) *err = msg;
  return code;
}

}  // namespace

int build_grid(const LatticeInfo &lat, int dim, const int32_t ext_in[3], int L,
               const MaskView *refine, const MaskView *solid, const FaceSpec faces[6],
               HostGrid *out, std::string *err) {
  if (dim != lat.D) return fail(err, -1, "dimension does not match the lattice");
  if (L < 1 || L > 8) return fail(err, -1, "level count must be 1..8");
  Ctx cx;
  cx.lat = &lat;
  cx.D = dim;
  cx.L = L;
  cx.B = lat.B;
  cx.faces = faces;
  for (int a = 0; a < 3; ++a) {
    cx.ext[a] = a < dim ? ext_in[a] : 1;
    if (cx.ext[a] < 1) return fail(err, -1, "extent must be positive");
    if (a < dim && ((int64_t)cx.ext[a] << (L - 1)) >= (1 << 21))
      return fail(err, -1, "finest extent exceeds 2^21 cells per axis");
  }
  for (int a = 0; a < 3; ++a) {
    cx.periodic[a] = false;
    if (a >= dim) continue;
    const bool p0 = faces[2 * a].kind == BC_PERIODIC, p1 = faces[2 * a + 1].kind == BC_PERIODIC;
    if (p0 != p1) return fail(err, -2, "periodic faces must come in pairs");
    cx.periodic[a] = p0;
    if (p0 && cx.ext[a] <= lat.B) return fail(err, -1, "periodic extent must exceed the lattice reach");
    for (int s = 0; s < 2; ++s)
      if (faces[2 * a + s].kind < 0 || faces[2 * a + s].kind > 4) return fail(err, -1, "unknown face kind");
  }
  const int D = dim, B = lat.B, Q = lat.Q, Qm = Q - 1, NCH = 1 << D;
  // windows must lie inside their level
  for (int l = 0; l + 1 < L; ++l)
    for (int a = 0; a < 3; ++a) {
      const int64_t E = a < dim ? ((int64_t)cx.ext[a] << l) : 1;
      if (refine[l].data && (refine[l].lo[a] < 0 || refine[l].n[a] < 0 || refine[l].lo[a] + refine[l].n[a] > E))
        return fail(err, -1, "refine mask window outside its level");
    }
  for (int l = 0; solid && l < L; ++l)
    for (int a = 0; a < 3; ++a) {
      const int64_t E = a < dim ? ((int64_t)cx.ext[a] << l) : 1;
      if (solid[l].data && (solid[l].lo[a] < 0 || solid[l].n[a] < 0 || solid[l].lo[a] + solid[l].n[a] > E))
        return fail(err, -1, "solid mask window outside its level");
    }

  std::vector<LevelTmp> lv(L);
  // ---- dense boxes and region membership ----------------------------------
  for (int l = 0; l < L; ++l) {
    LevelTmp &v = lv[l];
    for (int a = 0; a < 3; ++a) v.E[a] = a < dim ? (cx.ext[a] << l) : 1;
    if (l == 0) {
      for (int a = 0; a < 3; ++a) { v.lo[a] = 0; v.n[a] = v.E[a]; }
    } else {
      const MaskView &w = refine[l - 1];
      const LevelTmp &p = lv[l - 1];
      bool empty = !w.data;
      for (int a = 0; a < 3 && !empty; ++a) {
        if (a >= dim) { v.lo[a] = 0; v.n[a] = 1; continue; }
        const int32_t a0 = std::max(w.lo[a], p.lo[a]);
        const int32_t a1 = std::min(w.lo[a] + w.n[a], p.lo[a] + p.n[a]);
        if (a1 <= a0) { empty = true; break; }
        v.lo[a] = 2 * a0;
        v.n[a] = 2 * (a1 - a0);
      }
      if (empty)
        for (int a = 0; a < 3; ++a) { v.lo[a] = 0; v.n[a] = 0; }
    }
    const int64_t N = v.size();
    v.st.assign(N, 0);
    const MaskView *wp = l > 0 ? &refine[l - 1] : nullptr;
    const LevelTmp *pp = l > 0 ? &lv[l - 1] : nullptr;
#pragma omp parallel for schedule(static) collapse(2)
    for (int32_t z = 0; z < v.n[2]; ++z)
      for (int32_t y = 0; y < v.n[1]; ++y)
        for (int32_t x = 0; x < v.n[0]; ++x) {
          const int32_t X = x + v.lo[0], Y = y + v.lo[1], Z = z + v.lo[2];
          uint8_t s = 0;
          if (l == 0) {
            s = S_INR;
          } else {
            const int32_t PX = X >> 1, PY = Y >> 1, PZ = D == 3 ? Z >> 1 : 0;
            if ((pp->st[pp->lin(PX, PY, PZ)] & S_INR) && wp->at(PX, PY, PZ)) s = S_INR;
          }
          if (l + 1 < L && refine[l].at(X, Y, Z)) s |= S_REF;
          v.st[v.lin(X, Y, Z)] = s;
        }
    // nesting: every refined cell belongs to this level's region
    if (l + 1 < L && refine[l].data) {
      const MaskView &w = refine[l];
      bool bad = false;
#pragma omp parallel for schedule(static) collapse(2) reduction(|| : bad)
      for (int32_t z = 0; z < w.n[2]; ++z)
        for (int32_t y = 0; y < w.n[1]; ++y)
          for (int32_t x = 0; x < w.n[0]; ++x) {
            if (!w.data[x + (int64_t)w.n[0] * (y + (int64_t)w.n[1] * z)]) continue;
            const int32_t X = x + w.lo[0], Y = y + w.lo[1], Z = z + w.lo[2];
            if (!v.inside(X, Y, Z) || !(v.st[v.lin(X, Y, Z)] & S_INR)) bad = true;
          }
      if (bad) return fail(err, -2, "refine mask is not nested in its level");
    }
    // coarse-ghost strip: refined cells within Chebyshev distance B of an
    // unrefined in-domain cell (periodic faces wrap)
    if (l + 1 < L) {
      const MaskView &w = refine[l];
      const int RZ = D == 3 ? B : 0;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
      for (int32_t z = 0; z < v.n[2]; ++z)
        for (int32_t y = 0; y < v.n[1]; ++y)
          for (int32_t x = 0; x < v.n[0]; ++x) {
            const int64_t id = (int64_t)x + (int64_t)v.n[0] * ((int64_t)y + (int64_t)v.n[1] * z);
            if (!(v.st[id] & S_REF)) continue;
            const int32_t X = x + v.lo[0], Y = y + v.lo[1], Z = z + v.lo[2];
            bool hit = false;
            for (int dz = -RZ; dz <= RZ && !hit; ++dz)
              for (int dy = -B; dy <= B && !hit; ++dy)
                for (int dx = -B; dx <= B && !hit; ++dx) {
                  int32_t q[3] = {X + dx, Y + dy, Z + dz};
                  bool outside = false;
                  for (int a = 0; a < dim; ++a) {
                    if (q[a] >= 0 && q[a] < v.E[a]) continue;
                    if (cx.periodic[a]) q[a] = ((q[a] % v.E[a]) + v.E[a]) % v.E[a];
                    else outside = true;
                  }
                  if (!outside && !w.at(q[0], q[1], q[2])) hit = true;
                }
            if (hit) v.st[id] |= S_STRIP;
          }
    }
    // interfaces must be at least B cells of the coarser level apart
    if (l >= 1 && l + 1 < L) {
      const LevelTmp &p = lv[l - 1];
      bool bad = false;
#pragma omp parallel for schedule(static) reduction(|| : bad)
      for (int64_t id = 0; id < N; ++id) {
        if (!(v.st[id] & S_REF)) continue;
        const int32_t X = (int32_t)(id % v.n[0]) + v.lo[0];
        const int32_t Y = (int32_t)((id / v.n[0]) % v.n[1]) + v.lo[1];
        const int32_t Z = (int32_t)(id / ((int64_t)v.n[0] * v.n[1])) + v.lo[2];
        if (p.st[p.lin(X >> 1, Y >> 1, D == 3 ? Z >> 1 : 0)] & S_STRIP) bad = true;
      }
      if (bad) return fail(err, -2, "refinement interfaces are too close");
    }
    // existence
    const MaskView *sv = solid ? &solid[l] : nullptr;
#pragma omp parallel for schedule(static)
    for (int64_t id = 0; id < N; ++id) {
      uint8_t s = v.st[id];
      const bool pre = (s & S_INR) && (!(s & S_REF) || (s & S_STRIP));
      if (!pre) continue;
      s |= S_PRE;
      bool sol = false;
      if (sv && sv->data) {
        const int32_t X = (int32_t)(id % v.n[0]) + v.lo[0];
        const int32_t Y = (int32_t)((id / v.n[0]) % v.n[1]) + v.lo[1];
        const int32_t Z = (int32_t)(id / ((int64_t)v.n[0] * v.n[1])) + v.lo[2];
        sol = sv->at(X, Y, Z) != 0;
      }
      if (!sol) s |= S_EXIST;
      v.st[id] = s;
    }
  }
  // solid bodies must not cut interfaces: a fluid coarse ghost needs a fluid
  // child, a solid one has none
  for (int l = 0; l + 1 < L; ++l) {
    const LevelTmp &v = lv[l], &f = lv[l + 1];
    const int64_t N = v.size();
    bool bad = false;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t id = 0; id < N; ++id) {
      if (!(v.st[id] & S_STRIP)) continue;
      const int32_t X = (int32_t)(id % v.n[0]) + v.lo[0];
      const int32_t Y = (int32_t)((id / v.n[0]) % v.n[1]) + v.lo[1];
      const int32_t Z = (int32_t)(id / ((int64_t)v.n[0] * v.n[1])) + v.lo[2];
      int nf = 0;
      for (int o = 0; o < NCH; ++o) {
        const int32_t cx_ = 2 * X + (o & 1), cy_ = 2 * Y + ((o >> 1) & 1);
        const int32_t cz_ = D == 3 ? 2 * Z + ((o >> 2) & 1) : 0;
        if (f.inside(cx_, cy_, cz_) && (f.st[f.lin(cx_, cy_, cz_)] & S_EXIST)) ++nf;
      }
      const bool fluid = (v.st[id] & S_EXIST) != 0;
      if (fluid ? nf == 0 : nf != 0) bad = true;
    }
    if (bad) return fail(err, -2, "a solid body cuts a refinement interface");
  }

  // ---- canonical order: level-major, Z-order inside a level ----------------
  HostGrid &g = *out;
  g = HostGrid();
  g.D = D;
  g.L = L;
  g.Q = Q;
  g.B = B;
  for (int a = 0; a < 3; ++a) g.ext[a] = cx.ext[a];
  std::vector<std::vector<int64_t>> order(L);
  int64_t total = 0;
  for (int l = 0; l < L; ++l) {
    LevelTmp &v = lv[l];
    int32_t emax = std::max(v.E[0], std::max(v.E[1], D == 3 ? v.E[2] : 1));
    int32_t root = 1;
    while (root < emax) root <<= 1;
    if (v.size() > 0) zorder(v, D, 0, 0, 0, root, order[l]);
    g.off[l] = total;
    total += (int64_t)order[l].size();
  }
  g.off[L] = total;
  if (total >= INT32_MAX / 2) return fail(err, -1, "grid too large for 32-bit cell indices");
  const int64_t n = total;
  g.n = n;
  g.xyz.resize(3 * n);
  g.lev.resize(n);
  g.flag.assign(n, 0);
  for (int l = 0; l < L; ++l) {
    LevelTmp &v = lv[l];
    v.idx.assign(v.size(), -1);
    const std::vector<int64_t> &ord = order[l];
    const int64_t base = g.off[l];
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)ord.size(); ++k) {
      const int64_t id = ord[k];
      const int64_t c = base + k;
      g.xyz[3 * c] = (int32_t)(id % v.n[0]) + v.lo[0];
      g.xyz[3 * c + 1] = (int32_t)((id / v.n[0]) % v.n[1]) + v.lo[1];
      g.xyz[3 * c + 2] = (int32_t)(id / ((int64_t)v.n[0] * v.n[1])) + v.lo[2];
      g.lev[c] = (int8_t)l;
      v.idx[id] = (int32_t)c;
    }
    std::vector<int64_t>().swap(order[l]);
  }
  // ---- flags ----------------------------------------------------------------
  bool both = false;
#pragma omp parallel for schedule(static) reduction(|| : both)
  for (int64_t c = 0; c < n; ++c) {
    const int l = g.lev[c];
    const int32_t X = g.xyz[3 * c], Y = g.xyz[3 * c + 1], Z = g.xyz[3 * c + 2];
    uint8_t fl = 0;
    if (lv[l].st[lv[l].lin(X, Y, Z)] & S_STRIP) fl |= F_COARSE_GHOST;
    if (l > 0) {
      const LevelTmp &p = lv[l - 1];
      if (p.st[p.lin(X >> 1, Y >> 1, D == 3 ? Z >> 1 : 0)] & S_STRIP) fl |= F_FINE_GHOST;
    }
    if ((fl & (F_COARSE_GHOST | F_FINE_GHOST)) == (F_COARSE_GHOST | F_FINE_GHOST)) both = true;
    g.flag[c] = fl;
  }
  if (both) return fail(err, -2, "a cell is both a coarse and a fine ghost");
  // ---- pull neighbour list (canonical sentinels), SoA ----------------------
  g.nbr.resize((size_t)Qm * n);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < n; ++c) {
    const int l = g.lev[c];
    const LevelTmp &v = lv[l];
    for (int i = 1; i < Q; ++i) {
      int32_t q[3];
      int nout = 0, outf[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a) {
        q[a] = g.xyz[3 * c + a] - lat.c[i][a];
        if (a >= D) continue;
        if (q[a] >= 0 && q[a] < v.E[a]) continue;
        if (cx.periodic[a]) q[a] = ((q[a] % v.E[a]) + v.E[a]) % v.E[a];
        else outf[nout++] = 2 * a + (q[a] >= v.E[a] ? 1 : 0);
      }
      int32_t val = NBR_NONE;
      if (nout > 0) {
        bool wall = false;
        int mov = -1;
        for (int k = 0; k < nout; ++k) {
          const int kind = faces[outf[k]].kind;
          if (kind == BC_WALL) wall = true;
          if (kind == BC_MOVING_WALL && mov < 0) mov = outf[k];
        }
        val = wall ? NBR_SOLID : (mov >= 0 ? -3 - mov : NBR_NONE);
      } else if (v.inside(q[0], q[1], q[2])) {
        const int64_t id = v.lin(q[0], q[1], q[2]);
        if (v.st[id] & S_EXIST) val = v.idx[id];
        else if (v.st[id] & S_PRE) val = NBR_SOLID;
      }
      g.nbr[(size_t)(i - 1) * n + c] = val;
    }
  }
  // ---- boundary layers (B cells deep) on Neumann / equilibrium faces -------
  g.bc_src_all.assign(n, -1);
  std::vector<int8_t> bcf(n, -1);
  bool overlap = false, nosrc = false;
#pragma omp parallel for schedule(static) reduction(|| : overlap, nosrc)
  for (int64_t c = 0; c < n; ++c) {
    const int l = g.lev[c];
    int32_t src[3] = {g.xyz[3 * c], g.xyz[3 * c + 1], g.xyz[3 * c + 2]};
    int eqf = -1, nef = -1;
    for (int fc = 0; fc < 2 * D; ++fc) {
      const int kind = faces[fc].kind, a = fc / 2;
      if (kind != BC_NEUMANN && kind != BC_EQUILIBRIUM) continue;
      const int32_t E = lv[l].E[a], x = g.xyz[3 * c + a];
      const bool in = (fc & 1) ? x >= E - B : x < B;
      if (!in) continue;
      src[a] = (fc & 1) ? E - 1 - B : B;
      if (kind == BC_EQUILIBRIUM && eqf < 0) eqf = fc;
      if (kind == BC_NEUMANN && nef < 0) nef = fc;
    }
    if (eqf < 0 && nef < 0) continue;
    if (g.flag[c] & (F_COARSE_GHOST | F_FINE_GHOST)) { overlap = true; continue; }
    int32_t sid = -1;
    if (lv[l].inside(src[0], src[1], src[2])) sid = lv[l].idx[lv[l].lin(src[0], src[1], src[2])];
    if (sid < 0) { nosrc = true; continue; }
    g.bc_src_all[c] = sid;
    bcf[c] = (int8_t)(eqf >= 0 ? eqf : nef);
    g.flag[c] |= eqf >= 0 ? F_BC_EQ : F_BC_NEUMANN;
  }
  if (overlap) return fail(err, -2, "a boundary layer overlaps a refinement interface");
  if (nosrc) return fail(err, -2, "a boundary cell has no fluid source");
  bool srcbc = false, orphan = false;
#pragma omp parallel for schedule(static) reduction(|| : srcbc, orphan)
  for (int64_t c = 0; c < n; ++c) {
    const int32_t s = g.bc_src_all[c];
    if (s >= 0 && (g.flag[s] & (F_BC_EQ | F_BC_NEUMANN))) srcbc = true;
    if (g.flag[c] & (F_COARSE_GHOST | F_FINE_GHOST | F_BC_EQ | F_BC_NEUMANN)) continue;
    for (int i = 1; i < Q; ++i)
      if (g.nbr[(size_t)(i - 1) * n + c] == NBR_NONE) orphan = true;
  }
  if (srcbc) return fail(err, -2, "a boundary source lies in a boundary layer");
  if (orphan) return fail(err, -2, "a bulk cell has no streaming source");
  for (int l = 0; l < L; ++l) {
    g.boff[l] = (int64_t)g.bc_cell.size();
    for (int64_t c = g.off[l]; c < g.off[l + 1]; ++c)
      if (g.bc_src_all[c] >= 0) {
        g.bc_cell.push_back((int32_t)c);
        g.bc_src.push_back(g.bc_src_all[c]);
        g.bc_face.push_back(bcf[c]);
      }
  }
  g.boff[L] = (int64_t)g.bc_cell.size();
  // ---- pressure sponge: linear ramp over a band along each face ------------
  bool any_sponge = false;
  for (int fc = 0; fc < 2 * D; ++fc)
    if (faces[fc].kind != BC_PERIODIC && faces[fc].sponge_sigma_max > 0.0 && faces[fc].sponge_width > 0.0)
      any_sponge = true;
  if (any_sponge) {
    g.sigma.assign(n, 0.0);
    g.rho_inf.assign(n, 1.0);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
      const int l = g.lev[c];
      double best = 0.0, rinf = 1.0;
      for (int fc = 0; fc < 2 * D; ++fc) {
        const FaceSpec &F = faces[fc];
        if (F.kind == BC_PERIODIC || F.sponge_sigma_max <= 0.0 || F.sponge_width <= 0.0) continue;
        const int a = fc / 2;
        const double centre = (g.xyz[3 * c + a] + 0.5) / (double)(1 << l);
        const double dist = (fc & 1) ? cx.ext[a] - centre : centre;
        const double ramp = std::min(1.0, std::max(0.0, 1.0 - dist / F.sponge_width));
        const double s = F.sponge_sigma_max * ramp;
        if (s > best) { best = s; rinf = F.rho; }
      }
      g.sigma[c] = best;
      g.rho_inf[c] = rinf;
      if (best > 0.0) g.flag[c] |= F_SPONGE;
    }
  }
  // ---- coarse ghosts: child table and unknown populations ------------------
  for (int l = 0; l < L; ++l) {
    g.goff[l] = (int64_t)g.ghost_cell.size();
    for (int64_t c = g.off[l]; c < g.off[l + 1]; ++c)
      if (g.flag[c] & F_COARSE_GHOST) g.ghost_cell.push_back((int32_t)c);
  }
  g.goff[L] = (int64_t)g.ghost_cell.size();
  const int64_t ng = g.goff[L];
  g.child.assign((size_t)ng * NCH, -1);
  g.unknown.assign(ng, 0);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < ng; ++k) {
    const int64_t c = g.ghost_cell[k];
    const int l = g.lev[c];
    const LevelTmp &f = lv[l + 1];
    for (int o = 0; o < NCH; ++o) {
      const int32_t X = 2 * g.xyz[3 * c] + (o & 1), Y = 2 * g.xyz[3 * c + 1] + ((o >> 1) & 1);
      const int32_t Z = D == 3 ? 2 * g.xyz[3 * c + 2] + ((o >> 2) & 1) : 0;
      if (f.inside(X, Y, Z)) g.child[(size_t)k * NCH + o] = f.idx[f.lin(X, Y, Z)];
    }
    // coalesced: populations the coarse level does not supply itself, i.e.
    // whose pull source at this level is missing or is another coarse ghost
    // (in the overlap the fine level carries the flow; taking such a
    // population from the neighbouring ghost double-counts at corners)
    uint64_t m = 0;
    for (int i = 1; i < Q; ++i) {
      const int32_t v = g.nbr[(size_t)(i - 1) * n + c];
      if (v == NBR_NONE || (v >= 0 && (g.flag[v] & F_COARSE_GHOST))) m |= (uint64_t)1 << i;
    }
    g.unknown[k] = m;
  }
  return 0;
}

}  // namespace lbm
