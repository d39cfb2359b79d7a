// lattice.h -- velocity sets, weights and per-lattice constants of the
// library (App. A.1, Table "lattices_structure"; D3Q27 = D1Q3^3).
//
// The sets are generated at compile time: every integer vector of the
// lattice's shell list, rest velocity first, then ascending (|xi|^2, xi_x,
// xi_y, xi_z).  This canonical order defines the population index i and the
// columns of the neighbour list.
#pragma once

#include <cstdint>

namespace lbm {

enum LatticeKind { LAT_D2Q9 = 0, LAT_D3Q27 = 1, LAT_D2Q21 = 2, LAT_D2Q37 = 3, LAT_D2Q13 = 4 };

struct Vel {
  int x, y, z;
};

template <int Q>
struct VelSet {
  Vel v[Q];
  double w[Q];
  int opp[Q];
};

constexpr int iabs_c(int a) { return a < 0 ? -a : a; }

// Weight of velocity (x, y, z) in lattice `kind`, 0 when not a member.
// D2Q37: the unique solution of the eighth-order isotropy conditions (the
// tabulated 15-digit values are this solution truncated).
constexpr double weight_of(int kind, int x, int y, int z) {
  const int a = iabs_c(x), b = iabs_c(y), c = iabs_c(z);
  if (kind == LAT_D3Q27) {
    if (a > 1 || b > 1 || c > 1) return 0.0;
    const int nz = (a != 0) + (b != 0) + (c != 0);
    return nz == 0 ? 8.0 / 27.0 : nz == 1 ? 2.0 / 27.0 : nz == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
  }
  if (c != 0) return 0.0;
  const int hi = a > b ? a : b, lo = a > b ? b : a;
  if (kind == LAT_D2Q9) {
    if (hi == 0) return 4.0 / 9.0;
    if (hi == 1 && lo == 0) return 1.0 / 9.0;
    if (hi == 1 && lo == 1) return 1.0 / 36.0;
    return 0.0;
  }
  if (kind == LAT_D2Q13) {
    if (hi == 0) return 36.0 / 96.0;
    if (hi == 1 && lo == 0) return 8.0 / 96.0;
    if (hi == 1 && lo == 1) return 6.0 / 96.0;
    if (hi == 2 && lo == 0) return 1.0 / 96.0;
    return 0.0;
  }
  if (kind == LAT_D2Q21) {
    if (hi == 0) return 91.0 / 324.0;
    if (hi == 1 && lo == 0) return 1.0 / 12.0;
    if (hi == 1 && lo == 1) return 2.0 / 27.0;
    if (hi == 2 && lo == 0) return 7.0 / 360.0;
    if (hi == 2 && lo == 2) return 1.0 / 432.0;
    if (hi == 3 && lo == 0) return 1.0 / 1620.0;
    return 0.0;
  }
  // D2Q37
  if (hi == 0) return 0.233150669132352502286506704067;
  if (hi == 1 && lo == 0) return 0.107306091542219002412464287183;
  if (hi == 1 && lo == 1) return 0.0576678598887948820300692153933;
  if (hi == 2 && lo == 0) return 0.0142082161584507502646989423441;
  if (hi == 2 && lo == 1) return 0.00535304900051377523273150166219;
  if (hi == 2 && lo == 2) return 0.00101193759267357547541090850664;
  if (hi == 3 && lo == 0) return 0.000245301027757717345465916643268;
  if (hi == 3 && lo == 1) return 0.000283414252994198217400525294195;
  return 0.0;
}

constexpr bool vel_before(const Vel &a, const Vel &b) {
  const int na = a.x * a.x + a.y * a.y + a.z * a.z;
  const int nb = b.x * b.x + b.y * b.y + b.z * b.z;
  if (na != nb) return na < nb;
  if (a.x != b.x) return a.x < b.x;
  if (a.y != b.y) return a.y < b.y;
  return a.z < b.z;
}

template <int KIND, int Q, int D, int R>
constexpr VelSet<Q> make_set() {
  VelSet<Q> s{};
  int n = 0;
  for (int z = (D == 3 ? -R : 0); z <= (D == 3 ? R : 0); ++z)
    for (int y = -R; y <= R; ++y)
      for (int x = -R; x <= R; ++x)
        if (weight_of(KIND, x, y, z) > 0.0 && n < Q) {
          s.v[n] = Vel{x, y, z};
          ++n;
        }
  // insertion sort into the canonical order
  for (int i = 1; i < n; ++i) {
    Vel key = s.v[i];
    int j = i - 1;
    while (j >= 0 && vel_before(key, s.v[j])) {
      s.v[j + 1] = s.v[j];
      --j;
    }
    s.v[j + 1] = key;
  }
  for (int i = 0; i < Q; ++i) {
    s.w[i] = weight_of(KIND, s.v[i].x, s.v[i].y, s.v[i].z);
    for (int j = 0; j < Q; ++j)
      if (s.v[j].x == -s.v[i].x && s.v[j].y == -s.v[i].y && s.v[j].z == -s.v[i].z) s.opp[i] = j;
  }
  return s;
}

template <int KIND>
struct Lattice;

template <>
struct Lattice<LAT_D2Q9> {
  static constexpr int kind = LAT_D2Q9, D = 2, Q = 9, B = 1;
  static constexpr double cs2 = 1.0 / 3.0;
  static constexpr VelSet<9> S = make_set<LAT_D2Q9, 9, 2, 1>();
};

template <>
struct Lattice<LAT_D3Q27> {
  static constexpr int kind = LAT_D3Q27, D = 3, Q = 27, B = 1;
  static constexpr double cs2 = 1.0 / 3.0;
  static constexpr VelSet<27> S = make_set<LAT_D3Q27, 27, 3, 1>();
};

template <>
struct Lattice<LAT_D2Q13> {
  static constexpr int kind = LAT_D2Q13, D = 2, Q = 13, B = 2;
  static constexpr double cs2 = 0.5;
  static constexpr VelSet<13> S = make_set<LAT_D2Q13, 13, 2, 2>();
};

template <>
struct Lattice<LAT_D2Q21> {
  static constexpr int kind = LAT_D2Q21, D = 2, Q = 21, B = 3;
  static constexpr double cs2 = 2.0 / 3.0;
  static constexpr VelSet<21> S = make_set<LAT_D2Q21, 21, 2, 3>();
};

template <>
struct Lattice<LAT_D2Q37> {
  static constexpr int kind = LAT_D2Q37, D = 2, Q = 37, B = 3;
  static constexpr double cs2 = 0.697953322019683088238409055389;
  static constexpr VelSet<37> S = make_set<LAT_D2Q37, 37, 2, 3>();
};

// host-side description used by the grid builder and the C-ABI
struct LatticeInfo {
  int kind, D, Q, B;
  double cs2;
  int c[37][3];
  double w[37];
  int opp[37];
};

template <int KIND>
inline LatticeInfo lattice_info() {
  using L = Lattice<KIND>;
  LatticeInfo li{};
  li.kind = KIND;
  li.D = L::D;
  li.Q = L::Q;
  li.B = L::B;
  li.cs2 = L::cs2;
  for (int i = 0; i < L::Q; ++i) {
    li.c[i][0] = L::S.v[i].x;
    li.c[i][1] = L::S.v[i].y;
    li.c[i][2] = L::S.v[i].z;
    li.w[i] = L::S.w[i];
    li.opp[i] = L::S.opp[i];
  }
  return li;
}

inline bool get_lattice_info(int kind, LatticeInfo *out) {
  switch (kind) {
    case LAT_D2Q9: *out = lattice_info<LAT_D2Q9>(); return true;
    case LAT_D3Q27: *out = lattice_info<LAT_D3Q27>(); return true;
    case LAT_D2Q21: *out = lattice_info<LAT_D2Q21>(); return true;
    case LAT_D2Q37: *out = lattice_info<LAT_D2Q37>(); return true;
    case LAT_D2Q13: *out = lattice_info<LAT_D2Q13>(); return true;
    default: return false;
  }
}

}  // namespace lbm
