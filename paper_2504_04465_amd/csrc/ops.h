// ops.h -- argument blocks and launcher table shared by the host scheduler
// and the per-lattice kernel translation units.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace lbm {

enum CollisionKind { COLL_BGK = 0, COLL_RR = 1, COLL_DDF_POLY = 2, COLL_DDF_NEWTON = 3,
                     COLL_DDF_MLP = 4, COLL_DDF_MLP_NEWTON = 5 };
enum StorageKind { STO_FP64 = 0, STO_FP32 = 1, STO_FP16 = 2 };

// device counters (unsigned long long), CNT_COPIES copies of CNT_COUNT (one
// 64-byte line each): a block adds to copy blockIdx mod CNT_COPIES, the host
// sums the copies.  Every Newton cell counts its solve; with one copy, the
// atomics of all wavefronts of the device queued on a single line and took
// two thirds of the D2Q21 collide's time.
enum { CNT_NEWTON_CALLS = 0, CNT_NEWTON_ITERS = 1, CNT_NEWTON_FAIL = 2, CNT_NONFINITE = 3,
       CNT_MLP_FALLBACK = 4, CNT_HIST0 = 8, NHIST = 16, CNT_COUNT = 32, CNT_COPIES = 1024 };

constexpr int NLAM = 8;
// Population storage: the slots are grouped in chunks of PCH = 2^PCH_SH
// slots (64 bricks); a chunk holds its slots' population 0, then population
// 1, ..., so element (i, s) of a Q-population buffer is at
// ((s >> PCH_SH) * Q + i) * PCH + (s mod PCH).  The Q rows a wavefront reads
// and writes then lie within Q * PCH values instead of being a whole buffer
// apart, which the DRAM serves faster (about 10 % for the D3Q27 pull).  A
// buffer of stride slots (a multiple of PCH) holds Q * stride values.
constexpr int PCH_SH = 12;
constexpr int64_t PCH = (int64_t)1 << PCH_SH;
// conserved sums: at most SUM_BLOCKS blocks per level, each striding over
// the level's tiles, write one partial of the six quantities each; the
// partials of level l start at l * SUM_BLOCKS * 6
constexpr int SUM_BLOCKS = 1024, SUM_LEVELS = 8, SUM_Q = 6;
constexpr int SUM_PARTIALS = SUM_LEVELS * SUM_BLOCKS * SUM_Q;
constexpr int MLP_IN = 4, MLP_HID = 64, MLP_OUT = 8;

struct FaceVals {
  double rho[6], u[6][3], T[6];
  int extrap[6];
};

struct PhysArgs {
  double tau;          // relaxation time of the level
  double omega, krr;   // 1 / tau and 1 - 1 / tau, formed on the host
  double cs2w;         // denominator of the moving-wall term (cs2, or T0 for DDF)
  double uw[6][3];     // moving-wall velocity per face
  double Cv, sensor_A; // DDF
  int sensor_on, trace_eq;
  double newton_tol, fallback_tol;
  int newton_max_it, warm;
  const void *mlp;     // MLP operand block (device), or null
};

// pull topology of the slots: bricks of 64 slots with their neighbour
// bricks, and explicit rows for the cells the brick arithmetic does not give
struct Topo {
  const int32_t *nbrick;   // [bricks][row] neighbour brick ids (slot / 64)
  const uint64_t *xmask;   // [bricks] lanes with an exception row
  const int32_t *xbase;    // [bricks] first exception row of the brick
  const int32_t *xnbr;     // [Q-1][xstride] pull sources of the exception rows
  const uint64_t *xreg;    // [rows] bit i: the row's source of population i is the bulk gather's
  int64_t xstride;
  const double *xdu;       // [Q-1][xstride] xi_i . (inflow noise) of the rows, or null
  int off32;               // population buffers under 4 GB: the steady-state pull uses 32-bit byte offsets
};

// the collides of every level active at a substep in one launch: what
// differs between the levels (the rest of KArgs is common to them)
constexpr int MAX_LEVELS = 8;
struct MultiTable {
  int n;                    // active levels in the launch; 0: a per-level launch
  int parity[MAX_LEVELS];   // input buffer of each active level
  const void *f[2], *g[2];  // the two population buffers
  int64_t begin[MAX_LEVELS], count[MAX_LEVELS];
  double tau[MAX_LEVELS], omega[MAX_LEVELS], krr[MAX_LEVELS];
  int64_t block0[MAX_LEVELS + 1];  // first block of each (multiples of 8); block0[n] = grid size
};

// collide-and-stream of the slots [begin, begin + count) of one level
// (begin and count are multiples of 64)
struct KArgs {
  const void *fin;
  void *fout;
  const void *gin;
  void *gout;
  int64_t stride;      // slots per buffer (a multiple of PCH), and the SoA stride of lam
  int64_t vbase;       // first virtual (coalesced) slot
  Topo topo;
  const uint8_t *flags;
  const double *sigma, *rho_inf; // sponge (may be null)
  void *lam;           // multipliers [8][stride] (DDF_NEWTON family): FP64 for
                       // FP64 population storage, FP32 otherwise
  int64_t begin, count;
  PhysArgs ph;
  unsigned long long *counters;
  int aa;              // in-place streaming: 0 off, 1 even step, 2 odd step
  // in place on a refined grid: slot -> coalesced slot of a coarse ghost
  // (-1 elsewhere); a ghost leaves its post-collision populations there,
  // row i, for the explosion
  const int32_t *gslot;
  MultiTable multi;    // n > 0: every active level of a substep in one launch
};

// coalescence of the unknown populations of one level's coarse ghosts
struct CArgs {
  const void *fin_child;  // newest buffer of the fine level
  const void *gin_child;
  void *fout_coarse;      // newest buffer of the coarse level (virtual slots)
  void *gout_coarse;
  void *lam;           // multipliers, element type as in KArgs
  int64_t stride, vbase;
  const int32_t *xnbr;      // exception rows (children of coarse ghosts have one)
  int64_t xstride;
  const double *xdu;        // inflow noise of the rows, or null
  const int32_t *child;     // [ghost][2^D] child slots
  const int32_t *crow;      // [ghost][2^D] exception rows of the children
  const uint64_t *unknown;  // [ghost]
  const int32_t *ghost_cell;
  int64_t g0, count;        // ghosts [g0, g0 + count)
  double cs2w, uw[6][3];
  int ngrp;                 // population groups per child (set by the launcher)
  // in-place streaming: aa = 2 when the fine level's rows are swapped (odd
  // phase: the children are read as a swapped pull); swap = 1 when the
  // coarse level's are (the coalesced population i goes to row opp(i))
  int aa, swap;
};

// uniform explosion of coarse-ghost post-collision states into the children
struct EArgs {
  const void *fin_coarse;
  void *fout_fine;
  const void *gin_coarse;
  void *gout_fine;
  void *lam;           // multipliers, element type as in KArgs
  int64_t stride;
  const int32_t *child, *ghost_cell;
  int64_t g0, count;
  // in-place streaming (mode 0: two buffers): the coarse ghost's
  // post-collision populations are read from its coalesced slot (vbase +
  // ghost index, where its collide left them); mode 1, the fine level is at
  // an odd phase: child row opp(i) takes population i; mode 2, even phase:
  // population i goes to row i of the cell that pulls it from the child
  // (through the child's exception row), the bounce-back into the child's
  // own row opp(i) with the moving-wall term
  int mode;
  int64_t vbase, xstride;
  const int32_t *xnbr, *crow;
  double cs2w, uw[6][3];
};

// boundary-layer fill after the collision of one level
struct BArgs {
  void *f;
  void *g;
  void *lam;           // multipliers, element type as in KArgs
  int64_t stride;
  const int32_t *bc_cell, *bc_src;
  const int8_t *bc_face;
  int64_t b0, count;
  FaceVals fv;
  PhysArgs ph;
  unsigned long long *counters;
  // in-place streaming (mode 0: two buffers): the source cell's
  // post-collision populations are in its own rows opp(i) (mode 1, odd
  // phase) or in its staging slot stage[src] (mode 2, even phase); the
  // boundary cell's populations are written as its own store would leave
  // them: rows opp(i) (mode 1), or pushed through its exception row
  // bc_row[k] (mode 2)
  int mode;
  const int32_t *stage, *bc_row;
  const int32_t *xnbr;
  int64_t xstride;
};

// gathers of the synchronisation-point state: moments, populations, sums
struct MArgs {
  const void *fin;
  const void *gin;
  const void *lam;
  int64_t stride, vbase;
  Topo topo;
  const uint8_t *flags;
  const int32_t *cell_of;  // [slot] canonical cell, -1 for holes
  int64_t begin, count;    // slots
  double cs2w, uw[6][3], Cv;
  int mode;            // k_gather: 0 moments, 1 populations (+ multipliers),
                       // 3 populations of listed cells (k_sums: sums)
  const int32_t *cells_list;  // mode 3: canonical cells, entries [list_begin, list_begin + count)
  const int32_t *slot_of;     // mode 3: slot of a canonical cell
  int64_t list_begin;
  double *out;         // moments [n_mom][n] / populations [Q][n] (g after)
  double *lam_out;     // [8][n]
  int64_t n;
  double vol;          // cell volume 2^(-D l) for sums
  double *partials;    // k_sums: [gridDim.x][6] block partials
  int aa;              // 2: in-place buffer after an even step (rows swapped)
};

// initialisation from moments, or restore of a raw state
struct IArgs {
  void *f;
  void *g;
  void *lam;           // multipliers, element type as in KArgs
  int64_t stride, n;
  const int32_t *slot_of;  // [n] slot of a canonical cell
  const double *src;   // moments [n_mom][n] or populations [Q][n]
  const double *src_g, *src_lam;
  int mode;            // 0: equilibrium from moments, 1: raw populations
  PhysArgs ph;
  unsigned long long *counters;
};

struct Ops {
  void (*collide)(const KArgs &, bool pre, hipStream_t);
  // all active levels in one launch (steady state: no pre-collision input,
  // two buffers); null where the model keeps per-level launches
  void (*collide_multi)(const KArgs &, hipStream_t);
  int collide_block;        // threads per collide block
  void (*coalesce)(const CArgs &, bool pre_child, hipStream_t);
  void (*explode)(const EArgs &, hipStream_t);
  void (*bcfill)(const BArgs &, hipStream_t);
  void (*gather)(const MArgs &, bool pre, hipStream_t);
  void (*sums)(const MArgs &, bool pre, hipStream_t);  // sum_blocks(a.count) blocks of k_sums
  void (*init)(const IArgs &, hipStream_t);
  void (*sensor)(const MArgs &, const PhysArgs &, bool pre, hipStream_t);
  int sizeof_storage;
};

// blocks of the k_sums launch over `count` slots
inline int sum_blocks(int64_t count) {
  const int64_t t = (count + 255) / 256;
  return (int)(t < SUM_BLOCKS ? t : SUM_BLOCKS);
}

// final reduction of the conserved sums: out[k] = sum over levels l <
// n_levels and blocks b < nb[l] of partials[(l * SUM_BLOCKS + b) * 6 + k],
// in that order (one thread per quantity); enqueued on the stream
void launch_sum_partials(const double *partials, const int *nb, int n_levels, double *out, hipStream_t s);

// device address of the current GPU's static array of SUM_PARTIALS + SUM_Q
// doubles (looked up once per device, with that device current)
hipError_t sums_scratch(double **out);

bool get_ops_d2q9(int coll, int storage, Ops *out);
bool get_ops_d3q27(int coll, int storage, Ops *out);
bool get_ops_d2q21(int coll, int storage, Ops *out);
bool get_ops_d2q37(int coll, int storage, Ops *out);
bool get_ops_d2q13(int coll, int storage, Ops *out);

}  // namespace lbm
