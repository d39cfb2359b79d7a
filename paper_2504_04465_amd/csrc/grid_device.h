// grid_device.h -- the refined grid and its brick layout built on the GPU
// (Secs. 4.3-4.4 construction, Sec. 8 remeshing without the host tree
// build).  The result is the same HostGrid and DeviceLayout, value for
// value, as build_grid + build_layout produce on the host; the device
// arrays are copied back into them at the end.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "grid_builder.h"
#include "layout.h"
#include "lattice.h"

namespace lbm {

// device memory for the builder's temporaries (released before return)
struct DevAlloc {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*release)(void *p, void *ctx);
  void *ctx;
};

// Canonical tables the caller keeps on the device (allocated through the
// DevAlloc, owned by the caller): the coordinates and the neighbour list are
// then not copied into the HostGrid (its xyz and nbr stay empty; fetch them
// with fetch_host_mirror when a host reader needs them).  The caller may
// release nbr once it has formed the per-slot flags.
struct DeviceGridArrays {
  int32_t *xyz = nullptr;     // [n][3]
  int8_t *lev = nullptr;      // [n]
  uint8_t *flag = nullptr;    // [n] canonical flags
  int32_t *nbr = nullptr;     // [Q-1][n] canonical values
  int32_t *slot_of = nullptr; // [n]
  int64_t n = 0;
  int Qm = 0;
};

// Same arguments and validation as build_grid (periodic[a]: both faces of
// axis a are periodic).  Returns 0, -1 (argument error), -2 (mask error) or
// -3 (device allocation or runtime failure); *err receives the text.
// keep (may be null) receives the device tables above.  Synchronises the
// stream.
int build_grid_device(const LatticeInfo &lat, int dim, const int32_t ext[3], int L, const MaskView *refine,
                      const MaskView *solid, const FaceSpec faces[6], const bool periodic[3], const DevAlloc &da,
                      hipStream_t stream, HostGrid *g, DeviceLayout *y, DeviceGridArrays *keep, std::string *err);

// g->xyz and g->nbr from the kept device tables, where kept and not yet on
// the host.
int fetch_host_mirror(const DeviceGridArrays &dg, HostGrid *g, hipStream_t stream, std::string *err);

// per-slot device flags: the canonical flag, F_MOVING where a population is
// pulled from a moving wall, F_HOLE for slots without a cell
void launch_slot_flags(const DeviceGridArrays &dg, int64_t nslot, uint8_t *out, hipStream_t stream);

// remesh_sources on the device: for every cell of `nw` its sources among
// the flow cells (not fine ghosts) of `old`, same order and weights value
// for value, from the two grids' kept device tables (coordinates, levels,
// flags).  *off [n_new + 1], *src, *wt are device arrays from `da` that
// the caller releases.  Returns 0, -1 with *err set when a new cell covers
// no old flow cell (the lowest such cell is named), -3 on a device failure.
int remesh_sources_device(const HostGrid &old, const DeviceGridArrays &dold, const HostGrid &nw,
                          const DeviceGridArrays &dnew, const DevAlloc &da, hipStream_t stream, int64_t **off,
                          int32_t **src, double **wt, std::string *err);

}  // namespace lbm
