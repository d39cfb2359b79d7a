// remesh.h -- sources of the cells of a new tree in an old one (mesh
// adaptation, Sec. 8) and the device kernel that moves the state across.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <string>
#include <vector>

namespace lbm {

struct HostGrid;

// For every cell of `nw`, its sources among the cells of `old` other than
// fine ghosts (they tile the domain; in an overlap band the coarse ghost
// carries the state): the old cell at the same place and level, or
// the old cell that contains it (uniform explosion), or the old cells inside
// it with weights proportional to their volume (coalescence).  CSR layout:
// cell j reads src[off[j] .. off[j+1]) with weights wt.  Returns 0, or -1
// with *err set when a new cell covers no old flow cell.
int remesh_sources(const HostGrid &old, const HostGrid &nw, std::vector<int64_t> *off, std::vector<int32_t> *src,
                   std::vector<double> *wt, std::string *err);

// out[r][j] = sum_k wt[k] old[r][src[k]], k in [off[j], off[j+1]), r < rows
void launch_remap(const double *old, int64_t n_old, double *out, int64_t n_new, int rows, const int64_t *off,
                  const int32_t *src, const double *wt, hipStream_t s);

}  // namespace lbm
