// Host interface of the persistent multi-frame decode kernel.
#pragma once

#include "network.h"

namespace pswa {

struct PersistArgs {
  NetDims x;
  DevWeights w;
  PassCtx c;               // buffers; M, gpos and fid are set per step
  const int* row_start;    // [T+1]: rows of global step t are [row_start[t], row_start[t+1])
  const int* gpos_all;     // global position of each row
  const int* fid_all;      // frame of each row
  int T;
  unsigned* bar;           // barrier arrivals (zeroed before each launch)
  int* abort_flag;         // set when a barrier wait exceeds spin_limit
  long spin_limit;
};

size_t persistent_lds_bytes(const NetDims& x, int prec);
// Largest grid whose blocks can all be resident at once (0 on error).
int persistent_max_grid(const NetDims& x, int prec);
void launch_persistent(const PersistArgs& P, int grid, hipStream_t s);
void zero_ints(int* p, int n, hipStream_t s);

}  // namespace pswa
