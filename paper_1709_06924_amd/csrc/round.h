// A round of segmented launches for a batch of problems (the serving loop).
//
// Each problem of the batch records the launches of its next step -- in its
// own order, which is always a subsequence of the fixed kernel order below
// (history push, direction passes, trial point, grid build, cell geometry,
// quadrature, reductions, scalar gather) -- and issue() then makes one
// launch per kernel for all problems that recorded it: blockIdx.y selects
// the problem, whose arguments and own grid size come from one table copied
// to the device in a single transfer.  Every problem's blocks run exactly
// what its own single launch would, so its results do not depend on the
// batch.  The round ends with one gather of every problem's scalars into
// pinned host memory and one stream synchronisation.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <utility>
#include <vector>

#include "kernels.h"
#include "lbfgs.h"

namespace scvt {

// copy of `count` device doubles of one problem into the round's scalars
struct GatherArgs {
  const double* src;
  double* dst;  // device staging
  int count;
};

struct Round {
  std::vector<PushExtArgs> push_ext[2];  // by vector width (index vw - 1)
  std::vector<FinChain> fin_chain;
  std::vector<HistFinArgs> fin_back, fin_fwd, fin_gq;
  std::vector<HistPassArgs> q0[2], dir[2];
  std::vector<NormArgs> norm;
  std::vector<GridBuildArgs> grid;
  std::vector<CellArgs> cells;  // main path (certified passes, then fallback)
  std::vector<CellArgs> cells_all;  // small problems: every cell by the fallback
  std::map<std::pair<int, int>, std::vector<CellArgs>> quad;  // by (variant, mixed)
  std::vector<EvalRedArgs> reduce;
  std::vector<FinalizeArgs> fin;
  struct Out {
    const double* src;
    int count;
    double* host;  // where the gathered values go after the round
  };
  std::vector<Out> out;

  bool empty() const;
  void clear();
};

// Device and pinned staging of the rounds (one per server).
struct RoundBuffers {
  void* dev = nullptr;     // argument tables and grid sizes
  void* host = nullptr;    // pinned mirror
  size_t bytes = 0;
  double* dscal = nullptr;  // gathered scalars (device)
  double* hscal = nullptr;  // pinned
  int max_scal = 0;
};

// Issue the round on stream s and wait for it; the recorded scalars are
// then in their host destinations.  Returns a hipError_t value.
hipError_t round_run(Round& r, RoundBuffers& b, hipStream_t s);

// launch of the scalar gather (round.hip)
hipError_t launch_gather_many(const Seg<GatherArgs>& g, hipStream_t s);

}  // namespace scvt
