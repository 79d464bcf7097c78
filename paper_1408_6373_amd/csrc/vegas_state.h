// vegas_state.h -- a Vegas integral's state file (checkpoint and resume).
#pragma once
#include <string>
#include <vector>

#include "vegas_engine.h"

namespace ccuba {

// What a state file holds besides the settings it was written for: the
// state after its last iteration, the grid, and the per-iteration history.
struct StateFile {
  VState st{};
  std::vector<double> grid, I, var;
};

// Read `path' for the integral `sp'.  Returns 1 when there is no such file,
// 0 when `out' holds its contents, CCUBA_EINVAL when the file is unreadable
// or was written for other settings (dimension, bins, integrand, precision,
// flags, seed, stream, nstart, nincrease).
int state_read(const char *path, const VegasSpec &sp, StateFile &out);
// Write `path' atomically (a temporary file renamed over it).  CCUBA_EINVAL
// when it cannot be written.
int state_write(const char *path, const VegasSpec &sp, const StateFile &sf);

}  // namespace ccuba
