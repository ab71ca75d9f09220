// tune.h -- autotuner of the step kernels' tile shape (tune.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

namespace lbm {

// A candidate shape: vx, nw, flags as in lbm_set_tile; h = rows per
// workgroup (march form) or tiles per work item (batched kernels); ch =
// items per XCD chunk of the batched kernels (0 for single lattices).
struct TileCand {
    int vx, nw, h, flags, ch;
};

std::string device_arch();
bool tune_cache_get(const std::string& key, TileCand* out);
void tune_cache_put(const std::string& key, const TileCand& c, float us);
std::vector<TileCand> lattice_candidates(int dtype);
std::vector<TileCand> pool_candidates(int dtype);
int time_candidates(const std::vector<TileCand>& cands, int reps, hipStream_t st,
                    const std::function<hipError_t(const TileCand&)>& launch, float* best_us);

}  // namespace lbm
