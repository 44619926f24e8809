// mlp_device.h -- learned eddy-viscosity closure on the device (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lbm.h"
#include "lbm_device.h"

namespace lbmx {

// bytes of the device-side closure parameters (packed from the blob)
constexpr size_t kMlpDeviceBytes = 32768;

// Validate a closure blob and pack it into the device layout (dev:
// kMlpDeviceBytes) and the step's kernel-argument scalars (mc).  false with
// a reason for a bad magic, version, shape or size.
bool mlp_pack_blob(const void *blob, size_t nbytes, void *dev, MlpConst *mc, std::string *why);

// fused step with the learned closure: a persistent kernel of `grid` blocks
// (mlp_launch_grid: the blocks that fit on the device at once, a multiple of
// 8 so that each block's tiles stay on its XCD, at most ntiles)
hipError_t mlp_launch_grid(int storage, int flags, int ntiles, int *grid);
hipError_t launch_step_mlp(int storage, const StepArgs &a, int bx, int bz, int grid,
                           hipStream_t s);

// cells of the step with the given parity that fell back to Smagorinsky
lbm_status mlp_fallback_count(const void *dev, int parity, int64_t *count, hipStream_t s);

}  // namespace lbmx
