// Host-visible launchers of the demapping kernels (defined next to each kernel).
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace dm {

// Table row stride used by the kernels for a dimensionality D (1..8 exact, else 16 or 32).
int padded_dim(int D);

// Symbols per tile of the FP32 kernel (one lane per symbol).
int valu_tile_symbols();

// FP32 direct-difference demapper (one lane per symbol, persistent grid).
hipError_t launch_demap_valu(const LaunchArgs& a, int grid, hipStream_t st);

// Exact recomputation of the queued (symbol, bit) pairs whose far-subset sum underflowed.
hipError_t launch_fixup(const LaunchArgs& a, int grid, hipStream_t st);

}  // namespace dm
