// Host-visible launchers of the demapping kernels (defined next to each kernel).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"

namespace dm {

// Table row stride used by the kernels for a dimensionality D (1..8 exact, else 16 or 32).
int padded_dim(int D);

// Symbols per tile of the FP32 kernel (one lane per symbol).
int valu_tile_symbols();
int hard_tile_symbols();
hipError_t launch_hard_demap(const HardArgs& a, int grid, hipStream_t st);
int hard_mfma_block_symbols();
// MFMA decisions (split-FP16 operand table `frag` of the label-order points, r_max = max ||x||);
// ambiguous symbols go to `queue` (FixEntry n = symbol, tag = block) for launch_hard_fix.
hipError_t launch_hard_mfma(const HardArgs& a, const void* frag, float r_max, FixEntry* queue, uint32_t* qcount,
                            uint32_t qcap, int grid, hipStream_t st);
hipError_t launch_hard_fix(const HardArgs& a, const FixEntry* queue, const uint32_t* qcount, uint32_t qcap, int grid,
                           hipStream_t st);

// FP32 direct-difference demapper (one lane per symbol, persistent grid).
hipError_t launch_demap_valu(const LaunchArgs& a, int grid, hipStream_t st);

// Exact recomputation of the queued (symbol, bit) pairs whose far-subset sum underflowed.
hipError_t launch_fixup(const LaunchArgs& a, int grid, hipStream_t st);
// Exponent cache of the fix-up kernel (per wave, 4 waves per block) for an M-point constellation,
// and the blocks per CU that fit it within 160 KiB of LDS and the kernel's 8 waves per SIMD.
inline int fixup_cache_points(int M) { return M <= kFixCached ? ((M + 63) / 64) * 64 : 64; }
inline size_t fixup_lds_bytes(int M) { return (size_t)4 * fixup_cache_points(M) * sizeof(float); }
inline int fixup_blocks_per_cu(int M) { return (int)std::min<size_t>(8, (160 * 1024) / (fixup_lds_bytes(M) + 1024)); }

// K slots (multiple of 16) of the MFMA operand vectors for dimensionality D.
int mfma_slots(int D, bool split);

// Symbols per block iteration of the MFMA kernel.
int mfma_block_symbols();

// MFMA demapper specialised for M = 32..256 points and D in {2, 4, 8} (tile count and label
// bits known at compile time); hipErrorNotSupported for other shapes.
bool mfma_small_supported(int M, int D);
hipError_t launch_demap_mfma_small(const LaunchArgs& a, int prec, const void* frag, const void* pv, int grid,
                                   hipStream_t st);

// MFMA demapper: prec 1 = BF16, 2 = FP16, 3 = BF16 split, 4 = FP16 split.  `frag` is the
// point-side operand table in fragment order ([tile][mfma][lane] x 16 bytes); `pv` the same
// operands per label ([label][K slots], 16-bit), read for the transmitted points.
hipError_t launch_demap_mfma(const LaunchArgs& a, int prec, const void* frag, const void* pv, int grid, hipStream_t st);

// Symbols per work item of the batched kernel for an instance kind (kKindValu / kKindMfma).
int batched_tile_symbols(int kind);

// Allow the batched kernel of a precision its 128 KiB of dynamic LDS (call before launching or
// capturing it).
hipError_t prepare_batched(int prec);

// Persistent batched kernel (prec selects the MFMA operand variant used by MFMA instances).
hipError_t launch_demap_batched(const BatchArgs& a, int prec, int grid, hipStream_t st);

// Fix-up of queued symbols of any instance (tables with row stride 8).
hipError_t launch_batched_fixup(const BatchArgs& a, int grid, hipStream_t st);

// p[0..n) = 0 with a kernel (usable inside a captured graph).
hipError_t launch_zero_words(uint32_t* p, size_t n, hipStream_t st);

}  // namespace dm
