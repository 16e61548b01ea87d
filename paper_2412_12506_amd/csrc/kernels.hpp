// HIP kernels for gfx950 (CDNA4, wave64).
//
// Block-sparse (BSR) operators stream their blocks from HBM once per apply.
// A bs x bs block is stored "row-tiled": entry (r, c) sits at
//     ((c / V) * bs + r) * V + (c % V)
// where V is the vector width in elements (16-byte loads when bs allows), so
// that lane r of a wavefront reads row r of the block V entries at a time and
// one load instruction of the wave covers a contiguous run of memory.
//
// Lane mapping of the fast kernels (bs <= 64): a wavefront processes
// G = 64 / bs block rows at once, lane = (group g, block row r).  The vector
// entry a lane needs from another lane of its group is broadcast with a lane
// read (readlane when G == 1, a lane permute otherwise).  Larger blocks use
// the generic kernels (one lane per scalar row).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ldgmg {

// BF16 storage of a block entry: the upper 16 bits of the FP32 value (rounded
// to nearest even from FP32), widened back to FP32 exactly by a shift.
struct bf16s {
  uint16_t u;
};

// V: entries per vector load (16 bytes where bs allows it)
template <typename T, int BS>
struct BlkCfg {
  static constexpr int V = sizeof(T) == 8   ? (BS % 2 == 0 ? 2 : 1)
                           : sizeof(T) == 4 ? (BS % 4 == 0 ? 4 : 1)
                                            : (BS % 8 == 0 ? 8 : BS % 4 == 0 ? 4 : BS % 2 == 0 ? 2 : 1);
  static constexpr int G = 64 / BS;      // block rows per wavefront
  static constexpr int NV = BS / V;      // vector loads per lane per block
};

}  // namespace ldgmg
