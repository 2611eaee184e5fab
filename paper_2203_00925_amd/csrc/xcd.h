// Block order for gather kernels on the 8 XCDs of the chip.  Blocks are
// dealt to the XCDs in turn and each XCD has its own L2; with the grid
// padded to a multiple of 8, block b works on logical block
// (b % 8) * (grid / 8) + b / 8, so each XCD takes one contiguous eighth of
// the rows and the neighbour data that consecutive rows share (nearby cells
// of a space-filling-curve order) stays in one L2.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mifvm {

constexpr int kXcds = 8;

__device__ inline int64_t xcd_block() {
    const int64_t per = gridDim.x / kXcds;
    return int64_t(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}
__device__ inline int64_t gtid_m() { return xcd_block() * blockDim.x + threadIdx.x; }
// grid of blocks of `block` threads covering n rows, padded to a multiple of 8
inline unsigned rows_m(int64_t n, int block) {
    const int64_t b = (n + block - 1) / block;
    return unsigned((b + kXcds - 1) / kXcds * kXcds);
}

}  // namespace mifvm
