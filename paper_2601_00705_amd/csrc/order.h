// order.h -- argument block and launcher of the spatial storage order of a
// map (Morton cells, stable radix ranking, brick interleave).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsr {

#define GSR_RADIX_TILE 4096  // keys per block of a radix pass (256 threads x 16)
#define GSR_RADIX_BITS 8     // digit width; four passes cover the 31-bit codes
#define GSR_BOX_BLOCKS 256   // blocks of the box pass, one partial box each

// Workspace: two (code, value) buffers of n entries, the radix counts
// [256][blocks], the digit totals and the partial boxes.
struct OrderArgs {
    int64_t n;
    const float* mean;   // [3][n]
    uint32_t* box;       // [GSR_BOX_BLOCKS][8]: order-preserving images of lo x, y, z, then hi x, y, z
    uint32_t* code[2];   // [n] each: keys, ping-pong between passes
    uint32_t* val[2];    // [n] each: Gaussian indices, ping-pong
    uint32_t* hist;      // [256][blocks]: per-block digit counts, then their offsets within the digit
    uint32_t* tot;       // [256]: keys per digit of the pass
    int32_t blocks;      // radix tiles of GSR_RADIX_TILE keys
    int32_t brick;
    int64_t full;        // n / brick
    int64_t mult;        // the brick multiplier P
    int32_t* index;      // [n] out
};

hipError_t launch_spatial_order(const OrderArgs& a, hipStream_t s);

}  // namespace gsr
