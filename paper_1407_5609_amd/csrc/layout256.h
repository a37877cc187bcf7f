// Address layout of the 256x256 screen's K slices (shared by the kernel and
// by host-side checks of it).
//
// A slice holds 256 rows x 128 bytes of one operand. It is filled by
// 32 direct-to-LDS instructions of 16 bytes per lane: wave w (0..3) issues
// instruction q (0..7) for the 8-row block R0 = (8 w + q) * 8; lane i of it
// writes LDS bytes [R0 * 128 + 16 i, + 16), i.e. row R0 + i / 8, slot i % 8.
// Slot s of row r holds the 16-byte chunk c = s ^ (r & 7) of that row, so a
// lane loads global chunk (i % 8) ^ (i / 8) of its row (R0 is a multiple of 8).
// A fragment read of row r, chunk c therefore looks at slot c ^ (r & 7).
#pragma once

#include <stdint.h>

namespace cpmi {
namespace l256 {

constexpr int SLICE = 128;  // bytes of K per row and slice

// Source of direct-to-LDS load (wave, q, lane): row within the tile and byte
// column within the slice.
__host__ __device__ inline int dma_row(int wave, int q, int lane) { return (wave * 8 + q) * 8 + (lane >> 3); }
__host__ __device__ inline int dma_col(int lane) { return (((lane & 7) ^ (lane >> 3)) << 4); }
// Destination byte in the slice's LDS block.
__host__ __device__ inline int dma_lds(int wave, int q, int lane) { return (wave * 8 + q) * 8 * SLICE + lane * 16; }
// Byte position in the LDS block of (row, 16-byte chunk).
__host__ __device__ inline int frag_lds(int row, int chunk) { return row * SLICE + ((chunk ^ (row & 7)) << 4); }

}  // namespace l256
}  // namespace cpmi
