// Address layout of the 256x256 screen's K slices (shared by the kernel and
// by host-side checks of it).
//
// A slice holds 256 rows x 64 bytes of one operand. It is filled by 16
// direct-to-LDS instructions of 16 bytes per lane: wave w (0..3) issues
// instruction q (0..3) for the 16-row block R0 = (4 w + q) * 16; lane i of it
// writes LDS bytes [R0 * 64 + 16 i, + 16), i.e. row R0 + i / 4, slot i % 4.
// Slot s of row r holds the 16-byte chunk c = s ^ ((r >> 2) & 3) of that row,
// and a fragment read of row r, chunk c looks at slot c ^ ((r >> 2) & 3):
// 16 consecutive rows read at one chunk then cover the 16 combinations of
// (r % 4, slot), i.e. each of the 64 four-byte banks exactly once.
#pragma once

#include <stdint.h>

namespace cpmi {
namespace l256 {

constexpr int SLICE = 64;  // bytes of K per row and slice
constexpr int NQ = 4;      // 16-row blocks per wave and operand

__host__ __device__ inline int swz(int row) { return (row >> 2) & 3; }
// Source of direct-to-LDS load (wave, q, lane): row within the tile and byte
// column within the slice.
__host__ __device__ constexpr int dma_row(int wave, int q, int lane) { return (wave * NQ + q) * 16 + (lane >> 2); }
__host__ __device__ inline int dma_col(int wave, int q, int lane)
{
    return ((lane & 3) ^ swz(dma_row(wave, q, lane))) << 4;
}
// Destination byte in the slice's LDS block.
__host__ __device__ constexpr int dma_lds(int wave, int q, int lane) { return (wave * NQ + q) * 16 * SLICE + lane * 16; }
// Byte position in the LDS block of (row, 16-byte chunk).
__host__ __device__ inline int frag_lds(int row, int chunk) { return row * SLICE + ((chunk ^ swz(row)) << 4); }

// Byte offset, in the screen operand read by the 256-row screen, of byte b of
// row r (rows of `rowbytes` bytes, a multiple of 2 * SLICE). The operand is
// stored slice-major per block of 256 rows: block I holds the 64-byte slice 0
// of its 256 rows (16 KB), then slice 1, and so on. One direct-to-LDS load of
// 16 rows of a slice then reads 1 KB of consecutive memory (whole 128-byte
// lines) instead of half of 16 lines.
__host__ __device__ inline int64_t xs_offset(int64_t r, int64_t b, int64_t rowbytes)
{
    return ((r >> 8) * (rowbytes / SLICE) + b / SLICE) * (256 * SLICE) + (r & 255) * SLICE + (b % SLICE);
}

}  // namespace l256
}  // namespace cpmi
