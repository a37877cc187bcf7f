// Rigorous per-tile bound on |screen value - canonical d^2|.
//
// Notation for a row x (canonical vector: the float32 point promoted to double,
// or the FP64 z-normalised window), its screen operand x~ (FP32, BF16 or int8)
// and Delta = x - x~:
//   a = ||x||, at = ||x~||, r = ||Delta||, s^ = fp32(||x||^2).
// The screen value of a pair is  D~ = fl(s^_i + fl(s^_j - 2 G~_ij)),  with G~
// the matrix-core dot product of x~_i and x~_j (FP32 accumulation).
// Exact squared distance: delta^2 = s_i + s_j - 2<x_i, x_j>. Error sources:
//   1. accumulation in the matrix core: |G~ - <x~_i,x~_j>| <= gamma_K at_i at_j
//      (any summation order, one rounding per product and per addition,
//      unit 2^-23 so that truncating hardware is covered too);
//   2. operand rounding: <x,y> - <x~,y~> = <Delta_x, y> + <x~, Delta_y>, so
//      |.| <= r_i a_j + at_i r_j (Cauchy-Schwarz);
//   3. the two FP32 operations of the epilogue: <= 2^-23 (s^_i + s^_j + 2|G~|)
//      (taken with a factor 2 margin as 2^-22);
//   4. s^ vs ||x||^2: FP64 summation then rounding to FP32,
//      <= (2^-24 + gamma_{d+2}(2^-53)) ||x||^2 for each of i and j;
//   5. canonical FP64 d^2 vs exact delta^2: <= gamma_{d+2}(2^-53) (a_i + a_j)^2;
//   6. FP32 subnormal flushing inside the matrix core: < 2^-90 absolute.
// Taking maxima of s^, a, at, r over the rows of tile block I and of block J
// bounds every pair of the tile. The sum is formed in FP64 and scaled by
// (1 + 2^-16), which exceeds the rounding of the bound's own evaluation.
// For the int8 screen every step is exact integer arithmetic and the bound is 0.
//
// Folded form (SCREEN_FOLDED; the 256-row screen): the row scalars enter the
// matrix product itself. Each tile's accumulator starts from one extra
// matrix-core step whose operands carry c = -s^/4 split into three BF16 parts
// (or c = -s^/2 as one FP32 value) against ones, so that the accumulator
// holds fl(-(s^_i + s^_j)/2 + <x~_i, x~_j>) and D~ = -2 * acc (exact). Error
// sources, replacing 1 and 3 above:
//   1'. accumulation of the K products and of the folded terms:
//       <= gamma_K' (at_i at_j + (1 + 2^-6)(s^_i + s^_j)/2), doubled by the -2;
//   3'. the split c~ of c: |c~ - c| <= 2^-27 |c| (three RNE BF16 parts; exact
//       for FP32), i.e. <= 2^-27 (s^_i + s^_j) in D~; counted as 2^-24.
// 2, 4, 5 and 6 are unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpmi {

// Screen value forms: row scalars added in the epilogue, or folded into the
// matrix product (see above).
enum { SCREEN_EPILOGUE = 0, SCREEN_FOLDED = 1 };

__host__ __device__ inline double tile_bound(float4 bI, float4 bJ, int32_t kpad, int64_t d, int prec, int form)
{
    if (prec == 3) return 0.0;  // int8: exact
    const double u32 = 1.0 / 8388608.0;                       // 2^-23
    const double u64 = 1.0 / 9007199254740992.0;              // 2^-53
    const double D = (double)d + 2.0;
    const double g64 = D * u64 / (1.0 - D * u64);
    const double SI = bI.x, AI = bI.y, TI = bI.z, RI = bI.w;
    const double SJ = bJ.x, AJ = bJ.y, TJ = bJ.z, RJ = bJ.w;
    double e;
    if (form == SCREEN_FOLDED) {
        // K products plus at most 12 folded terms, with margin
        const double K = (double)kpad + 16.0;
        const double gK = K * u32 / (1.0 - K * u32);
        e = 2.0 * gK * (TI * TJ + (1.0 + 1.0 / 64.0) * 0.5 * (SI + SJ));   // 1'
        e += (SI + SJ) * (1.0 / 16777216.0);                                  // 3'
    } else {
        const double K = (double)kpad + 2.0;
        const double gK = K * u32 / (1.0 - K * u32);
        e = 2.0 * gK * TI * TJ;                                               // 1
        e += (1.0 / 4194304.0) * (SI + SJ + 2.0 * TI * TJ * (1.0 + gK));     // 3 (2^-22)
    }
    e += 2.0 * (RI * AJ + TI * RJ);                           // 2
    e += (SI + SJ) * (1.0 / 16777216.0 + g64) * (1.0 + 1.0 / 1048576.0); // 4
    e += g64 * (AI + AJ) * (AI + AJ);                         // 5
    e += 0x1p-90;                                             // 6
    return e * (1.0 + 1.0 / 65536.0);
}

// Smallest float >= x (x finite, non-negative or not).
__host__ __device__ inline float f32_up(double x)
{
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

// Largest float <= x.
__host__ __device__ inline float f32_down(double x)
{
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}

// Relative/absolute margin for one FP64 addition or subtraction of a and b.
__host__ __device__ inline double add_margin(double a, double b)
{
    return (fabs(a) + fabs(b)) * 0x1p-50;
}

}  // namespace cpmi
