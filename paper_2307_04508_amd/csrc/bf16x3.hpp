// BF16x3 contraction core shared by the polarizability SYRK and the B.W.B
// self-energy contraction.
//
// Each FP32 operand x is held as two BF16 numbers, hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest), and a product as
// hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16 (the lo*lo term and the
// split residuals cost at most 3 * 2^-18 of |x y|).  The split is made once
// per operand by a preparation kernel into library workspace, k-contiguous
// ([row][k], rows and k zero-padded to whole tiles), so the contraction
// kernels copy their tiles global -> LDS directly (global_load_lds, 16 bytes
// per lane) and run no conversion on the VALU.
//
// Tiles: 128 rows of A x 128 rows of B x 32 k per stage, 4 waves of 64 x 64
// (2 x 2 MFMA blocks of 32 x 32, three products each per 16 k).  An LDS tile
// row holds 32 k = 64 bytes in four 16-byte chunks; chunk c of row r is
// stored at position c ^ ((r >> 2) & 3), so the 16-byte operand reads of
// 16 consecutive rows hit 16 distinct bank groups.
#pragma once

#include "common.hpp"

namespace b3 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128;           // tile rows (A and B)
constexpr int BK = 32;            // k per stage
constexpr int NT = 256;           // threads per workgroup
constexpr int TILE = BM * BK;     // bf16 elements of one operand tile

// One pipeline stage of LDS: A hi, A lo, B hi, B lo (8 KB each).
struct Stage {
  __bf16 t[4][TILE];
};

// Copy rows row0 .. row0 + 127, k0 .. k0 + 31 of a split array (row stride
// ld elements, 16-byte aligned rows) into an LDS tile.  Each wave issues two
// instructions of 16 rows x 64 bytes; lane l fills LDS row 16 b + (l >> 2),
// chunk position l & 3, with the global chunk that position holds.
__device__ __forceinline__ void load_tile(const __bf16* __restrict__ g, int64_t ld,
                                          int64_t row0, int64_t k0, __bf16* lds, int wave,
                                          int lane) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int blk = wave * 2 + h;
    const int r = blk * 16 + (lane >> 2);
    const int cg = (lane & 3) ^ ((r >> 2) & 3);
    const __bf16* src = g + (row0 + r) * ld + k0 + 8 * cg;
    __builtin_amdgcn_global_load_lds(src, lds + blk * 16 * BK, 16, 0, 0);
  }
}

// The MFMA operand of row r, k chunk kc (8 consecutive k) of an LDS tile.
__device__ __forceinline__ bf16x8 frag(const __bf16* lds, int r, int kc) {
  return *reinterpret_cast<const bf16x8*>(lds + r * BK + 8 * (kc ^ ((r >> 2) & 3)));
}

// acc[i][j] += A rows (wy 64 + i 32 ..) x B rows (wx 64 + j 32 ..) over the
// 32 k of one stage, three BF16 products per term.
__device__ __forceinline__ void stage_mfma(const Stage& s, f32x16 (&acc)[2][2], int wy, int wx,
                                           int lane) {
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const int kc = 2 * ks + (lane >> 5);
    bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ra = wy * 64 + i * 32 + (lane & 31);
      const int rb = wx * 64 + i * 32 + (lane & 31);
      ah[i] = frag(s.t[0], ra, kc);
      al[i] = frag(s.t[1], ra, kc);
      bh[i] = frag(s.t[2], rb, kc);
      bl[i] = frag(s.t[3], rb, kc);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      }
  }
}

// Round-to-nearest split of x into hi + lo.
__device__ __forceinline__ void split(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

}  // namespace b3
