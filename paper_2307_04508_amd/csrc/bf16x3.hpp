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
// Tiles: 128 rows of A x 128 rows of B x BK k per stage (BK = 32 or 16),
// 4 waves of 64 x 64 or 8 waves of 64 x 32 (MFMA blocks of 32 x 32, three
// products each per 16 k).  An LDS tile row holds BK k in 16-byte chunks, XOR-swizzled by the
// row (32 k: position c ^ ((r >> 2) & 3); 16 k: c ^ ((r >> 3) & 1)), so the
// 16-byte operand reads of 16 consecutive rows hit 16 distinct bank groups.
#pragma once

#include "common.hpp"

namespace b3 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128;           // tile rows (A and B)
constexpr int NT = 256;           // threads per workgroup

// One pipeline stage of LDS for BKT k per stage: A hi, A lo, B hi, B lo.
template <int BKT>
struct StageT {
  __bf16 t[4][BM * BKT];
};
constexpr int BK = 32;            // the default stage depth
using Stage = StageT<BK>;

// Swizzled 16-byte chunk position of chunk c in tile row r.
template <int BKT>
__device__ __forceinline__ int swz(int r, int c) {
  return BKT == 32 ? (c ^ ((r >> 2) & 3)) : (c ^ ((r >> 3) & 1));
}

// Copy rows row0 .. row0 + 127, k0 .. k0 + BKT - 1 of a split array (row
// stride ld elements, 16-byte aligned rows) into an LDS tile of BKT-element
// rows, with NW waves.  A wave instruction fills 1 KB: 16 rows of 32 k (lane
// l: row l >> 2, position l & 3) or 32 rows of 16 k (row l >> 1, position
// l & 1); each position receives the global chunk the swizzle stores there.
template <int BKT, int NW = 4>
__device__ __forceinline__ void load_tile(const __bf16* __restrict__ g, int64_t ld,
                                          int64_t row0, int64_t k0, __bf16* lds, int wave,
                                          int lane) {
  constexpr int CH = BKT / 8;                 // 16-byte chunks per tile row
  constexpr int ROWS = 64 / CH;               // rows per wave instruction
  constexpr int PER_WAVE = BM / ROWS / NW;    // instructions per wave
  static_assert(PER_WAVE >= 1, "too many waves for the tile");
#pragma unroll
  for (int h = 0; h < PER_WAVE; ++h) {
    const int blk = wave * PER_WAVE + h;
    const int r = blk * ROWS + lane / CH;
    const int cg = swz<BKT>(r, lane % CH);    // the swizzle is an involution
    const __bf16* src = g + (row0 + r) * ld + k0 + 8 * cg;
    __builtin_amdgcn_global_load_lds(src, lds + blk * ROWS * BKT, 16, 0, 0);
  }
}

// The MFMA operand of row r, k chunk kc (8 consecutive k) of an LDS tile.
template <int BKT>
__device__ __forceinline__ bf16x8 frag(const __bf16* lds, int r, int kc) {
  return *reinterpret_cast<const bf16x8*>(lds + r * BKT + 8 * swz<BKT>(r, kc));
}

// acc[i][j] += A rows (ar + 32 i ..) x B rows (br + 32 j ..) over the BKT k
// of one stage, three BF16 products per term.
template <int BKT, int WI, int WJ>
__device__ __forceinline__ void stage_mfma(const StageT<BKT>& s, f32x16 (&acc)[WI][WJ], int ar,
                                           int br, int lane) {
#pragma unroll
  for (int ks = 0; ks < BKT / 16; ++ks) {
    const int kc = 2 * ks + (lane >> 5);
    bf16x8 ah[WI], al[WI], bh[WJ], bl[WJ];
#pragma unroll
    for (int i = 0; i < WI; ++i) {
      ah[i] = frag<BKT>(s.t[0], ar + i * 32 + (lane & 31), kc);
      al[i] = frag<BKT>(s.t[1], ar + i * 32 + (lane & 31), kc);
    }
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      bh[j] = frag<BKT>(s.t[2], br + j * 32 + (lane & 31), kc);
      bl[j] = frag<BKT>(s.t[3], br + j * 32 + (lane & 31), kc);
    }
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
      for (int j = 0; j < WJ; ++j) {
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
