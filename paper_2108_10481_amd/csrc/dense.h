// Assembled far field: shared between the single- and multi-right-hand-side paths.
#pragma once
#include <vector>

#include "pbm_internal.h"

namespace pbm {

// Dense row-major far-field matrix in the vertex basis.  Rows: [block row 0
// (V) | block row 1 (V)]; columns: [x1 (V) | 0 | x2 (V) | 0] with each column
// block padded to Vp (a multiple of 64) so 16-byte loads never straddle blocks.
struct Dense {
    int V = 0, n = 0;
    size_t Vp = 0;                 // column offset of the second block
    size_t ld = 0;                 // row stride in elements = 2 Vp
    double *A64 = nullptr;
    float *A32 = nullptr;
    uint16_t *A16 = nullptr;
    int kind16 = 0;                // 0 none, 1 bf16, 2 fp16
    float scale16[4] = {1, 1, 1, 1};   // fp16: stored = entry * scale (blocks 11, 12, 21, 22)
    int ncolor = 0;
    std::vector<int32_t> color_ptr;
    int32_t *color_tri = nullptr;  // target triangles grouped by colour
    // source tiles: consecutive Morton-ordered triangles, coloured so that
    // tiles of one colour touch disjoint vertices
    int tile = 256;
    int ntile = 0, ntcolor = 0;
    // targets one assembly block processes in turn against its tile
    int asm_group = 4;
    // one evaluation per unordered triangle pair (FP32 storage): per launch
    // (tile colour, target colour) the blocks {tile, first, end, 0} of targets
    // t < (tile + 1) * tile size, and the side matrix C (2V x Vp) of the
    // swapped pairs' non-symmetric values; C aliases A16 in mixed modes
    bool sym = false;
    std::vector<size_t> sym_ptr;
    int4 *sym_blocks = nullptr;
    float *C32 = nullptr;
    std::vector<int32_t> tcolor_ptr;
    int32_t *tcolor_tile = nullptr;
    int32_t *tv_ptr = nullptr, *tv_col = nullptr, *tv_eptr = nullptr, *te = nullptr;
    // dense index of each vertex (first touch in tile order) and its inverse
    int32_t *vpos = nullptr, *vperm = nullptr;
    float *x32 = nullptr;          // ld (padded) FP32 copy of x
    double *x64 = nullptr;         // ld (padded) FP64 copy of x
    double *gpart = nullptr;       // 2 n partial row sums of the split GEMV
    int level = 1;                 // 1: accurate operator, 0: 16-bit operator
    int gemv_hi = -1, gemv_lo = -1;   // autotuned GEMV variants (-1: not tuned yet)
    // multi right-hand side workspaces (allocated on first use)
    uint16_t *X16 = nullptr;       // 16 x ld
    double *Y16 = nullptr;         // 16 x n
    // the 16-bit copy in the MFMA GEMM's operand order (allocated on the first
    // batched product): for each 16-row tile and 32-column step, the 16 x 32
    // block as 64 lanes x 8 values (lane l: row l % 16, columns 8 (l / 16) ..),
    // so each of the GEMM's loads reads 1 KB of consecutive bytes; refreshed
    // when the 16-bit copy is rewritten (the versions differ)
    uint16_t *A16t = nullptr;
    bool a16t_failed = false;      // no room for it: the GEMM reads the row-major copy
    unsigned a16_version = 0, a16t_version = 0;
};

constexpr int kMaxBatch = 16;

}  // namespace pbm
