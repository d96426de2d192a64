// gemm_layout.h -- where the matrix-core engine keeps each value of an
// N = 256 block (16 x 16: sample n = 16 n1 + n2, bin k = k1 + 16 k2) in the
// registers of one 64-lane wave, and which DFT-matrix entry every lane feeds
// to each of its four products.  Host and device: a host build checks the
// layout against a float64 DFT.
//
// Matrix-core operand layout (v_mfma_f32_16x16x32_f16; lane l = 16 g + c):
//   A (16 x 32): lane (g, c) holds row c, contraction entries 8g .. 8g+7
//   B (32 x 16): lane (g, c) holds column c, contraction entries 8g .. 8g+7
//   D (16 x 16): lane (g, c) holds rows 4g .. 4g+3 of column c
// A complex contraction over 16 terms puts term t(g, j) (j < 4) of lane group
// g at entries 8g + j (real parts) and 8g + 4 + j (imaginary parts), except in
// S1, whose entries 8g + 2j, 8g + 2j + 1 hold the real and imaginary part as
// the samples are stored; only the pairing of entries between A and B
// matters, so each stage may order its 16 terms as it likes, provided both
// operands agree.
//
// The four products of one block (W[a][b] = w16^{ab}, w16 = exp(-j 2 pi/16)):
//   S1  D1[n2][k1] = sum_n1 x[n1][n2] W[n1][k1]      A = input, B = W
//   S2  X[k2][k1]  = sum_n2 W[k2][n2] T[n2][k1] D1   A = W, B = twiddled D1
//   S3  D3[k1][n2] = sum_k2 Y[k2][k1] conj W[k2][n2] A = Y (transposed), B = W
//                                                    (as conj(sum conj(Y) W))
//   S4  z[n1][n2]  = sum_k1 conj W[n1][k1] T* D3     A = conj W, B = twiddled D3
// with the twiddles T[n2][k1] = w256^{n2 k1}.  The accumulator layout of each
// product is the next one's operand layout, so a block stays in registers.
//
// Two row orders differ from the natural one:
//   * S1's 16 terms in lane group g are the input rows n1 = g + 4 j: for
//     M = 192 the next block's rows 0..3 are this block's rows 12..15, i.e.
//     slot 0 of the next block is slot 3 of this one, in the same lane;
//   * S4's output rows are the 4 x 4 transpose of D's (row 4 g + r of D holds
//     z[n1 = 4 r + g]): one store instruction (fixed r) then writes the 64
//     consecutive samples 16 (4 r + g) + c, whole 128-byte lines.
#pragma once

#include <hip/hip_runtime.h>

#define VBW_GL_HD __host__ __device__ __forceinline__

namespace vbw {
namespace gemm {

// input row n1 in slot j (j < 4) of lane group g
VBW_GL_HD constexpr int in_row(int g, int j) { return g + 4 * j; }
// 4 x 4 transpose of a row index: 4 a + b -> 4 b + a
VBW_GL_HD constexpr int transpose4(int i) { return 4 * (i & 3) + (i >> 2); }
// output row n1 in accumulator slot r (r < 4) of lane group g
VBW_GL_HD constexpr int out_row(int g, int r) { return transpose4(4 * g + r); }

// Exponent e (W = w16^e) of the DFT-matrix entry that lane (g, c) feeds to
// contraction term j of each product.
VBW_GL_HD constexpr int s1_w(int g, int c, int j) { return (in_row(g, j) * c) & 15; }        // W[n1][k1 = c]
VBW_GL_HD constexpr int s2_w(int g, int c, int j) { return (c * (4 * g + j)) & 15; }         // W[k2 = c][n2]
// S3's entries W[k2 = 4 g + j][n2 = c] equal S2's (W is symmetric): S3 runs
// as the conjugate of a forward product with S2's operand.
VBW_GL_HD constexpr int s4_w(int g, int c, int j) { return (transpose4(c) * (4 * g + j)) & 15; }  // W[n1][k1]
// Exponent of the twiddle w256^{n2 k1} in accumulator slot r of lane (g, c)
// (S1 output: n2 = 4 g + r, k1 = c; S3 output: k1 = 4 g + r, n2 = c).
VBW_GL_HD constexpr int tw_e(int g, int c, int r) { return ((4 * g + r) * c) & 255; }

}  // namespace gemm
}  // namespace vbw
